"""ctypes binding of libcorr.so, the MI355X FX-correlator library.

The functions carry the C ABI's names and only marshal arguments: torch
tensors become device pointers, the HIP stream defaults to torch's current
stream, and a non-OK status raises CorrError.  Every step of the correlator
runs in the library's HIP kernels; there is no Python or CPU fallback, and
loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  -- loads the process's HIP runtime before libcorr.so

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcorr.so")

CORR_OK = 0
CORR_E_INVALID_ARG = 1
CORR_E_UNSUPPORTED = 2
CORR_E_NOMEM = 3
CORR_E_OVERFLOW = 4
CORR_E_STATE = 5
CORR_E_HIP = 6

CORR_FP32, CORR_FP16, CORR_FP8_E4M3, CORR_INT8 = 0, 1, 2, 3
CORR_TRI_LOWER, CORR_TRI_UPPER, CORR_FULL = 0, 1, 2
CORR_CHAN_MAJOR, CORR_BASELINE_MAJOR = 0, 1
CORR_MIN_CHANNELS, CORR_MAX_CHANNELS, CORR_MAX_INPUTS = 16, 8192, 8192
CORR_INT8_MAX_INTEGRATE = 66572

PRECISIONS = {"fp32": CORR_FP32, "fp16": CORR_FP16, "fp8": CORR_FP8_E4M3, "int8": CORR_INT8}
LAYOUTS = {"lower": CORR_TRI_LOWER, "upper": CORR_TRI_UPPER, "full": CORR_FULL}
ORDERS = {"chan": CORR_CHAN_MAJOR, "baseline": CORR_BASELINE_MAJOR}
# element type of spectra per precision (re, im pairs)
SPECTRA_DTYPE = {CORR_FP32: torch.float32, CORR_FP16: torch.float16,
                 CORR_FP8_E4M3: torch.float8_e4m3fn, CORR_INT8: torch.int8}

# Header names of every exported function (checked by the ABI tests).
ABI_FUNCTIONS = (
    "corr_n_products", "corr_visibility_bytes", "corr_spectra_bytes", "corr_create",
    "corr_destroy", "corr_fengine", "corr_xengine", "corr_dump_visibilities",
    "corr_copy_spectra", "corr_get_counts", "corr_status_string", "corr_last_error",
    "corr_set_tile", "corr_autotune", "corr_create_batched", "corr_batch_get",
    "corr_xengine_batched", "corr_destroy_batched", "corr_xengine_rect", "corr_fengine_real8",
    "corr_fengine_at", "corr_fengine_real8_at", "corr_xengine_dump", "corr_xengine_noalloc", "corr_fx",
    "corr_set_spectra_layout", "corr_autotune_fx",
)


class corr_params(ctypes.Structure):
    _fields_ = [
        ("n_stations", ctypes.c_int32),
        ("n_pols", ctypes.c_int32),
        ("n_channels", ctypes.c_int32),
        ("n_integrate", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("device_mem_cap", ctypes.c_uint64),
    ]


class corr_tuning(ctypes.Structure):
    _fields_ = [
        ("tile", ctypes.c_int32),
        ("time_block_major", ctypes.c_int32),
        ("default_tile", ctypes.c_int32),
        ("default_time_block_major", ctypes.c_int32),
        ("ms_default", ctypes.c_float),
        ("ms_tuned", ctypes.c_float),
    ]


class CorrError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {corr_status_string(status)} ({detail})")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with paper_1305_5639_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        PP = ctypes.POINTER(corr_params)
        L.corr_n_products.argtypes = [PP]
        L.corr_n_products.restype = i64
        L.corr_visibility_bytes.argtypes = [PP]
        L.corr_visibility_bytes.restype = i64
        L.corr_spectra_bytes.argtypes = [PP, i32]
        L.corr_spectra_bytes.restype = i64
        L.corr_create.argtypes = [PP, P, ctypes.POINTER(P)]
        L.corr_destroy.argtypes = [P]
        L.corr_fengine.argtypes = [P, P, i64, i32, P]
        L.corr_fengine_real8.argtypes = [P, P, i64, i32, P]
        L.corr_fengine_at.argtypes = [P, P, i64, i32, P, i32]
        L.corr_fengine_real8_at.argtypes = [P, P, i64, i32, P, i32]
        L.corr_xengine.argtypes = [P, P, i32, P]
        L.corr_xengine_dump.argtypes = [P, P, i32, P, P]
        L.corr_dump_visibilities.argtypes = [P, P, i32, i32]
        L.corr_copy_spectra.argtypes = [P, P, i32]
        L.corr_get_counts.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.corr_status_string.argtypes = [i32]
        L.corr_status_string.restype = ctypes.c_char_p
        L.corr_last_error.argtypes = [P]
        L.corr_last_error.restype = ctypes.c_char_p
        L.corr_set_tile.argtypes = [P, i32]
        L.corr_autotune.argtypes = [P, i32, ctypes.POINTER(i32)]
        L.corr_create_batched.argtypes = [PP, i32, P, ctypes.POINTER(P)]
        L.corr_batch_get.argtypes = [P, i32, ctypes.POINTER(P)]
        L.corr_xengine_batched.argtypes = [P, ctypes.POINTER(i32)]
        L.corr_destroy_batched.argtypes = [P]
        L.corr_xengine_rect.argtypes = [P, i32, i32, i32, i32, i32, P, i32]
        L.corr_xengine_noalloc.argtypes = [PP, P, i32, P, P, i32, P]
        L.corr_fx.argtypes = [P, P, i64, i32, P, i32]
        L.corr_set_spectra_layout.argtypes = [P, i32]
        L.corr_autotune_fx.argtypes = [P, P, i64, i32, P, ctypes.POINTER(corr_tuning)]
        for f in ("corr_create", "corr_destroy", "corr_fengine", "corr_fengine_real8", "corr_fengine_at",
                  "corr_fengine_real8_at", "corr_xengine", "corr_xengine_dump",
                  "corr_xengine_rect", "corr_xengine_noalloc", "corr_fx",
                  "corr_dump_visibilities", "corr_copy_spectra", "corr_get_counts", "corr_set_tile",
                  "corr_autotune", "corr_create_batched", "corr_batch_get", "corr_xengine_batched",
                  "corr_destroy_batched", "corr_set_spectra_layout", "corr_autotune_fx"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------
def make_params(n_stations, n_pols, n_channels, n_integrate, precision="fp32", layout="lower",
                order="chan", device_mem_cap=0) -> corr_params:
    prec = PRECISIONS.get(precision, precision)
    lay = LAYOUTS.get(layout, layout)
    odr = ORDERS.get(order, order)
    return corr_params(int(n_stations), int(n_pols), int(n_channels), int(n_integrate), int(prec),
                       int(lay), int(odr), 0, int(device_mem_cap))


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    import numpy as np
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"cannot pass {type(x)} as a pointer")


def _on_device(x) -> int:
    return 1 if isinstance(x, torch.Tensor) and x.is_cuda else 0


def _check(status: int, where: str, h=None):
    if status != CORR_OK:
        raise CorrError(status, where, corr_last_error(h))


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return stream


# --------------------------------------------------------------------------
# the ABI, by name
# --------------------------------------------------------------------------
def corr_status_string(status: int) -> str:
    return lib().corr_status_string(int(status)).decode()


def corr_last_error(h=None) -> str:
    return lib().corr_last_error(h).decode()


def corr_n_products(params: corr_params) -> int:
    return int(lib().corr_n_products(ctypes.byref(params)))


def corr_visibility_bytes(params: corr_params) -> int:
    return int(lib().corr_visibility_bytes(ctypes.byref(params)))


def corr_spectra_bytes(params: corr_params, n_spectra: int) -> int:
    return int(lib().corr_spectra_bytes(ctypes.byref(params), int(n_spectra)))


def corr_create(params: corr_params, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().corr_create(ctypes.byref(params), _stream(stream), ctypes.byref(h)), "corr_create")
    return h


def corr_destroy(h) -> None:
    _check(lib().corr_destroy(h), "corr_destroy", h)


def _rows(x, ld_samples):
    """(pointer, ld) of a [rows][samples] buffer.  A 2-D tensor whose rows are
    contiguous but spaced further apart (a slice of a longer recording, say)
    is passed as is, its row stride as ld unless ld_samples is given."""
    if isinstance(x, torch.Tensor) and x.dim() == 2 and x.stride(-1) == 1 and not x.is_contiguous():
        return x.data_ptr(), (x.stride(0) if ld_samples is None else ld_samples)
    return _ptr(x), (x.shape[-1] if ld_samples is None else ld_samples)


def corr_fengine(h, volts, n_spectra: int, inv_scale=None, ld_samples: int | None = None,
                 first_spectrum: int = 0) -> None:
    """volts: complex64 [n_inputs][ld] voltages (device); rows may be a
    column slice of a wider tensor (ld = its row stride)."""
    ptr, ld_samples = _rows(volts, ld_samples)
    if first_spectrum:
        _check(lib().corr_fengine_at(h, ptr, int(ld_samples), int(n_spectra), _ptr(inv_scale),
                                     int(first_spectrum)), "corr_fengine_at", h)
    else:
        _check(lib().corr_fengine(h, ptr, int(ld_samples), int(n_spectra), _ptr(inv_scale)),
               "corr_fengine", h)


def corr_fengine_real8(h, samples, n_spectra: int, inv_scale=None, ld_samples: int | None = None,
                       first_spectrum: int = 0) -> None:
    """samples: int8 [n_inputs][ld] real samples (device); spectrum a of row p
    is the length-2C DFT of samples [a*2C, (a+1)*2C), channels 0..C-1.  Rows
    may be a column slice of a wider tensor (ld = its row stride)."""
    ptr, ld_samples = _rows(samples, ld_samples)
    if first_spectrum:
        _check(lib().corr_fengine_real8_at(h, ptr, int(ld_samples), int(n_spectra), _ptr(inv_scale),
                                           int(first_spectrum)), "corr_fengine_real8_at", h)
    else:
        _check(lib().corr_fengine_real8(h, ptr, int(ld_samples), int(n_spectra), _ptr(inv_scale)),
               "corr_fengine_real8", h)


def corr_xengine(h, spectra, n_spectra: int, inv_scale=None) -> None:
    _check(lib().corr_xengine(h, _ptr(spectra), int(n_spectra), _ptr(inv_scale)), "corr_xengine", h)


def corr_xengine_dump(h, spectra, n_spectra: int, inv_scale, dst) -> None:
    _check(lib().corr_xengine_dump(h, _ptr(spectra), int(n_spectra), _ptr(inv_scale), _ptr(dst)),
           "corr_xengine_dump", h)


def corr_xengine_rect(h, i0: int, ni: int, j0: int, nj: int, n_spectra: int, out, accumulate: bool = False) -> None:
    _check(lib().corr_xengine_rect(h, int(i0), int(ni), int(j0), int(nj), int(n_spectra), _ptr(out),
                                   int(bool(accumulate))), "corr_xengine_rect", h)


def corr_fx(h, volts, n_spectra: int, inv_scale, chunk_spectra: int, ld_samples: int | None = None) -> None:
    x, ld = _rows(volts, ld_samples)
    _check(lib().corr_fx(h, x, int(ld), int(n_spectra), _ptr(inv_scale), int(chunk_spectra)), "corr_fx", h)


def corr_xengine_noalloc(params: corr_params, spectra, n_spectra: int, inv_scale, vis, accumulate: bool = False,
                         stream=None) -> None:
    _check(lib().corr_xengine_noalloc(ctypes.byref(params), _ptr(spectra), int(n_spectra), _ptr(inv_scale),
                                      _ptr(vis), int(bool(accumulate)), _stream(stream)), "corr_xengine_noalloc")


def corr_dump_visibilities(h, dst, reset: bool = True, dst_on_device: int | None = None) -> None:
    dev = _on_device(dst) if dst_on_device is None else int(dst_on_device)
    _check(lib().corr_dump_visibilities(h, _ptr(dst), dev, int(bool(reset))), "corr_dump_visibilities", h)


def corr_copy_spectra(h, dst, dst_on_device: int | None = None) -> None:
    dev = _on_device(dst) if dst_on_device is None else int(dst_on_device)
    _check(lib().corr_copy_spectra(h, _ptr(dst), dev), "corr_copy_spectra", h)


def corr_get_counts(h) -> tuple[int, int]:
    a, b = ctypes.c_int32(), ctypes.c_int64()
    _check(lib().corr_get_counts(h, ctypes.byref(a), ctypes.byref(b)), "corr_get_counts", h)
    return a.value, b.value


def corr_set_tile(h, tile: int) -> None:
    _check(lib().corr_set_tile(h, int(tile)), "corr_set_tile", h)


def corr_autotune(h, n_spectra: int) -> int:
    t = ctypes.c_int32()
    _check(lib().corr_autotune(h, int(n_spectra), ctypes.byref(t)), "corr_autotune", h)
    return t.value


def corr_set_spectra_layout(h, time_block_major: int) -> None:
    _check(lib().corr_set_spectra_layout(h, int(time_block_major)), "corr_set_spectra_layout", h)


def corr_autotune_fx(h, volts, n_spectra: int, inv_scale=None, ld_samples: int | None = None) -> dict:
    x, ld = _rows(volts, ld_samples)
    t = corr_tuning()
    _check(lib().corr_autotune_fx(h, x, int(ld), int(n_spectra), _ptr(inv_scale), ctypes.byref(t)),
           "corr_autotune_fx", h)
    return {"tile": t.tile, "time_block_major": t.time_block_major,
            "default": {"tile": t.default_tile, "time_block_major": t.default_time_block_major},
            "ms_default": t.ms_default, "ms_tuned": t.ms_tuned}


def corr_create_batched(params_list, stream=None) -> ctypes.c_void_p:
    arr = (corr_params * len(params_list))(*params_list)
    b = ctypes.c_void_p()
    _check(lib().corr_create_batched(arr, len(params_list), _stream(stream), ctypes.byref(b)),
           "corr_create_batched")
    return b


def corr_batch_get(b, i: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().corr_batch_get(b, int(i), ctypes.byref(h)), "corr_batch_get")
    return h


def corr_xengine_batched(b, n_spectra) -> None:
    arr = (ctypes.c_int32 * len(n_spectra))(*[int(x) for x in n_spectra])
    _check(lib().corr_xengine_batched(b, arr), "corr_xengine_batched")


def corr_destroy_batched(b) -> None:
    _check(lib().corr_destroy_batched(b), "corr_destroy_batched")


# --------------------------------------------------------------------------
# small owning wrappers
# --------------------------------------------------------------------------
class Correlator:
    """Owns one handle; methods map one-to-one onto the ABI calls."""

    def __init__(self, n_stations, n_pols, n_channels, n_integrate, precision="fp32", layout="lower",
                 order="chan", device_mem_cap=0, stream=None, _borrowed=None):
        self.params = make_params(n_stations, n_pols, n_channels, n_integrate, precision, layout, order,
                                  device_mem_cap)
        self.n_inputs = n_stations * n_pols
        self.n_channels = n_channels
        self.precision = self.params.precision
        self._owned = _borrowed is None
        self.handle = corr_create(self.params, stream) if self._owned else _borrowed

    def fengine(self, volts, n_spectra, inv_scale=None, ld_samples=None, first_spectrum=0):
        """F-engine into the held spectra; first_spectrum > 0 appends at that
        (time-block aligned) offset."""
        corr_fengine(self.handle, volts, n_spectra, inv_scale, ld_samples, first_spectrum)

    def fengine_real8(self, samples, n_spectra, inv_scale=None, ld_samples=None, first_spectrum=0):
        corr_fengine_real8(self.handle, samples, n_spectra, inv_scale, ld_samples, first_spectrum)

    def xengine(self, n_spectra, spectra=None, inv_scale=None):
        corr_xengine(self.handle, spectra, n_spectra, inv_scale)

    def fx(self, volts, n_spectra, inv_scale=None, chunk_spectra=None, ld_samples=None):
        """F and X fused over time chunks (corr_fx)."""
        corr_fx(self.handle, volts, n_spectra, inv_scale,
                self.params.n_integrate if chunk_spectra is None else chunk_spectra, ld_samples)

    def xengine_dump(self, n_spectra, dst=None, spectra=None, inv_scale=None):
        """Last X-engine call of an integration, its result written straight to
        dst (a device tensor from new_visibilities()); the integration resets."""
        if dst is None:
            dst = self.new_visibilities()
        corr_xengine_dump(self.handle, spectra, n_spectra, inv_scale, dst)
        return dst

    def xengine_rect(self, i0, ni, j0, nj, n_spectra, out=None, accumulate=False):
        """Rows [i0, i0+ni) against columns [j0, j0+nj) of the held spectra:
        a [C][ni][nj][2] tensor (float32; int32 for int8), written or added to."""
        if out is None:
            dt = torch.int32 if self.precision == CORR_INT8 else torch.float32
            out = torch.empty((self.n_channels, ni, nj, 2), dtype=dt, device="cuda")
        corr_xengine_rect(self.handle, i0, ni, j0, nj, n_spectra, out, accumulate)
        return out

    def visibility_shape(self):
        """Shape of a dump as a tensor whose last axis is (re, im)."""
        N, C = self.n_inputs, self.n_channels
        B = N * N if self.params.layout == CORR_FULL else N * (N + 1) // 2
        return (C, B, 2) if self.params.order == CORR_CHAN_MAJOR else (B, C, 2)

    def new_visibilities(self, device="cuda"):
        dt = torch.int32 if self.precision == CORR_INT8 else torch.float32
        return torch.empty(self.visibility_shape(), dtype=dt, device=device)

    def dump(self, dst=None, reset=True, device="cuda"):
        if dst is None:
            dst = self.new_visibilities(device)
        corr_dump_visibilities(self.handle, dst, reset)
        return dst

    def spectra(self, device="cuda"):
        n_held, _ = corr_get_counts(self.handle)
        dst = torch.empty((n_held, self.n_channels, self.n_inputs, 2),
                          dtype=SPECTRA_DTYPE[self.precision], device=device)
        corr_copy_spectra(self.handle, dst)
        return dst

    def counts(self):
        return corr_get_counts(self.handle)

    def set_tile(self, tile):
        corr_set_tile(self.handle, tile)

    def autotune(self, n_spectra):
        return corr_autotune(self.handle, n_spectra)

    def set_spectra_layout(self, time_block_major):
        corr_set_spectra_layout(self.handle, time_block_major)

    def autotune_fx(self, volts, n_spectra, inv_scale=None, ld_samples=None):
        """Choose block size and spectra order on these voltages; the handle
        then holds their spectra (as after fengine)."""
        return corr_autotune_fx(self.handle, volts, n_spectra, inv_scale, ld_samples)

    def close(self):
        if self.handle and self._owned:
            corr_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns a batch of sub-arrays; sub-arrays are borrowed Correlator views."""

    def __init__(self, shapes, precision="fp16", layout="lower", order="chan", stream=None):
        """shapes: list of (n_stations, n_pols, n_channels, n_integrate)."""
        plist = [make_params(*sh, precision, layout, order) for sh in shapes]
        self.handle = corr_create_batched(plist, stream)
        self.subs = [Correlator(*sh, precision, layout, order, _borrowed=corr_batch_get(self.handle, i))
                     for i, sh in enumerate(shapes)]

    def __len__(self):
        return len(self.subs)

    def __getitem__(self, i):
        return self.subs[i]

    def xengine(self, n_spectra):
        corr_xengine_batched(self.handle, n_spectra)

    def close(self):
        if self.handle:
            for s in self.subs:
                s.handle = None
            corr_destroy_batched(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
