"""FX-correlator oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Plain float64 / exact-integer statements of the correlator hot path of Wang &
Harris (Exp. Astron. 2013): the F-engine DFT (Section 2, Eq. 1, for complex
samples and for the 8-bit real samples of Section 5), the X-engine
correlation over the triangle of non-redundant pairs (Section 2, Eq. 2 and
Section 4), the requantisers of the reduced-precision forms, and the emission
of the visibility triangle in the supported layouts and orders.

The arithmetic lives in ``oracle.c`` (plain C, float64 / int64, OpenMP over
independent outputs).  This module only marshals numpy arrays to it, plus the
layout emission, which is pure indexing.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Flags: no -march (the library may run on another host), no fast-math and no
# FMA contraction, so every product and sum is rounded as written.
CFLAGS = ["-O3", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it; returns the path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.oracle_fengine.argtypes = [P, i64, i32, i32, i32, P, i32, P]
        L.oracle_fengine_real8.argtypes = [P, i64, i32, i32, i32, P, i32, P]
        L.oracle_xengine_f64.argtypes = [P, i32, i32, i32, P]
        L.oracle_xengine_i8.argtypes = [P, i32, i32, i32, P]
        L.oracle_round_format.argtypes = [ctypes.c_double, i32, i32, ctypes.c_double]
        L.oracle_round_format.restype = ctypes.c_double
        for f in ("oracle_quant_f16", "oracle_quant_e4m3", "oracle_quant_int8"):
            getattr(L, f).argtypes = [P, i64, P]
        L.oracle_decode_e4m3.argtypes = [i32]
        L.oracle_decode_e4m3.restype = ctypes.c_double
        L.oracle_decode_f16.argtypes = [i32]
        L.oracle_decode_f16.restype = ctypes.c_double
        L.oracle_max_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# --------------------------------------------------------------------------
# Eq. 1
# --------------------------------------------------------------------------
def fengine(volts: np.ndarray, C: int, n_spectra: int, chans=None) -> np.ndarray:
    """Direct DFT (Eq. 1) of consecutive C-sample blocks.

    volts: complex64 [n_inputs][ld] with ld >= n_spectra*C.
    chans: channels to evaluate (default all C).
    Returns complex128 S[a][p][c] for a < n_spectra, p < n_inputs, c < len(chans).
    """
    v = np.ascontiguousarray(volts, dtype=np.complex64)
    n_inputs, ld = v.shape
    if ld < n_spectra * C:
        raise ValueError("voltage rows shorter than n_spectra*C")
    ch = np.arange(C, dtype=np.int32) if chans is None else np.ascontiguousarray(chans, dtype=np.int32)
    if ch.size and (ch.min() < 0 or ch.max() >= C):
        raise ValueError("channel out of range")
    S = np.empty((n_spectra, n_inputs, ch.size), dtype=np.complex128)
    lib().oracle_fengine(_ptr(v), ld, n_inputs, C, n_spectra, _ptr(ch), ch.size, _ptr(S))
    return S


def fengine_real8(samples: np.ndarray, C: int, n_spectra: int, chans=None) -> np.ndarray:
    """Real-input Eq. 1 (Section 5: 8-bit real samples): direct DFT of length 2C
    of consecutive 2C-sample blocks.

    samples: int8 [n_inputs][ld] with ld >= n_spectra*2C.
    chans: channels to evaluate, each in [0, C] (default 0..C-1; C is Nyquist).
    Returns complex128 S[a][p][c].
    """
    x = np.ascontiguousarray(samples, dtype=np.int8)
    n_inputs, ld = x.shape
    if ld < n_spectra * 2 * C:
        raise ValueError("sample rows shorter than n_spectra*2C")
    ch = np.arange(C, dtype=np.int32) if chans is None else np.ascontiguousarray(chans, dtype=np.int32)
    if ch.size and (ch.min() < 0 or ch.max() > C):
        raise ValueError("channel out of range")
    S = np.empty((n_spectra, n_inputs, ch.size), dtype=np.complex128)
    lib().oracle_fengine_real8(_ptr(x), ld, n_inputs, C, n_spectra, _ptr(ch), ch.size, _ptr(S))
    return S


# --------------------------------------------------------------------------
# Eq. 2
# --------------------------------------------------------------------------
def n_products(N: int) -> int:
    return N * (N + 1) // 2


def tri_lower_index(i, j):
    """b(i, j) = i(i+1)/2 + j for j <= i."""
    return i * (i + 1) // 2 + j


def xengine_f64(S: np.ndarray) -> np.ndarray:
    """S complex128 [A][N][K] -> V complex128 [K][N(N+1)/2] (lower triangle, Eq. 2)."""
    S = np.ascontiguousarray(S, dtype=np.complex128)
    A, N, K = S.shape
    V = np.empty((K, n_products(N)), dtype=np.complex128)
    lib().oracle_xengine_f64(_ptr(S), A, N, K, _ptr(V))
    return V


def xengine_i8(S: np.ndarray) -> np.ndarray:
    """S int8 [A][N][K][2] -> V int64 [K][N(N+1)/2][2], exact (Eq. 2)."""
    S = np.ascontiguousarray(S, dtype=np.int8)
    A, N, K, two = S.shape
    assert two == 2
    V = np.empty((K, n_products(N), 2), dtype=np.int64)
    lib().oracle_xengine_i8(_ptr(S), A, N, K, _ptr(V))
    return V


# --------------------------------------------------------------------------
# Requantisers and decoders
# --------------------------------------------------------------------------
def round_format(y: float, mbits: int, emin: int, maxval: float) -> float:
    return float(lib().oracle_round_format(float(y), mbits, emin, float(maxval)))


def quant_f16(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    q = np.empty_like(y)
    lib().oracle_quant_f16(_ptr(y), y.size, _ptr(q))
    return q


def quant_e4m3(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    q = np.empty_like(y)
    lib().oracle_quant_e4m3(_ptr(y), y.size, _ptr(q))
    return q


def quant_int8(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    q = np.empty(y.shape, dtype=np.int8)
    lib().oracle_quant_int8(_ptr(y), y.size, _ptr(q))
    return q


def quantise(S: np.ndarray, inv_scale: np.ndarray, precision: str) -> np.ndarray:
    """Requantise complex spectra S[..., k] with per-channel FP32 scale inv_s[k].

    y = S * inv_s[k] in float64, then the format's rounding on re and im.
    Returns int8 [..., 2] for 'int8', float64 [..., 2] (exact format values)
    for 'fp16' / 'fp8', and the unquantised float64 pair for 'fp32'.
    """
    y = np.ascontiguousarray(S, dtype=np.complex128) * np.asarray(inv_scale, dtype=np.float32).astype(np.float64)
    pair = np.stack([y.real, y.imag], axis=-1)
    if precision == "int8":
        return quant_int8(pair)
    if precision == "fp16":
        return quant_f16(pair)
    if precision == "fp8":
        return quant_e4m3(pair)
    if precision == "fp32":
        return pair
    raise ValueError(precision)


def decode_e4m3(codes: np.ndarray) -> np.ndarray:
    L = lib()
    table = np.array([L.oracle_decode_e4m3(c) for c in range(256)], dtype=np.float64)
    return table[np.asarray(codes, dtype=np.uint8)]


def decode_f16(codes: np.ndarray) -> np.ndarray:
    L = lib()
    table = np.array([L.oracle_decode_f16(c) for c in range(65536)], dtype=np.float64)
    return table[np.asarray(codes, dtype=np.uint16)]


# --------------------------------------------------------------------------
# Emission: layouts and orders of the visibility triangle
# --------------------------------------------------------------------------
LAYOUTS = ("lower", "upper", "full")
ORDERS = ("chan", "baseline")


def layout_pairs(N: int, layout: str):
    """The (i, j) pair of every stored product, in storage order.

    lower: rows i, columns j <= i, b = i(i+1)/2 + j.
    upper: rows i, columns j >= i, b = i*N - i(i-1)/2 + (j - i).
    full : all (i, j), b = i*N + j.
    """
    if layout == "lower":
        return [(i, j) for i in range(N) for j in range(i + 1)]
    if layout == "upper":
        return [(i, j) for i in range(N) for j in range(i, N)]
    if layout == "full":
        return [(i, j) for i in range(N) for j in range(N)]
    raise ValueError(layout)


def emit(V_lower: np.ndarray, N: int, layout: str = "lower", order: str = "chan") -> np.ndarray:
    """Re-express lower-triangle visibilities V[K][B] (any dtype; complex or
    trailing (re, im) pair) in the requested layout and order.

    C_ij for j > i is conj(C_ji) (Hermitian symmetry of Eq. 2).
    order 'chan' gives [K][b]; 'baseline' gives [b][K].
    """
    pairs = layout_pairs(N, layout)
    src = np.empty(len(pairs), dtype=np.int64)
    conj = np.zeros(len(pairs), dtype=bool)
    for t, (i, j) in enumerate(pairs):
        if j <= i:
            src[t] = tri_lower_index(i, j)
        else:
            src[t] = tri_lower_index(j, i)
            conj[t] = True
    out = V_lower[:, src].copy()
    if np.iscomplexobj(out):
        out[:, conj] = np.conj(out[:, conj])
    else:  # trailing (re, im)
        out[:, conj, 1] = -out[:, conj, 1]
    if order == "baseline":
        out = np.ascontiguousarray(np.swapaxes(out, 0, 1))
    elif order != "chan":
        raise ValueError(order)
    return out
