"""Comparison helpers for the GPU parity tests (no arithmetic of the method)."""
import math
import sys

import numpy as np


def say(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print(msg, flush=True)
    sys.stdout.flush()


def cplx(x: np.ndarray) -> np.ndarray:
    """[..., 2] (re, im) -> complex128."""
    x = np.asarray(x)
    return x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)


def spectra_akp_to_apk(S):
    """Public GPU spectra [A][C][N](...) -> oracle order [A][N][C](...)."""
    return np.ascontiguousarray(np.swapaxes(S, 1, 2))


def autos(V: np.ndarray, N: int) -> np.ndarray:
    """Auto products C_ii[k] (real) of lower-triangle visibilities V[K][B]."""
    idx = np.array([i * (i + 1) // 2 + i for i in range(N)])
    return np.real(V[:, idx])


def vis_errors(got: np.ndarray, ref: np.ndarray, N: int):
    """Per-channel relative Frobenius error e_F(k) = |V - V64|_F / |V64|_F and
    the largest normalised element error e_n = |V - V64| / sqrt(C_ii C_jj)
    (both over lower-triangle complex visibilities [K][B])."""
    eF = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    d = np.maximum(autos(ref, N), 1e-300)                     # [K][N]
    il, jl = np.tril_indices(N)
    norm = np.sqrt(d[:, il] * d[:, jl])
    en = np.abs(got - ref) / norm
    return eF, en


def tie_mismatches(q_gpu, q_ref, y_ref, eps):
    """Rounded codes may differ only where the float64 value sits within eps of
    the midpoint of the two codes (an FP32-vs-FP64 rounding tie).  Returns
    (number of mismatches, number of unexplained mismatches)."""
    q_gpu = np.asarray(q_gpu, np.float64)
    q_ref = np.asarray(q_ref, np.float64)
    mism = q_gpu != q_ref
    mid = 0.5 * (q_gpu + q_ref)
    eps = np.broadcast_to(eps, q_ref.shape)
    bad = mism & (np.abs(np.asarray(y_ref) - mid) > eps)
    return int(mism.sum()), int(bad.sum())


def fft_error_bound(C: int, rms: np.ndarray) -> np.ndarray:
    """A generous bound on the FP32 FFT error of a spectrum value: a few units
    of 2^-24 per radix stage times the channel RMS."""
    return 8.0 * max(1, int(math.log2(C))) * 2.0 ** -24 * rms
