"""Exact requantiser parity through the whole F-engine.

A constant block s[n] = v has the exact FFT S[0] = 16 v, S[k != 0] = 0 for
C = 16 (sums of equal values and zeros are exact in FP32), so with
inv_s[0] = 1/16 each block hands the value v, unrounded, to the requantiser.
Feeding chosen v (every E4M3 code, every tie between neighbouring codes,
values one float32 step either side of the ties, subnormals, saturation)
pins the GPU's int8 / binary16 / E4M3 rounding bit for bit against the
oracle's definitions."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
from helpers import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
C = 16


def _neighbours(vals):
    f = np.asarray(vals, np.float32)
    return np.concatenate([f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))])


def _cases(prec):
    if prec == "fp8":
        codes = oracle.decode_e4m3(np.arange(256, dtype=np.uint8))
        fin = np.unique(codes[np.isfinite(codes)])
        mids = (fin[:-1] + fin[1:]) / 2
        extra = [448.0, 449.0, 463.99, 464.0, 464.01, 480.0, 1e4, 1e30, 2.0 ** -10, 3 * 2.0 ** -11, 2.0 ** -12]
        v = np.concatenate([fin, _neighbours(mids), extra, -np.asarray(extra)])
    elif prec == "fp16":
        rng = np.random.default_rng(0)
        a = rng.standard_normal(3000).astype(np.float16).astype(np.float64)
        b = np.nextafter(a.astype(np.float16), np.float16(np.inf)).astype(np.float64)
        mids = (a + b) / 2                                    # exact binary16 ties
        sub = np.arange(1, 64) * 2.0 ** -24                     # subnormals
        extra = [65504.0, 65519.0, 65520.0, 70000.0, 1e30, 2.0 ** -25, 3 * 2.0 ** -26]
        v = np.concatenate([a, _neighbours(mids), sub, (sub[:-1] + sub[1:]) / 2, extra, -np.asarray(extra)])
    else:
        k = np.arange(-130, 131, dtype=np.float64)
        v = np.concatenate([k, _neighbours(k + 0.5), [1e6, -1e6, 127.49, -127.51]])
    return np.asarray(v, np.float32)


@pytest.mark.parametrize("prec", ["int8", "fp16", "fp8"])
def test_requantiser_bit_exact_on_exact_spectra(prec):
    vals = _cases(prec)
    n_pairs = (vals.size + 1) // 2
    N = 32
    A = -(-n_pairs // N)
    pad = np.zeros(2 * N * A, np.float32)
    pad[: vals.size] = vals
    pairs = pad.reshape(N, A, 2)                              # (re, im) level per block
    say(f"exact requantiser {prec}: {vals.size} values, N={N} A={A}")
    v = np.repeat(pairs[:, :, None, :], C, axis=2).reshape(N, A * C, 2)
    volts = torch.from_numpy(np.ascontiguousarray(v)).to(DEV).view(torch.complex64).reshape(N, A * C)
    inv = np.zeros(C, np.float32)
    inv[0] = 1.0 / 16.0
    inv[1:] = 1.0
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine(volts, A, torch.from_numpy(inv).to(DEV))
        sp = c.spectra().cpu()                               # [A][C][N][2]
    got = sp.numpy().astype(np.float64) if prec == "int8" else sp.to(torch.float64).numpy()
    y = np.transpose(pairs, (1, 0, 2)).astype(np.float64)     # [A][N][2], exact S[0] * inv_s[0]
    if prec == "int8":
        ref = oracle.quant_int8(y).astype(np.float64)
    elif prec == "fp16":
        ref = oracle.quant_f16(y)
    else:
        ref = oracle.quant_e4m3(y)
    ch0 = got[:, 0]
    bad = np.argwhere(ch0 != ref)
    assert bad.size == 0, [(y[tuple(b)], ch0[tuple(b)], ref[tuple(b)]) for b in bad[:8]]
    assert not got[:, 1:].any()                               # every other channel is exactly 0
