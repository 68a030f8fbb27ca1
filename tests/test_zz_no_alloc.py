"""The no-alloc X-engine (corr_xengine_noalloc) against the handle-based
X-engine on caller spectra (corr_xengine + dump), through the C ABI: two calls
in a row with the second smaller, a case that runs in several channel chunks,
accumulation, FP16 with per-channel scales and a ragged FP32 case; int8
results are also checked bit for bit against the integer oracle (Eq. 2)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, spectra_akp_to_apk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _handle_result(st, npol, C, A, prec, S, inv=None, calls=1):
    with corr.Correlator(st, npol, C, A, prec) as c:
        for _ in range(calls):
            c.xengine(A, S, inv)
        return c.dump()


def _noalloc(st, npol, C, A, prec, S, inv=None, vis=None, accumulate=False):
    p = corr.make_params(st, npol, C, 1, prec)
    if vis is None:
        N = st * npol
        dt = torch.int32 if prec == "int8" else torch.float32
        vis = torch.empty((C, N * (N + 1) // 2, 2), dtype=dt, device=DEV)
    corr.corr_xengine_noalloc(p, S, A, inv, vis, accumulate)
    return vis


@pytest.mark.parametrize("st,npol,C,A", [(75, 2, 64, 200), (20, 2, 32, 70)])
def test_noalloc_int8_two_calls_second_smaller(st, npol, C, A):
    say(f"noalloc int8 {st}x{npol} C={C} A={A}")
    S = synth.int8_spectra(A, C, st * npol, seed=st + A)
    Sd = torch.from_numpy(S).to(DEV)
    got = _noalloc(st, npol, C, A, "int8", Sd)
    ref = _handle_result(st, npol, C, A, "int8", Sd)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.xengine_i8(spectra_akp_to_apk(S)))


def test_noalloc_int8_many_chunks_and_accumulate():
    st, npol, C, A = 256, 2, 64, 2048                     # 2 MiB of staging per channel: 5 chunks
    say(f"noalloc int8 chunks {st}x{npol} C={C} A={A}")
    Sd = synth.int8_spectra(A, C, st * npol, seed=5, device=DEV)
    got = _noalloc(st, npol, C, A, "int8", Sd)
    got = _noalloc(st, npol, C, A, "int8", Sd, vis=got, accumulate=True)
    ref = _handle_result(st, npol, C, A, "int8", Sd, calls=2)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    chans = [0, 31, 63]
    q = Sd[:, chans].cpu().numpy()
    assert np.array_equal(got[chans].cpu().numpy().astype(np.int64),
                          2 * oracle.xengine_i8(spectra_akp_to_apk(q)))


def test_noalloc_fp16_scaled_accumulate():
    st, npol, C, A = 70, 1, 32, 96
    say("noalloc fp16 with scales")
    q = np.clip(synth.int8_spectra(A, C, st * npol, seed=9, rms=3.0), -8, 8).astype(np.float64)
    Sd = torch.from_numpy(q).to(torch.float16).to(DEV)
    inv = torch.from_numpy(np.linspace(0.5, 2.0, C).astype(np.float32)).to(DEV)
    got = _noalloc(st, npol, C, A, "fp16", Sd, inv)
    got = _noalloc(st, npol, C, A, "fp16", Sd, inv, vis=got, accumulate=True)
    ref = _handle_result(st, npol, C, A, "fp16", Sd, inv, calls=2)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_fp32_ragged():
    st, npol, C, A = 33, 1, 16, 45
    say("noalloc fp32 ragged")
    q = synth.int8_spectra(A, C, st * npol, seed=13, rms=2.0).astype(np.float32)
    Sd = torch.from_numpy(q).to(DEV)
    got = _noalloc(st, npol, C, A, "fp32", Sd)
    ref = _handle_result(st, npol, C, A, "fp32", Sd)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    exact = oracle.xengine_f64(spectra_akp_to_apk(cplx(q)))
    assert np.allclose(cplx(got.cpu().numpy()), exact, rtol=0, atol=1e-3)
