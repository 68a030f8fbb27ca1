"""F and X fused over time chunks (corr_fx): the same integration as one
F-engine + X-engine pass -- bit for bit for int8, against the integer oracle
(Eq. 2) on the requantised spectra, and within the FP32 bound of the float64
oracle (Eq. 1 then Eq. 2) -- for several chunk sizes, a ragged last chunk,
both F-engine forms (direct and chunked gather) and an integration longer
than the spectra the handle holds."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, spectra_akp_to_apk, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("st,C,A,chunk", [(20, 64, 300, 64), (20, 64, 300, 128), (33, 2048, 130, 64),
                                          (9, 256, 64, 64)])
def test_fx_int8_equals_unfused_and_oracle(st, C, A, chunk):
    say(f"fx int8 {st}x2 C={C} A={A} chunk={chunk}")
    w = synth.small(f"fx-{st}-{C}-{A}", st, 2, C, A, seed=st + C)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
    with corr.Correlator(st, 2, C, A, "int8") as c:
        c.fengine(v, A, inv)
        c.xengine(A)
        ref = c.dump()
        sp = c.spectra().cpu().numpy()
    with corr.Correlator(st, 2, C, chunk, "int8") as c:          # holds one chunk only
        c.fx(v, A, inv, chunk)
        got = c.dump()
        assert c.counts() == (min(chunk, A - (A - 1) // chunk * chunk), 0)
    assert torch.equal(got, ref)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), oracle.xengine_i8(spectra_akp_to_apk(sp)))


def test_fx_fp32_against_float64():
    st, C, A, chunk = 24, 128, 200, 48
    say(f"fx fp32 {st}x2 C={C} A={A} chunk={chunk}")
    w = synth.small("fx-fp32", st, 2, C, A, seed=77)
    vh = synth.voltages(w)
    with corr.Correlator(st, 2, C, 64, "fp32") as c:
        c.fx(torch.from_numpy(vh).to(DEV), A, None, chunk)
        last = A - (A - 1) // chunk * chunk                       # the spectra now held
        c.xengine(last)                                           # then continue the same integration
        got = cplx(c.dump().cpu().numpy())
    S = oracle.fengine(vh, C, A)
    ref = oracle.xengine_f64(S) + oracle.xengine_f64(S[A - last:])
    eF, en = vis_errors(got, ref, 2 * st)
    assert eF.max() < 1e-5 and en.max() < 1e-5


def test_fx_rejects():
    with corr.Correlator(4, 1, 64, 128, "int8") as c:
        v = torch.zeros((4, 256 * 64), dtype=torch.complex64, device=DEV)
        inv = torch.ones(64, device=DEV)
        for bad in (0, 32, 192, 256):                             # not a time block multiple, or > n_integrate
            with pytest.raises(corr.CorrError):
                c.fx(v, 256, inv, bad)
        with pytest.raises(corr.CorrError):
            c.fx(v, 256, None, 64)                                # int8 needs a scale
