"""Caller int8 spectra that hold -128, a valid int8 value outside the
symmetric range [-127, 127] the X-engine's exact negation and int32 bound
rely on: the library reads it as -127 (the requantiser's own clamp), and the
result is bit-exact against the integer oracle (Eq. 2) on the clamped
spectra."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
from helpers import say, spectra_akp_to_apk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _spectra_with_min(A, C, N, seed):
    rng = np.random.default_rng(seed)
    S = rng.integers(-128, 128, size=(A, C, N, 2), dtype=np.int16).astype(np.int8)
    # -128 in each plane on its own, in both planes at once, and on a whole input
    S[0, 0, 0, 0] = -128
    S[1, 0, 1, 1] = -128
    S[2, 1, 2, :] = -128
    S[:, :, N - 1, :] = -128
    return S


@pytest.mark.parametrize("N,C,A", [(7, 16, 70), (150, 16, 130), (64, 32, 64)])
def test_caller_int8_minus128_reads_as_minus127(N, C, A):
    say(f"int8 caller spectra with -128: N={N} C={C} A={A}")
    S = _spectra_with_min(A, C, N, seed=N + A)
    assert (S == -128).any()
    clamped = np.maximum(S, -127).astype(np.int8)
    ref = oracle.xengine_i8(spectra_akp_to_apk(clamped))
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))
        held = c.spectra().cpu().numpy()
        got = c.dump().cpu().numpy().astype(np.int64)
        # the fused dump path ingests the same way
        out = c.new_visibilities()
        c.xengine_dump(A, out, spectra=torch.from_numpy(S).to(DEV))
        fused = out.cpu().numpy().astype(np.int64)
    assert np.array_equal(held, clamped)
    assert np.array_equal(got, ref)
    assert np.array_equal(fused, ref)


def test_caller_int8_minus128_worst_case_autos():
    """Every value -128: each auto product reads 2 * 127^2 per spectrum, the
    bound CORR_INT8_MAX_INTEGRATE is derived from."""
    N, C, A = 3, 16, 64
    say("int8 caller spectra all -128")
    S = np.full((A, C, N, 2), -128, dtype=np.int8)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.dump().cpu().numpy().astype(np.int64)
    assert (got[..., 0] == 2 * 127 * 127 * A).all()
    assert (got[..., 1] == 0).all()
