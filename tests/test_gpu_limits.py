"""The largest array the library accepts: N = 8192 inputs (4096 stations x 2
pols).  Offsets within a channel's triangle then reach N(N+1)/2 - 1 =
33,558,527, and a channel has 64 row blocks of 128 (2080 blocks of its
triangle).  Caller spectra, 40 spectra (a ragged last time block in every
precision), two whole channels against the oracle in both block sizes."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
from helpers import cplx, say, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ST, P, C, A = 4096, 2, 16, 40
N = ST * P
CHANS = [0, C - 1]


@pytest.mark.timeout(600)
def test_max_inputs_int8_bit_exact():
    g = torch.Generator(device=DEV)
    g.manual_seed(21)
    S = torch.randint(-127, 128, (A, C, N, 2), generator=g, device=DEV, dtype=torch.int8)
    q = S[:, CHANS].cpu().numpy()
    say(f"int64 oracle, N={N}, channels {CHANS}")
    ref = oracle.xengine_i8(np.ascontiguousarray(np.swapaxes(q, 1, 2)))
    del q
    for tile in (64, 128):
        with corr.Correlator(ST, P, C, A, "int8") as c:
            c.set_tile(tile)
            c.xengine(A, S)
            vis = c.dump()
            got = vis[CHANS].cpu().numpy().astype(np.int64)
            del vis
        say(f"  tile {tile}: bit-exact {np.array_equal(got, ref)}")
        assert np.array_equal(got, ref)
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_max_inputs_fp32():
    g = torch.Generator(device=DEV)
    g.manual_seed(22)
    S = torch.randn((A, C, N, 2), generator=g, device=DEV, dtype=torch.float32)
    s = S[:, CHANS].cpu().numpy().astype(np.float64)
    say(f"float64 oracle, N={N}, channels {CHANS}")
    ref = oracle.xengine_f64(np.ascontiguousarray(np.swapaxes(s[..., 0] + 1j * s[..., 1], 1, 2)))
    del s
    for tile in (64, 128):
        with corr.Correlator(ST, P, C, A, "fp32") as c:
            c.set_tile(tile)
            c.xengine(A, S)
            vis = c.dump()
            got = cplx(vis[CHANS].cpu().numpy())
            del vis
        eF, en = vis_errors(got, ref, N)
        say(f"  tile {tile}: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
        assert eF.max() < 1e-5 and en.max() < 1e-5
    torch.cuda.empty_cache()
