"""The rectangle X-engine (corr_xengine_rect): one group of inputs against a
disjoint other group, the node product of the paper's space-division models
(Section 4).  Checked against the oracle's triangle (lower rectangles are
triangle entries, upper ones their conjugates), against the full-triangle
X-engine on the same spectra (triangle = diagonal triangles + rectangles), in
both block sizes, with ragged ranges and a ragged last time block."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
from helpers import cplx, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _int8_spectra(A, C, N, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return torch.randint(-127, 128, (A, C, N, 2), generator=g, device=DEV, dtype=torch.int8)


def _tri(i, j):
    return i * (i + 1) // 2 + j


@pytest.mark.parametrize("tile", [64, 128])
def test_rect_int8_bit_exact(tile):
    N, C, A = 200, 16, 70
    S = _int8_spectra(A, C, N, seed=31)
    ref = oracle.xengine_i8(np.ascontiguousarray(np.swapaxes(S.cpu().numpy(), 1, 2)))   # [C][B][2]
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.set_tile(tile)
        c.xengine(A, S)
        for (i0, ni, j0, nj) in ((130, 70, 3, 97), (0, 50, 60, 130), (199, 1, 0, 199), (5, 1, 6, 1)):
            got = c.xengine_rect(i0, ni, j0, nj, A).cpu().numpy().astype(np.int64)   # [C][ni][nj][2]
            ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj), indexing="ij")
            if i0 > j0:
                want = ref[:, _tri(ii, jj)]
            else:                                     # upper rectangle: conjugate of (j, i)
                want = ref[:, _tri(jj, ii)] * np.array([1, -1])
            say(f"  tile {tile} rows {i0}+{ni} cols {j0}+{nj}: equal {np.array_equal(got, want)}")
            assert np.array_equal(got, want)


def test_rect_fp32_union_equals_triangle_and_oracle():
    N, C, A, a = 160, 32, 33, 70
    g = torch.Generator(device=DEV)
    g.manual_seed(32)
    S = torch.randn((A, C, N, 2), generator=g, device=DEV, dtype=torch.float32)
    s = S.cpu().numpy().astype(np.float64)
    ref = oracle.xengine_f64(np.ascontiguousarray(np.swapaxes(s[..., 0] + 1j * s[..., 1], 1, 2)))
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.xengine(A, S)
        tri = cplx(c.dump().cpu().numpy())                                  # [C][B]
        got = cplx(c.xengine_rect(a, N - a, 0, a, A).cpu().numpy())         # [C][N-a][a]
    ii, jj = np.meshgrid(np.arange(a, N), np.arange(0, a), indexing="ij")
    part = tri[:, _tri(ii, jj)]
    d_tri = np.abs(got - part).max() / np.abs(part).max()
    want = ref[:, _tri(ii, jj)]
    rel = np.linalg.norm((got - want).reshape(C, -1), axis=1) / np.linalg.norm(want.reshape(C, -1), axis=1)
    say(f"  rect vs triangle kernel: max rel {d_tri:.1e}; vs float64 oracle: max e_F {rel.max():.1e}")
    assert d_tri < 1e-6
    assert rel.max() < 1e-5


def test_rect_accumulate_and_int8_valued_fp16():
    N, C, A = 96, 16, 40
    S8 = _int8_spectra(A, C, N, seed=33) // 8                              # |x| <= 16: exact in FP16 sums
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, S8)
        one = c.xengine_rect(40, 56, 0, 40, A)
        two = c.xengine_rect(40, 56, 0, 40, A)
        c.xengine_rect(40, 56, 0, 40, A, out=two, accumulate=True)
        assert torch.equal(two, 2 * one)
    with corr.Correlator(N, 1, C, A, "fp16") as c:
        c.xengine(A, S8.to(torch.float16))
        h = c.xengine_rect(40, 56, 0, 40, A)
    assert torch.equal(h.to(torch.int32), one)


def test_rect_errors():
    with corr.Correlator(8, 1, 16, 8, "fp32") as c:
        with pytest.raises(corr.CorrError) as ei:
            c.xengine_rect(4, 4, 0, 4, 8)                                   # nothing held yet
        assert ei.value.status == corr.CORR_E_STATE
        c.xengine(8, torch.zeros((8, 16, 8, 2), dtype=torch.float32, device=DEV))
        for args, st in (((2, 4, 0, 4, 8), corr.CORR_E_INVALID_ARG),        # overlap
                         ((4, 5, 0, 4, 8), corr.CORR_E_INVALID_ARG),        # rows past N
                         ((4, 0, 0, 4, 8), corr.CORR_E_INVALID_ARG),        # empty
                         ((4, 4, 0, 4, 9), corr.CORR_E_STATE)):             # more spectra than held
            with pytest.raises(corr.CorrError) as ei:
                c.xengine_rect(*args)
            assert ei.value.status == st
