"""Spectra order and the F + X autotuner.  Results may not depend on either:
the held spectra of both orders are identical element for element, the
int8 integration is bit for bit the same and equal to the integer oracle
(Eq. 2) on those spectra, the FP32 one stays within the float64 oracle's
bound (Eq. 1 then Eq. 2) -- under both orders forced, both block sizes, and
whatever configuration corr_autotune_fx picks (also when it comes from the
cache)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, spectra_akp_to_apk, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("st,C,A", [(20, 64, 300), (33, 2048, 130), (9, 256, 64)])
def test_int8_both_orders_and_tiles_are_exact(st, C, A):
    say(f"orders int8 {st}x2 C={C} A={A}")
    w = synth.small(f"order-{st}-{C}-{A}", st, 2, C, A, seed=3 * st + C)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
    vis, spec = [], []
    for order in (0, 1):
        for tile in (64, 128):
            with corr.Correlator(st, 2, C, A, "int8") as c:
                c.set_spectra_layout(order)
                c.set_tile(tile)
                c.fengine(v, A, inv)
                c.xengine(A)
                vis.append(c.dump())
                spec.append(c.spectra())
    for x in vis[1:]:
        assert torch.equal(x, vis[0])
    for s in spec[1:]:
        assert torch.equal(s, spec[0])
    ref = oracle.xengine_i8(spectra_akp_to_apk(spec[0].cpu().numpy()))
    assert np.array_equal(vis[0].cpu().numpy().astype(np.int64), ref)


def test_layout_switch_drops_held_spectra():
    with corr.Correlator(8, 2, 64, 64, "fp16") as c:
        v = torch.zeros((16, 64 * 64), dtype=torch.complex64, device=DEV)
        c.set_spectra_layout(0)
        c.fengine(v, 64)
        assert c.counts()[0] == 64
        c.set_spectra_layout(0)                                   # the order it already has: kept
        assert c.counts()[0] == 64
        c.set_spectra_layout(1)
        assert c.counts()[0] == 0
        with pytest.raises(corr.CorrError):
            c.xengine(64)
        with pytest.raises(corr.CorrError):
            c.set_spectra_layout(2)


@pytest.mark.parametrize("st,C,A", [(20, 64, 300), (33, 2048, 130)])
def test_autotuned_int8_matches_default(st, C, A):
    say(f"autotune_fx int8 {st}x2 C={C} A={A}")
    w = synth.small(f"tune-{st}-{C}-{A}", st, 2, C, A, seed=st * C + 1)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
    with corr.Correlator(st, 2, C, A, "int8") as c:
        c.fengine(v, A, inv)
        c.xengine(A)
        ref = c.dump()
        ref_spec = c.spectra()
    for attempt in range(2):                                      # measured, then from the cache
        with corr.Correlator(st, 2, C, A, "int8") as c:
            t = c.autotune_fx(v, A, inv)
            assert t["tile"] in (64, 128) and t["time_block_major"] in (0, 1)
            if attempt == 0:
                assert 0 < t["ms_tuned"] <= t["ms_default"]
            else:
                assert t["ms_tuned"] == -1.0 and t["ms_default"] == -1.0
                assert (t["tile"], t["time_block_major"]) == first
            first = (t["tile"], t["time_block_major"])
            assert c.counts() == (A, 0)                           # holds the spectra, nothing integrated
            assert torch.equal(c.spectra(), ref_spec)
            c.xengine(A)
            got = c.dump()
        assert torch.equal(got, ref)
    assert np.array_equal(got.cpu().numpy().astype(np.int64),
                          oracle.xengine_i8(spectra_akp_to_apk(ref_spec.cpu().numpy())))


def test_autotuned_fp32_against_float64():
    st, C, A = 24, 128, 200
    say(f"autotune_fx fp32 {st}x2 C={C} A={A}")
    w = synth.small("tune-fp32", st, 2, C, A, seed=91)
    vh = synth.voltages(w)
    with corr.Correlator(st, 2, C, A, "fp32") as c:
        t = c.autotune_fx(torch.from_numpy(vh).to(DEV), A)
        say(f"  chose tile {t['tile']} order {t['time_block_major']}")
        c.xengine(A)
        got = cplx(c.dump().cpu().numpy())
    ref = oracle.xengine_f64(oracle.fengine(vh, C, A))
    eF, en = vis_errors(got, ref, 2 * st)
    assert eF.max() < 1e-5 and en.max() < 1e-5


def test_autotune_fx_rejects():
    with corr.Correlator(4, 1, 64, 128, "int8") as c:
        v = torch.zeros((4, 256 * 64), dtype=torch.complex64, device=DEV)
        inv = torch.ones(64, device=DEV)
        for bad in (0, 129):                                      # empty, more than n_integrate
            with pytest.raises(corr.CorrError):
                c.autotune_fx(v, bad, inv)
        with pytest.raises(corr.CorrError):
            c.autotune_fx(v, 64, None)                            # int8 needs a scale


@pytest.mark.parametrize("order", [0, 1])
def test_forced_order_caller_spectra_rect_and_append_int8(order):
    """Every path that touches the held spectra under a forced order: caller
    spectra in and out, the triangle and the rectangle, and an integration
    appended in two F-engine pieces, bit-exact against the integer oracle."""
    N, C, A = 40, 256, 130
    say(f"forced order {order}: int8 N={N} C={C} A={A}")
    S = synth.int8_spectra(A, C, N, seed=order + 17)                  # [A][C][N][2]
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.set_spectra_layout(order)
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.dump().cpu().numpy().astype(np.int64)
        assert np.array_equal(c.spectra().cpu().numpy(), S)
        rect = c.xengine_rect(24, 16, 0, 24, A).cpu().numpy().astype(np.int64)     # rows 24..39 x columns 0..23
    Sc = spectra_akp_to_apk(S).astype(np.int64)                        # [A][N][C][2]
    assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(S)))
    x = Sc[..., 0] + 1j * Sc[..., 1]                                   # [A][N][C]
    ref_rect = np.einsum("aik,ajk->kij", np.conj(x[:, 24:40]), x[:, 0:24])
    assert np.array_equal(rect[..., 0], ref_rect.real.astype(np.int64))
    assert np.array_equal(rect[..., 1], ref_rect.imag.astype(np.int64))
    w = synth.small(f"order-append-{order}", 20, 2, C, A, seed=order + 5)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
    with corr.Correlator(20, 2, C, 128, "int8") as c:
        c.set_spectra_layout(order)
        c.fengine(v, 64, inv)                                          # spectra 0..63
        c.fengine(v[:, 64 * C:], 64, inv, ld_samples=v.shape[1], first_spectrum=64)   # 64..127
        c.xengine(128)
        got = c.dump().cpu().numpy().astype(np.int64)
        sp = c.spectra().cpu().numpy()
    assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(sp)))
