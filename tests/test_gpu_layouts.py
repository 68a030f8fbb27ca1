"""GPU parity on both spectra-buffer layouts.  The library picks one per
handle: time-block-major for 512 or more inputs, 2048 or more channels, or
rows narrower than 1024 bytes per channel (channels x element bytes), and
channel-major otherwise.  Every entry point that touches the held spectra
(F-engines, ingest of caller spectra, export, X-engine, fused dump, rectangle,
append, batched) is checked here on shapes from each side of that rule; the
int8 forms bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, spectra_akp_to_apk, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (N, C, A): channel-major (C >= 1024 bytes of int8 per row, N < 512, C < 2048)
# and time-block-major for each of the rule's three reasons.
INT8_SHAPES = [(40, 1024, 70), (40, 64, 70), (520, 16, 65), (20, 2048, 65)]


@pytest.mark.parametrize("N,C,A", INT8_SHAPES)
def test_caller_spectra_int8_round_trip_and_bit_exact(N, C, A):
    say(f"layout int8 caller spectra N={N} C={C} A={A}")
    S = synth.int8_spectra(A, C, N, seed=N + C + A)                # [A][C][N][2]
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.dump().cpu().numpy().astype(np.int64)
        back = c.spectra().cpu().numpy()
    assert np.array_equal(back, S)
    assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(S)))


@pytest.mark.parametrize("prec,N,C,A", [("fp32", 24, 256, 40), ("fp16", 24, 512, 70), ("fp8", 24, 1024, 70),
                                        ("fp32", 24, 64, 40), ("fp16", 520, 16, 70)])
def test_caller_spectra_float_forms(prec, N, C, A):
    """Exactly representable spectra: only the FP32 accumulation differs from
    the float64 oracle."""
    say(f"layout {prec} caller spectra N={N} C={C} A={A}")
    q = synth.int8_spectra(A, C, N, seed=N * 3 + C, rms=3.0).astype(np.float64)
    if prec == "fp8":
        q = np.clip(q, -8, 8)
    t = torch.from_numpy(q).to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]]).to(DEV)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.xengine(A, t)
        got = cplx(c.dump().cpu().numpy())
        back = c.spectra().cpu().to(torch.float64).numpy()
    assert np.array_equal(back, q)
    ref = oracle.xengine_f64(spectra_akp_to_apk(cplx(q)))
    eF, en = vis_errors(got, ref, N)
    say(f"  max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-6 and en.max() < 1e-6


@pytest.mark.parametrize("N,C,A", [(24, 1024, 150), (24, 64, 150)])
def test_fengine_held_spectra_feed_xengine_and_fused_dump(N, C, A):
    """F-engine writes and X-engine reads agree on the layout: the X-engine
    over held spectra, and the fused dump, equal the oracle on the exported
    spectra, bit for bit."""
    say(f"layout int8 F->X N={N} C={C} A={A}")
    w = synth.small("lay", N, 1, C, A, seed=70 + C)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.fengine(v, A, inv)
        c.xengine(A - 40)                                          # a prefix, ragged in its last block
        first = c.dump(reset=True).cpu().numpy().astype(np.int64)
        fused = c.xengine_dump(A).cpu().numpy().astype(np.int64)
        sp = c.spectra().cpu().numpy()
    S = spectra_akp_to_apk(sp)
    assert np.array_equal(first, oracle.xengine_i8(S[: A - 40]))
    assert np.array_equal(fused, oracle.xengine_i8(S))


def test_rect_channel_major_int8():
    N, C, A = 40, 1024, 70
    say(f"layout rect int8 N={N} C={C} A={A}")
    S = synth.int8_spectra(A, C, N, seed=77)
    ref = oracle.xengine_i8(spectra_akp_to_apk(S))                 # [C][B][2]
    i0, ni, j0, nj = 25, 15, 0, 20
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.xengine_rect(i0, ni, j0, nj, A).cpu().numpy().astype(np.int64)
    ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj), indexing="ij")
    assert np.array_equal(got, ref[:, ii * (ii + 1) // 2 + jj])


@pytest.mark.parametrize("prec,C", [("fp16", 512), ("int8", 1024)])
def test_append_pieces_channel_major(prec, C):
    N, A = 8, 150
    tb = {"fp16": 32, "int8": 64}[prec]
    say(f"layout append {prec} N={N} C={C} A={A}")
    w = synth.small("lay-ap", N, 1, C, A, seed=80 + C)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, prec)).to(DEV)
    with corr.Correlator(N, 1, C, A, prec) as whole, corr.Correlator(N, 1, C, A, prec) as parts:
        whole.fengine(v, A, inv)
        whole.xengine(A)
        first = 0
        for n in (tb, tb, A - 2 * tb):
            parts.fengine(v[:, first * C:(first + n) * C].contiguous(), n, inv, first_spectrum=first)
            first += n
        parts.xengine(A)
        assert torch.equal(whole.spectra(), parts.spectra())
        assert torch.equal(whole.dump(), parts.dump())


def test_real_input_channel_major_int8():
    N, C, A = 4, 1024, 70
    say(f"layout real8 int8 N={N} C={C} A={A}")
    rw = synth.small_real("lay-r8", N, C, A, seed=93)
    x = torch.from_numpy(synth.real8_samples(rw)).to(DEV)
    inv = torch.from_numpy(synth.real8_inv_scale(rw, "int8")).to(DEV)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.fengine_real8(x, A, inv)
        c.xengine(A)
        got = c.dump().cpu().numpy().astype(np.int64)
        sp = c.spectra().cpu().numpy()
    assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(sp)))


def test_batched_mixes_layouts():
    """Sub-arrays on different layouts in one persistent launch."""
    shapes = [(20, 1, 1024, 70), (20, 1, 64, 70), (5, 2, 16, 40), (10, 1, 2048, 65)]
    say("layout batched int8 mixed layouts")
    with corr.Batch(shapes, "int8") as b:
        for r, (ns, npol, C, A) in enumerate(shapes):
            w = synth.small(f"lay-b{r}", ns, npol, C, A, seed=100 + r)
            b.subs[r].fengine(torch.from_numpy(synth.voltages(w)).to(DEV), A,
                              torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV))
        b.xengine([A for (_, _, _, A) in shapes])
        for r, sub in enumerate(b.subs):
            got = sub.dump().cpu().numpy().astype(np.int64)
            sp = sub.spectra().cpu().numpy()
            assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(sp))), r
