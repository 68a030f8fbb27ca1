"""GPU parity of the block-size variants, the autotuner and the batched
persistent X-engine (one launch over uneven sub-arrays), including replay of
a captured HIP graph."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, spectra_akp_to_apk, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("N,C,A", [(1, 16, 5), (33, 16, 65), (64, 32, 64), (100, 16, 130), (130, 16, 70),
                                   (200, 16, 33)])
def test_tile_sizes_int8_bit_exact(tile, N, C, A):
    say(f"tile {tile} int8 N={N} C={C} A={A}")
    S = synth.int8_spectra(A, C, N, seed=N + tile + A)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.set_tile(tile)
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.dump().cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(S)))


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp8"])
def test_tile64_float_forms(prec):
    N, C, A = 70, 16, 96
    say(f"tile 64 {prec}")
    q = np.clip(synth.int8_spectra(A, C, N, seed=3, rms=3.0), -8, 8).astype(np.float64)
    t = torch.from_numpy(q).to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]]).to(DEV)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.set_tile(64)
        c.xengine(A, t)
        got = cplx(c.dump().cpu().numpy())
    ref = oracle.xengine_f64(spectra_akp_to_apk(cplx(q)))
    eF, en = vis_errors(got, ref, N)
    assert eF.max() < 1e-6 and en.max() < 1e-6


def test_autotune_picks_a_tile_and_keeps_parity():
    N, C, A = 90, 32, 64
    say("autotune")
    S = synth.int8_spectra(A, C, N, seed=17)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))          # holds the spectra (and integrates once)
        tile = c.autotune(A)
        assert tile in (64, 128)
        assert c.autotune(A) == tile                        # cached
        c.xengine(A)                                         # second integration with the tuned tile
        got = c.dump().cpu().numpy().astype(np.int64)
    assert np.array_equal(got, 2 * oracle.xengine_i8(spectra_akp_to_apk(S)))


SHAPES = [(1, 2, 16, 40), (16, 2, 32, 100), (35, 2, 16, 64), (65, 2, 16, 70), (100, 1, 64, 33), (150, 2, 16, 50)]


def _batch_inputs(prec, shapes, seed=0):
    vs, invs = [], []
    for r, (ns, npol, C, A) in enumerate(shapes):
        w = synth.small(f"b{r}", ns, npol, C, A, seed=seed + r)
        vs.append(synth.voltages(w))
        invs.append(synth.inv_scale(w, prec))
    return vs, invs


@pytest.mark.parametrize("tiles", ["auto", "mixed"])
def test_batched_int8_bit_exact(tiles):
    say(f"batched int8 {tiles}")
    vs, invs = _batch_inputs("int8", SHAPES)
    with corr.Batch(SHAPES, "int8") as b:
        for i, sub in enumerate(b.subs):
            if tiles == "mixed":
                sub.set_tile(64 if i % 2 else 128)
            sub.fengine(torch.from_numpy(vs[i]).to(DEV), SHAPES[i][3], torch.from_numpy(invs[i]).to(DEV))
        n = [A for (_, _, _, A) in SHAPES]
        n[2] = 0                                             # sub-array 2 skipped this call
        n[4] = 17                                            # a prefix of the held spectra
        b.xengine(n)
        for i, sub in enumerate(b.subs):
            sp = sub.spectra().cpu().numpy()
            got = sub.dump().cpu().numpy().astype(np.int64)
            if n[i] == 0:
                assert not got.any()
                continue
            ref = oracle.xengine_i8(spectra_akp_to_apk(sp[: n[i]]))
            assert np.array_equal(got, ref), i


def test_batched_matches_standalone_fp16_and_resumes():
    say("batched fp16 vs standalone")
    vs, invs = _batch_inputs("fp16", SHAPES, seed=10)
    n = [A for (_, _, _, A) in SHAPES]
    with corr.Batch(SHAPES, "fp16") as b:
        for i, sub in enumerate(b.subs):
            sub.fengine(torch.from_numpy(vs[i]).to(DEV), n[i], torch.from_numpy(invs[i]).to(DEV))
        b.xengine(n)
        b.xengine(n)                                         # integrates twice
        got = [sub.dump(reset=True).cpu().numpy() for sub in b.subs]
        b.xengine(n)                                         # after the reset: once
        once = [sub.dump(reset=True).cpu().numpy() for sub in b.subs]
    for i, (ns, npol, C, A) in enumerate(SHAPES):
        with corr.Correlator(ns, npol, C, A, "fp16") as c:
            c.fengine(torch.from_numpy(vs[i]).to(DEV), A, torch.from_numpy(invs[i]).to(DEV))
            c.xengine(A)
            ref = cplx(c.dump().cpu().numpy())
        N = ns * npol
        eF, en = vis_errors(cplx(got[i]), 2 * ref, N)
        assert eF.max() < 1e-6 and en.max() < 1e-6, i
        eF, en = vis_errors(cplx(once[i]), ref, N)
        assert eF.max() < 1e-6 and en.max() < 1e-6, i


def test_batched_graph_replay_matches_eager():
    """F-engines and the persistent X-engine captured in one graph; every replay
    (with eager dumps and synchronisations between) equals the eager result."""
    say("batched graph replay")
    shapes = SHAPES[:4]
    vs, invs = _batch_inputs("int8", shapes, seed=20)
    stream = torch.cuda.Stream()
    n = [A for (_, _, _, A) in shapes]
    with torch.cuda.stream(stream):
        vd = [torch.from_numpy(v).to(DEV) for v in vs]
        idd = [torch.from_numpy(x).to(DEV) for x in invs]
        b = corr.Batch(shapes, "int8", stream=stream)
        for i, sub in enumerate(b.subs):
            sub.fengine(vd[i], n[i], idd[i])
        b.xengine(n)                                         # eager reference (also fixes the work list)
        ref = [sub.dump(reset=True).cpu().numpy() for sub in b.subs]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for i, sub in enumerate(b.subs):
                sub.fengine(vd[i], n[i], idd[i])
            b.xengine(n)
        for rep in range(3):
            g.replay()
            stream.synchronize()
            got = [sub.dump(reset=True).cpu().numpy() for sub in b.subs]
            for i in range(len(shapes)):
                assert np.array_equal(got[i], ref[i]), (rep, i)
            torch.zeros(1000, device=DEV).sum().item()       # unrelated eager work between replays
        b.close()


def test_batched_direct_and_persistent_mix_int8():
    """A sub-array large enough to fill the GPU on its own (256 inputs x 1024
    channels: 3072 blocks of 128 inputs) runs as its own launch inside
    corr_xengine_batched, the small ones in the persistent launch; both
    integrate across calls (the zero flag of each is consumed once), bit-exact
    against the integer oracle, eagerly and replayed from a graph."""
    shapes = [(128, 2, 1024, 64)] + SHAPES[:3]
    say(f"batched direct + persistent int8 {shapes}")
    vs, invs = _batch_inputs("int8", shapes, seed=30)
    n = [A for (_, _, _, A) in shapes]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        vd = [torch.from_numpy(v).to(DEV) for v in vs]
        idd = [torch.from_numpy(x).to(DEV) for x in invs]
        b = corr.Batch(shapes, "int8", stream=stream)
        for i, sub in enumerate(b.subs):
            sub.fengine(vd[i], n[i], idd[i])
        b.xengine(n)
        b.xengine(n)                                         # integrates twice
        got = [sub.dump(reset=True).cpu().numpy().astype(np.int64) for sub in b.subs]
        sp = [sub.spectra().cpu().numpy() for sub in b.subs]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            b.xengine(n)
        for rep in range(2):
            g.replay()
            stream.synchronize()
            once = [sub.dump(reset=True).cpu().numpy().astype(np.int64) for sub in b.subs]
            for i in range(len(shapes)):
                assert np.array_equal(2 * once[i], got[i]), (rep, i)
        b.close()
    for i, (ns, npol, C, A) in enumerate(shapes):
        chans = sorted({0, 1, C // 2, C - 1})
        ref = oracle.xengine_i8(spectra_akp_to_apk(sp[i][:, chans]))
        assert np.array_equal(got[i][chans], 2 * ref), i


def test_batched_real_input_sub_arrays_int8_exact():
    """Sub-arrays fed by the real-input F-engine (8-bit real samples): the
    batched X-engine is exact against the integer oracle on each sub-array's
    spectra, and those spectra are the requantised float64 DFT of length 2C."""
    shapes = [(24, 1, 128, 130), (7, 1, 64, 64), (70, 1, 256, 40)]
    say("batched int8 on real-input sub-arrays")
    with corr.Batch(shapes, "int8") as b:
        xs, invs = [], []
        for i, (st, _, C, A) in enumerate(shapes):
            rw = synth.small_real(f"b-r8-{i}", st, C, A, seed=80 + i)
            xs.append(synth.real8_samples(rw))
            invs.append(synth.real8_inv_scale(rw, "int8"))
            b.subs[i].fengine_real8(torch.from_numpy(xs[i]).to(DEV), A, torch.from_numpy(invs[i]).to(DEV))
        b.xengine([A for (_, _, _, A) in shapes])
        for i, (st, _, C, A) in enumerate(shapes):
            sp = b.subs[i].spectra().cpu().numpy()
            got = b.subs[i].dump().cpu().numpy().astype(np.int64)
            assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(sp))), i
            y = oracle.fengine_real8(xs[i], C, A) * invs[i].astype(np.float64)[None, None, :]
            q = spectra_akp_to_apk(sp).astype(np.float64)
            assert max(np.max(np.abs(q[..., 0] - y.real)), np.max(np.abs(q[..., 1] - y.imag))) <= 0.5 + 1e-3, i


def _seed5_picks():
    """Four sub-arrays of the 64-sub-array seed-5 draw: the fewest inputs, the
    most inputs and two seeded others."""
    ws = synth.batched_workloads()
    by_n = sorted(range(len(ws)), key=lambda r: (ws[r].n_inputs, r))
    lo, hi = by_n[0], by_n[-1]
    rest = [r for r in range(len(ws)) if r not in (lo, hi)]
    picks = [lo, hi] + [int(x) for x in np.random.default_rng(55).choice(rest, size=2, replace=False)]
    return [ws[r] for r in picks]


@pytest.mark.timeout(600)
def test_batched_fp16_seed5_subarrays_vs_oracle():
    """The batched persistent X-engine in FP16 (FP32 accumulation) on four
    sub-arrays of the seed-5 uneven draw at their full shapes, F-engine
    included, against the oracle on sampled channels: the X-engine on the
    identical FP16 spectra (Eq. 2 in float64), and the whole F + X chain
    against the float64 DFT (Eq. 1) and Eq. 2."""
    ws = _seed5_picks()
    shapes = [(w.n_stations, w.n_pols, w.n_channels, w.n_integrate) for w in ws]
    say(f"batched fp16 seed-5 sub-arrays {shapes}")
    vs, invs = [], []
    with corr.Batch(shapes, "fp16") as b:
        for i, w in enumerate(ws):
            vs.append(synth.voltages(w, device=DEV))
            invs.append(synth.inv_scale(w, "fp16"))
            b.subs[i].fengine(vs[i], w.n_integrate, torch.from_numpy(invs[i]).to(DEV))
        b.xengine([w.n_integrate for w in ws])
        for i, w in enumerate(ws):
            N, C, A = w.n_inputs, w.n_channels, w.n_integrate
            chans = sorted({0, C // 2, C - 1, *w.tone_bins,
                            *[int(x) for x in np.random.default_rng(100 + i).choice(C, size=2, replace=False)]})
            got = cplx(b.subs[i].dump()[chans].cpu().numpy())
            sp = b.subs[i].spectra()                                   # [A][C][N][2] binary16
            q = sp[:, chans].to(torch.float64).cpu().numpy()
            del sp
            s2 = 1.0 / invs[i][chans].astype(np.float64) ** 2
            ref_q = oracle.xengine_f64(spectra_akp_to_apk(cplx(q))) * s2[:, None]
            eF, en = vis_errors(got, ref_q, N)
            say(f"  sub-array {i} ({N} inputs, {C} ch, {A} spectra) vs identical FP16 spectra: "
                f"max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
            assert eF.max() < 1e-5 and en.max() < 1e-5, i
            ref64 = oracle.xengine_f64(oracle.fengine(vs[i].cpu().numpy(), C, A, chans))
            eF, en = vis_errors(got, ref64, N)
            say(f"  sub-array {i} vs float64 F + X: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
            assert en.max() < 1e-3, i
            vs[i] = None
            torch.cuda.empty_cache()


def test_batch_member_per_array_calls_and_resets():
    """Per-array X-engine calls on batch sub-arrays follow the same device
    "zero since reset" flag as the batched launch: a reset makes the next call
    write, further calls add, and a dump before any call reads zeros."""
    say("batch member per-array calls and resets")
    shapes = SHAPES[:3]
    vs, invs = _batch_inputs("int8", shapes, seed=30)
    n = [A for (_, _, _, A) in shapes]
    with corr.Batch(shapes, "int8") as b:
        for i, sub in enumerate(b.subs):
            assert not sub.dump(reset=False).cpu().numpy().any()          # logically zero at creation
            sub.fengine(torch.from_numpy(vs[i]).to(DEV), n[i], torch.from_numpy(invs[i]).to(DEV))
        refs = [oracle.xengine_i8(spectra_akp_to_apk(sub.spectra().cpu().numpy())) for sub in b.subs]
        for i, sub in enumerate(b.subs):
            sub.xengine(n[i])
            sub.xengine(n[i])
        b.xengine(n)                                                     # three integrations in all
        for i, sub in enumerate(b.subs):
            assert np.array_equal(sub.dump(reset=True).cpu().numpy().astype(np.int64), 3 * refs[i]), i
            assert not sub.dump(reset=False).cpu().numpy().any(), i      # reset: zeros until the next call
            host = np.empty(sub.visibility_shape(), dtype=np.int32)
            sub.dump(host, reset=False)
            assert not host.any(), i
        b.xengine(n)
        for i, sub in enumerate(b.subs):
            sub.xengine(n[i])
            assert np.array_equal(sub.dump(reset=True).cpu().numpy().astype(np.int64), 2 * refs[i]), i
