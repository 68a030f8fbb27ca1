"""GPU parity of the chunked F-engine used from 2048 channels on: chunks of
time blocks (all inputs) or of one time block and a range of inputs go
through a bounded scratch buffer in the workgroups' natural order and are
gathered into the held rows.  Shapes here make several chunks of each kind;
the oracle evaluates sampled channels of sampled inputs one by one, the
X-engine is checked bit for bit on sampled channels, and appended pieces must
equal one call."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, fft_error_bound, say, spectra_akp_to_apk, tie_mismatches, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _chans(C, seed, n=12):
    rng = np.random.default_rng(seed)
    return sorted({0, 1, C // 2, C - 1, *[int(x) for x in rng.choice(C, n, replace=False)]})


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,N,C,A", [
    ("int8", 300, 8192, 70),      # 1 MB per (input, time block): chunks of 256 inputs, 2 x 2 chunks
    ("fp8", 300, 8192, 70),
    ("fp32", 600, 2048, 40),      # 150 MB per time block: one time block per chunk, 3 chunks
    ("fp16", 520, 4096, 70),      # 266 MB per time block: 2 x 3 chunks over inputs
])
def test_chunked_fengine_sampled_parity(prec, N, C, A):
    say(f"chunked F-engine {prec} N={N} C={C} A={A}")
    w = synth.small("fg", N, 1, C, A, seed=C + N)
    v = synth.voltages(w, device=DEV)
    inv_np = synth.inv_scale(w, prec)
    inv = torch.from_numpy(inv_np).to(DEV) if prec != "fp32" else None
    ins = sorted({0, 1, 255, 256, N // 2, N - 2, N - 1})
    chans = _chans(C, seed=N)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine(v, A, inv)
        c.xengine(A)
        vis = c.dump()                                              # [C][B][2]
        sp = c.spectra()                                            # [A][C][N][2]
        sub = sp[:, chans][:, :, ins].cpu()
        vis_s = vis[chans].cpu().numpy()
        spc = sp[:, chans].cpu()                                    # all inputs of the sampled channels
    del sp, vis
    vh = v[ins].cpu().numpy()
    del v
    torch.cuda.empty_cache()
    S = oracle.fengine(vh, C, A, chans)                             # [A][n_ins][n_ch]
    if prec == "fp32":
        got = cplx(sub.numpy())                                     # [A][n_ch][n_ins]
        ref = np.swapaxes(S, 1, 2)
        rms = np.sqrt(np.mean(np.abs(ref) ** 2))
        err = np.max(np.abs(got - ref)) / rms
        say(f"  sampled spectra: max |err| / rms = {err:.2e}")
        assert err < 1e-5
    else:
        q_gpu = sub.numpy().astype(np.float64) if prec == "int8" else sub.to(torch.float64).numpy()
        inv_c = inv_np[chans].astype(np.float64)
        q_ref = np.swapaxes(oracle.quantise(S, inv_np[chans], prec).astype(np.float64), 1, 2)
        y = np.swapaxes(S, 1, 2) * inv_c[None, :, None]
        y_pair = np.stack([y.real, y.imag], -1)
        rms_y = np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 2)))
        eps = fft_error_bound(C, rms_y)[None, :, None, None] + 1e-30
        n_mis, n_bad = tie_mismatches(q_gpu, q_ref, y_pair, eps)
        say(f"  sampled codes: mismatches {n_mis} of {q_ref.size}, unexplained {n_bad}")
        assert n_bad == 0
        assert n_mis <= max(2, q_ref.size // 100)
    # the X-engine over the held spectra, on the sampled channels
    if prec == "int8":
        ref_v = oracle.xengine_i8(spectra_akp_to_apk(spc.numpy()))
        assert np.array_equal(vis_s.astype(np.int64), ref_v)
    else:
        x = spc.to(torch.float64).numpy() if prec != "fp32" else spc.numpy().astype(np.float64)
        ref_v = oracle.xengine_f64(spectra_akp_to_apk(cplx(x)))
        s2 = 1.0 / inv_np[chans].astype(np.float64) ** 2 if prec != "fp32" else np.ones(len(chans))
        eF, en = vis_errors(cplx(vis_s), ref_v * s2[:, None], N)
        say(f"  sampled visibilities: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
        # FP8 MFMA sums its products at less than FP32 precision (the same
        # bar as the full-size FP8 test); FP16 and FP32 keep FP32 sums.
        tol = 1e-4 if prec == "fp8" else 1e-5
        assert eF.max() < tol and en.max() < tol


@pytest.mark.parametrize("prec,C", [("int8", 2048), ("fp16", 4096)])
def test_chunked_append_pieces_equal_one_call(prec, C):
    N, A = 40, 200
    tb = {"fp16": 32, "int8": 64}[prec]
    say(f"chunked append {prec} N={N} C={C} A={A}")
    w = synth.small("fg-ap", N, 1, C, A, seed=C + 3)
    v = synth.voltages(w, device=DEV)
    inv = torch.from_numpy(synth.inv_scale(w, prec)).to(DEV)
    with corr.Correlator(N, 1, C, A, prec) as whole, corr.Correlator(N, 1, C, A, prec) as parts:
        whole.fengine(v, A, inv)
        first = 0
        for n in (tb, 2 * tb, A - 3 * tb):
            parts.fengine(v[:, first * C:(first + n) * C].contiguous(), n, inv, first_spectrum=first)
            first += n
        assert torch.equal(whole.spectra(), parts.spectra())


@pytest.mark.parametrize("prec", ["int8", "fp32"])
def test_chunked_real_input_sampled(prec):
    """8-bit real samples at transform length 4096 (2048 channels)."""
    N, C, A = 6, 2048, 70
    say(f"chunked real8 {prec} N={N} C={C} A={A}")
    rw = synth.small_real("fg-r8", N, C, A, seed=94)
    x = synth.real8_samples(rw)
    inv_np = synth.real8_inv_scale(rw, prec)
    inv = torch.from_numpy(inv_np).to(DEV) if prec == "int8" else None
    chans = _chans(C, seed=5)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A, inv)
        sp = c.spectra().cpu()[:, chans]                           # [A][n_ch][N][2]
    S = oracle.fengine_real8(x, C, A, chans)                        # [A][N][n_ch]
    if prec == "fp32":
        got = cplx(sp.numpy())
        ref = np.swapaxes(S, 1, 2)
        err = np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
        say(f"  max |err| / rms = {err:.2e}")
        assert err < 1e-5
    else:
        y = np.swapaxes(S, 1, 2) * inv_np[chans].astype(np.float64)[None, :, None]
        q_ref = np.swapaxes(oracle.quantise(S, inv_np[chans], "int8").astype(np.float64), 1, 2)
        y_pair = np.stack([y.real, y.imag], -1)
        eps = fft_error_bound(2 * C, np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 2))))[None, :, None, None]
        n_mis, n_bad = tie_mismatches(sp.numpy().astype(np.float64), q_ref, y_pair, eps + 1e-30)
        say(f"  mismatches {n_mis} of {q_ref.size}, unexplained {n_bad}")
        assert n_bad == 0


def test_chunked_fengine_graph_replay():
    """A chunked F-engine (several F and gather launches per call) and the
    X-engine captured in one HIP graph right after a reset: every replay, with
    eager work between, equals the eager integration bit for bit (int8)."""
    N, C, A = 520, 2048, 128                     # two appended calls of one 136 MB time block each
    say(f"chunked graph replay int8 N={N} C={C} A={A}")
    w = synth.small("fg-g", N, 1, C, A, seed=96)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        v = synth.voltages(w, device=DEV)
        inv = torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV)
        with corr.Correlator(N, 1, C, A, "int8", stream=stream) as c:
            def run():
                c.fengine(v, 64, inv)
                c.fengine(v[:, 64 * C:], A - 64, inv, first_spectrum=64)
                c.xengine(A)
            run()
            ref = c.dump(reset=True).cpu().numpy()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                run()
            for rep in range(3):
                g.replay()
                stream.synchronize()
                got = c.dump(reset=False).cpu().numpy()
                assert np.array_equal(got, ref), rep
                torch.zeros(1000, device=DEV).sum().item()


def test_batched_with_chunked_subarrays_int8():
    """Sub-arrays from 2048 channels up (chunked F-engines, each with its own
    scratch) beside small ones in one batched X-engine launch."""
    shapes = [(20, 2, 2048, 70), (8, 1, 64, 100), (6, 2, 4096, 65)]
    say("batched int8 with chunked F-engines")
    with corr.Batch(shapes, "int8") as b:
        for r, (ns, npol, C, A) in enumerate(shapes):
            w = synth.small(f"fg-b{r}", ns, npol, C, A, seed=110 + r)
            b.subs[r].fengine(synth.voltages(w, device=DEV), A, torch.from_numpy(synth.inv_scale(w, "int8")).to(DEV))
        b.xengine([A for (_, _, _, A) in shapes])
        for r, sub in enumerate(b.subs):
            got = sub.dump().cpu().numpy().astype(np.int64)
            sp = sub.spectra().cpu().numpy()
            assert np.array_equal(got, oracle.xengine_i8(spectra_akp_to_apk(sp))), r
