"""GPU checks of the F-engines writing at an offset of the held spectra
(corr_fengine_at / corr_fengine_real8_at): an integration channelised in
pieces holds exactly the spectra of one call over the whole run, so one
X-engine call over it equals the single-call result, and the placement rules
(time-block alignment, no gap, capacity) are enforced."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import say, spectra_akp_to_apk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TB = {"fp32": 16, "fp16": 32, "fp8": 64, "int8": 64}


def _pieces(A, tb, sizes_in_blocks):
    """[(first, n)] covering [0, A): whole time blocks, the last one ragged."""
    out, first = [], 0
    for nb in sizes_in_blocks:
        n = min(nb * tb, A - first)
        if n <= 0:
            break
        out.append((first, n))
        first += n
    if first < A:
        out.append((first, A - first))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp8", "int8"])
def test_complex_pieces_equal_one_call(prec):
    N, C, A = 10, 64, 300
    say(f"append complex {prec} N={N} C={C} A={A}")
    w = synth.small("ap", N, 1, C, A, seed=90)
    v = torch.from_numpy(synth.voltages(w)).to(DEV)
    inv = torch.from_numpy(synth.inv_scale(w, prec)).to(DEV) if prec != "fp32" else None
    with corr.Correlator(N, 1, C, A, prec) as whole, corr.Correlator(N, 1, C, A, prec) as parts:
        whole.fengine(v, A, inv)
        whole.xengine(A)
        for first, n in _pieces(A, TB[prec], [2, 1, 3]):
            # each piece reads its own buffer: the samples of spectra [first, first + n)
            piece = v[:, first * C:(first + n) * C].contiguous()
            parts.fengine(piece, n, inv, first_spectrum=first)
        parts.xengine(A)
        assert torch.equal(whole.spectra(), parts.spectra())
        assert torch.equal(whole.dump(), parts.dump())


@pytest.mark.parametrize("prec", ["fp32", "int8"])
def test_real_input_pieces_equal_one_call_and_oracle(prec):
    N, C, A = 6, 128, 200
    say(f"append real8 {prec} N={N} C={C} A={A}")
    rw = synth.small_real("ap-r8", N, C, A, seed=91)
    x = synth.real8_samples(rw)
    xd = torch.from_numpy(x).to(DEV)
    inv = torch.from_numpy(synth.real8_inv_scale(rw, prec)).to(DEV) if prec == "int8" else None
    with corr.Correlator(N, 1, C, A, prec) as whole, corr.Correlator(N, 1, C, A, prec) as parts:
        whole.fengine_real8(xd, A, inv)
        whole.xengine(A)
        for first, n in _pieces(A, TB[prec], [1, 1]):
            parts.fengine_real8(xd[:, first * 2 * C:(first + n) * 2 * C].contiguous(), n, inv, first_spectrum=first)
        parts.xengine(A)
        assert torch.equal(whole.spectra(), parts.spectra())
        got = parts.dump().cpu().numpy()
        sp = parts.spectra().cpu().numpy()
    if prec == "int8":
        assert np.array_equal(got.astype(np.int64), oracle.xengine_i8(spectra_akp_to_apk(sp)))


def test_placement_rules():
    N, C, A = 4, 64, 256
    v = torch.zeros((N, A * C), dtype=torch.complex64, device=DEV)
    with corr.Correlator(N, 1, C, A, "fp16") as c:
        with pytest.raises(corr.CorrError):
            c.fengine(v, 32, first_spectrum=32)            # nothing held yet: a gap
        c.fengine(v, 64)
        with pytest.raises(corr.CorrError):
            c.fengine(v, 32, first_spectrum=16)            # not a multiple of the 32-spectrum time block
        with pytest.raises(corr.CorrError):
            c.fengine(v, 32, first_spectrum=96)            # gap after the 64 held spectra
        with pytest.raises(corr.CorrError):
            c.fengine(v, 224, first_spectrum=64)           # past n_integrate
        c.fengine(v, 192, first_spectrum=64)               # exactly fills the buffer
        counts = c.counts()
        assert counts[0] == 256
        c.fengine(v, 32, first_spectrum=32)                # overwrite from 32 on: the held set ends at 64
        assert c.counts()[0] == 64
        # caller spectra cannot be appended to
        c.xengine(32, torch.zeros((32, C, N, 2), dtype=torch.float16, device=DEV))
        with pytest.raises(corr.CorrError):
            c.fengine(v, 32, first_spectrum=32)


def test_graph_replay_of_real_input_pieces_and_xengine():
    """Real-input F-engine pieces and the X-engine of one handle captured in a
    HIP graph right after a reset (so the captured X-engine writes the
    accumulators): every replay, with eager work between, equals the eager
    integration, bit for bit (int8)."""
    N, C, A = 20, 128, 256
    say(f"graph replay real8 pieces N={N} C={C} A={A}")
    rw = synth.small_real("ap-g", N, C, A, seed=92)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        xd = torch.from_numpy(synth.real8_samples(rw)).to(DEV)
        inv = torch.from_numpy(synth.real8_inv_scale(rw, "int8")).to(DEV)
        pieces = [(f, n, xd[:, f * 2 * C:(f + n) * 2 * C].contiguous()) for f, n in _pieces(A, 64, [1, 2])]
        with corr.Correlator(N, 1, C, A, "int8", stream=stream) as c:
            def run():
                for f, n, buf in pieces:
                    c.fengine_real8(buf, n, inv, first_spectrum=f)
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
