"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the oracle computes a sample of channels one by one (all
inputs and spectra of those channels), and properties that hold at any size
(Parseval on the autos, real non-negative autos) are checked on every channel.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, say, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _sample(w, n_extra, seed=0):
    C = w.n_channels
    base = {0, C // 2, C - 1, *[b for b in w.tone_bins if b < C]}
    rng = np.random.default_rng(seed)
    extra = [int(x) for x in rng.permutation(C) if int(x) not in base][:n_extra]
    return sorted(base | set(extra))


def _autos_idx(N):
    return np.array([i * (i + 1) // 2 + i for i in range(N)])


@pytest.mark.timeout(900)
def test_mwa_fp32_full_size():
    w = synth.WORKLOADS["mwa-128x2-c1024"]
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    say(f"full size fp32 {w.name}")
    torch.cuda.empty_cache()
    v = synth.voltages(w, device=DEV)
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "fp32") as c:
        c.fengine(v, A)
        c.xengine(A)
        vis = c.dump()                                            # [C][B][2] on device
    # Parseval on every channel's autos: sum_k C_ii[k] = C sum_n |s_i[n]|^2
    power = (v.real.double() ** 2 + v.imag.double() ** 2).sum(dim=1).cpu().numpy()
    autos = vis[:, torch.as_tensor(_autos_idx(N), device=DEV), 0].double().sum(dim=0).cpu().numpy()
    rel = np.abs(autos - C * power) / (C * power)
    say(f"  Parseval on autos: max rel {rel.max():.2e}")
    assert rel.max() < 1e-5
    assert bool((vis[:, torch.as_tensor(_autos_idx(N), device=DEV), 1] == 0).all())
    chans = _sample(w, 6)
    got = cplx(vis[chans].cpu().numpy())
    vh = v.cpu().numpy()
    say(f"  oracle on channels {chans}")
    ref = oracle.xengine_f64(oracle.fengine(vh, C, A, chans))
    eF, en = vis_errors(got, ref, N)
    say(f"  sampled: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-5 and en.max() < 1e-5


@pytest.mark.timeout(900)
def test_int8_full_size_bit_exact_and_fp16_error():
    w = synth.WORKLOADS["int8-256x2-c2048"]
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    say(f"full size int8 {w.name}")
    torch.cuda.empty_cache()
    v = synth.voltages(w, device=DEV)
    inv = synth.inv_scale(w, "int8")
    chans = _sample(w, 2, seed=1)
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "int8") as c:
        c.fengine(v, A, torch.from_numpy(inv).to(DEV))
        c.xengine(A)
        vis = c.dump()
        sp = c.spectra()                                          # [A][C][N][2] int8
        sp_h = sp.cpu().numpy()                                   # every channel, 4.3 GB
        del sp
    q = sp_h[:, chans]                                            # [A][Cs][N][2]
    vis_h = vis.cpu().numpy()                                     # [C][B][2] int32
    got = vis_h[chans].astype(np.int64)
    # Eq. 2 in exact integers on EVERY channel, in channel chunks (bounded host
    # memory): the X-engine must equal the int64 oracle bit for bit.
    step = 256
    for c0 in range(0, C, step):
        say(f"  int64 oracle on the GPU's int8 spectra, channels [{c0}, {c0 + step})")
        ref = oracle.xengine_i8(np.ascontiguousarray(np.swapaxes(sp_h[:, c0:c0 + step], 1, 2)))
        assert np.array_equal(vis_h[c0:c0 + step].astype(np.int64), ref), c0
    del sp_h, vis_h
    # requantiser on the sample: codes equal the oracle's rounding of the
    # float64 DFT, up to rounding ties
    vh = v.cpu().numpy()
    S = oracle.fengine(vh, C, A, chans)                            # [A][N][Cs]
    q_ref = np.swapaxes(oracle.quantise(S, inv[chans], "int8"), 1, 2)
    mism = (q_ref != q).mean()
    say(f"  requantiser mismatch fraction {mism:.2e}")
    assert mism < 1e-4
    # the same integration in FP16 (FP32 accumulation): error against float64
    ref64 = oracle.xengine_f64(S)
    del vis
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "fp16") as c:
        c.fengine(v, A, torch.from_numpy(synth.inv_scale(w, "fp16")).to(DEV))
        c.xengine(A)
        g16 = cplx(c.dump()[chans].cpu().numpy())
    eF, en = vis_errors(g16, ref64, N)
    say(f"  fp16 vs float64: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert en.max() < 1e-3
    gi = cplx(got) * (1.0 / inv[chans].astype(np.float64) ** 2)[:, None]
    eF, en = vis_errors(gi, ref64, N)
    say(f"  int8 (16-LSB RMS) vs float64: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert en.max() < 0.05


@pytest.mark.timeout(900)
def test_ska_fp8_and_fp32_full_size():
    """1024 inputs x 4096 channels x 1024 spectra: the FP8 form and the plain
    FP32 path, each as a whole F + X step on complex64 voltages, against the
    float64 oracle (Eq. 1 then Eq. 2) on sampled channels that include 0, C/2
    and C - 1."""
    w = synth.WORKLOADS["ska-512x2-c4096"]
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    say(f"full size fp8 + fp32 {w.name}")
    torch.cuda.empty_cache()
    v = synth.voltages(w, device=DEV)
    inv = synth.inv_scale(w, "fp8")
    chans = _sample(w, 2, seed=2)
    assert {0, C // 2, C - 1} <= set(chans)
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "fp8") as c:
        c.fengine(v, A, torch.from_numpy(inv).to(DEV))
        c.xengine(A)
        vis = c.dump()
        got = cplx(vis[chans].cpu().numpy())
        autos_ok = bool((vis[:, torch.as_tensor(_autos_idx(N), device=DEV), 0] >= 0).all())
        del vis
        sp = c.spectra()
        q8 = sp.view(torch.uint8)[:, chans].cpu()
        q = q8.view(torch.float8_e4m3fn).to(torch.float64).numpy()
        del sp
    torch.cuda.empty_cache()
    assert autos_ok
    s2 = 1.0 / inv[chans].astype(np.float64) ** 2
    ref_q = oracle.xengine_f64(np.ascontiguousarray(np.swapaxes(cplx(q), 1, 2))) * s2[:, None]
    eF, en = vis_errors(got, ref_q, N)
    say(f"  vs identical FP8 spectra: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-4 and en.max() < 1e-4

    # the plain FP32 path on the same voltages
    say("  fp32 F + X at full size")
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "fp32") as c:
        c.fengine(v, A)
        c.xengine(A)
        vis = c.dump()
        got32 = cplx(vis[chans].cpu().numpy())
        autos = vis[:, torch.as_tensor(_autos_idx(N), device=DEV)]
        autos_real = bool((autos[..., 1] == 0).all()) and bool((autos[..., 0] >= 0).all())
        auto_sum = autos[..., 0].double().sum(dim=0).cpu().numpy()
        del vis, autos
    torch.cuda.empty_cache()
    assert autos_real
    # Parseval on every channel's autos: sum_k C_ii[k] = C sum_n |s_i[n]|^2
    power = (v.real.double() ** 2 + v.imag.double() ** 2).sum(dim=1).cpu().numpy()
    rel = np.abs(auto_sum - C * power) / (C * power)
    say(f"  fp32 Parseval on autos: max rel {rel.max():.2e}")
    assert rel.max() < 1e-5

    vh = v.cpu().numpy()
    del v
    torch.cuda.empty_cache()
    say(f"  float64 oracle DFT on channels {chans}")
    ref64 = oracle.xengine_f64(oracle.fengine(vh, C, A, chans))
    del vh
    eF, en = vis_errors(got32, ref64, N)
    say(f"  fp32 vs float64: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-5 and en.max() < 1e-5
    eF, en = vis_errors(got, ref64, N)
    say(f"  fp8 vs float64 per channel e_F {np.array2string(eF, precision=2)}  max e_n {en.max():.2e}")
    assert en.max() < 0.1
