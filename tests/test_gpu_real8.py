"""GPU parity of the real-input F-engine (8-bit real samples, transform length
2C, Section 5) and of the FX path it feeds, against the oracle, through the
C ABI: small shapes spanning every transform size, ragged spectrum counts and
padded rows, and the paper's own workload (2048 streams, transform length 256)
at full size on sampled streams and channels."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, fft_error_bound, say, tie_mismatches, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _samples(N, C, A, seed, ldpad=0, sigma=8.0):
    w = synth.small_real("r8", N, C, A, seed, sigma=sigma)
    x = synth.real8_samples(w)
    if ldpad:
        x = np.ascontiguousarray(np.pad(x, ((0, 0), (0, ldpad))))
    return w, x


@pytest.mark.parametrize("N,C,A,ldpad", [(3, 16, 5, 0), (2, 32, 1, 0), (2, 64, 130, 6), (3, 128, 17, 0),
                                         (4, 128, 64, 2), (5, 256, 33, 0), (2, 512, 16, 0),
                                         (4, 1024, 9, 0), (2, 2048, 5, 0), (1, 4096, 2, 4),
                                         (1, 8192, 3, 10)])
def test_fengine_real8_fp32_matches_dft(N, C, A, ldpad):
    say(f"fengine_real8 fp32 N={N} C={C} A={A} ldpad={ldpad}")
    w, x = _samples(N, C, A, seed=C + N, ldpad=ldpad)
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A)
        got = cplx(c.spectra().cpu().numpy())                     # [A][C][N]
    ref = np.swapaxes(oracle.fengine_real8(x, C, A), 1, 2)        # [A][C][N]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.max(np.abs(got - ref)) / rms
    say(f"  max |err| / rms = {err:.2e}")
    assert err < 1e-5
    # channel 0 of a real signal is real
    assert np.max(np.abs(got[:, 0, :].imag)) <= 1e-5 * rms


def test_fengine_real8_full_scale_samples():
    """Samples at the 8-bit limits (-128 and 127) and a constant row: the DC
    channel takes the whole sum and the others vanish."""
    N, C, A = 3, 128, 4
    rng = np.random.default_rng(3)
    x = rng.choice(np.array([-128, 127], np.int8), size=(N, A * 2 * C))
    x[2] = -128
    say(f"fengine_real8 full-scale N={N} C={C} A={A}")
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A)
        got = cplx(c.spectra().cpu().numpy())
    ref = np.swapaxes(oracle.fengine_real8(x, C, A), 1, 2)
    assert np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)) < 1e-5
    assert np.all(got[:, 0, 2] == -128.0 * 2 * C)
    assert np.max(np.abs(got[:, 1:, 2])) == 0.0


@pytest.mark.parametrize("prec", ["int8", "fp16", "fp8"])
@pytest.mark.parametrize("N,C,A", [(6, 128, 70), (3, 1024, 5), (2, 16, 200), (2, 8192, 3)])
def test_fengine_real8_requantiser_parity(prec, N, C, A):
    """Requantised real-input spectra equal the oracle's rounding of the
    float64 DFT, except at rounding ties closer than the FP32 FFT error."""
    say(f"requant real8 {prec} N={N} C={C} A={A}")
    w, x = _samples(N, C, A, seed=70 + C)
    inv = synth.real8_inv_scale(w, prec)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A, torch.from_numpy(inv).to(DEV))
        sp = c.spectra().cpu()
    q_gpu = sp.numpy().astype(np.float64) if prec == "int8" else sp.to(torch.float64).numpy()
    S = oracle.fengine_real8(x, C, A)                             # [A][N][C]
    q_ref = np.swapaxes(oracle.quantise(S, inv, prec).astype(np.float64), 1, 2)
    y = np.swapaxes(S, 1, 2) * inv.astype(np.float64)[None, :, None]
    y_pair = np.stack([y.real, y.imag], -1)
    rms_y = np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 2)))
    # the length-2C transform has one more radix-2 stage than the C-point FFT
    eps = fft_error_bound(2 * C, rms_y)[None, :, None, None] + 1e-30
    n_mis, n_bad = tie_mismatches(q_gpu, q_ref, y_pair, eps)
    say(f"  mismatches {n_mis} of {q_ref.size}, unexplained {n_bad}")
    assert n_bad == 0
    assert n_mis <= max(2, q_ref.size // 100)


def test_real8_fx_fp32_end_to_end():
    N, C, A = 24, 128, 300
    say(f"real8 FX fp32 N={N} C={C} A={A}")
    w, x = _samples(N, C, A, seed=5)
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A)
        c.xengine(A)
        got = cplx(c.dump().cpu().numpy())
    ref = oracle.xengine_f64(oracle.fengine_real8(x, C, A))
    eF, en = vis_errors(got, ref, N)
    say(f"  max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-5 and en.max() < 1e-5


@pytest.mark.parametrize("prec", ["int8", "fp16"])
def test_real8_fx_low_precision_end_to_end(prec):
    """The X-engine on the spectra the real-input F-engine produced: bit-exact
    (int8) or within FP32 accumulation error (FP16) of the oracle's
    correlation of those same spectra."""
    N, C, A = 40, 128, 256
    say(f"real8 FX {prec} N={N} C={C} A={A}")
    w, x = _samples(N, C, A, seed=6)
    inv = synth.real8_inv_scale(w, prec)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine_real8(torch.from_numpy(x).to(DEV), A, torch.from_numpy(inv).to(DEV))
        c.xengine(A)
        sp = c.spectra().cpu()
        vis = c.dump().cpu().numpy()
    if prec == "int8":
        S = np.swapaxes(sp.numpy(), 1, 2)                         # [A][N][C][2]
        ref = oracle.xengine_i8(S)
        assert np.array_equal(vis.astype(np.int64), ref)
    else:
        S = np.swapaxes(sp.to(torch.float64).numpy(), 1, 2)
        s2 = (1.0 / inv.astype(np.float64)) ** 2
        ref = oracle.xengine_f64(cplx(S)) * s2[:, None]
        eF, en = vis_errors(cplx(vis), ref, N)
        say(f"  max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
        assert eF.max() < 1e-5 and en.max() < 1e-5


def test_real8_argument_checks():
    N, C, A = 2, 64, 4
    x = torch.zeros((N, A * 2 * C + 2), dtype=torch.int8, device=DEV)
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        with pytest.raises(corr.CorrError):
            c.fengine_real8(x, A, ld_samples=A * 2 * C - 2)        # row shorter than the blocks
        with pytest.raises(corr.CorrError):
            c.fengine_real8(x, A, ld_samples=A * 2 * C + 1)        # odd stride
        with pytest.raises(corr.CorrError):
            c.fengine_real8(x.view(-1)[1:], 1, ld_samples=A * 2 * C)   # odd address
        with pytest.raises(corr.CorrError):
            c.fengine_real8(x, A + 1)                              # above n_integrate
    with corr.Correlator(N, 1, C, A, "int8") as c:
        with pytest.raises(corr.CorrError):
            c.fengine_real8(x, A)                                  # int8 needs a scale


def _autos_idx(N):
    return np.array([i * (i + 1) // 2 + i for i in range(N)])


@pytest.mark.timeout(900)
def test_paper_workload_full_size_int8_and_fp32():
    """2048 streams of 8-bit real samples, transform length 256, 1024 spectra
    (the benchmarked launch): int8 X bit-exact on sampled streams and
    channels; FP32 within 1e-5 of the float64 oracle on the same sample and
    the real-signal Parseval identity on every stream's autos."""
    w = synth.REAL_WORKLOADS["paper-2048-r256"]
    N, C, A = w.n_streams, w.n_channels, w.n_integrate
    torch.cuda.empty_cache()
    say(f"full size {w.name}: drawing samples")
    x = synth.real8_samples(w, device=DEV)
    rows = np.unique(np.concatenate([[0, 1, N - 1], np.random.default_rng(1).choice(N, 93, replace=False)]))
    chans = sorted({0, 1, w.tone_bin, C // 2, C - 1, 100})
    xs = x[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    S64 = oracle.fengine_real8(xs, C, A, chans)                   # [A][n][k]
    il, jl = np.tril_indices(rows.size)
    bsel = rows[il] * (rows[il] + 1) // 2 + rows[jl]

    say("  int8")
    inv = synth.real8_inv_scale(w, "int8")
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.fengine_real8(x, A, torch.from_numpy(inv).to(DEV))
        c.xengine(A)
        vis = c.dump()
        got = vis[torch.as_tensor(chans, device=DEV)][:, torch.as_tensor(bsel, device=DEV)].cpu().numpy()
        sp = c.spectra()[:, torch.as_tensor(chans, device=DEV)][:, :, torch.as_tensor(rows, device=DEV)]
        sp = sp.cpu().numpy()                                     # [A][k][n][2]
        del vis
    Sq = np.swapaxes(sp, 1, 2)                                    # [A][n][k][2]
    ref = oracle.xengine_i8(Sq)
    assert np.array_equal(got.astype(np.int64), ref)
    q_ref = oracle.quantise(S64, inv[chans], "int8").astype(np.float64)
    y = S64 * inv[chans].astype(np.float64)[None, None, :]
    eps = fft_error_bound(2 * C, np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 1))))[None, None, :, None]
    n_mis, n_bad = tie_mismatches(Sq.astype(np.float64), q_ref, np.stack([y.real, y.imag], -1), eps)
    say(f"  int8 spectra: mismatches {n_mis} of {q_ref.size}, unexplained {n_bad}")
    assert n_bad == 0 and n_mis <= max(2, q_ref.size // 100)

    say("  fp32")
    torch.cuda.empty_cache()
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.fengine_real8(x, A)
        c.xengine(A)
        vis = c.dump()
        autos = vis[:, torch.as_tensor(_autos_idx(N), device=DEV), 0].double()      # [C][N]
        got = cplx(vis[torch.as_tensor(chans, device=DEV)][:, torch.as_tensor(bsel, device=DEV)].cpu().numpy())
        del vis
    ref = oracle.xengine_f64(S64)
    eF, en = vis_errors(got, ref, rows.size)
    say(f"  fp32 sampled: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-5 and en.max() < 1e-5
    # 2C sum x^2 = X_0^2 + X_C^2 + 2 sum_{0<k<C} |X_k|^2 per spectrum, summed
    # over spectra; the Nyquist term X_C = sum_n (-1)^n x[n] comes from the samples.
    xb = x.view(N, A, 2 * C).double()
    sign = torch.ones(2 * C, dtype=torch.float64, device=DEV)
    sign[1::2] = -1
    nyq = ((xb * sign).sum(-1) ** 2).sum(-1)                      # [N]
    energy = (xb ** 2).sum(dim=(1, 2))
    lhs = (autos[0] + nyq + 2 * autos[1:].sum(0)).cpu().numpy()
    rhs = (2 * C * energy).cpu().numpy()
    rel = np.abs(lhs - rhs) / rhs
    say(f"  Parseval on autos: max rel {rel.max():.2e}")
    assert rel.max() < 1e-5
