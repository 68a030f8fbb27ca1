"""GPU parity of the HIP path against the oracle, at sizes the oracle finishes
in seconds that still span several MFMA tiles, several time blocks and ragged
tails.  Every call goes through the C ABI (paper_1305_5639_amd.corr)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_5639_amd as corr
import synth
from helpers import cplx, fft_error_bound, say, spectra_akp_to_apk, tie_mismatches, vis_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _volts(N, C, A, seed, ld=None):
    rng = np.random.default_rng(seed)
    ld = ld or A * C
    v = ((rng.standard_normal((N, ld)) + 1j * rng.standard_normal((N, ld))) * np.sqrt(0.5)).astype(np.complex64)
    return v


def _inputs_lower_ref(S_apk):
    return oracle.xengine_f64(S_apk)


# ------------------------------------------------------------ F-engine ----
@pytest.mark.parametrize("N,C,A,ldpad", [(3, 16, 5, 0), (2, 64, 130, 7), (4, 1024, 9, 0),
                                         (1, 8192, 3, 5), (5, 256, 33, 0), (2, 32, 1, 0),
                                         (3, 128, 17, 0), (2, 512, 16, 0), (2, 2048, 5, 0),
                                         (1, 4096, 2, 0)])
def test_fengine_fp32_matches_dft(N, C, A, ldpad):
    say(f"fengine fp32 N={N} C={C} A={A} ldpad={ldpad}")
    v = _volts(N, C, A, seed=C + N, ld=A * C + ldpad)
    with corr.Correlator(N, 1, C, A, "fp32") as c:
        c.fengine(torch.from_numpy(v).to(DEV), A)
        got = cplx(c.spectra().cpu().numpy())                     # [A][C][N]
    ref = np.swapaxes(oracle.fengine(v, C, A), 1, 2)              # [A][C][N]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.max(np.abs(got - ref)) / rms
    say(f"  max |err| / rms = {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("prec", ["int8", "fp16", "fp8"])
@pytest.mark.parametrize("N,C,A", [(6, 64, 70), (3, 1024, 5), (2, 16, 200), (2, 8192, 3), (3, 2048, 9),
                                   (2, 4096, 4)])
def test_fengine_requantiser_parity(prec, N, C, A):
    """Requantised spectra equal the oracle's rounding of the float64 DFT,
    except at rounding ties closer than the FP32 FFT error."""
    say(f"requant {prec} N={N} C={C} A={A}")
    w = synth.small("rq", N, 1, C, A, seed=40 + C)
    v = synth.voltages(w)
    inv = synth.inv_scale(w, prec)
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.fengine(torch.from_numpy(v).to(DEV), A, torch.from_numpy(inv).to(DEV))
        sp = c.spectra().cpu()
    if prec == "int8":
        q_gpu = sp.numpy().astype(np.float64)
    else:
        q_gpu = sp.to(torch.float64).numpy()
    S = oracle.fengine(v, C, A)                                   # [A][N][C]
    q_ref = np.swapaxes(oracle.quantise(S, inv, prec).astype(np.float64), 1, 2)   # [A][C][N][2]
    y = np.swapaxes(S, 1, 2) * inv.astype(np.float64)[None, :, None]
    y_pair = np.stack([y.real, y.imag], -1)
    rms_y = np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 2)))         # per channel
    eps = fft_error_bound(C, rms_y)[None, :, None, None] + 1e-30
    n_mis, n_bad = tie_mismatches(q_gpu, q_ref, y_pair, eps)
    say(f"  mismatches {n_mis} of {q_ref.size} ({100 * n_mis / q_ref.size:.3f}%), unexplained {n_bad}")
    assert n_bad == 0
    # every mismatch is a rounding tie within the FP32 FFT error; their rate
    # grows with log2 C and the fineness of the code grid (about 0.1% for
    # FP16 at 8192 channels).  A rate far above that would mean the bound
    # itself had grown too loose to be a check.
    assert n_mis <= max(2, q_ref.size // 100)


# ------------------------------------------------------------ X-engine ----
XSHAPES = [(1, 16, 1), (2, 16, 64), (33, 16, 65), (130, 32, 130), (256, 16, 200), (300, 16, 64),
           (129, 16, 3)]


@pytest.mark.parametrize("N,C,A", XSHAPES)
def test_xengine_int8_bit_exact(N, C, A):
    say(f"xengine int8 caller spectra N={N} C={C} A={A}")
    S = synth.int8_spectra(A, C, N, seed=N * 7 + A)               # [A][C][N][2]
    S[0, 0, :, :] = -127                                          # the range ends
    if A > 1:
        S[1, :, 0, 0] = 127
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(A, torch.from_numpy(S).to(DEV))
        got = c.dump().cpu().numpy().astype(np.int64)             # [C][B][2]
    ref = oracle.xengine_i8(spectra_akp_to_apk(S))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp8"])
@pytest.mark.parametrize("N,C,A", [(33, 16, 65), (130, 32, 100), (256, 16, 64), (17, 64, 7)])
def test_xengine_float_forms_on_exact_spectra(prec, N, C, A):
    """Caller spectra holding exactly representable values: only the FP32
    accumulation differs from the float64 oracle."""
    say(f"xengine {prec} caller spectra N={N} C={C} A={A}")
    q = synth.int8_spectra(A, C, N, seed=N + A, rms=3.0).astype(np.float64)
    if prec == "fp8":
        q = np.clip(q, -8, 8)                                     # integers exact in E4M3
    t = torch.from_numpy(q).to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]]).to(DEV)
    inv = None
    s2 = np.ones(C)
    if prec != "fp32":
        inv_np = (2.0 ** np.random.default_rng(C).integers(-3, 4, C)).astype(np.float32)
        inv = torch.from_numpy(inv_np).to(DEV)
        s2 = 1.0 / inv_np.astype(np.float64) ** 2
    with corr.Correlator(N, 1, C, A, prec) as c:
        c.xengine(A, t, inv)
        got = cplx(c.dump().cpu().numpy())
    ref = oracle.xengine_f64(spectra_akp_to_apk(cplx(q))) * s2[:, None]
    eF, en = vis_errors(got, ref, N)
    say(f"  max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-6 and en.max() < 1e-6


# --------------------------------------------------------------- F + X ----
def test_tiny_workload_fp32_end_to_end():
    """16 stations x 1 pol, 64 channels, 1024 spectra with a tone at channel 17."""
    w = synth.WORKLOADS["tiny-16x1-c64"]
    say(f"end-to-end fp32 {w.name}")
    v = synth.voltages(w)
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    with corr.Correlator(w.n_stations, w.n_pols, C, A, "fp32") as c:
        c.fengine(torch.from_numpy(v).to(DEV), A)
        c.xengine(A)
        got = cplx(c.dump().cpu().numpy())
    ref = oracle.xengine_f64(oracle.fengine(v, C, A))
    eF, en = vis_errors(got, ref, N)
    say(f"  max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert eF.max() < 1e-5 and en.max() < 1e-5
    # autos real and non-negative, tone phase per baseline
    d = [i * (i + 1) // 2 + i for i in range(N)]
    assert np.all(got[:, d].imag == 0) and np.all(got[:, d].real >= 0)
    for i in range(N):
        for j in range(i):
            ph = np.angle(got[17, i * (i + 1) // 2 + j] * np.exp(-1j * w.dphi * (j - i)))
            assert abs(ph) < 0.05


@pytest.mark.parametrize("prec", ["int8", "fp16", "fp8"])
def test_end_to_end_identical_spectra(prec):
    """F-engine in the reduced form, then X: the visibilities equal the oracle's
    correlation of the very spectra the GPU produced (exactly for int8)."""
    w = synth.small("e2e", 40, 2, 128, 150, seed=77)
    say(f"end-to-end {prec} {w.n_inputs} inputs C={w.n_channels} A={w.n_integrate}")
    v = synth.voltages(w)
    inv = synth.inv_scale(w, prec)
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    with corr.Correlator(w.n_stations, w.n_pols, C, A, prec) as c:
        c.fengine(torch.from_numpy(v).to(DEV), A, torch.from_numpy(inv).to(DEV))
        c.xengine(A)
        sp = c.spectra().cpu()
        got = c.dump().cpu().numpy()
    if prec == "int8":
        ref = oracle.xengine_i8(spectra_akp_to_apk(sp.numpy()))
        assert np.array_equal(got.astype(np.int64), ref)
        return
    q = cplx(sp.to(torch.float64).numpy())
    s2 = 1.0 / inv.astype(np.float64) ** 2
    ref = oracle.xengine_f64(spectra_akp_to_apk(q)) * s2[:, None]
    eF, en = vis_errors(cplx(got), ref, N)
    say(f"  vs identical spectra: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    # FP16 MFMA sums round like FP32; the FP8 (f8f6f4) MFMA's internal sum is
    # coarser (measured e_F ~1.2e-5), still far below the FP8 quantisation error.
    tol = 1e-6 if prec == "fp16" else 1e-4
    assert eF.max() < tol and en.max() < tol
    # and against the unquantised float64 path (quantisation error, reported)
    ref64 = oracle.xengine_f64(oracle.fengine(v, C, A))
    eF, en = vis_errors(cplx(got), ref64, N)
    say(f"  vs float64 unquantised: max e_F {eF.max():.2e}  max e_n {en.max():.2e}")
    assert en.max() < (2e-3 if prec == "fp16" else 0.1)


@pytest.mark.parametrize("layout,order", [("lower", "baseline"), ("upper", "chan"), ("upper", "baseline"),
                                          ("full", "chan"), ("full", "baseline")])
@pytest.mark.parametrize("prec", ["int8", "fp32"])
def test_dump_layouts_and_orders(layout, order, prec):
    N, C, A = 37, 16, 40
    say(f"dump {prec} {layout} {order}")
    S = synth.int8_spectra(A, C, N, seed=5)
    t = torch.from_numpy(S).to(DEV)
    if prec == "fp32":
        t = t.float()
    with corr.Correlator(N, 1, C, A, prec, layout, order) as c:
        c.xengine(A, t)
        got = c.dump().cpu().numpy()
        host = np.empty_like(got)
        c2 = corr.Correlator(N, 1, C, A, prec, layout, order)
        c2.xengine(A, t)
        corr.corr_dump_visibilities(c2.handle, host, reset=True)    # host destination
        c2.close()
    ref = oracle.emit(oracle.xengine_i8(spectra_akp_to_apk(S)), N, layout, order)
    assert np.array_equal(got.astype(np.int64), ref)
    assert np.array_equal(host, got)


def test_split_integration_and_resume_int8():
    """Two calls (40 + 60 spectra) equal one call of 100; a dump without reset
    keeps integrating; a reset starts again from zero."""
    N, C, A = 70, 32, 100
    say("resume int8")
    S = synth.int8_spectra(A, C, N, seed=9)
    d = torch.from_numpy(S).to(DEV)
    with corr.Correlator(N, 1, C, A, "int8") as c:
        c.xengine(40, d[:40].contiguous())
        part = c.dump(reset=False).cpu().numpy().astype(np.int64)
        c.xengine(60, d[40:].contiguous())
        assert c.counts() == (60, 100)
        whole = c.dump(reset=True).cpu().numpy().astype(np.int64)
        assert c.counts()[1] == 0
        zero = c.dump().cpu().numpy()
        assert not zero.any()
    ref40 = oracle.xengine_i8(spectra_akp_to_apk(S[:40]))
    ref = oracle.xengine_i8(spectra_akp_to_apk(S))
    assert np.array_equal(part, ref40)
    assert np.array_equal(whole, ref)


def test_prefix_of_held_spectra():
    """corr_xengine with n_spectra below the spectra held uses the first ones
    (the rest of the last time block is masked)."""
    w = synth.small("prefix", 12, 1, 64, 150, seed=3)
    say("prefix of held spectra")
    v = synth.voltages(w)
    inv = synth.inv_scale(w, "int8")
    with corr.Correlator(12, 1, 64, 150, "int8") as c:
        c.fengine(torch.from_numpy(v).to(DEV), 150, torch.from_numpy(inv).to(DEV))
        sp = c.spectra().cpu().numpy()
        c.xengine(77)
        got = c.dump().cpu().numpy().astype(np.int64)
    ref = oracle.xengine_i8(spectra_akp_to_apk(sp[:77]))
    assert np.array_equal(got, ref)


def test_runtime_state_errors():
    say("runtime state errors")
    with corr.Correlator(2, 1, 16, 8, "int8") as c:
        with pytest.raises(corr.CorrError) as e:
            c.xengine(4)
        assert e.value.status == corr.CORR_E_STATE
        with pytest.raises(corr.CorrError) as e:            # int8 needs a scale
            c.fengine(torch.zeros((2, 128), dtype=torch.complex64, device=DEV), 8)
        assert e.value.status == corr.CORR_E_INVALID_ARG
        inv = torch.ones(16, device=DEV)
        c.fengine(torch.zeros((2, 128), dtype=torch.complex64, device=DEV), 8, inv)
        with pytest.raises(corr.CorrError) as e:
            c.xengine(9)
        assert e.value.status == corr.CORR_E_STATE
    # int8 integration overflow is refused on the host before any launch
    with corr.Correlator(1, 1, 16, 40000, "int8") as c:
        S = torch.zeros((40000, 16, 1, 2), dtype=torch.int8, device=DEV)
        c.xengine(40000, S)
        with pytest.raises(corr.CorrError) as e:
            c.xengine(40000, S)
        assert e.value.status == corr.CORR_E_OVERFLOW
        assert c.counts()[1] == 40000


def test_nomem_from_device_budget():
    with pytest.raises(corr.CorrError) as e:
        corr.Correlator(4096, 2, 8192, 1000, "fp32")         # ~2 TB of accumulators
    assert e.value.status == corr.CORR_E_NOMEM
