"""Pins of the oracle against things other than itself (CPU only).

Each test ties one oracle routine to a library special case, a closed form,
an invariant, brute force on tiny inputs, or a hand-derived fixture, chosen so
that a dropped term, a wrong sign or index, or a transposed operand fails.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _crand(rng, shape, scale=1.0):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale).astype(np.complex64)


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------- Eq. 1 ----
@pytest.mark.parametrize("C", [4, 8, 16, 64, 256, 1024])
def test_dft_matches_numpy_fft(orc, C):
    """Library special case: numpy's FFT of complex128 blocks (Eq. 1, forward,
    unnormalised, natural order)."""
    rng = np.random.default_rng(C)
    A, N = 3, 4
    v = _crand(rng, (N, A * C))
    S = orc.fengine(v, C, A)                                   # [A][N][C]
    ref = np.fft.fft(v.astype(np.complex128).reshape(N, A, C), axis=-1).transpose(1, 0, 2)
    assert _rel(S, ref) < 1e-12


def test_dft_golden_exact_bin(orc):
    g = json.load(open(os.path.join(GOLDEN, "dft_exact_bin.json")))
    s = np.array([complex(*x) for x in g["s"]], dtype=np.complex64)[None, :]
    S = orc.fengine(s, g["C"], 1)[0, 0]
    ref = np.array([complex(*x) for x in g["S"]])
    assert np.max(np.abs(S - ref)) < 1e-14


@pytest.mark.parametrize("C,n0", [(16, 0), (16, 5), (64, 63), (256, 17)])
def test_dft_impulse(orc, C, n0):
    """An impulse at n0 gives exp(-j 2 pi k n0 / C): flat magnitude, linear phase."""
    v = np.zeros((1, C), np.complex64)
    v[0, n0] = 1
    S = orc.fengine(v, C, 1)[0, 0]
    k = np.arange(C)
    ref = np.exp(-2j * np.pi * ((k * n0) % C) / C)
    assert np.max(np.abs(S - ref)) < 1e-14
    assert np.allclose(np.abs(S), 1.0, atol=1e-14)


@pytest.mark.parametrize("C,k0,amp,phi", [(64, 17, 1.0, 0.3), (1024, 97, 0.5, -2.0), (4096, 4095, 2.0, 1.0)])
def test_dft_exact_bin_tone(orc, C, k0, amp, phi):
    """a exp(j(2 pi k0 n / C + phi)) -> a C exp(j phi) at k0 and ~0 elsewhere."""
    n = np.arange(C)
    v = (amp * np.exp(1j * (2 * np.pi * ((k0 * n) % C) / C + phi))).astype(np.complex64)[None]
    S = orc.fengine(v, C, 1)[0, 0]
    # tolerance covers the complex64 rounding of the input samples
    tol = amp * C * 1e-6
    assert abs(S[k0] - amp * C * np.exp(1j * phi)) < tol
    others = np.delete(S, k0)
    assert np.max(np.abs(others)) < tol


def test_dft_parseval(orc):
    rng = np.random.default_rng(7)
    C, A, N = 512, 2, 3
    v = _crand(rng, (N, A * C))
    S = orc.fengine(v, C, A)
    lhs = np.sum(np.abs(S) ** 2, axis=-1)                                   # [A][N]
    rhs = C * np.sum(np.abs(v.astype(np.complex128).reshape(N, A, C)) ** 2, axis=-1).T
    assert _rel(lhs, rhs) < 1e-12


def test_dft_shift_theorem(orc):
    rng = np.random.default_rng(8)
    C, d = 128, 9
    x = _crand(rng, (C,))
    v = np.stack([x, np.roll(x, d)])
    S = orc.fengine(v, C, 1)[0]
    k = np.arange(C)
    assert _rel(S[1], S[0] * np.exp(-2j * np.pi * ((k * d) % C) / C)) < 1e-12


def test_dft_channel_subset_and_blocks(orc):
    """A channel subset equals those entries of the full transform, and block a
    reads samples [aC, (a+1)C) of a row with a leading dimension ld > A*C."""
    rng = np.random.default_rng(9)
    C, A, N, ld = 32, 3, 2, 3 * 32 + 11
    v = _crand(rng, (N, ld))
    full = orc.fengine(v, C, A)
    ch = [31, 0, 5, 16]
    sub = orc.fengine(v, C, A, ch)
    assert np.array_equal(sub, full[:, :, ch])
    for a in range(A):
        ref = np.fft.fft(v[:, a * C:(a + 1) * C].astype(np.complex128), axis=-1)
        assert _rel(full[a], ref) < 1e-12


# ------------------------------------------- Eq. 1, 8-bit real samples ----
def _i8(rng, shape, lo=-128, hi=128):
    return rng.integers(lo, hi, shape, dtype=np.int8)


@pytest.mark.parametrize("C", [2, 8, 64, 128, 512])
def test_real8_matches_numpy_rfft(orc, C):
    """Library special case: numpy's real FFT of length 2C (forward,
    unnormalised, bins 0..C), blocks of 2C samples from rows with ld > A*2C."""
    rng = np.random.default_rng(100 + C)
    A, N = 3, 4
    ld = A * 2 * C + 5
    x = _i8(rng, (N, ld))
    chans = np.arange(C + 1)
    S = orc.fengine_real8(x, C, A, chans)                              # [A][N][C+1]
    ref = np.fft.rfft(x[:, :A * 2 * C].astype(np.float64).reshape(N, A, 2 * C), axis=-1).transpose(1, 0, 2)
    assert _rel(S, ref) < 1e-12
    assert np.array_equal(orc.fengine_real8(x, C, A), S[:, :, :C])      # default: channels 0..C-1


@pytest.mark.parametrize("C,n0", [(4, 0), (16, 5), (128, 255), (128, 17)])
def test_real8_impulse(orc, C, n0):
    """x[n0] = 1 gives exp(-j pi k n0 / C) at every channel 0..C."""
    x = np.zeros((1, 2 * C), np.int8)
    x[0, n0] = 1
    k = np.arange(C + 1)
    S = orc.fengine_real8(x, C, 1, k)[0, 0]
    ref = np.exp(-1j * np.pi * ((k * n0) % (2 * C)) / C)
    assert np.max(np.abs(S - ref)) < 1e-14


@pytest.mark.parametrize("C", [4, 128])
def test_real8_dc_nyquist_quarter(orc, C):
    """Closed forms with integer samples: a constant lands only in channel 0
    (2C times it), (-1)^n only in the Nyquist channel C, and the period-4
    sequences cos(pi n/2) = 1,0,-1,0 and sin(pi n/2) = 0,1,0,-1 only in
    channel C/2, as C and -jC."""
    n = np.arange(2 * C)
    x = np.stack([np.full(2 * C, -7), (-1) ** n, [1, 0, -1, 0][0:4] * (C // 2),
                  [0, 1, 0, -1] * (C // 2)]).astype(np.int8)
    k = np.arange(C + 1)
    S = orc.fengine_real8(x, C, 1, k)[0]
    ref = np.zeros((4, C + 1), complex)
    ref[0, 0] = -7 * 2 * C
    ref[1, C] = 2 * C
    ref[2, C // 2] = C
    ref[3, C // 2] = -1j * C
    assert np.max(np.abs(S - ref)) < 1e-12


def test_real8_equals_complex_dft_of_real_samples(orc):
    """The real-input transform equals the (separately pinned) complex DFT of
    length 2C of the same samples with zero imaginary part, channels 0..C."""
    rng = np.random.default_rng(11)
    C, A, N = 64, 2, 3
    x = _i8(rng, (N, A * 2 * C))
    k = np.arange(C + 1)
    S = orc.fengine_real8(x, C, A, k)
    Z = orc.fengine(x.astype(np.complex64), 2 * C, A, k)
    assert _rel(S, Z) < 1e-13


def test_real8_parseval(orc):
    """For real samples: 2C sum x^2 = |X_0|^2 + |X_C|^2 + 2 sum_{0<k<C} |X_k|^2."""
    rng = np.random.default_rng(12)
    C, A, N = 128, 3, 2
    x = _i8(rng, (N, A * 2 * C))
    S = orc.fengine_real8(x, C, A, np.arange(C + 1))
    P = np.abs(S) ** 2
    lhs = P[..., 0] + P[..., C] + 2 * P[..., 1:C].sum(-1)                # [A][N]
    rhs = 2 * C * (x.astype(np.float64).reshape(N, A, 2 * C) ** 2).sum(-1).T
    assert _rel(lhs, rhs) < 1e-12
    assert np.max(np.abs(S[..., 0].imag)) < 1e-9 and np.max(np.abs(S[..., C].imag)) < 1e-9


def test_real8_rejects_bad_arguments(orc):
    x = np.zeros((1, 16), np.int8)
    with pytest.raises(ValueError):
        orc.fengine_real8(x, 8, 2)
    with pytest.raises(ValueError):
        orc.fengine_real8(x, 8, 1, [9])


# ---------------------------------------------------------------- Eq. 2 ----
def _brute_xcorr(S):
    """Python-loop statement of Eq. 2 on complex numbers (tiny sizes only)."""
    A, N, K = S.shape
    out = np.zeros((K, N * (N + 1) // 2), dtype=np.complex128)
    for k in range(K):
        b = 0
        for i in range(N):
            for j in range(i + 1):
                out[k, b] = sum(np.conj(S[a, i, k]) * S[a, j, k] for a in range(A))
                b += 1
    return out


def test_xengine_golden_two_inputs(orc):
    g = json.load(open(os.path.join(GOLDEN, "xcorr_two_inputs.json")))
    S = np.array(g["S"], dtype=np.float64)                 # [A][N][K][2]
    Sc = S[..., 0] + 1j * S[..., 1]
    V = orc.xengine_f64(Sc)
    ref = np.array(g["V"], dtype=np.float64)
    assert np.array_equal(np.stack([V.real, V.imag], -1), ref)
    Vi = orc.xengine_i8(S.astype(np.int8))
    assert np.array_equal(Vi, ref.astype(np.int64))


@pytest.mark.parametrize("A,N,K", [(1, 1, 1), (4, 8, 8), (3, 5, 2), (2, 7, 3)])
def test_xengine_brute_force_and_matmul(orc, A, N, K):
    rng = np.random.default_rng(A * 100 + N * 10 + K)
    S = (rng.standard_normal((A, N, K)) + 1j * rng.standard_normal((A, N, K)))
    V = orc.xengine_f64(S)
    assert _rel(V, _brute_xcorr(S)) < 1e-13
    # library special case: X^H X per channel (numpy matmul), lower triangle
    for k in range(K):
        X = S[:, :, k]
        G = X.conj().T @ X                                  # G[i][j] = sum_a conj(X_ai) X_aj
        il, jl = np.tril_indices(N)
        assert _rel(V[k], G[il, jl]) < 1e-13


@pytest.mark.parametrize("A,N,K", [(1, 1, 1), (4, 8, 8), (5, 3, 4)])
def test_xengine_int8_exact(orc, A, N, K):
    rng = np.random.default_rng(N + K)
    S = rng.integers(-127, 128, size=(A, N, K, 2)).astype(np.int8)
    V = orc.xengine_i8(S)
    # exact Python integers
    Sc = S.astype(object)
    for k in range(K):
        b = 0
        for i in range(N):
            for j in range(i + 1):
                re = sum(Sc[a, i, k, 0] * Sc[a, j, k, 0] + Sc[a, i, k, 1] * Sc[a, j, k, 1] for a in range(A))
                im = sum(Sc[a, i, k, 0] * Sc[a, j, k, 1] - Sc[a, i, k, 1] * Sc[a, j, k, 0] for a in range(A))
                assert V[k, b, 0] == re and V[k, b, 1] == im
                b += 1


def test_xengine_int8_worst_case_magnitude(orc):
    """All entries -127 - 127j: autos reach 2*127^2*A exactly."""
    A, N, K = 64, 3, 2
    S = np.full((A, N, K, 2), -127, np.int8)
    V = orc.xengine_i8(S)
    assert np.all(V[..., 0] == 2 * 127 * 127 * A) and np.all(V[..., 1] == 0)


def test_xengine_hermitian_under_input_reversal(orc):
    """Reversing the input order maps lower-triangle products onto the upper
    triangle: C'_uv = C_{pi(u) pi(v)} = conj(C_{pi(v) pi(u)})."""
    rng = np.random.default_rng(3)
    A, N, K = 5, 6, 3
    S = rng.standard_normal((A, N, K)) + 1j * rng.standard_normal((A, N, K))
    V = orc.xengine_f64(S)
    Vr = orc.xengine_f64(S[:, ::-1, :])
    for u in range(N):
        for v in range(u + 1):
            i, j = N - 1 - u, N - 1 - v          # j >= i: upper triangle of C
            lower = orc.tri_lower_index(j, i)
            assert abs(Vr[:, orc.tri_lower_index(u, v)] - np.conj(V[:, lower])).max() < 1e-12


def test_xengine_autos_real_nonnegative(orc):
    rng = np.random.default_rng(4)
    S = rng.standard_normal((9, 7, 5)) + 1j * rng.standard_normal((9, 7, 5))
    V = orc.xengine_f64(S)
    d = [orc.tri_lower_index(i, i) for i in range(7)]
    assert np.all(V[:, d].imag == 0) and np.all(V[:, d].real >= 0)


def test_xengine_identical_inputs(orc):
    """Inputs p and q carrying the same signal: their rows agree and C_qp = C_pp."""
    rng = np.random.default_rng(5)
    A, N, K, p, q = 6, 5, 3, 1, 3
    S = rng.standard_normal((A, N, K)) + 1j * rng.standard_normal((A, N, K))
    S[:, q] = S[:, p]
    V = orc.xengine_f64(S)
    t = orc.tri_lower_index
    assert np.allclose(V[:, t(q, p)], V[:, t(p, p)], rtol=0, atol=1e-12)
    for r in range(N):
        vp = V[:, t(max(p, r), min(p, r))]
        vq = V[:, t(max(q, r), min(q, r))]
        # C_pr and C_qr agree (conjugated where the stored index order flips)
        vp = vp if r <= p else np.conj(vp)
        vq = vq if r <= q else np.conj(vq)
        assert np.allclose(vp, vq, atol=1e-12)


def test_xengine_additivity_and_zero_padding(orc):
    rng = np.random.default_rng(6)
    A1, A2, N, K = 4, 3, 5, 2
    S = rng.standard_normal((A1 + A2, N, K)) + 1j * rng.standard_normal((A1 + A2, N, K))
    V = orc.xengine_f64(S)
    assert np.allclose(V, orc.xengine_f64(S[:A1]) + orc.xengine_f64(S[A1:]), atol=1e-12)
    Sp = np.concatenate([S, np.zeros((5, N, K))], axis=0)              # zero spectra
    assert np.array_equal(orc.xengine_f64(Sp), V)
    Sn = np.concatenate([S, np.zeros((A1 + A2, 2, K))], axis=1)        # zero inputs
    Vn = orc.xengine_f64(Sn)
    B = N * (N + 1) // 2
    assert np.array_equal(Vn[:, :B], V) and np.all(Vn[:, B:] == 0)


# ------------------------------------------------------------- F + X -------
def test_fx_parseval_on_autos(orc):
    """sum_k C_ii[k] = C * sum_n |s_i[n]|^2 over the integrated samples."""
    rng = np.random.default_rng(10)
    C, A, N = 64, 16, 4
    v = _crand(rng, (N, A * C))
    V = orc.xengine_f64(orc.fengine(v, C, A))
    for i in range(N):
        lhs = V[:, orc.tri_lower_index(i, i)].real.sum()
        rhs = C * np.sum(np.abs(v[i].astype(np.complex128)) ** 2)
        assert abs(lhs - rhs) / rhs < 1e-12


def test_fx_tone_closed_form_noise_free(orc):
    """Noise-free twin of the tiny workload: s_p[n] = a exp(j(2 pi 17 n/64 + p dphi))
    gives C_ij[17] = A (64 a)^2 exp(j dphi (j - i)); every other channel ~0.
    The phase sign pins the conjugate on the first index of Eq. 2."""
    w0 = synth.WORKLOADS["tiny-16x1-c64"]
    w = synth.Workload(w0.name, w0.n_stations, 1, 64, 32, seed=1, tone_bins=(17,), tone_amps=(1.0,),
                       tone_phase="ramp", dphi=w0.dphi, noise=False)
    v = synth.voltages(w)
    V = orc.xengine_f64(orc.fengine(v, 64, w.n_integrate))
    A, a = w.n_integrate, 1.0
    for i in range(w.n_inputs):
        for j in range(i + 1):
            ref = A * (64 * a) ** 2 * np.exp(1j * w.dphi * (j - i))
            assert abs(V[17, orc.tri_lower_index(i, j)] - ref) < 1e-5 * abs(ref)
    mask = np.ones(64, bool)
    mask[17] = False
    assert np.max(np.abs(V[mask])) < 1e-5 * A * 64 ** 2


def test_fx_tone_with_noise_phase(orc):
    """Tiny workload with noise: the tone-bin phase per baseline is within
    0.05 rad of dphi (j - i)."""
    w = synth.WORKLOADS["tiny-16x1-c64"]
    v = synth.voltages(w)
    V = orc.xengine_f64(orc.fengine(v, 64, w.n_integrate, chans=[17]))
    for i in range(w.n_inputs):
        for j in range(i):
            d = np.angle(V[0, orc.tri_lower_index(i, j)] * np.exp(-1j * w.dphi * (j - i)))
            assert abs(d) < 0.05


def test_fx_noise_statistics(orc):
    """CN(0,1) noise: E[C_ii[k]] = A C with relative spread 1/sqrt(A); crosses
    have mean ~0 and magnitude ~sqrt(A) C."""
    w = synth.Workload("noise", 6, 1, 32, 400, seed=11)
    V = orc.xengine_f64(orc.fengine(synth.voltages(w), 32, 400))
    A, C = 400, 32
    autos = np.array([V[:, orc.tri_lower_index(i, i)].real for i in range(6)])
    assert abs(autos.mean() / (A * C) - 1) < 0.02
    assert autos.std() / (A * C) < 3 / math.sqrt(A)
    cross = np.array([V[:, orc.tri_lower_index(i, j)] for i in range(6) for j in range(i)])
    assert abs(cross.mean()) < 0.05 * A * C
    assert 0.5 < np.sqrt(np.mean(np.abs(cross) ** 2)) / (math.sqrt(A) * C) < 1.5


def test_fx_delayed_station_phase_slope(orc):
    """Input 1 is input 0 delayed by d samples: C_01[k] = sum conj(S_0) S_1 has
    phase -2 pi k d / C and magnitude ~ (1 - d/C) of the auto."""
    rng = np.random.default_rng(12)
    C, A, d = 64, 800, 4
    x = _crand(rng, (A * C + d,), scale=math.sqrt(0.5))
    v = np.stack([x[d:], x[:-d]])            # v1[n] = v0[n - d]
    V = orc.xengine_f64(orc.fengine(v, C, A))
    c01 = np.conj(V[:, orc.tri_lower_index(1, 0)])   # stored C_10; C_01 = conj(C_10)
    auto = V[:, 0].real
    k = np.arange(C)
    ph = np.angle(c01 * np.exp(2j * np.pi * k * d / C))
    assert np.max(np.abs(ph)) < 0.15
    ratio = np.abs(c01) / auto
    assert abs(ratio.mean() - (1 - d / C)) < 0.03


# ----------------------------------------------------------- quantisers ----
def test_e4m3_decode_all_codes_match_torch(orc):
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    mine = orc.decode_e4m3(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(mine), nan)
    assert np.array_equal(mine[~nan], ref[~nan])
    assert np.nanmax(mine) == 448.0 and orc.decode_e4m3(np.array([0x08]))[0] == 2.0 ** -6
    assert orc.decode_e4m3(np.array([0x01]))[0] == 2.0 ** -9


def test_f16_decode_all_codes_match_numpy(orc):
    codes = np.arange(65536, dtype=np.uint16)
    mine = orc.decode_f16(codes)
    ref = codes.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(mine), nan)
    assert np.array_equal(mine[~nan], ref[~nan])


def test_e4m3_round_trip_midpoints_and_saturation(orc):
    vals = orc.decode_e4m3(np.arange(256, dtype=np.uint8))
    finite = np.unique(vals[np.isfinite(vals)])
    assert np.array_equal(orc.quant_e4m3(finite), finite)
    # midpoints between neighbours round to the one with an even mantissa
    pos = finite[finite >= 0]
    codes = {v: c for c, v in enumerate(orc.decode_e4m3(np.arange(128, dtype=np.uint8))) if np.isfinite(v)}
    for lo, hi in zip(pos[:-1], pos[1:]):
        mid = (lo + hi) / 2
        even = lo if codes[lo] % 2 == 0 else hi
        assert orc.quant_e4m3(np.array([mid]))[0] == even
        assert orc.quant_e4m3(np.array([-mid]))[0] == -even
    big = np.array([448.0, 449.0, 463.9, 464.0, 470.0, 1e6, -500.0, -1e30])
    assert np.array_equal(orc.quant_e4m3(big), [448, 448, 448, 448, 448, 448, -448, -448])


def test_e4m3_matches_torch_in_range(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    y = (rng.standard_normal(200000) * 50).astype(np.float32)
    y = y[np.abs(y) <= 448]
    ref = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(orc.quant_e4m3(y.astype(np.float64)), ref)


def test_f16_matches_numpy_and_saturates(orc):
    rng = np.random.default_rng(14)
    y = np.concatenate([rng.standard_normal(200000) * 3000, rng.standard_normal(50000) * 1e-5])
    y = y[np.abs(y) <= 65504]
    assert np.array_equal(orc.quant_f16(y), y.astype(np.float16).astype(np.float64))
    assert np.array_equal(orc.quant_f16(np.array([65504.0, 65519.0, 65520.0, 1e9, -7e4])),
                          [65504, 65504, 65504, 65504, -65504])


def test_int8_rne_and_clamp(orc):
    y = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 0.49999, 126.5, 127.4, 127.5, 300, -127.5, -1e9])
    ref = np.array([0, 2, 2, 0, -2, -2, 0, 126, 127, 127, 127, -127, -127])
    assert np.array_equal(orc.quant_int8(y), ref)
    rng = np.random.default_rng(15)
    z = rng.standard_normal(100000) * 60
    assert np.array_equal(orc.quant_int8(z), np.clip(np.rint(z), -127, 127).astype(np.int8))


def test_quantise_applies_channel_scale(orc):
    S = np.array([[3.0 + 1j, 10.0 - 4j]])
    inv = np.array([0.5, 0.25], np.float32)
    q = orc.quantise(S, inv, "int8")
    assert np.array_equal(q, [[[2, 0], [2, -1]]])       # 1.5->2, 0.5->0, 2.5->2, -1->-1


# ------------------------------------------------------------- emission ----
def test_emit_layouts_and_orders(orc):
    rng = np.random.default_rng(16)
    A, N, K = 3, 4, 2
    S = rng.standard_normal((A, N, K)) + 1j * rng.standard_normal((A, N, K))
    V = orc.xengine_f64(S)
    full = orc.emit(V, N, "full")
    for k in range(K):
        X = S[:, :, k]
        assert _rel(full[k].reshape(N, N), X.conj().T @ X) < 1e-13
    up = orc.emit(V, N, "upper")
    iu, ju = np.triu_indices(N)
    assert _rel(up, full.reshape(K, N, N)[:, iu, ju]) < 1e-15
    bm = orc.emit(V, N, "lower", "baseline")
    assert np.array_equal(bm, V.T)
    Vi = orc.xengine_i8(rng.integers(-5, 6, (A, N, K, 2)).astype(np.int8))
    fi = orc.emit(Vi, N, "full")
    assert np.array_equal(fi[:, 1, 1], -fi[:, N, 1])    # C_01 = conj(C_10)
