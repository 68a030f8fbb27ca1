"""Seeded synthetic inputs for the FX correlator (shared by the GPU path's tests
and benchmark, and by the oracle's tests).

This module holds no step of the correlator's arithmetic: it only draws
station voltages (complex baseband, CN(0,1) noise plus exact-bin point-source
tones), per-channel requantisation scales, and the named workload shapes.

Workloads follow the shapes of the paper's setting (Wang & Harris, Exp. Astron.
2013, Sections 3-5: one stream per antenna and polarisation, an FFT length
equal to the channel count, spectra integrated over time), scaled to one GPU's
frequency share of an SKA-sized array.  No telescope data is used: every input
is drawn from a seeded generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TONE_BINS = (97, 411, 808)
TONE_AMPS = (0.5, 0.35, 0.25)


@dataclass(frozen=True)
class Workload:
    name: str
    n_stations: int
    n_pols: int
    n_channels: int
    n_integrate: int
    seed: int
    tone_bins: tuple = ()
    tone_amps: tuple = ()
    # "ramp": phase p*dphi per input; "geometric": 2 pi (u_s l_t + v_s m_t)
    tone_phase: str = "geometric"
    dphi: float = 0.0
    noise: bool = True

    @property
    def n_inputs(self) -> int:
        return self.n_stations * self.n_pols

    @property
    def n_samples(self) -> int:
        return self.n_channels * self.n_integrate

    @property
    def n_products(self) -> int:
        n = self.n_inputs
        return n * (n + 1) // 2

    @property
    def cmacs(self) -> int:
        """Algorithmic complex multiply-accumulates of one integration."""
        return self.n_products * self.n_channels * self.n_integrate


WORKLOADS = {
    # 16 stations x 1 pol, 64-point FFT, 1024 spectra; common tone at channel 17
    # with a per-station phase ramp of 2 pi / 16.
    "tiny-16x1-c64": Workload("tiny-16x1-c64", 16, 1, 64, 1024, seed=1,
                              tone_bins=(17,), tone_amps=(1.0,), tone_phase="ramp",
                              dphi=2 * math.pi / 16),
    # MWA-like: 128 stations x 2 pols = 256 inputs, 1024 channels, 1000 spectra.
    "mwa-128x2-c1024": Workload("mwa-128x2-c1024", 128, 2, 1024, 1000, seed=2,
                                tone_bins=TONE_BINS, tone_amps=TONE_AMPS),
    # 256 stations x 2 pols, 2048 channels, 2048 spectra (int8 / fp16 forms).
    "int8-256x2-c2048": Workload("int8-256x2-c2048", 256, 2, 2048, 2048, seed=3,
                                 tone_bins=TONE_BINS, tone_amps=TONE_AMPS),
    # One GPU's frequency share of an SKA-sized array: 512 x 2, 4096 channels.
    "ska-512x2-c4096": Workload("ska-512x2-c4096", 512, 2, 4096, 1024, seed=4,
                                tone_bins=TONE_BINS, tone_amps=TONE_AMPS),
}


def small(name: str, n_stations: int, n_pols: int, n_channels: int, n_integrate: int,
          seed: int, tones=True) -> Workload:
    """A reduced workload with the same structure (for parity at oracle sizes)."""
    bins = tuple(b % n_channels for b in TONE_BINS[:3]) if tones else ()
    bins = tuple(sorted(set(bins)))
    amps = TONE_AMPS[: len(bins)]
    return Workload(name, n_stations, n_pols, n_channels, n_integrate, seed,
                    tone_bins=bins, tone_amps=amps)


# --------------------------------------------------------------------------
# Tone phases
# --------------------------------------------------------------------------
def tone_phases(w: Workload) -> np.ndarray:
    """Phase of each tone at each input, float64 [n_tones][n_inputs].

    ramp      : phi_p = p * dphi.
    geometric : station positions (u, v) uniform in a disc of radius 4
                wavelengths and source direction cosines (l, m) uniform in
                [-0.5, 0.5], all seeded; phi = 2 pi (u l + v m); both
                polarisations of a station share the phase.
    """
    nt = len(w.tone_bins)
    if w.tone_phase == "ramp":
        p = np.arange(w.n_inputs, dtype=np.float64)
        return np.stack([p * w.dphi for _ in range(nt)]) if nt else np.zeros((0, w.n_inputs))
    rng = np.random.default_rng([w.seed, 7919])
    r = 4.0 * np.sqrt(rng.random(w.n_stations))
    th = 2 * math.pi * rng.random(w.n_stations)
    u, v = r * np.cos(th), r * np.sin(th)
    lm = rng.random((nt, 2)) - 0.5
    ph = np.empty((nt, w.n_inputs))
    for t in range(nt):
        st = 2 * math.pi * (u * lm[t, 0] + v * lm[t, 1])
        ph[t] = np.repeat(st, w.n_pols)
    return ph


def _tone_time_part(k: int, C: int, n: np.ndarray) -> np.ndarray:
    """exp(j 2 pi k n / C) with the argument reduced exactly mod C."""
    m = (np.int64(k) * n.astype(np.int64)) % C
    return np.exp(1j * 2 * math.pi * m.astype(np.float64) / C)


# --------------------------------------------------------------------------
# Voltages
# --------------------------------------------------------------------------
def voltages(w: Workload, n_spectra: int | None = None, device: str = "cpu",
             inputs: slice | None = None):
    """Complex64 voltages [n_inputs][n_spectra * C].

    Noise is CN(0,1) (re, im iid N(0, 1/2)); each tone adds
    a_t * exp(j (2 pi k_t n / C + phi_{t,p})).

    device 'cpu' returns a numpy array drawn with numpy's PCG64 keyed by the
    seed; a torch device ('cuda', 'cuda:0') returns a torch tensor drawn on
    that device with torch's Philox generator keyed by the same seed.  The two
    streams differ; a test that compares against the oracle copies the device
    tensor to the host.
    """
    A = w.n_integrate if n_spectra is None else n_spectra
    C = w.n_channels
    T = A * C
    ph = tone_phases(w)
    rows = range(w.n_inputs) if inputs is None else range(w.n_inputs)[inputs]
    rows = np.asarray(list(rows), dtype=np.int64)
    if device == "cpu":
        rng = np.random.default_rng(w.seed)
        if w.noise:
            full = rng.standard_normal((w.n_inputs, 2 * T), dtype=np.float32)
            x = full[rows]
            x *= np.float32(math.sqrt(0.5))
            v = x.view(np.complex64)
        else:
            v = np.zeros((rows.size, T), dtype=np.complex64)
        n = np.arange(T, dtype=np.int64)
        for t, (k, a) in enumerate(zip(w.tone_bins, w.tone_amps)):
            tp = _tone_time_part(k, C, n)
            amp = a * np.exp(1j * ph[t, rows])
            v += (amp[:, None] * tp[None, :]).astype(np.complex64)
        return np.ascontiguousarray(v)

    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(w.seed))
    if w.noise:
        v = torch.randn((w.n_inputs, T), dtype=torch.complex64, device=dev, generator=g)
        if inputs is not None:
            v = v[torch.as_tensor(rows, device=dev)].contiguous()
    else:
        v = torch.zeros((rows.size, T), dtype=torch.complex64, device=dev)
    if len(w.tone_bins):
        n = np.arange(C, dtype=np.int64)
        for t, (k, a) in enumerate(zip(w.tone_bins, w.tone_amps)):
            # exact-bin tone: the time part has period C
            tp = torch.as_tensor(_tone_time_part(k, C, n).astype(np.complex64), device=dev)
            amp = torch.as_tensor((a * np.exp(1j * ph[t, rows])).astype(np.complex64), device=dev)
            vv = v.view(rows.size, A, C)
            step = max(1, (1 << 28) // max(1, A * C))
            for p0 in range(0, rows.size, step):
                vv[p0:p0 + step] += amp[p0:p0 + step, None, None] * tp[None, None, :]
    return v


# --------------------------------------------------------------------------
# Per-channel requantisation scales
# --------------------------------------------------------------------------
TARGET_RMS = {"int8": 16.0, "fp8": 8.0, "fp16": 1.0, "fp32": 1.0}


def channel_rms(w: Workload) -> np.ndarray:
    """Expected per-component RMS of the C-point spectrum at each channel.

    CN(0,1) noise contributes C/2 per component; a tone of amplitude a in its
    bin contributes (a C)^2 / 2 per component on average over phase.
    """
    C = w.n_channels
    var = np.full(C, C / 2.0) if w.noise else np.zeros(C)
    for k, a in zip(w.tone_bins, w.tone_amps):
        var[k] += (a * C) ** 2 / 2.0
    var[var == 0] = 1.0
    return np.sqrt(var)


def inv_scale(w: Workload, precision: str) -> np.ndarray:
    """float32 inv_s[k] that maps the channel RMS to the precision's target."""
    return (TARGET_RMS[precision] / channel_rms(w)).astype(np.float32)


# --------------------------------------------------------------------------
# Quantised-valued spectra for X-engine-only tests and timing
# --------------------------------------------------------------------------
def int8_spectra(n_spectra: int, n_channels: int, n_inputs: int, seed: int, rms: float = 16.0,
                 device: str = "cpu"):
    """Random int8-valued complex spectra [A][C][N][2] in [-127, 127]
    (Gaussian of the given RMS, rounded and clipped), public spectra layout."""
    shape = (n_spectra, n_channels, n_inputs, 2)
    if device == "cpu":
        rng = np.random.default_rng(seed)
        x = np.rint(rng.standard_normal(shape, dtype=np.float32) * rms)
        return np.clip(x, -127, 127).astype(np.int8)
    import torch
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    x = torch.randn(shape, device=device, generator=g) * rms
    return torch.clamp(torch.round(x), -127, 127).to(torch.int8)


# --------------------------------------------------------------------------
# 8-bit real samples (the paper's own test streams, Section 5)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class RealWorkload:
    """n_streams streams of 8-bit real samples, transform length 2C (C
    channels kept), n_integrate spectra.  Each sample is
    clip(rint(sigma g + a cos(2 pi k0 n / 2C + phi_p)), -128, 127) with g
    standard normal and phi_p = 2 pi p 3 / n_streams (a phase ramp)."""
    name: str
    n_streams: int
    n_channels: int
    n_integrate: int
    seed: int
    sigma: float = 8.0
    tone_bin: int = 37
    tone_amp: float = 6.0

    @property
    def n_inputs(self) -> int:
        return self.n_streams

    @property
    def n_products(self) -> int:
        return self.n_streams * (self.n_streams + 1) // 2

    @property
    def cmacs(self) -> int:
        return self.n_products * self.n_channels * self.n_integrate


# The paper's tests: transform length 256 (128 channels kept), 64 to 3072
# streams, up to 2048 streams on one GPU in its time-division model.
REAL_WORKLOADS = {
    f"paper-{n}-r256": RealWorkload(f"paper-{n}-r256", n, 128, 1024, seed=60 + i)
    for i, n in enumerate((128, 512, 2048, 3072))
}


def small_real(name: str, n_streams: int, n_channels: int, n_integrate: int, seed: int,
               sigma: float = 8.0, tone_amp: float = 6.0) -> RealWorkload:
    return RealWorkload(name, n_streams, n_channels, n_integrate, seed, sigma,
                        tone_bin=37 % n_channels, tone_amp=tone_amp)


def _real_tone(w: RealWorkload) -> np.ndarray:
    """a cos(2 pi k0 n / 2C + phi_p) over one period n < 2C, float64 [N][2C]."""
    L = 2 * w.n_channels
    n = np.arange(L, dtype=np.int64)
    m = (np.int64(w.tone_bin) * n) % L
    phi = 2 * math.pi * 3.0 * np.arange(w.n_streams, dtype=np.float64) / w.n_streams
    return w.tone_amp * np.cos(2 * math.pi * m[None, :] / L + phi[:, None])


def real8_samples(w: RealWorkload, n_spectra: int | None = None, device: str = "cpu"):
    """int8 real samples [n_streams][n_spectra * 2C].  'cpu' draws with
    numpy's PCG64, a torch device with torch's Philox generator (different
    streams, same distribution), both keyed by the seed."""
    A = w.n_integrate if n_spectra is None else n_spectra
    L = 2 * w.n_channels
    tone = _real_tone(w)
    if device == "cpu":
        rng = np.random.default_rng(w.seed)
        x = rng.standard_normal((w.n_streams, A, L), dtype=np.float32) * np.float32(w.sigma)
        x += tone[:, None, :].astype(np.float32)
        return np.clip(np.rint(x), -128, 127).astype(np.int8).reshape(w.n_streams, A * L)
    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(w.seed))
    out = torch.empty((w.n_streams, A * L), dtype=torch.int8, device=dev)
    t = torch.as_tensor(tone.astype(np.float32), device=dev)
    step = max(1, (1 << 27) // max(1, A * L))
    for p0 in range(0, w.n_streams, step):
        p1 = min(w.n_streams, p0 + step)
        x = torch.randn((p1 - p0, A, L), device=dev, generator=g) * w.sigma + t[p0:p1, None, :]
        out[p0:p1] = torch.clamp(torch.round(x), -128, 127).to(torch.int8).view(p1 - p0, A * L)
    return out


def real8_inv_scale(w: RealWorkload, precision: str) -> np.ndarray:
    """float32 inv_s[k] mapping the expected per-component RMS of channel k of
    the length-2C spectrum to the precision's target: noise of variance
    sigma^2 + 1/12 (the rounding) gives C (sigma^2 + 1/12) per component, the
    tone adds (a C)^2 / 2 in its channel."""
    C = w.n_channels
    var = np.full(C, C * (w.sigma ** 2 + 1.0 / 12.0))
    var[w.tone_bin] += (w.tone_amp * C) ** 2 / 2.0
    return (TARGET_RMS[precision] / np.sqrt(var)).astype(np.float32)


# --------------------------------------------------------------------------
# Batched uneven sub-arrays
# --------------------------------------------------------------------------
def batched_workloads(n_arrays: int = 64, seed: int = 5, max_channels_log2: int = 12,
                      min_stations: int = 16, max_stations: int = 512,
                      min_integrate: int = 256, max_integrate: int = 2048) -> list:
    """Sub-arrays with station counts log-uniform in [16, 512] (2 pols),
    power-of-two channel counts 2^U{8..12} and integration U{256..2048};
    Gaussian noise plus one exact-bin tone each; sub-array r is seeded (seed, r)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_arrays):
        ns = int(round(math.exp(rng.uniform(math.log(min_stations), math.log(max_stations)))))
        C = 1 << int(rng.integers(8, max_channels_log2 + 1))
        A = int(rng.integers(min_integrate, max_integrate + 1))
        k = int(rng.integers(1, C))
        out.append(Workload(f"sub{r}", ns, 2, C, A, seed=seed * 1000 + r,
                            tone_bins=(k,), tone_amps=(0.5,)))
    return out
