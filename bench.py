"""Benchmark of the FX-correlator hot path on one MI355X.

One step = one pass of the whole hot path over one integration of synthetic
voltages already resident in HBM: F-engine (channelising FFT + requantise),
X-engine (Eq. 2 over the triangle of all input pairs, autos included), and the
dump of the visibilities to a device buffer with reset, fused into the
X-engine's epilogue (corr_xengine_dump).

Default workload: 512 stations x 2 pols (1024 inputs), 4096 channels (one
GPU's frequency share of a larger array), 1024 spectra per integration, FP32
-- the paper's single-precision arithmetic -- on complex64 Gaussian voltages
plus three point-source tones.  The value is algorithmic complex
multiply-accumulates (N(N+1)/2 * C * A per step) per second of the whole step.

Also reported on one JSON line:
  roofline     -- the dominant kernel (the X-engine), timed with HIP events on
                  the correlator's stream, against the MFMA peak of its type;
  forms        -- the same step in the FP8, FP16 and int8 forms, with X-engine
                  speed-ups over FP32 (the FP8 form is this workload's own
                  reduced-precision configuration);
  pipelined    -- the main step in the steady state of a streaming correlator:
                  two handles on two streams take alternate integrations, so
                  one's F-engine overlaps the other's X-engine;
  equal_accuracy -- the same int8-valued spectra through the FP32, FP16 and
                  int8 X-engines at the 512-input x 2048-channel x 2048-spectra
                  shape: every value is exact in all three element types, so
                  the int8 result is the exact sum and the float forms differ
                  from it by accumulation rounding only;
  xengine_shapes -- X-engine alone at the larger array shapes (512 inputs x
                  2048 channels x 2048 spectra for int8 / FP16, 1024 inputs x
                  4096 channels x 1024 spectra for FP8 / FP32), against each
                  type's MFMA peak, and the caller-spectra ingest (public
                  layout into the held rows) and export at those shapes;
  batched      -- 64 uneven sub-arrays: persistent batched X-engine vs
                  per-array launches, and the graph-replayed step;
  config_steps -- whole F + X steps of the 128 x 2-input / 1024-channel (FP32)
                  and 256 x 2-input / 2048-channel (int8, FP16) workloads;
  paper_workload -- 8-bit real samples, transform length 256, 128 to 3072
                  streams (the paper's own tests), FP32 and int8;
  cpu_baseline -- the oracle (float64 direct DFT + triple-loop correlation)
                  timed on a bounded channel sample on the host cores, which
                  also gives each form's error against float64, per sampled
                  channel.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "X-engine TCMAC/s & % MFMA peak; int8/fp16 vs fp32 speed-up at stated error"
# MI355X dense peaks (TFLOP/s or TOP/s); one CMAC = 8 real operations.
PEAK = {"fp32": 157.3, "fp16": 2500.0, "fp8": 5000.0, "int8": 5000.0}
DTYPE = {"fp32": "f32", "fp16": "f16", "fp8": "e4m3", "int8": "i8"}
HBM_PEAK_GBS = 8000.0
ELEM_BYTES = {"fp32": 4, "fp16": 2, "fp8": 1, "int8": 1}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ska-512x2-c4096")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--forms", default="fp8,fp16,int8",
                    help="other precisions to time on the same workload ('' for none)")
    ap.add_argument("--equal-workload", default="int8-256x2-c2048",
                    help="shape of the equal-accuracy comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-sub-array batched (persistent, graph-captured) section")
    ap.add_argument("--batched-blocks-per-x", type=int, default=8,
                    help="F-engine time blocks appended per batched X-engine launch (8: the whole integration)")
    ap.add_argument("--batched-steps", type=int, default=8,
                    help="graph replays per integration in the batched section")
    ap.add_argument("--cpu-channels", type=int, default=16,
                    help="channels of the oracle's bounded sample (0, C/2, C-1 and the tone bins included)")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the two-stream steady-state measurement of the main step")
    ap.add_argument("--no-equal-accuracy", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the whole F + X steps of the 2048- and 4096-channel workloads")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the 8-bit real-sample section (128 to 3072 streams, transform length 256)")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the X-engine timings at the 512- and 1024-input shapes")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the F + X autotuner (block size x spectra order) on the main workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "xengine_traffic.txt"),
                    help="rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the X-engine (HBM bytes per launch)")
    return ap.parse_args()


def source_hash(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(path, key):
    """HBM bytes per X-engine launch from a rocprofv3 counter summary, or None
    when the summary is missing or was taken on a different X-engine source.
    Lines read: 'xengine_source_sha256_16 = <hash>' and
    'traffic_bytes_per_launch <workload>/<precision> = <bytes>'."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    vals = {}
    for l in lines:
        if "=" in l:
            k, v = l.split("=", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_1305_5639_amd", "csrc", "xengine.hip")
    if vals.get("xengine_source_sha256_16") != source_hash(src):
        return None
    v = vals.get(f"traffic_bytes_per_launch {key}")
    return float(v) if v else None


def x_roofline(prec, N, C, A, ms):
    """The X-engine launch against its roofline: algorithmic bytes (spectra
    read, N(N+1)/2 x C x 8-byte visibilities written on a first call), their
    rate, and the fraction of the ceiling min(MFMA peak, AI x HBM peak)
    reached, as the time at that ceiling over the measured time."""
    cm = N * (N + 1) // 2 * C * A
    nbytes = N * C * A * 2 * ELEM_BYTES[prec] + N * (N + 1) // 2 * C * 8
    t_mfma = 8 * cm / (PEAK[prec] * 1e12)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    return {"algorithmic_bytes": nbytes, "algorithmic_gbs": nbytes / (ms * 1e-3) / 1e9,
            "bound": "mfma" if t_mfma >= t_hbm else "hbm",
            "ceiling_ms": 1e3 * max(t_mfma, t_hbm), "ceiling_frac": max(t_mfma, t_hbm) / (ms * 1e-3)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Timer:
    """HIP events recorded on the correlator's stream (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.torch.cuda.current_stream())
        return e

    def stop(self, s):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.torch.cuda.current_stream())
        self.pairs.append((s, e))

    def times(self):
        return [a.elapsed_time(b) for a, b in self.pairs]

    def mean_ms(self):
        return float(np.mean(self.times())) if self.pairs else float("nan")

    def stats(self):
        t = self.times()
        return {"mean": float(np.mean(t)), "median": float(np.median(t)), "min": float(np.min(t))}


def run_form(torch, corr, synth, w, prec, volts, steps, warmup):
    """Time steps of F + X + dump, the dump fused into the X-engine
    (corr_xengine_dump writes the integration to the output buffer and
    resets); F and X timed on their own with events."""
    inv = torch.from_numpy(synth.inv_scale(w, prec)).to("cuda") if prec != "fp32" else None
    c = corr.Correlator(w.n_stations, w.n_pols, w.n_channels, w.n_integrate, prec)
    out = c.new_visibilities()
    A = w.n_integrate
    ftimer, xtimer = Timer(torch), Timer(torch)

    def step(timed):
        if timed:
            s = ftimer.start()
        c.fengine(volts, A, inv)
        if timed:
            ftimer.stop(s)
            s = xtimer.start()
        c.xengine_dump(A, out)
        if timed:
            xtimer.stop(s)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    timing = {"fengine_ms": ftimer.stats(), "xengine_and_dump_ms": xtimer.stats()}
    return c, out, inv, wall, ftimer.mean_ms(), xtimer.mean_ms(), timing


def run_autotune(torch, corr, synth, w, volts, precs):
    """corr_autotune_fx on the main workload for each precision: the chosen
    X-engine block size and spectra order, the F + X time (X timed on 256
    channels and scaled) of the built-in choice and of the chosen one, and
    whether the tuned handle's integration equals the default one's."""
    A = w.n_integrate
    out = {}
    for prec in precs:
        inv = torch.from_numpy(synth.inv_scale(w, prec)).to("cuda") if prec != "fp32" else None
        with corr.Correlator(w.n_stations, w.n_pols, w.n_channels, A, prec) as c:
            c.fengine(volts, A, inv)
            c.xengine(A)
            ref = c.dump()
        with corr.Correlator(w.n_stations, w.n_pols, w.n_channels, A, prec) as c:
            t0 = time.perf_counter()
            t = c.autotune_fx(volts, A, inv)
            torch.cuda.synchronize()
            t["tuner_s"] = time.perf_counter() - t0
            c.xengine(A)
            t["output_equal_default"] = bool(torch.equal(c.dump(), ref))
        del ref
        t["gain"] = t["ms_default"] / t["ms_tuned"] if t["ms_tuned"] > 0 else None
        out[prec] = t
        log(f"autotune {prec}: tile {t['tile']} order {t['time_block_major']}, F+X {t['ms_default']:.3f} -> "
            f"{t['ms_tuned']:.3f} ms, equal {t['output_equal_default']}")
    return out


def run_pipelined(torch, corr, w, prec, volts, steps, warmup, ref):
    """Steady state of a correlator fed integration after integration: two
    handles on two streams take alternate integrations, so the F-engine of
    one can run while the X-engine of the previous one does.  Each step is
    the same full F + X + fused dump; every output must equal the
    single-stream step's."""
    A = w.n_integrate
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    hs = [corr.Correlator(w.n_stations, w.n_pols, w.n_channels, A, prec, stream=s) for s in streams]
    outs = [h.new_visibilities() for h in hs]
    torch.cuda.synchronize()

    def step(i):
        h = hs[i % 2]
        h.fengine(volts, A)
        h.xengine_dump(A, outs[i % 2])

    for i in range(max(warmup, 2)):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    equal = all(bool(torch.equal(o, ref)) for o in outs)
    for h in hs:
        h.close()
    return wall, equal


def int8_valued(torch, shape, seed):
    """Seeded device spectra with int8 values: Gaussian, 16 LSB rms, clamped to
    +-127 (the requantiser's default operating point)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    x = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32) * 16.0
    return x.round_().clamp_(-127, 127).to(torch.int8)


def time_x(torch, c, A, reps):
    """Mean X-engine time on held spectra, first call of an integration each
    time (the accumulators are reset by a device dump in between, untimed)."""
    dst = c.new_visibilities()
    ts = []
    for _ in range(reps):
        c.dump(dst, reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.xengine(A)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return dst, sum(ts) / len(ts)


def run_equal_accuracy(torch, corr, w, reps=5):
    """Same int8-valued spectra into the FP32, FP16 and int8 X-engines."""
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    S8 = int8_valued(torch, (A, C, N, 2), seed=7)
    cm = N * (N + 1) // 2 * C * A
    out, vis = {}, {}
    for prec in ("int8", "fp16", "fp32"):
        S = S8 if prec == "int8" else S8.to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]])
        c = corr.Correlator(w.n_stations, w.n_pols, C, A, prec)
        c.xengine(A, S)                                # ingest the caller spectra
        del S
        v, ms = time_x(torch, c, A, reps)
        c.xengine(A)
        c.dump(v, reset=True)
        vis[prec] = v.to(torch.float64)
        c.close()
        out[prec] = {"xengine_ms": ms, "xengine_tcmacs": cm / (ms * 1e-3) / 1e12,
                     "mfma_frac": 8 * cm / (ms * 1e-3) / 1e12 / PEAK[prec]}
    del S8
    exact = vis["int8"][..., 0] + 1j * vis["int8"][..., 1]    # [C, B]
    d = exact.real[:, torch.tensor([i * (i + 1) // 2 + i for i in range(N)], device=exact.device)]
    il, jl = (torch.as_tensor(x, device=exact.device) for x in np.tril_indices(N))
    norm = torch.sqrt(torch.clamp(d[:, il] * d[:, jl], min=1e-300))
    for prec in ("fp16", "fp32"):
        g = vis[prec][..., 0] + 1j * vis[prec][..., 1]
        eF = torch.linalg.norm(g - exact, dim=1) / torch.linalg.norm(exact, dim=1)
        en = torch.abs(g - exact) / norm
        out[prec]["error_vs_exact"] = {"max_rel_frobenius": float(eF.max()), "max_normalised": float(en.max())}
        out[prec]["speedup_vs_fp32"] = out["fp32"]["xengine_ms"] / out[prec]["xengine_ms"]
    out["int8"]["error_vs_exact"] = {"max_rel_frobenius": 0.0, "max_normalised": 0.0}
    out["int8"]["speedup_vs_fp32"] = out["fp32"]["xengine_ms"] / out["int8"]["xengine_ms"]
    out["fp32"]["speedup_vs_fp32"] = 1.0
    del vis, exact, d, norm
    torch.cuda.empty_cache()
    return {"workload": f"{w.name}: int8-valued spectra (16 LSB rms) shared by all three forms", **out}


def run_shapes(torch, corr, reps=3):
    """X-engine alone at the 512- and 1024-input shapes, int8-valued spectra."""
    res = {}
    for name, prec, st, C, A in (("512x2048x2048", "int8", 256, 2048, 2048),
                                 ("512x2048x2048", "fp16", 256, 2048, 2048),
                                 ("1024x4096x1024", "fp8", 512, 4096, 1024),
                                 ("1024x4096x1024", "fp32", 512, 4096, 1024)):
        N = 2 * st
        S = int8_valued(torch, (A, C, N, 2), seed=11)
        if prec != "int8":
            S = S.to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]])
        c = corr.Correlator(st, 2, C, A, prec)
        c.xengine(A, S)
        # caller spectra: the same first call, ingest (public layout -> held
        # rows) included; the ingest is its excess over the held-spectra call
        dst = c.new_visibilities()
        ts = []
        for _ in range(reps):
            c.dump(dst, reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            c.xengine(A, S)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        caller_ms = sum(ts) / len(ts)
        nbytes = S.numel() * S.element_size()
        del S, dst
        torch.cuda.empty_cache()
        dst, ms = time_x(torch, c, A, reps)
        del dst
        out = c.spectra()                          # export: held rows -> public layout
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            corr.corr_copy_spectra(c.handle, out)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        del out
        export_ms = sum(ts) / len(ts)
        torch.cuda.empty_cache()
        ingest_ms = caller_ms - ms
        cm = N * (N + 1) // 2 * C * A
        tc = cm / (ms * 1e-3) / 1e12
        res[f"{prec}/{name}"] = {"inputs": N, "channels": C, "spectra": A, "xengine_ms": ms,
                                 "xengine_tcmacs": tc, "mfma_frac": 8 * tc / PEAK[prec],
                                 "spectra_bytes": nbytes, "caller_spectra_xengine_ms": caller_ms,
                                 "ingest_ms": ingest_ms, "ingest_tbs": 2 * nbytes / (ingest_ms * 1e-3) / 1e12,
                                 "export_ms": export_ms, "export_tbs": 2 * nbytes / (export_ms * 1e-3) / 1e12,
                                 "x_roofline": x_roofline(prec, N, C, A, ms)}
        log(f"shape {name} {prec}: X {ms:.3f} ms, {tc:.1f} TCMAC/s, {100 * 8 * tc / PEAK[prec]:.1f}% of MFMA peak; "
            f"{nbytes / 1e9:.2f} GB caller spectra in {ingest_ms:.2f} ms, out {export_ms:.2f} ms")
        c.close()
        torch.cuda.empty_cache()
    # Rectangle (cross-only) X-engine: inputs [512, 1024) against [0, 512),
    # 2048 channels x 2048 spectra -- a space-division node's product.
    for prec in ("int8", "fp16"):
        N, C, A, h = 1024, 2048, 2048, 512
        S = int8_valued(torch, (A, C, N, 2), seed=12)
        if prec != "int8":
            S = S.to(corr.SPECTRA_DTYPE[corr.PRECISIONS[prec]])
        c = corr.Correlator(N // 2, 2, C, A, prec)
        c.xengine(A, S)
        del S
        torch.cuda.empty_cache()
        out = c.xengine_rect(h, N - h, 0, h, A)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            c.xengine_rect(h, N - h, 0, h, A, out=out)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sum(ts) / len(ts)
        cm = (N - h) * h * C * A
        tc = cm / (ms * 1e-3) / 1e12
        res[f"{prec}/rect512x512-of-1024x2048x2048"] = {"rows": N - h, "cols": h, "channels": C, "spectra": A,
                                                         "xengine_ms": ms, "xengine_tcmacs": tc,
                                                         "mfma_frac": 8 * tc / PEAK[prec]}
        log(f"rectangle 512x512 {prec}: X {ms:.3f} ms, {tc:.1f} TCMAC/s, {100 * 8 * tc / PEAK[prec]:.1f}% of MFMA peak")
        del out
        c.close()
        torch.cuda.empty_cache()
    return res


def run_config_steps(torch, corr, synth, reps=3):
    """Whole F + X steps (dump fused) of the other configured workloads:
    128 x 2 inputs, 1024 channels, 1000 spectra in FP32; 256 x 2 inputs, 2048
    channels, 2048 spectra in int8 and FP16.  Voltages drawn on the device."""
    res = {}
    for name, precs in (("mwa-128x2-c1024", ("fp32",)), ("int8-256x2-c2048", ("int8", "fp16"))):
        w = synth.WORKLOADS[name]
        N, C, A = w.n_inputs, w.n_channels, w.n_integrate
        volts = synth.voltages(w, device="cuda")
        for prec in precs:
            inv = torch.from_numpy(synth.inv_scale(w, prec)).to("cuda")
            c = corr.Correlator(w.n_stations, w.n_pols, C, A, prec)
            out = c.new_visibilities()
            c.fengine(volts, A, inv)
            c.xengine_dump(A, out)
            ft, xt = Timer(torch), Timer(torch)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s_ = ft.start()
                c.fengine(volts, A, inv)
                ft.stop(s_)
                s_ = xt.start()
                c.xengine_dump(A, out)
                xt.stop(s_)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            f_ms, x_ms = ft.mean_ms(), xt.mean_ms()
            cm = w.cmacs
            res[f"{prec}/{name}"] = {
                "inputs": N, "channels": C, "spectra": A, "step_ms": wall * 1e3, "fengine_ms": f_ms,
                "xengine_ms": x_ms, "step_tcmacs": cm / wall / 1e12,
                "xengine_tcmacs": cm / (x_ms * 1e-3) / 1e12,
                "xengine_mfma_frac": 8 * cm / (x_ms * 1e-3) / 1e12 / PEAK[prec],
                "fengine_hbm_gbs": N * A * C * (8 + 2 * ELEM_BYTES[prec]) / (f_ms * 1e-3) / 1e9}
            log(f"config {name} {prec}: step {wall * 1e3:.2f} ms, F {f_ms:.2f} ms "
                f"({res[f'{prec}/{name}']['fengine_hbm_gbs'] / 1e3:.2f} TB/s), X {x_ms:.2f} ms "
                f"({100 * res[f'{prec}/{name}']['xengine_mfma_frac']:.1f}% of MFMA peak)")
            del out
            c.close()
            torch.cuda.empty_cache()
        del volts
        torch.cuda.empty_cache()
    return res


def run_fused_fx(torch, corr, synth, reps=3):
    """F and X fused over time chunks (corr_fx) on 256 x 2 inputs, 2048
    channels, 2048 spectra, int8, beside the unfused F + X.  A chunk of
    64 spectra (one time block, 134 MB of int8 spectra) fits the memory-side
    cache; every chunk after the first reads and writes the 2.15 GB of
    accumulators once more."""
    w = synth.WORKLOADS["int8-256x2-c2048"]
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    volts = synth.voltages(w, device="cuda")
    inv = torch.from_numpy(synth.inv_scale(w, "int8")).to("cuda")
    acc_bytes = C * N * (N + 1) // 2 * 8
    res = {"workload": f"{w.name}: int8", "accumulator_bytes": acc_bytes}
    dst = None
    for chunk in (64, 256, 1024, A):
        c = corr.Correlator(w.n_stations, w.n_pols, C, chunk, "int8")
        dst = c.new_visibilities()
        fn = (lambda: (c.fengine(volts, A, inv), c.xengine(A))) if chunk == A else (lambda: c.fx(volts, A, inv, chunk))
        fn()
        c.dump(dst, reset=True)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
            c.dump(dst, reset=True)
        ms = float(np.median(ts))
        n_chunks = -(-A // chunk)
        key = "unfused" if chunk == A else f"chunk_{chunk}"
        res[key] = {"chunk_spectra": chunk, "chunks": n_chunks, "fx_ms": ms, "tcmacs": w.cmacs / (ms * 1e-3) / 1e12,
                    "extra_accumulator_bytes": 2 * (n_chunks - 1) * acc_bytes,
                    "spectra_bytes_per_chunk": N * C * 2 * min(chunk, A)}
        log(f"fused FX int8 chunk {chunk}: {ms:.2f} ms")
        c.close()
        del dst
        torch.cuda.empty_cache()
    del volts
    torch.cuda.empty_cache()
    return res


def run_paper_workload(torch, corr, synth, reps=3):
    """The paper's own test streams (Section 5): 8-bit real samples, transform
    length 256 (128 channels), 1024 spectra, 128 to 3072 streams; the
    real-input F-engine and the X-engine in FP32 (the paper's precision) and
    int8.  Rates in the paper's counting too: 2.5 L log2 L flops per real
    transform of length L and 8 per CMAC."""
    res = {}
    for name in ("paper-128-r256", "paper-512-r256", "paper-2048-r256", "paper-3072-r256"):
        w = synth.REAL_WORKLOADS[name]
        N, C, A = w.n_streams, w.n_channels, w.n_integrate
        L = 2 * C
        x = synth.real8_samples(w, device="cuda")
        for prec in ("fp32", "int8"):
            inv = torch.from_numpy(synth.real8_inv_scale(w, prec)).to("cuda") if prec == "int8" else None
            c = corr.Correlator(N, 1, C, A, prec)
            dst = c.new_visibilities()
            c.fengine_real8(x, A, inv)                 # warm-up
            c.xengine(A)
            c.dump(dst, reset=True)
            ft, xt = Timer(torch), Timer(torch)
            for _ in range(reps):
                s = ft.start()
                c.fengine_real8(x, A, inv)
                ft.stop(s)
                s = xt.start()
                c.xengine(A)
                xt.stop(s)
                c.dump(dst, reset=True)
            torch.cuda.synchronize()
            f_ms, x_ms = ft.mean_ms(), xt.mean_ms()
            step = f_ms + x_ms
            cm = w.cmacs
            flops = N * A * 2.5 * L * math.log2(L) + 8.0 * cm
            res[f"{prec}/{name}"] = {
                "streams": N, "transform_length": L, "channels": C, "spectra": A,
                "fengine_ms": f_ms, "xengine_ms": x_ms, "fx_ms": step,
                "xengine_tcmacs": cm / (x_ms * 1e-3) / 1e12,
                "xengine_mfma_frac": 8 * cm / (x_ms * 1e-3) / 1e12 / PEAK[prec],
                "fengine_hbm_gbs": N * A * (L + 2 * C * ELEM_BYTES[prec]) / (f_ms * 1e-3) / 1e9,
                "fx_gflops_paper_count": flops / (step * 1e-3) / 1e9,
                "samples_per_s_per_stream": A * L / (step * 1e-3)}
            log(f"paper workload {name} {prec}: F {f_ms:.3f} ms, X {x_ms:.3f} ms, "
                f"{res[f'{prec}/{name}']['fx_gflops_paper_count']:.0f} GFLOPS (paper count), "
                f"{res[f'{prec}/{name}']['samples_per_s_per_stream'] / 1e6:.1f} Msample/s per stream")
            del dst
            c.close()
            torch.cuda.empty_cache()
        del x
        torch.cuda.empty_cache()
    return {"reference": "paper: ~105 GFLOPS for F + X on one Tesla C2075 (single precision, 8-bit "
                         "real samples, transform length 256); context, not a target", **res}


def sample_channels(w, n_chan):
    """The oracle's bounded channel sample: 0, C/2, C-1, the tone bins and
    seeded others, n_chan in all."""
    C = w.n_channels
    rng = np.random.default_rng(12345)
    base = {0, C // 2, C - 1, *[b for b in w.tone_bins if b < C]}
    others = [int(x) for x in rng.permutation(C) if int(x) not in base]
    return sorted(base | set(others[: max(0, n_chan - len(base))]))


def cpu_baseline(torch, oracle, synth, w, volts, results, chans):
    """The oracle on a channel sample of the same integration; errors per form
    (results hold each form's visibilities of the sampled channels)."""
    C, N, A = w.n_channels, w.n_inputs, w.n_integrate
    log(f"cpu_baseline: copying voltages to the host, oracle on {len(chans)} channels")
    v = volts.cpu().numpy()
    t0 = time.perf_counter()
    S = oracle.fengine(v, C, A, chans)
    V64 = oracle.xengine_f64(S)
    t = time.perf_counter() - t0
    B = N * (N + 1) // 2
    cmacs = B * len(chans) * A
    errors = {}
    il, jl = np.tril_indices(N)
    d = np.real(V64[:, [i * (i + 1) // 2 + i for i in range(N)]])
    norm = np.sqrt(np.maximum(d[:, il] * d[:, jl], 1e-300))
    for prec, (vis, s2) in results.items():
        g = vis.astype(np.float64)
        g = g[..., 0] + 1j * g[..., 1]
        if s2 is not None:
            g = g * s2[chans][:, None]
        eF = np.linalg.norm(g - V64, axis=1) / np.linalg.norm(V64, axis=1)
        en = np.abs(g - V64) / norm
        errors[prec] = {"max_rel_frobenius": float(eF.max()), "max_normalised": float(en.max()),
                        "per_channel": {"channels": [int(k) for k in chans],
                                        "rel_frobenius": [float(x) for x in eF],
                                        "max_normalised": [float(x) for x in en.max(axis=1)]}}
    return {
        "value": cmacs / t / 1e12,
        "unit": "TCMAC/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": (f"float64 direct DFT (Eq. 1) + triple-loop correlation (Eq. 2) of {len(chans)} of "
                   f"{C} channels, all {N} inputs x {A} spectra of the same integration; "
                   f"{cmacs:.3e} CMAC in {t:.2f} s"),
        "seconds": t,
        "host": host_cpu(),
    }, errors


def host_cpu():
    """CPU model (name, family / model / stepping numbers, clock), logical CPU
    count and the threads this process may use, of the host the oracle ran on."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if info:
                    break
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            if k in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                info[k] = v
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return {"model": info.get("model name", ""), "vendor": info.get("vendor_id", ""),
            "family_model_stepping": [info.get("cpu family"), info.get("model"), info.get("stepping")],
            "mhz": info.get("cpu MHz"), "logical_cpus": os.cpu_count(), "usable_cpus": allowed}


def run_batched(torch, corr, synth, steps_per_integration, blocks_per_x=4, reps=3):
    """64 uneven sub-arrays, FP16 in / FP32 accumulate.  Each sub-array's
    integration A_s is channelised in `steps_per_integration` time blocks of
    n_s = ceil(A_s / steps) spectra (rounded up to whole 32-spectrum time
    blocks), appended into its held spectra; every `blocks_per_x` blocks ONE
    persistent X-engine launch correlates all sub-arrays' held spectra, so the
    accumulators are read and written steps / blocks_per_x times per
    integration.  One graph replay = blocks_per_x x 64 F-engine launches + the
    batched X-engine.  Reports the X-engine as one batched launch vs 64
    per-array launches (same tuned block sizes), and the graph-replayed step."""
    prec = "fp16"
    tb = 32
    ws = synth.batched_workloads()
    ns = [-(-(-(-w.n_integrate // steps_per_integration)) // tb) * tb for w in ws]
    held = [blocks_per_x * n for n in ns]
    shapes = [(w.n_stations, w.n_pols, w.n_channels, h) for w, h in zip(ws, held)]
    cm_step = sum(w.n_products * w.n_channels * h for w, h in zip(ws, held))
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        volts, invs = [], []
        for w, n in zip(ws, ns):
            volts.append(synth.voltages(w, n_spectra=n, device="cuda"))
            invs.append(torch.from_numpy(synth.inv_scale(w, prec)).to("cuda"))
        b = corr.Batch(shapes, prec, stream=stream)

        def f_blocks():
            for blk in range(blocks_per_x):
                for i, sub in enumerate(b.subs):
                    sub.fengine(volts[i], ns[i], invs[i], first_spectrum=blk * ns[i])

        t0 = time.perf_counter()
        f_blocks()
        tiles = [sub.autotune(h) for sub, h in zip(b.subs, held)]
        tune_s = time.perf_counter() - t0
        b.xengine(held)                                        # warm-up; fixes the work list
        stream.synchronize()

        def timed(fn, k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(k):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / k

        def per_array():
            for sub, h in zip(b.subs, held):
                sub.xengine(h)

        per_array()
        t_per = timed(per_array, reps)
        t_bat = timed(lambda: b.xengine(held), reps)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            f_blocks()
            b.xengine(held)
        g.replay()
        replays = max(1, steps_per_integration // blocks_per_x)
        t_step = timed(g.replay, replays)
        stream.synchronize()
        b.close()
        del volts, invs
    torch.cuda.empty_cache()
    # integration against its roofline: the FP16 MFMA peak for the X-engine
    # work, and the HBM bytes of the whole integration (voltages read and
    # FP16 spectra written by the F-engines, spectra read and visibilities
    # written by the X-engines, a read of the visibilities for every X call
    # after the first)
    integ_s = t_step * replays * 1e-3
    cm_integ = cm_step * replays
    x_calls = replays
    v_bytes = sum(w.n_inputs * n * w.n_channels * 8 for w, n in zip(ws, ns)) * steps_per_integration
    s_bytes = sum(w.n_inputs * w.n_channels * 4 * h for w, h in zip(ws, held)) * replays
    a_bytes = sum(w.n_products * w.n_channels * 8 for w in ws)
    hbm = v_bytes + 2 * s_bytes + a_bytes * (1 + 2 * (x_calls - 1))
    out = {
        "workload": "batched-64: 64 sub-arrays, stations log-uniform 16..512 x 2 pols, "
                    "channels 2^(8..12), integration 256..2048 (seed 5), FP16 in / FP32 accumulate",
        "n_subarrays": len(ws),
        "spectra_per_fengine_block": ns,
        "fengine_blocks_per_xengine": blocks_per_x,
        "cmac_per_step": cm_step,
        "tiles": tiles,
        "autotune_s": tune_s,
        "xengine_batched_ms": t_bat,
        "xengine_per_array_ms": t_per,
        "xengine_batched_tcmacs": cm_step / (t_bat * 1e-3) / 1e12,
        "xengine_per_array_tcmacs": cm_step / (t_per * 1e-3) / 1e12,
        "batched_speedup_vs_per_array": t_per / t_bat,
        "graph_step_ms": t_step,
        "graph_step_tcmacs": cm_step / (t_step * 1e-3) / 1e12,
        "integration_ms": t_step * replays,
        "graph_steps_per_integration": replays,
        "integration_roofline": {
            "cmac": cm_integ, "tcmacs": cm_integ / integ_s / 1e12,
            "mfma_frac": 8 * cm_integ / integ_s / 1e12 / PEAK[prec],
            "hbm_bytes": hbm, "hbm_gbs": hbm / integ_s / 1e9, "hbm_frac": hbm / integ_s / 1e9 / HBM_PEAK_GBS,
            "min_ms_at_peaks": 1e3 * max(8 * cm_integ / (PEAK[prec] * 1e12), hbm / (HBM_PEAK_GBS * 1e9))},
    }
    return out


def run_batched_small(torch, corr, synth, reps=5):
    """64 small sub-arrays (16..64 stations x 2 pols, 256..1024 channels,
    integration 256..2048; seed 6), FP16: one batched persistent X-engine
    launch against 64 per-array launches on the same held spectra."""
    prec = "fp16"
    ws = synth.batched_workloads(n_arrays=64, seed=6, max_channels_log2=10, min_stations=16, max_stations=64)
    shapes = [(w.n_stations, w.n_pols, w.n_channels, w.n_integrate) for w in ws]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = corr.Batch(shapes, prec, stream=stream)
        for i, w in enumerate(ws):
            v = synth.voltages(w, device="cuda")
            b.subs[i].fengine(v, w.n_integrate, torch.from_numpy(synth.inv_scale(w, prec)).to("cuda"))
            del v
        n = [w.n_integrate for w in ws]
        b.xengine(n)

        def per_array():
            for sub, a in zip(b.subs, n):
                sub.xengine(a)

        per_array()
        stream.synchronize()

        def timed(fn, k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(k):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / k

        t_per = timed(per_array, reps)
        t_bat = timed(lambda: b.xengine(n), reps)
        b.close()
    torch.cuda.empty_cache()
    cm = sum(w.n_products * w.n_channels * w.n_integrate for w in ws)
    return {"workload": "batched-small-64: 64 sub-arrays, stations log-uniform 16..64 x 2 pols, channels "
                        "2^(8..10), integration 256..2048 (seed 6), FP16 in / FP32 accumulate",
            "cmac_per_call": cm, "xengine_batched_ms": t_bat, "xengine_per_array_ms": t_per,
            "xengine_batched_tcmacs": cm / (t_bat * 1e-3) / 1e12,
            "xengine_per_array_tcmacs": cm / (t_per * 1e-3) / 1e12,
            "batched_speedup_vs_per_array": t_per / t_bat}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the correlator runs on one GPU; --gpus must be 1 "
                          "(splitting channels across GPUs is not implemented)"}))
        print("bench.py: only --gpus 1 is supported", file=sys.stderr)
        return 2

    import torch

    import paper_1305_5639_amd as corr
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # A plain copy of known size: 1 GiB read + 1 GiB written per launch.
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB device-to-device (elementwise copy kernel)")
        del src, dst
    w = synth.WORKLOADS[args.workload]
    N, C, A = w.n_inputs, w.n_channels, w.n_integrate
    B = N * (N + 1) // 2
    cmacs = B * C * A
    log(f"workload {w.name}: {N} inputs, {C} channels, {A} spectra, {cmacs:.3e} CMAC per step")
    volts = synth.voltages(w, device="cuda")
    torch.cuda.synchronize()

    prec = args.precision
    c, out, inv, wall, f_ms, x_ms, timing = run_form(torch, corr, synth, w, prec, volts, args.steps, args.warmup)
    s2_main = None
    if prec == "int8":
        s2_main = 1.0 / synth.inv_scale(w, prec).astype(np.float64) ** 2
    chans = sample_channels(w, args.cpu_channels)
    results = {prec: (out[chans].cpu().numpy(), s2_main)}
    c.close()
    log(f"{prec}: step {wall * 1e3:.3f} ms, F {f_ms:.3f} ms, X {x_ms:.3f} ms")
    pipelined = None
    if not args.no_pipelined and prec == "fp32":
        wall_p, equal_p = run_pipelined(torch, corr, w, prec, volts, args.steps, args.warmup, out)
        pipelined = {"ms_per_step": wall_p * 1e3, "step_tcmacs": cmacs / wall_p / 1e12,
                     "speedup_vs_one_stream": wall / wall_p, "outputs_equal_one_stream": equal_p,
                     "streams": 2, "handles": 2}
        log(f"{prec} two streams: step {wall_p * 1e3:.3f} ms ({wall / wall_p:.3f}x), outputs equal: {equal_p}")

    x_flops = 8.0 * cmacs
    x_achieved = x_flops / (x_ms * 1e-3) / 1e12
    traffic = read_traffic(args.traffic_file, f"{w.name}/{prec}")
    roofline = {"kernel": f"xengine_kernel<{prec}>", "bound": "mfma", "achieved": x_achieved,
                "peak": PEAK[prec], "unit": "TFLOP/s", "frac": x_achieved / PEAK[prec],
                "traffic": traffic}

    forms = {}
    for fp in [f for f in args.forms.split(",") if f and f != prec]:
        cf, of, invf, wall_f, f_ms_f, x_ms_f, timing_f = run_form(torch, corr, synth, w, fp, volts, args.steps,
                                                                   args.warmup)
        s2 = None
        if fp == "int8":
            s2 = 1.0 / synth.inv_scale(w, fp).astype(np.float64) ** 2
        results[fp] = (of[chans].cpu().numpy(), s2)
        cf.close()
        del of
        xt = cmacs / (x_ms_f * 1e-3) / 1e12
        forms[fp] = {"ms_per_step": wall_f * 1e3, "fengine_ms": f_ms_f, "xengine_ms": x_ms_f,
                     "fengine_hbm_gbs": (N * A * C * (8 + 2 * ELEM_BYTES[fp])) / (f_ms_f * 1e-3) / 1e9,
                     "xengine_tcmacs": xt, "xengine_mfma_frac": 8 * xt / PEAK[fp],
                     "xengine_speedup_vs_fp32": x_ms / x_ms_f if prec == "fp32" else None,
                     "step_tcmacs": cmacs / wall_f / 1e12, "timing": timing_f,
                     "x_roofline": x_roofline(fp, N, C, A, x_ms_f)}
        log(f"{fp}: step {wall_f * 1e3:.3f} ms, F {f_ms_f:.3f} ms, X {x_ms_f:.3f} ms")

    tuned = None
    if not args.no_autotune:
        tuned = run_autotune(torch, corr, synth, w, volts, [prec] + list(forms))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu, errors = cpu_baseline(torch, oracle, synth, w, volts, results, chans)
        for fp, e in errors.items():
            if fp != prec:
                forms[fp]["error_vs_float64"] = e
        if prec in errors:
            cpu["error_vs_float64_" + prec] = errors[prec]
    del volts, out, results
    torch.cuda.empty_cache()

    equal = None
    if not args.no_equal_accuracy:
        equal = run_equal_accuracy(torch, corr, synth.WORKLOADS[args.equal_workload])
        log("equal accuracy: X " + ", ".join(f"{p} {equal[p]['xengine_ms']:.3f} ms" for p in ("fp32", "fp16", "int8")))
    shapes = None
    if not args.no_shapes:
        shapes = run_shapes(torch, corr)

    configs = None
    if not args.no_configs:
        configs = run_config_steps(torch, corr, synth)

    fused = None
    if not args.no_configs:
        fused = run_fused_fx(torch, corr, synth)

    paper = None
    if not args.no_paper:
        paper = run_paper_workload(torch, corr, synth)

    batched = None
    if not args.no_batched:
        log("batched: 64 small sub-arrays")
        small = run_batched_small(torch, corr, synth)
        log(f"batched small: X {small['xengine_batched_ms']:.3f} ms (one launch) vs "
            f"{small['xengine_per_array_ms']:.3f} ms (64 launches)")
        log("batched: 64 uneven sub-arrays")
        batched = run_batched(torch, corr, synth, args.batched_steps, args.batched_blocks_per_x)
        log(f"batched: X {batched['xengine_batched_ms']:.3f} ms (one launch) vs "
            f"{batched['xengine_per_array_ms']:.3f} ms (64 launches); graph step {batched['graph_step_ms']:.3f} ms; "
            f"integration {batched['integration_ms']:.1f} ms")
        batched["small_subarrays"] = small

    line = {
        "metric": METRIC,
        "value": cmacs / wall / 1e12,
        "unit": "TCMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic (seeded complex Gaussian voltages plus point-source tones, resident in HBM)",
        "config": {"workload": w.name, "n_stations": w.n_stations, "n_pols": w.n_pols,
                   "n_inputs": N, "n_channels": C, "n_integrate": A, "precision": prec,
                   "products": B, "cmac_per_step": cmacs,
                   "step": "F-engine + X-engine with the dump to a device buffer (reset) fused into its epilogue"},
        "xengine_ms": x_ms,
        "fengine_ms": f_ms,
        "xengine_tcmacs": cmacs / (x_ms * 1e-3) / 1e12,
        "fengine_hbm_gbs": (N * A * C * (8 + 2 * ELEM_BYTES[prec])) / (f_ms * 1e-3) / 1e9,
        "timing": timing,
        "roofline": roofline,
        "x_roofline": x_roofline(prec, N, C, A, x_ms),
        "forms": forms,
        "pipelined": pipelined,
        "autotune": tuned,
        "equal_accuracy": equal,
        "xengine_shapes": shapes,
        "batched": batched,
        "config_steps": configs,
        "fused_fx": fused,
        "paper_workload": paper,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
