#!/usr/bin/env python3
"""PLV / iPLV / ciPLV throughput on one MI355X.

Workload (sensor/ROI scale): N = 1024 analytic signals of T = 60000 samples
(60 s at 1 kHz) as complex64 [N, T], from the seeded lagged-oscillator
generator with 32 latent 8-12 Hz oscillators, zero-lag mixing 0.3 on channel
pairs and N(0, 0.5) noise.  One step = one plv_from_analytic call: phasor
normalisation, the upper-triangle Gram on MFMA, the chunk sum and the fused
PLV/iPLV/ciPLV epilogue with mirrored stores, inputs already in HBM.

value = pair-samples/s of the split-BF16 path, pair-samples = N(N-1)/2 * T.
The plain FP32 path runs on the same input for comparison, and both are
checked against the FP64 oracle on a sample of pairs (in the CPU-baseline
leg, which also times the oracle).

Other workloads (--workload; each prints its own JSON line, same
conventions): ``small`` N = 64 real f64 signals, T = 2048 at 256 Hz, FP64
end to end; ``batch`` 512 trials of uneven N in {68, 148, 360, 1000} and T in
[500, 4000] at 1 kHz, five 4 Hz bands each, real f32, FFT analytic signal and
one grouped Gram launch; ``grad`` N = 2048 real f32 signals, T = 8192,
forward plus adjoint of the ciPLV target loss; ``brain`` N = 15000 unit
phasors, T = 1.2e6 (144 GB of complex64 made on the GPU), 200 planted lagged
pairs, 16-bit MFMA with FP64 sums across K-chunks; ``coherence`` coherency of
N = 1024 complex coefficient rows x T = 60000; ``trials`` PLV across 40 trials
for 148 signals at each of 4000 time points.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PLV/ciPLV pair-samples/s + %MFMA peak, split-BF16 vs FP32 at stated err"
PEAK_TFLOPS = {"split_bf16": 2500.0, "bf16": 2500.0, "f16": 2500.0, "f32": 157.3, "f64": 78.6}
# MFMA flops the contraction performs per pair-sample: one complex
# multiply-add is 4 real multiply-adds (8 flops); the split form does three.
FLOP_PER_PAIR_SAMPLE = {"split_bf16": 24, "bf16": 8, "f16": 8, "f32": 8, "f64": 8}
N_SIG, T_SAMP, FS = 1024, 60000, 1000.0


def step_times(fn, steps, warmup):
    """Run fn() `warmup` times untimed, then `steps` times, each between its
    own pair of events on the current stream (the stream the library
    launches on), with per-stage timing on.  Returns (median ms per step,
    mean ms per step, stage sums, per-call Gram launch times)."""
    import statistics

    import torch

    import paper_1710_08037_amd as plv

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    plv.timing_enable(True)
    plv.timing_read(reset=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    gram = [ms / max(ln, 1) for ms, ln in plv.timing_list("gram")]
    stages = plv.timing_read(reset=True)
    plv.timing_enable(False)
    return statistics.median(per), sum(per) / len(per), stages, gram


def run_gpu(z, prec, steps, warmup):
    import paper_1710_08037_amd as plv

    return step_times(lambda: plv.from_analytic(z, prec=prec), steps, warmup)


# arithmetic type each precision mode computes in (the Gram's MFMA inputs)
DTYPE = {"split_bf16": "bf16x3 (split hi+lo, fp32 accumulate)", "bf16": "bf16", "f16": "f16", "f32": "f32",
         "f64": "f64"}


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("herk.hip", "metrics.h", "plv_internal.h", "plv_plan.cpp"):
        with open(os.path.join(ROOT, "paper_1710_08037_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch recorded from rocprofv3 counters in profiles/traffic.txt,
    or None when the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    cur = _source_hash()
    with open(path) as fh:
        for line in fh:
            tok = line.split("#", 1)[0].split()
            if len(tok) >= 5 and tok[0] == kernel and tok[4] == workload and tok[1] == cur:
                return int(tok[2]) + int(tok[3])
    return None


def issued_flops(prec, n, t, bm=None):
    """MFMA work the Gram kernel issues: whole BM x BM tiles of the upper
    triangle (diagonal tiles in full, rows padded to the tile) over K padded
    to 32 samples.  bm: the tile edge (default: the largest of the mode)."""
    if bm is None:
        bm = 64 if prec == "f64" else 128
    ntile = -(-n // bm)
    return FLOP_PER_PAIR_SAMPLE[prec] * (ntile * (ntile + 1) // 2) * bm * bm * (-(-t // 32) * 32)


def roofline(prec, n, t, stages, gram_launch_ms):
    """Roofline of the Gram kernel from the median of its per-launch times
    (HIP events recorded by the library on the stream it launches on)."""
    import statistics

    per_launch_s = statistics.median(gram_launch_ms) / 1e3
    mean_launch_s = stages["gram"][0] / max(stages["gram"][2], 1) / 1e3
    flops = FLOP_PER_PAIR_SAMPLE[prec] * (n * (n - 1) // 2) * t
    achieved = flops / per_launch_s / 1e12
    peak = PEAK_TFLOPS[prec]
    issued_tf = issued_flops(prec, n, t) / per_launch_s / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic("herk_kernel<%s>" % prec, "n%d_t%d" % (n, t)),
            "kernel": "herk_kernel<%s>" % prec, "kernel_ms": round(per_launch_s * 1e3, 4),
            "kernel_ms_mean": round(mean_launch_s * 1e3, 4),
            "flop_per_pair_sample": FLOP_PER_PAIR_SAMPLE[prec],
            "useful_frac_8flop": round(8 * (n * (n - 1) // 2) * t / per_launch_s / 1e12 / peak, 4),
            "issued_achieved": round(issued_tf, 2), "issued_frac": round(issued_tf / peak, 4)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_gram_rate(z_np, budget_s=4.0):
    """The paper's own matrix method on this host, as context: FP64
    U @ U^H / T through torch's CPU BLAS on all cores (unit phasors made
    with numpy), on the first R rows, R sized for about `budget_s`.
    Returns (pair-samples/s, rows, threads, seconds)."""
    import numpy as np
    import torch

    t = z_np.shape[1]

    def run(r):
        u = z_np[:r].astype(np.complex128)
        u = u / np.where(np.abs(u) > 0, np.abs(u), 1.0)
        ut = torch.from_numpy(u)
        t0 = time.perf_counter()
        g = ut @ ut.conj().T / t
        dt = time.perf_counter() - t0
        del g
        return dt

    r = min(z_np.shape[0], 128)
    dt = run(r)
    rate = r * (r - 1) / 2 * t / dt
    r2 = int(min(z_np.shape[0], max(r, math.sqrt(2 * rate * budget_s / t))))
    if r2 > r:
        r, dt = r2, run(r2)
        rate = r * (r - 1) / 2 * t / dt
    return rate, r, torch.get_num_threads(), dt


def cpu_baseline(z_np, gpu_out, budget_s=15.0):
    """Time the FP64 oracle (per-pair angle / exp / mean) on all pairs among
    the first R rows of the same input, R sized for about `budget_s`, and
    check the GPU results on exactly those pairs."""
    import numpy as np

    import oracle

    nthreads = oracle.threads()
    t = z_np.shape[1]

    def run(r):
        zs = z_np[:r].astype(np.complex128)
        pr = oracle.upper_pairs(r)
        t0 = time.perf_counter()
        phi = oracle.phase(zs)
        g = oracle.pair_means(phi, pr, nthreads)
        dt = time.perf_counter() - t0
        return g, pr, dt

    # calibrate on enough rows that the threaded oracle runs at its full rate
    g, pr, dt = run(min(z_np.shape[0], 96))
    rate = len(pr) * t / dt
    want_pairs = rate * budget_s / t
    r = int(min(z_np.shape[0], max(32, math.sqrt(2 * want_pairs))))
    g, pr, dt = run(r)
    value = len(pr) * t / dt
    p, ip, cp = oracle.metrics(g)
    errs = {}
    for prec, out in gpu_out.items():
        a, b = pr[:, 0], pr[:, 1]
        gg = out["g"][a, b]
        e = max(np.abs(gg.real - g.real).max(), np.abs(gg.imag - g.imag).max())
        errs[prec] = {"g": float(e),
                      "plv": float(np.abs(out["plv"][a, b] - p).max()),
                      "iplv": float(np.abs(out["iplv"][a, b] - ip).max()),
                      "ciplv": float(np.abs(out["ciplv"][a, b] - cp).max())}
    base = {"value": round(value, 1), "unit": "pair-samples/s", "cores": nthreads, "kind": "oracle",
            "sample": "all %d pairs among the first %d signals x %d samples of the same input, %.1f s"
                      % (len(pr), r, t, dt), "cpu_model": cpu_model()}
    # the same oracle on one core, on a smaller sample
    r1 = int(max(16, min(r, math.sqrt(2 * (value / nthreads) * 4.0 / t))))
    zs = z_np[:r1].astype(np.complex128)
    pr1 = oracle.upper_pairs(r1)
    t0 = time.perf_counter()
    oracle.pair_means(oracle.phase(zs), pr1, 1)
    dt1 = time.perf_counter() - t0
    base["one_core"] = {"value": round(len(pr1) * t / dt1, 1), "cores": 1,
                        "sample": "all %d pairs among the first %d signals, %.1f s" % (len(pr1), r1, dt1)}
    rate, rg, thr, dtg = cpu_gram_rate(z_np)
    base["cpu_gram"] = {"value": round(rate, 1), "unit": "pair-samples/s", "threads": thr,
                        "kind": "FP64 U @ U^H / T, torch CPU BLAS (the paper's matrix method, context only)",
                        "sample": "first %d signals x %d samples, %.2f s" % (rg, t, dtg)}
    return base, errs


def timed(fn, steps, warmup):
    """(median ms per step, stage ms per step) of fn() on the current stream."""
    med, mean, stages, _ = step_times(fn, steps, warmup)
    per = {k: round(v[0] / steps, 4) for k, v in stages.items() if v[1]}
    per["mean_ms_per_step"] = round(mean, 4)
    return med, per


def line_for(workload, value, ms, args, dtype, config, extra):
    out = {"metric": METRIC, "value": round(value, 1), "unit": "pair-samples/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": dict(workload=workload, **config)}
    out.update(extra)
    return out


def bench_small(args):
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    x = torch.from_numpy(synth.glag_real(64, 2048, 256.0, 8, 10.0, seed=synth.seed_for(1))).cuda()
    ms, stages = timed(lambda: plv.from_real(x, 256.0, prec="f64"), args.steps, args.warmup)
    ps = 64 * 63 // 2 * 2048
    return line_for("small FP64: N=64 real f64 x T=2048 at 256 Hz, plain analytic signal", ps / (ms / 1e3), ms,
                    args, DTYPE["f64"], {"n": 64, "t": 2048, "prec": "f64"}, {"stage_ms": stages})


def bench_batch(args):
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    seed = synth.seed_for(4)
    shapes = synth.batch_shapes(512, seed)
    xs = [torch.from_numpy(synth.glag_real(n, t, 1000.0, 32, (2.0, 42.0), seed=seed + 1 + k,
                                           dtype=np.float32)).cuda() for k, (n, t) in enumerate(shapes)]
    bands = synth.bands_hz()
    if args.autotune:
        plv.autotune_batch(xs, prec=args.prec_batch, fs=1000.0, bands=bands)
    ms, stages = timed(lambda: plv.from_real_batch(xs, 1000.0, bands=bands, prec=args.prec_batch), args.steps,
                       args.warmup)
    ps = sum(n * (n - 1) // 2 * t for n, t in shapes) * len(bands)
    edges = {n: plv.tile_edge(n, args.prec_batch) for n in sorted({n for n, _ in shapes})}
    issued = sum(issued_flops(args.prec_batch, n, t, edges[n]) for n, t in shapes) * len(bands)
    useful = FLOP_PER_PAIR_SAMPLE[args.prec_batch] * ps
    return line_for("uneven batch: 512 trials, N in {68,148,360,1000}, T in [500,4000], 5 bands, real f32",
                    ps / (ms / 1e3), ms, args, DTYPE[args.prec_batch], {"trials": 512, "bands": len(bands),
                                                        "prec": args.prec_batch},
                    {"stage_ms": stages, "pair_samples": ps, "rows": sum(n for n, _ in shapes),
                     "tile_edges": {str(k): v for k, v in edges.items()}, "autotuned": bool(args.autotune),
                     "issued_over_useful_mfma": round(issued / useful, 4),
                     "gram_frac_of_peak": round(useful / (stages["gram"] / 1e3) / 1e12
                                                / PEAK_TFLOPS[args.prec_batch], 4) if stages.get("gram") else None})


def bench_grad(args):
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    n, t, fs = 2048, 8192, 1000.0
    x = torch.from_numpy(synth.glag_real(n, t, fs, 32, (8.0, 12.0), seed=synth.seed_for(5),
                                         dtype=np.float32)).cuda()
    cstar = torch.from_numpy(synth.sparse_target(n, seed=synth.seed_for(5, 1))).float().cuda()
    upper = torch.triu(torch.ones(n, n, device="cuda"), 1)

    def step():
        out = plv.from_real(x, fs, prec=args.prec_batch, want_g=True, want=("ciplv",))
        dc = (2 * (out["ciplv"][0] - cstar) * upper)[None]
        return plv.backward_batch([x], [out["g"]], [(None, None, dc)], fs=fs, prec=args.prec_batch)[0]

    ms, stages = timed(step, args.steps, args.warmup)
    ps = n * (n - 1) // 2 * t
    return line_for("differentiable ciPLV: N=2048 real f32 x T=8192, forward + adjoint", ps / (ms / 1e3), ms,
                    args, DTYPE[args.prec_batch], {"n": n, "t": t, "prec": args.prec_batch}, {"stage_ms": stages})


def bench_fir(args):
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    n, t, fs, order, pad = 2048, 8192, 1000.0, 2000, 2048
    x = torch.from_numpy(synth.glag_real(n, t, fs, 32, (8.0, 12.0), seed=synth.seed_for(7),
                                         dtype=np.float32)).cuda()
    prec = args.prec_batch
    bands = [(8.0, 12.0, order)]
    win = (pad, t - pad)
    ms, stages = timed(lambda: plv.from_real(x, fs, bands=bands, prec=prec, window=win), args.steps, args.warmup)
    tw = win[1] - win[0]
    ps = n * (n - 1) // 2 * tw
    extra = {"stage_ms": stages}
    if stages.get("gram"):
        flops = FLOP_PER_PAIR_SAMPLE[prec] * ps
        extra["gram_frac_of_peak"] = round(flops / (stages["gram"] / 1e3) / 1e12 / PEAK_TFLOPS[prec], 4)
    return line_for("FIR band-pass then PLV: N=2048 real f32 x T=8192 at 1 kHz (4096-sample epoch, 2048 "
                    "samples of padding each side), 8-12 Hz FIR of order 2000 applied forward and backward",
                    ps / (ms / 1e3), ms, args, DTYPE[prec], {"n": n, "t": t, "window": list(win), "fir_order": order,
                                                       "prec": prec}, extra)


def bench_coherence(args):
    """Coherency (Section II.B, Eq. 12) of N = 1024 complex rows x T = 60000
    samples (amplitude-modulated coupled coefficients, complex64)."""
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    n, t = N_SIG, T_SAMP
    z = torch.from_numpy(synth.coefficients_mixed(n, t, seed=synth.seed_for(6, 1), dtype=np.complex64)).cuda()
    prec = args.prec_batch
    ms, stages = timed(lambda: plv.coherence(z, prec=prec), args.steps, args.warmup)
    ps = n * (n - 1) // 2 * t
    extra = {"stage_ms": stages}
    if stages.get("gram"):
        flops = FLOP_PER_PAIR_SAMPLE[prec] * ps
        extra["gram_frac_of_peak"] = round(flops / (stages["gram"] / 1e3) / 1e12 / PEAK_TFLOPS[prec], 4)
        extra["gram_issued_frac_of_peak"] = round(issued_flops(prec, n, t) / (stages["gram"] / 1e3) / 1e12
                                                  / PEAK_TFLOPS[prec], 4)
    return line_for("coherency: N=1024 complex coefficient rows x T=60000, amplitude-modulated mixtures",
                    ps / (ms / 1e3), ms, args, DTYPE[prec], {"n": n, "t": t, "prec": prec}, extra)


def bench_coherence_stft(args):
    """Coherency over windowed segments (Section II.B, Eq. 12; Section III.B's
    Hamming-windowed overlapping segments): N = 1024 real f32 signals x 60 s
    at 1 kHz (lagged oscillators, 32 latents at 8-12 Hz), 1000-sample Hamming
    segments with 500 samples of overlap (119 segments), the five 1 Hz bins
    8..12 Hz; one coherency matrix per bin."""
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    n, t, seg, hop, bins = N_SIG, T_SAMP, 1000, 500, (8, 12)
    x = torch.from_numpy(synth.glag_real(n, t, FS, 32, (8.0, 12.0), seed=synth.seed_for(6, 7),
                                         dtype=np.float32)).cuda()
    prec = args.prec_batch
    ms, stages = timed(lambda: plv.coherence_stft(x, seg, hop, bins, "hamming", prec=prec), args.steps,
                       args.warmup)
    nseg = (t - seg) // hop + 1
    nb = bins[1] - bins[0] + 1
    ps = n * (n - 1) // 2 * nseg * nb
    extra = {"stage_ms": stages, "segments": nseg, "bins": nb,
             "coefficients_per_s": round(n * nseg * nb / (stages.get("stft", ms) / 1e3), 1)}
    return line_for("coherency over segments: N=1024 real f32 x T=60000 at 1 kHz, 1000-sample Hamming segments, "
                    "500 overlap, bins 8..12 Hz", ps / (ms / 1e3), ms, args, DTYPE[prec],
                    {"n": n, "t": t, "seg": seg, "hop": hop, "bins": list(bins), "prec": prec}, extra)


def bench_trials(args):
    """Lachaux's PLV across trials (Eq. 1): 148 signals x 40 trials x 4000 time
    points (4 s at 1 kHz), complex64 trial-major; one PLV matrix per time point."""
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    import synth

    n, ntr, t = 148, 40, 4000
    seed = synth.seed_for(7, 100)
    z = torch.from_numpy(np.stack([synth.glag_analytic(n, t, 1000.0, 8, (8.0, 12.0), seed=seed + k,
                                                       dtype=np.complex64) for k in range(ntr)])).cuda()
    prec = args.prec_batch
    ms, stages = timed(lambda: plv.over_trials(z, prec=prec), args.steps, args.warmup)
    ps = n * (n - 1) // 2 * ntr * t
    return line_for("PLV across trials: 148 signals x 40 trials x 4000 time points, complex64",
                    ps / (ms / 1e3), ms, args, DTYPE[prec], {"n": n, "trials": ntr, "t": t, "prec": prec},
                    {"stage_ms": stages, "matrices_per_s": round(t / (ms / 1e3), 1)})


def bench_brain(args):
    """Whole-brain scale: N = 15000 unit phasors of T = 1.2e6 samples (144 GB
    of complex64, generated on the GPU), 200 planted constant-lag pairs;
    16-bit MFMA with FP32 accumulation in K-chunks and FP64 sums across them."""
    import numpy as np
    import torch

    import paper_1710_08037_amd as plv
    from synth import seed_for
    from synth.device import phasors_planted_device

    n, t, npairs = 15000, 1200000, 200
    prec = args.prec_brain
    z, pairs, lags = phasors_planted_device(n, t, npairs, seed_for(3))
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    warm = max(1, min(args.warmup, 1))
    box = {}

    def step():
        box["out"] = plv.from_analytic(z, prec=prec, want=("plv", "iplv", "ciplv"))

    ms, stages = timed(step, steps, warm)
    ps = n * (n - 1) // 2 * t
    extra = {"stage_ms": stages, "pair_samples": ps}
    if stages.get("gram"):
        flops = FLOP_PER_PAIR_SAMPLE[prec] * ps
        extra["gram_tflops"] = round(flops / (stages["gram"] / 1e3) / 1e12, 1)
        extra["gram_frac_of_peak"] = round(flops / (stages["gram"] / 1e3) / 1e12 / PEAK_TFLOPS[prec], 4)
        extra["gram_issued_frac_of_peak"] = round(issued_flops(prec, n, t) / (stages["gram"] / 1e3) / 1e12
                                                  / PEAK_TFLOPS[prec], 4)
    if not args.no_cpu:
        extra["cpu_baseline"], extra["max_abs_err"] = brain_cpu_leg(z, pairs, box["out"])
    extra["steps_note"] = "at most 3 timed steps of about a second each"
    line = line_for("whole-brain: N=15000 unit phasors x T=1.2e6 (complex64, generated on the GPU), "
                    "200 planted lagged pairs", ps / (ms / 1e3), ms, args, DTYPE[prec], {"n": n, "t": t, "prec": prec},
                    extra)
    line["steps"] = steps
    line["warmup"] = warm
    return line


def brain_cpu_leg(z, pairs, out, budget_s=15.0):
    """The oracle on the planted pairs plus all pairs among R random other
    rows (R sized for about `budget_s`), timed, and the GPU results checked
    on exactly those pairs."""
    import numpy as np

    import oracle

    n, t = z.shape
    nthreads = oracle.threads()
    rng = np.random.default_rng(5)
    planted = np.unique(pairs.reshape(-1))
    rest = np.setdiff1d(np.arange(n), planted)
    probe = 16
    rows = np.sort(rng.choice(rest, size=probe, replace=False))
    zz = z[rows].cpu().numpy().astype(np.complex128)
    pr = oracle.upper_pairs(probe)
    t0 = time.perf_counter()
    oracle.pair_means(oracle.phase(zz), pr, nthreads)
    rate = len(pr) * t / (time.perf_counter() - t0)
    r = int(max(probe, math.sqrt(2 * max(rate * budget_s / t - len(pairs), 0))))
    rows = np.sort(np.concatenate([planted, rng.choice(rest, size=r, replace=False)]))
    zz = z[rows].cpu().numpy().astype(np.complex128)
    pos = {int(v): k for k, v in enumerate(rows)}
    rnd = np.array([pos[int(v)] for v in rows if int(v) not in set(planted.tolist())])
    loc = np.array([[pos[int(a)], pos[int(b)]] for a, b in pairs], dtype=np.int64)
    ii, jj = np.triu_indices(len(rnd), 1)
    loc = np.concatenate([loc, np.stack([rnd[ii], rnd[jj]], 1)])
    loc = np.stack([loc.min(1), loc.max(1)], 1)
    t0 = time.perf_counter()
    g = oracle.pair_means(oracle.phase(zz), loc, nthreads)
    dt = time.perf_counter() - t0
    p, ip, cp = oracle.metrics(g)
    a = rows[loc[:, 0]]
    b = rows[loc[:, 1]]
    errs = {}
    ia, ib = torch_index(a), torch_index(b)
    for k, ref in (("plv", p), ("iplv", ip), ("ciplv", cp)):
        got = out[k][ia, ib].cpu().numpy().astype(np.float64)
        errs[k] = float(np.abs(got - ref).max())
    base = {"value": round(len(loc) * t / dt, 1), "unit": "pair-samples/s", "cores": nthreads, "kind": "oracle",
            "sample": "the %d planted pairs and all %d pairs among %d other random signals, x %d samples, %.1f s"
                      % (len(pairs), len(loc) - len(pairs), len(rnd), t, dt)}
    return base, errs


def torch_index(a):
    import torch
    return torch.from_numpy(a).cuda()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU idles while the host makes the inputs; a few warm-up steps leave
    # the timed ones on a clock still ramping up (about 12% slower on the
    # sensor case), so the default warms up for as many steps as it times
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--prec", default="both", choices=["both", "split_bf16", "f32"],
                    help="paths to time (both: split-BF16 for `value`, FP32 beside it)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes 3 times (counter calibration) and exit")
    ap.add_argument("--workload", default="sensor", choices=["sensor", "small", "batch", "grad", "brain", "coherence", "trials", "fir",
                             "coherence_stft"])
    ap.add_argument("--prec-batch", default="split_bf16", help="precision of the batch and grad workloads")
    ap.add_argument("--autotune", action="store_true",
                    help="batch workload: measure the tile edge per row count (plv_autotune) before timing")
    ap.add_argument("--prec-brain", default="bf16", choices=["bf16", "f16"], help="precision of the brain workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth

    torch.cuda.set_device(0)
    if args.copy_ref:
        src = torch.empty(args.copy_ref, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": args.copy_ref}), flush=True)
        return
    if args.workload != "sensor":
        fn = {"small": bench_small, "batch": bench_batch, "grad": bench_grad, "brain": bench_brain, "fir": bench_fir,
              "coherence": bench_coherence, "trials": bench_trials,
              "coherence_stft": bench_coherence_stft}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    z_np = synth.glag_analytic(N_SIG, T_SAMP, FS, 32, (8.0, 12.0), seed=synth.seed_for(2), dtype=np.complex64)
    z = torch.from_numpy(z_np).cuda()

    results = {}
    precs = ("split_bf16", "f32") if args.prec == "both" else (args.prec,)
    for prec in precs:
        ms, mean, stages, gram = run_gpu(z, prec, args.steps, args.warmup)
        results[prec] = {"ms": ms, "mean": mean, "stages": stages, "gram": gram}
    if args.prec == "f32":
        print(json.dumps({"f32_ms_per_step": results["f32"]["ms"]}), flush=True)
        return

    pair_samples = N_SIG * (N_SIG - 1) // 2 * T_SAMP
    main_prec = "split_bf16"
    ms = results[main_prec]["ms"]
    line = {
        "metric": METRIC,
        "value": round(pair_samples / (ms / 1e3), 1),
        "unit": "pair-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[main_prec],
        "data": "synthetic",
        "config": {"workload": "sensor-scale analytic PLV: N=1024 complex64 signals x T=60000 samples, "
                               "lagged oscillators (32 latents, 8-12 Hz), split-BF16 Gram",
                   "n": N_SIG, "t": T_SAMP, "prec": main_prec},
        "roofline": roofline(main_prec, N_SIG, T_SAMP, results[main_prec]["stages"], results[main_prec]["gram"]),
        "mean_ms_per_step": round(results[main_prec]["mean"], 4),
        "timing": "median of per-step HIP event pairs on the launch stream; kernel_ms the median per launch",
    }
    stage_ms = {}
    for prec, r in results.items():
        stage_ms[prec] = {k: round(v[0] / max(v[1], 1), 4) for k, v in r["stages"].items() if v[1]}
    if "f32" in results:
        line["fp32"] = {"value": round(pair_samples / (results["f32"]["ms"] / 1e3), 1), "ms_per_step":
                        round(results["f32"]["ms"], 4), "roofline": roofline("f32", N_SIG, T_SAMP,
                                                                              results["f32"]["stages"],
                                                                              results["f32"]["gram"])}
        line["split_vs_fp32_speedup"] = round(results["f32"]["ms"] / ms, 3)
    line["stage_ms"] = stage_ms
    if not args.no_cpu:
        import paper_1710_08037_amd as plv
        gpu_out = {}
        for prec in precs:
            o = plv.from_analytic(z, prec=prec, want_g=True)
            torch.cuda.synchronize()
            gpu_out[prec] = {k: v.cpu().numpy().astype(np.complex128 if k == "g" else np.float64)
                             for k, v in o.items()}
        base, errs = cpu_baseline(z_np, gpu_out)
        line["cpu_baseline"] = base
        line["max_abs_err_vs_fp64"] = errs
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
