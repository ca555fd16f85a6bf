"""Throughput benchmark of the alpha-dense DFT on one MI355X.

Default workload: 256 complex64 signals, N = 65536 samples at dt = 1e-3 s
(T = 65.536 s), alpha = 8 -> 524288 bins per signal; each signal is 5 unit
complex tones at uniform random frequencies and phases plus complex Gaussian
noise (sigma = 0.05), seeded.  One step = one dense_dft_exec over the whole
batch, inputs resident in HBM.

Prints ONE JSON line: bins/s, per-kernel HIP-event durations, the HBM
roofline of the transform (algorithmic bytes = N*8 + alpha*N*8 per signal),
the rel. L2 error of the timed output against the FP64 oracle on a bin
sample, and the oracle's own rate on the host cores (cpu_baseline).

Other workloads (--workload): precision (1 x 2^22, alpha 16, c64),
plain_f64 (1 x 1024, alpha 4, real float64), uneven (1000 signals of uneven N
and alpha in one persistent launch vs 1000 plain launches) and serving
(Poisson request streams through the request server, batched vs plain,
p50/p99 latency) and ablation (the default shape against the FFT of the
zero-padded signals, by this library and by the platform FFT library).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


# Sources that fix the launches of the plain forward and inverse transforms
# and of the persistent batch (kernels, launch geometry, planner and tuner):
# the counter summaries are void once any changes.
TRAFFIC_SOURCES = ("dd_fft.hpp", "dd_kernels.hpp", "dd_inst.hpp", "dd_launch.hpp", "dd_host.hpp",
                   "dd_pass_f32.hip", "dd_single_f32.hip", "dd_misc.hip", "dd_api.cpp", "dd_tune.cpp",
                   "dd_inverse.hpp", "dd_inv_f32.hip",
                   "dd_batch.hip", "dd_batch.hpp", "dd_batch_host.hpp", "dd_batch_api.cpp")


def kernel_source_hash():
    """First 16 hex digits of sha256 over TRAFFIC_SOURCES."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2403_16665_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per step from the committed rocprofv3 counter summary, or None
    when it was taken for other kernel sources or another workload."""
    import glob
    import re
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        txt = open(path).read()
        t = re.search(r"^traffic_bytes_per_step:\s*(\d+)", txt, re.M)
        h = re.search(r"^source_hash:\s*(\w+)", txt, re.M)
        w = re.search(r"^workload:\s*(\w+)", txt, re.M)
        if t and h and w and w.group(1) == workload and h.group(1) == kernel_source_hash():
            return int(t.group(1))
    return None

WORKLOADS = {
    "batch_c64": dict(batch=256, N=65536, alpha=8, dt=1e-3, input="complex64"),
    "real_f32": dict(batch=256, N=65536, alpha=8, dt=1e-3, input="float32 real"),
    "precision": dict(batch=1, N=1 << 22, alpha=16, dt=1e-3, input="complex64"),
    "plain_f64": dict(batch=1, N=1024, alpha=4, dt=1e-3, input="float64"),
    "uneven": dict(batch=1000, N=0, alpha=0, dt=1e-3, input="complex64"),
    "serving": dict(batch=0, N=0, alpha=0, dt=1e-3, input="float32/complex64"),
    "ablation": dict(batch=256, N=65536, alpha=8, dt=1e-3, input="complex64"),
    "inverse": dict(batch=256, N=65536, alpha=8, dt=1e-3, input="complex64 spectra"),
    "decimated": dict(batch=256, N=65536, alpha=0, dt=1e-3, input="complex64"),
}


def make_inputs(name, w):
    import siggen
    N, batch, dt = w["N"], w["batch"], w["dt"]
    if name == "batch_c64":
        return np.stack([siggen.tones_complex(g, N, dt) for g in siggen.rngs(1, batch)])
    if name == "real_f32":
        return np.stack([siggen.tones_real(g, N, dt, w["alpha"])[0] for g in siggen.rngs(7, batch)]).astype(np.float32)
    if name == "precision":
        return siggen.precision_tones(siggen.rngs(2, 1)[0], N)[None, :]
    if name == "plain_f64":
        return siggen.tones_real(siggen.rngs(0, 1)[0], N, dt, w["alpha"])[0][None, :]
    raise ValueError(name)


def tune_classes(dd, classes, batch_kernel=True, plain_batch=1, dtypes=None):
    """Run the schedule tuner over (N, alpha) classes before timing: the batch
    kernel's schedule per class and, if plain_batch, the plain plan's (for a
    batch of plain_batch signals of each input dtype in `dtypes`, complex64
    by default).  Returns a summary."""
    t0 = time.perf_counter()
    gain_b, gain_p = [], []
    for N, a in sorted(set(classes)):
        if batch_kernel:
            try:
                r = dd.dense_dft_tune_batch(N, a)
                gain_b.append(r["ms_default"] / r["ms_best"])
            except dd.DenseDFTError:
                pass   # no batch-kernel schedule: plain fallback
        if plain_batch:
            for code in (dtypes or (dd.DD_C64,)):
                r = dd.dense_dft_tune(N, a, plain_batch, code)
                gain_p.append(r["ms_default"] / r["ms_best"])
    out = {"classes": len(set(classes)), "seconds": time.perf_counter() - t0}
    if gain_b:
        out["batch_kernel_speedup_over_rule"] = {"mean": float(np.mean(gain_b)), "max": float(np.max(gain_b))}
    if gain_p:
        out["plain_speedup_over_rule"] = {"mean": float(np.mean(gain_p)), "max": float(np.max(gain_p))}
    return out


def precision_errors(dd, xd, Xd, N, alpha, T):
    """The precision form: relative L2 error against the FP64 oracle on the
    workload's 16384 seeded bins (tests/golden fixture written by the oracle)
    with FP64-generated twiddles (Xd, the timed output) and with the
    FP32-twiddle variant."""
    import torch
    path = os.path.join(ROOT, "tests", "golden", "precision_2p22_a16_16384.npz")
    fx = np.load(path, allow_pickle=False)
    bins, ref = fx["bins"], fx["X"]
    idx = torch.from_numpy(bins).to(Xd.device)
    p32 = dd.dense_dft_plan(N, alpha, T, 1, dd.DD_C64, dd.DD_TWIDDLE_FP32)
    X32 = torch.empty_like(Xd)
    dd.dense_dft_exec(p32, xd, X32)
    torch.cuda.synchronize()
    out = {"bins": int(len(bins)), "bound": 1e-5, "reference": "FP64 oracle, " + os.path.relpath(path, ROOT)}
    for name, X in (("rel_l2_fp64_twiddles", Xd), ("rel_l2_fp32_twiddles", X32)):
        got = X[0][idx].cpu().numpy()
        out[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_rows, alpha, T, M, N, target_s=20.0):
    """Time the FP64 oracle on a bounded sample of the workload (host cores):
    all bins of signal 0, then of signal 1, ..., or a seeded subset of the
    last one, until about target_s seconds of work (the short probe that sets the
    sample size overestimates the cost per bin, so the run is about half that).  Returns
    [(signal, bins, reference)] and the cpu_baseline record."""
    import oracle
    import siggen
    rng = np.random.default_rng(123)
    probe = siggen.bin_subset(rng, M, min(M, 64 * oracle.threads()))   # several bins per thread
    t0 = time.perf_counter()
    oracle.alpha_dft_bins(x_rows[0], alpha, T, probe)
    rate = len(probe) / max(time.perf_counter() - t0, 1e-6)
    want = int(max(64, rate * target_s))
    samples, done, el = [], 0, 0.0
    for b in range(len(x_rows)):
        nb = min(M, want - done)
        if nb <= 0:
            break
        bins = siggen.bin_subset(rng, M, nb)
        t0 = time.perf_counter()
        ref = oracle.alpha_dft_bins(x_rows[b], alpha, T, bins)
        el += time.perf_counter() - t0
        samples.append((b, bins, ref))
        done += len(bins)
    nsig = len(samples)
    return samples, {"value": done / el, "unit": "bins/s", "cores": oracle.threads(), "cpu_model": cpu_model(),
                     "kind": "oracle",
                     "sample": f"{done} seeded bins of the first {nsig} signal(s) (each bin = {N} complex "
                               f"multiply-adds, FP64 direct sum), {el:.1f} s"}


def run_uneven(args):
    """1000 complex64 signals, (N, alpha) drawn log-uniformly (siggen.uneven_mix),
    tone-plus-noise content: one persistent batch launch vs 1000 plain launches."""
    import torch
    import paper_2403_16665_amd as dd
    import siggen
    dt = 1e-3
    mix = siggen.uneven_mix(siggen.rngs(3, 1)[0], 1000)
    gens = siggen.rngs(4, len(mix))
    xs_np = [siggen.tones_complex(g, N, dt) for g, (N, a) in zip(gens, mix)]
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    Xs = [torch.empty(a * N, dtype=torch.complex64, device="cuda") for (N, a) in mix]
    descs = [(N, a, N * dt, dd.DD_C64, xs[i], Xs[i]) for i, (N, a) in enumerate(mix)]
    tuning = None
    if args.tune_db and os.path.exists(args.tune_db):
        dd.dense_dft_tune_load(args.tune_db)  # the schedules of an earlier run, no tuner launches
        tuning = {"loaded": args.tune_db}
    elif args.tune:
        tuning = tune_classes(dd, mix)
        if args.tune_db:
            dd.dense_dft_tune_save(args.tune_db)
    b = dd.dense_dft_batch_plan(descs)
    tasks, grid, scratch, fb = dd.dense_dft_batch_info(b)
    plans = [dd.dense_dft_plan(N, a, N * dt, 1, dd.DD_C64) for (N, a) in mix]
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    bins = sum(a * N for N, a in mix)
    b_alg = sum(N * 8 + a * N * 8 for N, a in mix)

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, 1e3 * (time.perf_counter() - t0) / steps

    def plain():
        for p, x, X in zip(plans, xs, Xs):
            dd.dense_dft_exec(p, x, X, stream=sp)

    ms_b, wall_b = timed(lambda: dd.dense_dft_batch_exec(b, stream=sp), args.steps, args.warmup)
    assert dd.dense_dft_batch_status(b) == 0
    Xb = [X.clone() for X in Xs[:50]]
    ms_p, wall_p = timed(plain, max(3, args.steps // 10), max(1, args.warmup // 5))
    torch.cuda.synchronize()
    same = all(torch.allclose(a_, c_, rtol=0, atol=1e-5 * float(c_.abs().max()))
               for a_, c_ in zip(Xb, Xs[:50]))
    achieved = b_alg / (ms_b * 1e-3) / 1e9
    result = {
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": bins / (ms_b * 1e-3), "unit": "bins/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "wall_ms_per_step": wall_b,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uneven", "signals": len(mix), "bins_per_step": bins,
                   "N_range": [min(n for n, _ in mix), max(n for n, _ in mix)],
                   "alphas": sorted(set(a for _, a in mix)), "input": "complex64", "dt": dt},
        "batch": {"tasks": tasks, "grid": grid, "scratch_bytes": scratch, "fallback_signals": fb,
                  "launches_per_step": "1 staging kernel + 1 or 2 queue kernels"},
        "plain": {"value": bins / (ms_p * 1e-3), "ms_per_step": ms_p, "wall_ms_per_step": wall_p,
                  "launches_per_step": "1000 execs"},
        "batched_over_plain": ms_p / ms_b,
        "tuning": tuning,
        "batched_equals_plain": bool(same),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("uneven"),
                     "what": "whole batch per step: algorithmic bytes sum(N*8 + alpha*N*8) / step time"},
    }
    if result["roofline"]["traffic"]:
        result["roofline"]["amplification"] = result["roofline"]["traffic"] / b_alg
    if not args.no_cpu:
        N0, a0 = mix[0]
        samples, cpu = cpu_baseline([xs_np[0]], a0, N0 * dt, a0 * N0, N0)
        _, bins0, ref = samples[0]
        got = Xs[0].cpu().numpy()[bins0]
        result["rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def run_serving(args):
    """Open-loop Poisson request streams through the request server, batched
    (continuous batching, one persistent launch per batch) and plain (every
    request alone as one plain execution).  (N, alpha) as the uneven mix,
    float32 real or complex64 input half and half, tone-plus-noise content,
    inputs resident in HBM before the stream starts."""
    import ctypes
    import torch
    import paper_2403_16665_amd as dd
    import siggen
    dt = 1e-3
    rates = [float(r) for r in args.rates.split(",")]
    count = args.requests
    rng = siggen.rngs(5, 1)[0]
    mix = siggen.uneven_mix(rng, count)
    codes = [dd.DD_F32 if u < 0.5 else dd.DD_C64 for u in rng.random(count)]
    # one input per (N, dtype): requests read it, each writes its own output
    inputs = {}
    kinds = sorted(set((N, c) for (N, _), c in zip(mix, codes)))
    for g, (N, c) in zip(siggen.rngs(6, len(kinds)), kinds):
        if c == dd.DD_F32:
            inputs[(N, c)] = torch.from_numpy(siggen.tones_real(g, N, dt, 1)[0].astype(np.float32)).cuda()
        else:
            inputs[(N, c)] = torch.from_numpy(siggen.tones_complex(g, N, dt)).cuda()
    offs = np.concatenate([[0], np.cumsum([a * N for N, a in mix])])
    arena = torch.empty(int(offs[-1]), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    descs = [dd.dd_desc(N, a, N * dt, c, inputs[(N, c)].data_ptr(), arena[int(offs[i]):].data_ptr())
             for i, ((N, a), c) in enumerate(zip(mix, codes))]
    bins = np.array([a * N for N, a in mix], dtype=np.float64)
    balg = np.array([N * (4 if c == dd.DD_F32 else 8) + a * N * 8 for (N, a), c in zip(mix, codes)],
                    dtype=np.float64)
    budget = 16 << 30

    def stream_through(server, rate, seed):
        arr = siggen.poisson_arrivals(np.random.default_rng(seed), rate, count)
        t0 = dd.dense_dft_clock_ns() + 2_000_000
        due = [t0 + int(a_ * 1e9) for a_ in arr]
        tickets = dd.dense_dft_submit_many_at(server, descs, due)   # native open-loop generator
        res = [dd.dense_dft_wait(server, int(tk), 120_000_000) for tk in tickets]
        assert all(r["status"] == 0 for r in res)
        lat = np.array([r["t_done_ns"] - r["t_arrival_ns"] for r in res]) / 1e6
        span = (max(r["t_done_ns"] for r in res) - min(r["t_arrival_ns"] for r in res)) / 1e9
        return {"rate_req_s": rate, "requests": count, "bins_per_s": float(bins.sum() / span),
                "hbm_GBps": float(balg.sum() / span / 1e9), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_batch": float(np.mean([r["batch_requests"] for r in res]))}

    tuning = tune_classes(dd, mix, dtypes=(dd.DD_C64, dd.DD_F32)) if args.tune else None
    out = {}
    for mode, name in ((dd.DD_SERVE_PLAIN, "plain"), (dd.DD_SERVE_BATCHED, "batched")):
        srv = dd.dense_dft_server_create(mode=mode, hbm_budget_bytes=budget)
        for (N, a), c in sorted(set(zip(mix, codes))):
            dd.dense_dft_server_warm(srv, N, a, N * dt, c)
        stream_through(srv, rates[-1], 99)         # warm-up pass over every class
        out[name] = [stream_through(srv, r, 100 + k) for k, r in enumerate(rates)]
        out[name + "_stats"] = dd.dense_dft_server_stats(srv)
        dd.dense_dft_server_destroy(srv)
    # the arena holds the batched pass's outputs: 1% of the requests again
    # through a plain plan, compared by relative L2 over the whole spectrum
    checked, worst = 0, 0.0
    for i in range(0, count, 100):
        N, a = mix[i]
        c = codes[i]
        ref = dd.alpha_dft(inputs[(N, c)], a, N * dt)
        got = arena[int(offs[i]):int(offs[i + 1])]
        torch.cuda.synchronize()
        worst = max(worst, float((got - ref).abs().pow(2).sum().sqrt() / ref.abs().pow(2).sum().sqrt()))
        checked += 1
    top = out["batched"][-1]
    result = {
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": top["bins_per_s"], "unit": "bins/s", "n_gpus": 1, "steps": count, "warmup": count,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving", "requests_per_rate": count, "rates_req_s": rates,
                   "N_range": [min(n for n, _ in mix), max(n for n, _ in mix)], "alphas": [2, 3, 4, 8, 16],
                   "inputs": "float32 real / complex64, 1:1", "hbm_budget_bytes": budget},
        "serving": out,
        "tuning": tuning,
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
        "plain_at_top_rate": out["plain"][-1],
        "check": {"requests": checked, "max_rel_l2_vs_plain": worst, "bound": 1e-5},
        "roofline": {"bound": "hbm", "achieved": top["hbm_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": top["hbm_GBps"] / HBM_PEAK_GBS, "traffic": None,
                     "what": "served algorithmic bytes sum(N*s_in + alpha*N*8) / wall span at the top rate"},
    }
    print(json.dumps(result), flush=True)


def run_ablation(args):
    """The saving the paper claims over zero padding (Section 4), measured on
    the default workload's shape: the alpha-dense transform, against the
    length-alpha*N FFT of the zero-padded signals computed (b) by this
    library's own kernels (alpha = 1 at length alpha*N) and (c) by the
    platform FFT library through torch.fft, as a black box.  All three
    outputs are the same spectrum; each is checked against the first."""
    import torch
    import paper_2403_16665_amd as dd
    import siggen
    N, alpha, batch, dt = 65536, 8, 256, 1e-3
    T, M = N * dt, alpha * N
    x = np.stack([siggen.tones_complex(g, N, dt) for g in siggen.rngs(1, batch)])
    xd = torch.from_numpy(x).cuda()
    xp = torch.zeros(batch, M, dtype=torch.complex64, device="cuda")
    xp[:, :N] = xd
    X = torch.empty(batch, M, dtype=torch.complex64, device="cuda")
    Xp = torch.empty_like(X)
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    if args.tune:
        dd.dense_dft_tune(N, alpha, batch, dd.DD_C64)
        dd.dense_dft_tune(M, 1, batch, dd.DD_C64)
    plan = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_C64)
    plan_p = dd.dense_dft_plan(M, 1, T * alpha, batch, dd.DD_C64)   # (T/N) = (alpha T)/(alpha N)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record()
            for _ in range(args.steps):
                fn()
            e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_a = timed(lambda: dd.dense_dft_exec(plan, xd, X, stream=sp))
    ms_b = timed(lambda: dd.dense_dft_exec(plan_p, xp, Xp, stream=sp))
    with torch.cuda.stream(stream):
        Xf = torch.fft.fft(xp, dim=1)
    torch.cuda.synchronize()

    def lib_fft():
        nonlocal Xf
        Xf = torch.fft.fft(xp, dim=1)
    ms_c = timed(lib_fft)
    Xf = Xf * (T / N)
    torch.cuda.synchronize()

    def rel(a, b):
        return float((a - b).abs().pow(2).sum().sqrt() / b.abs().pow(2).sum().sqrt())
    bins = batch * M
    b_a = batch * (N * 8 + M * 8)
    b_pad = batch * (M * 8 + M * 8)
    res = {
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": bins / (ms_a * 1e-3), "unit": "bins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_a, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ablation", "batch": batch, "N": N, "alpha": alpha, "input": "complex64"},
        "ablation": {
            "alpha_dense": {"ms": ms_a, "bins_per_s": bins / (ms_a * 1e-3), "algorithmic_bytes": b_a,
                            "schedule": dd.dense_dft_plan_get_sched(plan)},
            "zero_padded_own_fft": {"ms": ms_b, "bins_per_s": bins / (ms_b * 1e-3), "algorithmic_bytes": b_pad,
                                    "schedule": dd.dense_dft_plan_get_sched(plan_p),
                                    "rel_l2_vs_alpha_dense": rel(Xp, X)},
            "zero_padded_platform_fft": {"ms": ms_c, "bins_per_s": bins / (ms_c * 1e-3),
                                         "algorithmic_bytes": b_pad, "library": "torch.fft (rocFFT)",
                                         "rel_l2_vs_alpha_dense": rel(Xf, X)},
            "speedup_over_own_padded": ms_b / ms_a,
            "speedup_over_platform_padded": ms_c / ms_a,
        },
        "roofline": {"bound": "hbm", "achieved": b_a / (ms_a * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b_a / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "what": "alpha-dense transform, end to end per step"},
    }
    print(json.dumps(res), flush=True)


def run_inverse(args):
    """The inverse transform on the default workload's shape: 256 spectra of
    alpha*N = 524288 bins (the forward transforms of the default signals) back
    to N = 65536 samples each; the round trip is checked against the signals."""
    import torch
    import paper_2403_16665_amd as dd
    import siggen
    N, alpha, batch, dt = 65536, 8, 256, 1e-3
    T, M = N * dt, alpha * N
    x = np.stack([siggen.tones_complex(g, N, dt) for g in siggen.rngs(1, batch)])
    xd = torch.from_numpy(x).cuda()
    if args.tune_db and os.path.exists(args.tune_db):
        dd.dense_dft_tune_load(args.tune_db)  # the schedule of an earlier run, no tuner launches
    elif args.tune:
        dd.dense_dft_tune(N, alpha, batch, dd.DD_C64)
        if args.tune_db:
            dd.dense_dft_tune_save(args.tune_db)
    plan = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_C64)
    X = torch.empty(batch, M, dtype=torch.complex64, device="cuda")
    dd.dense_dft_exec(plan, xd, X)
    back = torch.empty(batch, N, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    for _ in range(args.warmup):
        dd.dense_dft_exec_inverse(plan, X, back, stream=sp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        dd.dense_dft_exec_inverse(plan, X, back, stream=sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    dd.dense_dft_profile_begin(plan, 1 << 16)
    for _ in range(args.steps):
        dd.dense_dft_exec_inverse(plan, X, back, stream=sp)
    prof = dd.dense_dft_profile_end(plan, cap=1 << 16)
    kern = {}
    for kind, t in prof:
        kern.setdefault(kind, []).append(t)
    kernels = {k: {"launches": len(v), "avg_us": 1e3 * float(np.mean(v))} for k, v in kern.items()}
    kms = sum(sum(v) for v in kern.values()) / args.steps
    rt = float((back - xd).abs().pow(2).sum().sqrt() / xd.abs().pow(2).sum().sqrt())
    b_alg = batch * (M * 8 + N * 8)
    achieved = b_alg / (kms * 1e-3) / 1e9
    traffic = measured_traffic("inverse")
    print(json.dumps({
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": batch * M / (ms * 1e-3), "unit": "bins/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "inverse", "batch": batch, "N": N, "alpha": alpha, "input": "complex64 spectra",
                   "schedule": dd.dense_dft_plan_get_sched(plan)},
        "kernels": kernels,
        "round_trip_rel_l2": rt,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "amplification": traffic / b_alg if traffic else None,
                     "what": "inverse transform per step: algorithmic bytes batch*(alpha*N*8 + N*8) / summed "
                             "kernel durations"},
    }), flush=True)


def run_decimated(args):
    """The alpha = 1/p transform (Section 2, alpha < 1) on the default
    signals: 256 complex64 signals of N = 65536 samples, p = 4 -> 16384 bins
    spaced p/T apart; fold then the plain transform of length N/p."""
    import torch
    import paper_2403_16665_amd as dd
    import siggen
    N, p, batch, dt = 65536, 4, 256, 1e-3
    T = N * dt
    x = np.stack([siggen.tones_complex(g, N, dt) for g in siggen.rngs(1, batch)])
    xd = torch.from_numpy(x).cuda()
    if args.tune:
        dd.dense_dft_tune(N // p, 1, batch, dd.DD_C64)
    plan = dd.dense_dft_plan_decimated(N, p, T, batch, dd.DD_C64)
    X = torch.empty(batch, N // p, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    for _ in range(args.warmup):
        dd.dense_dft_exec(plan, xd, X, stream=sp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        dd.dense_dft_exec(plan, xd, X, stream=sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    b_alg = batch * (N * 8 + (N // p) * 8)
    res = {
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": batch * (N // p) / (ms * 1e-3), "unit": "bins/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "decimated", "batch": batch, "N": N, "alpha": f"1/{p}", "input": "complex64",
                   "schedule_of_length_N_over_p": dd.dense_dft_plan_get_sched(plan)},
        "roofline": {"bound": "hbm", "achieved": b_alg / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "what": "end to end per step (fold + transform): algorithmic bytes batch*(N*8 + N/p*8)"},
    }
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.decimated_dft(x[0], p, T)
        el = time.perf_counter() - t0
        got = X[0].cpu().numpy()
        res["rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["cpu_baseline"] = {"value": len(ref) / el, "unit": "bins/s", "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"all {len(ref)} bins of signal 0 ({N} complex multiply-adds each), {el:.1f} s"}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch_c64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing leg")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="use the planner's built-in schedule rules instead of tuning first")
    ap.add_argument("--rates", default="1000,2000,5000,10000,20000,50000,100000,200000,400000,800000",
                    help="serving: Poisson arrival rates (requests/s)")
    ap.add_argument("--requests", type=int, default=10000, help="serving: requests per rate")
    ap.add_argument("--tune-db", default="", metavar="PATH",
                    help="default, real-input, inverse and uneven workloads: load the tuning table "
                         "from PATH if it exists, else tune and save it there (profiling runs then "
                         "time the same schedules)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="instead of the transform, run --steps plain device copies of MIB MiB "
                         "(calibrates the profiler's HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the transform of a "
                                   "batch shards by signal with no exchange, so multi-GPU runs "
                                   "are not measured", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    if args.copy_calib:
        n = args.copy_calib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"copy_bytes_each": n, "copies": args.steps,
                          "GBps_read_plus_write": 2 * n * args.steps / el / 1e9}))
        return

    import paper_2403_16665_amd as dd

    if args.workload == "uneven":
        run_uneven(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return
    if args.workload == "ablation":
        run_ablation(args)
        return
    if args.workload == "inverse":
        run_inverse(args)
        return
    if args.workload == "decimated":
        run_decimated(args)
        return

    w = WORKLOADS[args.workload]
    N, alpha, batch, dt = w["N"], w["alpha"], w["batch"], w["dt"]
    T = N * dt
    M = alpha * N
    x = make_inputs(args.workload, w)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(x).to(dev)
    code = dd.dtype_code(xd.dtype)
    tuning = None
    if args.tune_db and os.path.exists(args.tune_db):
        # a table saved by an earlier run: the same schedules, no tuner launches
        dd.dense_dft_tune_load(args.tune_db)
        tuning = {"loaded": args.tune_db}
    elif args.tune:
        t_tune = time.perf_counter()
        tuning = dd.dense_dft_tune(N, alpha, batch, code)
        tuning["seconds"] = time.perf_counter() - t_tune
        if args.tune_db:
            dd.dense_dft_tune_save(args.tune_db)
    plan = dd.dense_dft_plan(N, alpha, T, batch, code)
    Xd = torch.empty((batch, M), dtype=dd.out_dtype(code), device=dev)
    stream = torch.cuda.Stream(device=dev)
    sp = stream.cuda_stream

    for _ in range(args.warmup):
        dd.dense_dft_exec(plan, xd, Xd, stream=sp)
    torch.cuda.synchronize()

    # timed region: exactly K steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        dd.dense_dft_exec(plan, xd, Xd, stream=sp)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps

    # per-step device times (p50 / p99): the same K steps, one event pair each
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    for e0, e1 in step_ev:
        e0.record(stream)
        dd.dense_dft_exec(plan, xd, Xd, stream=sp)
        e1.record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([e0.elapsed_time(e1) for e0, e1 in step_ev])

    # the copy ceiling on this device: a plain 1 GiB device-to-device copy
    cbuf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cdst = torch.empty_like(cbuf)
    cdst.copy_(cbuf)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(3):
        cdst.copy_(cbuf)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * (1 << 30) / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del cbuf, cdst

    # per-kernel durations: the same K steps with every launch bracketed by events
    dd.dense_dft_profile_begin(plan, 1 << 16)
    for _ in range(args.steps):
        dd.dense_dft_exec(plan, xd, Xd, stream=sp)
    prof = dd.dense_dft_profile_end(plan, cap=1 << 16)
    kern = {}
    for kind, ms in prof:
        kern.setdefault(kind, []).append(ms)
    kernels = {k: {"launches": len(v), "avg_us": 1e3 * float(np.mean(v))} for k, v in kern.items()}
    kernel_ms_per_step = sum(sum(v) for v in kern.values()) / args.steps

    in_bytes = xd.element_size()
    out_bytes = Xd.element_size()
    b_alg = batch * (N * in_bytes + M * out_bytes)        # algorithmic bytes per step
    bins_per_step = batch * M
    value = bins_per_step / (ms_per_step * 1e-3)
    achieved = b_alg / (kernel_ms_per_step * 1e-3) / 1e9
    result = {
        "metric": "dense-spectrum bins/s & % HBM peak, batched vs plain at rel L2<=1e-5; p50/p99",
        "value": value,
        "unit": "bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "wall_ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if out_bytes == 16 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "batch": batch, "N": N, "alpha": alpha,
                   "dt": dt, "T": T, "input": w["input"], "bins_per_signal": M,
                   "schedule": dd.dense_dft_plan_get_sched(plan)},
        "tuning": tuning,
        "hbm_frac_end_to_end": b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "copy_ceiling_GBps": copy_gbs,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                     "what": "whole transform per step (all its kernels): algorithmic bytes "
                             "batch*(N*s_in + alpha*N*s_out) / summed kernel durations"},
    }
    traffic = result["roofline"]["traffic"]
    if traffic:
        result["roofline"]["amplification"] = traffic / b_alg   # measured HBM bytes / algorithmic
    if args.workload == "precision":
        result["precision"] = precision_errors(dd, xd, Xd, N, alpha, T)
    if args.workload == "real_f32":
        # the same samples through the complex path, which transforms every
        # scratch row instead of the Hermitian half
        xc = xd.to(torch.complex64)
        if args.tune:
            dd.dense_dft_tune(N, alpha, batch, dd.DD_C64)
        plan_c = dd.dense_dft_plan(N, alpha, T, batch, dd.DD_C64)
        Xc = torch.empty_like(Xd)
        for _ in range(args.warmup):
            dd.dense_dft_exec(plan_c, xc, Xc, stream=sp)
        ev0.record(stream)
        for _ in range(args.steps):
            dd.dense_dft_exec(plan_c, xc, Xc, stream=sp)
        ev1.record(stream)
        torch.cuda.synchronize()
        c_ms = ev0.elapsed_time(ev1) / args.steps
        worst = 0.0
        for b in range(0, batch, 51):
            d = (Xd[b] - Xc[b]).abs().pow(2).sum().sqrt() / Xc[b].abs().pow(2).sum().sqrt()
            worst = max(worst, float(d))
        result["complex_path"] = {"ms_per_step": c_ms, "real_path_speedup": c_ms / ms_per_step,
                                  "max_rel_l2_real_vs_complex": worst,
                                  "schedule": dd.dense_dft_plan_get_sched(plan_c)}
        del xc, Xc
    if not args.no_cpu:
        samples, cpu = cpu_baseline(x, alpha, T, M, N)
        got = np.concatenate([Xd[b].cpu().numpy()[bins] for b, bins, _ in samples])
        ref = np.concatenate([r for _, _, r in samples])
        result["rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["rel_l2_bins"] = int(len(ref))
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
