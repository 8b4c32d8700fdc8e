#!/usr/bin/env python3
"""Benchmark of the RSM hot path on one MI355X.  Prints one JSON line.

Default (the metric's own workloads):
  * value: batched RSM, decompositions/s of one fused library call over a batch of 256
    uneven problems (m U[4096, 65536], n U[128, 1024], r U{2..16}, rho U[0.6, 0.9],
    l = r + 1, I = 4n, FP32 data and Gram, FP64 eigen-solves), inputs resident in HBM.
    One step = one batched call; the same problems one at a time (plain RSM) beside it,
    with oracle parity on a seeded 64-problem sample, and the roofline of the batch's
    gather + Gram step (algorithmic bytes over its event-timed duration);
  * served: Poisson arrivals drawn from the batch's size distribution for 60 s at 0.5x
    and 0.9x the batched saturation rate, continuous batching against first-in first-out
    plain RSM on the same trace, p50 / p99 latency, and a seeded 5% of the requests
    compared with the same request run alone (plus an oracle check of a few);
  * paper_scale: one 131072 x 1024 problem (r 8, l 9, rho 0.8, 8192 sub-matrices):
    throughput, latency, per-step times, the Gram roofline, oracle parity, the oracle's
    CPU rate and a rows-first (method M2) summary;
  * precision: the precision-stress problem with the FP64, FP32 and split-BF16 Grams;
  * plain_fp64: the 2000 x 200 FP64 problem, latency p50 / p99 over 200 repetitions;
  * cpu_baseline: the FP64 oracle on the host, on one core and on all cores.
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

METRIC = "decompositions/s + p99 latency, batched/served vs plain RSM on 1 GPU, ≤1e-4 rad"
HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="suite",
                    choices=["suite", "paper_scale", "plain_fp64", "precision", "batched",
                             "served", "table1", "rows_first"],
                    help="suite (default): the batched headline with every other workload "
                         "summarised beside it")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--served-seconds", type=float, default=60.0)
    ap.add_argument("--served-budget-gib", type=float, default=128.0)
    ap.add_argument("--served-sample", type=float, default=0.05,
                    help="fraction of served requests compared with the same request alone")
    ap.add_argument("--parity-problems", type=int, default=64,
                    help="problems of the batch checked against the oracle")
    ap.add_argument("--no-batched", action="store_true",
                    help="paper_scale: omit nothing else (kept for the profiling commands)")
    ap.add_argument("--no-rows-first", action="store_true",
                    help="paper_scale: omit the rows-first (method M2) summary")
    ap.add_argument("--plain-gram", action="store_true",
                    help="per-trial column-streaming Gram kernel instead of the tiled one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: omit the one-at-a-time leg (for profiling runs)")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in Gram tile shapes (no autotuning before timing)")
    ap.add_argument("--tune-file", default=None,
                    help="install this saved tile table instead of autotuning")
    ap.add_argument("--save-tune", default=None,
                    help="write the tile table used for the timed run to this file")
    ap.add_argument("--cpu-sample-trials", type=int, default=4096)
    ap.add_argument("--cpu-sample-rows", type=int, default=2048,
                    help="rows of U in the parity checks")
    ap.add_argument("--cpu-sample-u-rows", type=int, default=49152)
    ap.add_argument("--workers", type=int, default=0,
                    help="oracle worker processes (0: the host's cores, at most 16)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (calibrates the "
                         "byte counters of rocprofv3 --pmc) and exit")
    return ap.parse_args()


def progress(msg):
    """One line per finished phase on stderr (the JSON result stays alone on stdout)."""
    print(f"[bench {time.perf_counter() - T_START:6.1f}s] {msg}", file=sys.stderr, flush=True)


def workers_of(args):
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return args.workers or max(1, min(16, cores or 1))


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "cores_available": aff}


def copy_probe(mib):
    """A plain copy kernel of known size: the byte counters' calibration."""
    import torch
    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 3}), flush=True)


def traffic_from_profile(kernel_src, profile="k_gram_dma_paper_scale_counters.md",
                         key="hbm_bytes_per_launch"):
    """HBM bytes of the Gram step from a committed rocprofv3 counter summary, or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    with open(kernel_src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return int(vals[key])
    except (KeyError, ValueError):
        return None


def make_workload(name):
    import synth
    if name == "paper_scale":
        return synth.paper_scale()
    if name == "plain_fp64":
        return synth.plain_fp64()
    if name == "rows_first":
        # the paper-scale problem sampled rows first (method M2, k = r + 1 = 9 rows)
        p = synth.paper_scale()
        p.name = "paper-scale shape, rows first (M2, k = 9)"
        p.rows_first = True
        return p
    return synth.precision_stress()


def _rows_first(p):
    return bool(getattr(p, "rows_first", False))


# ------------------------------------------------------------------ oracle legs (host)

_G = {}


def _oracle_chunk(args):
    """N over a trial range (worker process; inherits the problem through fork)."""
    from threadpoolctl import threadpool_limits

    from oracle import rsm
    lo, hi = args
    p = _G["p"]
    with threadpool_limits(limits=1):   # one BLAS thread per worker process
        if _G["rows_first"]:
            return rsm.accumulate_N_rows_first(p.Y, p.W, _G["subsets"][lo:hi], p.r, p.r + 1)[0]
        return rsm.accumulate_N(p.Y, p.W, _G["subsets"][lo:hi], p.r, p.l - p.r, p.r)[0]


def _oracle_u_chunk(args):
    """Rows [lo, hi) of U-hat for the V-hat in _G (worker process)."""
    from threadpoolctl import threadpool_limits

    from oracle import rsm
    lo, hi = args
    p = _G["p"]
    with threadpool_limits(limits=1):
        U, _ = rsm.solve_U(p.Y, p.W, _G["V"], rows=range(lo, hi))
    return U[lo:hi]


def _pool(workers):
    import multiprocessing as mp
    return mp.get_context("fork").Pool(workers)


def oracle_N(p, workers, rows_first=False):
    from oracle import rng
    subsets = rng.draw_subsets(p.seed_rsm, p.m if rows_first else p.n, p.l, p.num_submatrices)
    _G.update(p=p, subsets=subsets, rows_first=rows_first)
    chunks = np.array_split(np.arange(p.num_submatrices), workers * 4)
    ranges = [(int(c[0]), int(c[-1]) + 1) for c in chunks if len(c)]
    with _pool(workers) as pool:
        parts = pool.map(_oracle_chunk, ranges)
    return np.sum(parts, axis=0)


def oracle_parity(p, V_gpu, U_gpu, sample_rows, workers, rows_first=None):
    """theta_max of V-hat and rel RMS of U V^T (sampled rows) against the FP64 oracle.
    V_gpu / U_gpu may be lists (several GPU results of the same problem).  rows_first:
    sampling M2 (default: the workload's own)."""
    from oracle import metrics, rsm
    rows_first = _rows_first(p) if rows_first is None else rows_first
    t0 = time.perf_counter()
    N = oracle_N(p, workers, rows_first)
    V_ora, _ = rsm.solve_V(N, p.r)
    rows = np.linspace(0, p.m - 1, sample_rows).astype(np.int64)
    U_ora, _ = rsm.solve_U(p.Y, p.W, V_ora, rows=rows)
    t_oracle = time.perf_counter() - t0
    single = not isinstance(V_gpu, list)
    Vs, Us = ([V_gpu], [U_gpu]) if single else (V_gpu, U_gpu)
    out = [(metrics.principal_angle_max(V, V_ora),
            metrics.rel_rms_known(p.W[rows], U[rows], V, U_ora[rows], V_ora)) for V, U in zip(Vs, Us)]
    if single:
        return out[0][0], out[0][1], t_oracle
    return out, t_oracle


def cpu_baseline(p, n_trials, n_rows):
    """The oracle on one host core over a bounded sample, scaled to one decomposition."""
    from threadpoolctl import threadpool_limits

    from oracle import rng, rsm
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        if _rows_first(p):
            subsets = rng.draw_subsets(p.seed_rsm, p.m, p.l, n_trials)
            N, _, _ = rsm.accumulate_N_rows_first(p.Y, p.W, subsets, p.r, p.r + 1)
        else:
            subsets = rng.draw_subsets(p.seed_rsm, p.n, p.l, n_trials)
            N, _, _ = rsm.accumulate_N(p.Y, p.W, subsets, p.r, p.l - p.r, p.r)
        t_trials = time.perf_counter() - t0
        t0 = time.perf_counter()
        N = N + np.eye(p.n) * 1e-3
        V, _ = rsm.solve_V(N, p.r)
        t_eig = time.perf_counter() - t0
        rows = np.arange(n_rows)
        t0 = time.perf_counter()
        rsm.solve_U(p.Y, p.W, V, rows=rows)
        t_u = time.perf_counter() - t0
    est = t_trials * (p.num_submatrices / n_trials) + t_eig + t_u * (p.m / n_rows)
    return {
        "value": 1.0 / est, "unit": "decompositions/s", "cores": 1, "kind": "oracle",
        "sample": (f"{n_trials} of {p.num_submatrices} trials, {n_rows} of {p.m} rows of U, "
                   f"one n x n eigh; scaled to one decomposition ({est:.1f} s estimated)"),
        "measured_s": round(t_trials + t_eig + t_u, 2),
    }


def cpu_all_cores(p, workers):
    """One whole decomposition by the oracle on `workers` host cores: the trials split over
    worker processes (one BLAS thread each), the partial N summed, eigh, then the rows of
    U-hat split over the workers."""
    from oracle import rsm
    t0 = time.perf_counter()
    N = oracle_N(p, workers)
    V, _ = rsm.solve_V(N, p.r)
    _G["V"] = V
    chunks = np.array_split(np.arange(p.m), workers * 4)
    with _pool(workers) as pool:
        pool.map(_oracle_u_chunk, [(int(c[0]), int(c[-1]) + 1) for c in chunks if len(c)])
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "decompositions/s", "cores": workers, "kind": "oracle",
            "sample": "one whole decomposition (every trial, every row of U-hat)",
            "measured_s": round(t, 2)}


def _oracle_item(k):
    """Oracle parity of one problem of _G["items"] (worker process): N from every trial,
    V-hat, U-hat on the sampled rows; (theta_max, rel RMS, seconds)."""
    from threadpoolctl import threadpool_limits

    from oracle import metrics, rng, rsm
    d = _G["items"][k]
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        n = d["W"].shape[1]
        subsets = rng.draw_subsets(d["seed"], n, d["l"], d["I"])
        N, _, _ = rsm.accumulate_N(d["Y"], d["W"], subsets, d["r"], d["l"] - d["r"], d["r"])
        V, _ = rsm.solve_V(N, d["r"])
        rows = d["rows"]
        U, _ = rsm.solve_U(d["Y"], d["W"], V, rows=rows)
    theta = metrics.principal_angle_max(d["V"], V)
    rms = metrics.rel_rms_known(d["W"][rows], d["U_rows"], d["V"], U[rows], V)
    return float(theta), float(rms), time.perf_counter() - t0


def _oracle_full(k):
    """One whole oracle decomposition of _G["items"][k] on one core; seconds."""
    from threadpoolctl import threadpool_limits

    from oracle import rsm
    d = _G["items"][k]
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        rsm.rsm(d["Y"], d["W"], d["r"], d["I"], seed=d["seed"], l=d["l"], with_e=False)
    return time.perf_counter() - t0


def oracle_items(items, workers, fn=_oracle_item):
    """fn over host problem records in chunks of `workers` forked processes."""
    out = []
    for k0 in range(0, len(items), workers):
        chunk = items[k0:k0 + workers]
        _G["items"] = chunk
        with _pool(min(workers, len(chunk))) as pool:
            out.extend(pool.map(fn, range(len(chunk))))
    _G.pop("items", None)
    return out


def _host_record(Y, W, r, I, seed, l, V=None, U=None, sample_rows=0, rows=None):
    """A problem on the host for the oracle legs (Y, W as (m, n) arrays)."""
    Yh, Wh = Y.cpu().numpy(), W.cpu().numpy().astype(bool)
    m = Yh.shape[0]
    if rows is None and sample_rows:
        rows = np.linspace(0, m - 1, min(m, sample_rows)).astype(np.int64)
    d = {"Y": Yh, "W": Wh, "r": r, "I": I, "seed": seed, "l": l, "rows": rows}
    if V is not None:
        d["V"] = V
        d["U_rows"] = U
    return d


# ------------------------------------------------------------------ C1: paper scale

def run_single(args, torch, p, steps, warmup, autotune=True):
    """Timed decompositions of one resident problem: throughput, latency, per-step times
    from HIP events on the launch stream, the Gram roofline, the last result."""
    from paper_1411_0814_amd import Request, _lib, decompose, tune, workspace_bytes
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(p.Yt).to(dev).T
    W = torch.from_numpy(p.Wt.view(bool)).to(dev).T
    gram = p.gram
    flags = _lib.PLAIN_GRAM if args.plain_gram else 0
    rows_first = _rows_first(p)
    if rows_first:
        flags = _lib.ROWS_FIRST
    stream = torch.cuda.current_stream(dev)
    req = Request(Y=Y, W=W, r=p.r, num_submatrices=p.num_submatrices, seed=p.seed_rsm, l=p.l,
                  gram=gram, flags=flags)
    tune.clear()
    tuned = None
    if autotune and not (args.no_tune or args.plain_gram or rows_first or gram == "f64"):
        tuned = _tune_for(args, [req])
    ws_need = workspace_bytes([req])
    ws = torch.empty(ws_need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + ws_need]
    nev = 2 * len(_lib.STEPS)

    def new_events():
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nev)]
        for e in evs:
            e.record(stream)  # materialise the handle
        return evs

    def run(evs):
        return decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram,
                         flags=flags, workspace=ws, events=evs, stream=stream)

    for _ in range(warmup):
        res = run(new_events())
    torch.cuda.synchronize()
    events = [new_events() for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run(events[k]) for k in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    names = _lib.STEPS
    per_step = {name: [] for name in names}
    latency = []
    for evs in events:
        for k, name in enumerate(names):
            if name == "error":
                continue
            per_step[name].append(evs[2 * k].elapsed_time(evs[2 * k + 1]))
        latency.append(evs[0].elapsed_time(evs[2 * names.index("usolve") + 1]))
    last = results[-1]
    info = last.info()
    gram_ms = float(np.mean(per_step["gram"]))
    elem = 4 if p.Yt.dtype == np.float32 else 8
    if rows_first:
        # M2: the k row words of the mask and the k x |C_t| qualifying values per trial
        b_alg = p.num_submatrices * p.l * ((p.n + 7) // 8) + info["rows_total"] * p.l * elem
        gram_name = "gram (M2: column qualification + k x k Gram)"
        traffic = None
    else:
        b_alg = p.num_submatrices * p.l * ((p.m + 7) // 8) + info["rows_total"] * p.l * elem
        gram_name = "gram (row qualification + Gram)"
        traffic = traffic_from_profile(
            os.path.join(ROOT, "paper_1411_0814_amd", "csrc", "k_gram.hip"))
    achieved = b_alg / (gram_ms * 1e-3) / 1e9
    out = {
        "decompositions_per_s": round(steps / elapsed, 3),
        "steps": steps, "warmup": warmup,
        "ms_per_step": round(elapsed / steps * 1e3, 4),
        "config": {"workload": p.name, "m": p.m, "n": p.n, "r": p.r, "l": p.l,
                   "num_submatrices": p.num_submatrices, "rho": p.rho, "gram": gram,
                   "sampling": "rows first (M2)" if rows_first else "columns first (M1)",
                   "gram_kernel": "plain" if args.plain_gram else "tiled",
                   "eig_solves": "f64"},
        "latency_ms": {"p50": round(float(np.percentile(latency, 50)), 4),
                       "p99": round(float(np.percentile(latency, 99)), 4)},
        "step_ms": {k: round(float(np.mean(v)), 4) for k, v in per_step.items() if v},
        "roofline": {"bound": "hbm", "kernel": gram_name,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_alg_per_launch": int(b_alg), "launch_ms": round(gram_ms, 4)},
        "info": {"accepted": info["accepted"],
                 "mean_rows": info["rows_total"] / max(1, p.num_submatrices),
                 "warnings": info["warnings"], "residual": info["residual"],
                 "eig_iterations": info["eig_iterations"],
                 "lambda_r": info["lambda"][p.r - 1], "lambda_r1": info["lambda"][p.r]},
    }
    if tuned is not None:
        out["autotune"] = {"seconds": tuned["seconds"], "entries": tuned["entries"],
                           "groups": tuned["groups"]}
    V, U = last.V.cpu().numpy(), last.U.cpu().numpy()
    return out, V, U, (Y, W, stream)


def run_paper_scale(args, torch):
    from paper_1411_0814_amd import tune
    t0 = time.perf_counter()
    p = make_workload("paper_scale")
    t_gen = time.perf_counter() - t0
    out, V, U, (Y, W, stream) = run_single(args, torch, p, 20, 3)
    out["gen_s"] = round(t_gen, 1)
    progress(f"paper scale: {out['ms_per_step']:.3f} ms per decomposition")
    if not args.no_rows_first:
        out["rows_first"] = run_rows_first(args, torch, p, Y, W, stream)
        progress("paper scale rows first done")
    del Y, W
    tune.clear()
    torch.cuda.empty_cache()
    return out, p, V, U


def paper_scale_host_legs(args, p, V, U, out):
    workers = workers_of(args)
    if not args.no_parity:
        theta, rms, t_or = oracle_parity(p, V, U, args.cpu_sample_rows, workers)
        out["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                         "rows_sampled_for_rms": args.cpu_sample_rows,
                         "oracle_s": round(t_or, 1), "oracle_workers": workers,
                         "pass": bool(theta <= 1e-4 and rms <= 1e-5)}
        progress(f"paper scale parity: theta {theta:.2e} rms {rms:.2e}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sample_trials, args.cpu_sample_u_rows)
        out["cpu_baseline_all_cores"] = cpu_all_cores(p, workers)
        progress("paper scale cpu baselines done")
    if "rows_first" in out and not args.no_parity:
        rf = out["rows_first"]
        theta, rms, _ = oracle_parity(p, rf.pop("_V"), rf.pop("_U"), args.cpu_sample_rows,
                                      workers, rows_first=True)
        rf["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                        "pass": bool(theta <= 1e-4 and rms <= 1e-5)}
    elif "rows_first" in out:
        out["rows_first"].pop("_V", None)
        out["rows_first"].pop("_U", None)


def run_rows_first(args, torch, p, Y, W, stream, steps=10, warmup=2):
    """The same resident problem sampled rows first (method M2, k = l rows per trial):
    decompositions/s over `steps` back-to-back calls (parity is added on the host later)."""
    from paper_1411_0814_amd import _lib, decompose
    kw = dict(l=p.l, gram=p.gram, flags=_lib.ROWS_FIRST, stream=stream)
    for _ in range(warmup):
        res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info = res.info()
    return {"decompositions_per_s": round(steps / elapsed, 3),
            "ms_per_decomposition": round(elapsed / steps * 1e3, 4),
            "k_rows_per_trial": p.l,
            "mean_qualifying_columns": info["rows_total"] / max(1, p.num_submatrices),
            "eig_iterations": info["eig_iterations"],
            "_V": res.V.cpu().numpy(), "_U": res.U.cpu().numpy()}


# ------------------------------------------------------------------ C3: batched

# The FP32 Gram's error in a trial's minor vectors grows as eps32 ||G_t|| / gap(G_t), and
# that gap closes as the trial's qualifying rows approach its l columns.  Problems whose
# expected qualifying rows per trial, m rho^l, fall below this many per column take the
# FP64 Gram (24 of the 256 problems of the mixed batch).
FP64_GRAM_BELOW_ROWS_PER_COLUMN = 4


def batch_gram(spec: dict) -> str:
    rows = spec["m"] * spec["rho"] ** spec["l"]
    return "f64" if rows < FP64_GRAM_BELOW_ROWS_PER_COLUMN * spec["l"] else "f32"


def _batch_setup(args, torch):
    """The mixed batch: 256 problems of uneven sizes drawn on the device, and requests."""
    import synth
    from paper_1411_0814_amd import Request
    specs = synth.batched_sizes(args.batch_count)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    inputs = [synth.batched_device(sp, dev) for sp in specs]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    reqs = [Request(Y=Y, W=W, r=sp["r"], num_submatrices=sp["num_submatrices"],
                    seed=sp["seed_rsm"], l=sp["l"], gram=batch_gram(sp))
            for sp, (Y, W) in zip(specs, inputs)]
    return specs, inputs, reqs, t_gen


def _tune_for(args, reqs):
    """The tile table for the timed runs: a saved one (--tune-file), else autotuned on
    these requests; optionally written out (--save-tune)."""
    from paper_1411_0814_amd import tune
    if args.tune_file:
        entries = tune.load(args.tune_file)
        out = {"seconds": 0.0, "entries": entries, "groups": [], "from_file": args.tune_file}
    else:
        out = tune.autotune(reqs, reps=3)
    if args.save_tune:
        tune.save(args.save_tune)
    return out


def _batch_ws(torch, reqs):
    from paper_1411_0814_amd import workspace_bytes
    ws_need = workspace_bytes(reqs)
    ws = torch.empty(ws_need + 256, dtype=torch.uint8, device="cuda")
    return ws[(-ws.data_ptr()) % 256:][:ws_need]


def _time_batch(reqs, steps, warmup, stream, torch, ws):
    """Seconds of each of `steps` fused calls over the batch (after `warmup` calls)."""
    from paper_1411_0814_amd import decompose_batched
    for _ in range(max(1, warmup)):
        res = decompose_batched(reqs, stream=stream, workspace=ws)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        res = decompose_batched(reqs, stream=stream, workspace=ws)
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs], res


def _batch_gram_roofline(reqs, stream, torch, ws):
    """One fused call with step events on one problem per Gram launch: the gather + Gram step
    of the batch (its launches run side by side on the library's lanes) from the first
    launch's start to the last one's end, and the algorithmic bytes of every problem's
    trials."""
    from dataclasses import replace

    from paper_1411_0814_amd import _lib, decompose_batched
    nev = 2 * len(_lib.STEPS)
    gi = _lib.STEPS.index("gram")
    # the library records a problem's step events around its launch group, and the Gram
    # step launches once per (l, precision) in this batch: one problem per group carries
    # events (recording 2 x 7 events for every problem would itself stretch the step)
    first = {}
    for k, q in enumerate(reqs):
        first.setdefault((q.l, q.gram), k)
    marked = sorted(first.values())
    evs = {}
    for k in marked:
        e = [torch.cuda.Event(enable_timing=True) for _ in range(nev)]
        for x in e:
            x.record(stream)
        evs[k] = e
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(stream)
    res = decompose_batched([replace(q, events=evs[k]) if k in evs else q
                             for k, q in enumerate(reqs)], stream=stream, workspace=ws)
    torch.cuda.synchronize()
    starts = [ref.elapsed_time(e[2 * gi]) for e in evs.values()]
    ends = [ref.elapsed_time(e[2 * gi + 1]) for e in evs.values()]
    span_ms = max(ends) - min(starts)
    b_alg = 0
    for q, r in zip(reqs, res):
        m, _ = q.Y.shape
        b_alg += q.num_submatrices * q.l * ((m + 7) // 8) + r.info()["rows_total"] * q.l * 4
    achieved = b_alg / (span_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "gram (row qualification + Gram), every problem of the batch",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(
                os.path.join(ROOT, "paper_1411_0814_amd", "csrc", "k_gram.hip"),
                "k_gram_dma_batched256_counters.md", "hbm_bytes_per_call"),
            "bytes_alg_per_launch": int(b_alg), "launch_ms": round(span_ms, 4),
            "note": "the step's launches (one per l and precision, side by side on four "
                    "streams) from the earliest start to the latest end of the step events of "
                    "one problem per launch; bytes summed over the batch; traffic from the "
                    "committed counters"}


def run_batched(args, torch):
    """Batched RSM (one fused call for the whole batch) vs plain RSM (the same problems one
    at a time through rsm_decompose on one stream).  The batch is timed with the built-in
    Gram tile shapes, then autotuned and timed again; the plain leg keeps the built-in
    shapes.  Returns the summary, the batch, and host records for the oracle legs."""
    from paper_1411_0814_amd import _lib, decompose, tune, workspace_bytes
    specs, inputs, reqs, t_gen = _batch_setup(args, torch)
    stream = torch.cuda.current_stream()
    ws = _batch_ws(torch, reqs)
    tune.clear()
    t_builtin, _ = _time_batch(reqs, 3, 1, stream, torch, ws)
    tuned = None
    if not args.no_tune:
        tuned = _tune_for(args, reqs)
    times, res = _time_batch(reqs, args.steps, args.warmup, stream, torch, ws)
    roof = _batch_gram_roofline(reqs, stream, torch, ws)
    progress(f"batched: {np.mean(times) * 1e3:.2f} ms per batch of {len(reqs)}")
    tune.clear()
    # plain: one at a time on one stream, one workspace sized for the largest problem
    plain_reqs = [] if args.no_plain else reqs
    ws1_need = max(workspace_bytes([q]) for q in reqs)
    ws1 = torch.empty(ws1_need + 256, dtype=torch.uint8, device="cuda")
    ws1 = ws1[(-ws1.data_ptr()) % 256:][:ws1_need]
    for q in plain_reqs[:8]:
        decompose(q.Y, q.W, q.r, q.num_submatrices, q.seed, l=q.l, gram=q.gram,
                  stream=stream, workspace=ws1)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in plain_reqs]
    t0 = time.perf_counter()
    for q, (a, b) in zip(plain_reqs, evs):
        a.record(stream)
        decompose(q.Y, q.W, q.r, q.num_submatrices, q.seed, l=q.l, gram=q.gram,
                  stream=stream, workspace=ws1)
        b.record(stream)
    torch.cuda.synchronize()
    t_plain = max(time.perf_counter() - t0, 1e-9)
    lat_plain = [a.elapsed_time(b) for a, b in evs] or [float("nan")]
    del ws1
    t_batch = float(np.mean(times))
    warn = [res[k].info() for k in range(len(reqs))]
    out = {
        "problems": len(reqs),
        "fp64_gram_problems": sum(q.gram == "f64" for q in reqs),
        "batched": {"decompositions_per_s": round(len(reqs) / t_batch, 1),
                    "ms_per_batch": round(t_batch * 1e3, 3),
                    "ms_per_batch_p50": round(float(np.percentile(times, 50)) * 1e3, 3),
                    "ms_per_batch_p99": round(float(np.percentile(times, 99)) * 1e3, 3),
                    "steps": args.steps, "warmup": args.warmup},
        "plain": {"decompositions_per_s": round(len(plain_reqs) / t_plain, 1),
                  "ms_total": round(t_plain * 1e3, 3),
                  "latency_ms": {"p50": round(float(np.percentile(lat_plain, 50)), 4),
                                 "p99": round(float(np.percentile(lat_plain, 99)), 4)}},
        "speedup": round(t_plain / t_batch, 2) if plain_reqs else None,
        "gen_s": round(t_gen, 2),
        "builtin_tiles": {"decompositions_per_s": round(len(reqs) / float(np.mean(t_builtin)), 1),
                          "ms_per_batch": round(float(np.mean(t_builtin)) * 1e3, 3)},
        "eig_iterations": {"max": max(i["eig_iterations"] for i in warn),
                           "median": float(np.median([i["eig_iterations"] for i in warn]))},
        "roofline": roof,
    }
    if tuned is not None:
        out["autotune"] = {"seconds": tuned["seconds"], "entries": len(tuned["entries"]),
                           "groups": tuned["groups"]}
    # the seeded parity sample, copied to the host now (the oracle runs later)
    records = []
    if not args.no_parity and args.parity_problems > 0:
        degenerate = _lib.W_NO_CONSTRAINTS | _lib.W_RANK_DEFICIENT
        pick = np.random.default_rng(7).choice(len(reqs), min(len(reqs), args.parity_problems),
                                               replace=False)
        flagged = []
        for k in sorted(int(x) for x in pick):
            if warn[k]["warn"] & degenerate:
                flagged.append({"problem": k, "warnings": warn[k]["warnings"]})
                continue
            q = reqs[k]
            m = q.Y.shape[0]
            rows = np.linspace(0, m - 1, min(m, args.cpu_sample_rows)).astype(np.int64)
            d = _host_record(q.Y, q.W, q.r, q.num_submatrices, q.seed, q.l,
                             V=res[k].V.cpu().numpy(), U=res[k].U.cpu().numpy()[rows], rows=rows)
            d["problem"] = k
            inf = warn[k]
            d["detail"] = {"problem": k, "m": int(m), "n": int(q.Y.shape[1]), "r": q.r,
                           "rho": float(specs[k]["rho"]), "I": q.num_submatrices,
                           "accepted": inf["accepted"],
                           "mean_rows": inf["rows_total"] / max(1, q.num_submatrices),
                           "lambda_r": inf["lambda"][q.r - 1], "lambda_r1": inf["lambda"][q.r],
                           "residual": inf["residual"], "eig_iterations": inf["eig_iterations"]}
            records.append(d)
        out["parity"] = {"flagged_not_gated": flagged}
    del res, ws
    return out, (specs, inputs, reqs), records


def batched_host_legs(args, out, records):
    workers = workers_of(args)
    if records:
        t0 = time.perf_counter()
        res = oracle_items(records, workers)
        thetas = [r[0] for r in res]
        rmss = [r[1] for r in res]
        worst = sorted(range(len(res)), key=lambda k: -thetas[k])[:3]
        out["parity"]["worst"] = [dict(records[k]["detail"], theta=thetas[k], rms=rmss[k])
                                  for k in worst]
        out["parity"].update({
            "problems_checked": [d["problem"] for d in records],
            "sample": f"seeded {len(records)} of {out['problems']} problems (U-hat on up to "
                      f"{args.cpu_sample_rows} rows each)",
            "theta_max_rad": max(thetas), "rel_rms_known": max(rmss),
            "theta_median_rad": float(np.median(thetas)),
            "oracle_s": round(time.perf_counter() - t0, 1), "oracle_workers": workers,
            "pass": bool(max(thetas) <= 1e-4 and max(rmss) <= 1e-5)})
        progress(f"batched parity: theta {max(thetas):.2e} rms {max(rmss):.2e}")


def batched_cpu_baselines(args, records):
    """The oracle's rate on problems of the batch: whole decompositions (every row of
    U-hat) on one core, about 15 s of work, and on all cores, two problems per worker."""
    workers = workers_of(args)
    _G["items"] = records
    done, t0 = 0, time.perf_counter()
    while done < len(records) and time.perf_counter() - t0 < 15.0:
        _oracle_full(done)
        done += 1
    t1 = time.perf_counter() - t0
    one = {"value": done / t1, "unit": "decompositions/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} whole decompositions of the seeded parity sample of the batch "
                     f"(every trial and every row of U-hat), one after another",
           "measured_s": round(t1, 2)}
    k_all = min(len(records), 2 * workers)
    t0 = time.perf_counter()
    oracle_items(records[:k_all], workers, fn=_oracle_full)
    t_all = time.perf_counter() - t0
    allc = {"value": k_all / t_all, "unit": "decompositions/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{k_all} whole decompositions of the same sample, one per worker "
                      "process at a time (one BLAS thread each)",
            "measured_s": round(t_all, 2)}
    return one, allc


# ------------------------------------------------------------------ C4: served

def run_served(args, torch, batch, saturation):
    """Poisson traces at 0.5x and 0.9x the batched saturation rate, served with continuous
    batching and, on the same trace, first-in first-out one at a time (plain) over the same
    window.  A seeded fraction of the served requests keeps V-hat and a row sample of U-hat;
    each is compared with the same request run alone."""
    from oracle import metrics
    from paper_1411_0814_amd import _lib, decompose, serve
    specs, inputs, reqs = batch
    degenerate = _lib.W_NO_CONSTRAINTS | _lib.W_RANK_DEFICIENT
    pool = [serve.PoolItem(Y=q.Y, W=q.W, r=q.r, num_submatrices=q.num_submatrices, l=q.l,
                           gram=q.gram) for q in reqs]
    budget = int(args.served_budget_gib * (1 << 30))
    dev_rows, host_rows = [], []
    for q in reqs:
        m = q.Y.shape[0]
        rows = np.linspace(0, m - 1, min(m, 256)).astype(np.int64)
        host_rows.append(rows)
        dev_rows.append(torch.from_numpy(rows).cuda())
    levels, oracle_jobs = [], []
    for frac in (0.5, 0.9):
        qps = frac * saturation
        trace = serve.poisson_trace(len(pool), qps, args.served_seconds, seed=11)
        rng = np.random.default_rng(17)
        picked = rng.random(len(trace)) < args.served_sample
        sample = {j.rid: dev_rows[j.item] for j, s in zip(trace, picked) if s}
        # memory cached for earlier streams goes back to the device first (the runtime
        # allocates kernel scratch for each new queue from what is free)
        torch.cuda.empty_cache()
        srv = serve.Server(pool, budget_bytes=budget, batching=True, max_inflight=3)
        st_b = srv.run(trace, sample=sample)
        torch.cuda.synchronize()
        del srv
        progress(f"served {frac}x: continuous batching done ({len(trace)} requests)")
        # alone vs in the mix; requests the library flags as having no unique V-hat (no
        # accepted trial, an uncovered column or no eigen-gap) are counted apart
        worst_t, worst_r, n_cmp, n_flag = 0.0, 0.0, 0, 0
        cmp_jobs = []
        for j in trace:
            if j.kept is None:
                continue
            raw = bytes(j.kept[2].cpu().numpy().tobytes())
            if _lib.Info.from_buffer_copy(raw).warn & degenerate:
                n_flag += 1
            else:
                cmp_jobs.append(j)
        for j in cmp_jobs:
            it = pool[j.item]
            a = decompose(it.Y, it.W, it.r, it.num_submatrices, j.seed, l=it.l, gram=it.gram)
            Va, Ua = a.V.cpu().numpy(), a.U[dev_rows[j.item]].cpu().numpy()
            Vm, Um = j.kept[0].cpu().numpy(), j.kept[1].cpu().numpy()
            Wr = reqs[j.item].W[dev_rows[j.item]].cpu().numpy().astype(bool)
            worst_t = max(worst_t, metrics.principal_angle_max(Vm, Va))
            worst_r = max(worst_r, metrics.rel_rms_known(Wr, Um, Vm, Ua, Va))
            n_cmp += 1
        # a few sampled requests against the oracle, on the host later
        for j in cmp_jobs[:4]:
            oracle_jobs.append((frac, j.item, j.seed, j.kept[0].cpu().numpy(),
                                j.kept[1].cpu().numpy()))
        for j in trace:
            j.kept = None
        progress(f"served {frac}x: {n_cmp} sampled requests compared alone")
        trace_p = serve.poisson_trace(len(pool), qps, args.served_seconds, seed=11)
        torch.cuda.empty_cache()
        st_p = serve.Server(pool, budget_bytes=budget, batching=False, max_inflight=1).run(
            trace_p, time_limit=args.served_seconds)
        torch.cuda.synchronize()
        progress(f"served {frac}x: plain FIFO done ({st_p['completed']} of {len(trace_p)})")
        levels.append({
            "qps": round(qps, 1), "fraction_of_saturation": frac,
            "continuous_batching": st_b,
            "alone_vs_mix": {"sample": f"seeded {args.served_sample:.0%} of requests "
                                       f"({n_cmp + n_flag}); V-hat and U-hat on 256 rows",
                             "compared": n_cmp, "flagged_not_gated": n_flag,
                             "theta_max_rad": worst_t, "rel_rms_known": worst_r,
                             "pass": bool(worst_t <= 1e-4 and worst_r <= 1e-5)},
            "plain_fifo": st_p,
            "plain_fifo_note": (f"same trace, admission stopped at {args.served_seconds:.0f} s; "
                                "latency_all_ms counts unserved requests at the stop "
                                "(lower bounds)")})
    return {"seconds_per_level": args.served_seconds, "budget_gib": args.served_budget_gib,
            "levels": levels}, (oracle_jobs, host_rows)


def served_host_legs(args, served, oracle_jobs, reqs):
    workers = workers_of(args)
    jobs, rows = oracle_jobs
    if not jobs:
        return
    records = []
    for frac, item, seed, V, U in jobs:
        q = reqs[item]
        d = _host_record(q.Y, q.W, q.r, q.num_submatrices, seed, q.l, V=V, U=U,
                         rows=rows[item])
        d["frac"] = frac
        records.append(d)
    res = oracle_items(records, workers)
    for lv in served["levels"]:
        got = [r for d, r in zip(records, res) if d["frac"] == lv["fraction_of_saturation"]]
        if got:
            lv["oracle_check"] = {"requests": len(got),
                                  "theta_max_rad": max(g[0] for g in got),
                                  "rel_rms_known": max(g[1] for g in got),
                                  "pass": bool(max(g[0] for g in got) <= 1e-4 and
                                               max(g[1] for g in got) <= 1e-5)}


# ------------------------------------------------------------------ C2 and C0

def run_precision(args, torch, steps=3, warmup=1):
    """Precision stress: the same problem with the FP64 (control), FP32 and split-BF16
    Grams, each timed; host legs add each one's parity with the FP64 oracle."""
    from paper_1411_0814_amd import decompose
    p = make_workload("precision")
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(p.Yt).to(dev).T
    W = torch.from_numpy(p.Wt.view(bool)).to(dev).T
    stream = torch.cuda.current_stream(dev)
    runs = {}
    for gram in ("f64", "f32", "bf16x2"):
        for _ in range(max(1, warmup)):
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram)
        torch.cuda.synchronize()
        evs = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram)
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in evs]
        inf = res.info()
        runs[gram] = {"decompositions_per_s": round(1e3 / float(np.mean(ms)), 2),
                      "ms_p50": round(float(np.percentile(ms, 50)), 4),
                      "eig_iterations": inf["eig_iterations"], "residual": inf["residual"],
                      "warnings": inf["warnings"],
                      "lambda_r": inf["lambda"][p.r - 1], "lambda_r1": inf["lambda"][p.r],
                      "_V": res.V.cpu().numpy(), "_U": res.U.cpu().numpy()}
    del Y, W, res
    torch.cuda.empty_cache()
    return runs, p


def precision_host_legs(args, runs, p):
    workers = workers_of(args)
    grams = list(runs)
    pairs, t_or = oracle_parity(p, [runs[g].pop("_V") for g in grams],
                                [runs[g].pop("_U") for g in grams], args.cpu_sample_rows, workers)
    for (theta, rms), g in zip(pairs, grams):
        runs[g].update(theta_max_rad=theta, rel_rms_known=rms)
    return {"config": {"workload": p.name, "m": p.m, "n": p.n, "r": p.r, "l": p.l,
                       "num_submatrices": p.num_submatrices, "rho": p.rho,
                       "singular_values": "geometric 1 .. 1e-3", "noise": 1e-5},
            "gram_modes": runs, "oracle_s": round(t_or, 1),
            "note": "the f64 leg is the control (FP64 Gram on the same FP32 data): it "
                    "separates the V-hat solver from the Gram's rounding"}


def run_plain_fp64(args, torch, reps=200):
    """The 2000 x 200 FP64 problem: latency p50 / p99 over `reps` decompositions."""
    from paper_1411_0814_amd import decompose
    p = make_workload("plain_fp64")
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(p.Yt).to(dev).T
    W = torch.from_numpy(p.Wt.view(bool)).to(dev).T
    stream = torch.cuda.current_stream(dev)
    for _ in range(10):
        res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram="f64")
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram="f64")
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    info = res.info()
    out = {"config": {"workload": p.name, "m": p.m, "n": p.n, "r": p.r, "l": p.l,
                      "num_submatrices": p.num_submatrices, "rho": p.rho, "gram": "f64"},
           "repetitions": reps,
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                          "p99": round(float(np.percentile(lat, 99)), 4)},
           "eig_iterations": info["eig_iterations"], "warnings": info["warnings"],
           "_V": res.V.cpu().numpy(), "_U": res.U.cpu().numpy()}
    return out, p


def plain_host_legs(args, out, p):
    theta, rms, _ = oracle_parity(p, out.pop("_V"), out.pop("_U"), p.m, workers_of(args))
    out["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                     "pass": bool(theta <= 1e-4 and rms <= 1e-5)}


# ------------------------------------------------------------------ entry points

def main_suite(args):
    import torch
    host = host_info()
    bout, batch, records = run_batched(args, torch)
    saturation = bout["batched"]["decompositions_per_s"]
    served, oracle_jobs = run_served(args, torch, batch, saturation)
    specs, inputs, reqs = batch
    # the served oracle checks need the inputs on the host: copy those few now
    ojobs, rows = oracle_jobs
    served_records = []
    for frac, item, seed, V, U in ojobs:
        q = reqs[item]
        d = _host_record(q.Y, q.W, q.r, q.num_submatrices, seed, q.l, V=V, U=U, rows=rows[item])
        d["frac"] = frac
        served_records.append(d)
    del batch, inputs, reqs, specs
    torch.cuda.empty_cache()
    c1, p1, V1, U1 = run_paper_scale(args, torch)
    prec, p2 = run_precision(args, torch)
    progress("precision stress done")
    c0, p0 = run_plain_fp64(args, torch)
    progress("plain fp64 done")
    # host legs: oracle parity and the oracle's own rate
    batched_host_legs(args, bout, records)
    if served_records:
        res = oracle_items(served_records, workers_of(args))
        for lv in served["levels"]:
            got = [r for d, r in zip(served_records, res)
                   if d["frac"] == lv["fraction_of_saturation"]]
            if got:
                lv["oracle_check"] = {"requests": len(got),
                                      "theta_max_rad": max(g[0] for g in got),
                                      "rel_rms_known": max(g[1] for g in got),
                                      "pass": bool(max(g[0] for g in got) <= 1e-4 and
                                                   max(g[1] for g in got) <= 1e-5)}
        progress("served oracle checks done")
    cpu_one, cpu_all = (None, None)
    if not args.no_cpu_baseline and records:
        cpu_one, cpu_all = batched_cpu_baselines(args, records)
        progress("batched cpu baselines done")
    paper_scale_host_legs(args, p1, V1, U1, c1)
    precision = precision_host_legs(args, prec, p2)
    progress("precision parity done")
    plain_host_legs(args, c0, p0)
    line = {
        "metric": METRIC, "value": bout["batched"]["decompositions_per_s"],
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": bout["batched"]["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched {bout['problems']} problems in one call: m U[4096,65536], "
                               "n U[128,1024], r U{2..16}, rho U[0.6,0.9], l=r+1, I=4n, no noise",
                   "gram": f"f32; f64 where m rho^l < {FP64_GRAM_BELOW_ROWS_PER_COLUMN} l "
                           f"({bout['fp64_gram_problems']} problems)",
                   "eig_solves": "f64", "step": "one batched call"},
        "latency_ms": {"p50": bout["batched"]["ms_per_batch_p50"],
                       "p99": bout["batched"]["ms_per_batch_p99"],
                       "of": "one batched call (all 256 problems)"},
        "roofline": bout["roofline"],
        "cpu_baseline": cpu_one,
        "cpu_baseline_all_cores": cpu_all,
        "host": host,
        "batched": bout,
        "served": served,
        "paper_scale": c1,
        "precision": precision,
        "plain_fp64": c0,
        "wall_s": round(time.perf_counter() - T_START, 1),
    }
    print(json.dumps(line), flush=True)


def main_batched(args):
    import torch
    bout, batch, records = run_batched(args, torch)
    line = {
        "metric": METRIC, "value": bout["batched"]["decompositions_per_s"],
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": bout["batched"]["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched {bout['problems']} problems: m U[4096,65536], "
                               "n U[128,1024], r U{2..16}, rho U[0.6,0.9], l=r+1, I=4n",
                   "gram": "f32", "eig_solves": "f64"},
        "roofline": bout["roofline"],
        "batched": bout,
    }
    if args.workload == "served":
        served, ojobs = run_served(args, torch, batch, bout["batched"]["decompositions_per_s"])
        served_host_legs(args, served, ojobs, batch[2])
        line["served"] = served
    batched_host_legs(args, bout, records)
    print(json.dumps(line), flush=True)


def _table1_golden():
    import csv
    path = os.path.join(ROOT, "tests", "golden", "table1_rsm.csv")
    with open(path) as f:
        return [row for row in csv.DictReader(line for line in f if not line.startswith("#"))]


def main_table1(args):
    """The paper's Table I workloads (r = 3, l = 4, M1, I = 25n, FP64 data): GPU time per
    decomposition and the error e of eq.(ep) next to the paper's printed e and its
    one-core Matlab time (context: another machine, another random instance)."""
    import torch

    import synth
    from paper_1411_0814_amd import _lib, decompose
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rows = []
    total_ms = 0.0
    for k, gold in enumerate(_table1_golden()):
        p = synth.table1(k)
        Y = torch.from_numpy(p.Yt).to(dev).T
        W = torch.from_numpy(p.Wt.view(bool)).to(dev).T
        for _ in range(max(1, args.warmup)):
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram="f64",
                            flags=_lib.COMPUTE_ERROR)
        torch.cuda.synchronize()
        evs = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram="f64",
                            flags=_lib.COMPUTE_ERROR)
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        total_ms += ms
        e = res.info()["e"]
        e_paper = float(gold["e_rsm"])
        rows.append({"m": p.m, "n": p.n, "rho": p.rho, "sigma": float(gold["sigma"]),
                     "I": p.num_submatrices, "gpu_ms": round(ms, 4), "e": round(e, 6),
                     "e_paper": e_paper, "e_within_1e-3": bool(abs(e - e_paper) <= 1e-3),
                     "paper_matlab_s": float(gold["t_rsm"])})
        del Y, W, res
        torch.cuda.empty_cache()
    line = {
        "metric": METRIC, "value": round(len(rows) / (total_ms * 1e-3), 2),
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total_ms / len(rows), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Table I shapes: r 3, l 4, M1, I 25n, m 65536..131072, "
                               "n 512..1024, rho 0.2..0.5, sigma 0.1..0.5", "gram": "f64"},
        "rows": rows,
        "paper_hardware": "Matlab, FP64, one core of an Intel i5-3470 at 3.2 GHz",
        "all_e_within_1e-3": all(r["e_within_1e-3"] for r in rows),
        "fig1": fig1_slopes(rows),
    }
    print(json.dumps(line), flush=True)


def fig1_slopes(rows):
    """Time against m (n fixed) and against n (m fixed) over the Table I rows that vary one
    of them, both divided by their smallest values and fitted by a straight line, as the
    paper's Fig. 1 does (a slope below 1: time grows more slowly than the size); with the
    log-log exponent and the same fits of the paper's printed one-core times."""
    def fit(xs, ts):
        x = np.asarray(xs, float) / min(xs)
        t = np.asarray(ts, float) / min(ts)
        slope = float(np.polyfit(x, t, 1)[0])
        expo = float(np.polyfit(np.log(x), np.log(t), 1)[0])
        return round(slope, 3), round(expo, 3)
    out = {}
    for name, key, other in (("time_vs_m", "m", "n"), ("time_vs_n", "n", "m")):
        ref = max(r[other] for r in rows)
        sel = [r for r in rows if r[other] == ref and r["rho"] == 0.2 and r["sigma"] == 0.2]
        sel.sort(key=lambda r: r[key])
        if len(sel) < 2:
            continue
        xs = [r[key] for r in sel]
        g_slope, g_exp = fit(xs, [r["gpu_ms"] for r in sel])
        p_slope, p_exp = fit(xs, [r["paper_matlab_s"] for r in sel])
        out[name] = {key: xs, f"fixed_{other}": ref, "gpu_ms": [r["gpu_ms"] for r in sel],
                     "gpu_slope": g_slope, "gpu_loglog_exponent": g_exp,
                     "paper_matlab_s": [r["paper_matlab_s"] for r in sel],
                     "paper_slope": p_slope, "paper_loglog_exponent": p_exp}
    return out


def main_single(args):
    """One resident problem (paper_scale, rows_first, plain_fp64): the per-workload line the
    profiling commands run."""
    import torch
    t0 = time.perf_counter()
    p = make_workload(args.workload)
    t_gen = time.perf_counter() - t0
    progress(f"workload {p.name} generated in {t_gen:.1f} s")
    out, V, U, (Y, W, stream) = run_single(args, torch, p, args.steps, args.warmup)
    progress(f"{args.steps} timed steps: {out['ms_per_step']:.3f} ms each")
    if not args.no_rows_first and args.workload == "paper_scale":
        out["rows_first"] = run_rows_first(args, torch, p, Y, W, stream)
    del Y, W
    if args.no_parity and "rows_first" in out:
        out["rows_first"].pop("_V")
        out["rows_first"].pop("_U")
    if not args.no_parity:
        workers = workers_of(args)
        theta, rms, t_or = oracle_parity(p, V, U, args.cpu_sample_rows, workers)
        progress(f"oracle parity: theta {theta:.3e} rms {rms:.3e} ({t_or:.1f} s)")
        out["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                         "rows_sampled_for_rms": args.cpu_sample_rows,
                         "oracle_s": round(t_or, 1), "oracle_workers": workers,
                         "pass": bool(theta <= 1e-4 and rms <= 1e-5)}
        if "rows_first" in out:
            rf = out["rows_first"]
            th2, rm2, _ = oracle_parity(p, rf.pop("_V"), rf.pop("_U"), args.cpu_sample_rows,
                                        workers, rows_first=True)
            rf["parity"] = {"theta_max_rad": th2, "rel_rms_known": rm2,
                            "pass": bool(th2 <= 1e-4 and rm2 <= 1e-5)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sample_trials, args.cpu_sample_u_rows)
    line = {"metric": METRIC, "value": out.pop("decompositions_per_s"),
            "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if p.gram == "f32" else p.gram, "data": "synthetic",
            "config": out.pop("config")}
    out.pop("steps"), out.pop("warmup")
    line.update(out)
    print(json.dumps(line), flush=True)


def main_precision(args):
    import torch
    runs, p = run_precision(args, torch, steps=args.steps, warmup=args.warmup)
    prec = precision_host_legs(args, runs, p)
    line = {
        "metric": METRIC, "value": runs["bf16x2"]["decompositions_per_s"],
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs["bf16x2"]["ms_p50"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x2", "data": "synthetic",
        "config": prec["config"], "gram_modes": prec["gram_modes"], "oracle_s": prec["oracle_s"],
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "suite":
        main_suite(args)
    elif args.workload in ("batched", "served"):
        main_batched(args)
    elif args.workload == "precision":
        main_precision(args)
    elif args.workload == "table1":
        main_table1(args)
    else:
        main_single(args)


if __name__ == "__main__":
    main()
