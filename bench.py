#!/usr/bin/env python3
"""Benchmark of the RSM hot path on one MI355X.

One step = one whole decomposition (steps a0..a7: mask packing, subset draw, row
qualification + Gram, minor vectors + N, V-hat, U-hat) of the paper-scale problem
131072 x 1024, r = 8, l = 9, rho = 0.8, 8192 sub-matrices, FP32 data and Gram, FP64
eigen-solves — with Y and W already resident in HBM.  Prints one JSON line.

Also reported:
  * latency p50 / p99 of one decomposition (HIP events on the launch stream);
  * the roofline of the dominant kernel (row qualification + Gram) against HBM, from its
    algorithmic bytes (the l mask bit-columns and the l values of every qualifying row, per
    trial) over its event-timed duration;
  * parity of the measured run against the FP64 oracle (largest principal angle of V-hat,
    relative RMS of U V^T on a sample of rows);
  * the oracle itself timed on the host on a bounded sample of the same workload.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper_scale",
                    choices=["paper_scale", "plain_fp64", "precision", "batched", "served",
                             "table1", "rows_first"])
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--served-seconds", type=float, default=5.0)
    ap.add_argument("--served-budget-gib", type=float, default=16.0)
    ap.add_argument("--parity-problems", type=int, default=16,
                    help="problems of the batch checked against the oracle")
    ap.add_argument("--no-batched", action="store_true",
                    help="omit the batched / served summaries from the default line")
    ap.add_argument("--no-rows-first", action="store_true",
                    help="omit the rows-first (method M2) summary from the default line")
    ap.add_argument("--plain-gram", action="store_true",
                    help="per-trial column-streaming Gram kernel instead of the tiled one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in Gram tile shapes (no autotuning before timing)")
    ap.add_argument("--tune-file", default=None,
                    help="install this saved tile table instead of autotuning")
    ap.add_argument("--save-tune", default=None,
                    help="write the tile table used for the timed run to this file")
    ap.add_argument("--cpu-sample-trials", type=int, default=4096)
    ap.add_argument("--cpu-sample-rows", type=int, default=2048,
                    help="rows of U in the parity check")
    ap.add_argument("--cpu-sample-u-rows", type=int, default=49152)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (calibrates the "
                         "byte counters of rocprofv3 --pmc) and exit")
    return ap.parse_args()


def progress(msg):
    """One line per finished phase on stderr (the JSON result stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def traffic_from_profile(kernel_src):
    """HBM bytes per launch of the Gram kernel from the committed rocprofv3 counter summary,
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_gram_tile_paper_scale_counters.md")
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
        return int(vals["hbm_bytes_per_launch"])
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


def _oracle_chunk(args):
    """N over a trial range (worker process; inherits the problem through fork)."""
    from threadpoolctl import threadpool_limits

    from oracle import rsm
    lo, hi = args
    p = _G["p"]
    with threadpool_limits(limits=1):   # one BLAS thread per worker process
        return _oracle_chunk_body(p, lo, hi, rsm, _G["rows_first"])


def _oracle_chunk_body(p, lo, hi, rsm, rows_first):
    if rows_first:
        return rsm.accumulate_N_rows_first(p.Y, p.W, _G["subsets"][lo:hi], p.r, p.r + 1)[0]
    return rsm.accumulate_N(p.Y, p.W, _G["subsets"][lo:hi], p.r, p.l - p.r, p.r)[0]


_G = {}


def oracle_parity(p, V_gpu, U_gpu, sample_rows, workers, rows_first=None):
    """theta_max of V-hat and rel RMS of U V^T (sampled rows) against the FP64 oracle.
    V_gpu / U_gpu may be lists (several GPU results of the same problem).  rows_first:
    sampling M2 (default: the workload's own)."""
    import multiprocessing as mp

    from oracle import metrics, rng, rsm
    rows_first = _rows_first(p) if rows_first is None else rows_first
    subsets = rng.draw_subsets(p.seed_rsm, p.m if rows_first else p.n, p.l, p.num_submatrices)
    _G.update(p=p, subsets=subsets, rows_first=rows_first)
    t0 = time.perf_counter()
    chunks = np.array_split(np.arange(p.num_submatrices), workers * 4)
    ranges = [(int(c[0]), int(c[-1]) + 1) for c in chunks if len(c)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_oracle_chunk, ranges)
    N = np.sum(parts, axis=0)
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


def run_rows_first(args, torch, p, Y, W, stream, steps=10, warmup=2):
    """The same resident problem sampled rows first (method M2, k = l rows per trial):
    decompositions/s over `steps` back-to-back calls and parity against the oracle."""
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
    out = {"decompositions_per_s": round(steps / elapsed, 3),
           "ms_per_decomposition": round(elapsed / steps * 1e3, 4),
           "k_rows_per_trial": p.l, "mean_qualifying_columns": info["rows_total"] / max(1, p.num_submatrices)}
    if not args.no_parity:
        workers = min(16, os.cpu_count() or 4)
        theta, rms, _ = oracle_parity(p, res.V.cpu().numpy(), res.U.cpu().numpy(),
                                      args.cpu_sample_rows, workers, rows_first=True)
        out["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                         "pass": bool(theta <= 1e-4 and rms <= 1e-5)}
    return out


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
                    seed=sp["seed_rsm"], l=sp["l"], gram="f32")
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


def _time_batch(reqs, reps, stream, torch):
    """Median seconds of one fused call over the batch (after one warm-up call)."""
    from paper_1411_0814_amd import decompose_batched, workspace_bytes
    ws_need = workspace_bytes(reqs)
    ws = torch.empty(ws_need + 256, dtype=torch.uint8, device="cuda")
    ws = ws[(-ws.data_ptr()) % 256:][:ws_need]
    res = decompose_batched(reqs, stream=stream, workspace=ws)   # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        res = decompose_batched(reqs, stream=stream, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    return float(np.median(times)), res


def run_batched(args, torch):
    """Batched RSM (one fused call for the whole batch) vs plain RSM (the same problems one
    at a time through rsm_decompose on one stream), with oracle parity on a sample.  The
    batch is timed with the built-in Gram tile shapes, then autotuned and timed again; the
    plain leg keeps the built-in shapes."""
    from paper_1411_0814_amd import decompose, tune, workspace_bytes
    specs, inputs, reqs, t_gen = _batch_setup(args, torch)
    stream = torch.cuda.current_stream()
    tune.clear()
    t_builtin, res = _time_batch(reqs, args.batch_reps, stream, torch)
    tuned = None
    if not args.no_tune:
        tuned = _tune_for(args, reqs)
        t_batch, res = _time_batch(reqs, args.batch_reps, stream, torch)
    else:
        t_batch = t_builtin
    # plain: one at a time on one stream, one workspace sized for the largest problem
    ws1_need = max(workspace_bytes([q]) for q in reqs)
    ws1 = torch.empty(ws1_need + 256, dtype=torch.uint8, device="cuda")
    ws1 = ws1[(-ws1.data_ptr()) % 256:][:ws1_need]
    for q in reqs[:8]:
        decompose(q.Y, q.W, q.r, q.num_submatrices, q.seed, l=q.l, gram=q.gram,
                  stream=stream, workspace=ws1)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in reqs]
    t0 = time.perf_counter()
    for q, (a, b) in zip(reqs, evs):
        a.record(stream)
        decompose(q.Y, q.W, q.r, q.num_submatrices, q.seed, l=q.l, gram=q.gram,
                  stream=stream, workspace=ws1)
        b.record(stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    lat_plain = [a.elapsed_time(b) for a, b in evs]
    out = {
        "problems": len(reqs),
        "batched": {"decompositions_per_s": round(len(reqs) / t_batch, 1),
                    "ms_per_batch": round(t_batch * 1e3, 3), "reps": args.batch_reps},
        "plain": {"decompositions_per_s": round(len(reqs) / t_plain, 1),
                  "ms_total": round(t_plain * 1e3, 3),
                  "latency_ms": {"p50": round(float(np.percentile(lat_plain, 50)), 4),
                                 "p99": round(float(np.percentile(lat_plain, 99)), 4)}},
        "speedup": round(t_plain / t_batch, 2),
        "gen_s": round(t_gen, 2),
        "builtin_tiles": {"decompositions_per_s": round(len(reqs) / t_builtin, 1),
                          "ms_per_batch": round(t_builtin * 1e3, 3)},
    }
    if tuned is not None:
        out["autotune"] = {"seconds": tuned["seconds"], "entries": len(tuned["entries"]),
                           "groups": tuned["groups"]}
    if not args.no_parity and args.parity_problems > 0:
        # a seeded sample of the batch against the oracle; problems the library flags as
        # having no well-defined V-hat (no accepted trial, or an uncovered column / no
        # eigen-gap) are listed apart and kept out of the angle gate
        from oracle import metrics, rsm
        from paper_1411_0814_amd import _lib
        degenerate = _lib.W_NO_CONSTRAINTS | _lib.W_RANK_DEFICIENT
        pick = np.random.default_rng(7).choice(len(reqs), args.parity_problems, replace=False)
        worst_t, worst_r, t_or = 0.0, 0.0, time.perf_counter()
        checked, flagged = [], []
        for k in sorted(int(x) for x in pick):
            info = res[k].info()
            if info["warn"] & degenerate:
                flagged.append({"problem": k, "warnings": info["warnings"]})
                continue
            Y = reqs[k].Y.cpu().numpy()
            W = reqs[k].W.cpu().numpy()
            ora = rsm.rsm(Y, W, reqs[k].r, reqs[k].num_submatrices, seed=reqs[k].seed,
                          l=reqs[k].l, with_e=False)
            V, U = res[k].V.cpu().numpy(), res[k].U.cpu().numpy()
            worst_t = max(worst_t, metrics.principal_angle_max(V, ora.V))
            worst_r = max(worst_r, metrics.rel_rms_known(W, U, V, ora.U, ora.V))
            checked.append(k)
        out["parity"] = {"problems_checked": checked, "flagged_not_gated": flagged,
                         "theta_max_rad": worst_t, "rel_rms_known": worst_r,
                         "oracle_s": round(time.perf_counter() - t_or, 1),
                         "pass": bool(worst_t <= 1e-4 and worst_r <= 1e-5)}
    return out, (specs, inputs, reqs)


def run_served(args, torch, batch, saturation):
    """Poisson traces at 0.5x and 0.9x the batched saturation rate, served with continuous
    batching and, on the same trace, first-in first-out one at a time (plain)."""
    from paper_1411_0814_amd import serve
    specs, inputs, reqs = batch
    pool = [serve.PoolItem(Y=q.Y, W=q.W, r=q.r, num_submatrices=q.num_submatrices, l=q.l,
                           gram=q.gram) for q in reqs]
    budget = int(args.served_budget_gib * (1 << 30))
    levels = []
    for frac in (0.5, 0.9):
        qps = frac * saturation
        trace = serve.poisson_trace(len(pool), qps, args.served_seconds, seed=11)
        srv = serve.Server(pool, budget_bytes=budget, batching=True, max_inflight=3)
        st_b = srv.run(trace)
        trace_p = serve.poisson_trace(len(pool), qps, args.served_seconds, seed=11)
        st_p = serve.Server(pool, budget_bytes=budget, batching=False, max_inflight=1).run(
            trace_p, time_limit=4 * args.served_seconds)
        torch.cuda.synchronize()
        levels.append({"qps": round(qps, 1), "fraction_of_saturation": frac,
                       "continuous_batching": st_b, "plain_fifo": st_p})
    return {"seconds_per_level": args.served_seconds, "budget_gib": args.served_budget_gib,
            "levels": levels}


def main_batched(args):
    import torch
    out, batch = run_batched(args, torch)
    line = {
        "metric": METRIC, "value": out["batched"]["decompositions_per_s"],
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.batch_reps, "warmup": 1,
        "ms_per_step": out["batched"]["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched {out['problems']} problems: m U[4096,65536], "
                               "n U[128,1024], r U{2..16}, rho U[0.6,0.9], l=r+1, I=4n",
                   "gram": "f32", "eig_solves": "f64"},
        "batched": out,
    }
    if args.workload == "served":
        line["served"] = run_served(args, torch, batch, out["batched"]["decompositions_per_s"])
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
    }
    print(json.dumps(line), flush=True)


def main_precision(args):
    """Precision stress: the same problem with the FP32 Gram and with the split-BF16 Gram on
    MFMA, each timed and compared with one FP64 oracle run."""
    import torch

    from paper_1411_0814_amd import decompose
    p = make_workload("precision")
    dev = torch.device("cuda:0")
    Y = torch.from_numpy(p.Yt).to(dev).T
    W = torch.from_numpy(p.Wt.view(bool)).to(dev).T
    stream = torch.cuda.current_stream(dev)
    runs = {}
    for gram in ("f64", "f32", "bf16x2"):
        for _ in range(max(1, args.warmup)):
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram)
        torch.cuda.synchronize()
        evs = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram)
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in evs]
        runs[gram] = {"decompositions_per_s": round(1e3 / float(np.mean(ms)), 2),
                      "ms_p50": round(float(np.percentile(ms, 50)), 4),
                      "ms_p99": round(float(np.percentile(ms, 99)), 4),
                      "V": res.V.cpu().numpy(), "U": res.U.cpu().numpy(),
                      "info": res.info()}
    workers = min(16, os.cpu_count() or 4)
    pairs, t_or = oracle_parity(p, [runs[g]["V"] for g in runs], [runs[g]["U"] for g in runs],
                                args.cpu_sample_rows, workers)
    # the generating V (orthonormal, strongest direction first): how much of it each
    # precision recovers, per leading k
    Vbar = np.linalg.qr(p.Vbar)[0]
    for (theta, rms), g in zip(pairs, runs):
        runs[g].update(theta_max_rad=theta, rel_rms_known=rms)
        Vg = np.linalg.qr(runs[g]["V"])[0]
        # largest angle between the leading k generating directions and span(V-hat)
        runs[g]["theta_vs_generating_V_leading_k"] = {
            str(k): float(np.arcsin(min(1.0, np.linalg.norm(
                Vbar[:, :k] - Vg @ (Vg.T @ Vbar[:, :k]), 2)))) for k in (4, 6, 7, 8)}
        inf = runs[g].pop("info")
        lam = inf["lambda"]
        runs[g]["lambda_r"], runs[g]["lambda_r1"] = lam[p.r - 1], lam[p.r]
        runs[g].update(eig_iterations=inf["eig_iterations"], residual=inf["residual"],
                       warnings=inf["warnings"])
        del runs[g]["V"], runs[g]["U"]
    line = {
        "metric": METRIC, "value": runs["bf16x2"]["decompositions_per_s"],
        "unit": "decompositions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": runs["bf16x2"]["ms_p50"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x2", "data": "synthetic",
        "config": {"workload": p.name, "m": p.m, "n": p.n, "r": p.r, "l": p.l,
                   "num_submatrices": p.num_submatrices, "rho": p.rho,
                   "singular_values": "geometric 1 .. 1e-3", "noise": 1e-5,
                   "eig_solves": "f64"},
        "gram_modes": runs,
        "oracle": {"s": round(t_or, 1), "workers": workers, "rows_sampled_for_rms": args.cpu_sample_rows},
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
    if args.workload in ("batched", "served"):
        main_batched(args)
        return
    if args.workload == "precision":
        main_precision(args)
        return
    if args.workload == "table1":
        main_table1(args)
        return
    import torch

    from paper_1411_0814_amd import _lib, decompose, workspace_bytes, Request

    t_gen = time.perf_counter()
    p = make_workload(args.workload)
    t_gen = time.perf_counter() - t_gen
    progress(f"workload {p.name} generated in {t_gen:.1f} s")
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
    from paper_1411_0814_amd import tune
    tune.clear()
    tuned = None if args.no_tune or args.plain_gram or rows_first else _tune_for(args, [req])
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

    for _ in range(args.warmup):
        res = run(new_events())
    torch.cuda.synchronize()
    progress(f"{args.warmup} warm-up steps done")
    events = [new_events() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run(events[k]) for k in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"{args.steps} timed steps: {elapsed / args.steps * 1e3:.3f} ms each")

    steps = _lib.STEPS
    per_step = {name: [] for name in steps}
    latency = []
    for evs in events:
        for k, name in enumerate(steps):
            if name == "error":
                continue
            per_step[name].append(evs[2 * k].elapsed_time(evs[2 * k + 1]))
        latency.append(evs[0].elapsed_time(evs[2 * steps.index("usolve") + 1]))
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
        "metric": METRIC,
        "value": round(args.steps / elapsed, 3),
        "unit": "decompositions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if gram == "f32" else gram,
        "data": "synthetic",
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
        "info": {"accepted": info["accepted"], "mean_rows": info["rows_total"] / max(1, p.num_submatrices),
                 "warnings": info["warnings"], "residual": info["residual"],
                 "lambda_r": info["lambda"][p.r - 1], "lambda_r1": info["lambda"][p.r]},
        "gen_s": round(t_gen, 1),
    }
    if tuned is not None:
        out["autotune"] = {"seconds": tuned["seconds"], "entries": tuned["entries"],
                           "groups": tuned["groups"]}
    if not args.no_parity:
        workers = min(16, os.cpu_count() or 4)
        theta, rms, t_or = oracle_parity(p, last.V.cpu().numpy(), last.U.cpu().numpy(),
                                         args.cpu_sample_rows, workers)
        progress(f"oracle parity: theta {theta:.3e} rms {rms:.3e} ({t_or:.1f} s)")
        out["parity"] = {"theta_max_rad": theta, "rel_rms_known": rms,
                         "rows_sampled_for_rms": args.cpu_sample_rows,
                         "oracle_s": round(t_or, 1), "oracle_workers": workers,
                         "pass": bool(theta <= 1e-4 and rms <= 1e-5)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_sample_trials, args.cpu_sample_u_rows)
        progress("cpu baseline done")
    if not args.no_rows_first and args.workload == "paper_scale":
        out["rows_first"] = run_rows_first(args, torch, p, Y, W, stream)
        progress("rows-first summary done")
    if not args.no_batched and args.workload == "paper_scale":
        del Y, W, ws, results, res, last
        torch.cuda.empty_cache()
        bout, batch = run_batched(args, torch)
        out["batched"] = bout
        out["served"] = run_served(args, torch, batch, bout["batched"]["decompositions_per_s"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
