"""Autotuner of the gather + Gram step's tile shapes.

The tiled Gram kernel (steps a2 + a3) has three free parameters per launch: how Y is
staged into LDS (through registers in 32-row chunks, or loaded straight into LDS in
16-row chunks, which leaves more registers for the trials' accumulators), the trials per
workgroup (one thread per trial, so also the workgroup size) and the number of workgroups
the launch aims for, which sets how many row splits each trial's Gram is cut into (their
partial Grams are summed afterwards, in the minor-vector step).  They trade occupancy
against re-reads of Y and partial-sum traffic, and the best choice depends on l, Y's
element type, the Gram precision and on whether the launch serves one problem or a batch.

`autotune(requests)` groups the requests the way the library groups its launches, times
every candidate pair on those very problems (the Gram and minor-vector steps, which hold
the partial-sum reduction, bracketed by stream events), and installs the fastest pair of
each group in the library's tile table.  `save` / `load` keep a table as JSON; a table
named by the environment variable RSM_TUNE_FILE is installed when the package is imported.
Problems with the DETERMINISTIC flag never use the table.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import replace

import numpy as np

from . import Request, _lib, decompose_batched

WGS_CANDIDATES = (128, 256, 512, 1024, 2048, 4096, 8192, 16384)
_GRAM, _MINOR = _lib.STEPS.index("gram"), _lib.STEPS.index("minor")


def table() -> list[dict]:
    """The library's current tile table."""
    return _lib.tune_get()


def install(entries: list[dict]) -> None:
    """Replace the library's tile table."""
    _lib.tune_set(entries)


def clear() -> None:
    _lib.tune_set([])


def save(path: str, entries: list[dict] | None = None) -> None:
    with open(path, "w") as f:
        json.dump({"entries": table() if entries is None else entries}, f, indent=1)


def load(path: str) -> list[dict]:
    """Read a saved table and install it; returns its entries."""
    with open(path) as f:
        entries = json.load(f)["entries"]
    install(entries)
    return entries


def _key(req: Request, torch) -> tuple[int, int, int]:
    l = req.l or req.r + 1
    ydt = _lib.F64 if req.Y.dtype == torch.float64 else _lib.F32
    return l, _lib.GRAM_MODES[req.gram], ydt


def _time_group(reqs, stream, reps, torch) -> float:
    """Median over `reps` calls of the Gram + minor-vector steps of one launch group."""
    times = []
    for k in range(reps + 1):                       # the first call warms up
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(_lib.STEPS))]
        for e in evs:
            e.record(stream)                        # create the handles the library records
        run = [replace(q, events=evs if j == 0 else None) for j, q in enumerate(reqs)]
        decompose_batched(run, stream=stream)
        stream.synchronize()
        if k:
            times.append(evs[2 * _GRAM].elapsed_time(evs[2 * _MINOR + 1]))
    return float(np.median(times))


def autotune(requests, *, wgs=WGS_CANDIDATES, reps: int = 3, stream=None,
             keep_existing: bool = True) -> dict:
    """Time the candidate tile shapes on `requests` and install the winners.

    The requests run with ACCUMULATE_ONLY into scratch N matrices, so only steps a0..a5
    execute; their inputs are not modified.  Returns the installed entries and, per
    launch group, the built-in time and the best time (milliseconds)."""
    import torch
    t_start = time.perf_counter()
    stream = stream or torch.cuda.current_stream()
    groups: dict[tuple, list] = {}
    for q in requests:
        if q.flags & (_lib.DETERMINISTIC | _lib.FINALIZE_ONLY) or q.num_submatrices <= 0:
            continue
        groups.setdefault(_key(q, torch), []).append(q)
    base = [e for e in table()] if keep_existing else []
    report = []
    for (l, prec, ydt), members in sorted(groups.items()):
        shapes = [(kern, nt) for kern in (_lib.GRAM_KERNEL_REGS, _lib.GRAM_KERNEL_DMA,
                                          _lib.GRAM_KERNEL_DMA2, _lib.GRAM_KERNEL_GATHER,
                                          _lib.GRAM_KERNEL_AUTO)
                  for nt in _lib.tune_threads(l, prec, ydt, kern)]
        if not shapes:
            continue                                 # per-trial streamer: nothing to tune
        batched = 1 if len(members) > 1 else 0
        others = [e for e in base if (e["l"], e["gram_prec"], e["y_dtype"], e["batched"])
                  != (l, prec, ydt, batched)]
        run = [replace(q, flags=(q.flags | _lib.ACCUMULATE_ONLY) & ~_lib.N_ACCUMULATE,
                       N=torch.zeros(q.Y.shape[1], q.Y.shape[1], dtype=torch.float64,
                                     device=q.Y.device), taps=False)
               for q in members]
        install(others)
        t_builtin = _time_group(run, stream, reps, torch)
        best, best_t = None, t_builtin
        for kern, nt in shapes:
            for w in wgs:
                cand = {"l": l, "gram_prec": prec, "y_dtype": ydt, "batched": batched,
                        "gram_threads": nt, "gram_wgs": int(w), "gram_kernel": kern}
                install(others + [cand])
                t = _time_group(run, stream, reps, torch)
                if t < best_t:
                    best, best_t = cand, t
        base = others + ([best] if best is not None else [])
        report.append({"l": l, "gram_prec": prec, "y_dtype": ydt, "batched": batched,
                       "problems": len(members), "builtin_ms": round(t_builtin, 4),
                       "best_ms": round(best_t, 4),
                       "choice": None if best is None else
                       {"gram_kernel": best["gram_kernel"], "gram_threads": best["gram_threads"],
                        "gram_wgs": best["gram_wgs"]}})
    install(base)
    return {"entries": base, "groups": report,
            "seconds": round(time.perf_counter() - t_start, 2)}


def load_from_env() -> None:
    path = os.environ.get("RSM_TUNE_FILE")
    if path:
        load(path)
