"""RSM (Random SubMatrix method, arXiv:1411.0814) on MI355X: Python binding of librsm.

Low-rank decomposition Y ~ U V^T of an m x n matrix with missing entries (eq.(problem)),
by the paper's three steps with method M1 and the L2 norm.  Every step runs in the HIP
kernels of librsm; this module only marshals arguments.  PyTorch provides the device
buffers and the stream.

    from paper_1411_0814_amd import decompose
    res = decompose(Y, W, r=8, num_submatrices=8192, seed=1)      # Y, W on cuda
    res.U, res.V, res.info()                                         # info() syncs

`Y` is a CUDA tensor (float32/float64), `W` a CUDA bool/uint8 tensor of the same shape
(True/nonzero = known).  Either may be row-major (a contiguous (m, n) tensor) or
column-major (the transpose of a contiguous (n, m) tensor); column-major Y is read in
place.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

from . import _lib
from ._lib import RSMError, LibraryMissing  # noqa: F401

__all__ = ["decompose", "decompose_noalloc", "decompose_batched", "workspace_bytes", "Request", "Result",
           "RSMError", "LibraryMissing"]


def _torch():
    import torch
    return torch


def _layout(t, name):
    """(layout, leading dimension) of a 2-D tensor, or raise."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    m, n = t.shape
    s0, s1 = t.stride()
    if s1 == 1 and (s0 >= n or m == 1):
        return _lib.ROW_MAJOR, max(s0, n)
    if s0 == 1 and (s1 >= m or n == 1):
        return _lib.COL_MAJOR, max(s1, m)
    raise ValueError(f"{name} must be row-major or column-major (got strides {t.stride()})")


@dataclass
class Request:
    """One decomposition: inputs on the device plus the method's parameters."""
    Y: object
    W: object
    r: int
    num_submatrices: int
    seed: int
    l: int = 0
    nvec: int = 0
    min_rows: int = 0
    gram: str = "f32"
    trial_begin: int = 0
    subsets: object = None          # optional (I, l) int32 CUDA tensor
    N: object = None                # optional (n, n) float64 CUDA tensor (in/out)
    flags: int = 0
    taps: bool = False              # also return the per-trial taps
    events: object = None           # optional list of 2 * len(STEPS) torch.cuda.Event


@dataclass
class Result:
    U: object
    V: object
    N: object
    info_raw: object                 # device bytes of rsm_info
    taps: dict = field(default_factory=dict)
    stream: object = None
    _keep: list = field(default_factory=list)   # host/device buffers that must outlive the call

    def full_N(self):
        """N as a full symmetric (n, n) float64 tensor (synchronises)."""
        torch = _torch()
        if self.stream is not None:
            self.stream.synchronize()
        A = self.N.T
        return torch.tril(A) + torch.tril(A, -1).T

    def info(self) -> dict:
        """Synchronise with the stream and decode rsm_info."""
        torch = _torch()
        if self.stream is not None:
            self.stream.synchronize()
        raw = bytes(self.info_raw.cpu().numpy().tobytes())
        inf = _lib.Info.from_buffer_copy(raw)
        warn = int(inf.warn)
        return {
            "warn": warn,
            "warnings": [name for bit, name in _lib.WARNINGS.items() if warn & bit],
            "uncovered": int(inf.uncovered),
            "accepted": int(inf.accepted),
            "rows_total": int(inf.rows_total),
            "rows_underdetermined": int(inf.rows_underdetermined),
            "known": int(inf.known),
            "eig_iterations": int(inf.eig_iterations),
            "lambda": [float(x) for x in inf.lambda_],
            "residual": float(inf.residual),
            "mu": float(inf.mu),
            "e": float(inf.e),
        }


def _problem(req: Request) -> _lib.Problem:
    torch = _torch()
    m, n = req.Y.shape
    if tuple(req.W.shape) != (m, n):
        raise ValueError("W must have the shape of Y")
    ylay, _ = _layout(req.Y, "Y")
    wlay, _ = _layout(req.W, "W")
    if req.Y.dtype == torch.float32:
        ydt = _lib.F32
    elif req.Y.dtype == torch.float64:
        ydt = _lib.F64
    else:
        raise ValueError("Y must be float32 or float64")
    if req.gram not in _lib.GRAM_MODES:
        raise ValueError(f"gram must be one of {sorted(_lib.GRAM_MODES)}")
    p = _lib.Problem()
    p.m, p.n = m, n
    p.r, p.l, p.nvec, p.min_rows = int(req.r), int(req.l or 0), int(req.nvec or 0), int(req.min_rows or 0)
    p.num_submatrices = int(req.num_submatrices)
    p.trial_begin = int(req.trial_begin)
    p.seed = int(req.seed) & (2**64 - 1)
    p.gram_prec = _lib.GRAM_MODES[req.gram]
    p.flags = int(req.flags)
    p.y_dtype, p.y_layout, p.w_layout = ydt, ylay, wlay
    p.reserved = 0
    return p


def workspace_bytes(requests: Sequence[Request]) -> int:
    return _lib.workspace_bytes([_problem(r) for r in requests])


def _check_device_tensor(t, name, dtype=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")


def _prepare(req: Request, p: _lib.Problem, device):
    """Allocate outputs; return (Input, Output, Result)."""
    torch = _torch()
    m, n, r = int(p.m), int(p.n), int(p.r)
    l = int(p.l) or r + 1
    nvec = int(p.nvec) or (l - r)
    I = int(p.num_submatrices)
    _check_device_tensor(req.Y, "Y")
    _check_device_tensor(req.W, "W")
    W = req.W
    if W.dtype == torch.bool:
        W = W.view(torch.uint8)
    elif W.dtype != torch.uint8:
        raise ValueError("W must be bool or uint8")
    _, ldy = _layout(req.Y, "Y")
    _, ldw = _layout(W, "W")
    inp = _lib.Input()
    inp.Y, inp.ldy = req.Y.data_ptr(), ldy
    inp.W, inp.ldw = W.data_ptr(), ldw
    if req.subsets is not None:
        _check_device_tensor(req.subsets, "subsets", torch.int32)
        if tuple(req.subsets.shape) != (I, l) or not req.subsets.is_contiguous():
            raise ValueError("subsets must be a contiguous (I, l) int32 tensor")
        inp.subsets = req.subsets.data_ptr()
    acc_only = bool(p.flags & _lib.ACCUMULATE_ONLY)
    V = None if acc_only else torch.empty((r, n), dtype=torch.float64, device=device).T
    U = None if acc_only else torch.empty((r, m), dtype=torch.float64, device=device).T
    N = req.N
    if N is None and (p.flags & (_lib.ACCUMULATE_ONLY | _lib.FINALIZE_ONLY | _lib.N_ACCUMULATE)):
        N = torch.zeros((n, n), dtype=torch.float64, device=device)
    if N is not None:
        _check_device_tensor(N, "N", torch.float64)
        if tuple(N.shape) != (n, n) or not N.is_contiguous():
            raise ValueError("N must be a contiguous (n, n) float64 tensor")
    info = torch.empty(C.sizeof(_lib.Info), dtype=torch.uint8, device=device)
    out = _lib.Output()
    out.V = V.data_ptr() if V is not None else None
    out.U = U.data_ptr() if U is not None else None
    out.N = N.data_ptr() if N is not None else None
    out.info = info.data_ptr()
    taps = {}
    if req.taps:
        taps["cols"] = torch.empty((I, l), dtype=torch.int32, device=device)
        taps["rows"] = torch.empty((I,), dtype=torch.int32, device=device)
        taps["gram"] = torch.empty((I, l, l), dtype=torch.float64, device=device)
        taps["eigs"] = torch.empty((I, l), dtype=torch.float64, device=device)
        out.trial_cols = taps["cols"].data_ptr()
        out.trial_rows = taps["rows"].data_ptr()
        out.trial_gram = taps["gram"].data_ptr()
        out.trial_eigs = taps["eigs"].data_ptr()
        # rows first (method M2): the taps hold S_t, |C_t|, H_t and its eigenvalues; the
        # trial's vectors are not kept
        if not (p.flags & _lib.ROWS_FIRST):
            taps["vecs"] = torch.empty((I, nvec, l), dtype=torch.float64, device=device)
            out.trial_vecs = taps["vecs"].data_ptr()
    keep = []
    if req.events is not None:
        if len(req.events) != 2 * len(_lib.STEPS):
            raise ValueError(f"events must hold {2 * len(_lib.STEPS)} torch.cuda.Event")
        handles = (C.c_void_p * len(req.events))()
        for k, ev in enumerate(req.events):
            handles[k] = ev.cuda_event
        out.step_events = C.cast(handles, C.c_void_p)
        keep.append(handles)
    # N is column-major n x n (ld n) with its lower triangle written, i.e. the upper
    # triangle of the (n, n) torch tensor; Result.full_N() returns the symmetric matrix.
    res = Result(U=U, V=V, N=N, info_raw=info, taps=taps)
    res._keep = keep
    return inp, out, res


def _workspace(nbytes, device):
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def decompose_batched(requests: Sequence[Request], stream=None, workspace=None) -> list[Result]:
    """Several independent decompositions in one library call."""
    torch = _torch()
    if not requests:
        return []
    L = _lib.lib()
    device = requests[0].Y.device
    stream = stream or torch.cuda.current_stream(device)
    probs = [_problem(r) for r in requests]
    ws_need = _lib.workspace_bytes(probs)
    # allocated on the stream the kernels run on, so the caching allocator does not hand
    # these blocks to other streams while the kernels may still use them
    with torch.cuda.stream(stream):
        prepared = [_prepare(r, p, device) for r, p in zip(requests, probs)]
        if workspace is None:
            ws_buf, ws_ptr = _workspace(ws_need, device)
    if workspace is not None:
        ws_buf, ws_ptr = workspace, workspace.data_ptr()
        if workspace.numel() * workspace.element_size() < ws_need or ws_ptr % 256:
            raise ValueError("workspace too small or misaligned")
    k = len(requests)
    parr = (_lib.Problem * k)(*probs)
    iarr = (_lib.Input * k)(*[x[0] for x in prepared])
    oarr = (_lib.Output * k)(*[x[1] for x in prepared])
    code = L.rsm_decompose_batched(k, parr, iarr, oarr, C.c_void_p(ws_ptr), C.c_size_t(ws_need),
                                   C.c_void_p(stream.cuda_stream))
    _lib.check(code, "rsm_decompose_batched")
    results = []
    for _, _, res in prepared:
        res.stream = stream
        res._keep.append(ws_buf)  # keep the scratch alive until the stream is done
        results.append(res)
    return results


def decompose(Y, W, r: int, num_submatrices: int, seed: int, *, l: int = 0, nvec: int = 0,
              min_rows: int = 0, gram: str = "f32", trial_begin: int = 0, subsets=None,
              N=None, flags: int = 0, taps: bool = False, stream=None,
              workspace=None, events=None) -> Result:
    """One RSM decomposition (steps a1..a7) enqueued on `stream` (default: current)."""
    torch = _torch()
    L = _lib.lib()
    req = Request(Y=Y, W=W, r=r, num_submatrices=num_submatrices, seed=seed, l=l, nvec=nvec,
                  min_rows=min_rows, gram=gram, trial_begin=trial_begin, subsets=subsets, N=N,
                  flags=flags, taps=taps, events=events)
    device = Y.device
    stream = stream or torch.cuda.current_stream(device)
    p = _problem(req)
    ws_need = _lib.workspace_bytes([p])
    # allocated on the launch stream (see decompose_batched)
    with torch.cuda.stream(stream):
        inp, out, res = _prepare(req, p, device)
        if workspace is None:
            ws_buf, ws_ptr = _workspace(ws_need, device)
    if workspace is not None:
        ws_buf, ws_ptr = workspace, workspace.data_ptr()
        if workspace.numel() * workspace.element_size() < ws_need or ws_ptr % 256:
            raise ValueError("workspace too small or misaligned")
    code = L.rsm_decompose(C.byref(p), C.byref(inp), C.byref(out), C.c_void_p(ws_ptr),
                           C.c_size_t(ws_need), C.c_void_p(stream.cuda_stream))
    _lib.check(code, "rsm_decompose")
    res.stream = stream
    res._keep.append(ws_buf)  # keep the scratch alive until the stream is done
    return res


def decompose_noalloc(Y, W, r: int, num_submatrices: int, seed: int, *, l: int = 0,
                      nvec: int = 0, min_rows: int = 0, gram: str = "f32", trial_begin: int = 0,
                      subsets=None, N=None, flags: int = 0, stream=None) -> Result:
    """As decompose, through rsm_decompose_noalloc: the library takes its workspace from its
    own per-device scratch array (no workspace tensor).  Outputs are still allocated here."""
    torch = _torch()
    L = _lib.lib()
    req = Request(Y=Y, W=W, r=r, num_submatrices=num_submatrices, seed=seed, l=l, nvec=nvec,
                  min_rows=min_rows, gram=gram, trial_begin=trial_begin, subsets=subsets, N=N,
                  flags=flags)
    device = Y.device
    stream = stream or torch.cuda.current_stream(device)
    p = _problem(req)
    with torch.cuda.stream(stream):
        inp, out, res = _prepare(req, p, device)
    code = L.rsm_decompose_noalloc(C.byref(p), C.byref(inp), C.byref(out),
                                   C.c_void_p(stream.cuda_stream))
    _lib.check(code, "rsm_decompose_noalloc")
    res.stream = stream
    return res


def _load_tune_file():
    import os
    if os.environ.get("RSM_TUNE_FILE"):
        from . import tune
        tune.load_from_env()


_load_tune_file()
