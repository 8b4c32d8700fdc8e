"""ctypes view of librsm's C ABI (include/rsm.h).

Only argument marshalling lives here: the structs mirror the header field by field and
the functions are the exported entry points.  Loading fails loudly when the library has
not been built — there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsm.so")

# ---------------------------------------------------------------- constants (rsm.h)
ABI_VERSION = 1
MAX_R = 16
MAX_L = 17
MAX_N = 2048

OK = 0
E_ARG = -1
E_WORKSPACE = -2
E_DEVICE = -3
E_UNSUPPORTED = -4
E_SCRATCH = -5
NOALLOC_MAX_BYTES = 64 << 20   # RSM_NOALLOC_MAX_BYTES

W_NO_CONSTRAINTS = 1
W_RANK_DEFICIENT = 2
W_ROWS_UNDERDETERMINED = 4
W_NOT_CONVERGED = 8
W_BAD_SUBSET = 16
W_PIVOT = 32
WARNINGS = {W_NO_CONSTRAINTS: "no_constraints", W_RANK_DEFICIENT: "rank_deficient",
            W_ROWS_UNDERDETERMINED: "rows_underdetermined", W_NOT_CONVERGED: "not_converged",
            W_BAD_SUBSET: "bad_subset", W_PIVOT: "pivot"}

F32, F64 = 0, 1
COL_MAJOR, ROW_MAJOR = 0, 1
GRAM_F64, GRAM_F32, GRAM_BF16X2 = 0, 1, 2
GRAM_MODES = {"f64": GRAM_F64, "f32": GRAM_F32, "bf16x2": GRAM_BF16X2}

ACCUMULATE_ONLY = 1 << 0
FINALIZE_ONLY = 1 << 1
N_ACCUMULATE = 1 << 2
COMPUTE_ERROR = 1 << 3
PLAIN_GRAM = 1 << 4
DETERMINISTIC = 1 << 5
ROWS_FIRST = 1 << 6         # method M2: k-row subsets, qualifying columns
SERIAL_STEPS = 1 << 7       # a step's launch groups in order on the caller's stream

STEPS = ["pack", "subsets", "gram", "minor", "eig", "usolve", "error"]


class Problem(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("n", C.c_int64),
        ("r", C.c_int32), ("l", C.c_int32), ("nvec", C.c_int32), ("min_rows", C.c_int32),
        ("num_submatrices", C.c_int64), ("trial_begin", C.c_int64),
        ("seed", C.c_uint64),
        ("gram_prec", C.c_int32), ("flags", C.c_uint32),
        ("y_dtype", C.c_int32), ("y_layout", C.c_int32), ("w_layout", C.c_int32),
        ("reserved", C.c_int32),
    ]


class Input(C.Structure):
    _fields_ = [
        ("Y", C.c_void_p), ("ldy", C.c_int64),
        ("W", C.c_void_p), ("ldw", C.c_int64),
        ("subsets", C.c_void_p),
    ]


class Info(C.Structure):
    _fields_ = [
        ("warn", C.c_uint32), ("uncovered", C.c_int32),
        ("accepted", C.c_int64), ("rows_total", C.c_int64),
        ("rows_underdetermined", C.c_int64), ("known", C.c_int64),
        ("eig_iterations", C.c_int32), ("reserved", C.c_int32),
        ("lambda_", C.c_double * (MAX_R + 1)),
        ("residual", C.c_double), ("mu", C.c_double), ("e", C.c_double),
    ]


class Output(C.Structure):
    _fields_ = [
        ("V", C.c_void_p), ("U", C.c_void_p), ("N", C.c_void_p), ("info", C.c_void_p),
        ("trial_cols", C.c_void_p), ("trial_rows", C.c_void_p), ("trial_gram", C.c_void_p),
        ("trial_vecs", C.c_void_p), ("trial_eigs", C.c_void_p),
        ("step_events", C.c_void_p),
    ]


class TuneEntry(C.Structure):
    _fields_ = [
        ("l", C.c_int32), ("gram_prec", C.c_int32), ("y_dtype", C.c_int32),
        ("batched", C.c_int32), ("gram_threads", C.c_int32), ("gram_wgs", C.c_int32),
        ("gram_kernel", C.c_int32),
    ]


GRAM_KERNEL_REGS, GRAM_KERNEL_DMA, GRAM_KERNEL_DMA2 = 1, 2, 3
GRAM_KERNEL_GATHER, GRAM_KERNEL_AUTO = 4, 5


EXPORTS = ["rsm_abi_version", "rsm_status_string", "rsm_workspace_bytes", "rsm_decompose",
           "rsm_decompose_batched", "rsm_tune_set", "rsm_tune_get", "rsm_tune_threads",
           "rsm_lemma1_c", "rsm_trials_bound", "rsm_plan_trials", "rsm_decompose_noalloc"]

_LIB = None


class LibraryMissing(RuntimeError):
    pass


def lib() -> C.CDLL:
    """The loaded library (raises LibraryMissing if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} not found: build it with `python -m paper_1411_0814_amd.build` "
                "(or __graft_entry__.build()); there is no CPU fallback")
        # torch first: the library must bind to the HIP runtime torch already carries
        # (the streams and buffers it is given are torch's); loaded first, it would pull a
        # second runtime into the process, where torch's stream handles are not valid
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        L.rsm_abi_version.restype = C.c_int32
        L.rsm_abi_version.argtypes = []
        L.rsm_status_string.restype = C.c_char_p
        L.rsm_status_string.argtypes = [C.c_int32]
        L.rsm_workspace_bytes.restype = C.c_int32
        L.rsm_workspace_bytes.argtypes = [C.POINTER(Problem), C.c_int32, C.POINTER(C.c_size_t)]
        L.rsm_decompose.restype = C.c_int32
        L.rsm_decompose.argtypes = [C.POINTER(Problem), C.POINTER(Input), C.POINTER(Output),
                                    C.c_void_p, C.c_size_t, C.c_void_p]
        L.rsm_decompose_noalloc.restype = C.c_int32
        L.rsm_decompose_noalloc.argtypes = [C.POINTER(Problem), C.POINTER(Input), C.POINTER(Output),
                                            C.c_void_p]
        L.rsm_decompose_batched.restype = C.c_int32
        L.rsm_decompose_batched.argtypes = [C.c_int32, C.POINTER(Problem), C.POINTER(Input),
                                            C.POINTER(Output), C.c_void_p, C.c_size_t,
                                            C.c_void_p]
        L.rsm_tune_set.restype = C.c_int32
        L.rsm_tune_set.argtypes = [C.POINTER(TuneEntry), C.c_int32]
        L.rsm_tune_get.restype = C.c_int32
        L.rsm_tune_get.argtypes = [C.POINTER(TuneEntry), C.c_int32, C.POINTER(C.c_int32)]
        L.rsm_tune_threads.restype = C.c_int32
        L.rsm_tune_threads.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
        L.rsm_lemma1_c.restype = C.c_int32
        L.rsm_lemma1_c.argtypes = [C.c_int64, C.c_double, C.c_int64, C.POINTER(C.c_double)]
        L.rsm_trials_bound.restype = C.c_int32
        L.rsm_trials_bound.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_int32, C.c_int32,
                                       C.c_double, C.c_int32, C.POINTER(C.c_double)]
        L.rsm_plan_trials.restype = C.c_int32
        L.rsm_plan_trials.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_int32, C.c_int32,
                                      C.c_double, C.c_int32, C.POINTER(C.c_int64)]
        if L.rsm_abi_version() != ABI_VERSION:
            raise LibraryMissing("librsm ABI version mismatch; rebuild the library")
        _LIB = L
    return _LIB


def status_string(code: int) -> str:
    return lib().rsm_status_string(int(code)).decode()


class RSMError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code


def check(code: int, where: str) -> None:
    if code != OK:
        raise RSMError(code, where)


def workspace_bytes(problems) -> int:
    arr = (Problem * len(problems))(*problems)
    out = C.c_size_t(0)
    check(lib().rsm_workspace_bytes(arr, len(problems), C.byref(out)), "rsm_workspace_bytes")
    return int(out.value)


TUNE_FIELDS = [f for f, _ in TuneEntry._fields_]


def tune_set(entries) -> None:
    """Replace the library's tile table with `entries` (dicts with TUNE_FIELDS keys)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for k, e in enumerate(entries):
        for f in TUNE_FIELDS:
            setattr(arr[k], f, int(e.get(f, 0)))
    check(lib().rsm_tune_set(arr, len(entries)), "rsm_tune_set")


def tune_get() -> list[dict]:
    count = C.c_int32(0)
    check(lib().rsm_tune_get(None, 0, C.byref(count)), "rsm_tune_get")
    arr = (TuneEntry * max(1, count.value))()
    check(lib().rsm_tune_get(arr, count.value, C.byref(count)), "rsm_tune_get")
    return [{f: int(getattr(arr[k], f)) for f in TUNE_FIELDS} for k in range(count.value)]


def tune_threads(l: int, gram_prec: int, y_dtype: int, kernel: int = GRAM_KERNEL_REGS) -> list[int]:
    buf = (C.c_int32 * 8)()
    count = C.c_int32(0)
    check(lib().rsm_tune_threads(l, gram_prec, y_dtype, kernel, buf, 8, C.byref(count)),
          "rsm_tune_threads")
    return [int(buf[k]) for k in range(min(count.value, 8))]
