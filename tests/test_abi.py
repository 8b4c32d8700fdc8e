"""The C ABI: symbols, struct layouts, and host-side argument validation (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1411_0814_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsm.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(rsm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared_functions()
    assert declared == sorted(_lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name
    assert L.rsm_abi_version() == _lib.ABI_VERSION
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}$", out, re.M), name


_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "rsm.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("rsm_problem %zu\nrsm_input %zu\nrsm_info %zu\nrsm_output %zu\n",
         sizeof(rsm_problem), sizeof(rsm_input), sizeof(rsm_info), sizeof(rsm_output));
  F(rsm_problem, m) F(rsm_problem, r) F(rsm_problem, num_submatrices) F(rsm_problem, seed)
  F(rsm_problem, gram_prec) F(rsm_problem, flags) F(rsm_problem, y_dtype) F(rsm_problem, reserved)
  F(rsm_input, Y) F(rsm_input, ldy) F(rsm_input, W) F(rsm_input, ldw) F(rsm_input, subsets)
  F(rsm_info, warn) F(rsm_info, accepted) F(rsm_info, known) F(rsm_info, eig_iterations)
  F(rsm_info, lambda) F(rsm_info, residual) F(rsm_info, mu) F(rsm_info, e)
  F(rsm_output, V) F(rsm_output, info) F(rsm_output, trial_cols) F(rsm_output, trial_eigs)
  F(rsm_output, step_events)
  printf("rsm_tune_entry %zu\n", sizeof(rsm_tune_entry));
  F(rsm_tune_entry, l) F(rsm_tune_entry, gram_prec) F(rsm_tune_entry, y_dtype)
  F(rsm_tune_entry, batched) F(rsm_tune_entry, gram_threads) F(rsm_tune_entry, gram_wgs)
  F(rsm_tune_entry, gram_kernel)
  printf("KERNELS %d %d\n", RSM_GRAM_KERNEL_REGS, RSM_GRAM_KERNEL_DMA);
  printf("STEPS %d\n", RSM_NUM_STEPS);
  printf("MAX %d %d %d %d\n", RSM_MAX_R, RSM_MAX_L, RSM_MAX_N, RSM_ABI_VERSION);
  return 0;
}
"""


def test_struct_layouts_match_header():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(_PROBE)
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{os.path.dirname(HEADER)}",
                        src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.strip().splitlines():
        k, *v = line.split()
        got[k] = v
    assert int(got["rsm_problem"][0]) == C.sizeof(_lib.Problem)
    assert int(got["rsm_input"][0]) == C.sizeof(_lib.Input)
    assert int(got["rsm_info"][0]) == C.sizeof(_lib.Info)
    assert int(got["rsm_output"][0]) == C.sizeof(_lib.Output)
    assert int(got["rsm_tune_entry"][0]) == C.sizeof(_lib.TuneEntry)
    pyname = {"lambda": "lambda_"}
    structs = {"rsm_problem": _lib.Problem, "rsm_input": _lib.Input, "rsm_info": _lib.Info,
               "rsm_output": _lib.Output, "rsm_tune_entry": _lib.TuneEntry}
    for k, v in got.items():
        if "." in k:
            s, f = k.split(".")
            assert getattr(structs[s], pyname.get(f, f)).offset == int(v[0]), k
    assert [int(x) for x in got["MAX"]] == [_lib.MAX_R, _lib.MAX_L, _lib.MAX_N, _lib.ABI_VERSION]
    assert int(got["STEPS"][0]) == len(_lib.STEPS)
    assert [int(x) for x in got["KERNELS"]] == [_lib.GRAM_KERNEL_REGS, _lib.GRAM_KERNEL_DMA]


def _prob(**kw):
    p = _lib.Problem()
    p.m, p.n, p.r, p.num_submatrices, p.seed = 2000, 200, 5, 800, 1
    p.gram_prec = _lib.GRAM_F64
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ws(p):
    out = C.c_size_t(0)
    code = _lib.lib().rsm_workspace_bytes(C.byref(p), 1, C.byref(out))
    return code, out.value


def test_split_bf16_accepted_for_fp32():
    code, nbytes = _ws(_prob(gram_prec=_lib.GRAM_BF16X2, y_dtype=_lib.F32, r=15, l=16))
    assert code == _lib.OK and nbytes > 0


def test_serial_steps_flag_accepted_and_changes_no_workspace():
    # a call-level scheduling choice: the same plan and workspace as without it
    code, base = _ws(_prob())
    code2, serial = _ws(_prob(flags=_lib.SERIAL_STEPS))
    assert code == code2 == _lib.OK and serial == base
    assert _ws(_prob(flags=1 << 8))[0] == _lib.E_ARG


def test_workspace_bytes_valid_and_monotone():
    code, small = _ws(_prob())
    assert code == _lib.OK and small > 0
    code, big = _ws(_prob(num_submatrices=8000))
    assert code == _lib.OK and big > small
    code, rm = _ws(_prob(y_layout=_lib.ROW_MAJOR))
    assert code == _lib.OK and rm >= small + 2000 * 200 * 4
    # batched: the parts' scratch plus one shared descriptor area (a few KiB) per call
    arr = (_lib.Problem * 2)(_prob(), _prob(num_submatrices=8000))
    out = C.c_size_t(0)
    assert _lib.lib().rsm_workspace_bytes(arr, 2, C.byref(out)) == _lib.OK
    assert small + big - 4096 <= out.value <= small + big
    assert out.value % 256 == 0


@pytest.mark.parametrize("kw,code", [
    (dict(r=0), _lib.E_ARG),
    (dict(r=200), _lib.E_ARG),                 # r >= min(m, n)
    (dict(l=5), _lib.E_ARG),                   # l <= r
    (dict(l=201), _lib.E_ARG),                 # l > n
    (dict(nvec=2), _lib.E_ARG),                # nvec > l - r
    (dict(num_submatrices=-1), _lib.E_ARG),
    (dict(trial_begin=-5), _lib.E_ARG),
    (dict(m=0), _lib.E_ARG),
    (dict(gram_prec=7), _lib.E_ARG),
    (dict(y_dtype=3), _lib.E_ARG),
    (dict(flags=1 << 20), _lib.E_ARG),
    (dict(flags=_lib.ACCUMULATE_ONLY | _lib.FINALIZE_ONLY), _lib.E_ARG),
    (dict(reserved=1), _lib.E_ARG),
    (dict(r=17, n=300, m=5000), _lib.E_UNSUPPORTED),
    (dict(l=18, r=5), _lib.E_UNSUPPORTED),
    (dict(n=5000, m=6000), _lib.E_UNSUPPORTED),
    # split-BF16 runs on the tiled MFMA kernel only: FP32 Y, l <= 16, not the plain kernel
    (dict(gram_prec=_lib.GRAM_BF16X2, y_dtype=_lib.F64), _lib.E_UNSUPPORTED),
    (dict(gram_prec=_lib.GRAM_BF16X2, y_dtype=_lib.F32, r=16, l=17), _lib.E_UNSUPPORTED),
    (dict(gram_prec=_lib.GRAM_BF16X2, y_dtype=_lib.F32, flags=_lib.PLAIN_GRAM), _lib.E_UNSUPPORTED),
])
def test_invalid_problems_rejected_on_host(kw, code):
    assert _ws(_prob(**kw))[0] == code


RF = _lib.ROWS_FIRST


@pytest.mark.parametrize("kw,code", [
    (dict(flags=RF), _lib.OK),
    (dict(flags=RF, l=9, r=8, n=1024, m=131072), _lib.OK),
    (dict(flags=RF, nvec=1), _lib.E_ARG),                       # every trial gives |C| - r
    (dict(flags=RF, min_rows=5), _lib.E_ARG),                   # a trial needs > r columns
    (dict(flags=RF, l=5), _lib.E_ARG),                          # k <= r
    (dict(flags=RF, l=2001), _lib.E_ARG),                       # k > m
    (dict(flags=RF, l=18), _lib.E_UNSUPPORTED),                 # k > RSM_MAX_L
    (dict(flags=RF, gram_prec=_lib.GRAM_BF16X2, y_dtype=_lib.F32), _lib.E_UNSUPPORTED),
    (dict(flags=RF | _lib.PLAIN_GRAM), _lib.E_UNSUPPORTED),
])
def test_rows_first_validation(kw, code):
    assert _ws(_prob(**kw))[0] == code


def test_rows_first_workspace_holds_row_planes_and_row_major_copy():
    # the row bit-planes (m x ceil(n/64) words), k x r doubles per trial and one copy of Y:
    # the row-major copy when Y is column-major, the column-major copy (for U-hat) when Y
    # is row-major
    p = _prob()
    code, rf = _ws(_prob(flags=RF))
    _, rf_rm = _ws(_prob(flags=RF, y_layout=_lib.ROW_MAJOR))
    assert code == _lib.OK
    words = p.m * ((p.n + 63) // 64) * 8
    ycopy = p.m * p.n * 4                                        # FP32 Y
    bmat = p.num_submatrices * (p.r + 1) * p.r * 8
    nn = p.n * p.n * 8
    assert rf >= words + ycopy + bmat + 3 * nn
    assert abs(rf - rf_rm) <= 1024


def _decompose_raw(p, inp, out, ws_ptr, ws_bytes):
    return _lib.lib().rsm_decompose(C.byref(p), C.byref(inp), C.byref(out), C.c_void_p(ws_ptr),
                                    C.c_size_t(ws_bytes), None)


def test_decompose_validates_before_any_launch():
    # Fake (never dereferenced) device addresses: every case below must be rejected on the
    # host before anything touches the device.
    fake = 1 << 40
    p = _prob()
    _, need = _ws(p)
    inp = _lib.Input(Y=fake, ldy=2000, W=fake, ldw=2000, subsets=None)
    out = _lib.Output(V=fake, U=fake, N=None, info=fake)
    assert _decompose_raw(p, inp, out, fake, need - 1) == _lib.E_WORKSPACE
    assert _decompose_raw(p, inp, out, fake + 8, need) == _lib.E_WORKSPACE      # misaligned
    assert _decompose_raw(p, inp, out, None, need) == _lib.E_WORKSPACE
    bad = _lib.Input(Y=fake, ldy=1999, W=fake, ldw=2000)                       # ldy < m
    assert _decompose_raw(p, bad, out, fake, need) == _lib.E_ARG
    bad = _lib.Input(Y=None, ldy=2000, W=fake, ldw=2000)
    assert _decompose_raw(p, bad, out, fake, need) == _lib.E_ARG
    assert _decompose_raw(p, inp, _lib.Output(V=fake, U=fake, info=None), fake, need) == _lib.E_ARG
    assert _decompose_raw(p, inp, _lib.Output(V=None, U=fake, info=fake), fake, need) == _lib.E_ARG
    # accumulate-only / finalize-only need N
    p2 = _prob(flags=_lib.ACCUMULATE_ONLY)
    _, need2 = _ws(p2)
    assert _decompose_raw(p2, inp, _lib.Output(info=fake), fake, need2) == _lib.E_ARG
    p3 = _prob(flags=_lib.FINALIZE_ONLY)
    assert _decompose_raw(p3, inp, out, fake, need2) == _lib.E_ARG
    # row-major W needs ldw >= n
    p4 = _prob(w_layout=_lib.ROW_MAJOR)
    _, need4 = _ws(p4)
    assert _decompose_raw(p4, _lib.Input(Y=fake, ldy=2000, W=fake, ldw=199), out, fake, need4) == _lib.E_ARG
    assert _lib.lib().rsm_decompose_batched(0, None, None, None, None, 0, None) == _lib.E_ARG


def test_noalloc_rejects_on_host_before_any_device_call():
    # no GPU is needed: a problem whose workspace exceeds the built-in scratch, and a NULL
    # problem, are rejected before the call looks at the device
    fake = 1 << 40
    L = _lib.lib()
    inp = _lib.Input(Y=fake, ldy=131072, W=fake, ldw=131072, subsets=None)
    out = _lib.Output(V=fake, U=fake, N=None, info=fake)
    big = _prob(m=131072, n=1024, r=8, l=9, num_submatrices=8192, y_dtype=_lib.F32,
                gram_prec=_lib.GRAM_F32)
    code, need = _ws(big)
    assert code == _lib.OK and need > _lib.NOALLOC_MAX_BYTES
    assert L.rsm_decompose_noalloc(C.byref(big), C.byref(inp), C.byref(out), None) == _lib.E_SCRATCH
    assert L.rsm_decompose_noalloc(None, C.byref(inp), C.byref(out), None) == _lib.E_ARG
    bad = _prob(r=0)
    assert L.rsm_decompose_noalloc(C.byref(bad), C.byref(inp), C.byref(out), None) == _lib.E_ARG


def test_status_strings():
    for code in [_lib.OK, _lib.E_ARG, _lib.E_WORKSPACE, _lib.E_DEVICE, _lib.E_UNSUPPORTED,
                 _lib.E_SCRATCH, *_lib.WARNINGS]:
        s = _lib.status_string(code)
        assert s and s != "unknown status"
    assert _lib.status_string(12345) == "unknown status"


@pytest.fixture
def empty_tune_table():
    _lib.tune_set([])
    yield
    _lib.tune_set([])


def _entry(**kw):
    e = {"l": 9, "gram_prec": _lib.GRAM_F32, "y_dtype": _lib.F32, "batched": 0,
         "gram_threads": 512, "gram_wgs": 1024, "gram_kernel": 0}
    e.update(kw)
    return e


def test_tune_threads_lists_built_kernels():
    F32, F64 = _lib.F32, _lib.F64
    DMA = _lib.GRAM_KERNEL_DMA
    assert _lib.tune_threads(17, _lib.GRAM_F32, F32, DMA) == [256, 512]
    assert _lib.tune_threads(3, _lib.GRAM_F32, F32, DMA) == [256, 512]
    assert _lib.tune_threads(6, _lib.GRAM_F64, F64, DMA) == []
    assert _lib.tune_threads(9, _lib.GRAM_BF16X2, F32, DMA) == []
    DB = _lib.GRAM_KERNEL_DMA2
    assert _lib.tune_threads(12, _lib.GRAM_F32, F32, DB) == [512, 1024]
    assert _lib.tune_threads(13, _lib.GRAM_F32, F32, DB) == [512]
    assert _lib.tune_threads(4, _lib.GRAM_F64, F64, DB) == []
    assert _lib.tune_threads(9, _lib.GRAM_F32, F32) == [256, 512]
    assert _lib.tune_threads(10, _lib.GRAM_F32, F32) == [256, 512]
    assert _lib.tune_threads(12, _lib.GRAM_F32, F32) == [256]
    assert _lib.tune_threads(6, _lib.GRAM_F64, F64) == [256, 512]
    assert _lib.tune_threads(7, _lib.GRAM_F64, F64) == [256]
    assert _lib.tune_threads(6, _lib.GRAM_F64, F32) == []        # REGS: no FP64 sums of FP32
    # FP64 sums of FP32 data: double-buffered direct-to-LDS only, 512 trials up to l = 14
    assert _lib.tune_threads(14, _lib.GRAM_F64, F32, DB) == [256, 512]
    assert _lib.tune_threads(15, _lib.GRAM_F64, F32, DB) == [256]
    assert _lib.tune_threads(6, _lib.GRAM_F64, F32, DMA) == []
    for kern in (_lib.GRAM_KERNEL_GATHER, _lib.GRAM_KERNEL_AUTO):  # as the two-buffer kernel
        assert _lib.tune_threads(12, _lib.GRAM_F32, F32, kern) == [512, 1024]
        assert _lib.tune_threads(13, _lib.GRAM_F32, F32, kern) == [512]
        assert _lib.tune_threads(14, _lib.GRAM_F64, F32, kern) == [256, 512]
        assert _lib.tune_threads(6, _lib.GRAM_F64, F64, kern) == [256, 512]   # FP64 data
        assert _lib.tune_threads(7, _lib.GRAM_F64, F64, kern) == [256]
        assert _lib.tune_threads(9, _lib.GRAM_BF16X2, F32, kern) == []
    assert _lib.tune_threads(16, _lib.GRAM_BF16X2, F32) == [64]
    assert _lib.tune_threads(17, _lib.GRAM_BF16X2, F32) == []


def test_tune_table_roundtrip_and_validation(empty_tune_table):
    good = [_entry(), _entry(l=12, gram_threads=256, batched=1, gram_wgs=0,
                             gram_kernel=_lib.GRAM_KERNEL_REGS),
            _entry(l=16, gram_prec=_lib.GRAM_BF16X2, gram_threads=64, gram_wgs=64),
            _entry(l=17, gram_threads=512, gram_kernel=_lib.GRAM_KERNEL_DMA),
            _entry(l=17, gram_threads=512),          # FP32 stages straight into LDS by default
            _entry(l=9, gram_threads=1024),
            _entry(l=14, gram_prec=_lib.GRAM_F64, gram_threads=512)]
    _lib.tune_set(good)
    assert _lib.tune_get() == good
    bad = [_entry(l=1), _entry(l=_lib.MAX_L + 1), _entry(gram_threads=384),
           _entry(l=12, gram_threads=512, gram_kernel=_lib.GRAM_KERNEL_REGS),
           _entry(l=13, gram_threads=1024),          # built-in kernel at l = 13: 512 only
           _entry(gram_kernel=6), _entry(gram_kernel=-1),
           _entry(l=13, gram_threads=1024, gram_kernel=_lib.GRAM_KERNEL_DMA2),
           _entry(l=6, gram_prec=_lib.GRAM_F64, y_dtype=_lib.F64, gram_threads=0,
                  gram_kernel=_lib.GRAM_KERNEL_DMA),
           _entry(gram_wgs=-1), _entry(gram_wgs=(1 << 20) + 1),
           _entry(batched=2), _entry(y_dtype=7), _entry(gram_prec=3),
           # FP64 sums of FP32 Y: straight-to-LDS only, 256 trials above l = 14
           _entry(l=15, gram_prec=_lib.GRAM_F64, gram_threads=512),
           _entry(gram_prec=_lib.GRAM_F64, gram_threads=256, gram_kernel=_lib.GRAM_KERNEL_REGS)]
    for e in bad:
        with pytest.raises(_lib.RSMError) as ei:
            _lib.tune_set(good[:1] + [e])
        assert ei.value.code == _lib.E_ARG, e
        assert _lib.tune_get() == good                           # unchanged on error
    _lib.tune_set([])
    assert _lib.tune_get() == []


def test_tune_table_sets_the_gram_shape(empty_tune_table):
    """A table entry changes the Gram row splits (part of the workspace) only for the launch
    kind it names, and never for deterministic problems."""
    p = _prob(m=131072, n=1024, r=8, l=9, num_submatrices=8192, gram_prec=_lib.GRAM_F32,
              y_dtype=_lib.F32)
    code, base = _ws(p)
    assert code == _lib.OK
    # built-in: 8 groups of 1024 trials x 32 splits; 512 trials and 8192 workgroups -> 16
    # groups x 512 splits
    _lib.tune_set([_entry(gram_wgs=8192)])
    code, more = _ws(p)
    part_row = 8192 * 45 * 4 + 8192 * 4            # partial Grams + partial row counts
    assert more - base >= (512 - 32) * part_row - 4096
    # a one-workgroup-per-group target: a single split
    _lib.tune_set([_entry(gram_threads=512, gram_wgs=1)])
    code, fewer = _ws(p)
    assert base - fewer >= 31 * part_row - 4096
    # entries for batched launches or another l do not apply to this lone problem
    _lib.tune_set([_entry(batched=1, gram_wgs=8192), _entry(l=10, gram_wgs=8192)])
    assert _ws(p)[1] == base
    _lib.tune_set([_entry(gram_wgs=8192)])
    assert _ws(_prob(m=131072, n=1024, r=8, l=9, num_submatrices=8192,
                     gram_prec=_lib.GRAM_F32, y_dtype=_lib.F32,
                     flags=_lib.DETERMINISTIC))[1] == base
