"""Host-only checks of the C ABI: the library loads, exports what the header
declares, the ctypes mirror matches the C layout, and plan validation rejects
bad set-ups with the documented status (no kernel runs here)."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2201_00451_amd import binding as B
from paper_2201_00451_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fstat.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libfstat.so is not built: run python paper_2201_00451_amd/build.py")
    return B.load_library()


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"FSTAT_API\s+[\w\s\*]+?\b(fstat_\w+)\s*\(", txt)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (fstat_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert hasattr(lib, f)
    assert B.version().startswith("fstat-gfx950")


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "fstat.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("fstat_detector %zu\nfstat_plan_desc %zu\nfstat_inputs %zu\n",
         sizeof(fstat_detector), sizeof(fstat_plan_desc), sizeof(fstat_inputs));
  F(fstat_plan_desc, det); F(fstat_plan_desc, dt); F(fstat_plan_desc, n_fft);
  F(fstat_plan_desc, flags); F(fstat_inputs, valid); F(fstat_inputs, n_eph);
  F(fstat_inputs, moments); F(fstat_detector, n); F(fstat_detector, noise_var);
  printf("fstat_sft_desc %zu\n", sizeof(fstat_sft_desc));
  F(fstat_sft_desc, n_sft); F(fstat_sft_desc, n_bins); F(fstat_sft_desc, reserved);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.strip().splitlines())
    want = {
        "fstat_detector": ctypes.sizeof(B.FstatDetector),
        "fstat_plan_desc": ctypes.sizeof(B.FstatPlanDesc),
        "fstat_inputs": ctypes.sizeof(B.FstatInputs),
        "fstat_plan_desc.det": B.FstatPlanDesc.det.offset,
        "fstat_plan_desc.dt": B.FstatPlanDesc.dt.offset,
        "fstat_plan_desc.n_fft": B.FstatPlanDesc.n_fft.offset,
        "fstat_plan_desc.flags": B.FstatPlanDesc.flags.offset,
        "fstat_inputs.valid": B.FstatInputs.valid.offset,
        "fstat_inputs.n_eph": B.FstatInputs.n_eph.offset,
        "fstat_inputs.moments": B.FstatInputs.moments.offset,
        "fstat_detector.n": B.FstatDetector.n.offset,
        "fstat_detector.noise_var": B.FstatDetector.noise_var.offset,
        "fstat_sft_desc": ctypes.sizeof(B.FstatSftDesc),
        "fstat_sft_desc.n_sft": B.FstatSftDesc.n_sft.offset,
        "fstat_sft_desc.n_bins": B.FstatSftDesc.n_bins.offset,
        "fstat_sft_desc.reserved": B.FstatSftDesc.reserved.offset,
    }
    assert {k: int(v) for k, v in got.items()} == want


def good_desc():
    ds = synth.small_case(seed=3, n=3000, n_fft=1 << 13, ndet=2)
    return ds, B.make_plan_desc(ds)


def status_of(desc):
    lib = B.load_library()
    h = ctypes.c_void_p()
    st = lib.fstat_plan_create(ctypes.byref(desc), ctypes.byref(h))
    if st == 0:
        lib.fstat_plan_destroy(h)
    return st, B.last_error()


def test_plan_accepts_valid_setup(lib):
    ds, d = good_desc()
    p = B.Plan(d)
    # every documented tuning choice is accepted (n_fft = 2^13: columns 2^6 x rows 2^7 by default)
    for log_len, cl, rl in ((7, 64, 32), (7, 32, 16), (6, 64, 32), (6, 32, 16)):
        for radix in (0, 16, 32):
            d2 = B.make_plan_desc(ds, dict(tune_col_log_len=log_len, tune_col_lines=cl,
                                           tune_row_lines=rl, tune_fft_radix=radix))
            B.Plan(d2)
    k_pad, lc, lr = p.info()
    assert (lc, lr) == (6, 7) and k_pad % (1 << lr) == 0 and k_pad % 512 == 0
    assert k_pad >= ds.detectors[0].n and k_pad <= ds.n_fft
    # header + one slot of two n_fft complex64 arrays
    assert p.workspace_size(1) >= 2 * 8 * ds.n_fft
    assert p.workspace_size(3) - p.workspace_size(2) == p.workspace_size(2) - p.workspace_size(1)


@pytest.mark.parametrize("mutate,needle", [
    (lambda d: setattr(d, "ndet", 0), "ndet"),
    (lambda d: setattr(d, "ndet", 5), "ndet"),
    (lambda d: setattr(d, "n_fft", 3 << 12), "power of two"),
    (lambda d: setattr(d, "n_fft", 1 << 11), "power of two"),
    (lambda d: setattr(d, "n_fft", 1 << 25), "power of two"),
    (lambda d: setattr(d, "n_bins", 0), "band"),
    (lambda d: setattr(d, "bin_lo", (1 << 13) - 5), "band"),
    (lambda d: setattr(d, "sinc_halfwidth", 1), "sinc_halfwidth"),
    (lambda d: setattr(d, "sinc_halfwidth", 7), "sinc_halfwidth"),
    (lambda d: setattr(d, "sinc_halfwidth", 33), "sinc_halfwidth"),
    (lambda d: setattr(d, "dt", 0.0), "dt"),
    (lambda d: setattr(d, "dt", float("nan")), "dt"),
    (lambda d: setattr(d, "sid_rate", -1.0), "sid_rate"),
    (lambda d: setattr(d, "flags", 2), "flags"),
    (lambda d: setattr(d.det[1], "noise_var", 0.0), "noise_var"),
    (lambda d: setattr(d.det[0], "n", 0), "n must be"),
    (lambda d: setattr(d.det[0], "az_y", d.det[0].az_x + 1.0), "orthogonal"),
    (lambda d: setattr(d, "tau0", 0.0), "grid origin"),
    (lambda d: setattr(d, "max_delay", float("inf")), "max_delay"),
    (lambda d: setattr(d, "tune_col_log_len", 5), "tune_col_log_len"),
    (lambda d: setattr(d, "tune_col_log_len", 13), "tune_col_log_len"),
    (lambda d: setattr(d, "tune_col_lines", 3), "tune_col_lines"),
    (lambda d: setattr(d, "tune_row_lines", 7), "tune_row_lines"),

    (lambda d: setattr(d, "tune_fft_radix", 8), "tune_fft_radix"),
    (lambda d: (setattr(d, "n_fft", 1 << 12), setattr(d, "n_bins", 1 << 12),
               setattr(d.det[0], "n", 4000)), "too short"),
])
def test_plan_rejects_invalid_setup(lib, mutate, needle):
    _, d = good_desc()
    mutate(d)
    st, msg = status_of(d)
    assert st == B.FSTAT_EINVAL
    assert needle in msg


def test_null_arguments_rejected_before_any_launch(lib):
    ds, d = good_desc()
    p = B.Plan(d)
    vp = ctypes.c_void_p
    inp = B.FstatInputs()
    # null inputs / templates / outputs / workspace: EINVAL from host validation
    assert lib.fstat_compute_2f(p.handle, None, vp(0), 1, vp(0), vp(0), vp(0), 0, vp(0)) == B.FSTAT_EINVAL
    assert "templates" in B.last_error()
    assert lib.fstat_compute_2f(p.handle, None, vp(4096), 1, vp(4096), vp(0), vp(0), 0,
                                vp(0)) == B.FSTAT_EINVAL
    assert "inputs" in B.last_error()
    assert lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(0), 1, vp(0), vp(0), vp(0), 0,
                                vp(0)) == B.FSTAT_EINVAL
    assert lib.fstat_compute_2f(None, ctypes.byref(inp), vp(0), 1, vp(0), vp(0), vp(0), 0,
                                vp(0)) == B.FSTAT_EINVAL
    # fake (never dereferenced) device pointers pass pointer checks; the
    # ephemeris does not cover the data span -> EINVAL
    for i in range(2):
        inp.x[i] = inp.ephem[i] = 4096
    inp.moments = 4096
    inp.n_eph, inp.eph_t0, inp.eph_dt = 10, 0.0, 60.0
    st = lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(0), vp(4096),
                              1 << 30, vp(0))
    assert st == B.FSTAT_EINVAL and "ephemeris" in B.last_error()
    # covering ephemeris, workspace too small -> EWORKSPACE; misaligned -> EINVAL
    inp.eph_t0, inp.n_eph = ds.eph_t0, ds.eph_tables[0].shape[0]
    st = lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(0), vp(4096),
                              1024, vp(0))
    assert st == B.FSTAT_EWORKSPACE
    st = lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(0), vp(4100),
                              1 << 30, vp(0))
    assert st == B.FSTAT_EINVAL and "aligned" in B.last_error()
    assert lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(4096), -1, vp(4096), vp(0),
                                vp(4096), 1 << 30, vp(0)) == B.FSTAT_EINVAL
    # zero templates is a no-op that succeeds without touching the device
    assert lib.fstat_compute_2f(p.handle, ctypes.byref(inp), vp(0), 0, vp(0), vp(0), vp(4096),
                                1 << 30, vp(0)) == B.FSTAT_OK


def test_gradient_entry_checks_arguments_before_any_launch(lib):
    ds, d = good_desc()
    p = B.Plan(d)
    vp = ctypes.c_void_p
    # adjoint slot: the forward slot plus two more n_fft arrays and the tile partials
    g1, g2 = p.grad_workspace_size(1), p.grad_workspace_size(2)
    assert g2 - g1 >= (p.workspace_size(2) - p.workspace_size(1)) + 2 * 8 * ds.n_fft
    assert g2 - g1 == p.grad_workspace_size(3) - g2 and (g2 - g1) % 256 == 0
    sz = ctypes.c_size_t()
    assert lib.fstat_grad_workspace_size(p.handle, 0, ctypes.byref(sz)) == B.FSTAT_EINVAL
    assert lib.fstat_grad_workspace_size(None, 1, ctypes.byref(sz)) == B.FSTAT_EINVAL
    inp = B.FstatInputs()
    for i in range(2):
        inp.x[i] = inp.ephem[i] = 4096
    inp.moments = 4096
    inp.eph_t0, inp.eph_dt, inp.n_eph = ds.eph_t0, ds.eph_dt, ds.eph_tables[0].shape[0]
    grad = lib.fstat_compute_2f_grad
    # null weights / gradient output / templates
    assert grad(p.handle, ctypes.byref(inp), vp(4096), 1, vp(0), vp(4096), vp(0), vp(4096),
                1 << 30, vp(0)) == B.FSTAT_EINVAL
    assert "grad" in B.last_error()
    assert grad(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(0), vp(0), vp(4096),
                1 << 30, vp(0)) == B.FSTAT_EINVAL
    assert grad(p.handle, ctypes.byref(inp), vp(0), 1, vp(4096), vp(4096), vp(0), vp(4096),
                1 << 30, vp(0)) == B.FSTAT_EINVAL
    # the forward workspace is too small for the adjoint
    assert grad(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(4096), vp(0), vp(4096),
                p.workspace_size(1), vp(0)) == B.FSTAT_EWORKSPACE
    assert grad(p.handle, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(4096), vp(0), vp(4100),
                g1, vp(0)) == B.FSTAT_EINVAL
    assert grad(p.handle, None, vp(4096), 1, vp(4096), vp(4096), vp(0), vp(4096), g1,
                vp(0)) == B.FSTAT_EINVAL
    assert grad(p.handle, ctypes.byref(inp), vp(4096), -1, vp(4096), vp(4096), vp(0), vp(4096),
                g1, vp(0)) == B.FSTAT_EINVAL
    assert grad(p.handle, ctypes.byref(inp), vp(0), 0, vp(0), vp(0), vp(0), vp(4096), g1,
                vp(0)) == B.FSTAT_OK


def test_search_plan_groups_and_chunks(lib):
    """Grouping of a bank on the host: runs of equal sky/orbit form one group;
    an isolated source ignores porb/tp; chunks hold `slots` templates."""
    ds, d = good_desc()
    p = B.Plan(d)
    rows = []
    for sky in range(3):
        for f1 in range(5):
            rows.append([1.0 + sky, -0.5, 0.0, 1e-10 * f1, 0.0, 0.0, 1.0 + f1, 7.0 * f1])
    rows.append([9.0, 0.1, 0, 0, 0, 0.3, 5000.0, 1.0])
    rows.append([9.0, 0.1, 0, 1e-10, 0, 0.3, 5000.0, 1.0])
    rows.append([9.0, 0.1, 0, 0, 0, 0.3, 5000.0, 2.0])     # other periastron time: new group
    tm = np.array(rows, dtype=np.float64)
    vp = ctypes.c_void_p
    for slots, nchunks in ((4, 5), (8, 3), (32, 1)):
        h = vp()
        assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), len(tm), slots, 0,
                                       ctypes.byref(h)) == 0
        ws, ng, nc = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_int64()
        assert lib.fstat_search_info(h, ctypes.byref(ws), ctypes.byref(ng), ctypes.byref(nc)) == 0
        assert (ng.value, nc.value) == (5, nchunks)
        assert ws.value >= slots * 2 * 8 * ds.n_fft
        lib.fstat_search_destroy(h)
    h = vp()
    assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), len(tm), 33, 0,
                                   ctypes.byref(h)) == B.FSTAT_EINVAL
    assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), len(tm), 4, 4,
                                   ctypes.byref(h)) == B.FSTAT_EINVAL
    # graph and accumulate flags together are accepted
    assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), len(tm), 4,
                                   B.SEARCH_GRAPH | B.SEARCH_ACCUMULATE, ctypes.byref(h)) == 0
    # candidate retention: argument checks come before any launch
    ws = ctypes.c_size_t()
    assert lib.fstat_search_info(h, ctypes.byref(ws), None, None) == 0
    inp = B.FstatInputs()
    run = lib.fstat_search_run_candidates
    assert run(h, ctypes.byref(inp), vp(4096), 70.0, vp(4096), 16, vp(0), vp(0), vp(4096),
               ws.value, vp(0)) == B.FSTAT_EINVAL and "count" in B.last_error()
    assert run(h, ctypes.byref(inp), vp(4096), 70.0, vp(0), 16, vp(4096), vp(0), vp(4096),
               ws.value, vp(0)) == B.FSTAT_EINVAL
    assert run(h, ctypes.byref(inp), vp(4096), 70.0, vp(4096), -1, vp(4096), vp(0), vp(4096),
               ws.value, vp(0)) == B.FSTAT_EINVAL
    assert run(h, ctypes.byref(inp), vp(4096), float("nan"), vp(4096), 16, vp(4096), vp(0),
               vp(4096), ws.value, vp(0)) == B.FSTAT_EINVAL and "threshold" in B.last_error()
    assert run(None, ctypes.byref(inp), vp(4096), 70.0, vp(4096), 16, vp(4096), vp(0),
               vp(4096), ws.value, vp(0)) == B.FSTAT_EINVAL
    lib.fstat_search_destroy(h)


def test_search_chunks_keep_groups_whole(lib):
    """A sky group that fits a launch sequence is not split over two: 10
    groups of 10 spin-downs with 25 slots give 5 sequences of 2 groups; a
    group larger than the slots fills whole sequences."""
    ds, d = good_desc()
    p = B.Plan(d)
    vp = ctypes.c_void_p
    rows = [[1.0 + 0.01 * g, -0.5, 0, 1e-11 * k, 0, 0, 1.0, 0] for g in range(10) for k in range(10)]
    for tm, slots, want in ((np.array(rows), 25, 5), (np.array(rows), 30, 4),
                            (np.array(rows[:10] * 1), 4, 3)):
        tm = np.ascontiguousarray(tm, dtype=np.float64)
        h = vp()
        assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), len(tm), slots, 0,
                                       ctypes.byref(h)) == 0
        ng, nc = ctypes.c_int64(), ctypes.c_int64()
        assert lib.fstat_search_info(h, None, ctypes.byref(ng), ctypes.byref(nc)) == 0
        assert nc.value == want, (slots, nc.value)
        lib.fstat_search_destroy(h)


def test_autotune_checks_arguments_before_any_launch(lib):
    ds, d = good_desc()
    vp = ctypes.c_void_p
    best = B.FstatPlanDesc()
    ms = ctypes.c_float()
    inp = B.FstatInputs()
    tune = lib.fstat_autotune
    assert tune(ctypes.byref(d), ctypes.byref(inp), vp(4096), 1, vp(4096), vp(4096), 1 << 30,
                vp(0), None, ctypes.byref(ms)) == B.FSTAT_EINVAL
    assert tune(None, ctypes.byref(inp), vp(4096), 1, vp(4096), vp(4096), 1 << 30, vp(0),
                ctypes.byref(best), ctypes.byref(ms)) == B.FSTAT_EINVAL
    assert tune(ctypes.byref(d), ctypes.byref(inp), vp(4096), 0, vp(4096), vp(4096), 1 << 30,
                vp(0), ctypes.byref(best), ctypes.byref(ms)) == B.FSTAT_EINVAL
    assert "sample" in B.last_error()
    bad = B.make_plan_desc(ds)
    bad.ndet = 0
    assert tune(ctypes.byref(bad), ctypes.byref(inp), vp(4096), 1, vp(4096), vp(4096), 1 << 30,
                vp(0), ctypes.byref(best), ctypes.byref(ms)) == B.FSTAT_EINVAL


def test_autotune_search_cache_hit_runs_nothing(lib, tmp_path):
    """fstat_autotune_search with a cache line for this set-up returns its
    shape without touching the device (here, with no GPU at all); a line for
    another set-up, or a shape the plan refuses, is not taken; the argument
    checks come first."""
    ds, d = good_desc()
    vp = ctypes.c_void_p
    best = B.FstatPlanDesc()
    ms = ctypes.c_float()
    hit = ctypes.c_int32(7)
    inp = B.FstatInputs()
    tm = np.zeros((1, 8))
    key = f"n_fft={d.n_fft} ndet={d.ndet} D={d.sinc_halfwidth} flags={d.flags} slots=4" + \
        "".join(f" n{x}={d.det[x].n}" for x in range(d.ndet))
    log_n = int(math.log2(d.n_fft))
    lr = log_n // 2
    # line counts the plan accepts: the largest that fits the LDS, or half
    cmax, rmax = min(16384 >> lr, 64), min(8192 >> (log_n - lr), 32)
    cache = tmp_path / "tune.jsonl"
    cache.write_text(
        '{"key": "' + key.replace("slots=4", "slots=5") + f'", "tune": [{lr}, {cmax}, {rmax}, '
        '16], "ms": 1.5}\n'
        '{"key": "' + key + f'", "tune": [{lr}, {cmax // 2}, {rmax}, 32], "ms": 2.25}}\n')
    call = lib.fstat_autotune_search
    args = lambda slots, reps, c: (ctypes.byref(d), ctypes.byref(inp), tm.ctypes.data_as(vp),
                                    vp(4096), 1, slots, reps, vp(4096), c, vp(0),
                                    ctypes.byref(best), ctypes.byref(ms), ctypes.byref(hit))
    assert call(*args(4, 2, str(cache).encode())) == B.FSTAT_EINVAL
    assert "repeats" in B.last_error()
    assert call(*args(0, 3, str(cache).encode())) == B.FSTAT_EINVAL
    assert call(*args(4, 3, str(cache).encode())) == B.FSTAT_OK
    assert hit.value == 1 and abs(ms.value - 2.25) < 1e-6
    assert (best.tune_col_log_len, best.tune_col_lines, best.tune_row_lines,
            best.tune_fft_radix) == (lr, cmax // 2, rmax, 32)
    assert best.n_fft == d.n_fft and best.ndet == d.ndet
    # a refused shape (column length outside [6, 12]) is not taken: the call
    # goes on to time shapes, which needs a device
    cache.write_text('{"key": "' + key + f'", "tune": [13, {cmax}, {rmax}, 32], "ms": 2.25}}\n')
    r = call(*args(4, 3, str(cache).encode()))
    assert r != B.FSTAT_OK and hit.value == 0


def test_batch_checks_arguments_before_any_launch(lib):
    """fstat_batch_create/run validate every argument on the host."""
    vp = ctypes.c_void_p
    p = B.Plan(good_desc()[1])
    tm = np.zeros((3, 8))
    tm[:, 6] = 1.0
    h = vp()
    assert lib.fstat_search_create(p.handle, tm.ctypes.data_as(vp), 3, 2, 0, ctypes.byref(h)) == 0
    arr = (vp * 1)(h)
    b = vp()
    assert lib.fstat_batch_create(None, 1, 2, ctypes.byref(b)) == B.FSTAT_EINVAL
    assert lib.fstat_batch_create(arr, 0, 2, ctypes.byref(b)) == B.FSTAT_EINVAL
    assert lib.fstat_batch_create(arr, 1, 0, ctypes.byref(b)) == B.FSTAT_EINVAL
    assert lib.fstat_batch_create(arr, 1, 17, ctypes.byref(b)) == B.FSTAT_EINVAL
    assert "lanes" in B.last_error()
    assert lib.fstat_batch_create((vp * 1)(None), 1, 2, ctypes.byref(b)) == B.FSTAT_EINVAL
    assert lib.fstat_batch_create(arr, 1, 2, None) == B.FSTAT_EINVAL
    assert lib.fstat_batch_create(arr, 1, 4, ctypes.byref(b)) == B.FSTAT_OK
    ins = (ctypes.POINTER(B.FstatInputs) * 1)(ctypes.pointer(B.FstatInputs()))
    ptrs = (vp * 1)(4096)
    sizes = (ctypes.c_size_t * 1)(1 << 30)
    run = lib.fstat_batch_run
    assert run(None, ins, ptrs, ptrs, ptrs, sizes, vp(4096)) == B.FSTAT_EINVAL
    assert run(b, None, ptrs, ptrs, ptrs, sizes, vp(4096)) == B.FSTAT_EINVAL
    assert run(b, ins, ptrs, ptrs, ptrs, sizes, vp(0)) == B.FSTAT_EINVAL
    assert "stream" in B.last_error()
    # invalid inputs of a member search are reported before any launch
    assert run(b, ins, ptrs, ptrs, ptrs, sizes, vp(4096)) == B.FSTAT_EINVAL
    lib.fstat_batch_destroy(b)
    lib.fstat_search_destroy(h)


def test_sft_entry_checks_arguments_before_any_launch(lib):
    """fstat_sfts_to_series: invalid descriptions are refused on the host."""
    buf = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails first

    def call(**kw):
        d = B.FstatSftDesc(0.0, 300.0, 10, 29925, 150, 0)
        for k, v in kw.items():
            setattr(d, k, v)
        return lib.fstat_sfts_to_series(ctypes.byref(d), buf, None, buf, None, None)

    assert lib.fstat_sfts_to_series(None, buf, None, buf, None, None) == B.FSTAT_EINVAL
    assert call(t_sft=0.0) == B.FSTAT_EINVAL
    assert call(n_sft=0) == B.FSTAT_EINVAL
    assert call(k0=-1) == B.FSTAT_EINVAL
    assert call(reserved=1) == B.FSTAT_EINVAL
    assert call(n_bins=151) == B.FSTAT_EUNSUPPORTED        # odd
    assert call(n_bins=2 * 7 * 11) == B.FSTAT_EUNSUPPORTED  # prime factors above 5
    assert call(n_bins=8192) == B.FSTAT_EUNSUPPORTED        # beyond 4096
    d = B.FstatSftDesc(0.0, 300.0, 10, 29925, 150, 0)
    assert lib.fstat_sfts_to_series(ctypes.byref(d), None, None, buf, None, None) == B.FSTAT_EINVAL


def test_sinc_halfwidth_for_accuracy_bound(lib):
    """The accuracy rule for D against the oracle's own kernel definition
    (Hann-windowed sinc, 2D taps) evaluated here: the chosen D meets the bound
    over the band and the next smaller choice does not."""
    from oracle import fstat_oracle as O
    import numpy as np

    def worst(D, frac):
        e = 0.0
        for nu in np.linspace(0.0, frac / 2, 33):
            for u in np.linspace(0.0, 1.0, 17)[:-1]:
                j = np.arange(-D + 1, D + 1)
                jr = np.arange(-31, 33)
                a = np.abs(np.sum(O.sinc_kernel(u - j, D) * np.exp(2j * np.pi * nu * (j - u)))) ** 2
                r = np.abs(np.sum(O.sinc_kernel(u - jr, 32) * np.exp(2j * np.pi * nu * (jr - u)))) ** 2
                e = max(e, abs(a / r - 1))
        return e

    choices = (4, 6, 8, 10, 12, 16)
    for frac, tol in ((0.3, 1e-3), (0.5, 1e-3), (0.5, 1e-2)):
        D, err = B.sinc_halfwidth_for(frac, tol)
        assert D in choices and err <= tol
        assert worst(D, frac) <= tol * 1.05
        if D != choices[0]:
            smaller = choices[choices.index(D) - 1]
            assert worst(smaller, frac) > tol
    with pytest.raises(B.FstatError):
        B.sinc_halfwidth_for(0.95, 1e-6)
