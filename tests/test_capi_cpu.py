"""C ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and host-side validation rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttgbf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:size_t|tt_status|const char\*|void|int32_t)\s+(tt_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("tt_kernel_build", "tt_predict", "tt_update", "tt_round", "tt_normalize_moments",
                 "tt_filter_run"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2501_07942_amd import binding as B
    lib = C.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(B.EXPORTED) == set(declared_functions())


def test_train_elems_and_version():
    from paper_2501_07942_amd import binding as B
    n = (C.c_int32 * 3)(4, 5, 6)
    cap = (C.c_int32 * 4)(1, 2, 3, 1)
    assert B.LIB.tt_train_elems(3, n, cap) == 1 * 4 * 2 + 2 * 5 * 3 + 3 * 6 * 1
    assert B.LIB.tt_train_elems(0, n, cap) == 0
    assert b"gfx950" in B.LIB.tt_version()


def test_host_validation_rejects_before_launch():
    from paper_2501_07942_amd import binding as B
    # null arguments
    st = B.LIB.tt_round(1, None, None, 1e-10, 4, None, 0, None)
    assert st == B.ERR_ARG
    assert b"null" in B.LIB.tt_last_error()
    # malformed train: cap[0] != 1 is rejected by the workspace query
    t = B.Train()
    t.d = 2
    t.n[0] = t.n[1] = 4
    t.cap[0], t.cap[1], t.cap[2] = 2, 2, 1
    t.dtype = B.F64
    t.cores = t.ranks = t.log_scale = t.status = 1024  # never dereferenced on the host
    arr = (B.Train * 1)(t)
    assert B.LIB.tt_round_workspace(1, arr, arr) == 0
    # eps < 0 rejected
    t.cap[0] = 1
    arr = (B.Train * 1)(t)
    st = B.LIB.tt_round(1, arr, arr, -1.0, 4, C.c_void_p(4096), 1 << 20, None)
    assert st == B.ERR_ARG
    # workspace too small
    need = B.LIB.tt_round_workspace(1, arr, arr)
    assert need > 0
    st = B.LIB.tt_round(1, arr, arr, 1e-10, 4, C.c_void_p(4096), 16, None)
    assert st == B.ERR_WORKSPACE
    # bad grid in kernel build
    g = B.make_grid(2, [1, 4], [0, 0], [1, 1])
    hw = (C.c_int32 * 2)(1, 1)
    capa = (C.c_int32 * 3)(1, 2, 1)
    assert B.LIB.tt_kernel_build_workspace(C.byref(g), hw, capa) == 0


def test_filter_run_workspace_query():
    from paper_2501_07942_amd import binding as B, runner, workload as wl
    specs, _, _ = wl.make_batch("range4d", batch=2, steps=3, d=3, n=32, cap=8)
    fs = runner.filter_specs(specs, [0, 0], 13, 64)
    arr = (B.FilterSpec * 2)(*fs)
    kt = B.Train()
    kt.d = 3
    for k in range(3):
        kt.n[k] = 2 * specs[0].halfwidths()[k] + 1
    kt.cap[0], kt.cap[1], kt.cap[2], kt.cap[3] = 1, 13, 13, 1
    kt.dtype = B.F64
    kt.cores = kt.ranks = kt.log_scale = kt.status = 4096  # never dereferenced on the host
    karr = (B.Train * 1)(kt)
    assert B.LIB.tt_filter_run_workspace(2, arr, karr, 1, B.F64) > 0
    assert B.LIB.tt_filter_run_workspace(2, arr, karr, 1, 7) == 0
    assert B.LIB.tt_filter_run_workspace(2, arr, None, 0, B.F64) == 0


def test_einsum_prediction_validation():
    from paper_2501_07942_amd import binding as B

    def train(d, n, caps):
        t = B.Train()
        t.d = d
        for k in range(d):
            t.n[k] = n[k]
        for k in range(d + 1):
            t.cap[k] = caps[k]
        t.dtype = B.F64
        t.cores = t.ranks = t.log_scale = t.status = 1024  # never dereferenced on the host
        return t

    p = train(2, [5, 6], [1, 3, 1])
    tpm = train(4, [5, 6, 5, 6], [1, 4, 9, 4, 1])
    P, T = (B.Train * 1)(p), (B.Train * 1)(tpm)
    need = B.LIB.tt_predict_einsum_workspace(1, T, P)
    assert need > 0
    # a transition train of the wrong length or mode sizes is rejected
    bad = (B.Train * 1)(train(3, [5, 6, 5], [1, 4, 9, 1]))
    assert B.LIB.tt_predict_einsum_workspace(1, bad, P) == 0
    bad = (B.Train * 1)(train(4, [5, 6, 5, 7], [1, 4, 9, 4, 1]))
    assert B.LIB.tt_predict_einsum_workspace(1, bad, P) == 0
    # an output whose capacities cannot hold the transition train's ranks
    small = (B.Train * 1)(train(2, [5, 6], [1, 2, 1]))
    st = B.LIB.tt_predict_einsum(1, T, P, small, C.c_void_p(4096), need, None)
    assert st == B.ERR_SHAPE
    ok = (B.Train * 1)(train(2, [5, 6], [1, 4, 1]))
    st = B.LIB.tt_predict_einsum(1, T, P, ok, C.c_void_p(4096), 16, None)
    assert st == B.ERR_WORKSPACE


def test_redesign_and_interpolation_validation():
    from paper_2501_07942_amd import binding as B

    def train(n, caps):
        t = B.Train()
        t.d = len(n)
        for k in range(t.d):
            t.n[k] = n[k]
        for k in range(t.d + 1):
            t.cap[k] = caps[k]
        t.dtype = B.F64
        t.cores = t.ranks = t.log_scale = t.status = 1024  # never dereferenced on the host
        return t

    g0 = B.make_grid(2, [8, 9], [-1.0, -1.0], [1.0, 1.0])
    g1 = B.make_grid(2, [8, 9], [-2.0, -1.0], [1.0, 2.0])
    gi = (B.Grid * 1)(g0)
    go = (B.Grid * 1)(g1)
    tin = (B.Train * 1)(train([8, 9], [1, 3, 1]))
    need = B.LIB.tt_interpolate_workspace(1)
    assert need > 0
    ws = C.c_void_p(4096)
    # grid and train disagree on a mode size
    bad = (B.Train * 1)(train([8, 10], [1, 3, 1]))
    assert B.LIB.tt_interpolate(1, gi, go, tin, bad, ws, need, None) == B.ERR_SHAPE
    # output capacity below the input's
    small = (B.Train * 1)(train([8, 9], [1, 2, 1]))
    assert B.LIB.tt_interpolate(1, gi, go, tin, small, ws, need, None) == B.ERR_SHAPE
    # an axis of one point has no spacing
    g2 = (B.Grid * 1)(B.make_grid(2, [1, 9], [-1.0, -1.0], [1.0, 1.0]))
    one = (B.Train * 1)(train([1, 9], [1, 3, 1]))
    assert B.LIB.tt_interpolate(1, g2, g2, one, one, ws, need, None) == B.ERR_SHAPE
    # grid re-design: a singular F and a non-positive nsigma are rejected
    # before anything reaches the device
    f = (C.c_double * 4)(1.0, 2.0, 2.0, 4.0)
    q = (C.c_double * 4)(1.0, 0.0, 0.0, 1.0)
    out = (B.Grid * 1)()
    rneed = B.LIB.tt_grid_redesign_workspace(1, 2)
    assert rneed > 0
    st = B.LIB.tt_grid_redesign(1, 2, f, q, 3.0, C.c_void_p(4096), C.c_void_p(4096), gi, out, ws, rneed, None)
    assert st == B.ERR_ARG and b"singular" in B.LIB.tt_last_error()
    f2 = (C.c_double * 4)(1.1, 0.1, -0.2, 1.1)
    st = B.LIB.tt_grid_redesign(1, 2, f2, q, 0.0, C.c_void_p(4096), C.c_void_p(4096), gi, out, ws, rneed, None)
    assert st == B.ERR_ARG


def test_status_strings():
    from paper_2501_07942_amd import binding as B
    assert B.status_string(B.OK).startswith("TT_OK")
    assert B.status_string(B.ERR_WORKSPACE).startswith("TT_ERR_WORKSPACE")
    assert B.status_string(99) == "unknown tt_status code"
    assert B.device_status_string(0) == "ok"
    both = B.device_status_string(B.STATUS_NONFINITE | B.STATUS_CAPACITY)
    assert "NONFINITE" in both and "CAPACITY" in both


def test_filter_state_rejects_bad_direction_before_launch():
    from paper_2501_07942_amd import binding as B
    st = B.LIB.tt_filter_state(1, None, None, 0, B.F64, 7, None, None, 0, None)
    assert st == B.ERR_ARG
    assert b"tt_filter_state" in B.LIB.tt_last_error()
