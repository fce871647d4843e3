"""GPU parity of the whole filter recursion (tt_filter_run) against the CPU
oracle: linear-Gaussian workload (also against the Kalman filter), reduced
range workloads in FP64 and FP32, ragged batches."""
import math

import numpy as np
import pytest

from oracle import filters as flt
from oracle import model as mdl
from oracle import tt as ttm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import binding, runner, workload
    assert torch.cuda.is_available()
    return binding, runner, workload


def oracle_run(s, z):
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    return flt.run_tt_filter(axes, s.q, s.halfwidths(), s.meas(), z, s.m0, s.p0_diag, s.cap, s.eps)


def test_kf2d_fp64_matches_oracle_and_kalman(mods):
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("kf2d")
    s, z = specs[0], zs[0]
    ref = oracle_run(s, z)
    kf = flt.run_kalman(s.q, np.eye(2) * s.sigma_lin ** 2, z, s.m0, np.diag(s.p0_diag))
    run, _ = runner.run_filters(specs, zs, B.F64)
    assert int(run.status.cpu()[0]) == 0
    lc = run.log_c.cpu().numpy()[0]
    mean = run.mean.cpu().numpy()[0]
    cov = run.cov.cpu().numpy()[0]
    assert np.abs(lc - ref["log_c"]).max() < 1e-10 * max(1.0, np.abs(ref["log_c"]).max())
    dx = (s.hi - s.lo) / (s.n - 1)
    assert np.abs(mean - ref["mean"]).max() < 1e-10 * dx
    assert np.abs(cov - ref["cov"]).max() < 1e-10
    assert np.abs(mean - kf["mean"]).max() < 1e-8
    assert abs(run.loglik.item() - ref["loglik"]) < 1e-9


@pytest.fixture
def predict_mode(mods, request):
    B = mods[0]
    B.set_predict_mode(request.param)
    yield request.param
    B.set_predict_mode(B.PREDICT_DIRECT)


@pytest.mark.parametrize("predict_mode", [0, 1, 2], indirect=True)
@pytest.mark.parametrize("d,n,cap,steps", [(3, 40, 8, 6), (4, 32, 8, 5)])
def test_range_fp64_matches_oracle(mods, d, n, cap, steps, predict_mode):
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=steps, d=d, n=n, cap=cap)
    s, z = specs[0], zs[0]
    ref = oracle_run(s, z)
    run, _ = runner.run_filters(specs, zs, B.F64)
    assert int(run.status.cpu()[0]) == 0
    lc = run.log_c.cpu().numpy()[0]
    mp = run.log_mpred.cpu().numpy()[0]
    mean = run.mean.cpu().numpy()[0]
    ranks = run.ranks.cpu().numpy()[0]
    dx = s.spacing()
    assert [list(r) for r in ranks] == [list(r) for r in ref["ranks_filt"]]
    assert np.abs(lc - ref["log_c"]).max() < 1e-10 * max(1.0, np.abs(ref["log_c"]).max())
    assert np.abs(mp[1:] - ref["log_mpred"]).max() < 1e-10
    assert np.abs(mean - ref["mean"]).max() < 1e-10 * dx


@pytest.mark.parametrize("predict_mode", [0, 1, 2], indirect=True)
def test_per_axis_kernel_widths_fp64(mods, predict_mode):
    # different process-noise scales per axis give kernel fibres of different
    # lengths in every core
    B, runner, wl = mods
    s = wl.spec_range(3, 36, 8, sigma_w=[1.0, 0.6, 1.4])
    assert len(set(s.halfwidths())) == 3
    x, z = wl.simulate(s, 5, __import__("numpy").random.SeedSequence(7))
    ref = oracle_run(s, z)
    run, _ = runner.run_filters([s], [z], B.F64)
    assert int(run.status.cpu()[0]) == 0
    lc = run.log_c.cpu().numpy()[0]
    assert np.abs(lc - ref["log_c"]).max() < 1e-10 * max(1.0, np.abs(ref["log_c"]).max())
    assert np.abs(run.mean.cpu().numpy()[0] - ref["mean"]).max() < 1e-10 * s.spacing()


@pytest.mark.parametrize("predict_mode", [0, 1, 2, 3], indirect=True)
def test_range_fp32_meets_reduced_precision_bars(mods, predict_mode):
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=6, d=3, n=40, cap=8)
    s, z = specs[0], zs[0]
    ref = oracle_run(s, z)
    run, _ = runner.run_filters(specs, zs, B.F32)
    assert int(run.status.cpu()[0]) == 0
    mean = run.mean.cpu().numpy()[0]
    lc = run.log_c.cpu().numpy()[0]
    dx = s.spacing()
    assert np.abs(mean - ref["mean"]).max() < 1e-3 * dx
    assert np.abs(lc - ref["log_c"]).max() < 1e-4


def test_ragged_batch_equals_single_runs(mods):
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range6d_ragged", batch=3, steps=3, d=3)
    for s, n in zip(specs, (32, 24, 40)):
        s.n = n
    for s, c in zip(specs, (4, 8, 6)):
        s.cap = c
    run, _ = runner.run_filters(specs, zs, B.F64)
    for b in range(3):
        one, _ = runner.run_filters([specs[b]], [zs[b]], B.F64)
        assert np.array_equal(one.log_c.cpu().numpy()[0], run.log_c.cpu().numpy()[b])
        assert np.array_equal(one.mean.cpu().numpy()[0], run.mean.cpu().numpy()[b])
        ref = oracle_run(specs[b], zs[b])
        assert np.abs(run.log_c.cpu().numpy()[b] - ref["log_c"]).max() < 1e-9


def fp32_bars(run, b, s, ref):
    assert int(run.status.cpu()[b]) == 0
    mean = run.mean.cpu().numpy()[b]
    lc = run.log_c.cpu().numpy()[b]
    assert np.abs(mean - ref["mean"]).max() < 1e-3 * s.spacing()
    assert np.abs(lc - ref["log_c"]).max() < 1e-4


@pytest.mark.parametrize("predict_mode", [0, 3], indirect=True)
def test_per_axis_kernel_widths_fp32(mods, predict_mode):
    # kernel fibres of different lengths per core on the FP32 prediction
    # kernels (matrix-core and vector-ALU); n = 36 leaves a ragged 16-row tile
    B, runner, wl = mods
    s = wl.spec_range(3, 36, 8, sigma_w=[1.0, 0.6, 1.4])
    x, z = wl.simulate(s, 5, np.random.SeedSequence(7))
    ref = oracle_run(s, z)
    run, _ = runner.run_filters([s], [z], B.F32)
    fp32_bars(run, 0, s, ref)


@pytest.mark.parametrize("predict_mode", [0, 3], indirect=True)
def test_wide_bond_fp32(mods, predict_mode):
    # rank cap 24: bonds that are not a multiple of 4 and more than 32
    # columns in the absorbed factor (two column passes of the MFMA kernel)
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=5, d=3, n=40, cap=24)
    s, z = specs[0], zs[0]
    ref = oracle_run(s, z)
    run, _ = runner.run_filters(specs, zs, B.F32)
    fp32_bars(run, 0, s, ref)


def test_fp32_batch_of_64_equals_single_runs(mods):
    # a batch large enough for the wide launch shapes gives every filter
    # bit-for-bit the result it gets alone
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range6d_ragged", batch=64, steps=3, d=3)
    for i, s in enumerate(specs):
        s.n = (24, 32, 40)[i % 3]
        s.cap = (4, 8, 6)[i % 3]
    run, _ = runner.run_filters(specs, zs, B.F32)
    for b in (0, 1, 2, 37, 63):
        one, _ = runner.run_filters([specs[b]], [zs[b]], B.F32)
        assert np.array_equal(one.log_c.cpu().numpy()[0], run.log_c.cpu().numpy()[b])
        assert np.array_equal(one.mean.cpu().numpy()[0], run.mean.cpu().numpy()[b])


@pytest.mark.parametrize("predict_mode", [0, 3], indirect=True)
@pytest.mark.parametrize("d,n,cap,steps", [(3, 40, 8, 6), (4, 32, 8, 5)])
def test_fp32_density_l1_against_dense_oracle(mods, d, n, cap, steps, predict_mode):
    # the reduced-precision bar on the density itself: L1 = sum |dP| delta of
    # the final filtering densities, reconstructed densely (N^d <= 1.1e6)
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=steps, d=d, n=n, cap=cap)
    s, z = specs[0], zs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    ref = flt.run_tt_filter(axes, s.q, s.halfwidths(), s.meas(), z, s.m0, s.p0_diag, s.cap, s.eps)
    run, _ = runner.run_filters(specs, zs, B.F32)
    assert int(run.status.cpu()[0]) == 0
    cores, st = run.save_state()[0].fetch_scaled()
    assert st == 0
    delta = mdl.cell_volume(axes)
    l1 = float(np.abs(ttm.full(cores) - ttm.full(ref["final"])).sum()) * delta
    print(f"fp32 d={d} N={n} cap={cap}: dense L1 of the final density {l1:.2e}")
    assert l1 <= 1e-4
