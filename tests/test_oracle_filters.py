"""Pins for the oracle filters: Kalman agreement on the linear-Gaussian
workload, dense vs TT agreement, Kalman closed form (CPU only)."""
import math

import numpy as np
import pytest

from oracle import filters as flt
from oracle import model as mdl
from oracle import tt as ttm
from paper_2501_07942_amd import workload as wl


def test_kalman_scalar_closed_form():
    # one update with prior N(1, 4), R = 1, z = 3: posterior mean 1 + 4/5*2,
    # variance 4 - 16/5, log c = log N(3; 1, 5); then predict with Q = 0.5
    q = np.array([[0.5]])
    out = flt.run_kalman(q, np.array([[1.0]]), np.array([[3.0], [2.0]]), [1.0], np.array([[4.0]]))
    assert abs(out["mean"][0][0] - 2.6) < 1e-15
    assert abs(out["cov"][0][0][0] - 0.8) < 1e-15
    assert abs(out["log_c"][0] - (-0.5 * (math.log(2 * math.pi * 5) + 4 / 5))) < 1e-14
    pm, pv = 2.6, 1.3
    assert abs(out["log_c"][1] - (-0.5 * (math.log(2 * math.pi * (pv + 1)) + (2 - pm) ** 2 / (pv + 1)))) < 1e-14
    assert abs(out["mean"][1][0] - (pm + pv / (pv + 1) * (2 - pm))) < 1e-14


def test_kf2d_tt_dense_kalman_agree():
    specs, xs, zs = wl.make_batch("kf2d")
    s, z = specs[0], zs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    h = s.halfwidths()
    tt = flt.run_tt_filter(axes, s.q, h, s.meas(), z, s.m0, s.p0_diag, s.cap, s.eps)
    de = flt.run_dense_pmf(axes, s.q, h, s.meas(), z, s.m0, s.p0_diag)
    kf = flt.run_kalman(s.q, np.eye(2) * s.sigma_lin ** 2, z, s.m0, np.diag(s.p0_diag))
    # separable model: every TT stays exactly rank one
    assert all(r == [1, 1, 1] for r in tt["ranks_filt"])
    assert np.abs(tt["log_c"] - de["log_c"]).max() < 1e-12
    assert np.abs(tt["mean"] - de["mean"]).max() < 1e-12
    assert np.abs(tt["cov"] - de["cov"]).max() < 1e-12
    # the grid truncates the Gaussians at the box edge (x0 ~ N(0,4) on
    # [-10,10]: 5 sigma), which moves log c_k by up to ~1e-6
    assert np.abs(tt["log_c"] - kf["log_c"]).max() < 1e-5
    assert np.abs(tt["mean"] - kf["mean"]).max() < 1e-8
    assert np.abs(tt["cov"] - kf["cov"]).max() < 1e-8


def test_dense_vs_tt_range_reduced():
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=6, d=3, n=32, cap=64)
    s, z = specs[0], zs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    h = s.halfwidths()
    tt = flt.run_tt_filter(axes, s.q, h, s.meas(), z, s.m0, s.p0_diag, s.cap, 1e-12)
    de = flt.run_dense_pmf(axes, s.q, h, s.meas(), z, s.m0, s.p0_diag, record_density=True)
    # cap not binding and tol 1e-12: the TT filter equals the dense filter to
    # the accumulated rounding tolerance
    assert np.abs(tt["log_c"] - de["log_c"]).max() < 1e-9
    assert np.abs(tt["mean"] - de["mean"]).max() < 1e-9
    fin = ttm.full(tt["final"])
    assert np.linalg.norm(fin - de["final"]) < 1e-9 * np.linalg.norm(de["final"])


def test_tt_filter_unit_mass_and_records():
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=4, d=3, n=32, cap=8)
    s, z = specs[0], zs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    out = flt.run_tt_filter(axes, s.q, s.halfwidths(), s.meas(), z, s.m0, s.p0_diag, s.cap, s.eps)
    mass, _, _ = mdl.moments_tt(out["final"], axes)
    assert abs(mass - 1.0) < 1e-13
    assert len(out["log_c"]) == 4 and len(out["log_mpred"]) == 3
    assert all(max(r) <= 8 for r in out["ranks_filt"])
    # a nonnegative PMD cannot gain more mass than the kernel carries
    ksum = mdl.kernel_dense(s.q, axes, s.halfwidths()).sum()
    assert np.all(out["log_mpred"] <= math.log(ksum) + 1e-12)


def test_marginal_min_is_the_smallest_dense_marginal_value():
    # the negativity monitor of the oracle filter against the dense marginals
    # of a TT with negative entries
    from oracle.filters import _marginal_min
    rng = np.random.default_rng(21)
    rk = [1, 2, 3, 1]
    a = [rng.standard_normal((rk[k], n, rk[k + 1])) for k, n in enumerate((4, 5, 3))]
    f = ttm.full(a)
    want = min(float(f.sum(axis=tuple(j for j in range(3) if j != l)).min()) for l in range(3))
    assert abs(_marginal_min(a) - want) < 1e-12 * np.abs(f).sum()
    assert want < 0.0


def test_rounding_tail_record_is_the_truncation_error_bound():
    # the per-rounding record of the oracle filter: sqrt(sum of the squared
    # discarded tails) / ||A||; for one bond it is the truncation error itself
    # (Eckart-Young), for several an upper bound of it (the TT-SVD bound)
    from oracle import tt as ttm
    from oracle.filters import _tail_rel
    rng = np.random.default_rng(11)
    m = rng.standard_normal((20, 7)) @ rng.standard_normal((7, 18)) + 1e-3 * rng.standard_normal((20, 18))
    a2 = [m.reshape(1, 20, 18), np.eye(18).reshape(18, 18, 1)]
    r2, info = ttm.tt_round(a2, 1e-12, 4, return_info=True)
    err = np.linalg.norm(ttm.full(r2) - m) / np.linalg.norm(m)
    assert abs(_tail_rel(info) - err) <= 1e-10 * err
    cores = [rng.standard_normal((1, 6, 5)), rng.standard_normal((5, 7, 6)), rng.standard_normal((6, 5, 4)),
             rng.standard_normal((4, 6, 1))]
    r4, info = ttm.tt_round(cores, 1e-12, 3, return_info=True)
    full = ttm.full(cores)
    err = np.linalg.norm(ttm.full(r4) - full) / np.linalg.norm(full)
    assert 0.0 < err <= _tail_rel(info) * (1 + 1e-10)
