"""Pins of the oracle's log-likelihood gradients (CPU).

Three independent routes are checked against each other and against closed
forms: the Kalman filter (exact for the linear-Gaussian model), the dense
point-mass filter differentiated by the complex step, and central
differences of the TT filter with its ranks replayed.
"""
import numpy as np
import pytest

from oracle import grad as og
from oracle import model as mdl
from paper_2501_07942_amd import workload as wl


def ctx_of(s, z, cap=None):
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    sw = np.sqrt(np.diag(s.q))
    return dict(axes=axes, corr=s.q / np.outer(sw, sw), halfwidths=s.halfwidths(), z=z, m0=s.m0,
                p0_diag=s.p0_diag, cap=cap or s.cap, eps=s.eps, meas_kind=s.meas_kind), sw


@pytest.fixture(scope="module")
def linear_case():
    s = wl.spec_kf2d()
    x, z = wl.simulate(s, 12, np.random.SeedSequence(11))
    ctx, sw = ctx_of(s, z)
    return ctx, np.concatenate([sw, [s.sigma_lin]])


@pytest.fixture(scope="module")
def range_case():
    s = wl.spec_range(2, 40, 40, lo=-10.0, hi=10.0, sigma_w=[1.0, 0.8])
    x, z = wl.simulate(s, 8, np.random.SeedSequence(5))
    ctx, sw = ctx_of(s, z)
    return ctx, np.concatenate([sw, [s.sigma_r, s.sigma_lin, s.sensor[0], s.sensor[1]]])


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_complex_step_equals_central_differences_on_kalman(linear_case):
    # the complex-step machinery against plain central differences of the
    # same analytic function
    ctx, th = linear_case
    g_cs = og.grad_complex_step(og.loglik_kalman_cs, th, ctx)
    g_fd = og.grad_fd(og.loglik_kalman_cs, th, ctx)
    assert rel(g_cs, g_fd) < 1e-8


def test_kalman_loglik_matches_closed_form_filter(linear_case):
    # the complex-capable Kalman LL is the real Kalman filter's LL
    from oracle import filters as flt
    ctx, th = linear_case
    sw, meas = og.unpack(th, 2, "linear")
    q = og.q_of(sw, ctx["corr"])
    ref = flt.run_kalman(q, np.eye(2) * meas["sigma_lin"] ** 2, ctx["z"], ctx["m0"], np.diag(ctx["p0_diag"]))
    assert abs(og.loglik_kalman_cs(th, ctx).real - ref["loglik"]) < 1e-12 * abs(ref["loglik"])


def test_dense_pmf_gradient_matches_kalman_gradient(linear_case):
    # linear-Gaussian model on a spectrally accurate grid: the dense point-mass
    # filter's exact (complex-step) gradient equals the Kalman gradient up to
    # the grid discretisation
    ctx, th = linear_case
    g_dense = og.grad_complex_step(og.loglik_dense_cs, th, ctx)
    g_kf = og.grad_complex_step(og.loglik_kalman_cs, th, ctx)
    assert rel(g_dense, g_kf) < 1e-7


def test_dense_loglik_matches_dense_filter(range_case):
    from oracle import filters as flt
    ctx, th = range_case
    sw, meas = og.unpack(th, 2, "range")
    q = og.q_of(sw, ctx["corr"])
    ref = flt.run_dense_pmf(ctx["axes"], q, ctx["halfwidths"], meas, ctx["z"], ctx["m0"], ctx["p0_diag"])
    assert abs(og.loglik_dense_cs(th, ctx).real - ref["loglik"]) < 1e-11 * abs(ref["loglik"])


def test_tt_replay_gradient_matches_dense_complex_step(range_case):
    # range measurement, rank cap not binding: the TT filter is the dense
    # filter to the rounding tolerance, and so are their gradients
    ctx, th = range_case
    ll, g_tt, base = og.grad_fd_tt(th, ctx)
    g_dense = og.grad_complex_step(og.loglik_dense_cs, th, ctx)
    assert rel(g_tt, g_dense) < 1e-7
    # sigma_lin does not enter a d = 2 range model
    assert g_tt[3] == 0.0 and g_dense[3] == 0.0


def test_rank_replay_reproduces_the_base_run(range_case):
    ctx, th = range_case
    c6 = dict(ctx, cap=6)
    base = og.loglik_tt(th, c6)
    again = og.loglik_tt(th, c6, {"ranks_pred": base["ranks_pred"], "ranks_filt": base["ranks_filt"]})
    assert again["loglik"] == base["loglik"]
    assert again["ranks_filt"] == base["ranks_filt"]


def test_replay_gradient_is_stable_when_the_cap_binds(range_case):
    # with the cap binding, central differences with replayed ranks converge
    # (h = 1e-4 and 1e-5 agree), and the gradient differs from the dense one
    # by the truncation, not by noise
    ctx, th = range_case
    c6 = dict(ctx, cap=6)
    _, g5, base = og.grad_fd_tt(th, c6, h_rel=1e-5)
    _, g4, _ = og.grad_fd_tt(th, c6, h_rel=1e-4)
    assert max(r for rr in base["ranks_filt"] for r in rr) == 6
    assert rel(g4, g5) < 1e-6
    g_dense = og.grad_complex_step(og.loglik_dense_cs, th, ctx)
    assert 1e-4 < rel(g5, g_dense) < 5e-2
