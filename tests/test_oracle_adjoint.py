"""Pins of the oracle's reverse-mode gradient (CPU).

Every adjoint is checked against something other than itself: directional
derivatives of the oracle's own forward routines (QR/SVD rounding, TT-SVD,
convolution, Hadamard, sum), the Kalman filter and the dense point-mass
filter differentiated by the complex step, and central differences of the
TT filter with replayed ranks.
"""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import grad as og
from oracle import model as mdl
from oracle import tt as ttm
from paper_2501_07942_amd import workload as wl

import os, sys  # noqa: E401
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from adjoint_helpers import full_vjp  # noqa: E402


def rand_tt(rng, n, r, decay=1.0):
    rk = [1] + list(r) + [1]
    cores = []
    for k in range(len(n)):
        g = rng.standard_normal((rk[k], n[k], rk[k + 1]))
        # geometric column scales give each unfolding a graded spectrum
        g *= decay ** np.arange(rk[k + 1])[None, None, :]
        cores.append(g)
    return cores


def inner(a, b):
    return float(sum(np.sum(x * y) for x, y in zip(a, b)))


def perturbed(cores, dirs, h):
    return [c + h * dc for c, dc in zip(cores, dirs)]


def test_sum_vjp_is_the_derivative_of_the_sum():
    rng = np.random.default_rng(1)
    a = rand_tt(rng, [4, 5, 3], [3, 2])
    da = rand_tt(rng, [4, 5, 3], [3, 2])
    # the sum is linear in each core: one core at a time
    g = oa.sum_vjp(a, 1.7)
    for k in range(3):
        dk = [np.zeros_like(x) for x in a]
        dk[k] = da[k]
        exact = 1.7 * (ttm.tt_sum(perturbed(a, dk, 1.0)) - ttm.tt_sum(a))
        assert abs(inner(g, dk) - exact) < 1e-12 * max(1.0, abs(exact))


def test_moments_vjp_matches_directional_differences():
    # the moments of model.moments_tt (means and covariance of the density
    # the TT holds, on its grid) differentiated along a random core direction,
    # against central differences of the moments themselves; the cell volume
    # cancels, so it is the derivative with respect to the cores
    rng = np.random.default_rng(4)
    n = [6, 7, 5]
    a = [np.abs(g) + 0.1 for g in rand_tt(rng, n, [3, 2])]
    da = rand_tt(rng, n, [3, 2])
    axes = mdl.grid_axes([-2.0, -1.0, 0.5], [3.0, 2.5, 4.0], n)
    mb = rng.standard_normal(3)
    cb = rng.standard_normal((3, 3))  # not symmetric: both entries of a pair count

    def f(cores):
        _, mean, cov = mdl.moments_tt(cores, axes)
        return float(mb @ mean + np.sum(cb * cov))

    g = oa.moments_vjp(a, axes, mb, cb)
    h = 1e-6
    fd = (f(perturbed(a, da, h)) - f(perturbed(a, da, -h))) / (2 * h)
    assert abs(inner(g, da) - fd) < 1e-7 * max(1.0, abs(fd))
    # only the means, only the covariance
    g1 = oa.moments_vjp(a, axes, mb, None)
    g2 = oa.moments_vjp(a, axes, None, cb)
    assert abs(inner(g1, da) + inner(g2, da) - inner(g, da)) < 1e-12 * max(1.0, abs(fd))
    # a scaled density has the same moments: the adjoint is orthogonal to it
    assert abs(inner(g, a)) < 1e-10 * max(1.0, float(np.sqrt(inner(g, g) * inner(a, a))))


def test_hadamard_and_conv_adjoint_identities():
    # <Cbar, dC> = <Abar, dA> + <Bbar, dB> for the bilinear maps, with the
    # forward maps taken from oracle.tt
    rng = np.random.default_rng(2)
    la = rand_tt(rng, [6, 7, 5], [2, 3])
    pb = rand_tt(rng, [6, 7, 5], [3, 2])
    dla = rand_tt(rng, [6, 7, 5], [2, 3])
    dpb = rand_tt(rng, [6, 7, 5], [3, 2])
    hb = [rng.standard_normal(g.shape) for g in ttm.hadamard(la, pb)]
    abar, bbar = oa.hadamard_vjp(la, pb, hb)
    lhs = inner(hb, ttm.hadamard(dla, pb)) + inner(hb, ttm.hadamard(la, dpb))
    assert abs(lhs - inner(abar, dla) - inner(bbar, dpb)) < 1e-10 * abs(lhs)
    hw = [2, 3, 1]
    kk = rand_tt(rng, [5, 7, 3], [2, 2])
    dkk = rand_tt(rng, [5, 7, 3], [2, 2])
    cb = [rng.standard_normal(g.shape) for g in ttm.conv(kk, pb, hw)]
    kbar, pbar = oa.conv_vjp(kk, pb, hw, cb)
    lhs = inner(cb, ttm.conv(dkk, pb, hw)) + inner(cb, ttm.conv(kk, dpb, hw))
    assert abs(lhs - inner(kbar, dkk) - inner(pbar, dpb)) < 1e-10 * abs(lhs)


def test_topvec_vjp_matches_eigenvector_differences():
    # f(S) = tr(U_r^T X U_r) depends on the leading subspace only
    rng = np.random.default_rng(3)
    m = rng.standard_normal((9, 6)) * (0.5 ** np.arange(6))[None, :]
    x = rng.standard_normal((9, 9))
    x = x + x.T
    dm = rng.standard_normal((9, 6))
    r = 3

    def f(mm):
        u, s, _ = np.linalg.svd(mm, full_matrices=False)
        ur = u[:, :r]
        return float(np.trace(ur.T @ x @ ur))

    u, s, _ = np.linalg.svd(m, full_matrices=False)
    ubar = 2.0 * x @ u[:, :r]
    sbar = oa.topvec_vjp(u, s, r, ubar)
    # S = M M^T: <Sbar, dS> with dS = dM M^T + M dM^T
    pred = float(np.sum(sbar * (dm @ m.T + m @ dm.T)))
    h = 1e-6
    fd = (f(m + h * dm) - f(m - h * dm)) / (2 * h)
    assert abs(pred - fd) < 1e-7 * max(1.0, abs(fd))


def test_round_vjp_matches_directional_differences_of_qr_svd_rounding():
    # the adjoint of the Gram-form rounding against central differences of
    # oracle.tt.tt_round (Householder QR + SVD) at the same forced ranks
    rng = np.random.default_rng(4)
    n = [4, 5, 4, 3]
    a = rand_tt(rng, n, [4, 6, 3], decay=0.6)
    da = rand_tt(rng, n, [4, 6, 3])
    forced = [1, 3, 3, 2, 1]
    y, tape = oa.round_fwd(a, forced)
    assert np.linalg.norm(ttm.full(y) - ttm.full(ttm.tt_round(a, 0.0, None, forced_ranks=forced))) \
        < 1e-12 * np.linalg.norm(ttm.full(y))
    t = rng.standard_normal(n)
    abar = oa.round_vjp(tape, full_vjp(y, t))
    h = 1e-6

    def f(cores):
        return float(np.sum(ttm.full(ttm.tt_round(cores, 0.0, None, forced_ranks=forced)) * t))

    fd = (f(perturbed(a, da, h)) - f(perturbed(a, da, -h))) / (2 * h)
    assert abs(inner(abar, da) - fd) < 1e-7 * abs(fd)


def test_tt_svd_vjp_matches_directional_differences():
    rng = np.random.default_rng(5)
    base = ttm.full(rand_tt(rng, [5, 4, 6], [3, 3], decay=0.5))
    x = base + 1e-9 * rng.standard_normal(base.shape)     # ranks 3, 3 at tol 1e-6
    dx = rng.standard_normal(base.shape)
    cores, tape = oa.tt_svd_fwd(x, 1e-6)
    assert ttm.ranks(cores) == [1, 3, 3, 1]
    t = rng.standard_normal(base.shape)
    xbar = oa.tt_svd_vjp(tape, full_vjp(cores, t))
    h = 1e-7

    def f(xx):
        c = ttm.tt_svd(xx, 1e-6)
        assert ttm.ranks(c) == [1, 3, 3, 1]
        return float(np.sum(ttm.full(c) * t))

    fd = (f(x + h * dx) - f(x - h * dx)) / (2 * h)
    assert abs(float(np.sum(xbar * dx)) - fd) < 1e-6 * abs(fd)


def ctx_of(s, z, cap=None):
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    sw = np.sqrt(np.diag(s.q))
    return dict(axes=axes, corr=s.q / np.outer(sw, sw), halfwidths=s.halfwidths(), z=z, m0=s.m0,
                p0_diag=s.p0_diag, cap=cap or s.cap, eps=s.eps, meas_kind=s.meas_kind), sw


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def replay_of(run):
    return {"ranks_pred": run["ranks_pred"], "ranks_filt": run["ranks_filt"]}


def test_adjoint_gradient_on_the_linear_gaussian_model():
    # every rank is one: the adjoint is the dense filter's exact gradient
    # (complex step) and, up to the grid, the Kalman gradient
    s = wl.spec_kf2d()
    x, z = wl.simulate(s, 12, np.random.SeedSequence(11))
    ctx, sw = ctx_of(s, z)
    th = np.concatenate([sw, [s.sigma_lin]])
    base = og.loglik_tt(th, ctx)
    ll, g = oa.loglik_grad_adjoint(th, ctx, replay_of(base))
    assert abs(ll - base["loglik"]) < 1e-12 * abs(ll)
    assert rel(g, og.grad_complex_step(og.loglik_dense_cs, th, ctx)) < 1e-12
    assert rel(g, og.grad_complex_step(og.loglik_kalman_cs, th, ctx)) < 1e-7


@pytest.fixture(scope="module")
def range2():
    s = wl.spec_range(2, 40, 40, lo=-10.0, hi=10.0, sigma_w=[1.0, 0.8])
    x, z = wl.simulate(s, 8, np.random.SeedSequence(5))
    ctx, sw = ctx_of(s, z)
    return ctx, np.concatenate([sw, [s.sigma_r, s.sigma_lin, s.sensor[0], s.sensor[1]]])


def test_adjoint_gradient_matches_dense_complex_step_when_the_cap_is_loose(range2):
    ctx, th = range2
    base = og.loglik_tt(th, ctx)
    ll, g = oa.loglik_grad_adjoint(th, ctx, replay_of(base))
    assert ll == base["loglik"] or abs(ll - base["loglik"]) < 1e-12 * abs(ll)
    assert rel(g, og.grad_complex_step(og.loglik_dense_cs, th, ctx)) < 1e-6
    assert g[3] == 0.0


def test_adjoint_gradient_matches_replay_differences_when_the_cap_binds(range2):
    ctx, th = range2
    c6 = dict(ctx, cap=6)
    ll, g_fd, base = og.grad_fd_tt(th, c6)
    _, g = oa.loglik_grad_adjoint(th, c6, replay_of(base))
    assert rel(g, g_fd) < 1e-5


def test_adjoint_gradient_d3_with_binding_cap():
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=5, d=3, n=32, cap=6)
    s, z = specs[0], zs[0]
    ctx, sw = ctx_of(s, z)
    th = np.concatenate([sw, [s.sigma_r, s.sigma_lin, s.sensor[0], s.sensor[1]]])
    ll, g_fd, base = og.grad_fd_tt(th, ctx)
    assert max(max(r) for r in base["ranks_filt"]) == 6
    _, g = oa.loglik_grad_adjoint(th, ctx, replay_of(base))
    assert rel(g, g_fd) < 1e-4
