"""GPU log-likelihood gradients (rank-replay central differences through
tt_filter_run) against the oracle's gradients."""
import numpy as np
import pytest

from oracle import grad as og
from oracle import model as mdl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import binding, grad, runner, workload
    assert torch.cuda.is_available()
    return binding, grad, runner, workload


def oracle_ctx(s, z):
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    sw = np.sqrt(np.diag(s.q))
    return dict(axes=axes, corr=s.q / np.outer(sw, sw), halfwidths=s.halfwidths(), z=z, m0=s.m0,
                p0_diag=s.p0_diag, cap=s.cap, eps=s.eps, meas_kind=s.meas_kind)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_replaying_recorded_ranks_reproduces_the_run(mods):
    B, G, runner, wl = mods
    import torch
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=5, d=3, n=32, cap=6)
    run, z = runner.run_filters(specs, zs, B.F64)
    kernels, kidx, kr = runner.build_kernels(specs, B.F64)
    again = B.FilterRun(runner.filter_specs(specs, kidx, kr, 64), kernels, 5, z.shape[2], B.F64)
    again(z, replay=(run.ranks_pred.clone(), run.ranks.clone()))
    torch.cuda.synchronize()
    assert np.array_equal(again.log_c.cpu().numpy(), run.log_c.cpu().numpy())
    assert np.array_equal(again.ranks.cpu().numpy(), run.ranks.cpu().numpy())
    assert np.array_equal(again.ranks_pred.cpu().numpy(), run.ranks_pred.cpu().numpy())
    # the predictive ranks are recorded: the prior is rank one, later ones bounded by the cap
    rp = run.ranks_pred.cpu().numpy()
    assert np.all(rp[:, 0] == 1) and rp.max() <= 6


def test_gradient_matches_oracle_replay_gradient(mods):
    # d = 3 range model with a binding cap: both sides differentiate the
    # computed log-likelihood with frozen ranks
    B, G, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=5, d=3, n=32, cap=6)
    s, z = specs[0], zs[0]
    ll, g, info = G.loglik_grad([s], [z])
    ctx = oracle_ctx(s, z)
    ll_o, g_o, base = og.grad_fd_tt(G.theta_of(s), ctx)
    assert abs(ll[0] - ll_o) < 1e-10 * abs(ll_o)
    assert rel(g[0], g_o) < 1e-6
    assert info["filters_perturbed"] == 2 * len(g_o)


def test_gradient_matches_dense_complex_step(mods):
    # d = 2 range model, cap not binding: the TT gradient is the dense
    # filter's exact gradient
    B, G, runner, wl = mods
    s = wl.spec_range(2, 40, 40, lo=-10.0, hi=10.0, sigma_w=[1.0, 0.8])
    x, z = wl.simulate(s, 8, np.random.SeedSequence(5))
    ll, g, _ = G.loglik_grad([s], [z])
    g_dense = og.grad_complex_step(og.loglik_dense_cs, G.theta_of(s), oracle_ctx(s, z))
    assert rel(g[0], g_dense) < 1e-6


def test_batched_gradient_equals_single_gradients(mods):
    B, G, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=3, steps=4, d=3, n=24, cap=5)
    ll, g, _ = G.loglik_grad(specs, zs)
    for b in range(3):
        l1, g1, _ = G.loglik_grad([specs[b]], [zs[b]])
        assert np.array_equal(g1[0], g[b]) and l1[0] == ll[b]


def test_autograd_wrapper(mods):
    B, G, runner, wl = mods
    import torch
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=4, d=3, n=24, cap=5)
    th0 = G.theta_of(specs[0])
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    w = torch.tensor([0.25, -1.5], dtype=torch.float64)
    # rank-replay differences behind the wrapper
    ll = G.TTFilterLogLik.apply(theta, specs, zs, method="differences")
    (ll * w).sum().backward()
    ll_ref, g_ref, _ = G.loglik_grad(specs, zs, np.tile(th0, (2, 1)))
    assert np.allclose(ll.detach().numpy(), ll_ref, rtol=0, atol=0)
    assert np.allclose(theta.grad.numpy(), 0.25 * g_ref[0] - 1.5 * g_ref[1], rtol=1e-12, atol=0)
    # the reverse sweep (default): same value as the composed adjoint, and
    # the same gradient as the differences to their accuracy
    from paper_2501_07942_amd import adjoint_grad as AG
    theta.grad = None
    ll = G.TTFilterLogLik.apply(theta, specs, zs)
    (ll * w).sum().backward()
    ll_a, g_a, _ = AG.loglik_grad_adjoint(specs, zs, np.tile(th0, (2, 1)))
    assert np.array_equal(ll.detach().numpy(), ll_a)
    # the backward seeds the reverse sweep with w (not a power of two: equal
    # up to the sweep's rounding noise)
    ga = 0.25 * g_a[0] - 1.5 * g_a[1]
    assert np.abs(theta.grad.numpy() - ga).max() <= 1e-6 * np.abs(ga).max()
    gw = 0.25 * g_ref[0] - 1.5 * g_ref[1]
    assert np.abs(theta.grad.numpy() - gw).max() < 1e-5 * np.abs(gw).max()
    with pytest.raises(ValueError):
        G.TTFilterLogLik.apply(theta, specs, zs, method="fd")
