"""The composed reverse-mode gradient on the GPU (adjoint_grad: forward
with checkpoints, reverse sweep through tt_*_adjoint) against the oracle's
reverse mode, replayed-rank central differences on the GPU, and the exact
gradients of the linear-Gaussian model."""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import grad as og
from oracle import model as mdl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import adjoint_grad, grad, workload
    assert torch.cuda.is_available()
    return adjoint_grad, grad, workload


def ctx_of(s, z):
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    sw = np.sqrt(np.diag(s.q))
    return dict(axes=axes, corr=s.q / np.outer(sw, sw), halfwidths=s.halfwidths(), z=z, m0=s.m0,
                p0_diag=s.p0_diag, cap=s.cap, eps=s.eps, meas_kind=s.meas_kind)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_adjoint_gradient_binding_cap_batch(mods):
    AG, G, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=5, d=3, n=32, cap=6)
    print("reverse sweep (tt_filter_run_adjoint): 2 filters, d=3, N=32, cap 6, 5 steps", flush=True)
    ll, g, _ = AG.loglik_grad_adjoint(specs, zs)
    ll_fd, g_fd, _ = G.loglik_grad(specs, zs)
    # checkpoint segments of two and of three steps recompute the same
    # steps: bit for bit the same; the tape (a checkpoint per step) hands the
    # rounding adjoint the forward's singular vectors of the same unfoldings,
    # equal up to rounding (amplified by the small kept singular values, well
    # below this case's distance to the differences)
    ll2, g2, _ = AG.loglik_grad_adjoint(specs, zs, ckpt_every=2)
    ll3, g3, _ = AG.loglik_grad_adjoint(specs, zs, ckpt_every=3)
    assert np.array_equal(ll2, ll3) and np.array_equal(g2, g3)
    assert np.array_equal(ll2, ll)
    for b in range(2):
        print(f"  filter {b}: tape vs checkpoints {rel(g[b], g2[b]):.1e}", flush=True)
        assert rel(g[b], g2[b]) < 1e-6
        ctx = ctx_of(specs[b], zs[b])
        base = og.loglik_tt(G.theta_of(specs[b]), ctx)
        # same log-likelihood as the oracle and the fused forward
        assert abs(ll[b] - base["loglik"]) < 1e-10 * abs(base["loglik"])
        assert abs(ll[b] - ll_fd[b]) < 1e-10 * abs(ll_fd[b])
        # the gradient: replayed differences on the GPU, the oracle's reverse mode
        _, g_or = oa.loglik_grad_adjoint(G.theta_of(specs[b]), ctx,
                                         {"ranks_pred": base["ranks_pred"], "ranks_filt": base["ranks_filt"]})
        print(f"  filter {b}: vs GPU differences {rel(g[b], g_fd[b]):.1e}, vs oracle {rel(g[b], g_or):.1e}",
              flush=True)
        assert rel(g[b], g_fd[b]) < 1e-5
        assert rel(g[b], g_or) < 1e-4


def test_autograd_wrapper_runs_the_reverse_sweep_in_backward(mods):
    # forward = the taped recursion only; backward = tt_filter_run_adjoint
    # seeded with the incoming gradient of LL
    import torch
    AG, G, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=4, d=3, n=24, cap=5)
    ll_ref, g_ref, _ = AG.loglik_grad_adjoint(specs, zs)
    # seeds that are powers of two scale every step exactly; others up to
    # the rounding noise of the reverse sweep
    for seed, tol in (([0.5, -2.0], 0.0), ([0.7, -1.3], 1e-6)):
        th = torch.tensor(np.stack([G.theta_of(s) for s in specs]), dtype=torch.float64, requires_grad=True)
        ll = G.TTFilterLogLik.apply(th, specs, zs)
        w = torch.tensor(seed, dtype=torch.float64)
        (ll * w).sum().backward()
        assert np.array_equal(ll.detach().numpy(), ll_ref)
        want = w.numpy()[:, None] * g_ref
        err = float(np.abs(th.grad.numpy() - want).max() / np.abs(want).max())
        print(f"  autograd seed {seed}: {err:.1e}", flush=True)
        assert err <= tol


def test_adjoint_gradient_linear_gaussian(mods):
    AG, G, wl = mods
    s = wl.spec_kf2d()
    x, z = wl.simulate(s, 12, np.random.SeedSequence(11))
    ll, g, _ = AG.loglik_grad_adjoint([s], [z])
    ctx, th = ctx_of(s, z), G.theta_of(s)
    g_dense = og.grad_complex_step(og.loglik_dense_cs, th, ctx)
    print(f"  linear Gaussian: vs dense {rel(g[0], g_dense):.1e}", flush=True)
    assert rel(g[0], g_dense) < 1e-8
    assert rel(g[0], og.grad_complex_step(og.loglik_kalman_cs, th, ctx)) < 1e-7


def test_adjoint_gradient_loose_cap_matches_dense_complex_step(mods):
    AG, G, wl = mods
    s = wl.spec_range(2, 40, 40, lo=-10.0, hi=10.0, sigma_w=[1.0, 0.8])
    x, z = wl.simulate(s, 8, np.random.SeedSequence(5))
    ll, g, _ = AG.loglik_grad_adjoint([s], [z])
    g_dense = og.grad_complex_step(og.loglik_dense_cs, G.theta_of(s), ctx_of(s, z))
    print(f"  loose cap: vs dense complex step {rel(g[0], g_dense):.1e}", flush=True)
    assert rel(g[0], g_dense) < 1e-5
    assert g[0][3] == 0.0


def test_adjoint_gradient_against_oracle_replay_differences_d4(mods):
    # an exact reference computed without the GPU: central differences of the
    # oracle's TT filter with every rounding's rank replayed from its base run
    # (d=4, N=32, binding cap 6, 8 steps); the GPU reverse sweep leaves kept
    # directions below 6e-6 sigma_1 of a bond out of the eigenvector adjoint
    AG, G, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=8, d=4, n=32, cap=6)
    print("composed adjoint vs oracle differences: 2 filters, d=4, N=32, cap 6, 8 steps", flush=True)
    ll, g, _ = AG.loglik_grad_adjoint(specs, zs)
    for b in range(2):
        ctx = ctx_of(specs[b], zs[b])
        ll_o, g_o, base = og.grad_fd_tt(G.theta_of(specs[b]), ctx)
        assert max(max(r) for r in base["ranks_filt"]) == 6
        err = rel(g[b], g_o)
        print(f"  filter {b}: |dLL|/|LL| {abs(ll[b] - ll_o) / abs(ll_o):.1e}, gradient vs oracle differences {err:.1e}",
              flush=True)
        assert abs(ll[b] - ll_o) < 1e-10 * abs(ll_o)
        assert err < 1e-4
