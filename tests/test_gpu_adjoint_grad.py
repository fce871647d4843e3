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
    print("composed adjoint: 2 filters, d=3, N=32, cap 6, 5 steps", flush=True)
    ll, g, _ = AG.loglik_grad_adjoint(specs, zs)
    ll_fd, g_fd, _ = G.loglik_grad(specs, zs)
    # checkpoint segments of two steps, and a checkpoint per step without
    # the tape: the same computations, bit for bit; with the tape the
    # rounding adjoint takes the forward's singular vectors of the same
    # unfoldings, equal up to rounding (amplified by the small kept singular
    # values, well below this case's distance to the differences)
    ll2, g2, _ = AG.loglik_grad_adjoint(specs, zs, ckpt_every=2)
    ll1, g1, _ = AG.loglik_grad_adjoint(specs, zs, tape=False)
    assert np.array_equal(ll1, ll2) and np.array_equal(g1, g2)
    assert np.array_equal(ll1, ll)
    for b in range(2):
        print(f"  filter {b}: with vs without the tape {rel(g[b], g1[b]):.1e}", flush=True)
        assert rel(g[b], g1[b]) < 1e-6
    # the parameter tangents by forward instead of central differences
    _, g_f, _ = AG.loglik_grad_adjoint(specs, zs, scheme="forward")
    with pytest.raises(ValueError):
        AG.loglik_grad_adjoint(specs, zs, scheme="backward")
    for b in range(2):
        print(f"  filter {b}: forward vs central tangents {rel(g_f[b], g[b]):.1e}", flush=True)
        assert rel(g_f[b], g[b]) < 1e-5
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


def test_adjoint_gradient_linear_gaussian(mods):
    AG, G, wl = mods
    s = wl.spec_kf2d()
    x, z = wl.simulate(s, 12, np.random.SeedSequence(11))
    # tangents by central differences (O(h^2), h = 1e-5, the default)
    ll, g, _ = AG.loglik_grad_adjoint([s], [z])
    ctx, th = ctx_of(s, z), G.theta_of(s)
    g_dense = og.grad_complex_step(og.loglik_dense_cs, th, ctx)
    print(f"  linear Gaussian: vs dense {rel(g[0], g_dense):.1e}", flush=True)
    assert rel(g[0], g_dense) < 1e-8
    assert rel(g[0], og.grad_complex_step(og.loglik_kalman_cs, th, ctx)) < 1e-7
    # forward differences (O(h), h = 1e-7)
    _, g_f, _ = AG.loglik_grad_adjoint([s], [z], scheme="forward")
    print(f"  linear Gaussian, forward tangents: vs dense {rel(g_f[0], g_dense):.1e}", flush=True)
    assert rel(g_f[0], g_dense) < 1e-6


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
