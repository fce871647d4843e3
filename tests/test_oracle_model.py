"""Pins for the oracle's grid, kernel, likelihood and moments against closed
forms and dense evaluation (CPU only)."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import model as mdl
from oracle import tt as ttm


def test_grid_inclusive_linspace_and_cell_volume():
    axes = mdl.grid_axes(-20.0, 20.0, [128, 128])
    assert axes[0][0] == -20.0 and abs(axes[0][-1] - 20.0) < 1e-12
    dx = 40.0 / 127.0
    assert np.allclose(np.diff(axes[0]), dx)
    assert abs(mdl.cell_volume(axes) - dx * dx) < 1e-15


def test_prior_unit_mass_and_moments():
    axes = mdl.grid_axes(-10.0, 10.0, [64, 64, 64])
    p = mdl.prior_tt(axes, [0.5, -1.0, 0.0], [4.0, 2.0, 3.0])
    assert ttm.ranks(p) == [1, 1, 1, 1]
    mass, mean, cov = mdl.moments_tt(p, axes)
    assert abs(mass - 1.0) < 1e-14
    # the Riemann sum of a Gaussian with sigma/Delta >= 4 is spectrally accurate;
    # the box edge at >= 5 sigma truncates ~1e-6 of the mass
    assert np.allclose(mean, [0.5, -1.0, 0.0], atol=2e-5)
    assert np.allclose(cov, np.diag([4.0, 2.0, 3.0]), atol=5e-4)


def test_kernel_separable_closed_form():
    # diagonal Q: K(m) = prod_l N(Delta_l m_l; 0, q_l) Delta_l; the sum over
    # the box approximates prod_l erf(h_l Delta_l / sqrt(2 q_l)) spectrally
    q = np.diag([1.0, 0.5, 2.0])
    axes = mdl.grid_axes(-20.0, 20.0, [128, 128, 128])
    h = mdl.kernel_halfwidths(q, axes)
    dx = mdl.spacings(axes)
    k = mdl.kernel_dense(q, axes, h)
    for l in range(3):
        m = np.arange(-h[l], h[l] + 1) * dx[l]
        one = np.exp(-0.5 * m ** 2 / q[l, l]) / math.sqrt(2 * math.pi * q[l, l]) * dx[l]
        shp = [1, 1, 1]
        shp[l] = -1
        k = k / one.reshape(shp)
    assert np.allclose(k, 1.0, rtol=1e-12)
    ksum = mdl.kernel_dense(q, axes, h).sum()
    closed = np.prod([special.erf((h[l] + 0.5) * dx[l] / math.sqrt(2 * q[l, l])) for l in range(3)])
    assert abs(ksum - closed) < 5e-4
    ttk = mdl.kernel_tt(q, axes, h)
    assert ttm.ranks(ttk) == [1, 1, 1, 1]


def test_kernel_halfwidths_match_4sigma_box():
    q = np.eye(4)
    for n, expect in [(64, 6), (96, 9), (128, 12)]:
        axes = mdl.grid_axes(-20.0, 20.0, [n] * 4)
        assert mdl.kernel_halfwidths(q, axes) == [expect] * 4


def test_kernel_tt_reproduces_dense():
    q = np.array([[1.0, 0.3, 0.0], [0.3, 1.0, 0.3], [0.0, 0.3, 1.0]])
    axes = mdl.grid_axes(-20.0, 20.0, [128] * 3)
    h = mdl.kernel_halfwidths(q, axes)
    kd = mdl.kernel_dense(q, axes, h)
    kt = mdl.kernel_tt(q, axes, h, 1e-12)
    assert np.linalg.norm(ttm.full(kt) - kd) <= 1e-12 * np.linalg.norm(kd)
    assert max(ttm.ranks(kt)) <= 20


def test_range_likelihood_tt_matches_dense():
    axes = mdl.grid_axes(-20.0, 20.0, [64, 64, 64])
    meas = {"kind": "range", "sensor": (3.0, -2.0), "sigma_r": 0.5, "sigma_lin": 1.0}
    z = np.array([7.3, 1.5])
    lt = mdl.likelihood_tt(axes, z, meas, 1e-12)
    ld = mdl.likelihood_dense(axes, z, meas)
    assert np.linalg.norm(ttm.full(lt) - ld) <= 2e-12 * np.linalg.norm(ld)
    # closed form at one grid point
    i = (10, 40, 20)
    x = [axes[l][i[l]] for l in range(3)]
    r = math.hypot(x[0] - 3.0, x[1] + 2.0)
    expect = (math.exp(-0.5 * (7.3 - r) ** 2 / 0.25) / math.sqrt(2 * math.pi * 0.25)
              * math.exp(-0.5 * (1.5 - x[2]) ** 2) / math.sqrt(2 * math.pi))
    assert abs(ld[i] - expect) < 1e-15
    assert abs(ttm.element(lt, i) - expect) < 1e-12 * ld.max()


def test_linear_likelihood_rank_one():
    axes = mdl.grid_axes(-10.0, 10.0, [64, 64])
    meas = {"kind": "linear", "sigma_lin": 1.0}
    lt = mdl.likelihood_tt(axes, np.array([1.0, -2.0]), meas)
    assert ttm.ranks(lt) == [1, 1, 1]
    assert np.allclose(ttm.full(lt), mdl.likelihood_dense(axes, np.array([1.0, -2.0]), meas))


def test_moments_of_correlated_gaussian():
    axes = mdl.grid_axes(-12.0, 12.0, [48, 48, 48])
    c = np.array([[4.0, 1.2, 0.3], [1.2, 3.0, -0.8], [0.3, -0.8, 2.5]])
    mu = np.array([0.7, -0.4, 1.1])
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1) - mu
    dens = np.exp(-0.5 * np.einsum("...i,ij,...j->...", g, np.linalg.inv(c), g))
    p = ttm.tt_svd(dens, 1e-13)
    mass, mean, cov = mdl.moments_tt(p, axes)
    m2, mean2, cov2 = mdl.moments_dense(dens, axes)
    assert np.allclose(mean, mean2, atol=1e-12) and np.allclose(cov, cov2, atol=1e-11)
    assert np.allclose(mean, mu, atol=1e-5) and np.allclose(cov, c, atol=1e-3)


def test_prediction_gaussian_closure():
    # a Gaussian PMD convolved with a Gaussian kernel is the Gaussian with the
    # summed covariance (CKE for x_{k+1} = x_k + w_k), away from the boundary
    axes = mdl.grid_axes(-20.0, 20.0, [96, 96, 96])
    q = np.array([[1.0, 0.3, 0.0], [0.3, 1.0, 0.3], [0.0, 0.3, 1.0]])
    h = mdl.kernel_halfwidths(q, axes)
    p = mdl.prior_tt(axes, [1.0, -0.5, 0.3], [2.0, 3.0, 1.5])
    k = mdl.kernel_tt(q, axes, h)
    c = ttm.tt_round(ttm.conv(k, p, h), 1e-12)
    mass, mean, cov = mdl.moments_tt(c, axes)
    # 4-sigma box keeps ~0.9997 of the kernel mass at d=3
    assert 0.999 < mass < 1.0
    assert np.allclose(mean, [1.0, -0.5, 0.3], atol=1e-4)
    assert np.allclose(cov, np.diag([2.0, 3.0, 1.5]) + q, atol=2e-2)


def test_prediction_translation_equivariance():
    axes = mdl.grid_axes(-10.0, 10.0, [40, 40])
    q = np.array([[0.8, 0.2], [0.2, 0.6]])
    h = mdl.kernel_halfwidths(q, axes)
    k = mdl.kernel_tt(q, axes, h)
    p1 = mdl.prior_tt(axes, [0.0, 0.0], [1.0, 1.0])
    dx = mdl.spacings(axes)
    p2 = mdl.prior_tt(axes, [3 * dx[0], -2 * dx[1]], [1.0, 1.0])
    c1 = ttm.full(ttm.conv(k, p1, h))
    c2 = ttm.full(ttm.conv(k, p2, h))
    assert np.allclose(np.roll(np.roll(c1, 3, axis=0), -2, axis=1)[5:-5, 5:-5], c2[5:-5, 5:-5],
                       rtol=1e-10, atol=1e-14)


def test_kernel_at_equals_dense_kernel_entries():
    # the pointwise kernel (used at sizes where the dense box is too large)
    # is the dense kernel's entry at every sampled offset
    q = np.array([[1.0, 0.3, 0.0], [0.3, 0.7, 0.3], [0.0, 0.3, 1.2]])
    axes = mdl.grid_axes(-6.0, 6.0, [25, 25, 25])
    h = mdl.kernel_halfwidths(q, axes)
    kd = mdl.kernel_dense(q, axes, h)
    rng = np.random.default_rng(3)
    offs = np.stack([rng.integers(-hh, hh + 1, 40) for hh in h], axis=1)
    got = mdl.kernel_at(q, axes, offs)
    ref = np.array([kd[tuple(o + np.array(h))] for o in offs])
    assert np.allclose(got, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("d,n,rho", [(3, 40, 0.3), (4, 24, 0.3), (7, 12, 0.3), (5, 16, 0.15)])
def test_pairwise_kernel_equals_dense_tt_svd(d, n, rho):
    # the kernel built from its diagonal and pairwise Gaussian factors without
    # the dense tensor: same ranks as the TT-SVD of the dense kernel and the
    # same tensor to 1e-11 (a dropped factor, a wrong sign of the coupling
    # or a mis-scaled constant moves it far beyond that)
    axes = mdl.grid_axes([-6.0] * d, [6.0] * d, [n] * d)
    sw = 1.0 + 0.1 * np.arange(d)
    corr = np.eye(d) + rho * (np.eye(d, k=1) + np.eye(d, k=-1))
    q = sw[:, None] * corr * sw[None, :]
    h = mdl.kernel_halfwidths(q, axes)
    dense = mdl.kernel_tt(q, axes, h, 1e-12)
    pair, info = mdl.kernel_tt_pairwise(q, axes, h, 1e-12, return_info=True)
    assert len(info["pair_ranks"]) == d * (d - 1) // 2
    assert ttm.ranks(pair) == ttm.ranks(dense)
    assert ttm.rel_diff(pair, dense) < 1e-11
    # its sum against the dense kernel's entries, summed directly
    kd = mdl.kernel_dense(q, axes, h)
    assert abs(ttm.tt_sum(pair) - kd.sum()) < 1e-12 * kd.sum()
