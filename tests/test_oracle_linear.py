"""Pins of the oracle's filter for linear dynamics on re-designed grids
(Alg. 3 with Alg. 4): the TT recursion against the same recursion on dense
arrays, both against the Kalman filter with the second-order convergence of
multilinear interpolation, and the geometric pieces against closed forms
(CPU only)."""
import numpy as np
import pytest

from oracle import linear as lin
from oracle import model as mdl
from oracle import tt as ttm

F_PAPER = np.array([[1.1, 0.1], [-0.2, 1.1]])   # the dynamics of the paper's 2-D experiment (Sec. 5)


def simulate(f, q, r, k, seed):
    rng = np.random.default_rng(seed)
    d = f.shape[0]
    x = np.zeros((k, d))
    x[0] = rng.normal(0.0, 2.0, d)
    for j in range(1, k):
        x[j] = f @ x[j - 1] + rng.multivariate_normal(np.zeros(d), q)
    z = x + rng.multivariate_normal(np.zeros(d), r, size=k)
    return x, z


def test_sheared_interpolation_reproduces_affine_functions():
    # multilinear interpolation in the lattice coordinates is exact for a
    # function affine in x (affine in u); points outside the lattice get zero
    f = F_PAPER
    lo, dx, n = np.array([-3.0, -2.0]), np.array([0.25, 0.2]), (24, 30)
    uu = np.meshgrid(*[np.arange(m) for m in n], indexing="ij")
    pts = np.stack([lo[l] + dx[l] * uu[l] for l in range(2)], axis=-1) @ f.T
    vals = 0.7 * pts[..., 0] - 1.3 * pts[..., 1] + 2.0
    axes_new = [np.linspace(-2.0, 1.0, 17), np.linspace(-1.0, 2.0, 13)]
    got = lin.sheared_interp_dense(vals, lo, dx, f, axes_new)
    g = np.meshgrid(*axes_new, indexing="ij")
    u = np.linalg.solve(f @ np.diag(dx), np.stack([g[0].ravel(), g[1].ravel()]) - (f @ lo)[:, None])
    inside = np.all((u >= 0) & (u <= np.array(n)[:, None] - 1), axis=0).reshape(g[0].shape)
    want = 0.7 * g[0] - 1.3 * g[1] + 2.0
    assert inside.sum() > 100
    assert np.abs(got[inside] - want[inside]).max() < 1e-12
    far = lin.sheared_interp_dense(vals, lo, dx, f, [np.array([50.0]), np.array([50.0])])
    assert far[0, 0] == 0.0


def test_lattice_box_and_kernel_box():
    lo, hi = np.array([-1.0, -2.0]), np.array([3.0, 1.0])
    blo, bhi = lin.lattice_box(np.eye(2), lo, hi)
    assert np.array_equal(blo, lo) and np.array_equal(bhi, hi)
    blo, bhi = lin.lattice_box(F_PAPER, lo, hi)
    # closed form of the bounding box of a linear image of a box
    c, h = (lo + hi) / 2, (hi - lo) / 2
    assert np.allclose(blo, F_PAPER @ c - np.abs(F_PAPER) @ h) and np.allclose(bhi, F_PAPER @ c + np.abs(F_PAPER) @ h)
    hw, qe = lin.kernel_box(np.eye(2), np.diag([1.0, 4.0]), np.array([0.5, 0.5]), [100, 100])
    assert hw == [8, 16] and np.allclose(qe, np.diag([1.0, 4.0]))


def test_tt_recursion_equals_the_dense_recursion():
    # loose cap: the TT filter is the dense filter up to its tolerances
    q, r = np.eye(2), np.eye(2)
    x, z = simulate(F_PAPER, q, r, 8, 1)
    meas = {"kind": "linear", "sigma_lin": 1.0}
    tt = lin.run_tt_filter_linear(F_PAPER, q, meas, z, np.zeros(2), np.full(2, 4.0), [-10, -10], [10, 10], 40, 40,
                                  1e-13)
    dn = lin.run_dense_pmf_linear(F_PAPER, q, meas, z, np.zeros(2), np.full(2, 4.0), [-10, -10], [10, 10], 40)
    assert np.abs(tt["log_c"] - dn["log_c"]).max() < 1e-8
    assert np.abs(tt["mean"] - dn["mean"]).max() < 1e-8
    assert np.abs(tt["log_mpred"] - dn["log_mpred"]).max() < 1e-8
    # the range model on the same dynamics (range block by truncated SVD)
    meas_r = {"kind": "range", "sensor": (3.0, -2.0), "sigma_r": 0.5, "sigma_lin": 1.0}
    zr = np.stack([np.hypot(x[:, 0] - 3.0, x[:, 1] + 2.0) + 0.5 * np.random.default_rng(2).standard_normal(8),
                   x[:, 1] + np.random.default_rng(3).standard_normal(8)], axis=1)
    tt = lin.run_tt_filter_linear(F_PAPER, q, meas_r, zr, np.zeros(2), np.full(2, 4.0), [-10, -10], [10, 10], 40, 40,
                                  1e-13)
    dn = lin.run_dense_pmf_linear(F_PAPER, q, meas_r, zr, np.zeros(2), np.full(2, 4.0), [-10, -10], [10, 10], 40)
    assert np.abs(tt["log_c"] - dn["log_c"]).max() < 1e-8


@pytest.mark.parametrize("f", [np.eye(2), F_PAPER], ids=["identity", "paper"])
def test_linear_gaussian_model_converges_to_the_kalman_filter(f):
    # the grids follow the density; the error is the multilinear
    # interpolation's, second order in the spacing
    q, r = np.eye(2), np.eye(2)
    x, z = simulate(f, q, r, 10, 4)
    meas = {"kind": "linear", "sigma_lin": 1.0}
    kf = lin.run_kalman_linear(f, q, r, z, np.zeros(2), 4.0 * np.eye(2))
    errs = []
    for n in (64, 128):
        tt = lin.run_tt_filter_linear(f, q, meas, z, np.zeros(2), np.full(2, 4.0), [-10, -10], [10, 10], n, n, 1e-12)
        errs.append(max(np.abs(tt["log_c"] - kf["log_c"]).max(), np.abs(tt["mean"] - kf["mean"]).max()))
        # the grid of every step holds the Kalman mean
        assert np.all(tt["grid_lo"] < kf["mean"]) and np.all(kf["mean"] < tt["grid_hi"])
    assert errs[0] < 0.03 and errs[1] < 0.008
    assert errs[0] / errs[1] > 2.5
