"""Pins of the oracle's grid re-design and TT interpolation (Alg. 4, Sec.
4.2 interpolation) against closed forms and library routines."""
import numpy as np
import pytest

from oracle import model as mdl
from oracle import redesign as rd
from oracle import tt as ttm


def rand_tt(rng, n, r):
    rk = [1] + list(r) + [1]
    return [rng.standard_normal((rk[k], n[k], rk[k + 1])) for k in range(len(n))]


def test_box_identity_dynamics_is_the_sigma_box():
    # F = I: the predictive box itself, m +- nsigma sqrt(diag(P + Q))
    m = np.array([0.3, -1.0, 2.0])
    p = np.array([[1.0, 0.2, 0.0], [0.2, 0.5, 0.1], [0.0, 0.1, 2.0]])
    q = np.diag([0.1, 0.2, 0.3])
    lo, hi = rd.redesign_box(m, p, np.eye(3), q, 4.0)
    half = 4.0 * np.sqrt(np.diag(p + q))
    assert np.allclose(lo, m - half, rtol=0, atol=1e-14)
    assert np.allclose(hi, m + half, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_box_is_the_bounding_box_of_the_mapped_box(seed):
    # the bounding box of the linear image A (c + [-h, h]) is A c +- |A| h:
    # a closed form independent of the corner enumeration
    rng = np.random.default_rng(seed)
    d = 3
    f = rng.standard_normal((d, d)) + 2.0 * np.eye(d)
    a = rng.standard_normal((d, d))
    p = a @ a.T + 0.5 * np.eye(d)
    q = np.diag(rng.uniform(0.1, 0.5, d))
    m = rng.standard_normal(d)
    lo, hi = rd.redesign_box(m, p, f, q, 3.0)
    mp = f @ m
    pp = f @ p @ f.T + q
    h = 3.0 * np.sqrt(np.diag(pp))
    finv = np.linalg.inv(f)
    c = finv @ mp
    w = np.abs(finv) @ h
    assert np.allclose(lo, c - w, rtol=1e-12, atol=1e-12)
    assert np.allclose(hi, c + w, rtol=1e-12, atol=1e-12)


def test_paper_dynamics_box_contains_the_mapped_corners():
    # the 2-D model of the paper's experiment (Sec. 5): every mapped corner
    # lies in the box and each box face touches a corner
    f = np.array([[1.1, 0.1], [-0.2, 1.1]])
    m, p, q = np.array([20.0, 5.0]), np.diag([4.0, 1.0]), np.eye(2)
    lo, hi = rd.redesign_box(m, p, f, q, 3.0)
    mp, pp = f @ m, f @ p @ f.T + q
    h = 3.0 * np.sqrt(np.diag(pp))
    corners = np.array([[mp[0] + s0 * h[0], mp[1] + s1 * h[1]] for s0 in (-1, 1) for s1 in (-1, 1)])
    back = np.linalg.solve(f, corners.T).T
    assert np.all(back >= lo - 1e-12) and np.all(back <= hi + 1e-12)
    assert np.allclose(back.min(axis=0), lo) and np.allclose(back.max(axis=0), hi)


def test_interpolation_onto_the_same_grid_is_the_identity():
    rng = np.random.default_rng(4)
    axes = mdl.grid_axes(-2.0, 3.0, [7, 5, 6])
    g = rand_tt(rng, [7, 5, 6], [3, 4])
    out = rd.interpolate_tt(g, axes, axes)
    for a, b in zip(out, g):
        assert np.array_equal(a, b)


def test_interpolation_matches_numpy_interp_per_axis():
    # dense brute force: np.interp along every axis of the full tensor, zero
    # off the old grid; the new grid overlaps the old one and extends beyond
    rng = np.random.default_rng(5)
    n_old, n_new = [6, 5, 7], [9, 4, 8]
    old = mdl.grid_axes([-1.0, 0.0, -2.0], [2.0, 3.0, 1.0], n_old)
    new = mdl.grid_axes([-1.5, 0.4, -2.0], [1.7, 3.6, 0.5], n_new)
    g = rand_tt(rng, n_old, [3, 2])
    got = ttm.full(rd.interpolate_tt(g, old, new))
    want = ttm.full(g)
    for ax in range(3):
        want = np.apply_along_axis(lambda v: np.interp(new[ax], old[ax], v, left=0.0, right=0.0), ax, want)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_interpolation_is_exact_for_multilinear_functions():
    # f(x) = prod_l (a_l + b_l x_l) is linear along each axis: interpolating
    # its grid values onto any grid inside the old box reproduces f there
    a, b = np.array([1.0, -0.5, 2.0]), np.array([0.3, 1.2, -0.7])
    old = mdl.grid_axes(-1.0, 2.0, [5, 6, 4])
    new = mdl.grid_axes(-0.8, 1.9, [11, 7, 9])
    cores = [(a[l] + b[l] * ax)[None, :, None] for l, ax in enumerate(old)]
    got = ttm.full(rd.interpolate_tt(cores, old, new))
    want = np.einsum("i,j,k->ijk", *[a[l] + b[l] * ax for l, ax in enumerate(new)])
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
