"""Pins of the oracle's deterministic TT-cross (maxvol pivots): maxvol's
local optimality by brute force, exact recovery of low-rank tensors, and the
transition kernel from point values against the dense TT-SVD, the pairwise
construction and direct evaluation (CPU only)."""
import itertools

import numpy as np
import pytest

from oracle import cross as cr
from oracle import model as mdl
from oracle import tt as ttm


def test_maxvol_is_locally_maximal_by_brute_force():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((12, 4)) * np.array([1.0, 0.1, 0.01, 1e-3])
    rows, b = cr.maxvol(a)
    assert len(set(rows.tolist())) == 4
    assert np.abs(b).max() <= 1.05 + 1e-12
    assert np.allclose(b, a @ np.linalg.inv(a[rows]), atol=1e-10)
    vol = abs(np.linalg.det(a[rows]))
    # no single swap of a chosen row for another row gains more than 1.05
    for j, i in itertools.product(range(4), range(12)):
        if i in rows:
            continue
        alt = rows.copy()
        alt[j] = i
        assert abs(np.linalg.det(a[alt])) <= 1.05 * vol * (1 + 1e-12)
    # on a small matrix it is within the local bound of the global maximum
    small = rng.standard_normal((7, 2))
    r2, _ = cr.maxvol(small)
    best = max(abs(np.linalg.det(small[list(c)])) for c in itertools.combinations(range(7), 2))
    assert abs(np.linalg.det(small[r2])) >= best / 1.05 ** 2


@pytest.mark.parametrize("ranks", [[2, 3, 2], [3, 7, 9, 4]])
def test_cross_recovers_a_low_rank_tensor(ranks):
    # ranks below and above the starting rank (the second doubles twice)
    rng = np.random.default_rng(len(ranks))
    n = [6, 9, 7, 8, 5][:len(ranks) + 1]
    rk = [1] + ranks + [1]
    a = [rng.standard_normal((rk[k], n[k], rk[k + 1])) for k in range(len(n))]
    full = ttm.full(a)
    c, info = cr.tt_cross(lambda idx: full[tuple(idx.T)], n, 1e-12, return_info=True)
    assert ttm.ranks(c) == rk
    assert np.linalg.norm(ttm.full(c) - full) <= 1e-12 * np.linalg.norm(full)


@pytest.mark.parametrize("d,n", [(3, 64), (4, 128), (6, 64)])
def test_cross_kernel_equals_dense_tt_svd(d, n):
    axes = mdl.grid_axes([-20.0] * d, [20.0] * d, [n] * d)
    q = np.eye(d) + 0.3 * (np.eye(d, k=1) + np.eye(d, k=-1))
    hw = mdl.kernel_halfwidths(q, axes)
    kc = cr.kernel_tt_cross(q, axes, hw, 1e-12)
    kd = mdl.kernel_tt(q, axes, hw, 1e-12)
    assert ttm.ranks(kc) == ttm.ranks(kd)
    assert ttm.rel_diff(kc, kd) <= 1e-11


def test_cross_kernel_at_d10_against_pairwise_factors_and_point_values():
    # no dense tensor at d = 10: two independent constructions and direct
    # evaluation of eq. TPMmat at scattered offsets
    d = 10
    axes = mdl.grid_axes([-25.0] * d, [25.0] * d, [64] * d)
    sw = 1.0 + 0.05 * np.arange(d)
    q = sw[:, None] * (np.eye(d) + 0.3 * (np.eye(d, k=1) + np.eye(d, k=-1))) * sw[None, :]
    hw = mdl.kernel_halfwidths(q, axes)
    kc = cr.kernel_tt_cross(q, axes, hw, 1e-12)
    kp = mdl.kernel_tt_pairwise(q, axes, hw, 1e-12)
    assert ttm.ranks(kc) == ttm.ranks(kp)
    assert ttm.rel_diff(kc, kp) <= 1e-11
    rng = np.random.default_rng(10)
    offs = np.stack([rng.integers(-h, h + 1, 400) for h in hw], axis=1)
    want = mdl.kernel_at(q, axes, offs)
    got = ttm.values(kc, offs + np.array(hw)[None, :])
    peak = float(mdl.kernel_at(q, axes, np.zeros((1, d)))[0])
    assert np.abs(got - want).max() <= 1e-11 * peak
