"""Pins for the oracle's TT toolkit against definitions, brute force and
library routines (CPU only)."""
import itertools
import math

import numpy as np
import pytest
from scipy import signal

from oracle import tt as ttm
from oracle import model as mdl


def rand_tt(rng, n, r, positive=False):
    d = len(n)
    rk = [1] + list(r) + [1]
    cores = []
    for k in range(d):
        g = rng.standard_normal((rk[k], n[k], rk[k + 1]))
        if positive:
            g = np.abs(g) + 0.1
        cores.append(g)
    return cores


def test_full_matches_elementwise_products():
    rng = np.random.default_rng(1)
    a = rand_tt(rng, [3, 4, 2, 5], [2, 3, 2])
    f = ttm.full(a)
    for idx in itertools.product(*[range(s) for s in f.shape]):
        # eq. ttd_exact written out: a product of matrices picked by the indices
        prod = np.eye(1)
        for g, i in zip(a, idx):
            prod = prod @ g[:, i, :]
        assert abs(f[idx] - prod[0, 0]) < 1e-12


def test_choose_rank_rule():
    s = np.array([4.0, 2.0, 1.0, 0.5])
    # tails: r=0 -> sqrt(21.25), r=1 -> sqrt(5.25), r=2 -> sqrt(1.25), r=3 -> 0.5, r=4 -> 0
    assert ttm.choose_rank(s, 0.5, None)[0] == 3          # tie 'tail <= delta' keeps 3
    assert ttm.choose_rank(s, 0.49, None)[0] == 4
    assert ttm.choose_rank(s, 100.0, None)[0] == 1        # never below one
    assert ttm.choose_rank(s, 0.0, 2)[0] == 2             # cap applied after tol
    assert ttm.choose_rank(s, math.sqrt(1.25), None)[0] == 2


def test_tt_svd_recovers_exact_low_rank():
    rng = np.random.default_rng(2)
    a = rand_tt(rng, [5, 6, 4, 5], [2, 3, 2])
    f = ttm.full(a)
    b = ttm.tt_svd(f, 1e-13)
    assert ttm.ranks(b) == [1, 2, 3, 2, 1]
    assert np.linalg.norm(ttm.full(b) - f) <= 1e-12 * np.linalg.norm(f)


def test_tt_svd_error_bound():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((6, 5, 6, 5))
    for eps in (0.5, 0.2, 0.05):
        b = ttm.tt_svd(f, eps)
        assert np.linalg.norm(ttm.full(b) - f) <= eps * np.linalg.norm(f) * (1 + 1e-12)


@pytest.mark.parametrize("cap", [None, 3, 1])
def test_round_equals_tt_svd_of_full(cap):
    # In exact arithmetic TT rounding (orthogonalise right-to-left, truncate
    # left-to-right with threshold eps*||A||/sqrt(d-1)) is the TT-SVD of the
    # dense tensor with the same threshold and cap.
    rng = np.random.default_rng(4)
    a = rand_tt(rng, [4, 5, 4, 5], [3, 5, 3], positive=True)
    b = ttm.add(a, ttm.scale(rand_tt(rng, [4, 5, 4, 5], [2, 2, 2], positive=True), 0.01))
    f = ttm.full(b)
    got = ttm.tt_round(b, 1e-3, cap)
    ref = ttm.tt_svd(f, 1e-3, cap)
    assert ttm.ranks(got) == ttm.ranks(ref)
    assert np.linalg.norm(ttm.full(got) - ttm.full(ref)) <= 1e-10 * np.linalg.norm(f)


def test_round_error_bound_and_idempotence():
    rng = np.random.default_rng(5)
    a = rand_tt(rng, [6, 6, 6, 6, 6], [4, 6, 6, 4])
    f = ttm.full(a)
    for eps in (1e-1, 1e-2):
        r = ttm.tt_round(a, eps)
        assert np.linalg.norm(ttm.full(r) - f) <= eps * np.linalg.norm(f) * (1 + 1e-10)
        r2 = ttm.tt_round(r, 1e-14)
        assert np.linalg.norm(ttm.full(r2) - ttm.full(r)) <= 1e-12 * np.linalg.norm(f)


def test_round_keeps_exact_rank_tensor():
    rng = np.random.default_rng(6)
    a = rand_tt(rng, [5, 4, 5, 4], [2, 3, 2])
    inflated = ttm.add(a, a)      # same tensor (2A) with doubled ranks
    r = ttm.tt_round(inflated, 1e-12)
    assert ttm.ranks(r) == [1, 2, 3, 2, 1]
    assert np.linalg.norm(ttm.full(r) - 2 * ttm.full(a)) <= 1e-13 * np.linalg.norm(ttm.full(a))


def test_hadamard_is_elementwise_and_ranks_multiply():
    rng = np.random.default_rng(7)
    a = rand_tt(rng, [3, 4, 5], [2, 3])
    b = rand_tt(rng, [3, 4, 5], [3, 2])
    h = ttm.hadamard(a, b)
    assert ttm.ranks(h) == [1, 6, 6, 1]
    assert np.allclose(ttm.full(h), ttm.full(a) * ttm.full(b), rtol=1e-13, atol=1e-13)


def test_sum_dot_norm():
    rng = np.random.default_rng(8)
    a = rand_tt(rng, [3, 4, 5, 2], [2, 3, 2])
    b = rand_tt(rng, [3, 4, 5, 2], [3, 2, 3])
    fa, fb = ttm.full(a), ttm.full(b)
    assert abs(ttm.tt_sum(a) - fa.sum()) < 1e-12 * np.abs(fa).sum()
    assert abs(ttm.tt_dot(a, b) - (fa * fb).sum()) < 1e-12 * np.abs(fa * fb).sum()
    assert abs(ttm.norm(a) - np.linalg.norm(fa)) < 1e-13 * np.linalg.norm(fa)
    v = [rng.standard_normal(s) for s in fa.shape]
    assert abs(ttm.contract_vectors(a, v) - np.einsum("ijkl,i,j,k,l->", fa, *v)) < 1e-11


def brute_conv(kfull, pfull, h):
    """d-dimensional direct sum over every offset; P is zero off the grid."""
    out = np.zeros_like(pfull)
    shape = pfull.shape
    for i in itertools.product(*[range(s) for s in shape]):
        acc = 0.0
        for m in itertools.product(*[range(-hh, hh + 1) for hh in h]):
            j = tuple(ii - mm for ii, mm in zip(i, m))
            if all(0 <= jj < s for jj, s in zip(j, shape)):
                acc += kfull[tuple(mm + hh for mm, hh in zip(m, h))] * pfull[j]
        out[i] = acc
    return out


@pytest.mark.parametrize("h", [[1, 2], [3, 0], [6, 6]])
def test_conv_matches_brute_force_2d(h):
    rng = np.random.default_rng(9)
    k = rand_tt(rng, [2 * h[0] + 1, 2 * h[1] + 1], [2])
    p = rand_tt(rng, [5, 6], [3])
    c = ttm.conv(k, p, h)
    assert ttm.ranks(c) == [1, 6, 1]
    assert np.allclose(ttm.full(c), brute_conv(ttm.full(k), ttm.full(p), h), rtol=1e-12, atol=1e-12)


def test_conv_matches_brute_force_3d_and_scipy():
    rng = np.random.default_rng(10)
    h = [1, 2, 1]
    k = rand_tt(rng, [3, 5, 3], [2, 2])
    p = rand_tt(rng, [4, 5, 4], [2, 3])
    got = ttm.full(ttm.conv(k, p, h))
    ref = brute_conv(ttm.full(k), ttm.full(p), h)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    # library routine: full linear convolution cropped at offset h
    full = signal.convolve(ttm.full(p), ttm.full(k), mode="full", method="direct")
    crop = full[tuple(slice(hh, hh + s) for hh, s in zip(h, got.shape))]
    assert np.allclose(got, crop, rtol=1e-12, atol=1e-12)


def test_alg1_einstein_summation_equals_convolution():
    # Alg. 1 contracts a 2d-core TT of the full transition tensor with the PMD
    # TT; for the random walk it must reproduce the convolution prediction.
    q = np.array([[0.6, 0.2, 0.0], [0.2, 0.5, 0.1], [0.0, 0.1, 0.7]])
    axes = mdl.grid_axes(-2.0, 2.0, [5, 6, 5])
    h = [4, 5, 4]           # untruncated: every grid offset
    t = mdl.tpm_dense(q, axes)
    t_tt = ttm.tt_svd(t, 1e-14)
    p = mdl.prior_tt(axes, [0.2, -0.1, 0.0], [0.8, 1.0, 0.6])
    p = ttm.add(p, ttm.scale(mdl.prior_tt(axes, [-0.5, 0.3, 0.2], [0.3, 0.4, 0.5]), 0.5))
    k_tt = ttm.tt_svd(mdl.kernel_dense(q, axes, h), 1e-14)
    via_alg1 = ttm.full(ttm.einsum_predict(t_tt, p))
    via_conv = ttm.full(ttm.conv(k_tt, p, h))
    dense = np.einsum("abcdef,def->abc", t, ttm.full(p))
    assert np.allclose(via_alg1, dense, rtol=1e-11, atol=1e-13)
    assert np.allclose(via_conv, dense, rtol=1e-11, atol=1e-13)


def test_storage_table1_bound():
    rng = np.random.default_rng(11)
    a = ttm.tt_round(rand_tt(rng, [7] * 5, [5, 9, 9, 5]), 1e-2, 6)
    npa, d = 7, 5
    assert ttm.storage(a) <= npa * d * max(ttm.ranks(a)) ** 2


def test_add_and_rel_diff():
    rng = np.random.default_rng(12)
    a = rand_tt(rng, [3, 4, 3], [2, 2])
    b = rand_tt(rng, [3, 4, 3], [3, 1])
    assert np.allclose(ttm.full(ttm.add(a, b)), ttm.full(a) + ttm.full(b))
    expect = np.linalg.norm(ttm.full(a) - ttm.full(b)) / np.linalg.norm(ttm.full(b))
    assert abs(ttm.rel_diff(a, b) - expect) < 1e-12 * expect


@pytest.mark.parametrize("keep", [(), (2,), (0, 3), (1, 2), (0, 1, 2, 3)])
def test_marginal_is_the_dense_sum_over_the_other_axes(keep):
    rng = np.random.default_rng(11)
    a = rand_tt(rng, [3, 4, 2, 5], [2, 3, 2])
    f = ttm.full(a)
    other = tuple(ax for ax in range(4) if ax not in keep)
    want = f.sum(axis=other) if other else f
    got = ttm.marginal(a, keep)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(f).sum())


def test_values_are_elements():
    rng = np.random.default_rng(12)
    a = rand_tt(rng, [3, 4, 2, 5], [2, 3, 2])
    f = ttm.full(a)
    idx = np.stack([rng.integers(0, s, 50) for s in f.shape], axis=1)
    assert np.allclose(ttm.values(a, idx), f[tuple(idx.T)], rtol=1e-13, atol=0)


def test_sample_probabilities_of_a_nonnegative_tt():
    # for A >= 0 the sequential conditionals multiply to A(i) / sum(A)
    rng = np.random.default_rng(13)
    a = rand_tt(rng, [3, 4, 2, 5], [2, 3, 2], positive=True)
    f = ttm.full(a)
    idx, q = ttm.sample(a, 400, np.random.default_rng(5))
    assert np.allclose(q, f[tuple(idx.T)] / f.sum(), rtol=1e-12, atol=0)


def test_sample_frequencies_and_negative_weights():
    # a 1-D train with a negative entry is never drawn there; the empirical
    # frequencies of a small 2-D tensor approach its probabilities
    a = [np.array([1.0, -0.5, 2.0]).reshape(1, 3, 1)]
    idx, q = ttm.sample(a, 2000, np.random.default_rng(1))
    assert not np.any(idx[:, 0] == 1)
    assert np.allclose(q[idx[:, 0] == 0], 1 / 3) and np.allclose(q[idx[:, 0] == 2], 2 / 3)
    rng = np.random.default_rng(14)
    b = rand_tt(rng, [3, 4], [2], positive=True)
    f = ttm.full(b)
    p = f / f.sum()
    idx, _ = ttm.sample(b, 200000, np.random.default_rng(2))
    freq = np.zeros_like(p)
    np.add.at(freq, (idx[:, 0], idx[:, 1]), 1.0)
    freq /= idx.shape[0]
    # binomial standard errors: every cell within 5 of them
    se = np.sqrt(p * (1 - p) / idx.shape[0])
    assert np.all(np.abs(freq - p) < 5 * se)
