"""Naive FP64 tensor-train toolkit (CPU oracle).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library.

A TT is a plain Python list of 3-way NumPy arrays ``G[k]`` of shape
``(r_{k-1}, n_k, r_k)`` with ``r_0 = r_d = 1`` (Sec. 3.1, eq. ttd_exact).
Every routine is written for clarity, not speed: library primitives
(``numpy.linalg.qr``/``svd``, ``einsum``) serve as single steps and there is
no blocking or fusion beyond what the definitions state.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# basic shape helpers
# ---------------------------------------------------------------------------

def ranks(tt):
    """TT ranks [r_0, ..., r_d] (Sec. 3.1, eq. ttd_exact)."""
    return [tt[0].shape[0]] + [g.shape[2] for g in tt]


def modes(tt):
    return [g.shape[1] for g in tt]


def storage(tt):
    """Number of stored values of a TT (Table 1 counts N_pa*d*max(R)^2)."""
    return int(sum(g.size for g in tt))


def full(tt):
    """Dense tensor from a TT by contracting the rank indices in order
    (Sec. 3.1, eq. ttd_exact).  Only for tiny tensors."""
    out = tt[0].reshape(tt[0].shape[1], tt[0].shape[2])
    shape = [tt[0].shape[1]]
    for g in tt[1:]:
        r0, n, r1 = g.shape
        out = out.reshape(-1, r0) @ g.reshape(r0, n * r1)
        shape.append(n)
    return out.reshape(shape)


def element(tt, idx):
    """A(i_1..i_d) as the product of core slices (Sec. 3.1, eq. ttd_exact)."""
    v = np.ones((1,))
    for g, i in zip(tt, idx):
        v = v @ g[:, i, :]
    return float(v[0])


# ---------------------------------------------------------------------------
# rank rule shared by TT-SVD and rounding
# ---------------------------------------------------------------------------

def choose_rank(s, delta, cap):
    """Smallest r whose discarded tail sqrt(sum_{j>r} s_j^2) is <= delta,
    then clipped to [1, cap].

    The paper rounds to a required accuracy with a maximum rank (Sec. 3.2,
    Sec. 4.1 'round'); the tie 'tail <= delta' and r >= 1 are this oracle's
    reading of the truncation rule of the TT-SVD that Sec. 3.1 cites."""
    s = np.asarray(s, dtype=np.float64)
    # tail[r] = sqrt(sum_{j>=r} s_j^2) for r = 0..len(s)
    tail = np.sqrt(np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]]))
    r = len(s)
    for cand in range(0, len(s) + 1):
        if tail[cand] <= delta:
            r = cand
            break
    r = max(1, r)
    if cap is not None:
        r = min(int(cap), r)
    return r, float(tail[r]) if r <= len(s) else 0.0


# ---------------------------------------------------------------------------
# TT-SVD of a dense tensor and TT rounding
# ---------------------------------------------------------------------------

def tt_svd(a, eps, cap=None):
    """Sequential truncated SVDs of the unfoldings of a dense tensor: the TT
    decomposition of Sec. 3.1 (eq. ttd_exact) computed to relative accuracy
    eps, with per-bond threshold eps*||A||_F/sqrt(d-1) and optional rank cap
    (Sec. 3.2)."""
    a = np.asarray(a, dtype=np.float64)
    d = a.ndim
    shape = a.shape
    if d == 1:
        return [a.reshape(1, shape[0], 1).copy()]
    delta = eps * np.linalg.norm(a.ravel()) / math.sqrt(d - 1)
    cores = []
    r_prev = 1
    rest = a.reshape(shape[0], -1)
    for k in range(d - 1):
        rest = rest.reshape(r_prev * shape[k], -1)
        u, s, vt = np.linalg.svd(rest, full_matrices=False)
        r, _ = choose_rank(s, delta, cap)
        cores.append(u[:, :r].reshape(r_prev, shape[k], r))
        rest = s[:r, None] * vt[:r]
        r_prev = r
    cores.append(rest.reshape(r_prev, shape[d - 1], 1))
    return cores


def orthogonalize_rl(tt):
    """Right-to-left orthogonalisation: cores d..2 become right-orthogonal
    via Householder QR (numpy.linalg.qr) and each R factor is absorbed into
    the core on its left (first sweep of TT rounding, Sec. 4.1 'round')."""
    cores = [g.copy() for g in tt]
    d = len(cores)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = cores[k].shape
        m = cores[k].reshape(r0, n * r1)
        q, r = np.linalg.qr(m.T, mode="reduced")
        rn = q.shape[1]
        cores[k] = q.T.reshape(rn, n, r1)
        a0, an, _ = cores[k - 1].shape
        cores[k - 1] = (cores[k - 1].reshape(a0 * an, r0) @ r.T).reshape(a0, an, rn)
    return cores


def tt_round(tt, eps, cap=None, return_info=False, forced_ranks=None):
    """TT rounding (Sec. 4.1 'round'): right-to-left QR orthogonalisation,
    then a left-to-right sweep of truncated SVDs.  The threshold per bond is
    eps*||A||_F/sqrt(d-1); ||A||_F is read off the first core after the
    orthogonalisation.  Ranks are capped at ``cap`` (Sec. 3.2).

    ``forced_ranks`` (d+1 integers) replaces the rank rule by the given
    ranks, clamped to the available singular values (rank replay: the
    derivative of the rounding with its ranks held fixed)."""
    d = len(tt)
    cores = orthogonalize_rl(tt)
    nrm = float(np.linalg.norm(cores[0].ravel()))
    delta = eps * nrm / math.sqrt(max(d - 1, 1))
    info = {"norm": nrm, "delta": delta, "tails": [], "gaps": [], "svals": []}
    for k in range(d - 1):
        r0, n, r1 = cores[k].shape
        m = cores[k].reshape(r0 * n, r1)
        u, s, vt = np.linalg.svd(m, full_matrices=False)
        r, tail = choose_rank(s, delta, cap)
        if forced_ranks is not None:
            r = max(1, min(int(forced_ranks[k + 1]), len(s)))
            tail = float(np.sqrt(np.sum(s[r:] ** 2)))
        info["tails"].append(tail)
        info["svals"].append(s.copy())
        info["gaps"].append(float(s[r - 1] - s[r]) if r < len(s) else float(s[r - 1]))
        cores[k] = u[:, :r].reshape(r0, n, r)
        w = s[:r, None] * vt[:r]
        b0, bn, b1 = cores[k + 1].shape
        cores[k + 1] = (w @ cores[k + 1].reshape(b0, bn * b1)).reshape(r, bn, b1)
    info["ranks"] = ranks(cores)
    if return_info:
        return cores, info
    return cores


# ---------------------------------------------------------------------------
# elementwise algebra (Sec. 4.1: times, sum, dot, mrdivide)
# ---------------------------------------------------------------------------

def hadamard(a, b):
    """Elementwise product of two TTs: each core slice is the Kronecker
    product of the two slices, so ranks multiply (Sec. 4.1 'times')."""
    out = []
    for ga, gb in zip(a, b):
        ra0, n, ra1 = ga.shape
        rb0, nb, rb1 = gb.shape
        assert n == nb
        c = np.einsum("aib,cid->acibd", ga, gb)
        out.append(c.reshape(ra0 * rb0, n, ra1 * rb1))
    return out


def contract_vectors(tt, vecs):
    """sum_{i_1..i_d} A(i_1..i_d) * v_1(i_1) * ... * v_d(i_d) by a left-to-right
    product of the vector-contracted cores (used for sum, mass and moments,
    Sec. 4.1 'sum', 'power', 'dot')."""
    acc = np.ones((1,))
    for g, v in zip(tt, vecs):
        acc = acc @ np.einsum("aib,i->ab", g, v)
    return float(acc[0])


def tt_sum(tt):
    """Sum of all elements (Sec. 4.1 'sum')."""
    return contract_vectors(tt, [np.ones(g.shape[1]) for g in tt])


def tt_dot(a, b):
    """Inner product <A,B> by a left-to-right sweep of per-core contractions
    (Sec. 4.1 'dot')."""
    acc = np.ones((1, 1))
    for ga, gb in zip(a, b):
        acc = np.einsum("ac,aib,cid->bd", acc, ga, gb)
    return float(acc[0, 0])


def marginal(tt, keep):
    """Sum of a TT over every index whose axis is not in ``keep``: a dense
    array over the kept axes, in ascending axis order (the 'sum' of Sec. 4.1
    taken over some axes only).  Cores of summed axes are reduced to their
    slice sums; cores of kept axes keep their grid index."""
    keep = sorted(set(int(k) for k in keep))
    acc = np.ones((1, 1))                  # (kept multi-index, rank)
    shape = []
    for k, g in enumerate(tt):
        if k in keep:
            acc = np.einsum("ma,aib->mib", acc, g).reshape(-1, g.shape[2])
            shape.append(g.shape[1])
        else:
            acc = acc @ g.sum(axis=1)
    return acc.reshape(shape) if shape else float(acc[0, 0])


def values(tt, idx):
    """A(i) at the grid multi-indices in the rows of ``idx`` (count x d), as
    products of core slices (Sec. 3.1, eq. ttd_exact) taken for all rows at
    once."""
    idx = np.asarray(idx, dtype=np.int64)
    v = np.ones((idx.shape[0], 1))
    for k, g in enumerate(tt):
        v = np.einsum("sa,asb->sb", v, g[:, idx[:, k], :])
    return v[:, 0]


def sample(tt, count, rng):
    """Draw ``count`` grid multi-indices from the distribution proportional
    to A (negative conditional weights, which truncation can leave in a
    density, count as zero), one axis after the other from its conditional
    given the axes already drawn.  Returns (idx [count, d], q [count]) with q
    the probability with which each drawn index was chosen; for a
    non-negative A, q = A(i) / sum(A)."""
    d = len(tt)
    right = [None] * (d + 1)
    right[d] = np.ones((1,))
    for k in range(d - 1, -1, -1):
        right[k] = tt[k].sum(axis=1) @ right[k + 1]
    left = np.ones((count, 1))
    idx = np.zeros((count, d), dtype=np.int64)
    q = np.ones(count)
    for k, g in enumerate(tt):
        w = np.einsum("sa,aib,b->si", left, g, right[k + 1])
        w = np.maximum(w, 0.0)
        w = w / w.sum(axis=1, keepdims=True)
        cdf = np.cumsum(w, axis=1)
        u = rng.random(count)[:, None]
        pick = np.minimum((u > cdf).sum(axis=1), g.shape[1] - 1)
        idx[:, k] = pick
        q *= w[np.arange(count), pick]
        left = np.einsum("sa,asb->sb", left, g[:, pick, :])
    return idx, q


def scale(tt, c):
    """Multiply a TT by a scalar (Sec. 4.1 'mrdivide' divides)."""
    out = [g.copy() for g in tt]
    out[0] = out[0] * c
    return out


def add(a, b):
    """A + B as a TT with block-diagonal cores (rank r_a + r_b)."""
    d = len(a)
    out = []
    for k, (ga, gb) in enumerate(zip(a, b)):
        ra0, n, ra1 = ga.shape
        rb0, _, rb1 = gb.shape
        if d == 1:
            out.append(ga + gb)
        elif k == 0:
            out.append(np.concatenate([ga, gb], axis=2))
        elif k == d - 1:
            out.append(np.concatenate([ga, gb], axis=0))
        else:
            c = np.zeros((ra0 + rb0, n, ra1 + rb1))
            c[:ra0, :, :ra1] = ga
            c[ra0:, :, ra1:] = gb
            out.append(c)
    return out


def norm(tt):
    """Frobenius norm of a TT, read off the first core after right-to-left
    orthogonalisation (no cancellation, unlike sqrt(<A,A>))."""
    return float(np.linalg.norm(orthogonalize_rl(tt)[0].ravel()))


def rel_diff(a, b):
    """||A - B||_F / ||B||_F with A - B formed as a TT."""
    return norm(add(a, scale(b, -1.0))) / norm(b)


# ---------------------------------------------------------------------------
# convolution of a TT with a TT kernel (Sec. 2.1 Tensor Form, Sec. 4.2)
# ---------------------------------------------------------------------------

def conv(kern, p, halfwidths):
    """Linear convolution of a TT on an N_1 x .. x N_d grid with a TT kernel
    defined on offsets m_l in [-h_l, h_l], cropped back to the grid:

        C(i) = sum_m K(m) P(i - m),   P = 0 off the grid.

    Sec. 4.2 states that the cores of a TT convolution are the convolutions
    of the cores (computed there with FFTs); here each core is formed by the
    direct tap sum, so the oracle owes nothing to FFT round-off:

        C_k(ab, i, a'b') = sum_m K_k(a, m + h_k, a') P_k(b, i - m, b').
    """
    out = []
    for gk, gp, h in zip(kern, p, halfwidths):
        rk0, taps, rk1 = gk.shape
        rp0, n, rp1 = gp.shape
        assert taps == 2 * h + 1
        c = np.zeros((rk0, rp0, n, rk1, rp1))
        for m in range(-h, h + 1):
            shifted = np.zeros_like(gp)
            lo, hi = max(0, m), min(n, n + m)
            if hi > lo:
                shifted[:, lo:hi, :] = gp[:, lo - m:hi - m, :]
            c += np.einsum("ab,cid->acibd", gk[:, m + h, :], shifted)
        out.append(c.reshape(rk0 * rp0, n, rk1 * rp1))
    return out


# ---------------------------------------------------------------------------
# Alg. 1: Einstein summation of a 2d-core TPM TT with a d-core PMD TT
# ---------------------------------------------------------------------------

def einsum_predict(t_cores, p_cores):
    """Prediction P'(i_1..i_d) = sum_{j} T(i_1..i_d, j_1..j_d) P(j_1..j_d)
    with T held as a 2d-core TT and P as a d-core TT (Sec. 4.2, Einstein
    Summation, eqs. ttConvolutionP/Z/M and the backward Z recursion,
    Alg. 1).

    For each second-half core of T a 4-way tensor M_k contracts the shared
    grid index with the matching core of P; Z is built backwards from
    Z^{(2d)} = 1, and the result keeps the first d cores of T with Z
    absorbed into the d-th.  (The paper's loop back to the construction of M is read as looping
    over all d second-half cores.)"""
    d = len(p_cores)
    assert len(t_cores) == 2 * d
    z = np.ones((1, 1))
    for j in range(d - 1, -1, -1):
        tk = t_cores[d + j]           # (R_{d+j-1}, N_j, R_{d+j})
        pk = p_cores[j]               # (R'_{j-1}, N_j, R'_j)
        m = np.einsum("aib,cid->acbd", tk, pk)   # M(r_{k-1}, r'_{k-1}, r_k, r'_k)
        z = np.einsum("acbd,bd->ac", m, z)
    out = [g.copy() for g in t_cores[:d]]
    r0, n, r1 = out[d - 1].shape
    out[d - 1] = (out[d - 1].reshape(r0 * n, r1) @ z).reshape(r0, n, 1)
    return out
