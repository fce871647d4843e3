"""Deterministic TT-cross approximation, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3.3 builds TTs of functions that are only available point by point
(the transition kernel, the likelihood, the interpolated density of Alg. 3)
by cross approximation: a matrix is approximated from r of its rows and r of
its columns, A ~ C A_hat^{-1} R, quasi-optimally when the r x r intersection
A_hat has (close to) the largest volume |det A_hat|.  The paper uses a
randomised greedy cross; this oracle takes the rows and columns of largest
volume deterministically (maxvol), so that two runs agree:

  maxvol(A)   rows of a tall m x r matrix whose r x r submatrix has locally
              maximal volume: start from the pivot rows of Gaussian
              elimination with partial pivoting, then swap in row i for
              pivot j while |B_ij| > 1 + tol, B = A A_I^{-1} (a swap
              multiplies the volume by |B_ij|).
  tt_cross    alternating sweeps over the cores.  With left index sets
              I_{<k} (r_{k-1} tuples of axes 0..k-1) and right index sets
              J_{>k} (r_k tuples of axes k+1..d-1), core k's fibre matrix
              C_k(alpha i, beta) = f(I_{<k}[alpha], i, J_{>k}[beta]) is
              evaluated; in a left-to-right sweep maxvol on the QR factor Q
              of C_k picks the r_k rows that form I_{<k+1}; right-to-left the
              same on the transposed fibre matrices updates J and gives the
              cores Q Q[rows]^{-1} (= C C[rows]^{-1} for full-rank C:
              interpolation form, the TT reproduces f on the chosen cross).
              The ranks start at r0 and double (up to rmax) until two
              consecutive sweeps agree to tol and rounding the result at tol
              leaves every rank at least two below the one used (or the
              bond's full rank was used); the result is rounded at tol
              (Sec. 4.1 'round').
"""
from __future__ import annotations

import math

import numpy as np

from . import tt as ttm


def maxvol(a, tol=0.05, max_swaps=1000):
    """(rows, B): r row indices of the m x r matrix a (m >= r, full column
    rank) with |B| <= 1 + tol entrywise for B = a a[rows]^{-1}."""
    a = np.asarray(a, dtype=np.float64)
    m, r = a.shape
    if m < r:
        raise ValueError("maxvol needs at least as many rows as columns")
    # initial rows: Gaussian elimination with partial pivoting, column by column
    work = a.copy()
    rows = []
    free = np.ones(m, dtype=bool)
    for j in range(r):
        col = np.abs(work[:, j]) * free
        p = int(np.argmax(col))
        rows.append(p)
        free[p] = False
        if work[p, j] != 0.0:
            work -= np.outer(work[:, j] / work[p, j], work[p, :]) * free[:, None]
    rows = np.array(rows)
    b = a @ np.linalg.inv(a[rows])
    for _ in range(max_swaps):
        i, j = np.unravel_index(int(np.argmax(np.abs(b))), b.shape)
        if abs(b[i, j]) <= 1.0 + tol:
            break
        # replace pivot j by row i: B <- B - B[:, j] (B[i, :] - e_j) / B[i, j]
        bij = b[i, j]
        ej = np.zeros(r)
        ej[j] = 1.0
        b = b - np.outer(b[:, j], b[i, :] - ej) / bij
        rows[j] = i
    return rows, b


def _fibre(fun, left, n, right):
    """C(alpha, i, beta) = fun(left[alpha] + (i,) + right[beta])."""
    ra, rb = left.shape[0], right.shape[0]
    idx = np.zeros((ra, n, rb, left.shape[1] + 1 + right.shape[1]), dtype=np.int64)
    idx[:, :, :, :left.shape[1]] = left[:, None, None, :]
    idx[:, :, :, left.shape[1]] = np.arange(n)[None, :, None]
    idx[:, :, :, left.shape[1] + 1:] = right[None, None, :, :]
    return np.asarray(fun(idx.reshape(-1, idx.shape[-1])), dtype=np.float64).reshape(ra, n, rb)


def _clip_ranks(n, r):
    d = len(n)
    out = [1] * (d + 1)
    for k in range(1, d):
        out[k] = int(min(r, np.prod(n[:k]), np.prod(n[k:])))
    return out


def _initial_right_sets(n, ranks, seed):
    """J_{>k} for k = 0..d-2: ranks[k+1] distinct tuples of axes k+1..d-1,
    drawn from a seeded generator (the first tuple is the middle point)."""
    d = len(n)
    gen = np.random.Generator(np.random.PCG64(seed))
    sets = [None] * d
    sets[d - 1] = np.zeros((1, 0), dtype=np.int64)
    for k in range(d - 2, -1, -1):
        r = ranks[k + 1]
        tail = n[k + 1:]
        seen = {tuple(int(x) // 2 for x in tail)}
        rows = [tuple(int(x) // 2 for x in tail)]
        while len(rows) < r:
            t = tuple(int(gen.integers(0, m)) for m in tail)
            if t not in seen:
                seen.add(t)
                rows.append(t)
        sets[k] = np.array(rows, dtype=np.int64)
    return sets


def _extend_right_sets(n, sets, ranks, seed):
    d = len(n)
    gen = np.random.Generator(np.random.PCG64(seed))
    out = list(sets)
    for k in range(d - 2, -1, -1):
        r = ranks[k + 1]
        rows = [tuple(int(x) for x in row) for row in sets[k]]
        seen = set(rows)
        tail = n[k + 1:]
        while len(rows) < r:
            t = tuple(int(gen.integers(0, m)) for m in tail)
            if t not in seen:
                seen.add(t)
                rows.append(t)
        out[k] = np.array(rows, dtype=np.int64)
    return out


def _sweep(fun, n, ranks, right):
    """One left-to-right sweep then one right-to-left sweep.  Returns the TT
    of the right-to-left sweep (interpolation form, first core the fibre
    matrix) and the updated right index sets."""
    d = len(n)
    left = [None] * d
    left[0] = np.zeros((1, 0), dtype=np.int64)
    for k in range(d - 1):
        c = _fibre(fun, left[k], n[k], right[k])
        m = c.reshape(-1, c.shape[2])
        q, _ = np.linalg.qr(m)
        rows, _ = maxvol(q)
        a, i = rows // n[k], rows % n[k]
        left[k + 1] = np.concatenate([left[k][a], i[:, None]], axis=1)
    cores = [None] * d
    new_right = [None] * d
    new_right[d - 1] = np.zeros((1, 0), dtype=np.int64)
    for k in range(d - 1, 0, -1):
        c = _fibre(fun, left[k], n[k], new_right[k])
        m = c.reshape(c.shape[0], -1).T            # (n_k r_k) x r_{k-1}
        q, _ = np.linalg.qr(m)
        rows, b = maxvol(q)
        i, bb = rows // c.shape[2], rows % c.shape[2]
        new_right[k - 1] = np.concatenate([i[:, None], new_right[k][bb]], axis=1)
        # Q Q[rows]^{-1} equals C C[rows]^{-1} when C has full column rank
        # and stays defined (still reproducing C) when it has not
        cores[k] = (q @ np.linalg.inv(q[rows])).T.reshape(-1, n[k], c.shape[2])
    cores[0] = _fibre(fun, left[0], n[0], new_right[0])
    return cores, new_right


def tt_cross(fun, n, tol=1e-12, r0=4, rmax=64, max_sweeps=12, seed=0, return_info=False):
    """TT of the function fun(idx) (idx: [M, d] integer multi-indices ->
    values [M]) on the grid of mode sizes n, to relative accuracy tol."""
    n = [int(x) for x in n]
    d = len(n)
    if d == 1:
        out = [np.asarray(fun(np.arange(n[0])[:, None]), dtype=np.float64).reshape(1, n[0], 1)]
        return (out, {"ranks_used": [1, 1], "sweeps": 0}) if return_info else out
    r = r0
    ranks = _clip_ranks(n, r)
    right = _initial_right_sets(n, ranks, seed)
    prev = None
    sweeps = 0
    while True:
        cores, right = _sweep(fun, n, ranks, right)
        sweeps += 1
        done = prev is not None and ttm.rel_diff(cores, prev) <= tol
        prev = cores
        if done or sweeps >= max_sweeps:
            rounded = ttm.tt_round(cores, tol)
            slack = all(rr + 2 <= rk or rk == full for rr, rk, full in
                        zip(ttm.ranks(rounded)[1:-1], ranks[1:-1], _clip_ranks(n, 10 ** 9)[1:-1]))
            if slack or r >= rmax:
                info = {"ranks_used": ranks, "sweeps": sweeps}
                return (rounded, info) if return_info else rounded
            r = min(2 * r, rmax)
            ranks = _clip_ranks(n, r)
            right = _extend_right_sets(n, right, ranks, seed + sweeps)
            prev = None
            sweeps = 0


def kernel_tt_cross(q, axes, halfwidths, tol=1e-12, **kw):
    """The transition kernel TT of eq. TPMmat (the Gaussian on the offset box
    times the cell volume) by cross approximation from point values."""
    from . import model as mdl
    hw = np.asarray(halfwidths, dtype=np.int64)

    def fun(idx):
        return mdl.kernel_at(q, axes, idx - hw[None, :])

    return tt_cross(fun, [2 * h + 1 for h in halfwidths], tol, **kw)
