"""Grid re-design and interpolation of a TT density onto a new grid (Sec.
4.2 'Interpolation in Tensor Train'; Alg. 3 and Alg. 4), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of points the paper leaves open:
  * predictive moments by the local (Kalman) prediction of the filtering
    moments, m' = F m, P' = F P F^T + Q (Alg. 4 names an extended or
    unscented Kalman filter; for linear F both reduce to this);
  * the predictive grid is the axis-aligned box m' +- nsigma sqrt(P'_ll)
    ("size based on P'" through a Chebyshev / sigma-ellipse bound: the
    number of standard deviations is a parameter);
  * the new filtering grid is the smallest axis-aligned box holding the
    2^d corners mapped by F^{-1}, with the old number of points per axis;
  * interpolation is multilinear on the axis-aligned grids (it acts core by
    core, as the paper's cited TT interpolation does), and the density is
    zero off the old grid.
"""
from __future__ import annotations

import itertools

import numpy as np


def predictive_moments(mean, cov, f, q):
    """Local Kalman prediction of the filtering moments."""
    f = np.asarray(f, dtype=np.float64)
    return f @ np.asarray(mean, dtype=np.float64), f @ np.asarray(cov, dtype=np.float64) @ f.T + np.asarray(q)


def redesign_box(mean, cov, f, q, nsigma):
    """Alg. 4: the predictive sigma box around m', its 2^d corners mapped to
    the filtering space by F^{-1}, and the smallest axis-aligned box holding
    them.  Returns (lo[d], hi[d])."""
    mp, pp = predictive_moments(mean, cov, f, q)
    half = nsigma * np.sqrt(np.diag(pp))
    d = len(mp)
    corners = np.array([mp + np.array(s) * half for s in itertools.product((-1.0, 1.0), repeat=d)])
    back = np.linalg.solve(np.asarray(f, dtype=np.float64), corners.T).T
    return back.min(axis=0), back.max(axis=0)


def interp_matrix(ax_old, ax_new):
    """Linear interpolation from the points ax_old to ax_new: W (N_new x
    N_old) with two weights per row inside [ax_old[0], ax_old[-1]] and a zero
    row outside it."""
    n0 = len(ax_old)
    w = np.zeros((len(ax_new), n0))
    step = (ax_old[-1] - ax_old[0]) / (n0 - 1)
    for i, x in enumerate(ax_new):
        if x < ax_old[0] or x > ax_old[-1]:
            continue
        j = min(int(np.floor((x - ax_old[0]) / step)), n0 - 2)
        t = (x - ax_old[j]) / (ax_old[j + 1] - ax_old[j])
        w[i, j] = 1.0 - t
        w[i, j + 1] = t
    return w


def interpolate_tt(cores, axes_old, axes_new):
    """Multilinear interpolation of a TT density onto a new axis-aligned
    grid: each core is contracted with its axis' interpolation matrix."""
    out = []
    for g, a0, a1 in zip(cores, axes_old, axes_new):
        out.append(np.einsum("ij,ajb->aib", interp_matrix(a0, a1), g))
    return out
