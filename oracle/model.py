"""FP64 CPU oracle: grid, point-mass densities, transition kernel and
likelihood of the random-walk state-space model.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of points the paper leaves open:
  * grid: inclusive linspace per axis, spacing (hi-lo)/(N-1), cell volume
    the product of spacings (Sec. 2, eq. pdf_pm, and the grid bullet of
    Sec. 4 state an equidistant grid with points at cell centres);
  * kernel: p_w evaluated at offset m times the spacing, times the cell
    volume (the TPM element of Sec. 2.1, eq. TPMmat, for a translation
    invariant model), on the box |m_l| <= h_l, not renormalised;
  * likelihood: full Gaussian densities including their constants.
"""
from __future__ import annotations

import math

import numpy as np

from . import tt as ttm


def grid_axes(lo, hi, n):
    """Per-axis grid vectors xi^l (Sec. 4 grid bullet: N_1+..+N_d numbers)."""
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (len(n),))
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (len(n),))
    return [lo[l] + (hi[l] - lo[l]) * np.arange(n[l]) / (n[l] - 1) for l in range(len(n))]


def spacings(axes):
    return np.array([ax[1] - ax[0] for ax in axes])


def cell_volume(axes):
    """delta: volume of one grid cell (Sec. 2, eq. pdf_pm)."""
    return float(np.prod(spacings(axes)))


def gauss1(x, mean, var):
    return np.exp(-0.5 * (x - mean) ** 2 / var) / math.sqrt(2.0 * math.pi * var)


# ---------------------------------------------------------------------------
# prior
# ---------------------------------------------------------------------------

def prior_tt(axes, m0, p0_diag):
    """Initial PMD weights P_0(i) = p(x_0 = x^(i)) for a Gaussian prior with
    diagonal covariance: exactly rank one.  Normalised so that
    sum_i P(i) * delta = 1 (Sec. 2: the PMD integrates to one)."""
    cores = [gauss1(ax, m0[l], p0_diag[l]).reshape(1, -1, 1) for l, ax in enumerate(axes)]
    mass = ttm.tt_sum(cores) * cell_volume(axes)
    return ttm.scale(cores, 1.0 / mass)


# ---------------------------------------------------------------------------
# transition kernel (middle row of the TPM)
# ---------------------------------------------------------------------------

def kernel_halfwidths(q, axes, nsigma=4.0, truncate=True):
    """Per-axis box |m_l| <= h_l = floor(nsigma*sqrt(Q_ll)/Delta_l); without
    truncation h_l = N_l - 1 (every offset between two grid points)."""
    dx = spacings(axes)
    if not truncate:
        return [len(ax) - 1 for ax in axes]
    return [int(math.floor(nsigma * math.sqrt(q[l, l]) / dx[l] + 1e-12)) for l in range(len(axes))]


def kernel_dense(q, axes, halfwidths):
    """K(m) = N(Delta o m; 0, Q) * delta on the offset box (Sec. 2.1,
    eq. TPMmat with x_{k+1} = x_k + w_k: the TPM depends on i - j only and
    its middle row, eq. tpmconvFFT, is this tensor).  The quadratic form is
    accumulated from broadcast 1-D offset vectors, one dense array in all."""
    d = len(axes)
    dx = spacings(axes)
    ys = []
    for l in range(d):
        shp = [1] * d
        shp[l] = -1
        ys.append((dx[l] * np.arange(-halfwidths[l], halfwidths[l] + 1)).reshape(shp))
    qinv = np.linalg.inv(q)
    quad = np.zeros([2 * h + 1 for h in halfwidths])
    for l in range(d):
        for j in range(d):
            if qinv[l, j] != 0.0:
                quad += qinv[l, j] * (ys[l] * ys[j])
    norm = (2.0 * math.pi) ** (-d / 2.0) / math.sqrt(np.linalg.det(q))
    return norm * np.exp(-0.5 * quad) * cell_volume(axes)


def kernel_at(q, axes, offsets):
    """K(m) at integer offsets m (rows of ``offsets``): the transition density
    p_w(Delta o m) = N(Delta o m; 0, Q) times the cell volume (Sec. 2.1,
    eq. TPMmat with x_{k+1} = x_k + w_k), evaluated point by point."""
    offsets = np.atleast_2d(np.asarray(offsets, dtype=np.float64))
    d = len(axes)
    y = offsets * spacings(axes)[None, :]
    qinv = np.linalg.inv(q)
    quad = np.einsum("pi,ij,pj->p", y, qinv, y)
    norm = (2.0 * math.pi) ** (-d / 2.0) / math.sqrt(np.linalg.det(q))
    return norm * np.exp(-0.5 * quad) * cell_volume(axes)


def kernel_tt(q, axes, halfwidths, tol=1e-12):
    """TT transition kernel: TT-SVD of the dense offset kernel (Sec. 3.1)."""
    return ttm.tt_svd(kernel_dense(q, axes, halfwidths), tol)


def kernel_tt_pairwise(q, axes, halfwidths, tol=1e-12, factor_tol=1e-14, return_info=False):
    """TT transition kernel without the dense tensor (any d): the Gaussian
    of eq. TPMmat on the offset box factorises as

      K(m) = c * prod_l exp(-Lam_ll y_l^2 / 2) * prod_{l<j} exp(-Lam_lj y_l y_j),

    y = Delta o m, Lam = Q^{-1}, c = (2 pi)^{-d/2} |Q|^{-1/2} delta.  The
    diagonal factors form a rank-one TT; every pairwise factor is a 2-D
    function whose truncated SVD (relative Frobenius tolerance factor_tol)
    gives a TT that carries its rank through the axes between l and j with
    identity cores.  The factors are multiplied in by Hadamard products
    (Sec. 4.1 'times'), column j of Lam after column j-1, each product
    followed by a rounding at factor_tol (Sec. 4.1 'round'); a last rounding
    at tol gives the kernel TT (Sec. 3.1).  Within a column the partial
    quadratic form can be indefinite: for strongly coupled Q (a tridiagonal
    correlation of -0.45 with growing sigma_w, say) the partial products grow
    at the corners of the box and the rounding's absolute error, relative to
    them, leaves about 1e-9 of the kernel; the random-walk models here
    (correlation 0.3) stay at 2e-13."""
    d = len(axes)
    dx = spacings(axes)
    ys = [dx[l] * np.arange(-halfwidths[l], halfwidths[l] + 1) for l in range(d)]
    lam = np.linalg.inv(np.asarray(q, dtype=np.float64))
    acc = [np.exp(-0.5 * lam[l, l] * ys[l] ** 2).reshape(1, -1, 1) for l in range(d)]
    info = {"pair_ranks": {}, "acc_ranks": []}
    # column by column: once the pairs (l, j), l < j, are in, the product's
    # quadratic form is the leading j+1 block of Lam plus the remaining
    # diagonal terms, positive definite, so no partial product grows beyond
    # the diagonal factors at the corners of the box
    for j in range(1, d):
        for l in range(j):
            if lam[l, j] == 0.0:
                continue
            e = np.exp(-lam[l, j] * np.outer(ys[l], ys[j]))
            u, sv, vt = np.linalg.svd(e, full_matrices=False)
            r, _ = ttm.choose_rank(sv, factor_tol * float(np.linalg.norm(sv)), None)
            fac = []
            for k in range(d):
                t = len(ys[k])
                if k == l:
                    fac.append((u[:, :r] * sv[:r]).reshape(1, t, r))
                elif k == j:
                    fac.append(vt[:r].reshape(r, t, 1))
                elif l < k < j:
                    fac.append(np.repeat(np.eye(r)[:, None, :], t, axis=1))
                else:
                    fac.append(np.ones((1, t, 1)))
            info["pair_ranks"][(l, j)] = r
            acc = ttm.tt_round(ttm.hadamard(acc, fac), factor_tol)
            info["acc_ranks"].append(ttm.ranks(acc))
    c = (2.0 * math.pi) ** (-d / 2.0) / math.sqrt(np.linalg.det(q)) * cell_volume(axes)
    acc[0] = acc[0] * c
    out = ttm.tt_round(acc, tol)
    return (out, info) if return_info else out


def tpm_dense(q, axes):
    """Full transition tensor T(i_1..i_d, j_1..j_d) = p(x^(i) | x^(j)) * delta
    (Sec. 2.1, eq. TPMmat; Sec. 4 tensor bullet).  Tiny grids only."""
    d = len(axes)
    pts = np.stack([g.ravel() for g in np.meshgrid(*axes, indexing="ij")], axis=1)  # N x d
    diff = pts[:, None, :] - pts[None, :, :]
    qinv = np.linalg.inv(q)
    quad = np.einsum("abi,ij,abj->ab", diff, qinv, diff)
    norm = (2.0 * math.pi) ** (-d / 2.0) / math.sqrt(np.linalg.det(q))
    t = norm * np.exp(-0.5 * quad) * cell_volume(axes)
    shape = [len(ax) for ax in axes]
    return t.reshape(shape + shape)


# ---------------------------------------------------------------------------
# likelihood
# ---------------------------------------------------------------------------

def range_block(ax1, ax2, z_range, sensor, sigma_r):
    """M(i_1, i_2) = N(z_r; ||(xi_1, xi_2) - s||, sigma_r^2) on the grid of
    the first two axes (Sec. 2.2: the likelihood p(z|x) at every grid
    point)."""
    x1, x2 = np.meshgrid(ax1, ax2, indexing="ij")
    rng = np.sqrt((x1 - sensor[0]) ** 2 + (x2 - sensor[1]) ** 2)
    return gauss1(z_range, rng, sigma_r ** 2)


def likelihood_tt(axes, z, meas, lik_tol=1e-12, lik_max_rank=None):
    """Likelihood tensor L (Sec. 2.2, Sec. 4 tensor bullet) as a TT.

    meas = {"kind": "linear", "sigma_lin": s}: z_l = x_l + v_l on every axis;
    each axis factor is a 1-D Gaussian and L has rank one.
    meas = {"kind": "range", "sensor": (s1, s2), "sigma_r": sr,
            "sigma_lin": s}: z_0 = ||(x_1,x_2) - s|| + v_0 and z_j = x_{j+1} + v_j
    for the remaining axes.  The (x_1, x_2) block is a dense N_1 x N_2 matrix
    truncated by SVD at relative tolerance lik_tol; the other axes are rank
    one."""
    d = len(axes)
    if meas["kind"] == "linear":
        s2 = meas["sigma_lin"] ** 2
        return [gauss1(z[l], axes[l], s2).reshape(1, -1, 1) for l in range(d)]
    m = range_block(axes[0], axes[1], z[0], meas["sensor"], meas["sigma_r"])
    u, s, vt = np.linalg.svd(m, full_matrices=False)
    r, _ = ttm.choose_rank(s, lik_tol * float(np.linalg.norm(s)), lik_max_rank)
    cores = [(u[:, :r] * s[:r]).reshape(1, -1, r), vt[:r].reshape(r, -1, 1)]
    s2 = meas["sigma_lin"] ** 2
    for l in range(2, d):
        cores.append(gauss1(z[l - 1], axes[l], s2).reshape(1, -1, 1))
    return cores


def likelihood_dense(axes, z, meas):
    """The same likelihood evaluated at every grid point (dense, no SVD)."""
    d = len(axes)
    if meas["kind"] == "linear":
        out = np.ones([len(a) for a in axes])
        for l in range(d):
            shp = [1] * d
            shp[l] = -1
            out = out * gauss1(z[l], axes[l], meas["sigma_lin"] ** 2).reshape(shp)
        return out
    m = range_block(axes[0], axes[1], z[0], meas["sensor"], meas["sigma_r"])
    out = m.reshape(m.shape + (1,) * (d - 2))
    for l in range(2, d):
        shp = [1] * d
        shp[l] = -1
        out = out * gauss1(z[l - 1], axes[l], meas["sigma_lin"] ** 2).reshape(shp)
    return out


# ---------------------------------------------------------------------------
# moments
# ---------------------------------------------------------------------------

def moments_tt(p, axes):
    """Mass, mean and covariance of a PMD held as a TT: contractions of the
    cores with the per-axis vectors 1, xi^l and (xi^l)^2 (Sec. 4.1 'power',
    'dot'; the moments of Alg. 2).  Returns (mass, mean[d], cov[d,d]) where mass is
    sum_i P(i) delta and the moments are of the normalised density."""
    d = len(axes)
    delta = cell_volume(axes)
    ones = [np.ones(len(ax)) for ax in axes]
    mass = ttm.contract_vectors(p, ones) * delta
    mean = np.zeros(d)
    for l in range(d):
        v = list(ones)
        v[l] = axes[l]
        mean[l] = ttm.contract_vectors(p, v) * delta / mass
    second = np.zeros((d, d))
    for l in range(d):
        for j in range(l, d):
            v = list(ones)
            if l == j:
                v[l] = axes[l] ** 2
            else:
                v[l] = axes[l]
                v[j] = axes[j]
            second[l, j] = second[j, l] = ttm.contract_vectors(p, v) * delta / mass
    cov = second - np.outer(mean, mean)
    return mass, mean, cov


def moments_dense(p, axes):
    d = len(axes)
    delta = cell_volume(axes)
    grids = np.meshgrid(*axes, indexing="ij")
    mass = float(p.sum() * delta)
    mean = np.array([float((p * grids[l]).sum() * delta / mass) for l in range(d)])
    cov = np.zeros((d, d))
    for l in range(d):
        for j in range(d):
            cov[l, j] = float((p * grids[l] * grids[j]).sum() * delta / mass) - mean[l] * mean[j]
    return mass, mean, cov
