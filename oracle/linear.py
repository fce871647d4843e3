"""FP64 CPU oracle of the point-mass filter for linear dynamics
x_{k+1} = F x_k + w_k on re-designed grids (Alg. 3 with Alg. 4), in TT
format and densely.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One step, after the update on the current axis-aligned grid G_k (Alg. 2):

  re-design 1 (Alg. 4)  moments of P_{k|k}, their local Kalman prediction,
                        the predictive sigma box, its corners mapped by F^{-1},
                        the bounding box G^ (same N): interpolate P_{k|k} onto
                        it (multilinear, core by core for the TT);
  time update (Alg. 3)  on the lattice x(j) = F xi^(j) the predictive is the
                        convolution of the weights with
                        T(m) = N(F (Delta^ o m); 0, Q) delta^
                             = N(Delta^ o m; 0, F^{-1} Q F^{-T}) delta^ / |det F|
                        (the transition density depends on j - j' only), on the
                        per-axis box |m_l| <= floor(4 sqrt((F^{-1}QF^{-T})_ll)
                        / Delta^_l) (capped at N - 1), cropped to the lattice;
  re-design 2 (Alg. 3)  the bounding box G_{k+1} of the lattice's corners
                        F xi^(corner) (same N); the predictive is interpolated
                        onto it (multilinear in the lattice coordinates
                        u = (F diag Delta^)^{-1} (x - F lo^), zero where a
                        neighbour is off the lattice) and normalised.

Readings (the paper leaves them open): the local filter of Alg. 4 is the
Kalman prediction (exact for linear F); nsigma of the predictive box is a
parameter (4 by default); the interpolation of step 5 is multilinear in the
lattice coordinates.  The TT filter forms that interpolation densely (tiny
grids: it is the definition the device's cross approximation is held to)
and decomposes it by TT-SVD at the filter's tolerance and cap.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import signal

from . import model as mdl
from . import redesign as rd
from . import tt as ttm


def kernel_box(f, q, dx, n, nsigma=4.0):
    """Per-axis half-widths of the time-update kernel on a grid of spacings dx."""
    fi = np.linalg.inv(np.asarray(f, dtype=np.float64))
    qe = fi @ np.asarray(q, dtype=np.float64) @ fi.T
    return [int(min(n[l] - 1, math.floor(nsigma * math.sqrt(qe[l, l]) / dx[l]))) for l in range(len(dx))], qe


def lattice_box(f, lo, hi):
    """The bounding box of the 2^d corners F x of the box [lo, hi]."""
    d = len(lo)
    corners = np.array([[hi[l] if s[l] else lo[l] for l in range(d)] for s in itertools.product((0, 1), repeat=d)])
    img = corners @ np.asarray(f, dtype=np.float64).T
    return img.min(axis=0), img.max(axis=0)


def sheared_interp_dense(pt, lo_h, dx_h, f, axes_new):
    """Values on the grid axes_new of the weights pt given on the lattice
    x(j) = F (lo_h + dx_h o j): multilinear in u = (F diag dx_h)^{-1} (x - F lo_h)
    over the 2^d lattice neighbours, zero for a neighbour off the lattice."""
    f = np.asarray(f, dtype=np.float64)
    d = len(axes_new)
    shape = pt.shape
    a = np.linalg.inv(f @ np.diag(dx_h))
    pts = np.stack([g.ravel() for g in np.meshgrid(*axes_new, indexing="ij")], axis=1)
    u = (pts - f @ np.asarray(lo_h)) @ a.T
    j0 = np.floor(u).astype(np.int64)
    t = u - j0
    out = np.zeros(len(pts))
    for corner in itertools.product((0, 1), repeat=d):
        idx = j0 + np.array(corner)[None, :]
        w = np.ones(len(pts))
        for l in range(d):
            w = w * (t[:, l] if corner[l] else 1.0 - t[:, l])
        ok = np.all((idx >= 0) & (idx < np.array(shape)[None, :]), axis=1)
        out[ok] += w[ok] * pt[tuple(idx[ok].T)]
    return out.reshape([len(ax) for ax in axes_new])


def _time_update_kernel(f, q, axes_h, nsigma_kernel, kernel_tol):
    dx = mdl.spacings(axes_h)
    hw, qe = kernel_box(f, q, dx, [len(a) for a in axes_h], nsigma_kernel)
    scale = 1.0 / abs(float(np.linalg.det(np.asarray(f, dtype=np.float64))))
    return hw, qe, scale


def run_tt_filter_linear(f, q, meas, z, m0, p0_diag, lo0, hi0, n, cap, eps, nsigma=4.0, nsigma_kernel=4.0,
                         kernel_tol=1e-12, lik_tol=1e-12, record_density=False):
    """The TT filter of Alg. 3 (module notes).  Returns per-step records
    (log_c, log_mpred, mean, cov, grids, ranks) and the final density."""
    d = len(m0)
    axes = mdl.grid_axes(lo0, hi0, [n] * d)
    p = mdl.prior_tt(axes, m0, p0_diag)
    rec = {"log_c": [], "log_mpred": [], "mean": [], "cov": [], "grid_lo": [], "grid_hi": [], "ranks": [],
           "densities": [], "lattice": []}
    for k in range(z.shape[0]):
        if k > 0:
            _, mean, cov = mdl.moments_tt(p, axes)
            lo_h, hi_h = rd.redesign_box(mean, cov, f, q, nsigma)
            axes_h = mdl.grid_axes(lo_h, hi_h, [n] * d)
            ph = rd.interpolate_tt(p, axes, axes_h)
            hw, qe, scale = _time_update_kernel(f, q, axes_h, nsigma_kernel, kernel_tol)
            kern = ttm.scale(mdl.kernel_tt(qe, axes_h, hw, kernel_tol), scale)
            pt = ttm.tt_round(ttm.conv(kern, ph, hw), eps, cap)
            lo_n, hi_n = lattice_box(f, lo_h, hi_h)
            axes = mdl.grid_axes(lo_n, hi_n, [n] * d)
            dense = sheared_interp_dense(ttm.full(pt), lo_h, mdl.spacings(axes_h), f, axes)
            p = ttm.tt_svd(dense, eps, cap)
            mpred = ttm.tt_sum(p) * mdl.cell_volume(axes)
            rec["log_mpred"].append(math.log(mpred))
            rec["lattice"].append((lo_h, hi_h))
            p = ttm.scale(p, 1.0 / mpred)
        delta = mdl.cell_volume(axes)
        lik = mdl.likelihood_tt(axes, z[k], meas, lik_tol)
        h = ttm.hadamard(lik, p)
        ck = ttm.tt_sum(h) * delta
        if not (ck > 0.0) or not math.isfinite(ck):
            raise FloatingPointError(f"non-positive or non-finite c_k at step {k}: {ck}")
        rec["log_c"].append(math.log(ck))
        hr = ttm.tt_round(h, eps, cap)
        p = ttm.scale(hr, 1.0 / (ttm.tt_sum(hr) * delta))
        _, mean, cov = mdl.moments_tt(p, axes)
        rec["mean"].append(mean)
        rec["cov"].append(cov)
        rec["grid_lo"].append(np.array([a[0] for a in axes]))
        rec["grid_hi"].append(np.array([a[-1] for a in axes]))
        rec["ranks"].append(ttm.ranks(p))
        if record_density:
            rec["densities"].append(p)
    out = {key: (np.array(v) if key in ("log_c", "log_mpred", "mean", "cov", "grid_lo", "grid_hi") else v)
           for key, v in rec.items()}
    out["loglik"] = float(np.sum(out["log_c"]))
    out["final"] = p
    out["axes"] = axes
    return out


def run_dense_pmf_linear(f, q, meas, z, m0, p0_diag, lo0, hi0, n, nsigma=4.0, nsigma_kernel=4.0):
    """The same recursion on dense arrays, nothing truncated: the first
    interpolation as the per-axis interpolation matrices applied to every
    axis, the time update as a zero-padded FFT convolution with the dense
    kernel cropped to the lattice, the second interpolation as above."""
    d = len(m0)
    axes = mdl.grid_axes(lo0, hi0, [n] * d)
    grids = np.meshgrid(*axes, indexing="ij")
    p = np.ones([n] * d)
    for l in range(d):
        p = p * mdl.gauss1(grids[l], m0[l], p0_diag[l])
    p = p / (p.sum() * mdl.cell_volume(axes))
    rec = {"log_c": [], "log_mpred": [], "mean": [], "cov": [], "densities": []}
    for k in range(z.shape[0]):
        if k > 0:
            _, mean, cov = mdl.moments_dense(p, axes)
            lo_h, hi_h = rd.redesign_box(mean, cov, f, q, nsigma)
            axes_h = mdl.grid_axes(lo_h, hi_h, [n] * d)
            ph = p
            for l in range(d):
                w = rd.interp_matrix(axes[l], axes_h[l])
                ph = np.moveaxis(np.tensordot(w, np.moveaxis(ph, l, 0), axes=(1, 0)), 0, l)
            hw, qe, scale = _time_update_kernel(f, q, axes_h, nsigma_kernel, 1e-12)
            kd = mdl.kernel_dense(qe, axes_h, hw) * scale
            full = signal.fftconvolve(ph, kd, mode="full")
            pt = full[tuple(slice(hw[l], hw[l] + n) for l in range(d))]
            lo_n, hi_n = lattice_box(f, lo_h, hi_h)
            axes = mdl.grid_axes(lo_n, hi_n, [n] * d)
            p = sheared_interp_dense(pt, lo_h, mdl.spacings(axes_h), f, axes)
            mpred = p.sum() * mdl.cell_volume(axes)
            rec["log_mpred"].append(math.log(mpred))
            p = p / mpred
        delta = mdl.cell_volume(axes)
        lik = mdl.likelihood_dense(axes, z[k], meas)
        h = lik * p
        ck = h.sum() * delta
        rec["log_c"].append(math.log(ck))
        p = h / ck
        _, mean, cov = mdl.moments_dense(p, axes)
        rec["mean"].append(mean)
        rec["cov"].append(cov)
        rec["densities"].append(p.copy())
    out = {key: np.array(v) if key != "densities" else v for key, v in rec.items()}
    out["loglik"] = float(np.sum(out["log_c"]))
    return out


def run_kalman_linear(f, q, r, z, m0, p0):
    """Kalman filter for x_{k+1} = F x_k + w_k, z_k = x_k + v_k (update at
    k = 0, predict then update afterwards); log c_k = log N(z_k; m^-, P^- + R)."""
    f = np.asarray(f, dtype=np.float64)
    m = np.array(m0, dtype=np.float64)
    p = np.array(p0, dtype=np.float64)
    d = len(m)
    rec = {"log_c": [], "mean": [], "cov": []}
    for k in range(z.shape[0]):
        if k > 0:
            m = f @ m
            p = f @ p @ f.T + q
        s = p + r
        innov = z[k] - m
        sinv = np.linalg.inv(s)
        _, logdet = np.linalg.slogdet(s)
        rec["log_c"].append(-0.5 * (d * math.log(2 * math.pi) + logdet + innov @ sinv @ innov))
        gain = p @ sinv
        m = m + gain @ innov
        p = (np.eye(d) - gain) @ p
        p = 0.5 * (p + p.T)
        rec["mean"].append(m.copy())
        rec["cov"].append(p.copy())
    out = {key: np.array(v) for key, v in rec.items()}
    out["loglik"] = float(np.sum(out["log_c"]))
    return out
