"""FP64 CPU oracle filters: the TT point-mass filter, a dense point-mass
filter and a Kalman filter for the random-walk model.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Step order (Alg. 2 with the FFT-form prediction of Alg. 3, fixed grid,
f = identity):
  k = 0 : update with z_0, round, normalise, moments;
  k >= 1: predict (convolution with the kernel), round, normalise
          (log m_pred records the mass that left the grid), update,
          c_k = sum(L o P_pred) * delta on the unrounded product,
          round, normalise, moments.
LL = sum_k log c_k (Sec. 2.2, eq. pmf_filtrace_b).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import signal

from . import model as mdl
from . import tt as ttm


def _marginal_min(p):
    """Minimum over all 1-D marginals of a TT (negativity monitor; the paper
    reports negative PMD values for d >= 3, Sec. 5.1, Sec. 6)."""
    d = len(p)
    mins = []
    for l in range(d):
        left = np.ones((1,))
        for k in range(l):
            left = left @ p[k].sum(axis=1)
        right = np.ones((1,))
        for k in range(d - 1, l, -1):
            right = p[k].sum(axis=1) @ right
        marg = np.einsum("a,aib,b->i", left, p[l], right)
        mins.append(float(marg.min()))
    return min(mins)


def _tail_rel(info):
    """The rounding's error bound relative to the input's norm: the square
    root of the sum over the bonds of the squared discarded tails, over
    ||A|| (the TT-SVD truncation bound, Sec. 3.2)."""
    return math.sqrt(sum(t * t for t in info["tails"])) / info["norm"] if info["norm"] > 0 else 0.0


def run_tt_filter(axes, q, halfwidths, meas, z, m0, p0_diag, cap, eps,
                  kernel_tol=1e-12, lik_tol=1e-12, lik_max_rank=None,
                  kernel=None, record_density=False, replay=None):
    """TT point-mass filter in FP64 (Alg. 2 loop order, Alg. 3's FFT
    prediction with F = I).  z has shape [K, b].  Returns a dict of per-step
    records and the final filtering TT.

    ``replay`` = {"ranks_pred": [...], "ranks_filt": [...]} (as recorded by a
    previous run) fixes the ranks of every rounding instead of the rank rule,
    so that a perturbed run follows the same rank pattern."""
    delta = mdl.cell_volume(axes)
    if kernel is None:
        kernel = mdl.kernel_tt(q, axes, halfwidths, kernel_tol)
    p = mdl.prior_tt(axes, m0, p0_diag)
    nsteps = z.shape[0]
    rec = {"log_c": [], "log_mpred": [], "mean": [], "cov": [], "ranks_pred": [],
           "ranks_filt": [], "ranks_unrounded": [], "marg_min": [], "tails": [], "tail_rel_pred": [],
           "tail_rel_filt": [],
           "densities": []}
    for k in range(nsteps):
        if k > 0:
            c = ttm.conv(kernel, p, halfwidths)
            rec["ranks_unrounded"].append(ttm.ranks(c))
            fr = None if replay is None else replay["ranks_pred"][k - 1]
            pt, info = ttm.tt_round(c, eps, cap, return_info=True, forced_ranks=fr)
            rec["tail_rel_pred"].append(_tail_rel(info))
            mpred = ttm.tt_sum(pt) * delta
            rec["log_mpred"].append(math.log(mpred))
            p = ttm.scale(pt, 1.0 / mpred)
            rec["ranks_pred"].append(ttm.ranks(p))
        lik = mdl.likelihood_tt(axes, z[k], meas, lik_tol, lik_max_rank)
        h = ttm.hadamard(lik, p)
        ck = ttm.tt_sum(h) * delta
        if not (ck > 0.0) or not math.isfinite(ck):
            raise FloatingPointError(f"non-positive or non-finite c_k at step {k}: {ck}")
        rec["log_c"].append(math.log(ck))
        fr = None if replay is None else replay["ranks_filt"][k]
        hr, info = ttm.tt_round(h, eps, cap, return_info=True, forced_ranks=fr)
        rec["tails"].append(info["tails"])
        rec["tail_rel_filt"].append(_tail_rel(info))
        mass = ttm.tt_sum(hr) * delta
        p = ttm.scale(hr, 1.0 / mass)
        rec["ranks_filt"].append(ttm.ranks(p))
        _, mean, cov = mdl.moments_tt(p, axes)
        rec["mean"].append(mean)
        rec["cov"].append(cov)
        rec["marg_min"].append(_marginal_min(p))
        if record_density:
            rec["densities"].append(p)
    out = {key: (np.array(v) if key in ("log_c", "log_mpred", "mean", "cov", "marg_min", "tail_rel_pred",
                                        "tail_rel_filt") else v)
           for key, v in rec.items()}
    out["loglik"] = float(np.sum(out["log_c"]))
    out["final"] = p
    out["kernel"] = kernel
    return out


def run_dense_pmf(axes, q, halfwidths, meas, z, m0, p0_diag, record_density=False):
    """Dense point-mass filter (Sec. 2, filter (ii) of Sec. 5): prediction
    by linear convolution with the dense kernel via zero-padded FFTs and a
    crop to the grid (eq. tpmconvFFT with P = 0 off the grid), Bayes update
    and normaliser (eqs. pmf_filtrace_a/b).  No rank truncation anywhere."""
    delta = mdl.cell_volume(axes)
    d = len(axes)
    kd = mdl.kernel_dense(q, axes, halfwidths)
    grids = np.meshgrid(*axes, indexing="ij")
    p = np.ones([len(a) for a in axes])
    for l in range(d):
        p = p * mdl.gauss1(grids[l], m0[l], p0_diag[l])
    p = p / (p.sum() * delta)
    rec = {"log_c": [], "log_mpred": [], "mean": [], "cov": [], "densities": []}
    for k in range(z.shape[0]):
        if k > 0:
            full = signal.fftconvolve(p, kd, mode="full")
            sl = tuple(slice(halfwidths[l], halfwidths[l] + len(axes[l])) for l in range(d))
            p = full[sl]
            mpred = p.sum() * delta
            rec["log_mpred"].append(math.log(mpred))
            p = p / mpred
        lik = mdl.likelihood_dense(axes, z[k], meas)
        h = lik * p
        ck = h.sum() * delta
        rec["log_c"].append(math.log(ck))
        p = h / ck
        _, mean, cov = mdl.moments_dense(p, axes)
        rec["mean"].append(mean)
        rec["cov"].append(cov)
        if record_density:
            rec["densities"].append(p.copy())
    out = {key: np.array(v) if key != "densities" else v for key, v in rec.items()}
    out["loglik"] = float(np.sum(out["log_c"]))
    out["final"] = p
    return out


def run_kalman(q, r, z, m0, p0):
    """Kalman filter for x_{k+1} = x_k + w_k, z_k = x_k + v_k (the linear
    Gaussian special case of eqs. asx/asz), same step order as the grid
    filters: update at k = 0, predict-then-update afterwards.
    log c_k = log N(z_k; m^-, P^- + R)."""
    m = np.array(m0, dtype=np.float64)
    p = np.array(p0, dtype=np.float64)
    d = len(m)
    rec = {"log_c": [], "mean": [], "cov": []}
    for k in range(z.shape[0]):
        if k > 0:
            p = p + q
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
