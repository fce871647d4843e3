"""FP64 CPU oracle: gradients of the log marginal likelihood
LL = sum_k log c_k (Sec. 2.2, eq. pmf_filtrace_b) with respect to the noise
and sensor parameters of the random-walk model.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Parameters theta, in this order:
  sigma_w[0..d-1]           process-noise standard deviations, Q = D C D with
                            D = diag(sigma_w) and a fixed correlation matrix C;
  sigma_r, sigma_lin, s1, s2  for the range measurement (sigma_r, the linear
                            measurements' sigma and the sensor position);
  sigma_lin                 for the all-linear measurement.

Three independent routes:
  * grad_fd_tt        central differences of the TT filter's LL with every
                      rounding's ranks replayed from the base run (the
                      derivative of the computed LL with its ranks frozen);
  * loglik_dense_cs   the dense point-mass filter written for complex
                      arithmetic, differentiated by the complex step
                      Im f(theta + i h e_j) / h (every operation of the dense
                      filter is analytic: exp, sqrt, sums, the linear
                      convolution, log), giving a machine-precision gradient;
  * loglik_kalman_cs  the Kalman filter for the linear-Gaussian case, also
                      complex-step differentiable.
The kernel box (the per-axis half widths) is held fixed at its base value:
it is a discretisation choice, not a function of theta.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import signal

from . import filters as flt
from . import model as mdl


def theta_names(d, meas_kind):
    names = [f"sigma_w{l}" for l in range(d)]
    if meas_kind == "range":
        return names + ["sigma_r", "sigma_lin", "s1", "s2"]
    return names + ["sigma_lin"]


def unpack(theta, d, meas_kind):
    """(sigma_w[d], meas dict) from theta (real or complex)."""
    theta = np.asarray(theta)
    sw = theta[:d]
    if meas_kind == "range":
        meas = {"kind": "range", "sigma_r": theta[d], "sigma_lin": theta[d + 1],
                "sensor": (theta[d + 2], theta[d + 3])}
    else:
        meas = {"kind": "linear", "sigma_lin": theta[d]}
    return sw, meas


def q_of(sigma_w, corr):
    """Q = diag(sigma_w) C diag(sigma_w)."""
    sw = np.asarray(sigma_w)
    return sw[:, None] * np.asarray(corr) * sw[None, :]


# ---------------------------------------------------------------------------
# TT filter: central differences with rank replay
# ---------------------------------------------------------------------------

def loglik_tt(theta, ctx, replay=None):
    """LL of the TT filter (oracle.filters.run_tt_filter) at theta; ctx holds
    axes, corr, halfwidths, z, m0, p0_diag, cap, eps, meas_kind and the
    kernel/likelihood tolerances."""
    d = len(ctx["axes"])
    sw, meas = unpack(np.asarray(theta, dtype=np.float64), d, ctx["meas_kind"])
    q = q_of(sw, ctx["corr"])
    return flt.run_tt_filter(ctx["axes"], q, ctx["halfwidths"], meas, ctx["z"], ctx["m0"],
                             ctx["p0_diag"], ctx["cap"], ctx["eps"], ctx.get("kernel_tol", 1e-12),
                             ctx.get("lik_tol", 1e-12), replay=replay)


def fd_steps(theta, h_rel):
    theta = np.asarray(theta, dtype=np.float64)
    return h_rel * np.maximum(1.0, np.abs(theta))


def grad_fd_tt(theta, ctx, h_rel=1e-5):
    """Central differences (h_j = h_rel * max(1, |theta_j|)) of the TT
    filter's LL, ranks of every rounding replayed from the run at theta.
    Returns (LL, gradient, base record)."""
    theta = np.asarray(theta, dtype=np.float64)
    base = loglik_tt(theta, ctx)
    replay = {"ranks_pred": base["ranks_pred"], "ranks_filt": base["ranks_filt"]}
    hs = fd_steps(theta, h_rel)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        tp = theta.copy()
        tm = theta.copy()
        tp[j] += hs[j]
        tm[j] -= hs[j]
        lp = loglik_tt(tp, ctx, replay)["loglik"]
        lm = loglik_tt(tm, ctx, replay)["loglik"]
        g[j] = (lp - lm) / (2.0 * hs[j])
    return base["loglik"], g, base


# ---------------------------------------------------------------------------
# dense point-mass filter in complex arithmetic (complex-step derivative)
# ---------------------------------------------------------------------------

def _cconv(a, b):
    """Full linear convolution of complex arrays as four real FFT
    convolutions of the parts, so that the rounding of the (large) real part
    never leaks into the (tiny) imaginary part the complex step reads."""
    ar, ai = np.real(a), np.imag(a)
    br, bi = np.real(b), np.imag(b)
    cv = lambda x, y: signal.fftconvolve(x, y, mode="full")
    return (cv(ar, br) - cv(ai, bi)) + 1j * (cv(ar, bi) + cv(ai, br))


def _gauss_c(x, mean, var):
    return np.exp(-0.5 * (x - mean) ** 2 / var) / np.sqrt(2.0 * np.pi * var)


def loglik_dense_cs(theta, ctx):
    """LL of the dense point-mass filter (the oracle's run_dense_pmf: linear
    convolution with the dense kernel on the offset box, crop, Bayes update,
    normaliser c_k = sum(L P) delta; Sec. 2, eqs. TPMmat, tpmconvFFT,
    pmf_filtrace_a/b) for a real or complex theta."""
    axes = ctx["axes"]
    d = len(axes)
    hw = ctx["halfwidths"]
    sw, meas = unpack(theta, d, ctx["meas_kind"])
    q = q_of(sw, ctx["corr"])
    delta = mdl.cell_volume(axes)
    dx = mdl.spacings(axes)
    # kernel K(m) = N(Delta o m; 0, Q) * delta on the box |m_l| <= h_l
    qinv = np.linalg.inv(q)
    quad = np.zeros([2 * h + 1 for h in hw], dtype=complex)
    ys = []
    for l in range(d):
        shp = [1] * d
        shp[l] = -1
        ys.append((dx[l] * np.arange(-hw[l], hw[l] + 1)).reshape(shp))
    for l in range(d):
        for j in range(d):
            quad = quad + qinv[l, j] * (ys[l] * ys[j])
    kd = (2.0 * np.pi) ** (-d / 2.0) / np.sqrt(np.linalg.det(q)) * np.exp(-0.5 * quad) * delta
    grids = np.meshgrid(*axes, indexing="ij")
    p = np.ones([len(a) for a in axes], dtype=complex)
    for l in range(d):
        p = p * _gauss_c(grids[l], ctx["m0"][l], ctx["p0_diag"][l])
    p = p / (p.sum() * delta)
    z = ctx["z"]
    ll = 0.0 + 0.0j
    for k in range(z.shape[0]):
        if k > 0:
            full = _cconv(p, kd)
            sl = tuple(slice(hw[l], hw[l] + len(axes[l])) for l in range(d))
            p = full[sl]
            p = p / (p.sum() * delta)
        if meas["kind"] == "linear":
            lik = np.ones_like(p)
            for l in range(d):
                lik = lik * _gauss_c(z[k][l], grids[l], meas["sigma_lin"] ** 2)
        else:
            s1, s2 = meas["sensor"]
            rng = np.sqrt((grids[0] - s1) ** 2 + (grids[1] - s2) ** 2)
            lik = _gauss_c(z[k][0], rng, meas["sigma_r"] ** 2)
            for l in range(2, d):
                lik = lik * _gauss_c(z[k][l - 1], grids[l], meas["sigma_lin"] ** 2)
        h = lik * p
        ck = h.sum() * delta
        ll = ll + np.log(ck)
        p = h / ck
    return ll


def loglik_kalman_cs(theta, ctx):
    """LL of the Kalman filter for z = x + v (the oracle's run_kalman, same
    step order), real or complex theta: log c_k = log N(z_k; m^-, P^- + R)."""
    d = len(ctx["m0"])
    sw, meas = unpack(theta, d, "linear")
    q = q_of(sw, ctx["corr"])
    r = np.eye(d) * meas["sigma_lin"] ** 2
    m = np.array(ctx["m0"], dtype=complex)
    p = np.diag(np.asarray(ctx["p0_diag"], dtype=float)).astype(complex)
    z = ctx["z"]
    ll = 0.0 + 0.0j
    for k in range(z.shape[0]):
        if k > 0:
            p = p + q
        s = p + r
        innov = z[k] - m
        sinv = np.linalg.inv(s)
        ll = ll - 0.5 * (d * math.log(2.0 * math.pi) + np.log(np.linalg.det(s)) + innov @ sinv @ innov)
        gain = p @ sinv
        m = m + gain @ innov
        p = (np.eye(d) - gain) @ p
        p = 0.5 * (p + p.T)
    return ll


def grad_complex_step(f, theta, ctx, h=1e-30):
    """d f / d theta_j = Im f(theta + i h e_j) / h for an analytic f."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        t = theta.astype(complex)
        t[j] += 1j * h
        g[j] = np.imag(f(t, ctx)) / h
    return g


def grad_fd(f, theta, ctx, h_rel=1e-5):
    """Central differences of a real function f(theta, ctx)."""
    theta = np.asarray(theta, dtype=np.float64)
    hs = fd_steps(theta, h_rel)
    g = np.zeros(len(theta))
    for j in range(len(theta)):
        tp = theta.copy()
        tm = theta.copy()
        tp[j] += hs[j]
        tm[j] -= hs[j]
        g[j] = (np.real(f(tp, ctx)) - np.real(f(tm, ctx))) / (2.0 * hs[j])
    return g
