"""FP64 CPU oracle: reverse-mode gradient of the TT filter's log marginal
likelihood LL = sum_k log c_k (Sec. 2.2, eq. pmf_filtrace_b) with respect to
the noise and sensor parameters, every rounding held at fixed ranks.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Each step of the recursion (Alg. 2 order, FFT-form prediction of Alg. 3 with
F = I) is re-run with a tape and then differentiated backwards:

  normalise and log c   P = X / (sum(X) delta),  LL += log(sum(L o P) delta)
  Hadamard              H_k = L_k (x) P_k slice by slice (Sec. 4.1 'times')
  convolution           C_k(ab,i,a'b') = sum_m K_k(a,m,a') P_k(b,i-m,b')
  rounding              the rounding of Sec. 4.1 'round' at fixed ranks
  likelihood            truncated SVD of the range block (Sec. 2.2)
  kernel                TT-SVD of the dense kernel (Sec. 3.1, eq. TPMmat)

Rounding at fixed ranks, written as a function of the input cores A_k only
(its value as a full tensor does not depend on the orthogonalisation used):

  Gram of the right part  G_d = 1,  G_{k-1} = sum_i A_k(:,i,:) G_k A_k(:,i,:)^T
  left-to-right           N_k = W_{k-1} x_1 A_k      ((r_{k-1} n_k) x R_k)
                          S_k = N_k G_k N_k^T,  U_k = leading r_k eigenvectors
                          of S_k (the left singular vectors of the unfolding),
                          output core k = U_k,  W_k = U_k^T N_k
  last core               W_{d-1} x_1 A_d.

The eigenpairs of S_k are read off the SVD of N_k F_k with F_k F_k^T = G_k
(F_k from Householder QR of the right part), which resolves singular values
far below sqrt(eps) of the largest.  The adjoint of the leading eigenvectors
keeps the couplings between kept and discarded directions (the discarded
singular values of a binding rank cap are not small); the couplings among
kept directions are dropped, which is exact because everything downstream
depends on the rounded tensor only, not on the basis of its cores.

Kept directions whose singular value is below TAU times the largest are left
out of the eigenvector adjoint.  Their terms are quotients of quantities that
carry rounding noise of order eps * sigma_1^2 by sigma_j^2, so they add noise
rather than signal; TAU = 6e-6 (about eps^(1/3)) balances that noise against
the dropped contribution, and the pins fix the resulting accuracy (1e-12 on
the linear-Gaussian model, 1e-6 against the dense complex step, 1e-4 against
replayed differences with a binding cap).

The kernel and the likelihood enter through their own truncated SVDs, which
are differentiated the same way; dK/dsigma and dM/dtheta are analytic.
"""
from __future__ import annotations

import math

import numpy as np

from . import model as mdl
from . import tt as ttm
from .grad import q_of, unpack


TAU = 6e-6

# ---------------------------------------------------------------------------
# leading-eigenvector adjoint of S = M M^T
# ---------------------------------------------------------------------------

def topvec_vjp(u_all, sig, r, ubar):
    """Adjoint Sbar of S = M M^T for its leading r eigenvectors U_r.

    ``u_all`` (p x q) and ``sig`` (q) are the thin SVD factors of M; the
    eigenvalues of S are sig^2 and zero on the complement of range(M).  For
    dU_j = sum_{i != j} u_i (u_i^T dS u_j) / (lam_j - lam_i) the adjoint is
    Sbar = sum_j x_j u_j^T with
      x_j = sum_{i discarded} u_i (u_i^T ubar_j) / (lam_j - lam_i)
            + (I - U U^T) ubar_j / lam_j.
    Couplings among kept vectors are omitted (see the module notes).  Only
    the symmetric part of Sbar is meaningful."""
    p = u_all.shape[0]
    lam = sig ** 2
    ur = u_all[:, :r]
    live = sig[:r] > TAU * sig[0]
    x = np.zeros((p, r))
    ud = u_all[:, r:]
    if ud.shape[1]:
        f = 1.0 / (lam[None, :r] - lam[r:, None])
        x += ud @ ((ud.T @ ubar) * f)
    x += (ubar - u_all @ (u_all.T @ ubar)) / lam[None, :r]
    x[:, ~live] = 0.0
    return x @ ur.T


# ---------------------------------------------------------------------------
# rounding at fixed ranks: forward with tape, adjoint
# ---------------------------------------------------------------------------

def round_fwd(a, ranks):
    """Rounding of the TT ``a`` to the ranks ``ranks`` (d+1 integers, each
    clamped to the available singular values), in the Gram form of the
    module notes.  Returns (cores, tape)."""
    d = len(a)
    a = [np.asarray(g, dtype=np.float64) for g in a]
    # right-part Grams and their square roots from the right-to-left QR sweep
    g = [None] * (d + 1)
    f = [None] * (d + 1)
    g[d - 1] = np.ones((1, 1))
    f[d - 1] = np.ones((1, 1))
    for k in range(d - 1, 0, -1):
        r0, n, r1 = a[k].shape
        gk = np.zeros((r0, r0))
        for i in range(n):
            gk += a[k][:, i, :] @ g[k] @ a[k][:, i, :].T
        g[k - 1] = gk
        # A_{>=k} = F_{k-1} (orthonormal rows): F from QR of the stacked blocks
        blk = np.concatenate([a[k][:, i, :] @ f[k] for i in range(n)], axis=1)
        _, rr = np.linalg.qr(blk.T, mode="reduced")
        f[k - 1] = rr.T
    out = []
    tape = {"a": a, "g": g, "n": [], "w": [np.ones((1, 1))], "u": [], "sig": [], "r": []}
    w = np.ones((1, 1))
    for k in range(d - 1):
        r0, n, r1 = a[k].shape
        nk = np.einsum("ac,cib->aib", w, a[k]).reshape(-1, r1)
        u, s, _ = np.linalg.svd(nk @ f[k], full_matrices=False)
        r = max(1, min(int(ranks[k + 1]), len(s)))
        uk = u[:, :r]
        w = uk.T @ nk
        out.append(uk.reshape(-1, n, r))
        tape["n"].append(nk)
        tape["u"].append(u)
        tape["sig"].append(s)
        tape["r"].append(r)
        tape["w"].append(w)
    out.append(np.einsum("ac,cib->aib", w, a[d - 1]))
    return out, tape


def round_vjp(tape, ybar):
    """Adjoint of round_fwd: output-core adjoints -> input-core adjoints."""
    a, g = tape["a"], tape["g"]
    d = len(a)
    abar = [np.zeros_like(x) for x in a]
    gbar = [np.zeros_like(x) if x is not None else None for x in g]
    # last core: Y_d = W_{d-1} x_1 A_d
    w = tape["w"][d - 1]
    wbar = np.einsum("aib,cib->ac", ybar[d - 1], a[d - 1])
    abar[d - 1] += np.einsum("ac,aib->cib", w, ybar[d - 1])
    for k in range(d - 2, -1, -1):
        r0, n, r1 = a[k].shape
        nk, u, s, r = tape["n"][k], tape["u"][k], tape["sig"][k], tape["r"][k]
        uk = u[:, :r]
        # W_k = U_k^T N_k
        nbar = uk @ wbar
        ubar = ybar[k].reshape(-1, r) + nk @ wbar.T
        # U_k = leading eigenvectors of S_k = N_k G_k N_k^T
        sbar = topvec_vjp(u, s, r, ubar)
        nbar += (sbar + sbar.T) @ nk @ g[k]
        gbar[k] += nk.T @ sbar @ nk
        # N_k = W_{k-1} x_1 A_k
        wprev = tape["w"][k]
        nb3 = nbar.reshape(wprev.shape[0], n, r1)
        wbar = np.einsum("aib,cib->ac", nb3, a[k])
        abar[k] += np.einsum("ac,aib->cib", wprev, nb3)
    # Gram recursion, G_{k-1} from A_k and G_k, taken back from the left
    for k in range(1, d):
        gb = gbar[k - 1] + gbar[k - 1].T
        for i in range(a[k].shape[1]):
            ai = a[k][:, i, :]
            abar[k][:, i, :] += gb @ ai @ g[k]
            gbar[k] += ai.T @ gbar[k - 1] @ ai
    return abar


# ---------------------------------------------------------------------------
# TT-SVD of a dense tensor: forward with tape, adjoint
# ---------------------------------------------------------------------------

def tt_svd_fwd(x, eps):
    """The TT-SVD of Sec. 3.1 (the same steps and rank rule as
    oracle.tt.tt_svd) with a tape."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    shape = x.shape
    delta = eps * np.linalg.norm(x.ravel()) / math.sqrt(max(d - 1, 1))
    tape = {"b": [], "u": [], "sig": [], "r": [], "shape": shape}
    cores = []
    rest = x.reshape(shape[0], -1)
    rp = 1
    for k in range(d - 1):
        rest = rest.reshape(rp * shape[k], -1)
        u, s, _ = np.linalg.svd(rest, full_matrices=False)
        r, _ = ttm.choose_rank(s, delta, None)
        tape["b"].append(rest)
        tape["u"].append(u)
        tape["sig"].append(s)
        tape["r"].append(r)
        cores.append(u[:, :r].reshape(rp, shape[k], r))
        rest = u[:, :r].T @ rest
        rp = r
    cores.append(rest.reshape(rp, shape[d - 1], 1))
    return cores, tape


def tt_svd_vjp(tape, ybar):
    """Adjoint of tt_svd_fwd: core adjoints -> dense-tensor adjoint.  Step k
    is B_{k+1} = U_k^T B_k (reshaped) with U_k the leading eigenvectors of
    B_k B_k^T."""
    shape = tape["shape"]
    d = len(shape)
    bbar_next = ybar[d - 1].reshape(tape["r"][-1], -1)
    for k in range(d - 2, -1, -1):
        b, u, s, r = tape["b"][k], tape["u"][k], tape["sig"][k], tape["r"][k]
        uk = u[:, :r]
        bn = bbar_next.reshape(r, -1)
        ubar = ybar[k].reshape(-1, r) + b @ bn.T
        bbar = uk @ bn
        sbar = topvec_vjp(u, s, r, ubar)
        bbar = bbar + (sbar + sbar.T) @ b
        bbar_next = bbar
    return np.asarray(bbar_next).reshape(shape)


# ---------------------------------------------------------------------------
# linear maps of the recursion and their adjoints
# ---------------------------------------------------------------------------

def sum_vjp(tt, sbar):
    """Adjoint of s = sum_i X(i) (Sec. 4.1 'sum'): core k receives
    sbar * left_k (x) ones (x) right_k."""
    d = len(tt)
    mats = [g.sum(axis=1) for g in tt]
    left = [np.ones((1,))]
    for k in range(d - 1):
        left.append(left[-1] @ mats[k])
    right = [None] * d
    acc = np.ones((1,))
    for k in range(d - 1, -1, -1):
        right[k] = acc
        acc = mats[k] @ acc
    return [sbar * np.einsum("a,i,b->aib", left[k], np.ones(tt[k].shape[1]), right[k]) for k in range(d)]


def weighted_sum_vjp(tt, weights, sbar):
    """Adjoint of s = sum_i w(i) X(i) for a rank-one weight
    w = w_0 (x) ... (x) w_{d-1} (a TT contraction with vectors, Sec. 4.1
    'dot'): core k receives sbar * left_k (x) w_k (x) right_k, with left and
    right the weighted prefix and suffix chains."""
    d = len(tt)
    mats = [np.einsum("i,aib->ab", w, g) for w, g in zip(weights, tt)]
    left = [np.ones((1,))]
    for k in range(d - 1):
        left.append(left[-1] @ mats[k])
    right = [None] * d
    acc = np.ones((1,))
    for k in range(d - 1, -1, -1):
        right[k] = acc
        acc = mats[k] @ acc
    return [sbar * np.einsum("a,i,b->aib", left[k], weights[k], right[k]) for k in range(d)]


def moments_vjp(tt, axes, mean_bar, cov_bar):
    """Adjoint with respect to the cores of the moments of a TT density
    (model.moments_tt: mean_l = M1_l / M0, cov_lj = M2_lj / M0 - mean_l
    mean_j, M_w = sum_i w(i) X(i); the cell volume cancels), given the
    adjoints of mean [d] and cov [d, d] (both entries of a symmetric pair
    count)."""
    d = len(tt)
    ones = [np.ones(len(ax)) for ax in axes]
    mean_bar = np.zeros(d) if mean_bar is None else np.asarray(mean_bar, dtype=np.float64)
    cov_bar = np.zeros((d, d)) if cov_bar is None else np.asarray(cov_bar, dtype=np.float64)

    def wvec(powers):
        return [np.asarray(axes[l], dtype=np.float64) ** powers.get(l, 0) if l in powers else ones[l]
                for l in range(d)]

    m0 = ttm.contract_vectors(tt, ones)
    m1 = np.array([ttm.contract_vectors(tt, wvec({l: 1})) for l in range(d)])
    mean = m1 / m0
    terms = []  # (weights, coefficient)
    mbar = mean_bar.copy()
    c0 = 0.0
    for l in range(d):
        for j in range(l, d):
            w = wvec({l: 2}) if l == j else wvec({l: 1, j: 1})
            m2 = ttm.contract_vectors(tt, w)
            cb = cov_bar[l, l] if l == j else cov_bar[l, j] + cov_bar[j, l]
            terms.append((w, cb / m0))
            c0 -= cb * m2 / m0 ** 2
            if l == j:
                mbar[l] -= 2.0 * cb * mean[l]
            else:
                mbar[l] -= cb * mean[j]
                mbar[j] -= cb * mean[l]
    for l in range(d):
        terms.append((wvec({l: 1}), mbar[l] / m0))
        c0 -= mbar[l] * mean[l] / m0
    terms.append((ones, c0))
    out = [np.zeros_like(g) for g in tt]
    for w, c in terms:
        tt_axpy(out, weighted_sum_vjp(tt, w, c))
    return out


def hadamard_vjp(a, b, hbar):
    """Adjoint of H_k((a,c), i, (b,d)) = A_k(a,i,b) B_k(c,i,d) (Sec. 4.1 'times')."""
    abar, bbar = [], []
    for ga, gb, hb in zip(a, b, hbar):
        ra0, n, ra1 = ga.shape
        rb0, _, rb1 = gb.shape
        h5 = hb.reshape(ra0, rb0, n, ra1, rb1)
        abar.append(np.einsum("acibd,cid->aib", h5, gb))
        bbar.append(np.einsum("acibd,aib->cid", h5, ga))
    return abar, bbar


def conv_vjp(kern, p, halfwidths, cbar):
    """Adjoint of the core-wise linear convolution of oracle.tt.conv:
    C_k((a,c), i, (b,d)) = sum_m K_k(a, m+h, b) P_k(c, i-m, d), P = 0 off the
    grid.  Returns (Kbar, Pbar)."""
    kbar, pbar = [], []
    for gk, gp, h, cb in zip(kern, p, halfwidths, cbar):
        rk0, taps, rk1 = gk.shape
        rp0, n, rp1 = gp.shape
        c5 = cb.reshape(rk0, rp0, n, rk1, rp1)
        kb = np.zeros_like(gk)
        pb = np.zeros_like(gp)
        for m in range(-h, h + 1):
            lo, hi = max(0, m), min(n, n + m)
            if hi <= lo:
                continue
            # output rows i in [lo, hi) read P rows i - m
            cs = c5[:, :, lo:hi, :, :]
            ps = gp[:, lo - m:hi - m, :]
            kb[:, m + h, :] += np.einsum("acibd,cid->ab", cs, ps)
            pb[:, lo - m:hi - m, :] += np.einsum("ab,acibd->cid", gk[:, m + h, :], cs)
        kbar.append(kb)
        pbar.append(pb)
    return kbar, pbar


def scale_vjp(x, c, ybar):
    """Adjoint of Y = c X applied to the first core: (Xbar, cbar)."""
    xbar = [yb.copy() for yb in ybar]
    xbar[0] = c * ybar[0]
    return xbar, float(np.sum(ybar[0] * x[0]))


def tt_axpy(dst, src, alpha=1.0):
    for k in range(len(dst)):
        dst[k] += alpha * src[k]


# ---------------------------------------------------------------------------
# analytic parameter derivatives of the kernel and the likelihood
# ---------------------------------------------------------------------------

def kernel_dsigma(q_sw, corr, axes, halfwidths):
    """dK/dsigma_j = K * q_j on the offset box, with
    q_j(y) = y_j (C^{-1} D^{-1} y)_j / sigma_j^2 - 1/sigma_j for
    Q = D C D (the derivative of the Gaussian in eq. TPMmat)."""
    sw = np.asarray(q_sw, dtype=np.float64)
    d = len(axes)
    kd = mdl.kernel_dense(q_of(sw, corr), axes, halfwidths)
    dx = mdl.spacings(axes)
    ys = []
    for l in range(d):
        shp = [1] * d
        shp[l] = -1
        ys.append((dx[l] * np.arange(-halfwidths[l], halfwidths[l] + 1)).reshape(shp))
    cinv = np.linalg.inv(np.asarray(corr, dtype=np.float64))
    out = []
    for j in range(d):
        cu = 0.0
        for l in range(d):
            if cinv[j, l] != 0.0:
                cu = cu + cinv[j, l] * ys[l] / sw[l]
        out.append(kd * (ys[j] * cu / sw[j] ** 2 - 1.0 / sw[j]))
    return kd, out


def _dgauss_dsigma(z, mean, sigma):
    """d/dsigma of N(z; mean, sigma^2)."""
    g = mdl.gauss1(z, mean, sigma ** 2)
    return g * ((z - mean) ** 2 / sigma ** 3 - 1.0 / sigma)


def range_block_grads(ax1, ax2, z_range, sensor, sigma_r):
    """M and dM/d(sigma_r, s1, s2) for M(i1,i2) = N(z; ||xi - s||, sigma_r^2)."""
    x1, x2 = np.meshgrid(ax1, ax2, indexing="ij")
    rng = np.sqrt((x1 - sensor[0]) ** 2 + (x2 - sensor[1]) ** 2)
    m = mdl.gauss1(z_range, rng, sigma_r ** 2)
    dm_dr = m * (z_range - rng) / sigma_r ** 2        # dM/d(range)
    with np.errstate(divide="ignore", invalid="ignore"):
        d1 = np.where(rng > 0, -(x1 - sensor[0]) / rng, 0.0)
        d2 = np.where(rng > 0, -(x2 - sensor[1]) / rng, 0.0)
    return m, _dgauss_dsigma(z_range, rng, sigma_r), dm_dr * d1, dm_dr * d2


# ---------------------------------------------------------------------------
# the whole filter
# ---------------------------------------------------------------------------

def _lik_fwd(axes, z, meas, lik_tol):
    """likelihood_tt with a tape (same truncation as oracle.model)."""
    d = len(axes)
    if meas["kind"] == "linear":
        return [mdl.gauss1(z[l], axes[l], meas["sigma_lin"] ** 2).reshape(1, -1, 1) for l in range(d)], None
    m = mdl.range_block(axes[0], axes[1], z[0], meas["sensor"], meas["sigma_r"])
    # right singular vectors as the leading eigenvectors of M^T M
    v, s, _ = np.linalg.svd(m.T, full_matrices=False)
    r, _ = ttm.choose_rank(s, lik_tol * float(np.linalg.norm(s)), None)
    vr = v[:, :r]
    cores = [(m @ vr).reshape(1, -1, r), vr.T.reshape(r, -1, 1)]
    for l in range(2, d):
        cores.append(mdl.gauss1(z[l - 1], axes[l], meas["sigma_lin"] ** 2).reshape(1, -1, 1))
    return cores, {"m": m, "v": v, "sig": s, "r": r}


def _lik_vjp(tape, lbar):
    """Adjoint of the range-block cores (M V_r, V_r^T) -> Mbar."""
    m, v, s, r = tape["m"], tape["v"], tape["sig"], tape["r"]
    vr = v[:, :r]
    c1b = lbar[0].reshape(-1, r)
    c2b = lbar[1].reshape(r, -1)
    mbar = c1b @ vr.T
    vbar = m.T @ c1b + c2b.T
    tbar = topvec_vjp(v, s, r, vbar)
    mbar += m @ (tbar + tbar.T)
    return mbar


def loglik_grad_adjoint(theta, ctx, replay):
    """LL and dLL/dtheta of the TT filter by reverse mode, ranks of every
    rounding fixed to ``replay`` = {"ranks_pred": [...], "ranks_filt": [...]}
    (as recorded by oracle.filters.run_tt_filter).  ctx as in
    oracle.grad.loglik_tt.  Returns (LL, gradient)."""
    theta = np.asarray(theta, dtype=np.float64)
    axes = ctx["axes"]
    d = len(axes)
    hw = ctx["halfwidths"]
    sw, meas = unpack(theta, d, ctx["meas_kind"])
    delta = mdl.cell_volume(axes)
    z = ctx["z"]
    lik_tol = ctx.get("lik_tol", 1e-12)
    kd, dk = kernel_dsigma(sw, ctx["corr"], axes, hw)
    kern, ktape = tt_svd_fwd(kd, ctx.get("kernel_tol", 1e-12))
    p = mdl.prior_tt(axes, ctx["m0"], ctx["p0_diag"])
    steps = []
    ll = 0.0
    for k in range(z.shape[0]):
        st = {}
        if k > 0:
            c = ttm.conv(kern, p, hw)
            pt, rtape = round_fwd(c, replay["ranks_pred"][k - 1])
            mpred = ttm.tt_sum(pt) * delta
            st.update(p_prev=p, pt=pt, rtape_pred=rtape, mpred=mpred)
            p = ttm.scale(pt, 1.0 / mpred)
        lik, ltape = _lik_fwd(axes, z[k], meas, lik_tol)
        h = ttm.hadamard(lik, p)
        ck = ttm.tt_sum(h) * delta
        ll += math.log(ck)
        hr, rtape = round_fwd(h, replay["ranks_filt"][k])
        mass = ttm.tt_sum(hr) * delta
        st.update(p_pred=p, lik=lik, ltape=ltape, h=h, ck=ck, hr=hr, rtape_filt=rtape, mass=mass)
        steps.append(st)
        p = ttm.scale(hr, 1.0 / mass)
    # reverse sweep
    kbar = [np.zeros_like(g) for g in kern]
    th_bar = np.zeros(len(theta))
    pbar = [np.zeros_like(g) for g in p]        # adjoint of the final filtering density: LL ignores it
    for k in range(z.shape[0] - 1, -1, -1):
        st = steps[k]
        # P = HR / mass, mass = sum(HR) delta
        hrbar, cbar_s = scale_vjp(st["hr"], 1.0 / st["mass"], pbar)
        mbar = -cbar_s / st["mass"] ** 2
        tt_axpy(hrbar, sum_vjp(st["hr"], mbar * delta))
        hbar = round_vjp(st["rtape_filt"], hrbar)
        # LL += log(sum(H) delta)
        tt_axpy(hbar, sum_vjp(st["h"], delta / st["ck"]))
        lbar, ppbar = hadamard_vjp(st["lik"], st["p_pred"], hbar)
        _lik_theta(th_bar, lbar, st, axes, z[k], meas, d)
        if k > 0:
            ptbar, cbar_s = scale_vjp(st["pt"], 1.0 / st["mpred"], ppbar)
            mbar = -cbar_s / st["mpred"] ** 2
            tt_axpy(ptbar, sum_vjp(st["pt"], mbar * delta))
            cbar = round_vjp(st["rtape_pred"], ptbar)
            kb, pbar = conv_vjp(kern, st["p_prev"], hw, cbar)
            tt_axpy(kbar, kb)
    kdbar = tt_svd_vjp(ktape, kbar)
    for j in range(d):
        th_bar[j] = float(np.sum(kdbar * dk[j]))
    return ll, th_bar


def _lik_theta(th_bar, lbar, st, axes, zk, meas, d):
    """Accumulate the measurement-parameter gradient of one step."""
    if meas["kind"] == "linear":
        for l in range(d):
            dl = _dgauss_dsigma(zk[l], axes[l], meas["sigma_lin"])
            th_bar[d] += float(np.sum(lbar[l].reshape(-1) * dl))
        return
    mbar = _lik_vjp(st["ltape"], lbar)
    _, dsr, ds1, ds2 = range_block_grads(axes[0], axes[1], zk[0], meas["sensor"], meas["sigma_r"])
    th_bar[d] += float(np.sum(mbar * dsr))
    th_bar[d + 2] += float(np.sum(mbar * ds1))
    th_bar[d + 3] += float(np.sum(mbar * ds2))
    for l in range(2, d):
        dl = _dgauss_dsigma(zk[l - 1], axes[l], meas["sigma_lin"])
        th_bar[d + 1] += float(np.sum(lbar[l].reshape(-1) * dl))
