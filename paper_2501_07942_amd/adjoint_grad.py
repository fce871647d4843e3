"""Reverse-mode gradient of the log marginal likelihood sum_k log c_k (Sec.
2.2, eq. pmf_filtrace_b) for a batch of FP64 filters, composed from the
library's forward and adjoint entry points.  Marshalling and sequencing
only: every arithmetic step runs in libttgbf.so.

Forward (Alg. 2 order, the prediction of Sec. 4.2 materialised):
  k = 0: P = normalise(prior)
  k >= 1: X = K (*) P;  Pt = round(X);  P_pred = normalise(Pt)
  every k: L_k = likelihood(z_k);  H = L_k o P_pred,  log c_k = log(sum(H) delta);
           HR = round(H);  P = normalise(HR)
Only the filtering densities P that start segments of ckpt_every steps
are kept (every one by default); the reverse sweep recomputes each segment
from its checkpoint, then each step of it, and runs the adjoints backwards
(tt_normalize_adjoint, tt_round_adjoint, tt_hadamard_adjoint,
tt_likelihood_adjoint, tt_predict_adjoint), collecting the adjoints of the
kernel train and of every likelihood train.

Parameters enter through the kernel TT (sigma_w) and the likelihood TTs
(sigma_r, sigma_lin, sensor).  The likelihood adjoints are carried through
the range block's truncated SVD (tt_likelihood_adjoint) onto the dense
likelihood P_k, whose parameter tangent is smooth; the kernel contribution
<Kbar, dK/dtheta> uses the tangent of the kernel's TT-SVD as the central
difference of the builds at theta +- h aligned to the base build's bond
bases (tt_align_signs).  Both tangents are central differences (or, optionally,
forward differences from the base builds) of dense-in-theta quantities; the
recursion itself is differentiated exactly.
Ranks of every rounding are those of the forward run (the same
deterministic calls reproduce them).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import binding as B
from . import grad as G
from . import runner


def _like(ts: Sequence[B.DeviceTT]) -> List[B.DeviceTT]:
    """Trains of the layouts of ts (one allocation for the batch)."""
    return B.DeviceTT.batch([t.n for t in ts], [t.cap for t in ts], ts[0].dtype)


def _zero_adj(ts: Sequence[B.DeviceTT]) -> List[B.DeviceTT]:
    """Adjoint trains of ts's layouts holding zeros, with ts's ranks."""
    zs = _like(ts)
    for z, t in zip(zs, ts):
        z.ranks.copy_(t.ranks)
    return zs


def _new(ns: Sequence[Sequence[int]], caps: Sequence[Sequence[int]]) -> List[B.DeviceTT]:
    return B.DeviceTT.batch(ns, caps, B.F64)


def _prod_caps(a: B.DeviceTT, b: B.DeviceTT) -> List[int]:
    return [x * y for x, y in zip(a.cap, b.cap)]


def _lik_caps(spec, lik_rank_cap: int) -> List[int]:
    caps = [1] * (spec.d + 1)
    if spec.meas_kind == "range":
        caps[1] = min(lik_rank_cap, spec.n)
    return caps


class _Step:
    pass


class ComposedGradient:
    """Forward run with checkpoints and the reverse sweep for one batch."""

    def __init__(self, specs: Sequence, zs: Sequence[np.ndarray], lik_rank_cap: int = 64, ckpt_every: int = 1,
                 tape: bool = True):
        import torch
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        self.C = int(ckpt_every)
        # with a checkpoint per step the forward also keeps each step's
        # rounded and normalised predictive, likelihood and update product
        # (a few MB per filter and step), so the reverse sweep recomputes only
        # the prediction product, not the two roundings; both roundings also
        # record the Grams, factors and SVDs their adjoints would otherwise
        # recompute
        self.tape = bool(tape) and self.C == 1
        self.torch = torch
        self.specs = list(specs)
        self.Bn = len(specs)
        self.K = zs[0].shape[0]
        self.lik_rank_cap = lik_rank_cap
        self.z, self.zdim = runner.z_tensor(zs)
        self.grids = [runner.grid_of(s) for s in self.specs]
        self.meas = [runner.meas_of(s) for s in self.specs]
        self.delta = [float(np.prod([(s.hi - s.lo) / (s.n - 1)] * s.d)) for s in self.specs]
        self.kern = []
        for s in self.specs:
            ks, _, _ = runner.build_kernels([s], B.F64)
            self.kern.append(ks[0])
        self.pcaps = [[1] + [s.cap] * (s.d - 1) + [1] for s in self.specs]

    # ---- forward pieces -------------------------------------------------
    def _zk(self, k):
        return self.z[:, k, :].contiguous()

    def _normalise(self, tts):
        lm = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
        B.tt_normalize_moments(self.grids, tts, lm)
        return lm

    def _round(self, xs, tape=None):
        outs = _new([x.n for x in xs], self.pcaps)
        groups = {}
        for i, s in enumerate(self.specs):
            groups.setdefault((s.eps, s.cap), []).append(i)
        for (eps, cap), idx in groups.items():    # one batched call per tolerance and cap
            B.tt_round([xs[i] for i in idx], [outs[i] for i in idx], eps, cap,
                       tape=tape.select(idx) if tape is not None else None)
        return outs

    def _likelihood(self, k, meas=None):
        ls = _new([[s.n] * s.d for s in self.specs], [_lik_caps(s, self.lik_rank_cap) for s in self.specs])
        B.tt_likelihood(self.grids, meas or self.meas, self._zk(k), ls, self.lik_rank_cap)
        return ls

    def _dense_likelihood(self, k, meas=None):
        ps = _new([[s.n] * s.d for s in self.specs], [_lik_caps(s, s.n) for s in self.specs])
        B.tt_likelihood_dense(self.grids, meas or self.meas, self._zk(k), ps)
        return ps

    def _step(self, k, p_prev, record=False):
        """Recompute step k from the filtering density p_prev (None at k = 0).
        record: keep the records of the prediction and update roundings
        (st.xtape, st.htape) for their adjoints."""
        st = _Step()
        st.xtape = None
        if k == 0:
            pt = _new([[s.n] * s.d for s in self.specs], self.pcaps)
            B.tt_prior(self.grids, np.array([s.m0 for s in self.specs]), np.array([s.p0_diag for s in self.specs]), pt)
            st.x = None
        else:
            st.x = _new([p.n for p in p_prev], [_prod_caps(kk, p) for kk, p in zip(self.kern, p_prev)])
            B.tt_predict(self.kern, p_prev, st.x)
            if record:
                st.xtape = B.RoundTape(st.x)
            pt = self._round(st.x, st.xtape)
        st.pt = pt
        self._normalise(pt)            # pt now holds P_pred (same cores)
        st.lik = self._likelihood(k)
        st.h = _new([p.n for p in pt], [_prod_caps(l, p) for l, p in zip(st.lik, pt)])
        log_c = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
        B.tt_update(self.grids, self.meas, self._zk(k), pt, st.h, self.lik_rank_cap, log_c)
        st.log_c = log_c
        st.htape = B.RoundTape(st.h) if record else None
        st.hr = self._round(st.h, st.htape)
        self._normalise(st.hr)         # hr now holds P_k
        return st

    def forward(self):
        """Log-likelihoods [B]; keeps the filtering TT that starts each segment
        of ckpt_every steps (P_{s-1} for s = C, 2C, ...)."""
        self.ckpt = {}
        self.tapes = {}
        ll = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
        p = None
        for k in range(self.K):
            st = self._step(k, p, record=self.tape)
            ll += st.log_c
            p = st.hr
            if (k + 1) % self.C == 0 and k + 1 < self.K:
                self.ckpt[k] = p
            if self.tape:
                st.x = None
                self.tapes[k] = st
        self.torch.cuda.synchronize()
        self.ll = ll.cpu().numpy()
        return self.ll

    # ---- reverse sweep --------------------------------------------------
    def reverse(self):
        """Adjoints of the kernel trains and of every likelihood train.  The
        segments of ckpt_every steps are taken from the last: each is
        recomputed from its checkpoint (the filtering TTs inside it kept),
        then every step of it is recomputed once more and run backwards."""
        kbar = _zero_adj(self.kern)
        self.lbar = [None] * self.K
        pbar = None
        for s0 in reversed(range(0, self.K, self.C)):
            s1 = min(s0 + self.C, self.K)
            seg = {}
            p = self.ckpt[s0 - 1] if s0 > 0 else None
            for k in range(s0, s1 - 1):
                p = self._step(k, p).hr
                seg[k] = p

            def prev(k):
                return None if k == 0 else (seg[k - 1] if (k - 1) in seg else self.ckpt[k - 1])

            for k in range(s1 - 1, s0 - 1, -1):
                pbar = self._reverse_step(k, prev(k), pbar, kbar)
        self.kbar = kbar
        self.torch.cuda.synchronize()

    def _reverse_step(self, k, pprev, pbar, kbar):
        """Recompute step k from P_{k-1} = pprev (or take its tape and
        recompute only the prediction product) and run its adjoints; returns
        the adjoint of P_{k-1} (None at k = 0)."""
        st = self.tapes.pop(k, None) if self.tape else None
        if st is None:
            st = self._step(k, pprev)
        elif k > 0:
            st.x = _new([p.n for p in pprev], [_prod_caps(kk, p) for kk, p in zip(self.kern, pprev)])
            B.tt_predict(self.kern, pprev, st.x)
        if pbar is None:
            pbar = _zero_adj(st.hr)
        # P_k = normalise(HR)
        hrbar = _like(st.hr)
        B.tt_normalize_adjoint(st.hr, pbar, None, hrbar)
        # HR = round(H)
        hbar = _like(st.h)
        B.tt_round_adjoint(st.h, st.hr, hrbar, hbar, tape=st.htape.structs if st.htape is not None else None)
        # log c_k = log(sum(H) delta): the log-mass adjoint of H with weight one
        cbar = _like(st.h)
        one = self.torch.ones(self.Bn, dtype=self.torch.float64, device="cuda")
        B.tt_normalize_adjoint(st.h, _zero_adj(st.h), one, cbar)
        B.tt_adjoint_axpy(1.0, cbar, hbar)
        # H = L o P_pred
        lbar = _like(st.lik)
        ppbar = _like(st.pt)
        B.tt_hadamard_adjoint(st.lik, st.pt, hbar, lbar, ppbar)
        # L = build(P): the adjoint onto the dense likelihood
        pd = self._dense_likelihood(k)
        pdbar = _like(pd)
        B.tt_likelihood_adjoint(self.meas, pd, st.lik, lbar, pdbar)
        self.lbar[k] = pdbar
        if k == 0:
            return None
        # P_pred = normalise(Pt), Pt = round(X), X = K (*) P_{k-1}
        ptbar = _like(st.pt)
        B.tt_normalize_adjoint(st.pt, ppbar, None, ptbar)
        xbar = _like(st.x)
        B.tt_round_adjoint(st.x, st.pt, ptbar, xbar, tape=st.xtape.structs if st.xtape is not None else None)
        pbar = _like(pprev)
        kb = _like(self.kern)
        B.tt_predict_adjoint(self.kern, pprev, xbar, pbar, kb)
        B.tt_adjoint_axpy(1.0, kb, kbar)
        return pbar

    # ---- parameter tangents -----------------------------------------------
    def _inner(self, abar, b):
        out = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
        B.tt_adjoint_inner(abar, b, out)
        return out

    def theta_grad(self, thetas: np.ndarray, h_rel: Optional[float] = None, scheme: str = "central") -> np.ndarray:
        """dLL/dtheta from the adjoints: the tangents of the kernel builds and
        of the dense likelihoods by central differences (scheme "central",
        h = 1e-5 max(1,|theta|) by default) or by forward differences from
        the base builds ("forward", 1e-7: one perturbed build per parameter
        instead of two, but the kernel TT-SVD's truncation noise, about 1e-12
        of the kernel, divided by h limits it to about 1e-4 relative)."""
        if scheme not in ("forward", "central"):
            raise ValueError(f"unknown difference scheme {scheme!r}")
        if h_rel is None:
            h_rel = 1e-7 if scheme == "forward" else 1e-5
        nt = thetas.shape[1]
        d = self.specs[0].d
        g = np.zeros((self.Bn, nt))
        boxes = [s.halfwidths() for s in self.specs]
        built = []
        signs = (1.0,) if scheme == "forward" else (1.0, -1.0)
        base_k = base_l = None
        if scheme == "forward":
            base_k = self._inner(self.kbar, self.kern)
            base_l = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
            for k in range(self.K):
                base_l += self._inner(self.lbar[k], self._dense_likelihood(k))
        for j in range(nt):
            hs = h_rel * np.maximum(1.0, np.abs(thetas[:, j]))
            vals = []
            for sgn in signs:
                th = thetas.copy()
                th[:, j] += sgn * hs
                sp = [G.spec_at(s, t, bx) for s, t, bx in zip(self.specs, th, boxes)]
                acc = self.torch.zeros(self.Bn, dtype=self.torch.float64, device="cuda")
                if j < d:
                    # built straight into the base kernels' capacities (their
                    # ranks), one batched build per offset box and tolerance;
                    # statuses checked at the end
                    kp = _like(self.kern)
                    groups = {}
                    for i, s in enumerate(sp):
                        groups.setdefault((tuple(int(h) for h in s.halfwidths()), s.kernel_tol), []).append(i)
                    for (hw, tol), idx in groups.items():
                        B.tt_kernel_build_batch([runner.grid_of(sp[i]) for i in idx], [sp[i].q for i in idx], hw, tol,
                                                [kp[i] for i in idx])
                    B.tt_align_signs(self.kern, kp)
                    acc += self._inner(self.kbar, kp)
                    built.extend(kp)
                else:
                    meas = [runner.meas_of(s) for s in sp]
                    for k in range(self.K):
                        acc += self._inner(self.lbar[k], self._dense_likelihood(k, meas))
                vals.append(acc)
            if scheme == "forward":
                base = base_k if j < d else base_l
                g[:, j] = ((vals[0] - base).cpu().numpy()) / hs
            else:
                g[:, j] = ((vals[0] - vals[1]).cpu().numpy()) / (2.0 * hs)
        if built:
            st = self.torch.stack([t.status for t in built]).cpu().numpy()
            if np.any(st != 0):
                raise B.TTError(f"perturbed kernel builds set status bits {np.unique(st)} (a rank moved)")
        return g


def loglik_grad_adjoint(specs: Sequence, zs: Sequence[np.ndarray], thetas: Optional[np.ndarray] = None,
                        h_rel: Optional[float] = None, lik_rank_cap: int = 64, scheme: str = "central",
                        ckpt_every: int = 1, tape: bool = True):
    """LL [B] and dLL/dtheta [B, n_theta] by the composed reverse sweep
    (FP64).  thetas: [B, n_theta] (None: each spec's own parameters);
    h_rel, scheme: the differences of the parameter tangents (theta_grad);
    ckpt_every: steps per checkpoint segment (1: every filtering TT kept);
    tape: with ckpt_every = 1, keep each step's intermediates except the
    prediction product (no recomputed roundings)."""
    specs = list(specs)
    if thetas is None:
        thetas = np.array([G.theta_of(s) for s in specs])
    boxes = [s.halfwidths() for s in specs]
    sp = [G.spec_at(s, t, bx) for s, t, bx in zip(specs, thetas, boxes)]
    cg = ComposedGradient(sp, zs, lik_rank_cap, ckpt_every, tape)
    ll = cg.forward()
    cg.reverse()
    return ll, cg.theta_grad(np.asarray(thetas, dtype=np.float64), h_rel, scheme), cg
