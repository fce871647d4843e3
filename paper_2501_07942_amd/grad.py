"""Gradient of the log marginal likelihood sum_k log c_k (Sec. 2.2,
eq. pmf_filtrace_b) with respect to the noise and sensor parameters, on the
GPU, by central differences with rank replay.

Parameters theta, per filter: sigma_w[0..d-1] (process-noise standard
deviations, Q = D C D with the filter's correlation matrix C fixed),
then sigma_r, sigma_lin, s1, s2 for the range measurement, or sigma_lin for
the all-linear one.

One call runs the base batch in FP64 recording the ranks of every rounding,
then all 2 n_theta perturbed copies of every filter as one batch that replays
those ranks (tt_filter_run's replay inputs): each perturbed run computes the
same sequence of fixed-rank operations, so (LL(theta + h) - LL(theta - h)) / 2h
is the derivative of the computed log-likelihood.  The kernel box is held at
the base value.  This is not an adjoint: its cost is 2 n_theta + 1 forward
runs, all batched.
"""
from __future__ import annotations

import copy
import time
from typing import List, Sequence

import numpy as np

from . import binding as B
from . import runner


def theta_of(spec) -> np.ndarray:
    sw = np.sqrt(np.diag(spec.q))
    if spec.meas_kind == "range":
        return np.concatenate([sw, [spec.sigma_r, spec.sigma_lin, spec.sensor[0], spec.sensor[1]]])
    return np.concatenate([sw, [spec.sigma_lin]])


def spec_at(spec, theta, box: List[int]):
    """Copy of spec with the model parameters theta and a fixed kernel box."""
    s = copy.deepcopy(spec)
    d = spec.d
    sw0 = np.sqrt(np.diag(spec.q))
    corr = np.asarray(spec.q) / np.outer(sw0, sw0)
    sw = np.asarray(theta[:d], dtype=np.float64)
    s.q = sw[:, None] * corr * sw[None, :]
    if spec.meas_kind == "range":
        s.sigma_r = float(theta[d])
        s.sigma_lin = float(theta[d + 1])
        s.sensor = (float(theta[d + 2]), float(theta[d + 3]))
    else:
        s.sigma_lin = float(theta[d])
    s.box = list(box)
    return s


def loglik_grad(specs: Sequence, zs: Sequence[np.ndarray], thetas=None, h_rel: float = 1e-5,
                precision: int = B.F64, lik_rank_cap: int = 64, ws_budget: float = 64e9):
    """LL [B] and dLL/dtheta [B, n_theta] for a batch of filters (FP64 by
    default).  thetas: [B, n_theta] parameters (None: each spec's own).  The
    perturbed filters run in chunks whose workspace fits ws_budget bytes.
    Returns (ll, grad, info) with info = {"ms_base", "ms_perturbed",
    "filters_perturbed", "chunks", "K"}."""
    import torch
    specs = list(specs)
    nb = len(specs)
    K = zs[0].shape[0]
    if thetas is None:
        thetas = np.stack([theta_of(s) for s in specs])
    thetas = np.asarray(thetas, dtype=np.float64)
    nt = thetas.shape[1]
    boxes = [s.halfwidths() for s in specs]
    base_specs = [spec_at(s, thetas[b], boxes[b]) for b, s in enumerate(specs)]
    z, zdim = runner.z_tensor(zs)
    # base run, ranks recorded
    kernels, kidx, kr = runner.build_kernels(base_specs, precision)
    base = B.FilterRun(runner.filter_specs(base_specs, kidx, kr, lik_rank_cap), kernels, K, zdim, precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base(z, moments=False)
    torch.cuda.synchronize()
    ms_base = (time.perf_counter() - t0) * 1e3
    # perturbed copies: filter (b, j, sign) at index (b * nt + j) * 2 + (0: +h, 1: -h)
    hs = h_rel * np.maximum(1.0, np.abs(thetas))
    pspecs, pz = [], []
    for b in range(nb):
        for j in range(nt):
            for sg in (1.0, -1.0):
                th = thetas[b].copy()
                th[j] += sg * hs[b, j]
                pspecs.append(spec_at(specs[b], th, boxes[b]))
                pz.append(zs[b])
    rep = 2 * nt
    rp = base.ranks_pred.repeat_interleave(rep, dim=0).contiguous()
    rf = base.ranks.repeat_interleave(rep, dim=0).contiguous()
    ll = base.loglik.cpu().numpy()
    st = [base.status.cpu().numpy()]
    del base
    pkern, pidx, pkr = runner.build_kernels(pspecs, precision)
    fps = runner.filter_specs(pspecs, pidx, max(kr, pkr), lik_rank_cap)
    zp, _ = runner.z_tensor(pz)
    per_filter = B.workspace_bytes(fps[:1], pkern, precision)
    chunk = int(max(1, min(len(fps), ws_budget // max(per_filter, 1))))
    llp = np.zeros(len(fps))
    ms_pert = 0.0
    nchunks = 0
    for c0 in range(0, len(fps), chunk):
        c1 = min(len(fps), c0 + chunk)
        prun = B.FilterRun(fps[c0:c1], pkern, K, zdim, precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prun(zp[c0:c1].contiguous(), moments=False, replay=(rp[c0:c1].contiguous(), rf[c0:c1].contiguous()))
        torch.cuda.synchronize()
        ms_pert += (time.perf_counter() - t0) * 1e3
        llp[c0:c1] = prun.loglik.cpu().numpy()
        st.append(prun.status.cpu().numpy())
        nchunks += 1
        del prun
    llp = llp.reshape(nb, nt, 2)
    grad = (llp[:, :, 0] - llp[:, :, 1]) / (2.0 * hs)
    st = np.concatenate(st)
    if np.any(st != 0):
        raise B.TTError(f"filter status bits set in the gradient runs: {np.unique(st)}")
    return ll, grad, {"ms_base": ms_base, "ms_perturbed": ms_pert, "filters_perturbed": len(pspecs),
                      "chunks": nchunks, "K": K}


class TTFilterLogLik:
    """torch.autograd.Function-style wrapper: apply(theta, specs, zs) returns
    LL[B] as a float64 tensor whose backward gives dLL/dtheta.  theta is
    [n_theta] (shared by the batch) or [B, n_theta].  method "adjoint" (the
    default): the forward runs tt_filter_run_taped (recursion with its tape)
    and the backward tt_filter_run_adjoint (the reverse sweep, seeded with
    the incoming gradient of LL); "differences": the forward takes the
    gradient from the batched rank-replay central differences of loglik_grad
    (step h_rel) and the backward scales it."""

    @staticmethod
    def apply(theta, specs, zs, h_rel: float = 1e-5, method: str = "adjoint", ckpt_every: int = 1):
        import torch
        if method not in ("adjoint", "differences"):
            raise ValueError(f"unknown gradient method {method!r}")

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, th):
                tcpu = th.detach().cpu().numpy().astype(np.float64)
                shared = tcpu.ndim == 1
                thetas = np.tile(tcpu, (len(specs), 1)) if shared else tcpu
                ctx.shared = shared
                if method == "adjoint":
                    from . import adjoint_grad
                    ctx.fg = adjoint_grad.filter_grad(specs, zs, thetas, ckpt_every=ckpt_every)
                    ll = ctx.fg.forward().clone()
                    return ll.to(dtype=th.dtype, device=th.device)
                ll, g, _ = loglik_grad(specs, zs, thetas, h_rel)
                ctx.fg = None
                ctx.save_for_backward(torch.as_tensor(g, dtype=th.dtype, device=th.device))
                return torch.as_tensor(ll, dtype=th.dtype, device=th.device)

            @staticmethod
            def backward(ctx, gout):
                if ctx.fg is not None:
                    gt = ctx.fg.backward(gout.to(device="cuda", dtype=torch.float64))
                    st = ctx.fg.status.cpu().numpy()
                    if np.any(st != 0):
                        raise B.TTError(f"gradient run status bits {np.unique(st)}")
                    gt = gt.to(dtype=gout.dtype, device=gout.device)
                else:
                    (g,) = ctx.saved_tensors
                    gt = gout[:, None] * g
                return gt.sum(0) if ctx.shared else gt

        return _Fn.apply(theta)
