"""Reverse-mode gradient of the log marginal likelihood sum_k log c_k (Sec.
2.2, eq. pmf_filtrace_b) for a batch of FP64 filters through the library's
tt_filter_run_taped / tt_filter_run_adjoint.  Marshalling only: the forward
with its tape or checkpoints, the reverse sweep through the adjoints of
normalisation, rounding (ranks of the forward held fixed), Hadamard update,
likelihood build and prediction, and the parameter tangents all run in
libttgbf.so.

Parameters theta per filter: sigma_w[0..d-1] (process-noise standard
deviations, Q = D C D with the filter's correlation C fixed), then sigma_r,
sigma_lin, s1, s2 for the range measurement, or sigma_lin for the all-linear
one.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import binding as B
from . import grad as G
from . import runner


def grad_spec(spec, lik_rank_cap: int = 64, kernel_cap: int = 16) -> B.GradSpec:
    """The C descriptor of one filter of the gradient workload."""
    gs = B.GradSpec()
    f = runner.filter_specs([spec], [0], kernel_cap, lik_rank_cap)[0]
    gs.f = f
    d = spec.d
    q = np.asarray(spec.q, dtype=np.float64)
    for i in range(d):
        for j in range(d):
            gs.q[i * d + j] = float(q[i, j])
    for l, h in enumerate(spec.halfwidths()):
        gs.halfwidths[l] = int(h)
    gs.kernel_tol = float(spec.kernel_tol)
    return gs


def filter_grad(specs: Sequence, zs: Sequence[np.ndarray], thetas: Optional[np.ndarray] = None,
                lik_rank_cap: int = 64, ckpt_every: int = 1, kernel_cap: Optional[int] = None) -> B.FilterGrad:
    """A FilterGrad over the filters at parameters thetas [B, n_theta]
    (None: each spec's own); kernel_cap (None: the largest rank of the
    kernels' device builds) sizes the kernel trains."""
    specs = list(specs)
    if thetas is None:
        thetas = np.array([G.theta_of(s) for s in specs])
    boxes = [s.halfwidths() for s in specs]
    sp = [G.spec_at(s, t, bx) for s, t, bx in zip(specs, thetas, boxes)]
    if kernel_cap is None:
        _, _, kernel_cap = runner.build_kernels(sp, B.F64)
    z, _ = runner.z_tensor(zs)
    return B.FilterGrad([grad_spec(s, lik_rank_cap, kernel_cap) for s in sp], z, ckpt_every)


def loglik_grad_adjoint(specs: Sequence, zs: Sequence[np.ndarray], thetas: Optional[np.ndarray] = None,
                        lik_rank_cap: int = 64, ckpt_every: int = 1):
    """LL [B] and dLL/dtheta [B, n_theta] by the reverse sweep (FP64), and
    the FilterGrad that ran it (its status word per filter is checked)."""
    import torch
    fg = filter_grad(specs, zs, thetas, lik_rank_cap, ckpt_every)
    ll = fg.forward()
    g = fg.backward(torch.ones(fg.B, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    st = fg.status.cpu().numpy()
    if np.any(st != 0):
        raise B.TTError(f"gradient run status bits {np.unique(st)} (a capacity was exceeded or a rank moved)")
    return ll.cpu().numpy(), g.cpu().numpy(), fg
