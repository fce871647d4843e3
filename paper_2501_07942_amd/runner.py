"""Set-up helpers around the C ABI: turn workload specifications into C
descriptors, build one transition-kernel TT per distinct grid and run the
batched filter.  Marshalling only; the arithmetic is in libttgbf.so."""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import binding as B
from .workload import FilterSpec as WSpec


def grid_of(spec: WSpec) -> B.Grid:
    return B.make_grid(spec.d, [spec.n] * spec.d, [spec.lo] * spec.d, [spec.hi] * spec.d)


def meas_of(spec: WSpec) -> B.Meas:
    kind = 0 if spec.meas_kind == "linear" else 1
    return B.make_meas(kind, spec.sensor, spec.sigma_r, spec.sigma_lin, spec.lik_tol, 0)


def kernel_key(spec: WSpec) -> Tuple:
    return (spec.d, spec.n, spec.lo, spec.hi, tuple(np.asarray(spec.q).ravel().tolist()),
            tuple(spec.halfwidths()), spec.kernel_tol)


def build_kernels(specs: Sequence[WSpec], precision: int, kernel_cap: int = 32):
    """One device kernel TT per distinct (grid, Q, box), re-packed with
    capacities equal to its ranks: the dense TT-SVD build up to d = 8 and
    2^28 taps, the TT-cross build beyond.  Returns (kernels, index per
    filter, largest interior kernel rank)."""
    kernels: List[B.DeviceTT] = []
    index: Dict[Tuple, int] = {}
    idx = []
    rmax = 1
    for s in specs:
        key = kernel_key(s)
        if key not in index:
            hw = s.halfwidths()
            taps = [2 * h + 1 for h in hw]
            # the device TT-SVD keeps rank*taps <= 1024 per unfolding
            cap = [1] + [min(kernel_cap, 1024 // taps[j], 1024 // taps[j - 1], int(np.prod(taps[:j])),
                             int(np.prod(taps[j:]))) for j in range(1, s.d)] + [1]
            kt = B.DeviceTT(taps, cap, precision)
            if s.d > 8 or float(np.prod([float(t) for t in taps])) > 2.0 ** 28:
                # no dense tensor: the kernel by TT-cross from point values
                kt = B.DeviceTT(taps, [1] + [min(kernel_cap, 64, int(min(np.prod(taps[:j]), np.prod(taps[j:]))))
                                             for j in range(1, s.d)] + [1], precision)
                B.tt_kernel_build_cross([grid_of(s)], [s.q], hw, s.kernel_tol, [kt], max_rank=64)
            else:
                B.tt_kernel_build(grid_of(s), s.q, hw, s.kernel_tol, kt)
            cores, ls, st = kt.fetch()
            if st != 0:
                raise B.TTError(f"kernel build status {st}")
            ranks = [1] + [g.shape[2] for g in cores]
            tight = B.DeviceTT(taps, ranks, precision)
            tight.load(cores, ls)
            rmax = max(rmax, max(ranks))
            index[key] = len(kernels)
            kernels.append(tight)
        idx.append(index[key])
    return kernels, idx, rmax


def filter_specs(specs: Sequence[WSpec], kidx: Sequence[int], kernel_cap: int = 16,
                 lik_rank_cap: int = 64) -> List[B.FilterSpec]:
    out = []
    for s, ki in zip(specs, kidx):
        f = B.FilterSpec()
        f.grid = grid_of(s)
        f.meas = meas_of(s)
        for l in range(s.d):
            f.m0[l] = float(s.m0[l])
            f.p0_diag[l] = float(s.p0_diag[l])
        f.cap = int(s.cap)
        f.eps = float(s.eps)
        f.kernel_index = int(ki)
        f.kernel_cap = int(kernel_cap)
        f.lik_rank_cap = int(lik_rank_cap)
        out.append(f)
    return out


def z_tensor(zs: Sequence[np.ndarray]):
    import torch
    zdim = max(z.shape[1] for z in zs)
    K = zs[0].shape[0]
    host = np.zeros((len(zs), K, zdim))
    for b, z in enumerate(zs):
        host[b, :, :z.shape[1]] = z
    return torch.from_numpy(host).cuda(), zdim


def run_filters(specs: Sequence[WSpec], zs: Sequence[np.ndarray], precision: int,
                lik_rank_cap: int = 64):
    """Build kernels and run the whole recursion once; returns the FilterRun
    (device outputs) after the stream has synchronised."""
    import torch
    kernels, kidx, kr = build_kernels(specs, precision)
    fspecs = filter_specs(specs, kidx, kr, lik_rank_cap)
    z, zdim = z_tensor(zs)
    run = B.FilterRun(fspecs, kernels, zs[0].shape[0], zdim, precision)
    run(z)
    torch.cuda.synchronize()
    return run, z
