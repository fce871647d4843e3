"""Seeded synthetic workloads for the TT grid-based filter.

This module holds model *specifications* and the simulation of truth and
measurements only; it contains none of the filter's arithmetic.  It is the
one module that both the HIP path's callers and the CPU checker read, so
that both consume identical inputs.

Model (random walk, Sec. 1 eqs. asx/asz with f = identity):
    x_{k+1} = x_k + w_k,  w_k ~ N(0, Q)
    z_k     = h(x_k) + v_k
with h either linear on every axis (z = x + v, v ~ N(0, sigma_lin^2 I)) or
the range to a sensor on (x_1, x_2) followed by linear measurements of the
remaining axes.  Q = D C D with D = diag(sigma_w) and C tridiagonal with unit
diagonal and rho on the first off-diagonals.

Truth trajectories are drawn with NumPy's PCG64 from
``SeedSequence(seed).spawn(B)``; a trajectory that leaves the central 75 % of
the grid box is redrawn (at most 1000 tries, then the last draw is kept).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

BASE_SEED = 20250114


def tridiag_q(d: int, sigma_w, rho: float = 0.3) -> np.ndarray:
    """Q = D C D, C = tridiag(rho, 1, rho), D = diag(sigma_w)."""
    sw = np.broadcast_to(np.asarray(sigma_w, dtype=np.float64), (d,))
    c = np.eye(d)
    for l in range(d - 1):
        c[l, l + 1] = c[l + 1, l] = rho
    return np.diag(sw) @ c @ np.diag(sw)


@dataclasses.dataclass
class FilterSpec:
    """One filter: grid, model, prior, rounding settings."""
    d: int
    n: int
    lo: float
    hi: float
    q: np.ndarray
    truncate_kernel: bool
    meas_kind: str                     # "linear" or "range"
    sensor: Tuple[float, float] = (3.0, -2.0)
    sigma_r: float = 0.5
    sigma_lin: float = 1.0
    m0: Optional[np.ndarray] = None
    p0_diag: Optional[np.ndarray] = None
    cap: int = 16
    eps: float = 1e-10
    kernel_tol: float = 1e-12
    lik_tol: float = 1e-12
    nsigma: float = 4.0
    box: Optional[List[int]] = None    # fixed kernel half widths (overrides the rule)

    @property
    def b(self) -> int:
        return self.d if self.meas_kind == "linear" else self.d - 1

    def meas(self) -> dict:
        if self.meas_kind == "linear":
            return {"kind": "linear", "sigma_lin": self.sigma_lin}
        return {"kind": "range", "sensor": tuple(self.sensor), "sigma_r": self.sigma_r,
                "sigma_lin": self.sigma_lin}

    def spacing(self) -> float:
        return (self.hi - self.lo) / (self.n - 1)

    def halfwidths(self) -> List[int]:
        """Offsets of the kernel box per axis: floor(nsigma*sqrt(Q_ll)/Delta),
        or N-1 (every grid offset) when the kernel is not truncated; ``box``
        when it is set."""
        if self.box is not None:
            return list(self.box)
        if not self.truncate_kernel:
            return [self.n - 1] * self.d
        dx = self.spacing()
        return [int(math.floor(self.nsigma * math.sqrt(self.q[l, l]) / dx + 1e-12))
                for l in range(self.d)]


def measure(spec: FilterSpec, x: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Simulated measurement h(x) + v."""
    if spec.meas_kind == "linear":
        return x + v
    rng = math.hypot(x[0] - spec.sensor[0], x[1] - spec.sensor[1])
    return np.concatenate([[rng], x[2:]]) + v


def simulate(spec: FilterSpec, steps: int, seed_seq: np.random.SeedSequence,
             central: float = 0.75, max_tries: int = 1000):
    """Truth x[0..K-1] and measurements z[0..K-1] for one filter."""
    gen = np.random.Generator(np.random.PCG64(seed_seq))
    chol_q = np.linalg.cholesky(spec.q)
    half = 0.5 * (spec.hi - spec.lo)
    mid = 0.5 * (spec.hi + spec.lo)
    noise_sd = np.full(spec.b, spec.sigma_lin)
    if spec.meas_kind == "range":
        noise_sd[0] = spec.sigma_r
    x = z = None
    for _ in range(max_tries):
        x = np.zeros((steps, spec.d))
        x[0] = spec.m0 + np.sqrt(spec.p0_diag) * gen.standard_normal(spec.d)
        for k in range(1, steps):
            x[k] = x[k - 1] + chol_q @ gen.standard_normal(spec.d)
        if np.all(np.abs(x - mid) <= central * half):
            break
    z = np.stack([measure(spec, x[k], noise_sd * gen.standard_normal(spec.b))
                  for k in range(steps)])
    return x, z


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def spec_kf2d() -> FilterSpec:
    """d=2, N=64 on [-10,10]^2, Q=diag(.5,.5) untruncated, z = x + v (R=I),
    x0 ~ N(0, 4I), rank cap 8, rounding tol 1e-10."""
    return FilterSpec(d=2, n=64, lo=-10.0, hi=10.0, q=np.diag([0.5, 0.5]),
                      truncate_kernel=False, meas_kind="linear", sigma_lin=1.0,
                      m0=np.zeros(2), p0_diag=np.full(2, 4.0), cap=8, eps=1e-10)


def spec_range(d: int, n: int, cap: int, lo: float = -20.0, hi: float = 20.0,
               sigma_w=1.0, rho: float = 0.3, sigma_r: float = 0.5,
               sigma_lin: float = 1.0, sensor=(3.0, -2.0), p0: float = 9.0,
               eps: float = 1e-10) -> FilterSpec:
    """Range on (x_1,x_2) plus linear x_3..x_d, tridiagonal-correlated random
    walk, kernel truncated at 4 sigma, x0 ~ N(0, p0 I)."""
    return FilterSpec(d=d, n=n, lo=lo, hi=hi, q=tridiag_q(d, sigma_w, rho),
                      truncate_kernel=True, meas_kind="range", sensor=tuple(sensor),
                      sigma_r=sigma_r, sigma_lin=sigma_lin, m0=np.zeros(d),
                      p0_diag=np.full(d, p0), cap=cap, eps=eps)


WORKLOADS = {
    # name: (description, builder(batch index) -> spec, filters, steps)
    "kf2d": ("d=2 N=64 linear-Gaussian, dense vs TT vs Kalman", 1, 20),
    "range4d": ("d=4 N=128 cap16 range+linear, FP64 single filter", 1, 50),
    "range6d_n128_c16": ("d=6 N=128 cap16 range+linear, uniform batch", 256, 100),
    "range6d_ragged": ("d=6 N in {64,96,128} cap in {8,16,24}, ragged batch", 256, 100),
    "range4d_grad": ("d=4 N=128 cap16 differentiated batch", 32, 50),
    "range10d_n256_c32": ("d=10 N=256 on [-25,25] cap32 range+linear, large batch", 64, 200),
}


def ragged_choice(seed_seq: np.random.SeedSequence) -> Tuple[int, int]:
    """(N, cap) drawn uniformly from {64,96,128} x {8,16,24} per filter."""
    gen = np.random.Generator(np.random.PCG64(seed_seq))
    n = int(gen.choice([64, 96, 128]))
    cap = int(gen.choice([8, 16, 24]))
    return n, cap


def make_batch(name: str, batch: Optional[int] = None, steps: Optional[int] = None,
               seed: int = BASE_SEED, n: Optional[int] = None, d: Optional[int] = None,
               cap: Optional[int] = None):
    """Specs, truths and measurements for a named workload.

    Returns (specs[B], x[B][K,d], z[B][K,b]).  ``n``, ``d`` and ``cap``
    override the grid size, dimension and rank cap (used for reduced parity
    cases)."""
    _, b_default, k_default = WORKLOADS[name]
    nb = b_default if batch is None else batch
    ks = k_default if steps is None else steps
    children = np.random.SeedSequence(seed).spawn(nb)
    specs, xs, zs = [], [], []
    for i in range(nb):
        sim_seq, choice_seq = children[i].spawn(2)
        if name == "kf2d":
            spec = spec_kf2d()
            if n is not None:
                spec.n = n
        elif name in ("range4d", "range4d_grad"):
            spec = spec_range(d or 4, n or 128, cap or 16)
        elif name == "range6d_n128_c16":
            spec = spec_range(d or 6, n or 128, cap or 16)
        elif name == "range10d_n256_c32":
            spec = spec_range(d or 10, n or 256, cap or 32, lo=-25.0, hi=25.0)
        elif name == "range6d_ragged":
            nn, cc = ragged_choice(choice_seq)
            spec = spec_range(d or 6, n or nn, cap or cc)
        else:
            raise KeyError(name)
        if cap is not None:
            spec.cap = cap
        x, z = simulate(spec, ks, sim_seq)
        specs.append(spec)
        xs.append(x)
        zs.append(z)
    return specs, xs, zs
