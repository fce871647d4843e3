"""Oracle parity of the whole recursion at the size of the throughput
workload: d=6, N=128 points per axis, rank cap 16, the 25-tap kernel TT of
ranks [1,15,16,16,16,15,1].  Steps 0..3 (an update, then three steps of
prediction, rounding, normalisation, update, rounding, normalisation in the
loop order of Alg. 2, with c_k of eq. pmf_filtrace_b) of sampled filters are
compared with the oracle's run of the same filter:

* the FP32-bulk batch of 256 filters in the launch configuration that the
  throughput measurement times (matrix-core prediction, 16 fibres per
  workgroup), run one step per call and saved after every step;
* the FP64 path on the same filters.

The filtering density itself is compared: for FP64 as the relative Frobenius
norm of the difference TT (normed by an orthogonalisation sweep, no
cancellation), for FP32 as the exact L1 error of every 1-D and 2-D marginal
and an importance-sampled estimate of the full L1 error (the dense 128^6
tensor cannot be formed)."""
import numpy as np
import pytest

import os
import sys

from oracle import filters as flt
from oracle import model as mdl
from oracle import tt as ttm

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_helpers import l1_marginals, l1_sampled, run_saving_states  # noqa: E402

pytestmark = pytest.mark.gpu

STEPS = 4
SAMPLED = (0, 97)
L1_SAMPLES = 20000


@pytest.fixture(scope="module")
def refs():
    from paper_2501_07942_amd import workload as wl
    specs, xs, zs = wl.make_batch("range6d_n128_c16", batch=256, steps=STEPS)
    s = specs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    kern = mdl.kernel_tt(s.q, axes, s.halfwidths(), s.kernel_tol)
    out = {}
    for b in SAMPLED:
        sb = specs[b]
        out[b] = flt.run_tt_filter(axes, sb.q, sb.halfwidths(), sb.meas(), zs[b], sb.m0, sb.p0_diag, sb.cap,
                                   sb.eps, kernel=kern, record_density=True)
    return specs, zs, axes, out


def test_fp64_path_matches_oracle_at_full_size(refs):
    from paper_2501_07942_amd import binding as B
    specs, zs, axes, ref = refs
    sub = [specs[b] for b in SAMPLED]
    out, dens = run_saving_states(sub, [zs[b] for b in SAMPLED], B.F64, range(len(SAMPLED)), STEPS)
    for i, b in enumerate(SAMPLED):
        r, s = ref[b], specs[b]
        assert out["status"][i] == 0
        assert [list(x) for x in out["ranks"][i]] == [list(x) for x in r["ranks_filt"]]
        assert [list(x) for x in out["ranks_pred"][i, 1:]] == [list(x) for x in r["ranks_pred"]]
        scale_c = max(1.0, float(np.abs(r["log_c"]).max()))
        err_c = float(np.abs(out["log_c"][i] - r["log_c"]).max())
        err_mp = float(np.abs(out["log_mpred"][i, 1:] - r["log_mpred"]).max())
        err_m = float(np.abs(out["mean"][i] - r["mean"]).max())
        err_p = max(ttm.rel_diff(g, o) for g, o in zip(dens[i], r["densities"]))
        print(f"fp64 filter {b}: |dlog c| {err_c:.2e} |dlog m_pred| {err_mp:.2e} |dmean|/dx {err_m / s.spacing():.2e}"
              f" max_k ||dP||/||P|| {err_p:.2e}")
        assert err_c <= 1e-10 * scale_c
        assert err_mp <= 1e-10 * max(1.0, float(np.abs(r["log_mpred"]).max()))
        assert err_m <= 1e-10 * s.spacing()
        assert err_p <= 1e-10


def test_fp32_batch_matches_oracle_at_full_size(refs):
    from paper_2501_07942_amd import binding as B
    specs, zs, axes, ref = refs
    out, dens = run_saving_states(specs, zs, B.F32, SAMPLED, STEPS)
    assert np.all(out["status"] == 0)
    dx = specs[0].spacing()
    for b in SAMPLED:
        r = ref[b]
        err_c = float(np.abs(out["log_c"][b] - r["log_c"]).max())
        err_m = float(np.abs(out["mean"][b] - r["mean"]).max())
        l1m = max(l1_marginals(g, o, dx) for g, o in zip(dens[b], r["densities"]))
        est = [l1_sampled(g, o, dx ** len(o), 100 + k, L1_SAMPLES) for k, (g, o) in enumerate(zip(dens[b], r["densities"]))]
        l1s, se = max(est)
        print(f"fp32 filter {b}: |dlog c| {err_c:.2e} |dmean|/dx {err_m / dx:.2e} marginal L1 {l1m:.2e}"
              f" sampled L1 {l1s:.2e} +- {se:.1e}")
        assert err_m <= 1e-3 * dx
        assert err_c <= 1e-4
        assert l1m <= 1e-4
        assert l1s + 3.0 * se <= 1e-4
