"""The per-step records of tt_filter_run_monitored against the oracle's run
of the same filters: the smallest 1-D marginal value of the filtering
density (the negativity monitor; the paper reports negative PMD values for
d >= 3, Sec. 5.1 and Sec. 6) and the relative error bound of both roundings
(sqrt of the sum of the squared discarded tails over ||A||, Sec. 3.2), FP64;
FP32 runs the same records; tt_marginal_min on single trains."""
import numpy as np
import pytest

from oracle import filters as flt
from oracle import model as mdl
from oracle import tt as ttm

pytestmark = pytest.mark.gpu

STEPS = 5


def test_monitor_records_match_the_oracle():
    import torch
    from paper_2501_07942_amd import binding as B, runner, workload as wl
    specs, xs, zs = wl.make_batch("range4d", batch=3, steps=STEPS, d=3, n=32, cap=6)
    kernels, kidx, kr = runner.build_kernels(specs, B.F64)
    fs = runner.filter_specs(specs, kidx, kr, 64)
    z, zdim = runner.z_tensor(zs)
    run = B.FilterRun(fs, kernels, STEPS, zdim, B.F64, monitor=True)
    run(z)
    torch.cuda.synchronize()
    assert np.all(run.status.cpu().numpy() == 0)
    mm = run.marg_min.cpu().numpy()
    tl = run.tails.cpu().numpy()
    for b, s in enumerate(specs):
        axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
        r = flt.run_tt_filter(axes, s.q, s.halfwidths(), s.meas(), zs[b], s.m0, s.p0_diag, s.cap, s.eps)
        # a 1-D marginal sums to sum(P) = 1/delta over its n points: compare
        # at 1e-10 of its mean value
        scale = 1.0 / (mdl.cell_volume(axes) * s.n)
        dmm = float(np.abs(mm[b] - r["marg_min"]).max())
        # the bound is a small difference of singular values: compared at 1e-4
        # of itself above the round-off floor of the largest singular value
        dtp = np.abs(tl[b, 1:, 0] - r["tail_rel_pred"]) - 1e-4 * r["tail_rel_pred"] - 1e-14
        dtf = np.abs(tl[b, :, 1] - r["tail_rel_filt"]) - 1e-4 * r["tail_rel_filt"] - 1e-14
        print(f"filter {b}: marg_min {mm[b].min():.3e} (|d| {dmm:.1e}), tails pred {tl[b, 1:, 0].max():.2e} "
              f"filt {tl[b, :, 1].max():.2e} (oracle {r['tail_rel_pred'].max():.2e} {r['tail_rel_filt'].max():.2e})",
              flush=True)
        assert dmm <= 1e-10 * scale
        assert tl[b, 0, 0] == 0.0
        assert np.all(dtp <= 0.0) and np.all(dtf <= 0.0)


def test_monitor_fp32_and_marginal_min_entry():
    import torch
    from paper_2501_07942_amd import binding as B, runner, workload as wl
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=STEPS, d=3, n=32, cap=6)
    kernels, kidx, kr = runner.build_kernels(specs, B.F32)
    fs = runner.filter_specs(specs, kidx, kr, 64)
    z, zdim = runner.z_tensor(zs)
    run = B.FilterRun(fs, kernels, STEPS, zdim, B.F32, monitor=True)
    run(z)
    torch.cuda.synchronize()
    assert np.all(run.status.cpu().numpy() == 0)
    assert np.all(np.isfinite(run.marg_min.cpu().numpy())) and np.all(run.tails.cpu().numpy() >= 0.0)
    # the stand-alone entry on random trains with negative entries, ragged ranks
    rng = np.random.default_rng(5)
    trains, refs = [], []
    for d, r in ((3, [4, 3]), (4, [2, 5, 3])):
        n = [7, 9, 6, 8][:d]
        rk = [1] + r + [1]
        cores = [rng.standard_normal((rk[k], n[k], rk[k + 1])) for k in range(d)]
        t = B.DeviceTT(n, [1] + [6] * (d - 1) + [1], B.F64)
        t.load(cores, 0.75)
        trains.append(t)
        full = ttm.full(cores) * np.exp(0.75)
        refs.append(min(full.sum(axis=tuple(a for a in range(d) if a != l)).min() for l in range(d)))
    for t, ref in zip(trains, refs):
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.tt_marginal_min([t], out)
        torch.cuda.synchronize()
        assert abs(float(out.item()) - ref) <= 1e-12 * max(1.0, abs(ref))
