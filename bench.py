#!/usr/bin/env python3
"""Throughput of the TT grid-based filter on one MI355X.

A step is one full recursion step (predict by per-core convolution, round,
normalise, likelihood + Hadamard update with c_k, round, normalise + moments)
for every filter of the batch.  The "grad" entry times the FP64 gradient of
sum_k log c_k on the differentiated workload (d=4, N=128, 32 filters) by the
reverse sweep, with rank-replay differences beside it.  The workload is d=6, N=128 points per axis on
[-20,20]^6, rank cap 16, 256 independent filters (range on (x1,x2) plus
linear x3..x6, tridiagonal-correlated random walk), synthetic seeded inputs.

Prints ONE JSON line.  `value` = filter steps per second of the FP32-bulk
batch (inputs resident in HBM).  Also reported: the plain FP64 single-filter
comparator, per-kernel-class times from HIP events, the roofline figure of
the dominant kernel and the CPU oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TT-GBF filter steps/s (d=6,N=128,rank≤16) FP32 batch vs FP64 plain; grad ms/step"
HBM_PEAK_GBS = 8000.0
# published dense FP32 matrix-core peak of MI355X (256 CUs x 2.4 GHz x 256
# flops/clk)
FP32_MFMA_PEAK_TFS = 157.3
# HBM bytes per launch of mfma_pred_kernel over the timed steps, from
# rocprofv3 FETCH_SIZE (x2.0) and WRITE_SIZE (x1.0), the factors measured on a
# plain 256 MiB device copy (profiles/mfma_pred_kernel_traffic_*.txt); reset to
# None whenever the kernel changes
TRAFFIC = 903468715


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_batch(B, runner, binding, wl, name, batch, steps, warmup, precision, profile_steps=0, seed=None,
              graph_replays=0, autotune=False, lik_rank_cap=64):
    import torch
    total = 1 + warmup + steps + profile_steps
    kw = {} if seed is None else {"seed": seed}
    specs, xs, zs = wl.make_batch(name, batch=batch, steps=total, **kw)
    t0 = time.time()
    kernels, kidx, kr = runner.build_kernels(specs, precision)
    fspecs = runner.filter_specs(specs, kidx, kr, lik_rank_cap)
    z, zdim = runner.z_tensor(zs)
    run = binding.FilterRun(fspecs, kernels, total, zdim, precision)
    torch.cuda.synchronize()
    log(f"[bench] {name} B={batch} prec={'f32' if precision == binding.F32 else 'f64'} setup {time.time() - t0:.1f}s "
        f"kernel ranks {kernels[0].cap}")
    tune = None
    if autotune and total >= 9:
        # pick the prediction's launch shape on this batch; the recursion then
        # restarts from the prior
        tune = run.autotune(z, warmup_steps=min(4, total - 9), rounds=2)
        log(f"[bench] autotune: {tune}")
    # warm-up: step 0 (update only) and `warmup` full steps, untimed
    run(z, k_begin=0, k_count=1 + warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    run(z, k_begin=1 + warmup, k_count=steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = None
    if profile_steps:
        binding.profile_begin()
        run(z, k_begin=1 + warmup + steps, k_count=profile_steps)
        torch.cuda.synchronize()
        prof = binding.profile_end()
    st = run.status.cpu().numpy()
    log(f"[bench] timed {steps} steps: {ms:.2f} ms, failed filters {int((st != 0).sum())}")
    graph = None
    if graph_replays:
        # the last step recorded once as a HIP graph, replayed as a streaming
        # filter fed the same measurement (timing only; the results are
        # checked against eager steps in the GPU tests)
        g = run.graph(z, k_begin=total - 1, k_count=1)
        g.launch()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(graph_replays):
            g.launch()
        ev1.record(stream)
        torch.cuda.synchronize()
        graph = {"ms_per_step": round(ev0.elapsed_time(ev1) / graph_replays, 3), "replays": graph_replays,
                 "eager_ms_per_step": round(ms / steps, 3)}
        g.destroy()
        log(f"[bench] graph replay: {graph}")
    return {"run": run, "ms": ms, "prof": prof, "specs": specs, "kernels": kernels, "zs": zs,
            "status": st, "total": total, "graph": graph, "autotune": tune}


def _shape_of(specs):
    """d, N and rank cap of the filters actually run (lists when they differ
    per filter, as in a ragged batch)."""
    def one(vals):
        vals = sorted(set(int(v) for v in vals))
        return vals[0] if len(vals) == 1 else vals
    return {"d": one(s.d for s in specs), "N": one(s.n for s in specs), "rank_cap": one(s.cap for s in specs)}


def cpu_baseline(wl, steps=6, warm=3):
    """The FP64 oracle on a bounded sample: one filter of the same workload,
    `warm` untimed full steps after step 0 (ranks reach the cap), then
    `steps` timed full steps, on the host cores."""
    import numpy as np
    from oracle import model as mdl
    from oracle import tt as ttm
    specs, xs, zs = wl.make_batch("range6d_n128_c16", batch=1, steps=1 + warm + steps)
    s, z = specs[0], zs[0]
    axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
    hw = s.halfwidths()
    t0 = time.time()
    kern = mdl.kernel_tt(s.q, axes, hw, s.kernel_tol)
    log(f"[bench] oracle kernel TT {ttm.ranks(kern)} in {time.time() - t0:.1f}s")
    delta = mdl.cell_volume(axes)
    p = mdl.prior_tt(axes, s.m0, s.p0_diag)
    lik = mdl.likelihood_tt(axes, z[0], s.meas(), s.lik_tol)
    p = ttm.tt_round(ttm.hadamard(lik, p), s.eps, s.cap)
    p = ttm.scale(p, 1.0 / (ttm.tt_sum(p) * delta))
    t0 = time.time()
    for k in range(1, 1 + warm + steps):
        if k == 1 + warm:
            t0 = time.time()
        c = ttm.conv(kern, p, hw)
        p = ttm.tt_round(c, s.eps, s.cap)
        p = ttm.scale(p, 1.0 / (ttm.tt_sum(p) * delta))
        lik = mdl.likelihood_tt(axes, z[k], s.meas(), s.lik_tol)
        h = ttm.hadamard(lik, p)
        p = ttm.tt_round(h, s.eps, s.cap)
        p = ttm.scale(p, 1.0 / (ttm.tt_sum(p) * delta))
        mdl.moments_tt(p, axes)
    dt = time.time() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    thr = os.environ.get("OMP_NUM_THREADS")
    if thr:
        cores = min(cores, int(thr))
    return {"value": steps / dt, "unit": "filter-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"1 filter x {steps} full steps (steps {1 + warm}..{warm + steps}, ranks at the cap) of "
                      f"d=6 N=128 cap16, FP64 NumPy oracle, {dt:.1f}s",
            "ranks": [int(r) for r in ttm.ranks(p)]}


def grad_bench(G, wl, steps, batch):
    """grad ms/step: the FP64 gradient of sum_k log c_k with respect to the
    noise and sensor parameters on the differentiated workload (d=4, N=128,
    cap 16, range + linear, 8 parameters), by the reverse sweep
    (tt_filter_run_taped / tt_filter_run_adjoint: forward with a tape per
    step, the adjoint of every step, parameter tangents of the kernel and
    likelihood builds) and, beside
    it, by batched rank-replay central differences.  One untimed call of each
    over two steps first (kernel builds, first launches), then one timed call
    each over `steps` steps (50 by default: the differentiated workload's
    horizon)."""
    import numpy as np
    import torch
    from paper_2501_07942_amd import adjoint_grad as AG
    specs, xs, zs = wl.make_batch("range4d_grad", batch=batch, steps=steps)
    # warm calls over the first two steps (kernel builds, first launches)
    warm = [z[:2] for z in zs]
    AG.loglik_grad_adjoint(specs, warm)
    G.loglik_grad(specs, warm)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    ll_a, g_a, _ = AG.loglik_grad_adjoint(specs, zs)
    torch.cuda.synchronize()
    ms_adj = (time.perf_counter() - t0) * 1e3
    peak_gb = (torch.cuda.max_memory_allocated() - base_mem) / 1e9
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ll, g, info = G.loglik_grad(specs, zs)
    torch.cuda.synchronize()
    ms_fd_wall = (time.perf_counter() - t0) * 1e3
    ms_fd = info["ms_base"] + info["ms_perturbed"]
    agree = float(np.max(np.abs(g_a - g).max(axis=1) / np.abs(g).max(axis=1)))
    return {"value": round(ms_adj / steps, 2), "unit": "ms per batched step (forward + gradient)",
            "filter_steps_per_s": round(batch * steps / (ms_adj / 1000.0), 1),
            "workload": "range4d_grad", "d": 4, "N": 128, "rank_cap": 16, "filters": batch, "steps": steps,
            "n_theta": int(g.shape[1]), "precision": "fp64",
            "method": "tt_filter_run_taped + tt_filter_run_adjoint: forward with a tape per step, adjoints of "
                      "prediction, rounding (fixed ranks), Hadamard update, normalisation and likelihood build; "
                      "measurement parameters by the analytic derivative of the dense likelihood, process-noise "
                      "parameters by central differences of the kernel TT-SVD builds",
            "checkpoint_every": 1, "peak_hbm_GB": round(peak_gb, 2),
            "max_rel_diff_vs_differences": agree, "max_abs_dll": float(np.abs(ll_a - ll).max()),
            "differences": {"value": round(ms_fd_wall / steps, 2), "unit": "ms per batched step (forward + gradient)",
                            "runs_only_ms_per_step": round(ms_fd / steps, 2),
                            "method": "rank-replay central differences, h = 1e-5 max(1,|theta|), "
                                      "2 n_theta + 1 batched forward runs",
                            "perturbed_filters": info["filters_perturbed"],
                            "ms_base": round(info["ms_base"], 1), "ms_perturbed": round(info["ms_perturbed"], 1)}}


def grad_large_bench(wl, steps=20, batch=16, ckpt=10):
    """The FP64 gradient on the large workload (d=10, N=256 on [-25,25]^10,
    cap 32; 14 parameters: ten process-noise deviations, range and linear
    deviations, sensor position) by the reverse sweep with a checkpoint every
    `ckpt` steps, the kernel TT and its tangents by TT-cross: one untimed call
    over two steps, then one timed call over `steps` steps for `batch`
    filters (the FP64 workspace of one filter is about 13 GB)."""
    import torch
    from paper_2501_07942_amd import adjoint_grad as AG
    specs, xs, zs = wl.make_batch("range10d_n256_c32", batch=batch, steps=steps)
    AG.loglik_grad_adjoint(specs, [z[:2] for z in zs], ckpt_every=ckpt)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    ll, g, _ = AG.loglik_grad_adjoint(specs, zs, ckpt_every=ckpt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    peak_gb = (torch.cuda.max_memory_allocated() - base_mem) / 1e9
    return {"value": round(ms / steps, 2), "unit": "ms per batched step (forward + gradient)",
            "filter_steps_per_s": round(batch * steps / (ms / 1000.0), 2), "workload": "range10d_n256_c32",
            "d": 10, "N": 256, "rank_cap": 32, "filters": batch, "steps": steps, "n_theta": int(g.shape[1]),
            "precision": "fp64", "checkpoint_every": ckpt, "peak_hbm_GB": round(peak_gb, 2),
            "method": "tt_filter_run_taped + tt_filter_run_adjoint with checkpoints (segments recomputed), "
                      "kernel TT and its 2d perturbed builds by TT-cross in one batched call"}


def einsum_bench(binding, batch=64, d=4, n=64, rt=64, rp=16, calls=10):
    """The Einstein-summation prediction (Alg. 1, tt_predict_einsum) on a
    batch of FP64 filters with random 2d-core transition trains (inner
    ranks rt) and densities (inner ranks rp): ms per batched call (host
    marshalling included) and, from the library's launch events, the kernel
    time and the HBM rate of its algorithmic bytes (every transition core read once, the
    first d-1 written once, the density read once, the output's last core
    written); the CPU baseline leg times the oracle's Alg. 1 beside it."""
    import torch
    tc = [1] + [rt] * (2 * d - 1) + [1]
    pc = [1] + [rp] * (d - 1) + [1]
    T = binding.DeviceTT.batch([[n] * (2 * d)] * batch, [tc] * batch, binding.F64)
    P = binding.DeviceTT.batch([[n] * d] * batch, [pc] * batch, binding.F64)
    O = binding.DeviceTT.batch([[n] * d] * batch, [tc[:d] + [1]] * batch, binding.F64)
    gen = torch.Generator(device="cuda").manual_seed(20250114)
    for t, c in [(x, tc) for x in T] + [(x, pc) for x in P]:
        t.cores.normal_(generator=gen)
        t.ranks.copy_(torch.tensor(c, dtype=torch.int32))
    binding.tt_predict_einsum(T, P, O)  # warm
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(calls):
        binding.tt_predict_einsum(T, P, O)
    e1.record(st)
    torch.cuda.synchronize()
    ms_call = e0.elapsed_time(e1) / calls
    # the kernels alone: library events around the launches of each call
    binding.profile_begin(("einsum",))
    for _ in range(calls):
        binding.tt_predict_einsum(T, P, O)
    torch.cuda.synchronize()
    kms, kn = binding.profile_end()["einsum"][:2]
    ms = kms / max(kn, 1)
    core = lambda a, b: a * n * b
    tbytes = sum(core(tc[k], tc[k + 1]) for k in range(2 * d)) + sum(core(tc[k], tc[k + 1]) for k in range(d - 1))
    byts = 8 * batch * (tbytes + sum(core(pc[k], pc[k + 1]) for k in range(d)) + tc[d - 1] * n)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": f"random 2d-core transition trains, d={d} N={n} rank {rt}, densities rank {rp}",
            "filters": batch, "precision": "fp64", "ms_per_call": round(ms_call, 4),
            "filter_calls_per_s": round(batch / (ms_call * 1e-3), 1), "kernel_ms_per_call": round(ms, 4),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_call": byts}}


def interp_bench(binding, batch=256, d=6, n=128, r=16, calls=10):
    """Interpolation of filtering densities onto re-designed grids (Alg. 4,
    tt_interpolate) at the metric workload's shapes (FP32 cores, rank r):
    ms per batched call (host marshalling included) and, from the library's
    launch events, the kernel time and the HBM rate of its algorithmic bytes
    (the input cores read once, the output cores written once)."""
    import torch
    caps = [1] + [r] * (d - 1) + [1]
    T_in = binding.DeviceTT.batch([[n] * d] * batch, [caps] * batch, binding.F32)
    T_out = binding.DeviceTT.batch([[n] * d] * batch, [caps] * batch, binding.F32)
    gen = torch.Generator(device="cuda").manual_seed(20250114)
    for t in T_in:
        t.cores.normal_(generator=gen)
        t.ranks.copy_(torch.tensor(caps, dtype=torch.int32))
    old = [binding.make_grid(d, [n] * d, [-20.0] * d, [20.0] * d)] * batch
    new = [binding.make_grid(d, [n] * d, [-17.0 + 0.01 * b] * d, [22.5 - 0.01 * b] * d) for b in range(batch)]
    binding.tt_interpolate(old, new, T_in, T_out)  # warm
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(calls):
        binding.tt_interpolate(old, new, T_in, T_out)
    e1.record(st)
    torch.cuda.synchronize()
    ms_call = e0.elapsed_time(e1) / calls
    binding.profile_begin(("interp",))
    for _ in range(calls):
        binding.tt_interpolate(old, new, T_in, T_out)
    torch.cuda.synchronize()
    kms, kn = binding.profile_end()["interp"][:2]
    ms = kms / max(kn, 1)
    elems = sum(caps[k] * n * caps[k + 1] for k in range(d))
    byts = 4 * batch * 2 * elems
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": f"filtering densities d={d} N={n} rank {r} onto shifted and rescaled grids",
            "filters": batch, "precision": "fp32", "ms_per_call": round(ms_call, 4),
            "filter_calls_per_s": round(batch / (ms_call * 1e-3), 1), "kernel_ms_per_call": round(ms, 4),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_call": byts}}


def conv_bench(binding, runner, wl, batch=32, r=16, calls=5):
    """The materialised prediction (tt_predict: per-core convolution of the
    kernel TT with the density TT, ranks multiplied, not rounded) at the
    metric workload's shapes (d=6, N=128, FP32, density rank r, its kernel
    TT): kernel time per batched call from the library's launch events and
    the HBM rate of its algorithmic bytes (the product written once, the
    kernel and density cores read once)."""
    import torch
    specs, _, _ = wl.make_batch("range6d_n128_c16", batch=1, steps=1)
    kern, _, _ = runner.build_kernels(specs, binding.F32)
    K = kern[0]
    d, n = specs[0].d, specs[0].n
    pc = [1] + [r] * (d - 1) + [1]
    P = binding.DeviceTT.batch([[n] * d] * batch, [pc] * batch, binding.F32)
    gen = torch.Generator(device="cuda").manual_seed(20250114)
    for t in P:
        t.cores.uniform_(generator=gen)
        t.ranks.copy_(torch.tensor(pc, dtype=torch.int32))
    kr = K.ranks.cpu().numpy().tolist()
    xc = [a * b for a, b in zip(K.cap, pc)]
    X = binding.DeviceTT.batch([[n] * d] * batch, [xc] * batch, binding.F32)
    binding.tt_predict([K] * batch, P, X)  # warm
    torch.cuda.synchronize()
    binding.profile_begin(("conv",))
    for _ in range(calls):
        binding.tt_predict([K] * batch, P, X)
    torch.cuda.synchronize()
    kms, kn = binding.profile_end()["conv"][:2]
    ms = kms / max(kn, 1)
    xr = [a * b for a, b in zip(kr, pc)]
    out_elems = sum(xr[k] * n * xr[k + 1] for k in range(d))
    in_elems = sum(pc[k] * n * pc[k + 1] for k in range(d)) + sum(kr[k] * K.n[k] * kr[k + 1] for k in range(d))
    byts = 4 * batch * (out_elems + in_elems)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": f"range6d_n128_c16 densities (d={d}, N={n}, rank {r}) times its kernel TT, ranks {xr}",
            "filters": batch, "precision": "fp32", "kernel": "conv_kernel<float>", "kernel_ms_per_call": round(ms, 4),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_call": byts}}


def cross_bench(binding, wl, runner, batch=4):
    """The transition kernel of the d=10, N=256 workload (41 taps per axis,
    1.3e16 entries, no dense tensor) by the device TT-cross
    (tt_kernel_build_cross): ms per batched build of `batch` kernels and the
    ranks; the oracle's cross on the host for one kernel beside it."""
    import numpy as np
    import torch
    specs, _, _ = wl.make_batch("range10d_n256_c32", batch=batch, steps=2)
    s = specs[0]
    hw = s.halfwidths()
    taps = [2 * h + 1 for h in hw]
    outs = [binding.DeviceTT(taps, [1] + [32] * (s.d - 1) + [1], binding.F64) for _ in specs]
    grids = [runner.grid_of(x) for x in specs]
    qs = [x.q for x in specs]
    binding.tt_kernel_build_cross(grids, qs, hw, s.kernel_tol, outs)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    binding.tt_kernel_build_cross(grids, qs, hw, s.kernel_tol, outs)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ranks = outs[0].ranks.cpu().numpy().tolist()
    from oracle import cross as ocr
    from oracle import model as mdl
    axes = mdl.grid_axes([s.lo] * s.d, [s.hi] * s.d, [s.n] * s.d)
    t0 = time.perf_counter()
    ocr.kernel_tt_cross(s.q, axes, hw, s.kernel_tol)
    cpu_s = time.perf_counter() - t0
    return {"workload": f"kernel TT d={s.d}, {taps[0]} taps per axis (N={s.n} on [{s.lo},{s.hi}]), tol {s.kernel_tol}",
            "kernels": batch, "ms_per_batched_build": round(ms, 1), "ranks": ranks,
            "cpu_baseline": {"value": round(cpu_s * 1e3, 1), "unit": "ms per kernel", "kind": "oracle",
                             "sample": "1 kernel, the oracle's deterministic TT-cross, FP64 NumPy"}}


def linear_bench(binding, runner, batch=64, n=64, steps=10):
    """The filter for linear dynamics on re-designed grids (Alg. 3 with
    Alg. 4, tt_filter_run_linear) on the paper's 2-D dynamics
    F = [[1.1, 0.1], [-0.2, 1.1]], Q = I, range + linear measurement, N = 64,
    cap 16, FP64: ms per batched step; the oracle's run of one filter beside
    it."""
    import numpy as np
    import torch
    from paper_2501_07942_amd import workload as wl
    f = np.array([[1.1, 0.1], [-0.2, 1.1]])
    q = np.eye(2)
    rng = np.random.default_rng(20250114)
    specs, zs = [], []
    for b in range(batch):
        spec = wl.FilterSpec(d=2, n=n, lo=-10.0, hi=10.0, q=q, truncate_kernel=True, meas_kind="range",
                             m0=np.zeros(2), p0_diag=np.full(2, 4.0), cap=16)
        x = np.zeros((steps, 2))
        x[0] = rng.normal(0.0, 2.0, 2)
        for k in range(1, steps):
            x[k] = f @ x[k - 1] + rng.standard_normal(2)
        rho = np.hypot(x[:, 0] - spec.sensor[0], x[:, 1] - spec.sensor[1])
        zs.append(np.stack([rho + spec.sigma_r * rng.standard_normal(steps), x[:, 1] + rng.standard_normal(steps)],
                           axis=1))
        specs.append(spec)
    fs = runner.filter_specs(specs, [0] * batch, 16, 64)
    z = torch.tensor(np.stack(zs), dtype=torch.float64, device="cuda")
    binding.filter_run_linear(fs[:1], f, q, z[:1].contiguous())  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = binding.filter_run_linear(fs, f, q, z)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    from oracle import linear as lin
    t0 = time.perf_counter()
    lin.run_tt_filter_linear(f, q, specs[0].meas(), zs[0], specs[0].m0, specs[0].p0_diag, [-10.0] * 2, [10.0] * 2, n,
                             16, 1e-10)
    cpu_s = time.perf_counter() - t0
    return {"workload": f"Alg. 3 (re-designed grids) on the paper's 2-D dynamics, range + linear, N={n}, cap 16",
            "filters": batch, "steps": steps, "precision": "fp64", "ms_per_batched_step": round(ms / steps, 2),
            "filter_steps_per_s": round(batch * steps / (ms * 1e-3), 1),
            "failed_filters": int((out["status"].cpu().numpy() != 0).sum()),
            "cpu_baseline": {"value": round(steps / cpu_s, 2), "unit": "filter-steps/s", "kind": "oracle",
                             "sample": f"1 filter x {steps} steps, FP64 NumPy (dense second interpolation)"}}


def interp_cpu_baseline(d=6, n=128, r=16):
    """The oracle's interpolation on one filter of the interp_bench shapes
    (part of the CPU baseline leg)."""
    import numpy as np
    from oracle import model as mdl
    from oracle import redesign as rd
    caps = [1] + [r] * (d - 1) + [1]
    rng = np.random.default_rng(20250114)
    cores = [rng.standard_normal((caps[k], n, caps[k + 1])) for k in range(d)]
    t0 = time.perf_counter()
    rd.interpolate_tt(cores, mdl.grid_axes(-20.0, 20.0, [n] * d), mdl.grid_axes(-17.0, 22.5, [n] * d))
    return {"value": round(1.0 / (time.perf_counter() - t0), 2), "unit": "filter-calls/s", "kind": "oracle",
            "sample": f"1 filter, d={d} N={n} rank {r}, FP64 NumPy"}


def einsum_cpu_baseline(d=4, n=64, rt=64, rp=16):
    """The oracle's Alg. 1 on one filter of the einsum_bench shapes (host
    cores; part of the CPU baseline leg)."""
    import numpy as np
    from oracle import tt as ttm
    tc = [1] + [rt] * (2 * d - 1) + [1]
    pc = [1] + [rp] * (d - 1) + [1]
    rng = np.random.default_rng(20250114)
    tt = [rng.standard_normal((tc[k], n, tc[k + 1])) for k in range(2 * d)]
    pp = [rng.standard_normal((pc[k], n, pc[k + 1])) for k in range(d)]
    t0 = time.perf_counter()
    ttm.einsum_predict(tt, pp)
    return {"value": round(1.0 / (time.perf_counter() - t0), 2), "unit": "filter-calls/s", "kind": "oracle",
            "sample": f"1 filter, d={d} N={n} rank {rt}, density rank {rp}, FP64 NumPy"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--workload", default="range6d_n128_c16")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 single-filter comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient timing")
    ap.add_argument("--no-einsum", action="store_true",
                    help="skip the Einstein-summation, interpolation and materialised-convolution timings")
    ap.add_argument("--extra-only", action="store_true",
                    help="only time the Einstein-summation prediction, the interpolation onto a new grid and the "
                         "materialised convolution")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged batch (N and cap drawn per filter)")
    ap.add_argument("--no-large", action="store_true", help="skip the d=10, N=256, cap-32 batch of 64 filters")
    ap.add_argument("--grad-steps", type=int, default=50)
    ap.add_argument("--grad-batch", type=int, default=32)
    ap.add_argument("--grad-only", action="store_true",
                    help="only time the gradient (prints {\"grad\": ...}; for profiling the reverse sweep)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default prediction launch shape")
    ap.add_argument("--graph-replays", type=int, default=3,
                    help="replays of one step recorded as a HIP graph (0: skip)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              f"(independent filters shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_07942_amd import binding, runner, workload as wl
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration > 0:
        nel = int(args.copy_calibration * 2 ** 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nel * 4, "copy_bytes_written": nel * 4, "copies": 5}), flush=True)
        return

    if args.extra_only:
        print(json.dumps({"einsum_predict": einsum_bench(binding), "interpolate": interp_bench(binding),
                          "conv_hbm": conv_bench(binding, runner, wl)}), flush=True)
        return
    if args.grad_only:
        from paper_2501_07942_amd import grad as G
        print(json.dumps({"grad": grad_bench(G, wl, args.grad_steps, args.grad_batch)}), flush=True)
        return

    main_res = run_batch(None, runner, binding, wl, args.workload, args.batch, args.steps, args.warmup,
                         binding.F32, profile_steps=args.profile_steps, graph_replays=args.graph_replays,
                         autotune=not args.no_autotune)
    B = args.batch
    ms = main_res["ms"]
    value = B * args.steps / (ms / 1000.0)

    # roofline of the dominant kernel from the profiled window: the fused
    # prediction (convolution + absorption of the next factor), a dense FP32
    # contraction on the matrix cores; its algorithmic flops and bytes come
    # from the library's work model evaluated on the device-resident ranks
    prof = main_res["prof"] or {}
    kernel_ms = {k: round(v[0] / max(args.profile_steps, 1), 3) for k, v in prof.items() if v[1]}
    roof = None
    if prof and prof["pred"][1] > 0 and prof["pred"][2] > 0:
        ms_p, n_p, fl_p, by_p = prof["pred"]
        avg_s = ms_p / n_p / 1000.0
        achieved = fl_p / n_p / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_MFMA_PEAK_TFS, 4), "traffic": TRAFFIC,
                "kernel": "mfma_pred_kernel<float, FFused<float>>", "avg_launch_ms": round(ms_p / n_p, 4),
                "launches": n_p, "algorithmic_flops_per_launch": round(fl_p / n_p),
                "algorithmic_bytes_per_launch": round(by_p / n_p),
                "algorithmic_GBs": round(by_p / n_p / avg_s / 1e9, 1)}
    # the HBM-bound update product: algorithmic bytes (write H, read L and P)
    # per launch over its HIP-event time
    hbm = None
    if prof and prof["hadamard"][1] > 0 and prof["hadamard"][3] > 0:
        ms_h, n_h, _, by_h = prof["hadamard"]
        gbs = by_h / n_h / (ms_h / n_h / 1000.0) / 1e9
        hbm = {"kernel": "hadamard_kernel<float>", "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_launch_ms": round(ms_h / n_h, 4),
               "algorithmic_bytes_per_launch": round(by_h / n_h)}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "filter-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-walk trajectories and range/linear measurements)",
        "config": {"workload": args.workload, **_shape_of(main_res["specs"]), "filters": B,
                   "precision": "fp32 bulk, fp64 Gram/pivoted-Cholesky/Jacobi, fp64 log-normaliser",
                   "failed_filters": int((main_res["status"] != 0).sum()),
                   "workspace_GB": round(main_res["run"].ws.numel() * main_res["run"].ws.element_size() / 1e9, 2)},
        "roofline": roof,
        "kernel_ms_per_step": kernel_ms,
        "hadamard_hbm": hbm,
        "graph_step": main_res["graph"],
        "autotune": main_res["autotune"],
    }
    if not args.no_einsum:
        out["kernel_cross"] = cross_bench(binding, wl, runner)
        out["linear_dynamics"] = linear_bench(binding, runner)
        torch.cuda.empty_cache()
    if not args.no_ragged:
        # the ragged batch: N and rank cap drawn per filter, same model
        rg = run_batch(None, runner, binding, wl, "range6d_ragged", B, args.steps, args.warmup, binding.F32)
        mix = {}
        for s in rg["specs"]:
            key = f"N{s.n}_c{s.cap}"
            mix[key] = mix.get(key, 0) + 1
        out["ragged"] = {"workload": "range6d_ragged", "value": round(B * args.steps / (rg["ms"] / 1000.0), 2),
                         "unit": "filter-steps/s", "ms_per_step": round(rg["ms"] / args.steps, 3), "filters": B,
                         "mix": dict(sorted(mix.items())), "failed_filters": int((rg["status"] != 0).sum()),
                         "workspace_GB": round(rg["run"].ws.numel() * rg["run"].ws.element_size() / 1e9, 2),
                         "precision": "fp32 bulk, fp64 Gram/pivoted-Cholesky/Jacobi, fp64 log-normaliser"}
        rg.clear()
        torch.cuda.empty_cache()
    if not args.no_einsum:
        out["einsum_predict"] = einsum_bench(binding)
        torch.cuda.empty_cache()
        out["interpolate"] = interp_bench(binding)
        torch.cuda.empty_cache()
        out["conv_hbm"] = conv_bench(binding, runner, wl)
        torch.cuda.empty_cache()
    if not args.no_plain:
        plain = run_batch(None, runner, binding, wl, args.workload, 1, args.steps, args.warmup, binding.F64)
        out["fp64_plain"] = {"value": round(args.steps / (plain["ms"] / 1000.0), 3), "unit": "filter-steps/s",
                             "ms_per_step": round(plain["ms"] / args.steps, 3), "filters": 1,
                             "failed_filters": int((plain["status"] != 0).sum())}
        out["fp32_batch_over_fp64_plain"] = round(value / out["fp64_plain"]["value"], 2)
        plain.clear()
    if not args.no_grad:
        from paper_2501_07942_amd import grad as G
        main_res.clear()  # release the batch's workspace before the gradient runs
        torch.cuda.empty_cache()
        out["grad"] = grad_bench(G, wl, args.grad_steps, args.grad_batch)
    if not args.no_large:
        # the large workload: d=10, N=256 on [-25,25]^10, cap 32, 64 filters,
        # all 200 steps (10 untimed after the first update, 187 timed, the
        # last 2 profiled for the prediction's roofline); the kernel TT by
        # TT-cross, likelihood blocks up to rank 96
        main_res.clear()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        lg = run_batch(None, runner, binding, wl, "range10d_n256_c32", 64, 187, 10, binding.F32, lik_rank_cap=96,
                       profile_steps=2, autotune=not args.no_autotune)
        st = lg["status"]
        lroof = None
        lprof = lg["prof"] or {}
        if lprof and lprof["pred"][1] > 0 and lprof["pred"][2] > 0:
            ms_p, n_p, fl_p, by_p = lprof["pred"]
            achieved = fl_p / n_p / (ms_p / n_p / 1000.0) / 1e12
            lroof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_MFMA_PEAK_TFS, 4),
                     "kernel": "mfma_pred_kernel<float, FFused<float>, true> (single-buffer variant)",
                     "avg_launch_ms": round(ms_p / n_p, 4), "launches": n_p,
                     "algorithmic_flops_per_launch": round(fl_p / n_p)}
        out["large_d10"] = {"workload": "range10d_n256_c32",
                            "value": round(64 * 187 / (lg["ms"] / 1000.0), 2), "unit": "filter-steps/s",
                            "ms_per_step": round(lg["ms"] / 187, 3), "filters": 64, "timed_steps": 187,
                            "roofline": lroof,
                            "failed_filters": int((st != 0).sum()),
                            "max_rank_last_step": int(lg["run"].ranks[:, -1].max().item()),
                            "workspace_GB": round(lg["run"].ws.numel() * lg["run"].ws.element_size() / 1e9, 2),
                            "peak_hbm_GB": round(torch.cuda.max_memory_allocated() / 1e9, 2),
                            "precision": "fp32 bulk, fp64 Gram/pivoted-Cholesky/Jacobi, fp64 log-normaliser"}
        lg.clear()
        torch.cuda.empty_cache()
        if not args.no_grad:
            out["large_d10"]["grad"] = grad_large_bench(wl)
            torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
        if "einsum_predict" in out:
            out["einsum_predict"]["cpu_baseline"] = einsum_cpu_baseline()
        if "interpolate" in out:
            out["interpolate"]["cpu_baseline"] = interp_cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
