"""Shared helpers of the GPU tests (not collected)."""
import itertools
import math

import numpy as np

from oracle import tt as ttm


def rand_pos_tt(rng, n, r):
    rk = [1] + list(r) + [1]
    return [np.abs(rng.standard_normal((rk[k], n[k], rk[k + 1]))) + 0.05 for k in range(len(n))]


def caps_of(cores, extra=0):
    return [1] + [g.shape[2] + extra for g in cores[:-1]] + [1]


def to_dev(B, cores, dtype, cap=None, log_scale=0.0):
    n = [g.shape[1] for g in cores]
    t = B.DeviceTT(n, cap or caps_of(cores), dtype)
    t.load(cores, log_scale)
    return t


def fetch_full(t):
    cores, st = t.fetch_scaled()
    return ttm.full(cores), cores, st


def run_saving_states(specs, zs, precision, keep, steps):
    """tt_filter_run one step per call; after each step the states of the
    filters in ``keep`` are saved (tt_filter_state) and fetched."""
    import torch
    from paper_2501_07942_amd import binding as B, runner
    kernels, kidx, kr = runner.build_kernels(specs, precision)
    fspecs = runner.filter_specs(specs, kidx, kr, 64)
    z, zdim = runner.z_tensor(zs)
    run = B.FilterRun(fspecs, kernels, steps, zdim, precision)
    trains = run.state_trains()
    dens = {b: [] for b in keep}
    for k in range(steps):
        run(z, k_begin=k, k_count=1)
        run.save_state(trains)
        for b in keep:
            cores, st = trains[b].fetch_scaled()
            assert st == 0
            dens[b].append(cores)
    torch.cuda.synchronize()
    out = {k: getattr(run, k).cpu().numpy() for k in ("log_c", "log_mpred", "mean", "cov", "ranks", "ranks_pred",
                                                      "status", "loglik")}
    del run, trains
    torch.cuda.empty_cache()
    return out, dens


def l1_marginals(p_gpu, p_ora, delta):
    """Exact L1 error sum |dm| * (cell volume of the marginal) of every 1-D
    and 2-D marginal of two densities on the same grid (delta = the spacing
    per axis); returns the largest."""
    d = len(p_ora)
    worst = 0.0
    for keep in itertools.chain(((l,) for l in range(d)), itertools.combinations(range(d), 2)):
        dm = ttm.marginal(p_gpu, keep) - ttm.marginal(p_ora, keep)
        worst = max(worst, float(np.abs(dm).sum()) * delta ** d)
    return worst


def l1_sampled(p_gpu, p_ora, delta, seed, count):
    """Importance-sampled full L1 error sum_i |dP(i)| delta with indices
    drawn from the oracle's density: mean and standard error."""
    idx, q = ttm.sample(p_ora, count, np.random.default_rng(seed))
    w = np.abs(ttm.values(p_gpu, idx) - ttm.values(p_ora, idx)) * delta / q
    return float(w.mean()), float(w.std() / math.sqrt(len(w)))
