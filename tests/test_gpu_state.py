"""Saving and restoring the filter state (tt_filter_state): a recursion split
at any step and continued from a saved density, in the same or in a fresh
workspace, is bitwise the uninterrupted recursion (Alg. 2's loop carries only
the filtering density from one step to the next)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import binding, runner, workload
    assert torch.cuda.is_available()
    return binding, runner, workload


def _setup(B, runner, specs, zs, precision, K):
    kernels, kidx, kr = runner.build_kernels(specs, precision)
    fspecs = runner.filter_specs(specs, kidx, kr, 64)
    z, zdim = runner.z_tensor(zs)
    return kernels, fspecs, z, zdim


@pytest.mark.parametrize("precision", [0, 1])
def test_split_run_with_saved_state_is_bitwise_the_whole_run(mods, precision):
    import torch
    B, runner, wl = mods
    K, split = 10, 5
    specs, xs, zs = wl.make_batch("range6d_ragged", batch=3, steps=K, d=3)
    for s, n, c in zip(specs, (32, 24, 40), (4, 8, 6)):
        s.n, s.cap = n, c
    kernels, fspecs, z, zdim = _setup(B, runner, specs, zs, precision, K)
    whole = B.FilterRun(fspecs, kernels, K, zdim, precision)
    whole(z)
    first = B.FilterRun(fspecs, kernels, K, zdim, precision)
    first(z, k_begin=0, k_count=split)
    saved = first.save_state()
    second = B.FilterRun(fspecs, kernels, K, zdim, precision)   # a fresh workspace
    second.log_c.copy_(first.log_c)
    second.load_state(saved)
    second(z, k_begin=split, k_count=K - split)
    torch.cuda.synchronize()
    # the caps 4 and 6 bind below the batch's largest cap 8: each filter's
    # rank rule stops at its own cap without a capacity flag
    assert np.all(whole.status.cpu().numpy() == 0)
    assert whole.ranks.cpu().numpy()[0].max() == 4 and whole.ranks.cpu().numpy()[2].max() == 6
    assert np.all(second.status.cpu().numpy() == 0)
    for name in ("log_c", "log_mpred", "mean", "cov", "ranks"):
        a = getattr(whole, name).cpu().numpy()[:, split:]
        b = getattr(second, name).cpu().numpy()[:, split:]
        assert np.array_equal(a, b), name
    assert np.array_equal(whole.loglik.cpu().numpy(), second.loglik.cpu().numpy())
    end_a = whole.save_state()
    end_b = second.save_state()
    for ta, tb in zip(end_a, end_b):
        ca, la, _ = ta.fetch()
        cb, lb, _ = tb.fetch()
        assert la == lb and all(np.array_equal(x, y) for x, y in zip(ca, cb))


def test_state_that_does_not_fit_is_flagged(mods):
    import torch
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=3, d=3, n=32, cap=8)
    kernels, fspecs, z, zdim = _setup(B, runner, specs, zs, B.F64, 3)
    run = B.FilterRun(fspecs, kernels, 3, zdim, B.F64)
    run(z)
    ranks = run.ranks.cpu().numpy()[0, -1]
    assert ranks.max() > 2
    small = B.DeviceTT([32] * 3, [1, 2, 2, 1], B.F64)
    small.cores.fill_(7.0)
    run.save_state([small])
    torch.cuda.synchronize()
    assert int(small.status.cpu().item()) == B.STATUS_CAPACITY
    assert float(small.cores[0].item()) == 7.0        # nothing copied
    assert B.device_status_string(B.STATUS_CAPACITY).startswith("TT_STATUS_CAPACITY")
