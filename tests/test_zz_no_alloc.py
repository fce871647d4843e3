"""tt_normalize_moments_noalloc (the allocation-free variant for callers
that cannot allocate device memory) against tt_normalize_moments: the same
kernels on the library's static scratch give bitwise the same log-masses,
moments and normalised trains, on two calls in a row (the second with a
smaller batch, d and rank capacity, over the first call's leftovers)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(B, rng, batch, d, n, r, dtype):
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from gpu_helpers import rand_pos_tt, to_dev
    cores = [rand_pos_tt(rng, [n] * d, [r] * (d - 1)) for _ in range(batch)]
    cap = [1] + [r + 3] * (d - 1) + [1]
    pair = [[to_dev(B, c, dtype, cap=cap, log_scale=0.3 * i) for i, c in enumerate(cores)] for _ in range(2)]
    grids = [B.make_grid(d, [n] * d, [-5.0 - i] * d, [6.0 + i] * d) for i in range(batch)]
    return grids, pair


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_matches_the_workspace_entry_point_on_two_calls(dtype):
    import torch
    from paper_2501_07942_amd import binding as B
    rng = np.random.default_rng(17)
    for batch, d, n, r in ((24, 6, 48, 12), (3, 3, 20, 4)):
        grids, (ta, tb) = _case(B, rng, batch, d, n, r, dtype)
        outs = []
        for fn, ts in ((B.tt_normalize_moments, ta), (B.tt_normalize_moments_noalloc, tb)):
            lm = torch.zeros(batch, dtype=torch.float64, device="cuda")
            mu = torch.zeros(batch, d, dtype=torch.float64, device="cuda")
            cv = torch.zeros(batch, d, d, dtype=torch.float64, device="cuda")
            fn(grids, ts, lm, mu, cv)
            torch.cuda.synchronize()
            outs.append((lm.cpu().numpy(), mu.cpu().numpy(), cv.cpu().numpy()))
        for x, y in zip(outs[0], outs[1]):
            assert np.all(np.isfinite(x)) and np.array_equal(x, y)
        for a, b in zip(ta, tb):
            ca, la, sa = a.fetch()
            cb, lb, sb = b.fetch()
            assert sa == sb == 0 and la == lb
            assert all(np.array_equal(x, y) for x, y in zip(ca, cb))


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch
    from paper_2501_07942_amd import binding as B
    d, n, cap = 8, 4, [1] + [64] * 7 + [1]
    ts = B.DeviceTT.batch([[n] * d] * 64, [cap] * 64, B.F64)
    grids = [B.make_grid(d, [n] * d, [-1.0] * d, [1.0] * d)] * 64
    lm = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(B.TTError, match="TT_ERR_WORKSPACE"):
        B.tt_normalize_moments_noalloc(grids, ts, lm)
