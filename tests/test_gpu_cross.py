"""The transition kernel by deterministic TT-cross on the device
(tt_kernel_build_cross) against the dense TT-SVD build and the oracle: same
ranks and the same tensor at d <= 6 (the dense tensor exists), and at d = 10
on the 41-tap box of N = 256 on [-25, 25] (1.3e16 entries, no dense
tensor) against the oracle's cross and direct evaluation of eq. TPMmat."""
import numpy as np
import pytest

from oracle import cross as ocr
from oracle import model as mdl
from oracle import tt as ttm

pytestmark = pytest.mark.gpu


def q_of(d, sw):
    sw = np.asarray(sw, dtype=np.float64)
    return sw[:, None] * (np.eye(d) + 0.3 * (np.eye(d, k=1) + np.eye(d, k=-1))) * sw[None, :]


def build_cross(B, grids, qs, hw, caps, dtype=0):
    outs = [B.DeviceTT([2 * h + 1 for h in hw], caps, dtype) for _ in qs]
    B.tt_kernel_build_cross(grids, qs, hw, 1e-12, outs)
    return outs


@pytest.mark.parametrize("d,n", [(3, 64), (4, 128), (6, 128)])
def test_cross_kernel_equals_dense_device_build(d, n):
    from paper_2501_07942_amd import binding as B
    grid = B.make_grid(d, [n] * d, [-20.0] * d, [20.0] * d)
    axes = mdl.grid_axes([-20.0] * d, [20.0] * d, [n] * d)
    sws = ([1.0] * d, list(1.0 + 0.1 * np.arange(d)))
    qs = [q_of(d, sw) for sw in sws]
    hw = mdl.kernel_halfwidths(qs[0], axes)
    caps = [1] + [32] * (d - 1) + [1]
    print(f"cross kernel d={d} N={n} taps {2 * hw[0] + 1}", flush=True)
    outs = build_cross(B, [grid, grid], qs, hw, caps)
    for q, o in zip(qs, outs):
        dense = B.DeviceTT([2 * h + 1 for h in hw], caps, B.F64)
        B.tt_kernel_build(grid, q, hw, 1e-12, dense)
        cc, sc = o.fetch_scaled()
        cd, sd = dense.fetch_scaled()
        assert sc == 0 and sd == 0
        print(f"  ranks cross {ttm.ranks(cc)} dense {ttm.ranks(cd)} rel {ttm.rel_diff(cc, cd):.1e}", flush=True)
        assert ttm.ranks(cc) == ttm.ranks(cd)
        assert ttm.rel_diff(cc, cd) <= 1e-11
        if d <= 4:
            assert ttm.rel_diff(cc, mdl.kernel_tt(q, axes, hw, 1e-12)) <= 1e-11


def test_cross_kernel_d10_n256_against_oracle_and_point_values():
    from paper_2501_07942_amd import binding as B
    d, n = 10, 256
    grid = B.make_grid(d, [n] * d, [-25.0] * d, [25.0] * d)
    axes = mdl.grid_axes([-25.0] * d, [25.0] * d, [n] * d)
    q = q_of(d, np.ones(d))
    hw = mdl.kernel_halfwidths(q, axes)
    assert hw == [20] * d
    caps = [1] + [32] * (d - 1) + [1]
    (o,) = build_cross(B, [grid], [q], hw, caps)
    f32 = build_cross(B, [grid], [q], hw, caps, dtype=B.F32)[0]
    cc, st = o.fetch_scaled()
    assert st == 0
    ref = ocr.kernel_tt_cross(q, axes, hw, 1e-12)
    print(f"d=10 cross ranks {ttm.ranks(cc)}, oracle {ttm.ranks(ref)}, rel {ttm.rel_diff(cc, ref):.1e}", flush=True)
    assert ttm.ranks(cc) == ttm.ranks(ref)
    assert ttm.rel_diff(cc, ref) <= 1e-11
    rng = np.random.default_rng(7)
    offs = np.stack([rng.integers(-h, h + 1, 500) for h in hw], axis=1)
    want = mdl.kernel_at(q, axes, offs)
    peak = float(mdl.kernel_at(q, axes, np.zeros((1, d)))[0])
    got = ttm.values(cc, offs + np.array(hw)[None, :])
    assert np.abs(got - want).max() <= 1e-11 * peak
    c32, s32 = f32.fetch_scaled()
    assert s32 == 0 and ttm.ranks(c32) == ttm.ranks(cc)
    assert np.abs(ttm.values(c32, offs + np.array(hw)[None, :]) - want).max() <= 1e-6 * peak


@pytest.mark.parametrize("d,n,r", [(2, 48, 6), (3, 24, 4)])
def test_lattice_interpolation_matches_the_dense_definition(d, n, r):
    # Alg. 3's second interpolation: a TT on the lattice F xi(lattice) onto
    # the axis-aligned box of the lattice's corners, against the oracle's
    # dense multilinear interpolation in the lattice coordinates
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from gpu_helpers import rand_pos_tt, to_dev
    from oracle import linear as lin
    from paper_2501_07942_amd import binding as B
    rng = np.random.default_rng(d)
    f = np.eye(d) + 0.15 * rng.standard_normal((d, d))
    lo_l, hi_l = -np.linspace(3.0, 4.0, d), np.linspace(2.0, 5.0, d)
    lo_t, hi_t = lin.lattice_box(f, lo_l, hi_l)
    src = rand_pos_tt(rng, [n] * d, [r] * (d - 1))
    tin = to_dev(B, src, B.F64, log_scale=0.4)
    outs = {dt: B.DeviceTT([n] * d, [1] + [64] * (d - 1) + [1], dt) for dt in (B.F64, B.F32)}
    lat = B.make_grid(d, [n] * d, list(lo_l), list(hi_l))
    tg = B.make_grid(d, [n] * d, list(lo_t), list(hi_t))
    for dt, o in outs.items():
        B.tt_interpolate_lattice(f, [lat], [tg], [tin], [o], 1e-12, 64)
    axes_l = mdl.grid_axes(lo_l, hi_l, [n] * d)
    want = lin.sheared_interp_dense(ttm.full(src) * np.exp(0.4), lo_l, mdl.spacings(axes_l), f,
                                    mdl.grid_axes(lo_t, hi_t, [n] * d))
    for dt, o in outs.items():
        cores, st = o.fetch_scaled()
        assert st == 0
        err = np.linalg.norm(ttm.full(cores) - want) / np.linalg.norm(want)
        print(f"lattice interpolation d={d} N={n} {'f64' if dt == B.F64 else 'f32'}: ranks {ttm.ranks(cores)} "
              f"rel {err:.1e}", flush=True)
        assert err <= (1e-10 if dt == B.F64 else 1e-6)
