"""GPU adjoint of the likelihood build (tt_likelihood_dense,
tt_likelihood_adjoint): the range block's truncated SVD differentiated on
the GPU against the oracle's adjoint of the same build at the same rank,
for a gauge-invariant scalar <T, L> of the likelihood tensor."""
import math

import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import tt as ttm

import os, sys  # noqa: E401
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from adjoint_helpers import full_vjp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import binding, runner, workload
    assert torch.cuda.is_available()
    return binding, runner, workload


def lik_caps(s, cap):
    c = [1] * (s.d + 1)
    if s.meas_kind == "range":
        c[1] = min(cap, s.n)
    return c


@pytest.mark.parametrize("lik_tol", [1e-6, 1e-12])
def test_likelihood_adjoint_matches_oracle_svd_adjoint(mods, lik_tol):
    B, runner, wl = mods
    import dataclasses
    import torch
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=3, d=3, n=40, cap=6)
    specs = [dataclasses.replace(s, lik_tol=lik_tol) for s in specs]
    # one linear-model filter of the same d rides along (p_bar = l_bar there)
    lin = dataclasses.replace(specs[0], meas_kind="linear")
    _, zl = wl.simulate(lin, 3, np.random.SeedSequence(3))
    specs = specs + [lin]
    zs = list(zs) + [zl]
    print(f"likelihood adjoint: lik_tol {lik_tol}, 2 range + 1 linear filters, d=3, N=40", flush=True)
    z, _ = runner.z_tensor(zs)
    zk = z[:, 1, :].contiguous()
    grids = [runner.grid_of(s) for s in specs]
    meas = [runner.meas_of(s) for s in specs]
    L = [B.DeviceTT([s.n] * s.d, lik_caps(s, 64), B.F64) for s in specs]
    P = [B.DeviceTT([s.n] * s.d, lik_caps(s, s.n), B.F64) for s in specs]
    B.tt_likelihood(grids, meas, zk, L, 64)
    B.tt_likelihood_dense(grids, meas, zk, P)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    LB, host = [], []
    for s, l in zip(specs, L):
        lc, ls, st = l.fetch()
        assert st == 0
        t = rng.standard_normal([s.n] * s.d)
        sc = math.exp(ls)
        lb = [sc * g for g in full_vjp(lc, t)]
        sbar = sc * float(np.sum(ttm.full(lc) * t))
        tb = B.DeviceTT([s.n] * s.d, l.cap, B.F64)
        tb.load(lb, sbar)
        LB.append(tb)
        host.append((lc, ls, t, lb, sbar))
    PB = [B.DeviceTT(p.n, p.cap, B.F64) for p in P]
    B.tt_likelihood_adjoint(meas, P, L, LB, PB)
    torch.cuda.synchronize()
    for s, p, pb, (lc, ls, t, lb, sbar) in zip(specs, P, PB, host):
        pc, pls, pst = p.fetch()
        bc, bls, bst = pb.fetch()
        assert pst == 0 and bst == 0
        assert pls == ls
        assert bls == sbar
        if s.meas_kind != "range":
            for a, b in zip(bc, lb):
                assert np.array_equal(a, b)
            continue
        m = pc[0][0]
        r = lc[0].shape[2]
        # the build at the GPU's rank, differentiated by the oracle
        v, sig, _ = np.linalg.svd(m.T, full_matrices=False)
        vr = v[:, :r]
        oc = [(m @ vr).reshape(1, -1, r), vr.T.reshape(r, -1, 1)] + list(lc[2:])
        assert np.linalg.norm(ttm.full(oc) - ttm.full(lc)) < 1e-10 * np.linalg.norm(ttm.full(lc))
        ob = [math.exp(ls) * g for g in full_vjp(oc, t)]
        mbar = oa._lik_vjp({"m": m, "v": v, "sig": sig, "r": r}, ob)
        err = np.abs(bc[0][0] - mbar).max() / np.abs(mbar).max()
        print(f"  rank {r}, sigma_r/sigma_1 {sig[r - 1] / sig[0]:.1e}: Mbar rel {err:.2e}", flush=True)
        assert err < 1e-7
        assert not np.any(bc[1])
        for a, b in zip(bc[2:], lb[2:]):
            assert np.array_equal(a, b)


def test_update_adjoint_matches_oracle(mods):
    # tt_update_adjoint for g = <full(H), T> + w log c_k on two range filters
    # and (a call of its own: the parameter layout differs) one linear
    # filter, d = 3, N = 40: the adjoint of P_pred and the measurement-
    # parameter gradient against the oracle's reverse mode of the same update
    # (likelihood build with its SVD adjoint, Hadamard, the log c_k term)
    B, runner, wl = mods
    import dataclasses
    import torch
    from oracle import model as mdl
    specs, xs, zs = wl.make_batch("range4d", batch=2, steps=3, d=3, n=40, cap=6)
    lin = dataclasses.replace(specs[0], meas_kind="linear")
    _, zl = wl.simulate(lin, 3, np.random.SeedSequence(3))
    rng = np.random.default_rng(23)
    for group, gz in (((specs[0], specs[1]), (zs[0], zs[1])), ((lin,), (zl,))):
        z, _ = runner.z_tensor(list(gz))
        zk = z[:, 1, :].contiguous()
        grids = [runner.grid_of(s) for s in group]
        meas = [runner.meas_of(s) for s in group]
        P, H, HB, PB, refs = [], [], [], [], []
        for s in group:
            pc = [np.abs(g) + 0.05 for g in (rng.standard_normal((1, s.n, 3)), rng.standard_normal((3, s.n, 2)),
                                             rng.standard_normal((2, s.n, 1)))]
            P.append(B.DeviceTT([s.n] * 3, [1, 3, 2, 1], B.F64))
            P[-1].load(pc)
            lc = 40 if s.meas_kind == "range" else 1
            H.append(B.DeviceTT([s.n] * 3, [1, 3 * lc, 2, 1], B.F64))
            PB.append(B.DeviceTT([s.n] * 3, [1, 3, 2, 1], B.F64))
            refs.append(pc)
        log_c = torch.zeros(len(group), dtype=torch.float64, device="cuda")
        B.tt_update(grids, meas, zk, P, H, 40, log_c)
        torch.cuda.synchronize()
        w = rng.standard_normal(len(group))
        nth = 7 if group[0].meas_kind == "range" else 4
        theta = torch.zeros(len(group), nth, dtype=torch.float64, device="cuda")
        ts = []
        for f, s in enumerate(group):
            hc, hls, hst = H[f].fetch()
            assert hst == 0
            t = rng.standard_normal([s.n] * 3)
            ts.append(t)
            hb = B.DeviceTT([s.n] * 3, H[f].cap, B.F64)
            hb.load([g * math.exp(hls) for g in full_vjp(hc, t)], float(np.sum(ttm.full(hc) * t)) * math.exp(hls))
            HB.append(hb)
        lcb = torch.tensor(w, dtype=torch.float64, device="cuda")
        print(f"update adjoint: {len(group)} {group[0].meas_kind} filter(s), d=3, N=40", flush=True)
        B.tt_update_adjoint(grids, meas, zk, P, H, HB, lcb, 40, PB, theta)
        torch.cuda.synchronize()
        th = theta.cpu().numpy()
        zh = zk.cpu().numpy()
        for f, s in enumerate(group):
            axes = mdl.grid_axes(s.lo, s.hi, [s.n] * s.d)
            delta = mdl.cell_volume(axes)
            m = s.meas()
            lik, ltape = oa._lik_fwd(axes, zh[f], m, s.lik_tol)
            h = ttm.hadamard(lik, refs[f])
            c = ttm.tt_sum(h) * delta
            hbar = full_vjp(h, ts[f])
            oa.tt_axpy(hbar, oa.sum_vjp(h, w[f] * delta / c))
            lbar, pbar = oa.hadamard_vjp(lik, refs[f], hbar)
            thb = np.zeros(nth)
            oa._lik_theta(thb, lbar, {"ltape": ltape}, axes, zh[f], m, 3)
            pb, _, st = PB[f].fetch()
            assert st == 0
            err_p = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(pb, pbar))
            err_t = float(np.abs(th[f, 3:] - thb[3:]).max() / max(1e-300, np.abs(thb[3:]).max()))
            print(f"  filter {f}: p_pred_bar {err_p:.1e}, theta_bar {err_t:.1e}", flush=True)
            assert err_p < 1e-10
            assert err_t < 1e-7
            assert np.all(th[f, :3] == 0.0)
