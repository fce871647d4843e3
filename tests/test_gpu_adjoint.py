"""GPU adjoints of the linear steps (tt_predict_adjoint, tt_hadamard_adjoint,
tt_normalize_adjoint) against the oracle's reverse-mode functions, element
by element, on seeded random trains spanning several tiles and ragged
ranks."""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import tt as ttm

import os, sys  # noqa: E401
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from adjoint_helpers import full_vjp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2501_07942_amd import binding
    assert torch.cuda.is_available()
    return binding


def rand_tt(rng, n, r):
    rk = [1] + list(r) + [1]
    return [rng.standard_normal((rk[k], n[k], rk[k + 1])) for k in range(len(n))]


def dev(B, cores, cap, prec, log_scale=0.0):
    t = B.DeviceTT([g.shape[1] for g in cores], cap, prec)
    t.load(cores, log_scale)
    return t


def empty_like(B, cores, cap, prec):
    return B.DeviceTT([g.shape[1] for g in cores], cap, prec)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


TOL = {"f64": 1e-12, "f32": 2e-5}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_predict_adjoint_matches_oracle(B, prec):
    import torch
    pr = B.F64 if prec == "f64" else B.F32
    rng = np.random.default_rng(7)
    n = [37, 29, 41]
    batch = []
    for f, (rp, rk, taps) in enumerate([([3, 5], [2, 4], [5, 7, 3]), ([6, 2], [3, 3], [9, 3, 5])]):
        p = rand_tt(rng, n, rp)
        k = rand_tt(rng, taps, rk)
        hw = [(t - 1) // 2 for t in taps]
        c = ttm.conv(k, p, hw)
        cb = [rng.standard_normal(g.shape) for g in c]
        kb_o, pb_o = oa.conv_vjp(k, p, hw, cb)
        batch.append((p, k, cb, kb_o, pb_o))
    print(f"predict adjoint {prec}: 2 filters, n={n}", flush=True)
    pcap, kcap, ccap = [1, 8, 8, 1], [1, 4, 4, 1], [1, 32, 32, 1]
    P = [dev(B, x[0], pcap, pr) for x in batch]
    K = [dev(B, x[1], kcap, pr) for x in batch]
    CB = [dev(B, x[2], ccap, pr, log_scale=0.25) for x in batch]
    PB = [empty_like(B, x[0], pcap, pr) for x in batch]
    KB = [empty_like(B, x[1], kcap, pr) for x in batch]
    B.tt_predict_adjoint(K, P, CB, PB, KB)
    torch.cuda.synchronize()
    for f, x in enumerate(batch):
        pb, ls, st = PB[f].fetch()
        kb, lsk, stk = KB[f].fetch()
        assert st == 0 and stk == 0 and ls == 0.25 and lsk == 0.25
        for k in range(3):
            assert rel(pb[k], x[4][k]) < TOL[prec], (f, k)
            assert rel(kb[k], x[3][k]) < TOL[prec], (f, k)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hadamard_adjoint_matches_oracle(B, prec):
    import torch
    pr = B.F64 if prec == "f64" else B.F32
    rng = np.random.default_rng(8)
    n = [33, 18, 21, 5]
    la = rand_tt(rng, n, [7, 1, 1])
    pb_ = rand_tt(rng, n, [5, 6, 3])
    hb = [rng.standard_normal(g.shape) for g in ttm.hadamard(la, pb_)]
    ab_o, bb_o = oa.hadamard_vjp(la, pb_, hb)
    print(f"hadamard adjoint {prec}: n={n}", flush=True)
    A = dev(B, la, [1, 8, 2, 2, 1], B.F64)
    Bt = dev(B, pb_, [1, 6, 6, 4, 1], pr)
    HB = dev(B, hb, [1, 48, 12, 8, 1], pr, log_scale=-1.5)
    AB = empty_like(B, la, [1, 8, 2, 2, 1], B.F64)
    BB = empty_like(B, pb_, [1, 6, 6, 4, 1], pr)
    B.tt_hadamard_adjoint([A], [Bt], [HB], [AB], [BB])
    torch.cuda.synchronize()
    ab, lsa, sta = AB.fetch()
    bb, lsb, stb = BB.fetch()
    assert sta == 0 and stb == 0 and lsa == -1.5 and lsb == -1.5
    for k in range(4):
        assert rel(ab[k], ab_o[k]) < TOL[prec], k
        assert rel(bb[k], bb_o[k]) < TOL[prec], k


def test_hadamard_adjoint_flags_mismatched_ranks(B):
    import torch
    rng = np.random.default_rng(9)
    n = [6, 7]
    la = rand_tt(rng, n, [2])
    pb_ = rand_tt(rng, n, [3])
    wrong = rand_tt(rng, n, [5])      # not 2 * 3
    A = dev(B, la, [1, 2, 1], B.F64)
    Bt = dev(B, pb_, [1, 3, 1], B.F64)
    HB = dev(B, wrong, [1, 6, 1], B.F64)
    BB = empty_like(B, pb_, [1, 3, 1], B.F64)
    B.tt_hadamard_adjoint([A], [Bt], [HB], None, [BB])
    torch.cuda.synchronize()
    assert BB.fetch()[2] == 4   # TT_STATUS_CAPACITY


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [([9, 11, 7], [4, 3]), ([6, 13, 5, 4], [300, 70, 2])],
                         ids=["small", "wide_bonds"])
def test_normalize_adjoint_matches_oracle(B, prec, shape):
    # downstream g(P) = <full(P), T> + w * log m for P = X / (sum(X) delta):
    # the GPU representation keeps the cores and moves the scale into the
    # log-scale; both must give the same derivative with respect to X's cores
    import math
    import torch
    pr = B.F64 if prec == "f64" else B.F32
    rng = np.random.default_rng(10)
    n, r = shape
    caps = [1] + list(r) + [1]
    x = [np.abs(g) + 0.2 for g in rand_tt(rng, n, r)]
    delta = 0.37
    t = rng.standard_normal(n)
    w = 0.8
    s = ttm.tt_sum(x)
    m = s * delta
    p_or = ttm.scale(x, 1.0 / m)
    # oracle: P = scale(X, 1/m) with m = sum(X) delta, plus w log m
    pbar_or = full_vjp(p_or, t)
    xbar_or, cb = oa.scale_vjp(x, 1.0 / m, pbar_or)
    mbar = -cb / m ** 2 + w / m
    oa.tt_axpy(xbar_or, oa.sum_vjp(x, mbar * delta))
    # GPU: P keeps X's cores, log_scale(P) = -log(S delta)
    ls_p = -math.log(s * delta)
    pbar_gpu = [g * math.exp(ls_p) for g in full_vjp(x, t)]
    sbar_p = float(np.sum(ttm.full(x) * t)) * math.exp(ls_p)
    X = dev(B, x, caps, pr)
    PB = dev(B, pbar_gpu, caps, pr, log_scale=sbar_p)
    XB = empty_like(B, x, caps, pr)
    lmb = torch.tensor([w], dtype=torch.float64, device="cuda")
    print(f"normalize adjoint {prec}: n={n}", flush=True)
    B.tt_normalize_adjoint([X], [PB], lmb, [XB])
    torch.cuda.synchronize()
    xb, ls, st = XB.fetch()
    assert st == 0 and ls == w
    for k in range(len(n)):
        assert rel(xb[k], xbar_or[k]) < (1e-12 if prec == "f64" else 1e-5), k


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_normalize_moments_adjoint_matches_oracle(B, prec):
    # the normalisation's adjoint plus that of the moments: downstream
    # g = <full(P), T> + w log m + <mb, mean> + <cb, cov>, a batch of two
    # filters with different grids and ranks; the oracle adds moments_vjp
    import math
    import torch
    from oracle import model as mdl
    pr = B.F64 if prec == "f64" else B.F32
    rng = np.random.default_rng(12)
    shapes = [([9, 11, 7], [4, 3], [-2.0, -1.0, 0.5], [3.0, 2.5, 4.0]),
              ([6, 13, 5], [2, 5], [0.0, -4.0, -1.0], [1.5, 4.0, 2.0])]
    X, PB, XB, grids, refs = [], [], [], [], []
    mbs, cbs, lms = [], [], []
    for n, r, lo, hi in shapes:
        caps = [1] + list(r) + [1]
        x = [np.abs(g) + 0.2 for g in rand_tt(rng, n, r)]
        axes = mdl.grid_axes(lo, hi, n)
        delta = mdl.cell_volume(axes)
        t = rng.standard_normal(n)
        w = float(rng.standard_normal())
        mb = rng.standard_normal(3)
        cb = rng.standard_normal((3, 3))
        s = ttm.tt_sum(x)
        m = s * delta
        p_or = ttm.scale(x, 1.0 / m)
        pbar_or = full_vjp(p_or, t)
        xbar_or, cbs_ = oa.scale_vjp(x, 1.0 / m, pbar_or)
        oa.tt_axpy(xbar_or, oa.sum_vjp(x, (-cbs_ / m ** 2 + w / m) * delta))
        oa.tt_axpy(xbar_or, oa.moments_vjp(x, axes, mb, cb))
        refs.append(xbar_or)
        ls_p = -math.log(s * delta)
        pbar_gpu = [g * math.exp(ls_p) for g in full_vjp(x, t)]
        sbar_p = float(np.sum(ttm.full(x) * t)) * math.exp(ls_p)
        X.append(dev(B, x, caps, pr))
        PB.append(dev(B, pbar_gpu, caps, pr, log_scale=sbar_p))
        XB.append(empty_like(B, x, caps, pr))
        grids.append(B.make_grid(3, n, lo, hi))
        mbs.append(mb)
        cbs.append(cb)
        lms.append(w)
    lmb = torch.tensor(lms, dtype=torch.float64, device="cuda")
    mbt = torch.tensor(np.stack(mbs), dtype=torch.float64, device="cuda")
    cbt = torch.tensor(np.stack(cbs), dtype=torch.float64, device="cuda")
    print(f"normalize + moments adjoint {prec}: 2 filters", flush=True)
    B.tt_normalize_moments_adjoint(grids, X, PB, lmb, XB, mbt, cbt)
    torch.cuda.synchronize()
    for f, ref in enumerate(refs):
        xb, ls, st = XB[f].fetch()
        assert st == 0 and ls == lms[f]
        for k in range(3):
            assert rel(xb[k], ref[k]) < (1e-11 if prec == "f64" else 1e-4), (f, k, rel(xb[k], ref[k]))
