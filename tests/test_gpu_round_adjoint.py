"""GPU adjoint of the rounding (tt_round_adjoint) against the oracle's
reverse mode of the same rounding at the same ranks, and against central
differences of the oracle's QR/SVD rounding."""
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
def B():
    import torch
    from paper_2501_07942_amd import binding
    assert torch.cuda.is_available()
    return binding


def rand_tt(rng, n, r, decay):
    rk = [1] + list(r) + [1]
    out = []
    for k in range(len(n)):
        g = rng.standard_normal((rk[k], n[k], rk[k + 1]))
        g *= decay ** np.arange(rk[k + 1])[None, None, :]
        out.append(g)
    return out


# modes, input ranks, rank cap, decay of the column scales; a batch shares d
CASES = [
    ([5, 4, 6, 3], [6, 10, 5], 4, 0.55),
    ([4, 7, 5, 6], [4, 8, 7], 3, 0.6),
]
CASES_D3 = [([6, 7, 5], [8, 9], 3, 0.6)]
# a wide first bond over rank-one bonds (the update rounding of the first step)
CASES_R1 = [([40, 6, 5, 4], [9, 1, 1], 8, 0.6)]
# unfoldings with n r = 4096 columns: the long products split their K
CASES_LONG = [([8, 64, 64, 6], [8, 64, 6], 5, 0.7)]


def run_case(B, cases, seed, taped=False):
    import torch
    rng = np.random.default_rng(seed)
    A, Y, YB, AB, host = [], [], [], [], []
    for n, r, cap, decay in cases:
        a = rand_tt(rng, n, r, decay)
        acap = [1] + [x + 2 for x in r] + [1]
        ta = B.DeviceTT(n, acap, B.F64)
        ta.load(a)
        ycap = [1] + [min(cap, x) for x in r] + [1]
        ty = B.DeviceTT(n, ycap, B.F64)
        A.append(ta)
        Y.append(ty)
        host.append((a, n, cap))
    tape = B.RoundTape(A) if taped else None
    for i, (a, n, cap) in enumerate(host):
        B.tt_round([A[i]], [Y[i]], 0.0, cap, tape=tape.select([i]) if taped else None)
    torch.cuda.synchronize()
    outs = []
    for i, (a, n, cap) in enumerate(host):
        ycores, ls, st = Y[i].fetch()
        assert st == 0
        t = rng.standard_normal(n)
        scale = math.exp(ls)
        yb = [scale * g for g in full_vjp(ycores, t)]
        sbar = scale * float(np.sum(ttm.full(ycores) * t))
        tyb = B.DeviceTT(n, Y[i].cap, B.F64)
        tyb.load(yb, sbar)
        YB.append(tyb)
        AB.append(B.DeviceTT(n, A[i].cap, B.F64))
        outs.append((a, [1] + [g.shape[2] for g in ycores], t, sbar))
    B.tt_round_adjoint(A, Y, YB, AB, tape=tape.structs if taped else None)
    torch.cuda.synchronize()
    if taped:
        outs = [o + (tape.valid[i].cpu().numpy(),) for i, o in enumerate(outs)]
    return outs, AB


@pytest.mark.parametrize("cases", [CASES, CASES_D3, CASES_R1, CASES_LONG],
                         ids=["d4_batch2", "d3", "rank_one_bonds", "long_products"])
def test_round_adjoint_with_forward_record(B, cases):
    """The adjoint fed the forward rounding's recorded right Grams and
    factors equals the one that recomputes them (same recursion, same
    thresholds), and the oracle's reverse mode."""
    print(f"round adjoint with record: {len(cases)} filter(s), d={len(cases[0][0])}", flush=True)
    outs0, AB0 = run_case(B, cases, 21)
    outs1, AB1 = run_case(B, cases, 21, taped=True)
    for (a, ranks, t, sbar, valid), o0, t0, t1 in zip(outs1, outs0, AB0, AB1):
        d = len(a)
        # every bond's Gram and factor is recorded (bond 1 folded with the
        # first core as such), and every left-to-right SVD of a tall unfolding
        want = [0] + [1 | 4] * (d - 1) + [0]
        if a[0].shape[2] > a[0].shape[1]:
            want[1] = 2  # its adjoint works from S_0: no SVD record
        assert list(valid) == want, valid
        ab0, _, _ = t0.fetch()
        ab1, ls, st = t1.fetch()
        assert st == 0 and ls == sbar
        y_or, tape = oa.round_fwd(a, ranks)
        ab_or = oa.round_vjp(tape, full_vjp(y_or, t))
        for k in range(d):
            sc = np.abs(ab_or[k]).max()
            assert np.abs(ab1[k] - ab0[k]).max() / sc < 1e-10, k
            assert np.abs(ab1[k] - ab_or[k]).max() / sc < 1e-8, k


@pytest.mark.parametrize("cases", [CASES, CASES_D3, CASES_R1, CASES_LONG],
                         ids=["d4_batch2", "d3", "rank_one_bonds", "long_products"])
def test_round_adjoint_matches_oracle_reverse_mode(B, cases):
    print(f"round adjoint: {len(cases)} filter(s), d={len(cases[0][0])}, binding caps", flush=True)
    outs, AB = run_case(B, cases, 21)
    for (a, ranks, t, sbar), tab in zip(outs, AB):
        y_or, tape = oa.round_fwd(a, ranks)
        ab_or = oa.round_vjp(tape, full_vjp(y_or, t))
        ab, ls, st = tab.fetch()
        assert st == 0 and ls == sbar
        for k in range(len(a)):
            err = np.abs(ab[k] - ab_or[k]).max() / np.abs(ab_or[k]).max()
            assert err < 1e-8, (k, err)


def test_round_adjoint_matches_differences_of_qr_svd_rounding(B):
    outs, AB = run_case(B, CASES_D3, 22)
    (a, ranks, t, sbar), tab = outs[0], AB[0]
    ab, _, _ = tab.fetch()
    rng = np.random.default_rng(23)
    da = [rng.standard_normal(g.shape) for g in a]

    def f(cores):
        return float(np.sum(ttm.full(ttm.tt_round(cores, 0.0, None, forced_ranks=ranks)) * t))

    h = 1e-6
    fd = (f([x + h * y for x, y in zip(a, da)]) - f([x - h * y for x, y in zip(a, da)])) / (2 * h)
    pred = sum(float(np.sum(x * y)) for x, y in zip(ab, da))
    assert abs(pred - fd) < 1e-7 * abs(fd)
