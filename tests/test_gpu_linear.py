"""The filter for linear dynamics on re-designed grids (Alg. 3 with Alg. 4:
tt_filter_run_linear) against the oracle's run of the same recursion, on the
paper's 2-D dynamics F = [[1.1, 0.1], [-0.2, 1.1]], Q = I (Sec. 5), with
linear measurements and with the range model, and at d = 3 with a sheared
F: the grids of every step, log c_k, the predictive mass and the means."""
import numpy as np
import pytest

from oracle import linear as lin

pytestmark = pytest.mark.gpu

F_PAPER = np.array([[1.1, 0.1], [-0.2, 1.1]])


def make(d, f, kind, n, steps, seed):
    from paper_2501_07942_amd import workload as wl
    rng = np.random.default_rng(seed)
    q = np.eye(d)
    x = np.zeros((steps, d))
    x[0] = rng.normal(0.0, 2.0, d)
    for k in range(1, steps):
        x[k] = f @ x[k - 1] + rng.standard_normal(d)
    spec = wl.FilterSpec(d=d, n=n, lo=-10.0, hi=10.0, q=q, truncate_kernel=True, meas_kind=kind,
                         m0=np.zeros(d), p0_diag=np.full(d, 4.0), cap=16)
    if kind == "linear":
        z = x + rng.standard_normal((steps, d))
    else:
        rho = np.hypot(x[:, 0] - spec.sensor[0], x[:, 1] - spec.sensor[1])
        z = np.concatenate([(rho + spec.sigma_r * rng.standard_normal(steps))[:, None],
                            x[:, 2:] + rng.standard_normal((steps, d - 2))], axis=1)
    return spec, q, z


@pytest.mark.parametrize("d,kind,n", [(2, "linear", 48), (2, "range", 64), (3, "linear", 24)])
def test_linear_dynamics_filter_matches_oracle(d, kind, n):
    import torch
    from paper_2501_07942_amd import binding as B, runner
    f = F_PAPER if d == 2 else np.array([[1.05, 0.1, 0.0], [-0.15, 1.0, 0.05], [0.0, 0.1, 0.95]])
    steps = 8
    spec, q, z = make(d, f, kind, n, steps, 20 + d)
    print(f"linear dynamics: d={d} {kind} N={n} {steps} steps", flush=True)
    fs = runner.filter_specs([spec], [0], 16, 64)
    zt = torch.tensor(z[None, :, :], dtype=torch.float64, device="cuda")
    out = B.filter_run_linear(fs, f, q, zt)
    torch.cuda.synchronize()
    assert int(out["status"].cpu()[0]) == 0
    ref = lin.run_tt_filter_linear(f, q, spec.meas(), z, spec.m0, spec.p0_diag, [spec.lo] * d, [spec.hi] * d, n,
                                   spec.cap, spec.eps)
    grids = out["grids"][0]
    err_g = max(np.abs(grids[:, :d] - ref["grid_lo"]).max(), np.abs(grids[:, d:] - ref["grid_hi"]).max())
    lc = out["log_c"].cpu().numpy()[0]
    lm = out["log_mpred"].cpu().numpy()[0, 1:]
    mean = out["mean"].cpu().numpy()[0]
    dx = (ref["grid_hi"] - ref["grid_lo"]) / (n - 1)
    err_c = float(np.abs(lc - ref["log_c"]).max())
    err_mp = float(np.abs(lm - ref["log_mpred"]).max())
    err_m = float((np.abs(mean - ref["mean"]) / dx).max())
    print(f"  grids {err_g:.1e} |dlog c| {err_c:.1e} |dlog m_pred| {err_mp:.1e} |dmean|/dx {err_m:.1e}", flush=True)
    assert err_g <= 1e-9
    assert err_c <= 1e-8 * max(1.0, float(np.abs(ref["log_c"]).max()))
    assert err_mp <= 1e-8
    assert err_m <= 1e-8
    assert abs(float(out["loglik"].cpu()[0]) - ref["loglik"]) <= 1e-8 * abs(ref["loglik"])
