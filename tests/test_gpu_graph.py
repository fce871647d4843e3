"""A filter step recorded as a HIP graph (tt_filter_graph_*) and replayed
as a streaming filter: every replay must equal the eager recursion bit for
bit, with eager work and synchronisations between the replays."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    from paper_2501_07942_amd import binding, runner, workload
    assert torch.cuda.is_available()
    return binding, runner, workload


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_graph_replays_equal_the_eager_recursion(mods, precision):
    B, runner, wl = mods
    import torch
    prec = B.F64 if precision == "f64" else B.F32
    K = 6
    specs, xs, zs = wl.make_batch("range4d", batch=3, steps=K, d=3, n=32, cap=6)
    print(f"graph replay: {precision}, B=3, d=3, N=32, cap 6, K={K}", flush=True)
    ref, z = runner.run_filters(specs, zs, prec)
    kernels, kidx, kr = runner.build_kernels(specs, prec)
    fspecs = runner.filter_specs(specs, kidx, kr, 64)
    # streaming run over a two-row measurement buffer: row 0 for the prior
    # update, row 1 rewritten before every replay of the steady step
    zs2 = z[:, :2, :].clone()
    run = B.FilterRun(fspecs, kernels, 2, z.shape[2], prec)
    run(zs2, k_begin=0, k_count=1)
    g = run.graph(zs2, k_begin=1, k_count=1)
    lc_ref = ref.log_c.cpu().numpy()
    mean_ref = ref.mean.cpu().numpy()
    ranks_ref = ref.ranks.cpu().numpy()
    for k in range(1, K):
        zs2[:, 1, :].copy_(z[:, k, :])
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(run.log_c[:, 1].cpu().numpy(), lc_ref[:, k]), k
        assert np.array_equal(run.mean[:, 1].cpu().numpy(), mean_ref[:, k]), k
        assert np.array_equal(run.ranks[:, 1].cpu().numpy(), ranks_ref[:, k]), k
        # unrelated eager work between replays
        torch.ones(1000, device="cuda").sum().item()
    assert int(run.status.abs().sum().item()) == 0
    g.destroy()


def test_graph_create_rejects_step_zero(mods):
    B, runner, wl = mods
    specs, xs, zs = wl.make_batch("range4d", batch=1, steps=3, d=3, n=24, cap=4)
    kernels, kidx, kr = runner.build_kernels(specs, B.F64)
    z, zdim = runner.z_tensor(zs)
    run = B.FilterRun(runner.filter_specs(specs, kidx, kr, 64), kernels, 3, zdim, B.F64)
    with pytest.raises(B.TTError):
        run.graph(z, k_begin=0)


def test_autotuned_prediction_shape_changes_no_result_bit(mods):
    # the tuner picks the fibres per workgroup of the matrix-core prediction;
    # a run after tuning equals the run before it bit for bit
    B, runner, wl = mods
    import torch
    K = 9
    specs, xs, zs = wl.make_batch("range4d", batch=4, steps=K, d=4, n=48, cap=8)
    print("autotune: FP32, B=4, d=4, N=48, cap 8", flush=True)
    before, z = runner.run_filters(specs, zs, B.F32)
    kernels, kidx, kr = runner.build_kernels(specs, B.F32)
    run = B.FilterRun(runner.filter_specs(specs, kidx, kr, 64), kernels, K, z.shape[2], B.F32)
    res = run.autotune(z, warmup_steps=0, rounds=2)
    torch.cuda.synchronize()
    assert res["best_bb"] in (2, 4, 8, 16)
    assert all(v > 0 for v in res["ms_per_step"].values())
    run(z)
    torch.cuda.synchronize()
    assert np.array_equal(run.log_c.cpu().numpy(), before.log_c.cpu().numpy())
    assert np.array_equal(run.mean.cpu().numpy(), before.mean.cpu().numpy())
    # the decision persists: saved as JSON keyed by architecture and shape,
    # adopted again by a load; entries of another architecture are ignored
    import json
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        path = tmp + "/tune.json"
        B.autotune_save(path)
        entries = json.load(open(path))
        mine = [e for e in entries if e["batch"] == 4 and e["n"] == 48 and e["dtype"] == "f32"]
        assert len(mine) == 1 and mine[0]["value"] == res["best_bb"]
        assert mine[0]["arch"].startswith("gfx") and mine[0]["rank_cap"] == 8
        assert B.autotune_load(path) == len(entries)
        other = [dict(e, arch="gfx000") for e in entries]
        json.dump(other, open(tmp + "/other.json", "w"))
        assert B.autotune_load(tmp + "/other.json") == 0
        open(tmp + "/bad.json", "w").write('[{"arch": "gfx950", "value": 3}]')
        with pytest.raises(B.TTError):
            B.autotune_load(tmp + "/bad.json")
