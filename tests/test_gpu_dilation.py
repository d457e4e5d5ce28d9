"""GPU parity of the scalar-dilation variant (one dilation value over the horizon) against
the oracle, through the C ABI.

The variant restricts every subproblem to s_1 = ... = s_K; the GPU kernel projects the
dilation values onto their mean (summed in node order through LDS), the oracle does the
same projection in FP64 with plain loops.
"""
import numpy as np
import pytest

import oracle
from paper_2404_18034_amd import api
from paper_2404_18034_amd import instances as I
from test_gpu_parity import TOL_F64, _errors, _gpu, _report, _valid, check_fp32_bar

pytestmark = pytest.mark.gpu


def _one_value(g, inst):
    for b in range(len(inst["K"])):
        s = g["u"][b, :inst["K"][b], 3]
        assert np.ptp(s) == 0.0, "instance %d holds more than one dilation value" % b


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scalar_dilation_short_horizon_all_instances(dtype):
    # mixed K in one batch, three subproblems, every instance
    print("case: scalar dilation, C2 x 24, 3 subproblems, %s" % dtype, flush=True)
    cfg = I.solver_settings("C2", scalar_dilation=1, scp_iters_max=3, early_exit=0)
    inst = I.make_instances("C2", B=24)
    g = _gpu(cfg, inst, dtype, k_max=30)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    _one_value(g, inst)
    if dtype == "f64":
        errs = _errors(cfg, g, o)
        _report("C2 scalar dilation fp64 3 subproblems", errs)
        for e in errs:
            assert e.max() <= TOL_F64
    else:
        assert check_fp32_bar(cfg, inst, g, o, "C2 scalar dilation fp32 3 subproblems").all()


def test_scalar_dilation_full_solve_fp64():
    # whole solves with early exit: statuses, iteration counts and trajectories on every
    # instance
    print("case: scalar dilation, C2 x 24, full solve, f64", flush=True)
    cfg = I.solver_settings("C2", scalar_dilation=1)
    inst = I.make_instances("C2", B=24)
    g = _gpu(cfg, inst, "f64", k_max=30)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    print("oracle status counts %s" % np.bincount(o["status"], minlength=3).tolist())
    errs = _errors(cfg, g, o)
    _report("C2 scalar dilation fp64", errs)
    for e in errs:
        assert e.max() <= TOL_F64
    for k in ("status", "scp_iters", "pipg_iters"):
        np.testing.assert_array_equal(g[k], o[k])
    _one_value(g, inst)
    np.testing.assert_allclose(g["t_f"], g["u"][:, 0, 3], rtol=1e-14)


def test_scalar_dilation_fp32_monte_carlo_sample():
    # the 1,024-instance Monte Carlo configuration (15 SCP x 1,000 PIPG, fixed work) on a
    # 32-instance sample, FP32 against the oracle at the fixed FP32 bar
    # (runs the oracle itself leaves non-finite are dropped from the sample first)
    print("case: scalar dilation, C1 x 32, f32", flush=True)
    cfg = I.solver_settings("C1", scalar_dilation=1)
    inst = I.make_instances("C1", B=32)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    ids = np.flatnonzero(o["status"] != 2)
    assert ids.size >= 28
    inst = I.make_instances("C1", ids=ids)
    o = {k: v[ids] for k, v in o.items()}
    g = _gpu(cfg, inst, "f32")
    _valid(g, inst)
    _one_value(g, inst)
    assert check_fp32_bar(cfg, inst, g, o, "C1 scalar dilation fp32").all()


@pytest.mark.parametrize("mode", [1, 2, 4])
def test_scalar_dilation_dispatch_modes_match_plain_launches(mode):
    # graph replay, K-ordered dispatch and the K-bucketed launches compute the same thing as
    # plain launches, bit for bit
    import torch
    print("case: scalar dilation, C2 x 40, mode %d" % mode, flush=True)
    cfg = I.solver_settings("C2", scalar_dilation=1)
    inst = I.make_instances("C2", B=40)
    ref = _gpu(cfg, inst, "f32", k_max=30)
    s = api.BatchSolver(dict(cfg, mode=mode), dtype="f32", k_max=30, max_batch=64)
    try:
        sol = s.solve(s.to_device(inst))
        torch.cuda.synchronize()
        for k in ref:
            np.testing.assert_array_equal(sol[k].cpu().numpy(), ref[k], err_msg=k)
    finally:
        s.close()


@pytest.mark.parametrize("over", [dict(mode=3), dict(grad_pipg_steps=20, grad_ckpt_every=5)])
def test_scalar_dilation_unsupported_combinations(over):
    cfg = I.solver_settings("C2", scalar_dilation=1, **over)
    with pytest.raises(api.ScpError) as e:
        api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=8)
    assert e.value.code == 8


def test_scalar_dilation_autotune_times_modes_1_2_4_only():
    # one register budget whatever the occupancy setting, no persistent form: the autotuner
    # times (1, 0), (2, 0) and (4, 0) and keeps the results of plain launches
    import torch
    print("case: scalar dilation, autotune, C2 x 40", flush=True)
    cfg = I.solver_settings("C2", scalar_dilation=1)
    inst = I.make_instances("C2", B=40)
    ref = _gpu(cfg, inst, "f32", k_max=30)
    s = api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=64)
    try:
        prob = s.to_device(inst)
        sol = s.alloc_solution(40)
        best, ms = s.autotune(prob, sol)
        assert set(ms) == {(1, 0), (2, 0), (4, 0)}, ms
        assert best in ms
        s.solve_into(prob, sol)
        torch.cuda.synchronize()
        for k in ref:
            np.testing.assert_array_equal(sol[k].cpu().numpy(), ref[k], err_msg=k)
    finally:
        s.close()
