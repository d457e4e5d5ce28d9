"""GPU parity of the full control set (section "6-DoF Powered Descent Guidance"): the
reaction-control torque gamma joins the thrust, u = (T, gamma, s), with its bound through the
CTCS integrand; the paper's Monte Carlo with the torque (workload F2) against the oracle built
with n_u = 7, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2404_18034_amd import api
from paper_2404_18034_amd import instances as I
from test_gpu_parity import TOL_F64, _errors, _gpu, _report, _valid, check_fp32_bar

pytestmark = pytest.mark.gpu


def test_torque_short_horizon_fp64_uneven_k():
    # every instance, K in {10, 20, 30}, three subproblems of 300 PIPG steps
    print("case: torque, 24 runs, K in {10,20,30}, 3 x 300, fp64", flush=True)
    cfg = I.solver_settings("F2", scp_iters_max=3, pipg_iters_max=300, early_exit=0)
    inst = I.make_instances("F2", B=24)
    inst["K"] = np.array([10, 20, 30] * 8, dtype=np.int32)
    g = _gpu(cfg, inst, "f64", k_max=30)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    assert g["u"].shape[-1] == 7
    errs = _errors(cfg, g, o)
    _report("torque fp64 3 subproblems", errs)
    for e in errs:
        assert e.max() <= TOL_F64
    # the torque is in use
    assert np.abs(g["u"][:, :, 3:6]).max() > 1e-3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_torque_monte_carlo_whole_solve(dtype):
    # 64 runs of the paper's Monte Carlo with the torque (at most 25 SCP iterations of 2,500
    # PIPG iterations, SCP early exit): statuses, iteration counts and trajectories
    print("case: torque, 64 runs, whole solve, %s" % dtype, flush=True)
    cfg = I.solver_settings("F2")
    inst = I.make_instances("F2", B=64)
    g = _gpu(cfg, inst, dtype, k_max=30)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    print("oracle status counts %s, GPU %s" % (np.bincount(o["status"], minlength=3).tolist(),
                                                np.bincount(g["status"], minlength=3).tolist()))
    if dtype == "f64":
        errs = _errors(cfg, g, o)
        _report("torque fp64 whole solve", errs)
        for e in errs:
            assert e.max() <= TOL_F64
        for k in ("status", "scp_iters", "pipg_iters"):
            np.testing.assert_array_equal(g[k], o[k])
    else:
        check_fp32_bar(cfg, inst, g, o, "torque fp32 whole solve")
    _valid(g, inst)
    gam = np.linalg.norm(g["u"][:, :, 3:6], axis=2)
    assert gam.max() <= inst["params"][0, 23] * 1.1


@pytest.mark.parametrize("mode,occupancy", [(1, 0), (2, 0), (3, 0), (4, 0), (0, 5), (1, 6)])
def test_torque_dispatch_modes_match_plain_launches(mode, occupancy):
    import torch
    print("case: torque, 40 runs, mode %d occupancy %d" % (mode, occupancy), flush=True)
    cfg = I.solver_settings("F2", scp_iters_max=4, pipg_iters_max=300, pipg_check_every=10)
    inst = I.make_instances("F2", B=40)
    inst["K"] = np.array([10, 20, 30, 13, 27] * 8, dtype=np.int32)
    ref = _gpu(cfg, inst, "f32", k_max=30)
    s = api.BatchSolver(dict(cfg, mode=mode, occupancy=occupancy), dtype="f32", k_max=30,
                        max_batch=64)
    try:
        prob = s.to_device(inst)
        sol = s.alloc_solution(40)
        for rep in range(2):
            for v in sol.values():
                v.zero_()
            s.solve_into(prob, sol)
            torch.cuda.synchronize()
            for k in ref:
                np.testing.assert_array_equal(sol[k].cpu().numpy(), ref[k],
                                              err_msg="%s rep %d" % (k, rep))
    finally:
        s.close()


def test_torque_node_counts_up_to_50_fp64():
    # the 1,024-lane workgroup variant with the torque layout, every node-wise set on
    print("case: torque, K up to 50, fp64, 2 x 200", flush=True)
    cfg = I.solver_settings("F2", node_projections=31, scp_iters_max=2, pipg_iters_max=200,
                            early_exit=0)
    inst = I.make_instances("F2", B=6)
    inst["K"] = np.array([41, 50, 44, 12, 47, 2], dtype=np.int32)
    g = _gpu(cfg, inst, "f64", k_max=50)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=50)
    errs = _errors(cfg, g, o)
    _report("torque K<=50 fp64", errs)
    for e in errs:
        assert e.max() <= TOL_F64


def test_torque_select_best_copies_seven_controls():
    # multi-start choice on torque solutions: the chosen start's trajectory, all 7 controls
    import torch
    cfg = I.solver_settings("F2", scp_iters_max=3, pipg_iters_max=200, early_exit=0)
    inst = I.make_instances("F2", B=4)
    rep = I.multistart(inst, (4.0, 6.0))
    s = api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=8)
    try:
        prob = s.to_device(rep)
        sol = s.alloc_solution(8)
        s.solve_into(prob, sol)
        best, out = s.select_best(sol, 4, 2)
        torch.cuda.synchronize()
        every = {k: v.cpu().numpy() for k, v in sol.items()}
        b = best.cpu().numpy()
        o = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        s.close()
    expect = oracle.select_best(every["status"], every["objective"], 4, 2)
    np.testing.assert_array_equal(b, expect)
    assert o["u"].shape[-1] == 7
    src = np.arange(4) * 2 + np.maximum(expect, 0)
    for k in every:
        np.testing.assert_array_equal(o[k], every[k][src], err_msg=k)


@pytest.mark.parametrize("over", [dict(scalar_dilation=1), dict(grad_pipg_steps=20, grad_ckpt_every=5)])
def test_torque_unsupported_combinations(over):
    cfg = I.solver_settings("F2", **over)
    with pytest.raises(api.ScpError) as e:
        api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=8)
    assert e.value.code == 8
