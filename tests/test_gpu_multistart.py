"""Multi-start on the GPU (scp_batch_select_best): the selection kernel against the oracle's
choice on synthetic solutions (ties, no converged start, one start), argument validation,
and the whole multi-start solve of the paper's Monte Carlo at K = 20 against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2404_18034_amd import api
from paper_2404_18034_amd import instances as I

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-9


def _fake_solution(solver, n, rng):
    import torch
    sol = solver.alloc_solution(n)
    dt = solver.dtype
    sol["x"].copy_(torch.as_tensor(rng.normal(size=tuple(sol["x"].shape)), dtype=dt))
    sol["u"].copy_(torch.as_tensor(rng.normal(size=tuple(sol["u"].shape)), dtype=dt))
    for k in ("t_f", "m_f", "defect_inf", "ctcs_viol"):
        sol[k].copy_(torch.as_tensor(rng.normal(size=n), dtype=sol[k].dtype))
    sol["status"].copy_(torch.as_tensor(rng.integers(0, 3, n), dtype=torch.int32))
    sol["scp_iters"].copy_(torch.as_tensor(rng.integers(1, 26, n), dtype=torch.int32))
    sol["pipg_iters"].copy_(torch.as_tensor(rng.integers(1, 60000, n), dtype=torch.int32))
    # coarse costs so that ties occur
    sol["objective"].copy_(torch.as_tensor(np.round(rng.normal(size=n), 1), dtype=torch.float64))
    return sol


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("problems,starts", [(97, 4), (64, 1), (33, 7), (0, 3)])
def test_select_best_kernel_matches_oracle(dtype, problems, starts):
    import torch
    print("case: select_best %s problems %d starts %d" % (dtype, problems, starts), flush=True)
    cfg = I.solver_settings("C1")
    s = api.BatchSolver(cfg, dtype=dtype, k_max=12, max_batch=max(problems * starts, 1))
    try:
        rng = np.random.default_rng(problems * 10 + starts)
        n = problems * starts
        sol = _fake_solution(s, max(n, 1), rng)
        best, out = s.select_best(sol, problems, starts)
        torch.cuda.synchronize()
        h = {k: v.cpu().numpy() for k, v in sol.items()}
        b = best.cpu().numpy()
        o = {k: v.cpu().numpy() for k, v in out.items()}
        expect = oracle.select_best(h["status"][:n], h["objective"][:n], problems, starts)
        np.testing.assert_array_equal(b[:problems], expect)
        src = np.arange(problems) * starts + np.maximum(expect, 0)
        for k in h:
            np.testing.assert_array_equal(o[k][:problems], h[k][src], err_msg=k)
    finally:
        s.close()


def test_select_best_rejects_bad_arguments():
    cfg = I.solver_settings("C1")
    s = api.BatchSolver(cfg, dtype="f32", k_max=12, max_batch=8)
    try:
        sol = s.alloc_solution(8)
        with pytest.raises(api.ScpError):       # out aliases the solved batch
            s.select_best_into(sol, 2, 4, s.torch.empty(2, dtype=s.torch.int32,
                                                        device="cuda:0"), sol)
        with pytest.raises(api.ScpError):       # more instances than max_batch
            s.select_best(s.alloc_solution(9), 3, 3)
        with pytest.raises(api.ScpError):       # no start
            s.select_best(sol, 2, 0)
    finally:
        s.close()


def test_multistart_paper_monte_carlo_k20_fp64():
    # the paper's Monte Carlo at K = 20 with the node-wise convex sets on and starts s_init in
    # {4, 5, 6, 7}: the GPU's choice and the chosen trajectories match the oracle's; every
    # problem converges, where the single start s_init = 5 leaves eight cycling
    print("case: multi-start paper Monte Carlo K=20 fp64", flush=True)
    cfg = I.solver_settings("F1", node_projections=31)
    inst = I.make_instances("F1")
    inst["K"] = np.full(256, 20, np.int32)
    s_init = (4.0, 5.0, 6.0, 7.0)
    out, best, every = api.solve_multistart(cfg, inst, s_init, dtype="f64", k_max=20)
    rep = I.multistart(inst, s_init)
    o = oracle.solve(cfg, rep["x0"], rep["xf"], rep["params"], rep["K"], kmax=20)
    ob = oracle.select_best(o["status"], o["objective"], 256, 4)
    single = np.sum(o["status"].reshape(256, 4)[:, 1] == 0)
    print("converged: one start (s_init = 5) %d / 256, multi-start GPU %d / 256, oracle %d / 256"
          % (single, np.sum(best >= 0), np.sum(ob >= 0)))
    np.testing.assert_array_equal(every["status"], o["status"])
    np.testing.assert_array_equal(every["scp_iters"], o["scp_iters"])
    # the choice agrees wherever the runner-up's cost is not within FP64 noise of the best
    obj = o["objective"].reshape(256, 4)
    conv = o["status"].reshape(256, 4) == 0
    srt = np.sort(np.where(conv, obj, np.inf), axis=1)
    clear = (ob >= 0) & ((srt[:, 1] - srt[:, 0]) > 1e-9)
    np.testing.assert_array_equal(best[clear], ob[clear])
    assert np.all(best >= 0) and single < 256
    px, pu = np.array(cfg["px"]), np.array(cfg["pu"])
    src = np.arange(256) * 4 + ob
    ex = np.max(np.abs(out["x"] - o["x"][src]) / px, axis=(1, 2))
    eu = np.max(np.abs(out["u"] - o["u"][src]) / pu, axis=(1, 2))
    print("chosen trajectories: x %.2e u %.2e" % (ex[clear].max(), eu[clear].max()))
    assert ex[clear].max() <= TOL_F64 and eu[clear].max() <= TOL_F64
