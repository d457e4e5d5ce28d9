"""Pins of the oracle's prox-linear SCP loop (section "Sequential Convex Programming") on the
single-instance workload and small Monte Carlo samples."""
import numpy as np
import pytest

import oracle
from paper_2404_18034_amd import instances as I

NX, NU = 15, 4


@pytest.fixture(scope="module")
def c0():
    cfg = I.solver_settings("C0")
    inst = I.make_instances("C0")
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    return cfg, inst, r


def test_c0_converges(c0):
    cfg, inst, r = c0
    assert r["status"][0] == 0
    assert 1 <= r["scp_iters"][0] <= cfg["scp_iters_max"]
    assert r["defect_inf"][0] <= cfg["feas_tol"]


def test_c0_boundary_conditions_exact(c0):
    cfg, inst, r = c0
    K = int(inst["K"][0])
    x = r["x"][0, :K]
    np.testing.assert_allclose(x[0, :14], inst["x0"][0, :14], atol=1e-12)
    assert abs(x[0, 14]) <= 1e-12
    fixed = [1, 2, 3, 4, 5, 6, 9, 10, 12, 13]
    np.testing.assert_allclose(x[K - 1, fixed], inst["xf"][0, [i - 1 for i in fixed]], atol=1e-12)


def test_c0_physical_outcome(c0):
    cfg, inst, r = c0
    p = inst["params"][0]
    assert p[1] < r["m_f"][0] < inst["x0"][0, 0]
    assert 0.0 < r["t_f"][0] < 20.0
    u = r["u"][0, :int(inst["K"][0])]
    assert np.all(u[:, 3] >= p[18] - 1e-9) and np.all(u[:, 3] <= p[19] + 1e-9)
    # t_f is the integral of the first-order-hold dilation
    K = int(inst["K"][0])
    assert r["t_f"][0] == pytest.approx(np.sum(0.5 * (u[1:, 3] + u[:-1, 3])) / (K - 1), rel=1e-14)


def test_c0_fine_repropagation(c0):
    # The converged trajectory is dynamically feasible: re-integrating each interval with a
    # step 8x finer reproduces the next node to the integrator's error, and the CTCS integral
    # of the constraint violation over each interval stays within eps.
    cfg, inst, r = c0
    K = int(inst["K"][0])
    p = inst["params"][0]
    x, u = r["x"][0, :K], r["u"][0, :K]
    px = np.array(cfg["px"])
    worst, worst_y = 0.0, 0.0
    for k in range(K - 1):
        xe, *_ = oracle.discretize_interval(x[k], u[k], u[k + 1], p, 1.0 / (K - 1),
                                            8 * cfg["rk4_substeps"])
        worst = max(worst, np.max(np.abs(xe[:14] - x[k + 1, :14]) / px[:14]))
        worst_y = max(worst_y, xe[14] - x[k, 14])
    assert worst < 1e-3
    assert worst_y <= p[20] * 1.01


def test_c0_dense_constraint_sampling(c0):
    # Between nodes the path constraints hold up to the CTCS tolerance: the violation on a
    # dense grid is bounded by the level implied by the eps budget.
    cfg, inst, r = c0
    K = int(inst["K"][0])
    p = inst["params"][0]
    x, u = r["x"][0, :K], r["u"][0, :K]
    dtau = 1.0 / (K - 1)
    viol = 0.0
    for k in range(K - 1):
        xs = x[k].copy()
        for j in range(20):
            a0, a1 = j / 20, (j + 1) / 20
            u0 = (1 - a0) * u[k] + a0 * u[k + 1]
            u1 = (1 - a1) * u[k] + a1 * u[k + 1]
            xs, *_ = oracle.discretize_interval(xs, u0, u1, p, dtau / 20, 4)
            viol = max(viol, np.max(oracle.constraints(xs, u1, p)))
    # [g]_+^2 integrated over an interval of duration ~0.5 is <= eps = 1e-4
    assert viol < np.sqrt(p[20] / 0.05)


def test_final_subproblem_is_stationary(c0):
    # At a converged point, the next convex subproblem returns (almost) a zero step.
    cfg, inst, r = c0
    K = int(inst["K"][0])
    x0, xf, p = inst["x0"][0], inst["xf"][0], inst["params"][0]
    xb, ub = r["x"][0, :K], r["u"][0, :K]
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, cfg["rk4_substeps"])
    qp = oracle.build_qp(cfg, p, K, x0, xf, xb, ub, xe, A, Bm, Bp)
    sigma, _ = oracle.power(cfg, qp)
    sol, _ = oracle.pipg(cfg, qp, sigma, 20000, 0, ref=(xb, ub, p))
    assert max(np.abs(sol["x"]).max(), np.abs(sol["u"]).max()) < 20 * cfg["scp_tol"]


def test_batch_threads_and_single_agree():
    cfg = I.solver_settings("C1", scp_iters_max=3, pipg_iters_max=200)
    inst = I.make_instances("C1", B=6)
    a = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], nthreads=1)
    b = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], nthreads=4)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    t = oracle.solve_trace(cfg, inst["x0"][2], inst["xf"][2], inst["params"][2], 20)
    np.testing.assert_array_equal(t["x"], a["x"][2])
    assert t["scp_iters"] == 3 and t["pipg_iters"] == 600


def test_uneven_node_counts_and_padding():
    cfg = I.solver_settings("C2", scp_iters_max=2, pipg_iters_max=50)
    inst = I.make_instances("C2", B=12)
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    for b in range(12):
        K = int(inst["K"][b])
        assert np.all(r["x"][b, K:] == 0.0) and np.all(r["u"][b, K:] == 0.0)
        one = oracle.solve(cfg, inst["x0"][b:b + 1], inst["xf"][b:b + 1],
                           inst["params"][b:b + 1], inst["K"][b:b + 1], kmax=30)
        np.testing.assert_array_equal(one["x"][0], r["x"][b])


def test_non_finite_input_is_flagged_not_raised():
    cfg = I.solver_settings("C1", scp_iters_max=2, pipg_iters_max=20)
    inst = I.make_instances("C1", B=3)
    inst["x0"][1, 2] = np.nan
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert r["status"][1] == 2
    assert r["status"][0] != 2 and r["status"][2] != 2
    good = oracle.solve(cfg, inst["x0"][[0, 2]], inst["xf"][[0, 2]], inst["params"][[0, 2]],
                        inst["K"][[0, 2]])
    np.testing.assert_array_equal(good["x"][0], r["x"][0])


def test_invalid_node_count_rejected():
    cfg = I.solver_settings("C1")
    inst = I.make_instances("C1", B=2)
    inst["K"][1] = 1
    with pytest.raises(ValueError):
        oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=20)


def test_minimum_node_count_two():
    cfg = I.solver_settings("C1", scp_iters_max=3, pipg_iters_max=300)
    inst = I.make_instances("C1", B=1)
    inst["K"][:] = 2
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert np.all(np.isfinite(r["x"])) and r["scp_iters"][0] == 3


def test_monte_carlo_sample_mostly_converges():
    cfg = I.solver_settings("C1")
    inst = I.make_instances("C1", B=24)
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert np.all(r["status"] != 2)
    assert np.mean(r["status"] == 0) >= 0.6
    assert np.all(r["defect_inf"] < 1e-2)


def test_truncated_map_reproduces_last_iteration_and_is_smooth():
    cfg = I.solver_settings("C1", scp_iters_max=4, pipg_iters_max=300)
    inst = I.make_instances("C1", ids=[5])
    x0, xf, p, K = inst["x0"][0], inst["xf"][0], inst["params"][0], int(inst["K"][0])
    last = oracle.lastiter_state(cfg, x0, xf, p, K)
    theta = oracle.theta_of(x0, p)
    out = oracle.truncated_map(cfg, x0, xf, p, K, theta, last, cfg["pipg_iters_max"])
    full = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert out[0] == pytest.approx(full["m_f"][0], abs=1e-13)
    assert out[1] == pytest.approx(full["t_f"][0], abs=1e-13)
    # central differences at two step sizes agree (the map is smooth at this point)
    for i in (1, 4, 16, 17):
        d = []
        for h in (1e-5, 1e-6):
            e = np.zeros(18); e[i] = h
            d.append((oracle.truncated_map(cfg, x0, xf, p, K, theta + e, last, 200)
                      - oracle.truncated_map(cfg, x0, xf, p, K, theta - e, last, 200)) / (2 * h))
        np.testing.assert_allclose(d[0], d[1], rtol=1e-3, atol=1e-6)


def test_prox_linear_iteration_creeps_instead_of_settling():
    # Why the differentiated unit is the last SCP iteration and not an implicit adjoint of
    # the whole solve (section "Sequential Convex Programming"): run on far past the paper's
    # tolerances (PIPG to 1e-13 with up to 20,000 steps per subproblem), the scaled SCP step
    # of a paper Monte Carlo run settles at a constant nonzero value while the trajectory
    # stays dynamically feasible and drifts steadily (final mass up, flight time down), so the
    # iteration has no isolated fixed point for the implicit function theorem to use.
    inst = I.make_instances("F1", B=1)
    base = dict(pipg_iters_max=20000, pipg_check_every=10, scp_tol=1e-12, feas_tol=1e-12,
                pipg_eps_abs=1e-13, pipg_eps_rel=1e-13, early_exit=0)
    out = {}
    for n in (24, 36):
        cfg = I.solver_settings("F1", scp_iters_max=n, **base)
        out[n] = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    a, b = out[24], out[36]
    print("\nstep %.3e %.3e, defect %.1e %.1e, m_f %+.2e, t_f %+.2e over 12 iterations" % (
        a["step"][0], b["step"][0], a["defect_inf"][0], b["defect_inf"][0],
        b["m_f"][0] - a["m_f"][0], b["t_f"][0] - a["t_f"][0]))
    for r in (a, b):
        assert r["defect_inf"][0] < 1e-7
        assert r["step"][0] > 1e-5
    assert abs(b["step"][0] - a["step"][0]) <= 0.05 * a["step"][0]
    assert b["m_f"][0] - a["m_f"][0] > 5e-6
    assert b["t_f"][0] - a["t_f"][0] < -1e-4
