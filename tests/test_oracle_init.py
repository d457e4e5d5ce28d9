"""Pins of the oracle's caller-supplied first reference (x_init, u_init): the initial guess of
the SCP iteration (section "Sequential Convex Programming": the iteration starts from a
reference trajectory, which the caller may give instead of the built-in straight line)."""
import numpy as np
import pytest

import oracle
from paper_2404_18034_amd import instances as I


def _guess(inst, kmax, nu=4):
    B = inst["K"].shape[0]
    x = np.zeros((B, kmax, 15))
    u = np.zeros((B, kmax, nu))
    for b in range(B):
        K = int(inst["K"][b])
        x[b, :K], u[b, :K] = oracle.init_guess(K, inst["x0"][b], inst["xf"][b],
                                               inst["params"][b], nu=nu)
    return x, u


def test_supplying_the_builtin_guess_changes_nothing():
    cfg = I.solver_settings("C2", scp_iters_max=4, pipg_iters_max=200)
    inst = I.make_instances("C2", B=6)
    xg, ug = _guess(inst, 30)
    a = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30)
    b = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"], kmax=30,
                     x_init=xg, u_init=ug)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_a_converged_solution_is_a_fixed_point():
    # restarted from its own converged trajectory, the prox-linear iteration stops after the
    # first subproblem (the convergence test needs one step) and stays where it was
    cfg = I.solver_settings("F1", scp_iters_max=25)
    inst = I.make_instances("F1", B=6)
    a = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert np.all(a["status"] == 0) and np.all(a["scp_iters"] > 3)
    b = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"],
                     x_init=a["x"], u_init=a["u"])
    assert np.all(b["status"] == 0) and np.all(b["scp_iters"] == 1)
    px = np.array(cfg["px"])
    assert np.max(np.abs(b["x"] - a["x"]) / px) <= 2e-4
    assert np.max(np.abs(b["t_f"] - a["t_f"]) / a["t_f"]) <= 1e-4


def test_one_side_given_and_a_different_start():
    # a perturbed start (only the states, only the controls, or both) is taken: the iteration
    # still converges onto the boundary values, along a different path (the problem is
    # nonconvex, so it may end at a different stationary trajectory)
    cfg = I.solver_settings("F1", scp_iters_max=25)
    inst = I.make_instances("F1", B=4)
    a = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    xg, ug = _guess(inst, 30)
    rng = np.random.default_rng(3)
    tau = np.linspace(0.0, 1.0, 30)[None, :, None]
    xp = xg.copy()
    xp[:, :, 1:4] += 0.3 * np.sin(np.pi * tau) * rng.normal(size=(4, 1, 3))
    up = ug.copy()
    up[:, :, 3] *= 1.1
    fixed = [1, 2, 3, 4, 5, 6, 9, 10, 12, 13]
    for xi, ui in ((xp, None), (None, up), (xp, up)):
        b = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"],
                         x_init=xi, u_init=ui)
        assert np.all(b["status"] == 0)
        np.testing.assert_allclose(b["x"][:, 0, :14], inst["x0"][:, :14], atol=1e-9)
        np.testing.assert_allclose(b["x"][:, -1, fixed], inst["xf"][:, [i - 1 for i in fixed]],
                                   atol=1e-9)
        assert np.any(b["scp_iters"] != a["scp_iters"]) or np.any(b["x"] != a["x"])


def test_shapes_are_checked():
    cfg = I.solver_settings("C1")
    inst = I.make_instances("C1", B=2)
    with pytest.raises(ValueError):
        oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"],
                     x_init=np.zeros((2, 19, 15)))
    with pytest.raises(ValueError):
        oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"],
                     u_init=np.zeros((2, 20, 7)))
