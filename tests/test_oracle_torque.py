"""Pins of the oracle's full control set (section "6-DoF Powered Descent Guidance"): the
reaction-control torque gamma joins the thrust, u = (T, gamma, s) (n_u = 7), with the row
||gamma||^2 - gamma_max^2 among the path constraints."""
import numpy as np
import pytest

import dense_qp as DQ
import oracle
from paper_2404_18034_amd import instances as I

NX = 15


def _point(rng, p):
    x = np.r_[1.8, rng.uniform(1, 4, 3), rng.normal(size=3), 0.0, 0.0, 0.0, 0.0,
              rng.normal(size=3) * 0.3, 0.0]
    q = rng.normal(size=4)
    x[7:11] = q / np.linalg.norm(q)
    u = np.r_[rng.uniform(1, 3), rng.normal(size=2) * 0.5, rng.normal(size=3) * 0.01, 5.0]
    return x, u


def test_torque_closed_forms():
    # at rest with no thrust and isotropic inertia the rates grow as gamma / J; the mass flow
    # and the translational dynamics do not see the torque
    p = I.nominal_params()
    x = np.r_[2.0, 4, 4, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0]
    gam = np.array([0.003, -0.002, 0.001])
    s = 3.0
    f7 = oracle.dynamics(x, np.r_[0.0, 0.0, 0.0, gam, s], p)
    np.testing.assert_allclose(f7[11:14], s * gam / p[6:9], rtol=1e-15)
    f4 = oracle.dynamics(x, np.r_[0.0, 0.0, 0.0, s], p)
    np.testing.assert_array_equal(f7[:11], f4[:11])
    # with thrust too the torque adds to the thrust torque r_T x T
    T = np.array([2.0, 0.1, -0.2])
    f7 = oracle.dynamics(x, np.r_[T, gam, s], p)
    f4 = oracle.dynamics(x, np.r_[T, s], p)
    np.testing.assert_allclose(f7[11:14] - f4[11:14], s * gam / p[6:9], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(f7[:11], f4[:11])


def test_torque_bound_row():
    p = I.nominal_params()
    x = np.r_[2.0, 4, 4, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0]
    gam = np.array([0.004, 0.0, 0.003])                    # |gamma| = 0.005 = gamma_max
    g = oracle.constraints(x, np.r_[2.0, 0, 0, gam, 5.0], p)
    assert g[8] == pytest.approx(0.0, abs=1e-18)
    g = oracle.constraints(x, np.r_[2.0, 0, 0, 2 * gam, 5.0], p)
    assert g[8] == pytest.approx(4 * 0.005 ** 2 - 0.005 ** 2, rel=1e-12)
    # the thrust-only model and an unbounded torque have the constant -1 there
    assert oracle.constraints(x, np.r_[2.0, 0, 0, 5.0], p)[8] == -1.0
    pinf = p.copy(); pinf[23] = np.inf
    assert oracle.constraints(x, np.r_[2.0, 0, 0, gam, 5.0], pinf)[8] == -1.0
    # the CTCS rate gains s [g_9]_+^2 when the bound is violated
    f_in = oracle.dynamics(x, np.r_[2.0, 0, 0, gam, 5.0], p)
    f_out = oracle.dynamics(x, np.r_[2.0, 0, 0, 2 * gam, 5.0], p)
    assert f_out[14] - f_in[14] == pytest.approx(5.0 * (3 * 0.005 ** 2) ** 2, rel=1e-9)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_torque_jacobians_against_central_differences(seed):
    rng = np.random.default_rng(seed)
    p = I.nominal_params()
    p[23] = 0.002                       # the torque bound is active at the random points
    for _ in range(5):
        x, u = _point(rng, p)
        A, B = oracle.jacobians(x, u, p)
        assert B.shape == (NX, 7)
        h = 1e-6
        for j in range(NX):
            e = np.zeros(NX); e[j] = h
            fd = (oracle.dynamics(x + e, u, p) - oracle.dynamics(x - e, u, p)) / (2 * h)
            np.testing.assert_allclose(A[:, j], fd, rtol=1e-6, atol=1e-8)
        for j in range(7):
            e = np.zeros(7); e[j] = h
            fd = (oracle.dynamics(x, u + e, p) - oracle.dynamics(x, u - e, p)) / (2 * e[j])
            np.testing.assert_allclose(B[:, j], fd, rtol=1e-6, atol=1e-8)


def test_torque_discretization_extends_the_thrust_only_one():
    # with the torque guess at zero, the n_u = 7 discretization reproduces the thrust-only
    # one on the shared columns, and its torque columns are those of J^-1 integrated
    cfg = I.solver_settings("F2")
    inst = I.make_instances("F2", ids=[0])
    x0, xf, p = inst["x0"][0], inst["xf"][0], inst["params"][0]
    K = 6
    xb, ub7 = oracle.init_guess(K, x0, xf, p, nu=7)
    xb4, ub4 = oracle.init_guess(K, x0, xf, p)
    np.testing.assert_array_equal(xb, xb4)
    np.testing.assert_array_equal(ub7[:, [0, 1, 2, 6]], ub4)
    assert np.all(ub7[:, 3:6] == 0.0)
    xe7, A7, Bm7, Bp7 = oracle.discretize(K, xb, ub7, p, cfg["rk4_substeps"])
    xe4, A4, Bm4, Bp4 = oracle.discretize(K, xb, ub4, p, cfg["rk4_substeps"])
    np.testing.assert_allclose(xe7, xe4, rtol=0, atol=1e-14)
    np.testing.assert_allclose(A7, A4, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Bm7[:, :, [0, 1, 2, 6]], Bm4, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Bp7[:, :, [0, 1, 2, 6]], Bp4, rtol=0, atol=1e-13)
    # torque columns: nonzero only through the rate rows (and what they drive)
    assert np.abs(Bm7[:, 11:14, 3:6]).max() > 0
    np.testing.assert_array_equal(Bm7[:, 0, 3:6], 0.0)


@pytest.mark.parametrize("K,n_iter", [(4, 30), (6, 60)])
def test_torque_pipg_custom_equals_generic_pipg(K, n_iter):
    cfg = I.solver_settings("F2")
    inst = I.make_instances("F2", ids=[3])
    x0, xf, p = inst["x0"][0], inst["xf"][0], inst["params"][0]
    xb, ub = oracle.init_guess(K, x0, xf, p, nu=7)
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, cfg["rk4_substeps"])
    qp = oracle.build_qp(cfg, p, K, x0, xf, xb, ub, xe, A, Bm, Bp)
    assert qp["Bm"].shape[-1] == 7
    assert np.all(np.isinf(qp["umin"][:, :6])) and np.all(np.isfinite(qp["umin"][:, 6]))
    sigma, _ = oracle.power(cfg, qp)
    a = 2.0 / (cfg["w_prox"] + np.sqrt(cfg["w_prox"] ** 2 + 4 * cfg["omega"] * sigma))
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z, w, v = DQ.pipg_generic(D, qp, a, cfg["omega"] * a, cfg["rho"], n_iter)
    sol, n = oracle.pipg(cfg, qp, sigma, n_iter, 0)
    np.testing.assert_allclose(DQ.join(sol), z, atol=1e-11)
    np.testing.assert_allclose(sol["phi"].ravel(), w, atol=1e-11)
    # the power iteration against the SVD of the dense operator
    Kmat = np.vstack([D["G"], D["H"]])
    smax2 = np.linalg.svd(Kmat, compute_uv=False)[0] ** 2
    assert sigma >= smax2 and sigma / (1 + cfg["power_buff"]) <= smax2 * (1 + 1e-12)


def test_torque_monte_carlo_sample_solves():
    # 16 runs of the paper's Monte Carlo with the torque: every run converges, lands on its
    # boundary values, keeps the torque within its bound up to the CTCS tolerance, and uses
    # less propellant than with thrust alone
    cfg = I.solver_settings("F2")
    inst = I.make_instances("F2", B=16)
    o = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert o["u"].shape[-1] == 7
    assert np.all(o["status"] == 0)
    np.testing.assert_allclose(o["x"][:, 0, :14], inst["x0"][:, :14], atol=1e-9)
    fixed = [1, 2, 3, 4, 5, 6, 9, 10, 12, 13]
    np.testing.assert_allclose(o["x"][:, -1, fixed], inst["xf"][:, [i - 1 for i in fixed]],
                               atol=1e-9)
    gam = np.linalg.norm(o["u"][:, :, 3:6], axis=2)
    assert gam.max() <= inst["params"][0, 23] * 1.1
    assert np.sum(gam.max(axis=1) > 0.5 * inst["params"][0, 23]) >= 8   # the torque is used
    o4 = oracle.solve(I.solver_settings("F1"), inst["x0"], inst["xf"], inst["params"], inst["K"])
    assert np.median(o["m_f"] - o4["m_f"]) > 0
