"""Pins of the oracle's scalar-dilation variant: one dilation value over the whole horizon.

In the per-node form the dilation s is a first-order-hold control with a value per node
(section "Free-Final-Time Problem": the time dilation enters the augmented dynamics as a
control).  The scalar variant keeps one value sigma for every node, so that the dilation's
contribution to interval k is sigma times S_k = (B^-_k + B^+_k) restricted to the s column.
The oracle realises it inside PIPG as a projection onto {s_1 = ... = s_K}; these tests pin
that against the reduced QP written with the S_k column (dense linear algebra), against a
library scalar minimiser for the projection, and against the per-node solver where the two
problems coincide.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import dense_qp as DQ
import oracle
from paper_2404_18034_amd import instances as I

NX, NU = 15, 4


def reference_qp(K, **over):
    cfg = I.solver_settings("C0", scalar_dilation=1, **over)
    inst = I.make_instances("C0", ids=[0])
    x0, xf, p = inst["x0"][0], inst["xf"][0], inst["params"][0]
    xb, ub = oracle.init_guess(K, x0, xf, p)
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, cfg["rk4_substeps"])
    qp = oracle.build_qp(cfg, p, K, x0, xf, xb, ub, xe, A, Bm, Bp)
    return cfg, qp


def expansion(K):
    """E maps the reduced variables (x_1..x_K, T_1..T_K, sigma) to (x, u): sigma is copied
    into the s slot of every node."""
    nx = K * NX
    nr = nx + 3 * K + 1
    E = np.zeros((nx + K * NU, nr))
    E[:nx, :nx] = np.eye(nx)
    for k in range(K):
        for j in range(3):
            E[nx + k * NU + j, nx + 3 * k + j] = 1.0
        E[nx + k * NU + 3, nr - 1] = 1.0
    return E


def test_initial_guess_has_one_dilation_value():
    inst = I.make_instances("C0", ids=[0])
    _, ub = oracle.init_guess(10, inst["x0"][0], inst["xf"][0], inst["params"][0])
    assert np.ptp(ub[:, 3]) == 0.0


def test_reduced_qp_with_s_column_equality_only():
    # Hard dynamics only: min 1/2 z'Pz + p'z over z = E zeta subject to G z = g and the
    # boundary values.  Written with the S_k column, G E has for interval k the column
    # B^-_k[:, s] + B^+_k[:, s] on sigma.  PIPG with the scalar dilation must reach the
    # KKT point of that reduced problem.
    K = 4
    cfg, qp = reference_qp(K, node_projections=0, w_ep=1e6)
    qp["umin"][:, 3] = -1e30
    qp["umax"][:, 3] = 1e30
    qp["eps"][:] = 1e3
    sigma, _ = oracle.power(cfg, qp)
    sol, _ = oracle.pipg(cfg, qp, sigma, 80000, 0)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    M, nx, nu, nm, n = DQ.sizes(K)
    nxu = nx + nu
    E = expansion(K)
    GE = D["G"][:, :nxu] @ E
    # the sigma column of G E is the sum of the s columns of B^- and B^+ (S_k)
    S = np.concatenate([qp["Bm"][k][:, 3] + qp["Bp"][k][:, 3] for k in range(M)])
    np.testing.assert_allclose(GE[:, -1], S, rtol=0, atol=1e-15)
    Pr = E.T @ np.diag(D["P"][:nxu]) @ E
    pr = E.T @ D["p"][:nxu]
    nr = E.shape[1]
    fixed = np.zeros(nr, bool)
    fixed[:NX] = True
    for i in DQ.FINAL_FIXED:
        fixed[(K - 1) * NX + i] = True
    zfix = np.zeros(nr)
    zfix[:NX] = qp["zi"]
    for i in DQ.FINAL_FIXED:
        zfix[(K - 1) * NX + i] = qp["zf"][i - 1]
    Gf, Gc = GE[:, ~fixed], GE[:, fixed]
    nf = int((~fixed).sum())
    KKT = np.block([[Pr[np.ix_(~fixed, ~fixed)], Gf.T], [Gf, np.zeros((Gf.shape[0],) * 2)]])
    rhs = np.concatenate([-pr[~fixed] - Pr[np.ix_(~fixed, fixed)] @ zfix[fixed],
                          D["g"] - Gc @ zfix[fixed]])
    sol_kkt = np.linalg.lstsq(KKT, rhs, rcond=None)[0]
    zeta = zfix.copy()
    zeta[~fixed] = sol_kkt[:nf]
    got = np.concatenate([sol["x"].ravel(), sol["u"].ravel()])
    np.testing.assert_allclose(got, E @ zeta, atol=1e-8)
    assert np.ptp(sol["u"][:, 3]) == 0.0


def project_scalar(z, qp, K):
    """Projection onto the paper's set with one dilation value, the s part by a library
    bounded scalar minimiser of sum_k (v_k - c)^2 over the common box."""
    d = DQ.split(DQ.project(z, qp, K), K)
    v = DQ.split(z, K)["u"][:, 3]
    lo, hi = qp["umin"][:, 3].max(), qp["umax"][:, 3].min()
    r = minimize_scalar(lambda c: np.sum((v - c) ** 2), bounds=(lo, hi), method="bounded",
                        options=dict(xatol=1e-13))
    d["u"][:, 3] = r.x
    return DQ.join(d)


def test_projection_onto_one_dilation_value_by_minimiser():
    # One PIPG step from a random point: the oracle's fresh dilation values must be the
    # minimiser's projection of the gradient step (both boxes active and inactive).
    K = 5
    cfg, qp = reference_qp(K, node_projections=0)
    rng = np.random.default_rng(7)
    sigma, _ = oracle.power(cfg, qp)
    a = 2.0 / (cfg["w_prox"] + np.sqrt(cfg["w_prox"] ** 2 + 4 * cfg["omega"] * sigma))
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    for scale, box in ((0.1, None), (3.0, None), (0.1, (-0.02, 0.01))):
        if box is not None:
            qp["umin"][:, 3], qp["umax"][:, 3] = box
        ws = dict(x=scale * rng.standard_normal((K, NX)), u=scale * rng.standard_normal((K, NU)),
                  mup=np.abs(rng.standard_normal((K - 1, NX))),
                  mum=np.abs(rng.standard_normal((K - 1, NX))),
                  phi=rng.standard_normal((K - 1, NX)), th=np.abs(rng.standard_normal(K - 1)))
        sol, _ = oracle.pipg(cfg, qp, sigma, 1, 0, ws=ws)
        z = DQ.join(ws)
        grad = D["P"] * z + D["p"] + D["G"].T @ ws["phi"].ravel() + D["H"].T @ ws["th"]
        want = DQ.split(project_scalar(z - a * grad, qp, K), K)
        np.testing.assert_allclose(sol["u"][:, 3], want["u"][:, 3], rtol=0, atol=1e-9)
        np.testing.assert_allclose(sol["u"][:, :3], want["u"][:, :3], rtol=0, atol=1e-12)


def test_fixed_point_certificate_with_one_dilation_value():
    # Converged PIPG: z = Pi'(z - alpha grad L) with Pi' the minimiser-based projection,
    # primal feasibility and complementarity.
    K = 5
    cfg, qp = reference_qp(K, node_projections=0)
    sigma, _ = oracle.power(cfg, qp)
    a = 2.0 / (cfg["w_prox"] + np.sqrt(cfg["w_prox"] ** 2 + 4 * cfg["omega"] * sigma))
    sol, _ = oracle.pipg(cfg, qp, sigma, 100000, 0)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z = DQ.join(sol)
    grad = D["P"] * z + D["p"] + D["G"].T @ sol["phi"].ravel() + D["H"].T @ sol["th"]
    assert np.abs(project_scalar(z - a * grad, qp, K) - z).max() < 1e-7
    assert np.abs(D["G"] @ z - D["g"]).max() < 1e-7
    slack = D["H"] @ z - D["h"]
    assert slack.max() < 1e-7
    assert np.abs(sol["th"] * slack).max() < 1e-7


def test_solve_keeps_one_dilation_value_and_t_f():
    # Every SCP solution has one dilation value, and t_f = integral of s over tau in [0, 1]
    # is that value.
    cfg = I.solver_settings("C2", scalar_dilation=1)
    inst = I.make_instances("C2", B=4)
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    for b in range(4):
        K = inst["K"][b]
        s = r["u"][b, :K, 3]
        assert np.ptp(s) == 0.0
        np.testing.assert_allclose(r["t_f"][b], s[0], rtol=1e-14)
    assert (r["status"] == 0).sum() >= 3


def test_degenerate_box_coincides_with_per_node_dilation():
    # With s_min = s_max (= s_init) both forms fix s at that value on every node: the
    # solutions are identical bit for bit.
    inst = I.make_instances("C2", B=3)
    p = inst["params"].copy()
    p[:, 18] = p[:, 19] = p[:, 21] = 4.5
    base = I.solver_settings("C2")
    r0 = oracle.solve(base, inst["x0"], inst["xf"], p, inst["K"])
    r1 = oracle.solve(dict(base, scalar_dilation=1), inst["x0"], inst["xf"], p, inst["K"])
    for key in r0:
        np.testing.assert_array_equal(r0[key], r1[key])


@pytest.mark.parametrize("flag", [0, 1])
def test_per_node_default_unchanged(flag):
    # The flag only acts on the dilation components: with it off the default settings give
    # the per-node form (a solve whose dilation varies along the trajectory).
    cfg = I.solver_settings("C0", scalar_dilation=flag)
    inst = I.make_instances("C0", ids=[0])
    r = oracle.solve(cfg, inst["x0"], inst["xf"], inst["params"], inst["K"])
    spread = np.ptp(r["u"][0, :inst["K"][0], 3])
    assert (spread == 0.0) == bool(flag)
