"""Pins of the oracle's convex-subproblem pieces: the prescaled QP (eq.
cvx-subproblem-custom), the customized power iteration, PIPG_custom, its stopping rule and
the node-wise projections."""
import numpy as np
import pytest
from scipy.optimize import minimize

import dense_qp as DQ
import oracle
from paper_2404_18034_amd import instances as I

NX, NU = 15, 4


def reference_qp(K=5, cfg_name="C0", b=0, iters=0, **over):
    """QP data at the initial guess (optionally after a few oracle SCP steps)."""
    cfg = I.solver_settings(cfg_name, **over)
    inst = I.make_instances(cfg_name, ids=[b])
    x0, xf, p = inst["x0"][0], inst["xf"][0], inst["params"][0]
    xb, ub = oracle.init_guess(K, x0, xf, p)
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, cfg["rk4_substeps"])
    qp = oracle.build_qp(cfg, p, K, x0, xf, xb, ub, xe, A, Bm, Bp)
    return cfg, dict(x0=x0, xf=xf, p=p, xb=xb, ub=ub, xe=xe, A=A, Bm=Bm, Bp=Bp), qp


def test_qp_build_identities():
    # For any (x, u): Px^-1 times the linearized residual (paper's w_k) equals the scaled
    # residual A^- x^ - x^_k+1 + B^- u^_k + B^+ u^_k+1 + w^_k.
    cfg, d, qp = reference_qp(K=6)
    K = 6
    px, pu = np.array(cfg["px"]), np.array(cfg["pu"])
    rng = np.random.default_rng(3)
    x = d["xb"] + rng.normal(size=(K, NX)) * 0.1
    u = d["ub"] + rng.normal(size=(K, NU)) * 0.1
    xh, uh = (x - d["xb"]) / px, (u - d["ub"]) / pu
    for k in range(K - 1):
        wk = d["xe"][k] - d["A"][k] @ d["xb"][k] - d["Bm"][k] @ d["ub"][k] - d["Bp"][k] @ d["ub"][k + 1]
        res = d["A"][k] @ x[k] + d["Bm"][k] @ u[k] + d["Bp"][k] @ u[k + 1] + wk - x[k + 1]
        sres = (qp["Am"][k] @ xh[k] - xh[k + 1] + qp["Bm"][k] @ uh[k] + qp["Bp"][k] @ uh[k + 1]
                + qp["w"][k])
        np.testing.assert_allclose(sres, res / px, atol=1e-12)
        # CTCS row: y_k+1 - y_k <= eps  <=>  y^_k+1 - y^_k <= eps^_k
        lhs = (x[k + 1, 14] - x[k, 14] - d["p"][20]) / px[14]
        assert xh[k + 1, 14] - xh[k, 14] - qp["eps"][k] == pytest.approx(lhs, abs=1e-12)
    # boundary values reproduce x_1 = (z_i, 0) and the fixed final components
    np.testing.assert_allclose(d["xb"][0] + px * qp["zi"], np.r_[d["x0"][:14], 0.0], atol=1e-15)
    np.testing.assert_allclose(d["xb"][-1, 1:14] + px[1:14] * qp["zf"], d["xf"], atol=1e-15)
    # scaled dilation bounds
    np.testing.assert_allclose(d["ub"][:, 3] + pu[3] * qp["umin"][:, 3], d["p"][18])
    np.testing.assert_allclose(d["ub"][:, 3] + pu[3] * qp["umax"][:, 3], d["p"][19])
    assert np.all(np.isinf(qp["umin"][:, :3])) and np.all(np.isinf(qp["umax"][:, :3]))


@pytest.mark.parametrize("K", [2, 3, 5])
def test_power_iteration_against_svd(K):
    cfg, _, qp = reference_qp(K=K, power_iters_max=20000, power_eps_rel=0.0)
    D = DQ.assemble(qp, 1.0, 0.0, 0.0)
    Kmat = np.vstack([D["G"], D["H"]])
    sv2 = np.linalg.svd(Kmat, compute_uv=False) ** 2
    smax2 = sv2[0]
    sigma, its = oracle.power(cfg, qp)
    est = sigma / (1.0 + cfg["power_buff"])
    # ||K^T K z|| / ||z|| never exceeds lambda_max(K^T K) and converges to it; when the top
    # two eigenvalues nearly coincide the estimate settles between them
    assert est <= smax2 * (1 + 1e-12)
    assert est >= min(smax2 * (1 - 1e-6), sv2[1] * (1 - 1e-9))
    assert sigma >= smax2


def test_power_iteration_stops_on_relative_change():
    cfg, _, qp = reference_qp(K=5)
    sigma, its = oracle.power(cfg, qp)
    assert its < cfg["power_iters_max"]
    cfg2 = dict(cfg, power_iters_max=1)
    _, its1 = oracle.power(cfg2, qp)
    assert its1 == 1


def _alpha_beta(cfg, sigma):
    a = 2.0 / (cfg["w_prox"] + np.sqrt(cfg["w_prox"] ** 2 + 4 * cfg["omega"] * sigma))
    return a, cfg["omega"] * a


@pytest.mark.parametrize("K,n_iter", [(3, 1), (4, 7), (6, 60)])
def test_pipg_custom_equals_generic_pipg(K, n_iter):
    # The customized solver exploits the block structure; the generic extrapolated PIPG on
    # the dense canonical form must produce the same iterates.
    cfg, _, qp = reference_qp(K=K, node_projections=0)
    sigma, _ = oracle.power(cfg, qp)
    alpha, beta = _alpha_beta(cfg, sigma)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z, w, v = DQ.pipg_generic(D, qp, alpha, beta, cfg["rho"], n_iter)
    sol, n = oracle.pipg(cfg, qp, sigma, n_iter, 0)
    assert n == n_iter
    np.testing.assert_allclose(DQ.join(sol), z, atol=1e-11)
    np.testing.assert_allclose(sol["phi"].ravel(), w, atol=1e-11)
    np.testing.assert_allclose(sol["th"], v, atol=1e-11)


def test_pipg_custom_equals_generic_pipg_warm_started():
    cfg, _, qp = reference_qp(K=5, node_projections=0)
    K = 5
    sigma, _ = oracle.power(cfg, qp)
    alpha, beta = _alpha_beta(cfg, sigma)
    rng = np.random.default_rng(11)
    ws = oracle.zero_warm_start(K)
    for k in ws:
        ws[k] = rng.normal(size=ws[k].shape) * 0.1
    ws["mup"] = np.abs(ws["mup"]); ws["mum"] = np.abs(ws["mum"]); ws["th"] = np.abs(ws["th"])
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z, w, v = DQ.pipg_generic(D, qp, alpha, beta, cfg["rho"], 25, z0=DQ.join(ws),
                              eta0=ws["phi"].ravel(), chi0=ws["th"])
    sol, _ = oracle.pipg(cfg, qp, sigma, 25, 0, ws)
    np.testing.assert_allclose(DQ.join(sol), z, atol=1e-11)
    np.testing.assert_allclose(sol["phi"].ravel(), w, atol=1e-11)


def test_pipg_converges_to_dense_kkt_solution_equality_only():
    # Hard dynamics only (no active inequality): the QP is min 1/2 w_prox ||z||^2 + c.z
    # subject to G z = g and the boundary values; PIPG must reach the KKT solution.
    cfg, _, qp = reference_qp(K=4, node_projections=0, w_ep=1e6)
    K = 4
    qp["umin"][:, 3] = -1e30; qp["umax"][:, 3] = 1e30
    qp["eps"][:] = 1e3
    sigma, _ = oracle.power(cfg, qp)
    sol, _ = oracle.pipg(cfg, qp, sigma, 60000, 0)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    M, nx, nu, nm, n = DQ.sizes(K)
    nxu = nx + nu
    fixed = np.zeros(nxu, bool)
    fixed[:NX] = True
    for i in DQ.FINAL_FIXED:
        fixed[(K - 1) * NX + i] = True
    zfix = np.zeros(nxu)
    zfix[:NX] = qp["zi"]
    for i in DQ.FINAL_FIXED:
        zfix[(K - 1) * NX + i] = qp["zf"][i - 1]
    G = D["G"][:, :nxu]
    Gf, Gc = G[:, ~fixed], G[:, fixed]
    nf = int((~fixed).sum())
    KKT = np.block([[cfg["w_prox"] * np.eye(nf), Gf.T], [Gf, np.zeros((Gf.shape[0],) * 2)]])
    rhs = np.concatenate([-D["p"][:nxu][~fixed], D["g"] - Gc @ zfix[fixed]])
    sol_kkt = np.linalg.lstsq(KKT, rhs, rcond=None)[0]
    z = zfix.copy()
    z[~fixed] = sol_kkt[:nf]
    got = np.concatenate([sol["x"].ravel(), sol["u"].ravel()])
    np.testing.assert_allclose(got, z, atol=1e-8)
    assert np.abs(sol["mup"]).max() == 0.0 and np.abs(sol["mum"]).max() == 0.0


def test_pipg_fixed_point_certificate_full_qp():
    # After many iterations the returned point satisfies the projected-gradient fixed point
    # z = Pi(z - alpha grad L(z, phi, theta)), primal feasibility and complementarity.
    cfg, _, qp = reference_qp(K=5, node_projections=0)
    K = 5
    sigma, _ = oracle.power(cfg, qp)
    alpha, beta = _alpha_beta(cfg, sigma)
    sol, _ = oracle.pipg(cfg, qp, sigma, 100000, 0)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z = DQ.join(sol)
    grad = D["P"] * z + D["p"] + D["G"].T @ sol["phi"].ravel() + D["H"].T @ sol["th"]
    assert np.abs(DQ.project(z - alpha * grad, qp, K) - z).max() < 1e-7
    assert np.abs(D["G"] @ z - D["g"]).max() < 1e-7
    slack = D["H"] @ z - D["h"]
    assert slack.max() < 1e-7
    assert np.abs(sol["th"] * slack).max() < 1e-7


def test_stopping_rule_hand_computed():
    K = 3
    base = oracle.zero_warm_start(K)
    old = {k: v.copy() for k, v in base.items()}
    new = {k: v.copy() for k, v in base.items()}
    old["x"][1, 2] = 1.0; new["x"][1, 2] = 1.0 + 2e-5      # dz = 2e-5, max|z| = 1 + 2e-5
    old["phi"][0, 0] = 2.0; new["phi"][0, 0] = 2.0          # dr = 0
    # eabs + erel*max = 1e-5 + 1e-5*(1+2e-5) ~ 2.00002e-5 >= 2e-5 -> terminate
    assert oracle.stopping(new, old, 1e-5, 1e-5)
    new["x"][1, 2] = 1.0 + 2.1e-5
    assert not oracle.stopping(new, old, 1e-5, 1e-5)
    new["x"][1, 2] = 1.0
    new["th"][1] = 3.5e-5                                    # dr = 3.5e-5 > 1e-5 + 1e-5*2
    assert not oracle.stopping(new, old, 1e-5, 1e-5)
    assert oracle.stopping(new, old, 1e-5, 2e-5)             # 1e-5 + 4e-5 >= 3.5e-5


def _in_sets(p, x, u, tol=1e-12):
    lat = np.linalg.norm(x[2:4])
    return (x[0] >= p[1] - tol and np.tan(p[15]) * lat <= x[1] + tol
            and x[9] ** 2 + x[10] ** 2 <= 0.5 * (1 - np.cos(p[16])) + tol
            and np.linalg.norm(x[11:14]) <= p[17] + tol
            and np.linalg.norm(u[:3]) * np.cos(p[14]) <= u[0] + tol
            and np.linalg.norm(u[:3]) <= p[13] + tol)


def test_node_projections_are_projections():
    p = I.nominal_params()
    p[16] = np.radians(45.0)
    rng = np.random.default_rng(5)
    for _ in range(200):
        x = rng.normal(size=NX) * 2; x[0] = rng.uniform(0, 3)
        u = rng.normal(size=NU) * 4
        px_, pu_ = oracle.project_node(p, x, u)
        assert _in_sets(p, px_, pu_, 1e-10)
        # idempotent
        a, b = oracle.project_node(p, px_, pu_)
        np.testing.assert_allclose(a, px_, atol=1e-12); np.testing.assert_allclose(b, pu_, atol=1e-12)
        # variational inequality against random members of the set
        for _ in range(5):
            y = rng.normal(size=NX) * 2; v = rng.normal(size=NU) * 4
            y, v = oracle.project_node(p, y, v)
            assert np.dot(x - px_, y - px_) <= 1e-9
            assert np.dot(u - pu_, v - pu_) <= 1e-9
        # untouched coordinates: q0, q1, y and the dilation
        assert px_[7] == x[7] and px_[8] == x[8] and px_[14] == x[14] and pu_[3] == u[3]


def test_thrust_projection_brute_force():
    p = I.nominal_params()
    rng = np.random.default_rng(9)
    cons = [{"type": "ineq", "fun": lambda T: T[0] - np.cos(p[14]) * np.linalg.norm(T)},
            {"type": "ineq", "fun": lambda T: p[13] - np.linalg.norm(T)}]
    for _ in range(10):
        T = rng.normal(size=3) * 4
        _, pu_ = oracle.project_node(p, np.r_[2.0, 4, 0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0], np.r_[T, 1.0])
        r = minimize(lambda z: np.sum((z - T) ** 2), x0=np.array([1.0, 0, 0]), constraints=cons,
                     method="SLSQP", options=dict(ftol=1e-14, maxiter=500))
        np.testing.assert_allclose(pu_[:3], r.x, atol=1e-5)


def _node_set_qp(K, over_params, xf_w=(0.0, 0.0, 0.0), iters=0):
    """Scaled QP at the initial guess of the single-instance problem with parameters changed
    so that every node-wise set binds early (tight thrust ball and gimbal, glide slope near the
    straight-line guess, small tilt and rate bounds, dry mass near the wet mass), and a landing
    condition with nonzero transverse rates; returns (cfg, qp, node) with the reference and
    scales the node-wise projections act through."""
    cfg = I.solver_settings("C0", node_projections=31)
    inst = I.make_instances("C0")
    x0, xf, p = inst["x0"][0].copy(), inst["xf"][0].copy(), inst["params"][0].copy()
    for i, v in over_params.items():
        p[i] = v
    xf[10:13] = xf_w
    xb, ub = oracle.init_guess(K, x0, xf, p)
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, cfg["rk4_substeps"])
    qp = oracle.build_qp(cfg, p, K, x0, xf, xb, ub, xe, A, Bm, Bp)
    node = dict(xbar=xb, ubar=ub, px=cfg["px"], pu=cfg["pu"], p=p, mask=31)
    return cfg, qp, node


TIGHT = {1: 1.995, 13: 2.02, 14: np.radians(4.0), 15: np.radians(44.0), 16: np.radians(1.5),
         17: 0.0075}


@pytest.mark.parametrize("K,n_iter", [(4, 40), (6, 60)])
def test_pipg_custom_equals_generic_pipg_node_sets(K, n_iter):
    # with every node-wise convex set on, at the real prescaling and a nonzero reference: the
    # block solver (projections through the reference and the scales, the rate ball's slice at
    # the last node) gives the iterates of the generic PIPG on the dense form, whose projection
    # is written from the sets' geometry; every set binds during the run
    cfg, qp, node = _node_set_qp(K, TIGHT, xf_w=(0.004, 0.0055, -0.005))
    sigma, _ = oracle.power(cfg, qp)
    alpha, beta = _alpha_beta(cfg, sigma)
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    active = {}
    z, w, v = DQ.pipg_generic(D, qp, alpha, beta, cfg["rho"], n_iter, node=node, active=active)
    sol, n = oracle.pipg(cfg, qp, sigma, n_iter, 0, ref=(node["xbar"], node["ubar"], node["p"]))
    print("\nsets that moved an iterate (count over nodes and steps):", active)
    assert set(active) >= {"mass", "glide", "tilt", "rate", "rate slice", "thrust"}
    np.testing.assert_allclose(DQ.join(sol), z, atol=1e-10)
    np.testing.assert_allclose(sol["phi"].ravel(), w, atol=1e-10)
    np.testing.assert_allclose(sol["th"], v, atol=1e-10)


def test_pipg_fixed_point_certificate_node_sets():
    # the returned point of a long run with every node-wise set on satisfies the
    # projected-gradient fixed point with the dense projection, primal feasibility and
    # complementarity, and lies in every set
    K = 5
    cfg, qp, node = _node_set_qp(K, TIGHT, xf_w=(0.004, 0.0055, -0.005))
    sigma, _ = oracle.power(cfg, qp)
    alpha, beta = _alpha_beta(cfg, sigma)
    sol, _ = oracle.pipg(cfg, qp, sigma, 800000, 0, ref=(node["xbar"], node["ubar"], node["p"]))
    D = DQ.assemble(qp, cfg["w_prox"], cfg["w_cost"], cfg["w_ep"])
    z = DQ.join(sol)
    grad = D["P"] * z + D["p"] + D["G"].T @ sol["phi"].ravel() + D["H"].T @ sol["th"]
    active = {}
    assert np.abs(DQ.project(z - alpha * grad, qp, K, node, active) - z).max() < 1e-7
    print("\nsets active at the fixed point:", active)
    assert len(active) >= 2
    assert np.abs(D["G"] @ z - D["g"]).max() < 1e-7
    slack = D["H"] @ z - D["h"]
    assert slack.max() < 1e-7
    assert np.abs(sol["th"] * slack).max() < 1e-7
    # the point is its own projection (it lies in every set)
    np.testing.assert_allclose(DQ.project(z, qp, K, node), z, atol=1e-12)


def test_dense_cone_projection_against_brute_force():
    # the dense module's geometric cone projection is itself pinned by constrained minimization
    rng = np.random.default_rng(21)
    for a in (0.3, 1.0, 2.7):
        for _ in range(10):
            t, z = rng.normal() * 2, rng.normal(size=2) * 2
            pt, pz = DQ.cone_project(t, z, a)
            cons = [{"type": "ineq", "fun": lambda v: a * v[0] - np.linalg.norm(v[1:])}]
            r = minimize(lambda v: np.sum((v - np.r_[t, z]) ** 2), x0=np.array([1.0, 0, 0]),
                         constraints=cons, method="SLSQP",
                         options=dict(ftol=1e-15, maxiter=500))
            np.testing.assert_allclose(np.r_[pt, pz], r.x, atol=1e-5)
