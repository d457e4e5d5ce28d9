"""Pins of the oracle's 6-DoF model (section "6-DoF Powered Descent Guidance") against closed
forms, finite differences and a library matrix exponential."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from paper_2404_18034_amd import instances as I

RNG = np.random.default_rng(20240418)


def rand_state(rng, scale=1.0):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return np.concatenate([[1.5 + 0.4 * rng.random()], rng.normal(size=3) * 3 * scale,
                           rng.normal(size=3) * scale, q, rng.normal(size=3) * 0.5 * scale,
                           [0.01]])


def rand_params(rng):
    p = I.nominal_params()
    p[6:9] = 0.01 * (1 + 0.2 * rng.uniform(-1, 1, 3))      # anisotropic inertia
    p[9:12] = [-0.01, 0.002 * rng.normal(), 0.002 * rng.normal()]
    p[22] = 1.0 + rng.random()                              # a speed bound (active at |v| > 2)
    return p


def skew(a):
    return np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])


def rodrigues(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.cos(ang) * np.eye(3) + (1 - np.cos(ang)) * np.outer(a, a) + np.sin(ang) * skew(a)


def dcm_from_dynamics(q, T, m, p):
    """Recover C(q) T from v_dot = C T / m + g, with s = 1."""
    x = np.zeros(15); x[0] = m; x[7:11] = q
    f = oracle.dynamics(x, np.concatenate([T, [1.0]]), p)
    return (f[4:7] - p[3:6]) * m


def test_dcm_matches_rodrigues():
    # q = (cos(a/2), sin(a/2) n) is a rotation by angle a about n (body -> inertial)
    p = I.nominal_params()
    for _ in range(5):
        n = RNG.normal(size=3); n /= np.linalg.norm(n)
        a = RNG.uniform(0, np.pi)
        q = np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * n])
        R = rodrigues(n, a)
        C = np.stack([dcm_from_dynamics(q, e, 1.0, p) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(C, R, atol=1e-14)


def test_free_fall_closed_form():
    # T = 0: no mass flow, v_dot = g, r_dot = v; isotropic J -> w_dot = 0
    p = I.nominal_params()
    x = rand_state(RNG)
    f = oracle.dynamics(x, np.array([0.0, 0.0, 0.0, 2.5]), p)
    assert f[0] == 0.0
    np.testing.assert_allclose(f[1:4], 2.5 * x[4:7], rtol=1e-15)
    np.testing.assert_allclose(f[4:7], 2.5 * p[3:6], rtol=1e-15)
    np.testing.assert_allclose(f[11:14], 0.0, atol=1e-15)


def test_mass_flow_and_torque():
    p = rand_params(RNG)
    x = rand_state(RNG)
    T = np.array([2.0, 0.3, -0.4])
    f = oracle.dynamics(x, np.concatenate([T, [1.0]]), p)
    assert f[0] == pytest.approx(-p[2] * np.linalg.norm(T), rel=1e-15)
    w, J, rT = x[11:14], p[6:9], p[9:12]
    want = (np.cross(rT, T) - np.cross(w, J * w)) / J
    np.testing.assert_allclose(f[11:14], want, rtol=1e-13)


def test_quaternion_kinematics_against_expm():
    # q_dot = 0.5 Omega(w) q with constant body rate: C(q(t)) = C(q0) expm(t [w x]).
    # T = 0 and isotropic J keep w constant; integrate with many small RK4 steps.
    p = I.nominal_params()
    w = np.array([0.3, -0.2, 0.5])
    q0 = np.array([np.cos(0.2), np.sin(0.2), 0.0, 0.0])
    x = np.zeros(15); x[0] = 2.0; x[7:11] = q0; x[11:14] = w
    u = np.array([0.0, 0.0, 0.0, 1.0])
    xe, *_ = oracle.discretize_interval(x, u, u, p, 1.0, 200)
    Cq = lambda q: np.stack([dcm_from_dynamics(q, e, 1.0, p) for e in np.eye(3)], axis=1)
    np.testing.assert_allclose(Cq(xe[7:11]), Cq(q0) @ expm(skew(w)), atol=1e-10)
    assert np.linalg.norm(xe[7:11]) == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("trial", range(6))
def test_jacobians_against_central_differences(trial):
    rng = np.random.default_rng(trial)
    p = rand_params(rng)
    x = rand_state(rng, scale=2.0)        # large enough to activate several constraints
    u = np.concatenate([rng.normal(size=3) * 3, [3.0 + rng.random()]])
    A, B = oracle.jacobians(x, u, p)
    h = 1e-6
    Af = np.stack([(oracle.dynamics(x + h * e, u, p) - oracle.dynamics(x - h * e, u, p)) / (2 * h)
                   for e in np.eye(15)], axis=1)
    Bf = np.stack([(oracle.dynamics(x, u + h * e, p) - oracle.dynamics(x, u - h * e, p)) / (2 * h)
                   for e in np.eye(4)], axis=1)
    scale = max(1.0, np.abs(A).max())
    assert np.abs(A - Af).max() <= 1e-6 * scale
    assert np.abs(B - Bf).max() <= 1e-6 * max(1.0, np.abs(B).max())


def test_ctcs_integrand_is_sum_of_squared_violations():
    p = I.nominal_params()
    x = rand_state(RNG, scale=2.0)
    u = np.array([0.1, 2.0, 0.0, 3.0])         # gimbal and T_min rows violated
    g = oracle.constraints(x, u, p)
    f = oracle.dynamics(x, u, p)
    assert f[14] == pytest.approx(3.0 * np.sum(np.maximum(g, 0.0) ** 2), rel=1e-14)


def test_speed_bound_row():
    # the speed row ||v||^2 - v_max^2 of the constraint list; without a bound (v_max = inf,
    # the nominal value) it is the constant -1 and never enters the CTCS integrand
    p = I.nominal_params()
    assert np.isinf(p[22])
    x = rand_state(RNG)
    x[4:7] = [1.5, -2.0, 0.5]
    u = np.array([2.0, 0.0, 0.0, 3.0])
    assert oracle.constraints(x, u, p)[7] == -1.0
    pv = p.copy(); pv[22] = 2.0
    g = oracle.constraints(x, u, pv)
    assert g[7] == pytest.approx(1.5 ** 2 + 2.0 ** 2 + 0.5 ** 2 - 4.0, abs=1e-14)
    np.testing.assert_array_equal(g[:7], oracle.constraints(x, u, p)[:7])
    # the augmented dynamics gain s * [g_8]_+^2 in the y row and nothing else
    f, fv = oracle.dynamics(x, u, p), oracle.dynamics(x, u, pv)
    np.testing.assert_array_equal(f[:14], fv[:14])
    assert fv[14] - f[14] == pytest.approx(3.0 * g[7] ** 2, rel=1e-12)
    # on the bound the row is zero
    x[4:7] *= 2.0 / np.linalg.norm(x[4:7])
    assert oracle.constraints(x, u, pv)[7] == pytest.approx(0.0, abs=1e-14)


def test_constraint_readings():
    p = I.nominal_params()
    # glide slope: the boundary point tan(gamma)*||(r2, r3)|| = r1 gives g2 = 0
    x = rand_state(RNG)
    lat = np.array([1.2, -0.7]); x[2:4] = lat
    x[1] = np.tan(p[15]) * np.linalg.norm(lat)
    assert oracle.constraints(x, np.array([1, 0, 0, 1.0]), p)[1] == pytest.approx(0.0, abs=1e-14)
    # tilt: g3 <= 0  <=>  the body x axis is within theta_max of vertical (C11 >= cos theta_max)
    for _ in range(50):
        q = RNG.normal(size=4); q /= np.linalg.norm(q)
        x[7:11] = q
        C11 = dcm_from_dynamics(q, np.array([1.0, 0, 0]), 1.0, p)[0]
        for th in (np.radians(30.0), np.radians(90.0)):
            pp = p.copy(); pp[16] = th
            g3 = oracle.constraints(x, np.array([1, 0, 0, 1.0]), pp)[2]
            assert g3 == pytest.approx(np.cos(th) - C11, abs=1e-14)
    # gimbal: a thrust exactly on the cone edge is on the boundary
    d = p[14]
    T = np.array([np.cos(d), np.sin(d), 0.0]) * 2.0
    assert oracle.constraints(x, np.concatenate([T, [1.0]]), p)[4] == pytest.approx(0, abs=1e-14)


def test_initial_condition_is_feasible():
    inst = I.make_instances("C1", B=64)
    for b in range(64):
        x0 = inst["x0"][b]
        u = np.array([x0[0], 0.0, 0.0, 5.0])
        assert np.all(oracle.constraints(x0, u, inst["params"][b]) <= 1e-12)
