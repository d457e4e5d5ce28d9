"""Pins of the oracle's discretization (section "Gradient of Discretized Dynamics"): RK4 on
the state and variational equations with a first-order-hold control."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from paper_2404_18034_amd import instances as I

NX, NU = 15, 4


def rk4_poly(Z):
    """Stability polynomial of classical RK4: I + Z + Z^2/2 + Z^3/6 + Z^4/24."""
    n = Z.shape[0]
    out, term = np.eye(n), np.eye(n)
    for j in range(1, 5):
        term = term @ Z / j
        out = out + term
    return out


def linear_model(rng):
    A0 = rng.normal(size=(NX, NX)) * 0.4
    B0 = rng.normal(size=(NX, NU)) * 0.4
    return A0, B0


def foh_generator(A0, B0, dtau):
    """Autonomous LTI form of x' = A0 x + B0 (u_k + (u_k+1 - u_k) sigma / dtau):
    state (x, v0, v1) with v0 the held input and v1 its constant slope."""
    n = NX + 2 * NU
    Mg = np.zeros((n, n))
    Mg[:NX, :NX] = A0
    Mg[:NX, NX:NX + NU] = B0
    Mg[NX:NX + NU, NX + NU:] = np.eye(NU)
    return Mg


def split_foh(E, dtau):
    """x(dtau) = Exx x0 + Ex0 u_k + Ex1 (u_k+1 - u_k)/dtau  ->  (A, B-, B+)."""
    Exx, Ex0, Ex1 = E[:NX, :NX], E[:NX, NX:NX + NU], E[:NX, NX + NU:]
    return Exx, Ex0 - Ex1 / dtau, Ex1 / dtau


@pytest.mark.parametrize("nsub", [1, 3, 10])
def test_linear_model_equals_rk4_polynomial(nsub):
    # RK4 applied to a linear autonomous system is exactly R(hM)^n: every block of the
    # jointly integrated variational system must match it to rounding.
    rng = np.random.default_rng(nsub)
    A0, B0 = linear_model(rng)
    dtau = 0.3
    h = dtau / nsub
    xk, uk, uk1 = rng.normal(size=NX), rng.normal(size=NU), rng.normal(size=NU)
    xe, A, Bm, Bp = oracle.discretize_interval(xk, uk, uk1, None, dtau, nsub, A0, B0)
    Mg = foh_generator(A0, B0, dtau)
    E = np.linalg.matrix_power(rk4_poly(h * Mg), nsub)
    Ae, Bme, Bpe = split_foh(E, dtau)
    np.testing.assert_allclose(A, np.linalg.matrix_power(rk4_poly(h * A0), nsub), atol=1e-13)
    np.testing.assert_allclose(A, Ae, atol=1e-13)
    np.testing.assert_allclose(Bm, Bme, atol=1e-13)
    np.testing.assert_allclose(Bp, Bpe, atol=1e-13)
    np.testing.assert_allclose(xe, Ae @ xk + Bme @ uk + Bpe @ uk1, atol=1e-13)


def test_linear_model_converges_to_matrix_exponential_at_fourth_order():
    rng = np.random.default_rng(7)
    A0, B0 = linear_model(rng)
    dtau = 0.5
    xk, uk, uk1 = rng.normal(size=NX), rng.normal(size=NU), rng.normal(size=NU)
    Ae, Bme, Bpe = split_foh(expm(dtau * foh_generator(A0, B0, dtau)), dtau)
    errs = []
    for nsub in (4, 8, 16):
        _, A, Bm, Bp = oracle.discretize_interval(xk, uk, uk1, None, dtau, nsub, A0, B0)
        errs.append(max(np.abs(A - Ae).max(), np.abs(Bm - Bme).max(), np.abs(Bp - Bpe).max()))
    assert errs[-1] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0          # O(h^4): error ratio ~16 on halving h


@pytest.mark.parametrize("trial", range(3))
def test_variational_equals_jacobian_of_rk4_map(trial):
    # Integrating the variational equations jointly with RK4 gives the exact Jacobian of
    # the discrete RK4 endpoint map, so central differences agree to their own error.
    rng = np.random.default_rng(100 + trial)
    inst = I.make_instances("C4", ids=[trial])
    p = inst["params"][0]
    q = rng.normal(size=4); q /= np.linalg.norm(q)
    x = np.concatenate([[1.9], rng.normal(size=3) * 3, rng.normal(size=3), q,
                        rng.normal(size=3) * 0.5, [0.0]])
    uk = np.concatenate([rng.normal(size=3) + [2, 0, 0], [4.0]])
    uk1 = np.concatenate([rng.normal(size=3) + [2, 0, 0], [5.0]])
    dtau, nsub, h = 1.0 / 19, 5, 1e-6
    end = lambda a, b, c: oracle.discretize_interval(a, b, c, p, dtau, nsub)[0]
    _, A, Bm, Bp = oracle.discretize_interval(x, uk, uk1, p, dtau, nsub)
    Af = np.stack([(end(x + h * e, uk, uk1) - end(x - h * e, uk, uk1)) / (2 * h)
                   for e in np.eye(NX)], axis=1)
    Bmf = np.stack([(end(x, uk + h * e, uk1) - end(x, uk - h * e, uk1)) / (2 * h)
                    for e in np.eye(NU)], axis=1)
    Bpf = np.stack([(end(x, uk, uk1 + h * e) - end(x, uk, uk1 - h * e)) / (2 * h)
                    for e in np.eye(NU)], axis=1)
    for got, want in ((A, Af), (Bm, Bmf), (Bp, Bpf)):
        assert np.abs(got - want).max() <= 1e-7 * max(1.0, np.abs(want).max())


def test_free_fall_interval_is_exact():
    # T = 0, constant s: r and v are polynomials of degree <= 2, which RK4 integrates exactly
    p = I.nominal_params()
    x = np.zeros(NX); x[0] = 2.0; x[1:4] = [4, 4, 0]; x[4:7] = [-1, -2, 0]; x[7] = 1.0
    u = np.array([0.0, 0.0, 0.0, 4.0])
    dtau = 0.25
    xe, A, Bm, Bp = oracle.discretize_interval(x, u, u, p, dtau, 3)
    t = 4.0 * dtau
    np.testing.assert_allclose(xe[1:4], x[1:4] + x[4:7] * t + 0.5 * p[3:6] * t * t, atol=1e-14)
    np.testing.assert_allclose(xe[4:7], x[4:7] + p[3:6] * t, atol=1e-14)
    assert xe[0] == 2.0
    # the mass row of A is e_m and the y column is e_y (nothing depends on y)
    np.testing.assert_array_equal(A[0], np.eye(NX)[0])
    np.testing.assert_array_equal(A[:, 14], np.eye(NX)[14])


def test_discretize_all_intervals_matches_single():
    inst = I.make_instances("C0")
    x0, xf, p, K = inst["x0"][0], inst["xf"][0], inst["params"][0], int(inst["K"][0])
    xb, ub = oracle.init_guess(K, x0, xf, p)
    xe, A, Bm, Bp = oracle.discretize(K, xb, ub, p, 5)
    for k in (0, K // 2, K - 2):
        r = oracle.discretize_interval(xb[k], ub[k], ub[k + 1], p, 1.0 / (K - 1), 5)
        for a, b in zip(r, (xe[k], A[k], Bm[k], Bp[k])):
            np.testing.assert_array_equal(a, b)


def test_initial_guess_reading():
    inst = I.make_instances("C1", B=3)
    for b in range(3):
        x0, xf, p = inst["x0"][b], inst["xf"][b], inst["params"][b]
        xb, ub = oracle.init_guess(20, x0, xf, p)
        np.testing.assert_array_equal(xb[0, :7], x0[:7])
        np.testing.assert_array_equal(xb[0, 11:14], x0[11:14])
        # q is normalized (float32-rounded inputs are unit only to ~1e-7)
        np.testing.assert_allclose(xb[0, 7:11], x0[7:11] / np.linalg.norm(x0[7:11]), atol=1e-15)
        np.testing.assert_allclose(xb[-1, 1:14], xf, atol=1e-15)
        np.testing.assert_allclose(np.linalg.norm(xb[:, 7:11], axis=1), 1.0, atol=1e-15)
        assert np.all(xb[:, 0] == x0[0]) and np.all(xb[:, 14] == 0.0)
        np.testing.assert_allclose(ub[:, 0], x0[0] * np.linalg.norm(p[3:6]))
        assert np.all(ub[:, 1:3] == 0.0) and np.all(ub[:, 3] == p[21])
