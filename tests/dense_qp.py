"""Dense canonical form of the scaled convex subproblem, assembled from its blocks.

Test helper: it writes out the canonical QP data (P, p, G, g, H, h) of the paper's
"Convex Optimization Solver" section, so that the block-structured solver can be checked
against generic dense linear algebra.  Variable order z = (x_1..x_N, u_1..u_N, mu+, mu-);
the dynamics rows carry +mu+ and -mu- (the subproblem's constraint as printed).
"""
import numpy as np

NX, NU = 15, 4
IY = 14


def sizes(K):
    M = K - 1
    nx, nu, nm = K * NX, K * NU, M * NX
    return M, nx, nu, nm, nx + nu + 2 * nm


def assemble(qp, w_prox, w_cost, w_ep):
    Am, Bm, Bp = qp["Am"], qp["Bm"], qp["Bp"]
    K = Am.shape[0] + 1
    M, nx, nu, nm, n = sizes(K)
    G = np.zeros((M * NX, n))
    for k in range(M):
        r = slice(k * NX, (k + 1) * NX)
        G[r, k * NX:(k + 1) * NX] = Am[k]
        G[r, (k + 1) * NX:(k + 2) * NX] = -np.eye(NX)
        G[r, nx + k * NU:nx + (k + 1) * NU] = Bm[k]
        G[r, nx + (k + 1) * NU:nx + (k + 2) * NU] = Bp[k]
        G[r, nx + nu + k * NX:nx + nu + (k + 1) * NX] = np.eye(NX)
        G[r, nx + nu + nm + k * NX:nx + nu + nm + (k + 1) * NX] = -np.eye(NX)
    g = -qp["w"].reshape(-1) if "w" in qp else np.zeros(M * NX)
    H = np.zeros((M, n))
    for k in range(M):
        H[k, k * NX + IY] = -1.0
        H[k, (k + 1) * NX + IY] = 1.0
    h = qp["eps"].copy() if "eps" in qp else np.zeros(M)
    P = np.zeros(n)
    P[:nx + nu] = w_prox
    p = np.zeros(n)
    p[(K - 1) * NX + 0] = -w_cost          # e_cost = -e_m on the final node
    p[nx + nu:] = w_ep
    return dict(P=P, p=p, G=G, g=g, H=H, h=h, K=K, n=n)


def split(z, K):
    M, nx, nu, nm, n = sizes(K)
    return dict(x=z[:nx].reshape(K, NX), u=z[nx:nx + nu].reshape(K, NU),
                mup=z[nx + nu:nx + nu + nm].reshape(M, NX),
                mum=z[nx + nu + nm:].reshape(M, NX))


def join(d):
    return np.concatenate([d["x"].ravel(), d["u"].ravel(), d["mup"].ravel(), d["mum"].ravel()])


FINAL_FIXED = [1, 2, 3, 4, 5, 6, 9, 10, 12, 13]   # r, v, (q2, q3), (w2, w3)


def project(z, qp, K):
    """Projection onto the paper's set: boundary values, the u box, mu >= 0."""
    d = split(z.copy(), K)
    d["x"][0, :] = qp["zi"]
    for i in FINAL_FIXED:
        d["x"][K - 1, i] = qp["zf"][i - 1]
    d["u"] = np.minimum(np.maximum(d["u"], qp["umin"]), qp["umax"])
    d["mup"] = np.maximum(d["mup"], 0.0)
    d["mum"] = np.maximum(d["mum"], 0.0)
    return join(d)


def pipg_generic(D, qp, alpha, beta, rho, n_iter, z0=None, eta0=None, chi0=None):
    """The generic extrapolated PIPG (Algorithm 1) on the dense data."""
    K = D["K"]
    zeta = np.zeros(D["n"]) if z0 is None else z0.copy()
    eta = np.zeros(D["G"].shape[0]) if eta0 is None else eta0.copy()
    chi = np.zeros(D["H"].shape[0]) if chi0 is None else chi0.copy()
    for _ in range(n_iter):
        grad = D["P"] * zeta + D["p"] + D["G"].T @ eta + D["H"].T @ chi
        z = project(zeta - alpha * grad, qp, K)
        w = eta + beta * (D["G"] @ (2 * z - zeta) - D["g"])
        v = np.maximum(0.0, chi + beta * (D["H"] @ (2 * z - zeta) - D["h"]))
        zeta = (1 - rho) * zeta + rho * z
        eta = (1 - rho) * eta + rho * w
        chi = (1 - rho) * chi + rho * v
    return z, w, v
