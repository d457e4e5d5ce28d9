"""Dense canonical form of the scaled convex subproblem, assembled from its blocks.

Test helper: it writes out the canonical QP data (P, p, G, g, H, h) of the paper's
"Convex Optimization Solver" section, so that the block-structured solver can be checked
against generic dense linear algebra.  Variable order z = (x_1..x_N, u_1..u_N, mu+, mu-);
the dynamics rows carry +mu+ and -mu- (the subproblem's constraint as printed).  The
node-wise convex sets are projected here from their geometry, independently of the oracle's
closed forms.
"""
import numpy as np

NX, NU = 15, 4
IY = 14


def sizes(K, n_u=NU):
    M = K - 1
    nx, nu, nm = K * NX, K * n_u, M * NX
    return M, nx, nu, nm, nx + nu + 2 * nm


def assemble(qp, w_prox, w_cost, w_ep):
    Am, Bm, Bp = qp["Am"], qp["Bm"], qp["Bp"]
    K = Am.shape[0] + 1
    n_u = Bm.shape[-1]
    M, nx, nu, nm, n = sizes(K, n_u)
    G = np.zeros((M * NX, n))
    for k in range(M):
        r = slice(k * NX, (k + 1) * NX)
        G[r, k * NX:(k + 1) * NX] = Am[k]
        G[r, (k + 1) * NX:(k + 2) * NX] = -np.eye(NX)
        G[r, nx + k * n_u:nx + (k + 1) * n_u] = Bm[k]
        G[r, nx + (k + 1) * n_u:nx + (k + 2) * n_u] = Bp[k]
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
    return dict(P=P, p=p, G=G, g=g, H=H, h=h, K=K, n=n, n_u=n_u)


def split(z, K, n_u=NU):
    M, nx, nu, nm, n = sizes(K, n_u)
    return dict(x=z[:nx].reshape(K, NX), u=z[nx:nx + nu].reshape(K, n_u),
                mup=z[nx + nu:nx + nu + nm].reshape(M, NX),
                mum=z[nx + nu + nm:].reshape(M, NX))


def join(d):
    return np.concatenate([d["x"].ravel(), d["u"].ravel(), d["mup"].ravel(), d["mum"].ravel()])


FINAL_FIXED = [1, 2, 3, 4, 5, 6, 9, 10, 12, 13]   # r, v, (q2, q3), (w2, w3)


def cone_project(t, z, a):
    """Projection of (t, z) onto the cone {||z|| <= a t}, from its geometry: with half-angle
    b = atan(a) and phi the angle between (t, z) and the axis, a point with phi <= b is kept,
    one with phi >= b + pi/2 (the polar cone) goes to the apex, and any other goes to the
    nearest generator, the ray at angle b in the plane of the axis and the point, at distance
    |(t, z)| cos(phi - b) from the apex."""
    z = np.asarray(z, dtype=np.float64)
    nz = np.linalg.norm(z)
    phi = np.arctan2(nz, t)
    b = np.arctan(a)
    if phi <= b:
        return t, z.copy()
    if phi >= b + np.pi / 2:
        return 0.0, np.zeros_like(z)
    L = np.hypot(t, nz) * np.cos(phi - b)
    return L * np.cos(b), L * np.sin(b) * z / nz


def ball_project(z, rad):
    n = np.linalg.norm(z)
    return z * (rad / n) if n > rad else z.copy()


def node_sets_project(x, u, p, mask, last, active=None):
    """The node-wise convex sets in original units (bits: 1 dry mass, 2 glide-slope cone on r,
    4 tilt disk on (q2, q3), 8 rate ball on w, 16 gimbal cone and T_max ball on T), for a node
    whose boundary values are already in x.  At the last node r, v, (q2, q3) and (w2, w3) are
    fixed: only the mass bound and the slice of the rate ball through the fixed transverse
    rates act there.  `active` (a dict) counts the sets that moved the point."""
    x, u = x.copy(), u.copy()

    def mark(name, before, after):
        if active is not None and not np.allclose(before, after, rtol=0, atol=0):
            active[name] = active.get(name, 0) + 1

    if mask & 1:
        m = max(x[0], p[1])
        mark("mass", x[0], m)
        x[0] = m
    if (mask & 2) and not last:
        t, z = cone_project(x[1], x[2:4], 1.0 / np.tan(p[15]))
        mark("glide", x[1:4], np.r_[t, z])
        x[1], x[2:4] = t, z
    if (mask & 4) and not last:
        q = ball_project(x[9:11], np.sqrt(0.5 * (1.0 - np.cos(p[16]))))
        mark("tilt", x[9:11], q)
        x[9:11] = q
    if mask & 8:
        if last:
            r = np.sqrt(max(p[17] ** 2 - x[12] ** 2 - x[13] ** 2, 0.0))
            w1 = min(max(x[11], -r), r)
            mark("rate slice", x[11], w1)
            x[11] = w1
        else:
            w = ball_project(x[11:14], p[17])
            mark("rate", x[11:14], w)
            x[11:14] = w
    if mask & 16:
        t, z = cone_project(u[0], u[1:3], np.tan(p[14]))
        T = ball_project(np.r_[t, z], p[13])
        mark("thrust", u[:3], T)
        u[:3] = T
    return x, u


def project(z, qp, K, node=None, active=None):
    """Projection onto the subproblem's constraint set: boundary values, the u box, mu >= 0
    (the paper's set), and with `node` = dict(xbar, ubar, px, pu, p, mask) the node-wise
    convex sets, which act in original units x = xbar + px x^, u = ubar + pu u^."""
    d = split(z.copy(), K, qp["umin"].shape[-1])
    d["x"][0, :] = qp["zi"]
    for i in FINAL_FIXED:
        d["x"][K - 1, i] = qp["zf"][i - 1]
    d["u"] = np.minimum(np.maximum(d["u"], qp["umin"]), qp["umax"])
    if node is not None and node["mask"]:
        px, pu = np.asarray(node["px"]), np.asarray(node["pu"])
        for k in range(K):
            x = node["xbar"][k] + px * d["x"][k]
            u = node["ubar"][k] + pu * d["u"][k]
            if k == 0:
                mask = node["mask"] & 16          # the first node's state is fixed entirely
            else:
                mask = node["mask"]
            x, u = node_sets_project(x, u, node["p"], mask, k == K - 1 and k > 0, active)
            d["x"][k] = (x - node["xbar"][k]) / px
            d["u"][k] = (u - node["ubar"][k]) / pu
    d["mup"] = np.maximum(d["mup"], 0.0)
    d["mum"] = np.maximum(d["mum"], 0.0)
    return join(d)


def pipg_generic(D, qp, alpha, beta, rho, n_iter, z0=None, eta0=None, chi0=None, node=None,
                 active=None):
    """The generic extrapolated PIPG (Algorithm 1) on the dense data."""
    K = D["K"]
    zeta = np.zeros(D["n"]) if z0 is None else z0.copy()
    eta = np.zeros(D["G"].shape[0]) if eta0 is None else eta0.copy()
    chi = np.zeros(D["H"].shape[0]) if chi0 is None else chi0.copy()
    for _ in range(n_iter):
        grad = D["P"] * zeta + D["p"] + D["G"].T @ eta + D["H"].T @ chi
        z = project(zeta - alpha * grad, qp, K, node, active)
        w = eta + beta * (D["G"] @ (2 * z - zeta) - D["g"])
        v = np.maximum(0.0, chi + beta * (D["H"] @ (2 * z - zeta) - D["h"]))
        zeta = (1 - rho) * zeta + rho * z
        eta = (1 - rho) * eta + rho * w
        chi = (1 - rho) * chi + rho * v
    return z, w, v
