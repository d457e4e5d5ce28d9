"""Seeded synthetic Monte Carlo instances and solver configurations.

This module only draws inputs: it holds none of the solver's arithmetic, so that the GPU
library and the independent CPU oracle can be fed exactly the same problem data.

Random numbers come from a counter-based SplitMix64 generator (Steele, Lea, Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): draw ``d`` of instance ``i``
under seed ``s`` is ``splitmix64(splitmix64(s) + 64*i + d)``, whose top 53 bits give a
uniform number in [0, 1).  Any instance can be regenerated on its own from (seed, i).

Instance layout (float64, row-major), matching the library's boundary:
  x0[B,15] = (m0, r0[3], v0[3], q0[4], w0[3], y0 = 0)
  xf[B,13] = (r_f[3], v_f[3], q_f[4], w_f[3])
  params[B,24] = m_wet, m_dry, alpha_mdot, g[3], J_diag[3], r_T[3], T_min, T_max,
                 delta_max, gamma_gs, theta_max, omega_max, s_min, s_max, eps_ctcs, s_init,
                 v_max (+inf: no speed bound), gamma_max (bound of the reaction-control
                 torque; read only by solves with the torque input, n_u = 7)
  K[B] int32 node counts.
The nominal vehicle is the nondimensional lander of the paper's 6-DoF example with the
values stated for the single-instance case (g = (-1,0,0), m_wet = 2, m_dry = 1,
J = 0.01 I, r_T = (-0.01,0,0), alpha = 0.01, T in [0.3, 5], 20 deg gimbal and glide slope,
90 deg tilt, 60 deg/s rate); dispersions are uniform around it.
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1

# Draw ids inside one instance's counter block.
D_R0, D_V0, D_M0, D_TILT, D_PSI, D_K, D_J, D_RT = 0, 3, 6, 7, 8, 9, 10, 13


def splitmix64(z):
    """One SplitMix64 output for a 64-bit state increment (vectorised over uint64 arrays)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, idx, draw):
    """U[0,1) for instance ids ``idx`` (array) and draw id ``draw`` under ``seed``."""
    base = splitmix64(np.uint64(seed & MASK64))
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = base + idx * np.uint64(64) + np.uint64(draw)
    z = splitmix64(ctr)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def sym(seed, idx, draw, half):
    """U(-half, +half)."""
    return (2.0 * uniform01(seed, idx, draw) - 1.0) * half


NOMINAL = dict(
    m_wet=2.0, m_dry=1.0, alpha_mdot=0.01, g=(-1.0, 0.0, 0.0), J=(0.01, 0.01, 0.01),
    r_T=(-0.01, 0.0, 0.0), T_min=0.3, T_max=5.0, delta_max=math.radians(20.0),
    gamma_gs=math.radians(20.0), theta_max=math.radians(90.0), omega_max=math.radians(60.0),
    s_min=0.1, s_max=20.0, eps_ctcs=1e-4, s_init=5.0, v_max=math.inf, gamma_max=0.005,
    r0=(4.0, 4.0, 0.0), v0=(-1.0, -2.0, 0.0), rf=(0.0, 0.0, 0.0), vf=(-0.1, 0.0, 0.0),
)


def nominal_params():
    n = NOMINAL
    return np.array([n["m_wet"], n["m_dry"], n["alpha_mdot"], *n["g"], *n["J"], *n["r_T"],
                     n["T_min"], n["T_max"], n["delta_max"], n["gamma_gs"], n["theta_max"],
                     n["omega_max"], n["s_min"], n["s_max"], n["eps_ctcs"], n["s_init"],
                     n["v_max"], n["gamma_max"]],
                    dtype=np.float64)


# Frozen solver settings shared by every configuration (the paper leaves them open; they
# were chosen once on the oracle and are used unchanged by both implementations).
HYPER = dict(
    pipg_check_every=10, rk4_substeps=5, power_iters_max=50, node_projections=0, pad=0,
    scp_tol=1e-4, feas_tol=1e-4, pipg_eps_abs=1e-5, pipg_eps_rel=1e-5,
    power_eps_abs=0.0, power_eps_rel=1e-6, power_buff=0.1,
    w_cost=0.005, w_prox=0.3, w_ep=100.0, omega=16.0, rho=1.9,
    px=(1.0, 4.0, 4.0, 4.0, 2.0, 2.0, 2.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.1),
    pu=(5.0, 5.0, 5.0, 5.0),
)

# The workloads: dtype, batch, node counts, dispersion widths, solver budget, seed.
CONFIGS = {
    "C0": dict(name="single instance, FP64", B=1, K=(10,), dtype="f64", disp=None,
               scp_iters_max=15, pipg_iters_max=2000, early_exit=1, seed=0),
    "C1": dict(name="Monte Carlo 1,024 x K=20, FP32", B=1024, K=(20,), dtype="f32",
               disp=dict(r=0.5, v=0.2, m=0.05, tilt_deg=10.0, JrT=0.0),
               scp_iters_max=15, pipg_iters_max=1000, early_exit=0, seed=1),
    "C2": dict(name="uneven 16,384 x K in {10,20,30}, FP32", B=16384, K=(10, 20, 30),
               dtype="f32", disp=dict(r=1.0, v=0.4, m=0.1, tilt_deg=20.0, JrT=0.0),
               scp_iters_max=15, pipg_iters_max=1000, early_exit=1, seed=2),
    "C3": dict(name="differentiation 4,096 x K=20, FP32", B=4096, K=(20,), dtype="f32",
               disp=dict(r=0.5, v=0.2, m=0.05, tilt_deg=10.0, JrT=0.0),
               scp_iters_max=15, pipg_iters_max=1000, early_exit=0, seed=3,
               grad_pipg_steps=200, grad_ckpt_every=20),
    "C4": dict(name="throughput 65,536 x K=30, FP32", B=65536, K=(30,), dtype="f32",
               disp=dict(r=1.0, v=0.4, m=0.1, tilt_deg=20.0, JrT=0.1),
               scp_iters_max=15, pipg_iters_max=1000, early_exit=0, seed=4),
    # The paper's own Monte Carlo (section "Numerical Results"): 256 runs with the initial
    # position drawn from U(6,9) x U(3,6) x U(1,2), at most 25 SCP iterations, 2,500 PIPG
    # iterations per subproblem (a stopping-test period beyond the budget: never tested),
    # every other value nominal.  The paper does not state its node count: at K = 30 (and 25)
    # every one of these 256 runs converges within 25 SCP iterations, as the paper reports for
    # its own; at K = 20 eight of them (large r_x, small r_y) cycle without converging.
    "F1": dict(name="paper's Monte Carlo 256 x K=30, FP32", B=256, K=(30,), dtype="f32",
               disp=dict(r_box=((6.0, 9.0), (3.0, 6.0), (1.0, 2.0)), r=0.0, v=0.0, m=0.0,
                         tilt_deg=0.0, JrT=0.0),
               scp_iters_max=25, pipg_iters_max=2500, early_exit=1, pipg_check_every=2501,
               seed=5),
    # The same runs with the paper's speed bound ||v|| <= v_max (a path constraint of section
    # "6-DoF Powered Descent Guidance", enforced through the CTCS integrand) at v_max = 2.4:
    # every run starts at |v| = 2.24 and, unbounded, peaks between 2.42 and 2.50, so the bound
    # shapes every trajectory.
    "F1S": dict(name="paper's Monte Carlo 256 x K=30 with speed bound, FP32", B=256, K=(30,),
                dtype="f32",
                disp=dict(r_box=((6.0, 9.0), (3.0, 6.0), (1.0, 2.0)), r=0.0, v=0.0, m=0.0,
                          tilt_deg=0.0, JrT=0.0),
                scp_iters_max=25, pipg_iters_max=2500, early_exit=1, pipg_check_every=2501,
                seed=5, v_max=2.4),
    # The paper's full control set (section "6-DoF Powered Descent Guidance"): the same 256
    # runs with the reaction-control torque gamma as a control input beside the thrust,
    # u = (T, gamma, s), bounded by ||gamma|| <= gamma_max = 0.005 through the CTCS integrand
    # (a quarter of the largest torque the gimbaled thrust can exert); its prescaling is the
    # bound itself.
    "F2": dict(name="paper's Monte Carlo 256 x K=30 with torque control, FP32", B=256, K=(30,),
               dtype="f32",
               disp=dict(r_box=((6.0, 9.0), (3.0, 6.0), (1.0, 2.0)), r=0.0, v=0.0, m=0.0,
                         tilt_deg=0.0, JrT=0.0),
               scp_iters_max=25, pipg_iters_max=2500, early_exit=1, pipg_check_every=2501,
               seed=5, settings=dict(n_u=7, pu=(5.0, 5.0, 5.0, 0.005, 0.005, 0.005, 5.0))),
}


def solver_settings(config, **overrides):
    """Plain dict of solver settings for a configuration name (or a config dict)."""
    cfg = CONFIGS[config] if isinstance(config, str) else config
    s = dict(HYPER)
    for k in ("scp_iters_max", "pipg_iters_max", "early_exit"):
        s[k] = cfg[k]
    for k in ("grad_pipg_steps", "grad_ckpt_every", "pipg_check_every"):
        if k in cfg:
            s[k] = cfg[k]
    s.update(cfg.get("settings", {}))
    s.update(overrides)
    return s


def make_instances(config, B=None, ids=None, seed=None):
    """Generate instances of a configuration.

    ``ids`` selects instance ids (default ``range(B)``); an instance depends only on
    (seed, id).  FP32 configurations round every value to float32 (the GPU consumes the
    float32 values; the oracle consumes the same values widened to float64).
    Returns dict(x0, xf, params, K) of numpy arrays.
    """
    cfg = CONFIGS[config] if isinstance(config, str) else config
    seed = cfg["seed"] if seed is None else seed
    if ids is None:
        ids = np.arange(cfg["B"] if B is None else B, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    n = ids.shape[0]
    nom = NOMINAL
    r0 = np.tile(np.array(nom["r0"]), (n, 1))
    v0 = np.tile(np.array(nom["v0"]), (n, 1))
    m0 = np.full(n, nom["m_wet"])
    q0 = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    params = np.tile(nominal_params(), (n, 1))
    d = cfg["disp"]
    if d is not None:
        for a in range(3):
            if "r_box" in d:  # absolute box: r0[a] ~ U(lo, hi)
                lo, hi = d["r_box"][a]
                r0[:, a] = lo + (hi - lo) * uniform01(seed, ids, D_R0 + a)
            r0[:, a] += sym(seed, ids, D_R0 + a, d["r"])
            v0[:, a] += sym(seed, ids, D_V0 + a, d["v"])
        m0 += sym(seed, ids, D_M0, d["m"])
        tilt = uniform01(seed, ids, D_TILT) * math.radians(d["tilt_deg"])
        psi = uniform01(seed, ids, D_PSI) * 2.0 * math.pi
        # rotation by `tilt` about the horizontal axis (0, cos psi, sin psi)
        q0 = np.stack([np.cos(tilt / 2), np.zeros(n), np.sin(tilt / 2) * np.cos(psi),
                       np.sin(tilt / 2) * np.sin(psi)], axis=1)
        if d["JrT"] > 0.0:
            for a in range(3):
                params[:, 6 + a] *= 1.0 + sym(seed, ids, D_J + a, d["JrT"])
                params[:, 9 + a] *= 1.0 + sym(seed, ids, D_RT + a, d["JrT"])
    params[:, 0] = m0
    if "v_max" in cfg:
        params[:, 22] = cfg["v_max"]
    Ks = np.array(cfg["K"], dtype=np.int32)
    if len(Ks) == 1:
        K = np.full(n, Ks[0], dtype=np.int32)
    else:
        pick = np.minimum((uniform01(seed, ids, D_K) * len(Ks)).astype(np.int64), len(Ks) - 1)
        K = Ks[pick]
    x0 = np.concatenate([m0[:, None], r0, v0, q0, np.zeros((n, 3)), np.zeros((n, 1))], axis=1)
    xf = np.tile(np.array([*nom["rf"], *nom["vf"], 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]), (n, 1))
    out = dict(x0=x0, xf=xf, params=params, K=K)
    if cfg["dtype"] == "f32":
        for k in ("x0", "xf", "params"):
            out[k] = out[k].astype(np.float32).astype(np.float64)
    return out


def multistart(inst, s_init):
    """Multi-start batch: problem p of `inst` repeated once per initial dilation guess, the
    copies of p at rows p*M .. p*M + M - 1 (M = len(s_init)), copy j with s_init[j] in the
    s_init column of params; nothing else changes."""
    M = len(s_init)
    out = {k: np.repeat(np.asarray(v), M, axis=0) for k, v in inst.items()}
    out["params"] = out["params"].copy()
    out["params"][:, 21] = np.tile(np.asarray(s_init, dtype=np.float64), len(inst["K"]))
    return out
