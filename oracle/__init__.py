"""FP64 CPU oracle for batched prox-linear SCP + CTCS + customized PIPG (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference implementation that the
GPU library is checked against.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does, and the oracle never
imports the GPU library.  The C source (``scp_oracle.c``) is compiled with gcc, without
fast-math and without FMA contraction, into ``_scp_oracle.so`` next to it.

Layouts (row-major float64 numpy arrays):
  x0[B,15], xf[B,13], params[B,24], K[B] (int32); trajectories x[B,kmax,15], u[B,kmax,n_u].
The controls are u = (T, s) (n_u = 4) or, for a settings dict with n_u = 7, u = (T, gamma, s)
with the reaction-control torque gamma: the same C source built with -DNU=7
(``_scp_oracle_nu7.so``).

``solve_f32`` runs the same C source compiled with float in place of double
(``_scp_oracle_f32.so``): a single-precision evaluation of the same algorithm; with
``contract=True`` the same source built with fused multiply-adds allowed
(``_scp_oracle_f32fma.so``), another equally valid single-precision rounding pattern.  Tests
use them only to measure how far FP32 rounding alone moves an instance's result (its FP32
conditioning); they are never an expected value.
"""
import ctypes
import os
import subprocess

import numpy as np

NX, NU, NP, NXF = 15, 4, 24, 13
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scp_oracle.c")
_SO = os.path.join(_HERE, "_scp_oracle.so")
_SO32 = os.path.join(_HERE, "_scp_oracle_f32.so")
_SO32F = os.path.join(_HERE, "_scp_oracle_f32fma.so")
_SO7 = os.path.join(_HERE, "_scp_oracle_nu7.so")

CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-D_POSIX_C_SOURCE=200809L", "-pthread"]


def build(force=False):
    """Compile the oracle with gcc (idempotent unless ``force``), and its single-precision
    twin (every ``double`` of the source read as ``float``)."""
    import re
    import tempfile
    if (not force and all(os.path.exists(p) and os.path.getmtime(p) >= os.path.getmtime(_SRC)
                          for p in (_SO, _SO32, _SO32F, _SO7))):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    tmp = _SO7 + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-DNU=7", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO7)
    with tempfile.TemporaryDirectory() as d:
        src32 = os.path.join(d, "scp_oracle_f32.c")
        with open(_SRC) as f:
            text = f.read()
        with open(src32, "w") as f:
            f.write(re.sub(r"\bdouble\b", "float", text))
        tmp = _SO32 + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src32, "-lm"])
        os.replace(tmp, _SO32)
        flags = [f for f in CFLAGS if f != "-ffp-contract=off"] + ["-ffp-contract=fast", "-mfma"]
        tmp = _SO32F + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *flags, "-o", tmp, src32, "-lm"])
        os.replace(tmp, _SO32F)
    return _SO


class Settings(ctypes.Structure):
    _fields_ = [
        ("scp_iters_max", ctypes.c_int32), ("pipg_iters_max", ctypes.c_int32),
        ("pipg_check_every", ctypes.c_int32), ("rk4_substeps", ctypes.c_int32),
        ("power_iters_max", ctypes.c_int32), ("early_exit", ctypes.c_int32),
        ("node_projections", ctypes.c_int32), ("scalar_dilation", ctypes.c_int32),
        ("scp_tol", ctypes.c_double), ("feas_tol", ctypes.c_double),
        ("pipg_eps_abs", ctypes.c_double), ("pipg_eps_rel", ctypes.c_double),
        ("power_eps_abs", ctypes.c_double), ("power_eps_rel", ctypes.c_double),
        ("power_buff", ctypes.c_double),
        ("w_cost", ctypes.c_double), ("w_prox", ctypes.c_double), ("w_ep", ctypes.c_double),
        ("omega", ctypes.c_double), ("rho", ctypes.c_double),
        ("px", ctypes.c_double * NX), ("pu", ctypes.c_double * NU),
    ]


class Settings7(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double * 7 if n == "pu" else t) for n, t in Settings._fields_]


class Settings32(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float if t is ctypes.c_double else
                 (ctypes.c_float * NX if n == "px" else ctypes.c_float * NU if n == "pu" else t))
                for n, t in Settings._fields_]


def n_u(cfg):
    """Number of controls of a settings dict: 4 (thrust, dilation) or 7 (with the torque)."""
    return int(cfg.get("n_u", NU))


def make_settings(cfg, cls=None):
    """Build the oracle's settings struct from a plain dict of solver settings."""
    if cls is None:
        cls = Settings7 if n_u(cfg) == 7 else Settings
    s = cls()
    for name, _ in Settings._fields_:
        if name in ("px", "pu"):
            continue
        setattr(s, name, cfg.get(name, 0) if name == "scalar_dilation" else cfg[name])
    for i, v in enumerate(cfg["px"]):
        s.px[i] = float(v)
    for i, v in enumerate(cfg["pu"]):
        s.pu[i] = float(v)
    return s


_lib = None
_lib7 = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def lib(nu=NU):
    """The oracle library for n_u controls (4, or 7 with the reaction-control torque)."""
    global _lib, _lib7
    if nu == 7:
        if _lib7 is None:
            build()
            _lib7 = _bind(ctypes.CDLL(_SO7), Settings7)
        return _lib7
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_SO), Settings)
    return _lib


def _bind(L, settings_cls):
    if True:
        S = ctypes.POINTER(settings_cls)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        sig = {
            "orc_dynamics": [_D, _D, _D, _D],
            "orc_jacobians": [_D, _D, _D, _D, _D],
            "orc_constraints": [_D, _D, _D, _D],
            "orc_discretize_interval": [_D, _D, _D, _D, _D, _D, c_double, c_int, _D, _D, _D, _D],
            "orc_discretize": [c_int, _D, _D, _D, c_int, _D, _D, _D, _D],
            "orc_init_guess": [c_int, _D, _D, _D, _D, _D],
            "orc_build_qp": [S, _D, c_int, _D, _D, _D, _D, _D, _D, _D, _D,
                             _D, _D, _D, _D, _D, _D, _D, _D, _D],
            "orc_power": [S, c_int, _D, _D, _D, _I],
            "orc_pipg": [S, c_int, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, c_double,
                         c_int, c_int, _D, _D, _D, _D, _D, _D],
            "orc_solve_batch": [S, c_int, c_int, _D, _D, _D, _I, c_int, _D, _D, _D, _D, _I, _I,
                                _I, _D, _D, _D, _D, _D, _D],
            "orc_solve_trace": [S, c_int, _D, _D, _D, _D, _D, _D, _I, c_int, _D],
            "orc_lastiter_state": [S, c_int, _D, _D, _D, _D, _D, _D, _D],
            "orc_iter_len": [c_int],
            "orc_truncated_map": [S, c_int, _D, _D, _D, _D, _D, _D, _D, c_double, c_int, _D],
            "orc_stopping": [c_int] + [_D] * 12 + [c_double, c_double],
            "orc_project_node": [_D, _D, _D],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
        L.orc_power.restype = c_double
        L.orc_pipg.restype = c_int
        L.orc_solve_batch.restype = c_int
        L.orc_iter_len.restype = c_int
        L.orc_lastiter_state.restype = c_int
        L.orc_stopping.restype = c_int
    return L


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else ctypes.cast(None, _D)


# ----------------------------------------------------------------------------- model ----
def dynamics(x, u, p):
    """f(x, u) of the lander; u has 4 or 7 entries (the latter with the torque)."""
    x, xp = _d(x); u, up = _d(u); p, pp = _d(p)
    f = np.zeros(NX)
    lib(u.size).orc_dynamics(xp, up, pp, _p(f))
    return f


def jacobians(x, u, p):
    x, xp = _d(x); u, up = _d(u); p, pp = _d(p)
    A = np.zeros((NX, NX)); B = np.zeros((NX, u.size))
    lib(u.size).orc_jacobians(xp, up, pp, _p(A), _p(B))
    return A, B


def constraints(x, u, p):
    x, xp = _d(x); u, up = _d(u); p, pp = _d(p)
    g = np.zeros(9)
    lib(u.size).orc_constraints(xp, up, pp, _p(g))
    return g


# ---------------------------------------------------------------------- discretization ----
def discretize_interval(xk, uk, uk1, p, dtau, nsub, A0=None, B0=None):
    """One interval; with A0/B0 given, the linear test model f = A0 x + B0 u is used."""
    xk, a = _d(xk); uk, b = _d(uk); uk1, c = _d(uk1)
    p = np.zeros(NP) if p is None else p
    p, pp = _d(p)
    nu = uk.size
    A0c = None if A0 is None else np.ascontiguousarray(A0, dtype=np.float64)
    B0c = None if B0 is None else np.ascontiguousarray(B0, dtype=np.float64)
    xe = np.zeros(NX); A = np.zeros((NX, NX)); Bm = np.zeros((NX, nu)); Bp = np.zeros((NX, nu))
    lib(nu).orc_discretize_interval(a, b, c, pp, _p(A0c), _p(B0c), float(dtau), int(nsub),
                                  _p(xe), _p(A), _p(Bm), _p(Bp))
    return xe, A, Bm, Bp


def discretize(K, xbar, ubar, p, nsub):
    xbar, xp = _d(xbar); ubar, up = _d(ubar); p, pp = _d(p)
    M = K - 1
    nu = ubar.shape[-1]
    xe = np.zeros((M, NX)); A = np.zeros((M, NX, NX))
    Bm = np.zeros((M, NX, nu)); Bp = np.zeros((M, NX, nu))
    lib(nu).orc_discretize(K, xp, up, pp, int(nsub), _p(xe), _p(A), _p(Bm), _p(Bp))
    return xe, A, Bm, Bp


def init_guess(K, x0, xf, p, nu=NU):
    x0, a = _d(x0); xf, b = _d(xf); p, c = _d(p)
    xb = np.zeros((K, NX)); ub = np.zeros((K, nu))
    lib(nu).orc_init_guess(K, a, b, c, _p(xb), _p(ub))
    return xb, ub


# ------------------------------------------------------------------------------ QP -------
def build_qp(cfg, p, K, x0, xf, xbar, ubar, xend, A, Bm, Bp):
    st = make_settings(cfg)
    args = [_d(v) for v in (p, x0, xf, xbar, ubar, xend, A, Bm, Bp)]
    M = K - 1
    nu = n_u(cfg)
    out = dict(Am=np.zeros((M, NX, NX)), Bm=np.zeros((M, NX, nu)), Bp=np.zeros((M, NX, nu)),
               w=np.zeros((M, NX)), eps=np.zeros(M), umin=np.zeros((K, nu)),
               umax=np.zeros((K, nu)), zi=np.zeros(NX), zf=np.zeros(NXF))
    a = [x[1] for x in args]
    lib(nu).orc_build_qp(ctypes.byref(st), a[0], K, a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8],
                       *[_p(out[k]) for k in ("Am", "Bm", "Bp", "w", "eps", "umin", "umax",
                                              "zi", "zf")])
    return out


def power(cfg, qp):
    st = make_settings(cfg)
    K = qp["umin"].shape[0] if "umin" in qp else qp["Am"].shape[0] + 1
    Am, a = _d(qp["Am"]); Bm, b = _d(qp["Bm"]); Bp, c = _d(qp["Bp"])
    it = ctypes.c_int32(0)
    sigma = lib(n_u(cfg)).orc_power(ctypes.byref(st), K, a, b, c, ctypes.byref(it))
    return sigma, it.value


def zero_warm_start(K, nu=NU):
    M = K - 1
    return dict(x=np.zeros((K, NX)), u=np.zeros((K, nu)), mup=np.zeros((M, NX)),
                mum=np.zeros((M, NX)), phi=np.zeros((M, NX)), th=np.zeros(M))


def pipg(cfg, qp, sigma, jmax, check, ws=None, ref=None):
    """Run PIPG_custom on scaled QP data; returns (solution dict, iterations).

    ``ref`` = (xbar, ubar, params) is needed only when node projections are enabled."""
    st = make_settings(cfg)
    K = qp["umin"].shape[0]
    ws = zero_warm_start(K, n_u(cfg)) if ws is None else ws
    out = {k: np.array(v, dtype=np.float64, copy=True) for k, v in ws.items()}
    q = {k: np.ascontiguousarray(qp[k], dtype=np.float64)
         for k in ("Am", "Bm", "Bp", "w", "eps", "umin", "umax", "zi", "zf")}
    refs = [None, None, None] if ref is None else [np.ascontiguousarray(r, dtype=np.float64)
                                                   for r in ref]
    n = lib(n_u(cfg)).orc_pipg(ctypes.byref(st), K, *[_p(q[k]) for k in ("Am", "Bm", "Bp", "w", "eps",
                                                                 "umin", "umax", "zi", "zf")],
                       *[_p(r) for r in refs], float(sigma), int(jmax), int(check),
                       *[_p(out[k]) for k in ("x", "u", "mup", "mum", "phi", "th")])
    if n < 0:
        raise ValueError("oracle: node projections need the reference and parameters")
    return out, n


# ----------------------------------------------------------------------------- SCP -------
def solve(cfg, x0, xf, params, K, kmax=None, nthreads=None, x_init=None, u_init=None):
    """Solve a batch; returns a dict of numpy arrays (same names as the GPU library).
    x_init [B][kmax][15] and u_init [B][kmax][n_u] (each optional) replace the initial guess
    on the first K_b nodes of instance b."""
    st = make_settings(cfg)
    x0, a = _d(x0); xf, b = _d(xf); params, c = _d(params)
    K = np.ascontiguousarray(K, dtype=np.int32)
    B = x0.shape[0]
    nu = n_u(cfg)
    kmax = int(K.max()) if kmax is None else int(kmax)
    xi = ui = None
    if x_init is not None:
        xi = np.ascontiguousarray(x_init, dtype=np.float64)
        if xi.shape != (B, kmax, NX):
            raise ValueError("oracle: x_init must have shape (B, kmax, 15)")
    if u_init is not None:
        ui = np.ascontiguousarray(u_init, dtype=np.float64)
        if ui.shape != (B, kmax, nu):
            raise ValueError("oracle: u_init must have shape (B, kmax, n_u)")
    nthreads = os.cpu_count() if nthreads is None else int(nthreads)
    out = dict(x=np.zeros((B, kmax, NX)), u=np.zeros((B, kmax, nu)), t_f=np.zeros(B),
               m_f=np.zeros(B), status=np.zeros(B, np.int32), scp_iters=np.zeros(B, np.int32),
               pipg_iters=np.zeros(B, np.int32), defect_inf=np.zeros(B), ctcs_viol=np.zeros(B),
               objective=np.zeros(B), step=np.zeros(B))
    rc = lib(nu).orc_solve_batch(
        ctypes.byref(st), B, kmax, a, b, c, K.ctypes.data_as(_I), nthreads,
        _p(out["x"]), _p(out["u"]), _p(out["t_f"]), _p(out["m_f"]),
        out["status"].ctypes.data_as(_I), out["scp_iters"].ctypes.data_as(_I),
        out["pipg_iters"].ctypes.data_as(_I), _p(out["defect_inf"]), _p(out["ctcs_viol"]),
        _p(out["objective"]), _p(out["step"]), None if xi is None else _p(xi),
        None if ui is None else _p(ui))
    if rc != 0:
        raise ValueError("oracle: invalid node count")
    return out


_lib32 = {}


def solve_f32(cfg, x0, xf, params, K, kmax=None, nthreads=None, contract=False):
    """The same solve evaluated in single precision (see the module note); float64 results.
    ``contract``: the build with fused multiply-adds."""
    if n_u(cfg) != NU:
        raise ValueError("the single-precision oracle builds have n_u = 4 only")
    if contract not in _lib32:
        build()
        _lib32[contract] = ctypes.CDLL(_SO32F if contract else _SO32)
    lib32 = _lib32[contract]
    st = make_settings(cfg, Settings32)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    x0, xf, params = f(x0), f(xf), f(params)
    K = np.ascontiguousarray(K, dtype=np.int32)
    B = x0.shape[0]
    kmax = int(K.max()) if kmax is None else int(kmax)
    nthreads = os.cpu_count() if nthreads is None else int(nthreads)
    out = dict(x=np.zeros((B, kmax, NX), np.float32), u=np.zeros((B, kmax, NU), np.float32),
               t_f=np.zeros(B, np.float32), m_f=np.zeros(B, np.float32),
               status=np.zeros(B, np.int32), scp_iters=np.zeros(B, np.int32),
               pipg_iters=np.zeros(B, np.int32), defect_inf=np.zeros(B, np.float32),
               ctcs_viol=np.zeros(B, np.float32), objective=np.zeros(B, np.float32),
               step=np.zeros(B, np.float32))
    v = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib32.orc_solve_batch(
        ctypes.byref(st), B, kmax, v(x0), v(xf), v(params), v(K), nthreads, v(out["x"]),
        v(out["u"]), v(out["t_f"]), v(out["m_f"]), v(out["status"]), v(out["scp_iters"]),
        v(out["pipg_iters"]), v(out["defect_inf"]), v(out["ctcs_viol"]), v(out["objective"]),
        v(out["step"]), None, None)
    if rc != 0:
        raise ValueError("oracle: invalid node count")
    return {k: (a.astype(np.float64) if a.dtype == np.float32 else a) for k, a in out.items()}


def select_best(status, objective, problems, starts):
    """Multi-start choice (the paper's Conclusion: several initial guesses per problem, the
    converged trajectory of lowest cost kept): for problem p, whose starts are rows
    p*starts .. p*starts + starts - 1, the start j with status 0 and the smallest objective,
    the first such j on ties, or -1 when no start converged.  Plain loops."""
    best = []
    for p in range(problems):
        pick, cost = -1, None
        for j in range(starts):
            r = p * starts + j
            if int(status[r]) == 0 and (pick < 0 or float(objective[r]) < cost):
                pick, cost = j, float(objective[r])
        best.append(pick)
    return np.array(best, dtype=np.int32)


def solve_trace(cfg, x0, xf, p, K, trace_n=64):
    st = make_settings(cfg)
    x0, a = _d(x0); xf, b = _d(xf); p, c = _d(p)
    xb = np.zeros((K, NX)); ub = np.zeros((K, n_u(cfg)))
    sc = np.zeros(6); ints = np.zeros(3, np.int32); tr = np.zeros((trace_n, 4))
    lib(n_u(cfg)).orc_solve_trace(ctypes.byref(st), int(K), a, b, c, _p(xb), _p(ub), _p(sc),
                          ints.ctypes.data_as(_I), int(trace_n), _p(tr))
    n = int(ints[1])
    return dict(x=xb, u=ub, t_f=sc[0], m_f=sc[1], defect_inf=sc[2], ctcs_viol=sc[3],
                objective=sc[4], step=sc[5], status=int(ints[0]), scp_iters=n,
                pipg_iters=int(ints[2]), trace=tr[:n])


def lastiter_state(cfg, x0, xf, p, K):
    """Reference, warm start and sigma of the last SCP iteration of a fixed-work solve."""
    st = make_settings(cfg)
    x0, a = _d(x0); xf, b = _d(xf); p, c = _d(p)
    nu = n_u(cfg)
    n = lib(nu).orc_iter_len(int(K))
    xb = np.zeros((K, NX)); ub = np.zeros((K, nu)); ws = np.zeros(n); sg = ctypes.c_double(0)
    rc = lib(nu).orc_lastiter_state(ctypes.byref(st), int(K), a, b, c, _p(xb), _p(ub), _p(ws),
                                  ctypes.byref(sg))
    if rc != 0:
        raise RuntimeError("oracle: no last iteration recorded")
    return dict(xbar=xb, ubar=ub, ws=ws, sigma=sg.value)


def truncated_map(cfg, x0, xf, p, K, theta, last, n_steps):
    """(m_f, t_f) of the last SCP iteration as a function of theta (18 values)."""
    st = make_settings(cfg)
    x0, a = _d(x0); xf, b = _d(xf); p, c = _d(p); th, t = _d(theta)
    out = np.zeros(2)
    xb, xbp = _d(last["xbar"]); ub, ubp = _d(last["ubar"]); ws, wsp = _d(last["ws"])
    lib(n_u(cfg)).orc_truncated_map(ctypes.byref(st), int(K), a, b, c, t, xbp, ubp, wsp,
                            float(last["sigma"]), int(n_steps), _p(out))
    return out


def theta_of(x0, p):
    """The 18 differentiated inputs: x0 (15), m_wet, alpha_mdot, T_max."""
    return np.concatenate([np.asarray(x0, np.float64), [p[0], p[2], p[13]]])


def stopping(new, old, eabs, erel):
    """The customized stopping test on two iterate dicts (keys x, u, mup, mum, phi, th)."""
    K = new["x"].shape[0]
    nu = new["u"].shape[-1]
    keys = ("x", "u", "mup", "mum", "phi", "th")
    a = [np.ascontiguousarray(new[k], dtype=np.float64) for k in keys]
    b = [np.ascontiguousarray(old[k], dtype=np.float64) for k in keys]
    return bool(lib(nu).orc_stopping(K, *[_p(v) for v in a], *[_p(v) for v in b], float(eabs),
                                   float(erel)))


def project_node(p, x, u):
    """Node-wise convex-set projection of a state (15) and control (4), original units."""
    p, pp = _d(p)
    x = np.array(x, dtype=np.float64, copy=True); u = np.array(u, dtype=np.float64, copy=True)
    lib(u.size).orc_project_node(pp, _p(x), _p(u))
    return x, u
