"""Python binding of the batched 6-DoF SCP library (argument marshalling only).

Every step of the solve runs in the HIP library ``libscp_batch.so``; this module only
allocates device tensors with PyTorch, hands their pointers and the current stream to the
C ABI declared in ``include/scp_batch.h``, and wraps the results.  There is no CPU
fallback: if the library or a GPU is missing, the calls raise.
"""
import ctypes
import os

import numpy as np

NX, NU, NP, NXF = 15, 4, 24, 13
NU_MAX = 7  # controls with the reaction-control torque: (T, gamma, s)
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscp_batch.so")

SCP_F32, SCP_F64 = 0, 1
STATUS = {0: "SCP_OK", 1: "SCP_ERR_ARG", 2: "SCP_ERR_SHAPE", 3: "SCP_ERR_DTYPE",
          4: "SCP_ERR_DEVICE", 5: "SCP_ERR_HIP", 6: "SCP_ERR_WORKSPACE", 7: "SCP_ERR_STATE",
          8: "SCP_ERR_UNSUPPORTED"}

# Symbols the header declares (checked by the test-suite without a GPU).
EXPORTS = ["scp_batch_workspace_bytes", "scp_batch_create", "scp_batch_solve",
           "scp_batch_set_stream", "scp_batch_last_error", "scp_batch_create_error",
           "scp_batch_profile", "scp_batch_profile_read", "scp_batch_autotune",
           "scp_batch_mode", "scp_batch_solve_record", "scp_batch_grad",
           "scp_batch_select_best", "scp_batch_destroy", "scp_batch_solve_noalloc"]
KERNEL_CLASSES = ("init", "discretize", "subproblem", "prepare")  # SCP_KERNEL_CLASSES order


class ScpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


# launch variants timed by scp_batch_autotune: (dispatch mode, occupancy)
TUNE_VARIANTS = ((1, 0), (2, 0), (3, 0), (1, 5), (2, 5), (1, 6), (2, 6), (4, 0), (4, 5), (4, 6))


class Settings(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32), ("k_max", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("scp_iters_max", ctypes.c_int32), ("pipg_iters_max", ctypes.c_int32),
        ("pipg_check_every", ctypes.c_int32), ("rk4_substeps", ctypes.c_int32),
        ("power_iters_max", ctypes.c_int32), ("early_exit", ctypes.c_int32),
        ("node_projections", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("grad_pipg_steps", ctypes.c_int32), ("grad_ckpt_every", ctypes.c_int32),
        ("occupancy", ctypes.c_int32), ("grad_rk4_tangent", ctypes.c_int32),
        ("scalar_dilation", ctypes.c_int32), ("n_u", ctypes.c_int32),
        ("power_fp32", ctypes.c_int32),
        ("scp_tol", ctypes.c_double), ("feas_tol", ctypes.c_double),
        ("pipg_eps_abs", ctypes.c_double), ("pipg_eps_rel", ctypes.c_double),
        ("power_eps_abs", ctypes.c_double), ("power_eps_rel", ctypes.c_double),
        ("power_buff", ctypes.c_double), ("w_cost", ctypes.c_double),
        ("w_prox", ctypes.c_double), ("w_ep", ctypes.c_double), ("omega", ctypes.c_double),
        ("rho", ctypes.c_double), ("px", ctypes.c_double * NX), ("pu", ctypes.c_double * NU_MAX),
    ]


class Problem(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("x0", ctypes.c_void_p), ("xf", ctypes.c_void_p),
                ("params", ctypes.c_void_p), ("K", ctypes.c_void_p), ("x_init", ctypes.c_void_p),
                ("u_init", ctypes.c_void_p)]


def _problem_struct(prob):
    """scp_problem of a dict of device tensors (x_init / u_init optional)."""
    opt = lambda k: prob[k].data_ptr() if prob.get(k) is not None else None
    return Problem(int(prob["x0"].shape[0]), prob["x0"].data_ptr(), prob["xf"].data_ptr(),
                   prob["params"].data_ptr(), prob["K"].data_ptr(), opt("x_init"),
                   opt("u_init"))


class Solution(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "u", "t_f", "m_f", "status", "scp_iters",
                                               "pipg_iters", "defect_inf", "ctcs_viol",
                                               "objective")]


LASTITER_FIELDS = ("xbar", "ubar", "mup", "mum", "phi", "th", "sigma")


class LastIter(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in LASTITER_FIELDS]


_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libscp_batch.so is not built; run __graft_entry__.build() or "
                               "python paper_2404_18034_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        L.scp_batch_workspace_bytes.argtypes = [ctypes.POINTER(Settings)]
        L.scp_batch_workspace_bytes.restype = ctypes.c_size_t
        L.scp_batch_create.argtypes = [ctypes.POINTER(Settings), ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.scp_batch_create.restype = ctypes.c_int
        L.scp_batch_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                      ctypes.POINTER(Solution)]
        L.scp_batch_solve.restype = ctypes.c_int
        L.scp_batch_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.scp_batch_set_stream.restype = ctypes.c_int
        L.scp_batch_last_error.argtypes = [ctypes.c_void_p]
        L.scp_batch_last_error.restype = ctypes.c_char_p
        L.scp_batch_create_error.argtypes = []
        L.scp_batch_create_error.restype = ctypes.c_char_p
        L.scp_batch_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.scp_batch_profile.restype = ctypes.c_int
        L.scp_batch_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int32)]
        L.scp_batch_profile_read.restype = ctypes.c_int
        L.scp_batch_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                         ctypes.POINTER(Solution), ctypes.c_char_p,
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double)]
        L.scp_batch_autotune.restype = ctypes.c_int
        L.scp_batch_mode.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
        L.scp_batch_mode.restype = ctypes.c_int
        L.scp_batch_solve_record.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                             ctypes.POINTER(Solution), ctypes.POINTER(LastIter)]
        L.scp_batch_solve_record.restype = ctypes.c_int
        L.scp_batch_grad.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem),
                                     ctypes.POINTER(LastIter), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.scp_batch_grad.restype = ctypes.c_int
        L.scp_batch_select_best.argtypes = [ctypes.c_void_p, ctypes.POINTER(Solution),
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(Solution)]
        L.scp_batch_select_best.restype = ctypes.c_int
        L.scp_batch_destroy.argtypes = [ctypes.c_void_p]
        L.scp_batch_destroy.restype = ctypes.c_int
        L.scp_batch_solve_noalloc.argtypes = [ctypes.POINTER(Settings), ctypes.c_int,
                                              ctypes.c_void_p, ctypes.POINTER(Problem),
                                              ctypes.POINTER(Solution)]
        L.scp_batch_solve_noalloc.restype = ctypes.c_int
        _lib = L
    return _lib


def make_settings(cfg, dtype="f32", k_max=None, max_batch=0):
    """C settings struct from a dict of solver settings (see instances.solver_settings)."""
    s = Settings()
    s.dtype = SCP_F64 if dtype in ("f64", "float64", SCP_F64) else SCP_F32
    s.k_max = int(k_max)
    s.max_batch = int(max_batch)
    for name in ("scp_iters_max", "pipg_iters_max", "pipg_check_every", "rk4_substeps",
                 "power_iters_max", "early_exit", "node_projections"):
        setattr(s, name, int(cfg[name]))
    s.mode = int(cfg.get("mode", 0))
    s.occupancy = int(cfg.get("occupancy", 0))
    # the tangent form of the RK4 share is the cheaper one for the two parameters that reach
    # the discretization (the reverse sweep stays available and is checked against it)
    s.grad_rk4_tangent = int(cfg.get("grad_rk4_tangent", 1))
    s.scalar_dilation = int(cfg.get("scalar_dilation", 0))
    s.power_fp32 = int(cfg.get("power_fp32", 0))
    s.n_u = int(cfg.get("n_u", NU))
    s.grad_pipg_steps = int(cfg.get("grad_pipg_steps", 0))
    s.grad_ckpt_every = int(cfg.get("grad_ckpt_every", 0))
    for name in ("scp_tol", "feas_tol", "pipg_eps_abs", "pipg_eps_rel", "power_eps_abs",
                 "power_eps_rel", "power_buff", "w_cost", "w_prox", "w_ep", "omega", "rho"):
        setattr(s, name, float(cfg[name]))
    for i, v in enumerate(cfg["px"]):
        s.px[i] = float(v)
    for i, v in enumerate(cfg["pu"]):
        s.pu[i] = float(v)
    return s


def workspace_bytes(settings):
    return int(load().scp_batch_workspace_bytes(ctypes.byref(settings)))


class BatchSolver:
    """A library handle with its caller-owned workspace (a torch uint8 device tensor)."""

    def __init__(self, cfg, dtype="f32", k_max=30, max_batch=1024, device=0, stream=None):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("BatchSolver needs a HIP GPU; none is visible")
        L = load()
        self.settings = make_settings(cfg, dtype, k_max, max_batch)
        self.dtype = torch.float64 if self.settings.dtype == SCP_F64 else torch.float32
        self.k_max, self.max_batch, self.device = int(k_max), int(max_batch), int(device)
        self.n_u = int(self.settings.n_u)
        nbytes = workspace_bytes(self.settings)
        if nbytes == 0:
            raise ScpError(1, "invalid settings")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8,
                                     device="cuda:%d" % self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.stream = stream
        h = ctypes.c_void_p()
        rc = L.scp_batch_create(ctypes.byref(self.settings), self.device,
                                ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(aligned),
                                ctypes.c_size_t(nbytes), ctypes.byref(h))
        if rc != 0:
            raise ScpError(rc, L.scp_batch_create_error().decode())
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().scp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise ScpError(rc, load().scp_batch_last_error(self.handle).decode())

    def alloc_solution(self, B):
        t = self.torch
        dev = "cuda:%d" % self.device
        return dict(
            x=t.empty((B, self.k_max, NX), dtype=self.dtype, device=dev),
            u=t.empty((B, self.k_max, self.n_u), dtype=self.dtype, device=dev),
            t_f=t.empty(B, dtype=self.dtype, device=dev),
            m_f=t.empty(B, dtype=self.dtype, device=dev),
            status=t.empty(B, dtype=t.int32, device=dev),
            scp_iters=t.empty(B, dtype=t.int32, device=dev),
            pipg_iters=t.empty(B, dtype=t.int32, device=dev),
            defect_inf=t.empty(B, dtype=t.float64, device=dev),
            ctcs_viol=t.empty(B, dtype=t.float64, device=dev),
            objective=t.empty(B, dtype=t.float64, device=dev))

    def to_device(self, inst):
        """Problem dict of numpy arrays -> device tensors of the handle's dtype (x_init and
        u_init, the optional first reference [B, k_max, 15] and [B, k_max, n_u], when
        present)."""
        t = self.torch
        dev = "cuda:%d" % self.device
        real = lambda a: t.as_tensor(np.ascontiguousarray(a), dtype=self.dtype).to(dev)
        out = dict(x0=real(inst["x0"]), xf=real(inst["xf"]), params=real(inst["params"]),
                   K=t.as_tensor(np.ascontiguousarray(inst["K"]), dtype=t.int32).to(dev))
        for k in ("x_init", "u_init"):
            if inst.get(k) is not None:
                out[k] = real(inst[k])
        return out

    def _structs(self, prob, sol):
        p = _problem_struct(prob)
        if sol is None:
            return p, None
        s = Solution(*[sol[n].data_ptr() for n in ("x", "u", "t_f", "m_f", "status",
                                                    "scp_iters", "pipg_iters", "defect_inf",
                                                    "ctcs_viol", "objective")])
        return p, s

    def autotune(self, prob, sol, cache_path=None):
        """Time the launch variants on this batch and keep the fastest (see
        scp_batch_autotune); returns ((mode, occupancy), {(mode, occupancy): ms})."""
        p, s = self._structs(prob, sol)
        var = ctypes.c_int32(-1)
        ms = (ctypes.c_double * len(TUNE_VARIANTS))()
        path = None if cache_path is None else str(cache_path).encode()
        self._check(load().scp_batch_autotune(self.handle, ctypes.byref(p), ctypes.byref(s),
                                              path, ctypes.byref(var), ms))
        return TUNE_VARIANTS[var.value], {TUNE_VARIANTS[v]: ms[v]
                                          for v in range(len(TUNE_VARIANTS)) if ms[v] >= 0}

    def mode(self):
        """(dispatch mode, occupancy variant) in use."""
        m, o = ctypes.c_int32(-1), ctypes.c_int32(-1)
        self._check(load().scp_batch_mode(self.handle, ctypes.byref(m), ctypes.byref(o)))
        return m.value, o.value

    def _on_device(self, name, v):
        if v.device.type != "cuda" or v.device.index != self.device:
            raise ScpError(2, "%s must be on cuda:%d" % (name, self.device))

    def _check_problem(self, prob):
        B = int(prob["x0"].shape[0])
        for k in ("x0", "xf", "params", "K", "x_init", "u_init"):
            if prob.get(k) is not None:
                self._on_device(k, prob[k])
        for k, shape in (("x0", (B, NX)), ("xf", (B, NXF)), ("params", (B, NP))):
            v = prob[k]
            if tuple(v.shape) != shape or v.dtype != self.dtype or not v.is_contiguous():
                raise ScpError(2, "%s must be a contiguous %s tensor of shape %s" %
                               (k, self.dtype, shape))
        if tuple(prob["K"].shape) != (B,) or prob["K"].dtype != self.torch.int32:
            raise ScpError(2, "K must be an int32 tensor of shape (B,)")
        for k, shape in (("x_init", (B, self.k_max, NX)), ("u_init", (B, self.k_max, self.n_u))):
            v = prob.get(k)
            if v is not None and (tuple(v.shape) != shape or v.dtype != self.dtype or
                                  not v.is_contiguous()):
                raise ScpError(2, "%s must be a contiguous %s tensor of shape %s" %
                               (k, self.dtype, shape))
        return B

    def _check_real(self, name, v, shape, dtype=None):
        dtype = self.dtype if dtype is None else dtype
        if tuple(v.shape) != tuple(shape) or v.dtype != dtype or not v.is_contiguous():
            raise ScpError(2, "%s must be a contiguous %s tensor of shape %s" % (name, dtype, shape))

    def _check_solution(self, sol, B):
        t = self.torch
        for k, tail, dtype in (("x", (self.k_max, NX), self.dtype),
                               ("u", (self.k_max, self.n_u), self.dtype),
                               ("t_f", (), self.dtype), ("m_f", (), self.dtype),
                               ("status", (), t.int32), ("scp_iters", (), t.int32),
                               ("pipg_iters", (), t.int32), ("defect_inf", (), t.float64),
                               ("ctcs_viol", (), t.float64), ("objective", (), t.float64)):
            v = sol[k]
            self._on_device(k, v)
            if (v.dim() != 1 + len(tail) or v.shape[0] < B or tuple(v.shape[1:]) != tail
                    or v.dtype != dtype or not v.is_contiguous()):
                raise ScpError(2, "solution array %s must be a contiguous %s tensor of shape "
                                  "(>= %d,) + %s" % (k, dtype, B, tail))

    def solve_into(self, prob, sol):
        """Enqueue a solve of device problem tensors into preallocated solution tensors."""
        self._check_solution(sol, self._check_problem(prob))
        p, s = self._structs(prob, sol)
        self._check(load().scp_batch_solve(self.handle, ctypes.byref(p), ctypes.byref(s)))
        return sol

    def alloc_lastiter(self, B):
        """Device buffers for the starting point of each instance's last subproblem."""
        t = self.torch
        dev = "cuda:%d" % self.device
        km, M = self.k_max, self.k_max - 1
        return dict(xbar=t.zeros((B, km, NX), dtype=self.dtype, device=dev),
                    ubar=t.zeros((B, km, NU), dtype=self.dtype, device=dev),
                    mup=t.zeros((B, M, NX), dtype=self.dtype, device=dev),
                    mum=t.zeros((B, M, NX), dtype=self.dtype, device=dev),
                    phi=t.zeros((B, M, NX), dtype=self.dtype, device=dev),
                    th=t.zeros((B, M), dtype=self.dtype, device=dev),
                    sigma=t.zeros(B, dtype=t.float64, device=dev))

    def _lastiter_struct(self, last, B):
        km, M = self.k_max, self.k_max - 1
        shapes = dict(xbar=(B, km, NX), ubar=(B, km, NU), mup=(B, M, NX), mum=(B, M, NX),
                      phi=(B, M, NX), th=(B, M), sigma=(B,))
        for k, shp in shapes.items():
            self._check_real(k, last[k], shp, self.torch.float64 if k == "sigma" else None)
        return LastIter(*[last[n].data_ptr() for n in LASTITER_FIELDS])

    def solve_record_into(self, prob, sol, last):
        """Solve, and record into `last` the starting point of each instance's last
        subproblem (scp_batch_solve_record)."""
        B = self._check_problem(prob)
        p, s = self._structs(prob, sol)
        r = self._lastiter_struct(last, B)
        self._check(load().scp_batch_solve_record(self.handle, ctypes.byref(p), ctypes.byref(s),
                                                  ctypes.byref(r)))
        return sol, last

    def grad_into(self, prob, last, cot, grad, value=None):
        """Vector-Jacobian product of the last SCP iteration (scp_batch_grad):
        grad[B, 18] = cot[:, 0] dm_f/dtheta + cot[:, 1] dt_f/dtheta, theta = (x0, m_wet,
        alpha_mdot, T_max); value[B, 2] (optional) receives (m_f, t_f) of that map."""
        B = self._check_problem(prob)
        p, _ = self._structs(prob, None)
        r = self._lastiter_struct(last, B)
        self._check_real("cot", cot, (B, 2))
        self._check_real("grad", grad, (B, 18))
        if value is not None:
            self._check_real("value", value, (B, 2))
        self._check(load().scp_batch_grad(self.handle, ctypes.byref(p), ctypes.byref(r),
                                          ctypes.c_void_p(cot.data_ptr()),
                                          ctypes.c_void_p(grad.data_ptr()),
                                          None if value is None else
                                          ctypes.c_void_p(value.data_ptr())))
        return grad

    def profile(self, enable=True):
        """Turn per-launch HIP-event timing on or off (see scp_batch_profile)."""
        self._check(load().scp_batch_profile(self.handle, int(bool(enable))))

    def profile_read(self):
        """{kernel class: (summed ms, launches)} of the last solve."""
        ms = (ctypes.c_double * len(KERNEL_CLASSES))()
        n = (ctypes.c_int32 * len(KERNEL_CLASSES))()
        self._check(load().scp_batch_profile_read(self.handle, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def solve(self, prob):
        B = int(prob["x0"].shape[0])
        sol = self.alloc_solution(B)
        return self.solve_into(prob, sol)

    def select_best_into(self, sol, problems, starts, best, out):
        """Enqueue the multi-start selection (scp_batch_select_best): `sol` holds
        problems * starts solved instances, the starts of problem p consecutive; best
        (int32 [problems]) and `out` (a solution of `problems` instances) are written."""
        problems, starts = int(problems), int(starts)
        n = problems * starts
        for k, v in sol.items():
            if v.shape[0] < n:
                raise ScpError(2, "solution array %s holds fewer than problems * starts rows" % k)
        for k, v in out.items():
            if v.shape[0] < problems:
                raise ScpError(2, "out array %s holds fewer than `problems` rows" % k)
        if best.dtype != self.torch.int32 or best.shape[0] < problems or not best.is_contiguous():
            raise ScpError(2, "best must be a contiguous int32 tensor of at least `problems` rows")
        names = ("x", "u", "t_f", "m_f", "status", "scp_iters", "pipg_iters", "defect_inf",
                 "ctcs_viol", "objective")
        s = Solution(*[sol[k].data_ptr() for k in names])
        o = Solution(*[out[k].data_ptr() for k in names])
        self._check(load().scp_batch_select_best(self.handle, ctypes.byref(s), problems, starts,
                                                 best.data_ptr(), ctypes.byref(o)))
        return best, out

    def select_best(self, sol, problems, starts):
        best = self.torch.empty(int(problems), dtype=self.torch.int32,
                                device="cuda:%d" % self.device)
        return self.select_best_into(sol, problems, starts, best, self.alloc_solution(problems))


def solve_noalloc_into(cfg, dtype, k_max, max_batch, prob, sol, device=0, stream=None):
    """scp_batch_solve_noalloc: solve `prob` into `sol` (dicts of device tensors, as
    BatchSolver.to_device / alloc_solution make them) with the library's fixed scratch as the
    workspace; no handle, nothing allocated.  Asynchronous on `stream` (default: the current
    stream of `device`)."""
    import torch
    L = load()
    s = make_settings(cfg, dtype, k_max, max_batch)
    B = int(prob["x0"].shape[0])
    p = _problem_struct(prob)
    so = Solution(*[sol[n].data_ptr() for n in ("x", "u", "t_f", "m_f", "status", "scp_iters",
                                                 "pipg_iters", "defect_inf", "ctcs_viol",
                                                 "objective")])
    stream = torch.cuda.current_stream(device) if stream is None else stream
    rc = L.scp_batch_solve_noalloc(ctypes.byref(s), int(device),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(p),
                                   ctypes.byref(so))
    if rc != 0:
        raise ScpError(rc, L.scp_batch_create_error().decode())


def solve(cfg, inst, dtype="f32", k_max=None, device=0):
    """One-shot convenience: numpy problem dict in, dict of numpy arrays out."""
    import torch
    K = np.asarray(inst["K"])
    k_max = int(K.max()) if k_max is None else int(k_max)
    B = int(K.shape[0])
    s = BatchSolver(cfg, dtype=dtype, k_max=k_max, max_batch=max(B, 1), device=device)
    try:
        sol = s.solve(s.to_device(inst))
        torch.cuda.synchronize(device)
        return {k: v.cpu().numpy() for k, v in sol.items()}
    finally:
        s.close()


def solve_multistart(cfg, inst, s_init, dtype="f32", k_max=None, device=0):
    """Multi-start one-shot: every problem of `inst` is solved once per initial dilation guess
    in `s_init` (all starts in one batch, see instances.multistart) and the converged start of
    lowest cost is kept.  Returns (numpy solution dict of the problems, best start per problem
    or -1, numpy solution dict of every start)."""
    import torch
    from . import instances
    starts = len(s_init)
    rep = instances.multistart(inst, s_init)
    K = np.asarray(rep["K"])
    k_max = int(K.max()) if k_max is None else int(k_max)
    P = int(np.asarray(inst["K"]).shape[0])
    s = BatchSolver(cfg, dtype=dtype, k_max=k_max, max_batch=max(P * starts, 1), device=device)
    try:
        sol = s.solve(s.to_device(rep))
        best, out = s.select_best(sol, P, starts)
        torch.cuda.synchronize(device)
        return ({k: v.cpu().numpy() for k, v in out.items()}, best.cpu().numpy(),
                {k: v.cpu().numpy() for k, v in sol.items()})
    finally:
        s.close()


_SOLVE_FN = None


def _solve_fn():
    global _SOLVE_FN
    if _SOLVE_FN is None:
        import torch

        class ScpSolve(torch.autograd.Function):
            """Forward: the batched solve, recording each instance's last subproblem; returns
            (m_f, t_f).  Backward: the vector-Jacobian product of the last SCP iteration
            (scp_batch_grad: the discretization, the subproblem and grad_pipg_steps PIPG steps
            at the recorded starting point) with respect to x0 and to the params columns
            alpha_mdot (2) and T_max (13).  The solve takes the initial mass from x0[0], so
            params column 0 (m_wet) and the other columns receive no gradient."""

            @staticmethod
            def forward(ctx, x0, params, solver, xf, K):
                prob = dict(x0=x0.detach().contiguous(), xf=xf.detach().contiguous(),
                            params=params.detach().contiguous(), K=K)
                B = int(x0.shape[0])
                sol = solver.alloc_solution(B)
                last = solver.alloc_lastiter(B)
                solver.solve_record_into(prob, sol, last)
                ctx.solver, ctx.prob, ctx.last = solver, prob, last
                return sol["m_f"].clone(), sol["t_f"].clone()

            @staticmethod
            def backward(ctx, g_m, g_t):
                solver, prob = ctx.solver, ctx.prob
                B = int(prob["x0"].shape[0])
                dev = prob["x0"].device
                z = torch.zeros(B, dtype=solver.dtype, device=dev)
                cot = torch.stack([z if g_m is None else g_m.to(solver.dtype),
                                   z if g_t is None else g_t.to(solver.dtype)], dim=1).contiguous()
                g = torch.empty((B, 18), dtype=solver.dtype, device=dev)
                solver.grad_into(prob, ctx.last, cot, g)
                g_x0 = g[:, :NX].clone()
                g_p = torch.zeros_like(prob["params"])
                g_p[:, 2] = g[:, 16]
                g_p[:, 13] = g[:, 17]
                return g_x0, g_p, None, None, None

        _SOLVE_FN = ScpSolve
    return _SOLVE_FN


def solve_differentiable(solver, x0, params, xf, K):
    """(m_f, t_f) of the batched solve as torch functions of x0 [B, 15] and params [B, 23]
    (device tensors of the solver's dtype); gradients flow through the last SCP iteration.
    The solver must have been created with grad_pipg_steps > 0."""
    return _solve_fn().apply(x0, params, solver, xf, K)
