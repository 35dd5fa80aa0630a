"""Thin ctypes binding of libfdd.so (the C ABI in include/fdd.h).

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
PyTorch supplies device memory (the workspace and the vectors) and the HIP stream.
The binding raises if the shared library is missing; there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdd.so")

FDD_OK = 0
FDD_NOT_CONVERGED = 1
FDD_E_ARG = -1
FDD_E_NOMEM = -2
FDD_E_HIP = -3
FDD_E_RA = -4
FDD_E_BREAKDOWN = -5
FDD_E_NONFINITE = -6
FDD_E_WORKSPACE = -7
FDD_E_STATE = -8
FDD_FP64 = 0
FDD_MIXED = 1
FDD_RA_PRECOND = 0
FDD_RA_OPERATOR = 1

STATUS_NAMES = {
    FDD_OK: "FDD_OK", FDD_NOT_CONVERGED: "FDD_NOT_CONVERGED", FDD_E_ARG: "FDD_E_ARG",
    FDD_E_NOMEM: "FDD_E_NOMEM", FDD_E_HIP: "FDD_E_HIP", FDD_E_RA: "FDD_E_RA",
    FDD_E_BREAKDOWN: "FDD_E_BREAKDOWN", FDD_E_NONFINITE: "FDD_E_NONFINITE",
    FDD_E_WORKSPACE: "FDD_E_WORKSPACE", FDD_E_STATE: "FDD_E_STATE",
}

# every symbol declared in include/fdd.h
EXPORTED = [
    "fdd_opts_default", "fdd_setup_mesh", "fdd_setup_model", "fdd_setup_hdiv", "fdd_problem_info", "fdd_workspace_bytes",
    "fdd_bind_workspace", "fdd_build_rational_pc", "fdd_ratpc_from_table", "fdd_ratpc_query",
    "fdd_interior_solve", "fdd_schur_apply", "fdd_precond_apply", "fdd_precond_apply_static",
    "fdd_apply_operator", "fdd_dd_precond_apply", "fdd_solve_full",
    "fdd_solve", "fdd_set_kernel_timer", "fdd_get_kernel_timer", "fdd_destroy_problem",
    "fdd_destroy_ratpc", "fdd_last_error", "fdd_version", "fdd_batch_create",
    "fdd_batch_set_mid_tile", "fdd_batch_tile_edges", "fdd_batch_workspace_bytes", "fdd_batch_bind_workspace", "fdd_solve_batched",
    "fdd_batch_destroy", "fdd_batch_set_kernel_timer", "fdd_batch_get_kernel_timer",
    "fdd_cnn_create", "fdd_cnn_param_count", "fdd_cnn_workspace_bytes", "fdd_cnn_bind_workspace",
    "fdd_cnn_set_params", "fdd_cnn_forward", "fdd_cnn_loss", "fdd_cnn_backward",
    "fdd_cnn_adam_step", "fdd_cnn_destroy",
    "fdd_setup_darcy_stokes", "fdd_ds_sizes", "fdd_ds_opts_default", "fdd_ds_precond_apply",
    "fdd_ds_solve",
]
FDD_KT_NONE, FDD_KT_DOWN0, FDD_KT_UP0, FDD_KT_COARSE = 0, 1, 2, 3


class FddDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("K", ctypes.c_double),
                ("mu", ctypes.c_double)]


class FddOpts(ctypes.Structure):
    _fields_ = [("outer_rtol", ctypes.c_double), ("outer_maxit", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("precision", ctypes.c_int), ("mg_nu", ctypes.c_int),
                ("step_rtol", ctypes.c_double), ("check_true_residual", ctypes.c_int),
                ("warmstart", ctypes.c_void_p), ("use_graph", ctypes.c_int),
                ("back_solve", ctypes.c_int)]


class FddStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_its", ctypes.c_int),
                ("inner_solves", ctypes.c_int), ("inner_its_total", ctypes.c_int),
                ("inner_its_max", ctypes.c_int), ("refine_steps", ctypes.c_int),
                ("rel_precond_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("warm_starts", ctypes.c_int),
                ("warm_accepted", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class FddDsOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("velocity_rtol", ctypes.c_double), ("velocity_maxit", ctypes.c_int),
                ("mg_nu", ctypes.c_int), ("pressure_rtol", ctypes.c_double),
                ("pressure_maxit", ctypes.c_int), ("darcy_rtol", ctypes.c_double),
                ("darcy_maxit", ctypes.c_int), ("darcy_precision", ctypes.c_int),
                ("darcy_mg_nu", ctypes.c_int), ("check_true_residual", ctypes.c_int)]


class FddDsStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("its", ctypes.c_int),
                ("velocity_its_total", ctypes.c_int), ("velocity_its_max", ctypes.c_int),
                ("pressure_its_total", ctypes.c_int), ("darcy_its_total", ctypes.c_int),
                ("darcy_its_max", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("true_rel_res", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class FddError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Loads libfdd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with paper_2211_15308_amd.build_lib")
    lib = ctypes.CDLL(LIB_PATH)
    P, V, I, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.fdd_opts_default.argtypes = [ctypes.POINTER(FddOpts)]
    lib.fdd_opts_default.restype = None
    lib.fdd_setup_mesh.argtypes = [ctypes.POINTER(FddDesc), I, ctypes.POINTER(P)]
    lib.fdd_setup_model.argtypes = [I, D, D, D, I, ctypes.POINTER(P)]
    lib.fdd_setup_hdiv.argtypes = [I, D, D, I, ctypes.POINTER(P)]
    lib.fdd_problem_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.fdd_workspace_bytes.argtypes = [P, ctypes.POINTER(FddOpts), ctypes.POINTER(ctypes.c_size_t)]
    lib.fdd_bind_workspace.argtypes = [P, V, ctypes.c_size_t, V]
    lib.fdd_build_rational_pc.argtypes = [P, I, D, I, ctypes.POINTER(P)]
    lib.fdd_ratpc_from_table.argtypes = [P, I, I, D, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(P)]
    lib.fdd_ratpc_query.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D),
                                    ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.fdd_interior_solve.argtypes = [P, V, V, ctypes.POINTER(FddOpts), V, ctypes.POINTER(I)]
    lib.fdd_schur_apply.argtypes = [P, P, V, V, ctypes.POINTER(FddOpts), V]
    lib.fdd_precond_apply.argtypes = [P, P, V, V, V]
    lib.fdd_precond_apply_static.argtypes = [P, P, V, V, V]
    lib.fdd_apply_operator.argtypes = [P, P, V, V, V]
    lib.fdd_solve.argtypes = [P, P, P, V, V, ctypes.POINTER(FddOpts), V, ctypes.POINTER(FddStats)]
    lib.fdd_dd_precond_apply.argtypes = [P, P, V, V, ctypes.POINTER(FddOpts), V]
    lib.fdd_solve_full.argtypes = [P, P, P, V, V, ctypes.POINTER(FddOpts), V, ctypes.POINTER(FddStats)]
    lib.fdd_set_kernel_timer.argtypes = [P, I, D]
    lib.fdd_get_kernel_timer.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D),
                                         ctypes.POINTER(ctypes.c_int64)]
    lib.fdd_destroy_problem.argtypes = [P]
    lib.fdd_destroy_problem.restype = None
    lib.fdd_destroy_ratpc.argtypes = [P]
    lib.fdd_destroy_ratpc.restype = None
    lib.fdd_batch_create.argtypes = [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P)]
    lib.fdd_batch_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdd_batch_set_mid_tile.argtypes = [P, I]
    lib.fdd_batch_tile_edges.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.fdd_batch_bind_workspace.argtypes = [P, V, ctypes.c_size_t, V]
    lib.fdd_solve_batched.argtypes = [P, ctypes.POINTER(V), ctypes.POINTER(V), ctypes.POINTER(FddOpts), V,
                                      ctypes.POINTER(FddStats)]
    lib.fdd_batch_set_kernel_timer.argtypes = [P, I, D]
    lib.fdd_batch_get_kernel_timer.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D),
                                               ctypes.POINTER(ctypes.c_int64)]
    lib.fdd_batch_destroy.argtypes = [P]
    lib.fdd_batch_destroy.restype = None
    F_ = ctypes.c_float
    lib.fdd_cnn_create.argtypes = [I, I, I, I, ctypes.POINTER(P)]
    lib.fdd_cnn_param_count.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.fdd_cnn_workspace_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdd_cnn_bind_workspace.argtypes = [P, V, ctypes.c_size_t, V]
    lib.fdd_cnn_set_params.argtypes = [P, V, V]
    lib.fdd_cnn_forward.argtypes = [P, V, I, I, I, V, V, V, I, V]
    lib.fdd_cnn_loss.argtypes = [P, V, V, I, I, V, V]
    lib.fdd_cnn_backward.argtypes = [P, I, I, V, V]
    lib.fdd_cnn_adam_step.argtypes = [P, V, V, V, V, F_, F_, F_, F_, I, V]
    lib.fdd_cnn_destroy.argtypes = [P]
    lib.fdd_cnn_destroy.restype = None
    lib.fdd_setup_darcy_stokes.argtypes = [I, D, D, D, I, I, ctypes.POINTER(P)]
    lib.fdd_ds_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]
    lib.fdd_ds_opts_default.argtypes = [ctypes.POINTER(FddDsOpts)]
    lib.fdd_ds_opts_default.restype = None
    lib.fdd_ds_precond_apply.argtypes = [P, P, P, V, V, ctypes.POINTER(FddDsOpts), V,
                                         ctypes.POINTER(FddDsStats)]
    lib.fdd_ds_solve.argtypes = [P, P, P, V, V, ctypes.POINTER(FddDsOpts), V, ctypes.POINTER(FddDsStats)]
    lib.fdd_last_error.restype = ctypes.c_char_p
    lib.fdd_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc, allow=(FDD_OK,)):
    if rc not in allow:
        raise FddError(rc, load().fdd_last_error().decode())
    return rc


def opts_default(**kw):
    o = FddOpts()
    load().fdd_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _ptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


_DTYPES = {"f64": "float64", "f32": "float32"}


def _vec(t, numel, device, name, dtype="f64", at_least=False):
    """Pointer of a contiguous device tensor after checking what the kernels assume of it: its
    dtype, that it lives on the problem's device, and its length (the kernels index it up to
    numel without bounds, so a short or mistyped vector must never reach them)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if (t.numel() < numel) if at_least else (t.numel() != numel):
        raise ValueError(f"{name} has {t.numel()} entries, expected {'>= ' if at_least else ''}{numel}")
    want = getattr(torch, _DTYPES[dtype])
    if t.dtype != want:
        raise ValueError(f"{name} must be {want} (got {t.dtype})")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device} (got {t.device})")
    return _ptr(t)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class RationalTable:
    """One rational-approximation table (eq. (RA)); owns the library handle."""

    def __init__(self, handle, which):
        self.h = handle
        self.which = which

    def query(self):
        lib = load()
        m = ctypes.c_int()
        lib.fdd_ratpc_query(self.h, ctypes.byref(m), None, None, None, None)
        c = (ctypes.c_double * max(m.value, 1))()
        p = (ctypes.c_double * max(m.value, 1))()
        c0 = ctypes.c_double()
        err = ctypes.c_double()
        _check(lib.fdd_ratpc_query(self.h, ctypes.byref(m), ctypes.byref(c0), c, p, ctypes.byref(err)))
        return dict(m=m.value, c0=c0.value, c=list(c)[:m.value], p=list(p)[:m.value], max_rel_err=err.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fdd_destroy_ratpc(self.h)
            self.h = None


def _th(T):
    """The handle of a rational table, or NULL for None (the H(div) problem has no operator table)."""
    return None if T is None else T.h


class Problem:
    """A set-up problem (fdd_setup_mesh); host only until bind_workspace is called."""

    def __init__(self, n, K, mu, dim=2, device=0, model_t=None, hdiv=False):
        """model_t is None: eq. (riesz) with Gamma a facet (fdd_setup_mesh); otherwise the paper's
        model problem with Gamma the whole boundary, gamma = mu and exponent t = model_t
        (fdd_setup_model).  hdiv: the H(div) problem of eq. (graddiv) with gamma = mu
        (fdd_setup_hdiv)."""
        lib = load()
        h = ctypes.c_void_p()
        if hdiv:
            _check(lib.fdd_setup_hdiv(n, K, mu, device, ctypes.byref(h)))
        elif model_t is None:
            d = FddDesc(dim, n, K, mu)
            _check(lib.fdd_setup_mesh(ctypes.byref(d), device, ctypes.byref(h)))
        else:
            _check(lib.fdd_setup_model(n, K, mu, model_t, device, ctypes.byref(h)))
        self.h = h
        self.n, self.K, self.mu, self.dim = n, K, mu, dim
        self.model_t = model_t
        self.hdiv = hdiv
        self.device = device
        self.workspace = None
        N, NI, NG = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(lib.fdd_problem_info(h, ctypes.byref(N), ctypes.byref(NI), ctypes.byref(NG),
                                    ctypes.byref(lo), ctypes.byref(hi)))
        self.N, self.NI, self.NG = N.value, NI.value, NG.value
        self.lam_lo, self.lam_hi = lo.value, hi.value

    def _v(self, t, numel, name):
        return _vec(t, numel, self.device, name)

    def workspace_bytes(self, opts=None):
        b = ctypes.c_size_t()
        _check(load().fdd_workspace_bytes(self.h, ctypes.byref(opts or opts_default()), ctypes.byref(b)))
        return b.value

    def bind_workspace(self, workspace=None, stream=None):
        """Binds a uint8 CUDA tensor (allocated here if not given) as the solver workspace."""
        import torch
        nbytes = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        ptr = workspace.data_ptr()
        off = (-ptr) % 256
        _check(load().fdd_bind_workspace(self.h, ctypes.c_void_p(ptr + off), workspace.numel() - off,
                                         _stream(stream)))
        self.workspace = workspace
        return self

    def build_rational_pc(self, which=FDD_RA_PRECOND, tol=1e-12, max_poles=64):
        h = ctypes.c_void_p()
        _check(load().fdd_build_rational_pc(self.h, which, tol, max_poles, ctypes.byref(h)))
        return RationalTable(h, which)

    def ratpc_from_table(self, which, c0, c, p):
        m = len(c)
        ca = (ctypes.c_double * max(m, 1))(*c)
        pa = (ctypes.c_double * max(m, 1))(*p)
        h = ctypes.c_void_p()
        _check(load().fdd_ratpc_from_table(self.h, which, m, c0, ca, pa, ctypes.byref(h)))
        return RationalTable(h, which)

    def interior_solve(self, f, u, opts=None, stream=None):
        its = ctypes.c_int()
        rc = load().fdd_interior_solve(self.h, self._v(f, self.NI, "f"), self._v(u, self.NI, "u"),
                                       ctypes.byref(opts or opts_default()),
                                       _stream(stream), ctypes.byref(its))
        _check(rc)
        return its.value

    def schur_apply(self, H, x_G, y_G, opts=None, stream=None):
        _check(load().fdd_schur_apply(self.h, _th(H), self._v(x_G, self.NG, "x_G"), self._v(y_G, self.NG, "y_G"),
                                      ctypes.byref(opts or opts_default()), _stream(stream)))

    def precond_apply(self, P, r_G, z_G, stream=None):
        _check(load().fdd_precond_apply(self.h, P.h, self._v(r_G, self.NG, "r_G"), self._v(z_G, self.NG, "z_G"),
                                        _stream(stream)))

    def precond_apply_static(self, P, r_G, z_G, stream=None):
        """fdd_precond_apply_static: the same product with no workspace and no allocation."""
        _check(load().fdd_precond_apply_static(self.h, P.h, self._v(r_G, self.NG, "r_G"),
                                               self._v(z_G, self.NG, "z_G"), _stream(stream)))

    def apply_operator(self, H, x, y, stream=None):
        _check(load().fdd_apply_operator(self.h, _th(H), self._v(x, self.N, "x"), self._v(y, self.N, "y"),
                                         _stream(stream)))

    def solve(self, P, H, b, x, opts=None, stream=None, allow_not_converged=False):
        st = FddStats()
        rc = load().fdd_solve(self.h, P.h, _th(H), self._v(b, self.N, "b"), self._v(x, self.N, "x"),
                              ctypes.byref(opts or opts_default()),
                              _stream(stream), ctypes.byref(st))
        _check(rc, (FDD_OK, FDD_NOT_CONVERGED) if allow_not_converged else (FDD_OK,))
        return st.as_dict()

    def dd_precond_apply(self, P, r, z, opts=None, stream=None):
        """z = B r with the lazy block preconditioner (fdd_dd_precond_apply)."""
        _check(load().fdd_dd_precond_apply(self.h, P.h, self._v(r, self.N, "r"), self._v(z, self.N, "z"),
                                           ctypes.byref(opts or opts_default()), _stream(stream)))

    def solve_full(self, P, H, b, x, opts=None, stream=None, allow_not_converged=False):
        """Full-system PCG with the lazy block preconditioner (fdd_solve_full)."""
        st = FddStats()
        rc = load().fdd_solve_full(self.h, P.h, H.h, self._v(b, self.N, "b"), self._v(x, self.N, "x"),
                                   ctypes.byref(opts or opts_default()), _stream(stream), ctypes.byref(st))
        _check(rc, (FDD_OK, FDD_NOT_CONVERGED) if allow_not_converged else (FDD_OK,))
        return st.as_dict()

    def set_kernel_timer(self, kind, split_us=8.0):
        _check(load().fdd_set_kernel_timer(self.h, kind, split_us))

    def kernel_timer(self):
        """(launches, total_ms, long_launches, long_ms, untimed) of the kernel timer."""
        n, ms, nl, lms, un = (ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(),
                              ctypes.c_int64())
        _check(load().fdd_get_kernel_timer(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nl),
                                           ctypes.byref(lms), ctypes.byref(un)))
        return n.value, ms.value, nl.value, lms.value, un.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fdd_destroy_problem(self.h)
            self.h = None


def ds_opts_default(**kw):
    o = FddDsOpts()
    load().fdd_ds_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class DarcyStokes(Problem):
    """The coupled Darcy-Stokes problem of eq. (darcy_stokes) (fdd_setup_darcy_stokes): FGMRES
    with the block-diagonal preconditioner of eq. (darcy_stokes_precond).  Rational tables are the
    Darcy block's (the facet problem with the same n, K, mu)."""

    def __init__(self, n, K, mu, alpha=0.0, krylov=200, device=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.fdd_setup_darcy_stokes(n, K, mu, alpha, krylov, device, ctypes.byref(h)))
        self.h = h
        self.n, self.K, self.mu, self.dim = n, K, mu, 2
        self.alpha, self.krylov = alpha, krylov
        self.model_t, self.hdiv = None, False
        self.device = device
        self.workspace = None
        N, NI, NG = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(lib.fdd_problem_info(h, ctypes.byref(N), ctypes.byref(NI), ctypes.byref(NG),
                                    ctypes.byref(lo), ctypes.byref(hi)))
        self.N, self.NI, self.NG = N.value, NI.value, NG.value
        self.lam_lo, self.lam_hi = lo.value, hi.value
        nu, np_, nd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fdd_ds_sizes(h, ctypes.byref(nu), ctypes.byref(np_), ctypes.byref(nd)))
        self.Nu, self.Np, self.ND = nu.value, np_.value, nd.value

    def precond_apply(self, P, H, r, z, opts=None, stream=None):
        """z = B r (fdd_ds_precond_apply); returns the inner counts."""
        st = FddDsStats()
        _check(load().fdd_ds_precond_apply(self.h, P.h, H.h, self._v(r, self.N, "r"), self._v(z, self.N, "z"),
                                           ctypes.byref(opts or ds_opts_default()), _stream(stream),
                                           ctypes.byref(st)))
        return st.as_dict()

    def solve(self, P, H, b, x, opts=None, stream=None, allow_not_converged=False):
        """x = A^{-1} b by FGMRES (fdd_ds_solve)."""
        st = FddDsStats()
        rc = load().fdd_ds_solve(self.h, P.h, H.h, self._v(b, self.N, "b"), self._v(x, self.N, "x"),
                                 ctypes.byref(opts or ds_opts_default()), _stream(stream), ctypes.byref(st))
        _check(rc, (FDD_OK, FDD_NOT_CONVERGED) if allow_not_converged else (FDD_OK,))
        return st.as_dict()


class Batch:
    """A batch of set-up problems solved together (fdd_batch_create / fdd_solve_batched).

    problems: Problem objects with workspaces bound; P, H: their RationalTable pairs.  The batch
    keeps references to all of them.
    """

    def __init__(self, problems, P, H, stream=None):
        lib = load()
        n = len(problems)
        if not (n == len(P) == len(H)) or n == 0:
            raise ValueError("problems, P and H must be non-empty and of equal length")
        self.problems, self.P, self.H = list(problems), list(P), list(H)
        arr = lambda hs: (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in hs])
        h = ctypes.c_void_p()
        _check(lib.fdd_batch_create(n, arr([p.h for p in problems]), arr([t.h for t in P]),
                                    arr([t.h for t in H]), ctypes.byref(h)))
        self.h = h
        self.count = n
        import torch
        nb = ctypes.c_size_t()
        _check(lib.fdd_batch_workspace_bytes(h, ctypes.byref(nb)))
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=f"cuda:{problems[0].device}")
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        _check(lib.fdd_batch_bind_workspace(h, ctypes.c_void_p(ptr + off), ws.numel() - off, _stream(stream)))
        self.workspace = ws

    def solve(self, bs, xs, opts=None, stream=None, allow_not_converged=False):
        """Solves every instance; returns the list of per-instance stats dicts."""
        n = self.count
        if len(bs) != n or len(xs) != n:
            raise ValueError("one b and one x per instance")
        ba = (ctypes.c_void_p * n)(*[_vec(b, p.N, p.device, f"b[{i}]").value
                                     for i, (p, b) in enumerate(zip(self.problems, bs))])
        xa = (ctypes.c_void_p * n)(*[_vec(x, p.N, p.device, f"x[{i}]").value
                                     for i, (p, x) in enumerate(zip(self.problems, xs))])
        st = (FddStats * n)()
        rc = load().fdd_solve_batched(self.h, ba, xa, ctypes.byref(opts or opts_default()),
                                      _stream(stream), st)
        _check(rc, (FDD_OK, FDD_NOT_CONVERGED) if allow_not_converged else (FDD_OK,))
        return [s.as_dict() for s in st]

    def set_mid_tile(self, edge):
        """Tile edge of the intermediate levels: 16, 32, or 0 (by tile count)."""
        _check(load().fdd_batch_set_mid_tile(self.h, edge))

    def tile_edges(self):
        levels = ctypes.c_int()
        edges = (ctypes.c_int * 16)()
        _check(load().fdd_batch_tile_edges(self.h, ctypes.byref(levels), edges))
        return list(edges)[:levels.value]

    def set_kernel_timer(self, kind, split_us=8.0):
        _check(load().fdd_batch_set_kernel_timer(self.h, kind, split_us))

    def kernel_timer(self):
        """(launches, total_ms, long_launches, long_ms, untimed) of the kernel timer."""
        n, ms, nl, lms, un = (ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(),
                              ctypes.c_int64())
        _check(load().fdd_batch_get_kernel_timer(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nl),
                                                 ctypes.byref(lms), ctypes.byref(un)))
        return n.value, ms.value, nl.value, lms.value, un.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fdd_batch_destroy(self.h)
            self.h = None


class Cnn:
    """The warm-start network (fdd_cnn_*): a handle plus its bound workspace.

    Parameters, gradients and Adam moments are caller-owned FP32 CUDA tensors of length
    param_count in the layout of include/fdd.h (per layer W[3][3][c_in][c_out], then b).
    """

    def __init__(self, batch_max, n_max, train=False, device=0, stream=None):
        import torch
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.fdd_cnn_create(batch_max, n_max, 1 if train else 0, device, ctypes.byref(h)))
        self.h = h
        self.batch_max, self.n_max, self.train = batch_max, n_max, train
        self.device = device
        c = ctypes.c_int64()
        _check(lib.fdd_cnn_param_count(h, ctypes.byref(c)))
        self.param_count = c.value
        nb = ctypes.c_size_t()
        _check(lib.fdd_cnn_workspace_bytes(h, ctypes.byref(nb)))
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=f"cuda:{device}")
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        _check(lib.fdd_cnn_bind_workspace(h, ctypes.c_void_p(ptr + off), ws.numel() - off, _stream(stream)))
        self.workspace = ws

    def _p(self, t, name):
        return _vec(t, self.param_count, self.device, name, "f32")

    def set_params(self, theta, stream=None):
        _check(load().fdd_cnn_set_params(self.h, self._p(theta, "theta"), _stream(stream)))

    def forward(self, traces, log10K, log10mu, out, n, rescale=True, stream=None):
        if traces.dim() != 2 or traces.shape[1] < n - 1:
            raise ValueError("traces must be (batch, >= n - 1)")
        B = traces.shape[0]
        d = self.device
        tr = _vec(traces, B * traces.shape[1], d, "traces")
        _check(load().fdd_cnn_forward(self.h, tr, traces.stride(0), B, n, _vec(log10K, B, d, "log10K"),
                                      _vec(log10mu, B, d, "log10mu"),
                                      _vec(out, B * (n - 1) ** 2, d, "out", "f32"), 1 if rescale else 0,
                                      _stream(stream)))

    def loss(self, out, target, n, loss=None, stream=None):
        B = out.shape[0]
        d = self.device
        _check(load().fdd_cnn_loss(self.h, _vec(out, B * (n - 1) ** 2, d, "out", "f32"),
                                   _vec(target, B * (n - 1) ** 2, d, "target", "f32"), B, n,
                                   None if loss is None else _vec(loss, 1, d, "loss"), _stream(stream)))

    def backward(self, batch, n, grad, stream=None):
        _check(load().fdd_cnn_backward(self.h, batch, n, self._p(grad, "grad"), _stream(stream)))

    def adam_step(self, theta, grad, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        _check(load().fdd_cnn_adam_step(self.h, self._p(theta, "theta"), self._p(grad, "grad"), self._p(m, "m"),
                                        self._p(v, "v"), lr, b1, b2, eps, step, _stream(stream)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.fdd_cnn_destroy(self.h)
            self.h = None


def pack_params(params):
    """Flattens [(W (3, 3, c_in, c_out), b)] into the library's parameter order (numpy)."""
    import numpy as np
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unpack_params(theta, widths=(5, 32, 32, 32, 32, 32, 1)):
    """Inverse of pack_params."""
    import numpy as np
    theta = np.asarray(theta)
    out, o = [], 0
    for a, c in zip(widths[:-1], widths[1:]):
        W = theta[o:o + 9 * a * c].reshape(3, 3, a, c)
        o += 9 * a * c
        b = theta[o:o + c]
        o += c
        out.append((W, b))
    return out


# names of the C ABI calls
def setup_mesh(n, K, mu, dim=2, device=0):
    return Problem(n, K, mu, dim, device)


def setup_model(n, K, gamma, t, device=0):
    """The paper's model problem (Gamma = the whole boundary, exponent t): fdd_setup_model."""
    return Problem(n, K, gamma, 2, device, model_t=t)


def setup_hdiv(n, K, gamma, device=0):
    """The H(div) problem of eq. (graddiv) (BDM1, Gamma = the whole boundary): fdd_setup_hdiv."""
    return Problem(n, K, gamma, 2, device, hdiv=True)


def setup_darcy_stokes(n, K, mu, alpha=0.0, krylov=200, device=0):
    """The coupled Darcy-Stokes problem of eq. (darcy_stokes): fdd_setup_darcy_stokes."""
    return DarcyStokes(n, K, mu, alpha, krylov, device)


def build_rational_pc(prob, which=FDD_RA_PRECOND, tol=1e-12, max_poles=64):
    return prob.build_rational_pc(which, tol, max_poles)


def schur_apply(prob, H, x_G, y_G, opts=None, stream=None):
    return prob.schur_apply(H, x_G, y_G, opts, stream)


def precond_apply(prob, P, r_G, z_G, stream=None):
    return prob.precond_apply(P, r_G, z_G, stream)


def solve(prob, P, H, b, x, opts=None, stream=None):
    return prob.solve(P, H, b, x, opts, stream)


def solve_batched(batch, bs, xs, opts=None, stream=None):
    return batch.solve(bs, xs, opts, stream)
