"""ctypes binding of ``libstwr.so`` (argument marshalling only).

Names mirror the C ABI in ``include/stwr.h``.  Vectors are torch tensors on
the CUDA (HIP) device, float64, contiguous; the binding passes their data
pointers and the current torch stream.  The library must be built
(``python -m paper_2407_13997_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstwr.so")

STWR_OK = 0
STATUS = {0: "STWR_OK", -1: "STWR_ERR_ARG", -2: "STWR_ERR_OOM", -3: "STWR_ERR_BUDGET",
          -4: "STWR_ERR_DEVICE", -5: "STWR_ERR_SINGULAR", -6: "STWR_ERR_NONFINITE",
          -7: "STWR_ERR_NOT_CONVERGED", -8: "STWR_ERR_STATE"}
FP64, FP32 = 0, 1

EXPORTED = [
    "stwr_default_opts", "stwr_ctx_create", "stwr_ctx_destroy", "stwr_ctx_set_stream",
    "stwr_last_error", "stwr_ctx_bytes_in_use", "stwr_problem_bytes", "stwr_problem_n_st", "stwr_mesh_info",
    "stwr_problem_create", "stwr_problem_destroy", "stwr_problem_sizes", "stwr_patch_sizes",
    "stwr_level_time_chunks",
    "stwr_set_opts",
    "stwr_nonlinear_residual", "stwr_linear_rhs", "stwr_velocity_l2_error", "stwr_expand",
    "stwr_assemble",
    "stwr_get_operator", "stwr_apply",
    "stwr_residual", "stwr_patch_factor", "stwr_patch_apply", "stwr_patch_apply_noalloc",
    "stwr_eig_estimate",
    "stwr_relax", "stwr_restrict", "stwr_prolong_add", "stwr_coarse_solve",
    "stwr_setup_smoothers", "stwr_vcycle", "stwr_fgmres", "stwr_newton_solve",
    "stwr_project_pressure", "stwr_ctx_set_timing", "stwr_ctx_kernel_times", "stwr_ctx_read_rate",
    "stwr_ctx_set_alloc_mode", "stwr_server_create", "stwr_server_submit", "stwr_server_poll",
    "stwr_server_wait", "stwr_server_now", "stwr_server_destroy",
    "stwr_batch_create", "stwr_batch_add", "stwr_batch_step", "stwr_batch_poll", "stwr_batch_info",
    "stwr_batch_destroy", "stwr_level_patches", "stwr_level_transfer",
]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("mesh_n", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("q", ctypes.c_int32),
                ("n_slabs", ctypes.c_int32), ("t_final", ctypes.c_double),
                ("reynolds", ctypes.c_double), ("n_psi_modes", ctypes.c_int32),
                ("n_p_modes", ctypes.c_int32), ("psi_ab", ctypes.POINTER(ctypes.c_int32)),
                ("psi_coef", ctypes.POINTER(ctypes.c_double)),
                ("p_ab", ctypes.POINTER(ctypes.c_int32)),
                ("p_coef", ctypes.POINTER(ctypes.c_double)), ("flow", ctypes.c_int32),
                ("temporal_nodes", ctypes.c_int32), ("equation", ctypes.c_int32),
                ("degree", ctypes.c_int32)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("eig_steps", ctypes.c_int32), ("smoother_prec", ctypes.c_int32),
                ("gmres_restart", ctypes.c_int32), ("gmres_maxit", ctypes.c_int32),
                ("gmres_rtol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
                ("newton_rtol", ctypes.c_double), ("vcycle_graph", ctypes.c_int32),
                ("newton_ew", ctypes.c_int32), ("gmres_atol", ctypes.c_double),
                ("time_chunks", ctypes.c_int32), ("factor_mfma", ctypes.c_int32),
                ("deterministic", ctypes.c_int32)]


MAX_NEWTON, MAX_LEVELS = 64, 16


class Stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("linear_its_total", ctypes.c_int32),
                ("linear_its", ctypes.c_int32 * MAX_NEWTON),
                ("fnorm", ctypes.c_double * (MAX_NEWTON + 1)),
                ("lambda_", ctypes.c_double * MAX_LEVELS),
                ("final_rel_residual", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double),
                ("linear_rel", ctypes.c_double * MAX_NEWTON)]

    def as_dict(self):
        k = self.newton_its
        return {"newton": k, "linear": list(self.linear_its[:max(k, 1)]),
                "linear_total": self.linear_its_total,
                "fnorm": list(self.fnorm[:k + 1]), "lambda": list(self.lambda_),
                "final_rel_residual": self.final_rel_residual,
                "setup_seconds": self.setup_seconds, "solve_seconds": self.solve_seconds,
                "linear_rel": list(self.linear_rel[:max(k, 1)])}


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("newton_its", ctypes.c_int32),
                ("linear_its", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("submit_time", ctypes.c_double), ("start_time", ctypes.c_double),
                ("end_time", ctypes.c_double), ("fnorm_ratio", ctypes.c_double),
                ("bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StwrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str | None = None):
    """Load the library (``STWR_LIBRARY`` overrides the in-tree path); raises if
    it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("STWR_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2407_13997_amd.build")
    lib = ctypes.CDLL(path)
    P, V = ctypes.c_void_p, ctypes.c_void_p
    i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    sig = {
        "stwr_default_opts": [ctypes.POINTER(SolverOpts)],
        "stwr_ctx_create": [i32, V, u64, ctypes.POINTER(P)],
        "stwr_ctx_destroy": [P],
        "stwr_ctx_set_stream": [P, V],
        "stwr_ctx_bytes_in_use": [P, ctypes.POINTER(u64)],
        "stwr_problem_bytes": [ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolverOpts), ctypes.POINTER(u64)],
        "stwr_problem_n_st": [ctypes.POINTER(ProblemDesc), ctypes.POINTER(i64)],
        "stwr_mesh_info": [i32, ctypes.POINTER(i64)],
        "stwr_problem_create": [P, ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolverOpts), ctypes.POINTER(P)],
        "stwr_problem_destroy": [P],
        "stwr_problem_sizes": [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)],
        "stwr_set_opts": [P, ctypes.POINTER(SolverOpts)],
        "stwr_nonlinear_residual": [P, V, V],
        "stwr_velocity_l2_error": [P, V, ctypes.POINTER(f64)],
        "stwr_expand": [P, V, V],
        "stwr_assemble": [P, V],
        "stwr_get_operator": [P, i32, ctypes.POINTER(i64), V, V, V, V],
        "stwr_apply": [P, i32, V, V],
        "stwr_residual": [P, i32, V, V, V],
        "stwr_patch_factor": [P, i32, i32],
        "stwr_patch_apply": [P, i32, V, V],
        "stwr_patch_apply_noalloc": [P, i32, V, V],
        "stwr_eig_estimate": [P, i32, ctypes.POINTER(f64)],
        "stwr_relax": [P, i32, V, V, i32, f64, f64],
        "stwr_restrict": [P, i32, V, V],
        "stwr_prolong_add": [P, i32, V, V],
        "stwr_coarse_solve": [P, V, V],
        "stwr_setup_smoothers": [P],
        "stwr_vcycle": [P, V, V],
        "stwr_fgmres": [P, V, V, ctypes.POINTER(Stats)],
        "stwr_newton_solve": [P, V, ctypes.POINTER(Stats)],
        "stwr_project_pressure": [P, i32, V],
        "stwr_ctx_set_timing": [P, i32],
        "stwr_ctx_kernel_times": [P, ctypes.POINTER(f64), ctypes.POINTER(i64)],
        "stwr_ctx_read_rate": [P, V, u64, i32, ctypes.POINTER(f64)],
        "stwr_ctx_set_alloc_mode": [P, i32],
        "stwr_server_create": [i32, i32, u64, ctypes.POINTER(P)],
        "stwr_server_submit": [P, ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolverOpts), V,
                               ctypes.POINTER(i64)],
        "stwr_server_poll": [P, ctypes.POINTER(Result), i32, ctypes.POINTER(i32)],
        "stwr_server_wait": [P, f64],
        "stwr_server_now": [P, ctypes.POINTER(f64)],
        "stwr_server_destroy": [P],
        "stwr_batch_create": [P, i32, ctypes.POINTER(P)],
        "stwr_batch_add": [P, ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolverOpts), V, ctypes.POINTER(i64)],
        "stwr_batch_step": [P, ctypes.POINTER(i32)],
        "stwr_batch_poll": [P, ctypes.POINTER(Result), i32, ctypes.POINTER(i32)],
        "stwr_batch_info": [P, ctypes.POINTER(i64)],
        "stwr_batch_destroy": [P],
        "stwr_level_patches": [i32, i32, ctypes.POINTER(i64), V, V],
        "stwr_level_transfer": [i32, i32, ctypes.POINTER(i64), V, V, V, V],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    lib.stwr_last_error.argtypes = [P]
    lib.stwr_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def default_opts() -> SolverOpts:
    o = SolverOpts()
    load().stwr_default_opts(ctypes.byref(o))
    return o


def make_desc(prob):
    """ProblemDesc from a stwr_workloads.Problem; returns (desc, keepalive)."""
    psi_ab = np.ascontiguousarray(prob.psi_ab, dtype=np.int32)
    psi_coef = np.ascontiguousarray(prob.psi_coef, dtype=np.float64)
    p_ab = np.ascontiguousarray(prob.p_ab, dtype=np.int32)
    p_coef = np.ascontiguousarray(prob.p_coef, dtype=np.float64)
    d = ProblemDesc(prob.mesh_n, prob.n_levels, prob.q, prob.n_slabs, prob.t_final, prob.reynolds,
                    len(psi_ab), len(p_ab),
                    psi_ab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    psi_coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    p_ab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    p_coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    int(getattr(prob, "flow", 0)), int(getattr(prob, "nodes", 0)),
                    int(getattr(prob, "equation", 0)), int(getattr(prob, "degree", 0)))
    return d, (psi_ab, psi_coef, p_ab, p_coef)


def problem_bytes(prob, opts=None) -> int:
    lib = load()
    d, keep = make_desc(prob)
    opts = opts or default_opts()
    out = ctypes.c_uint64()
    rc = lib.stwr_problem_bytes(ctypes.byref(d), ctypes.byref(opts), ctypes.byref(out))
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    return int(out.value)


def problem_n_st(prob) -> int:
    """Length of the problem's level-0 space-time vectors (stwr_problem_n_st)."""
    lib = load()
    d, keep = make_desc(prob)
    out = ctypes.c_int64()
    rc = lib.stwr_problem_n_st(ctypes.byref(d), ctypes.byref(out))
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    return int(out.value)


def mesh_info(mesh_n: int) -> np.ndarray:
    lib = load()
    out = np.zeros(52, dtype=np.int64)
    rc = lib.stwr_mesh_info(mesh_n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    return out


def level_patches(mesh_n: int, degree: int = 1):
    """(counts, patch_ptr, patch_dofs) of the host-built Vanka+star patches
    (stwr_level_patches)."""
    lib = load()
    counts = np.zeros(7, dtype=np.int64)
    cp = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.stwr_level_patches(mesh_n, degree, cp, None, None)
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    ptr = np.zeros(counts[1] + 1, dtype=np.int32)
    dofs = np.zeros(counts[2], dtype=np.int32)
    rc = lib.stwr_level_patches(mesh_n, degree, cp, ptr.ctypes.data_as(ctypes.c_void_p),
                                dofs.ctypes.data_as(ctypes.c_void_p))
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    return counts, ptr, dofs


def level_transfer(mesh_n: int, degree: int = 1):
    """(P as scipy CSR of fine x coarse free DoFs, inject) from stwr_level_transfer."""
    import scipy.sparse as sp
    lib = load()
    counts = np.zeros(3, dtype=np.int64)
    cp = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib.stwr_level_transfer(mesh_n, degree, cp, None, None, None, None)
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    nf, nc, nnz = (int(v) for v in counts)
    ptr = np.zeros(nf + 1, dtype=np.int32)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz)
    inj = np.zeros(nc, dtype=np.int32)
    rc = lib.stwr_level_transfer(mesh_n, degree, cp, ptr.ctypes.data_as(ctypes.c_void_p),
                                 col.ctypes.data_as(ctypes.c_void_p), val.ctypes.data_as(ctypes.c_void_p),
                                 inj.ctypes.data_as(ctypes.c_void_p))
    if rc != STWR_OK:
        raise StwrError(rc, lib.stwr_last_error(None).decode())
    return sp.csr_matrix((val, col, ptr), shape=(nf, nc)), inj


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "need a contiguous float64 device tensor"
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Library context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        rc = self.lib.stwr_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), hbm_budget,
                                      ctypes.byref(h))
        if rc != STWR_OK:
            raise StwrError(rc, self.lib.stwr_last_error(None).decode())
        self.h = h
        self.device = device

    def set_stream(self, stream):
        self.lib.stwr_ctx_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream))

    def bytes_in_use(self) -> int:
        out = ctypes.c_uint64()
        self.lib.stwr_ctx_bytes_in_use(self.h, ctypes.byref(out))
        return int(out.value)

    def set_timing(self, enable: bool):
        self.check(self.lib.stwr_ctx_set_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        """{class: (total_ms, launches)} since the last call; classes sweep/operator/gather."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        self.check(self.lib.stwr_ctx_kernel_times(self.h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("sweep", "operator", "gather"))}

    def read_rate(self, buf, reps: int = 5) -> float:
        """Attainable HBM read rate in GB/s, measured on the contiguous device
        tensor `buf` (at least 64 MiB, a multiple of 16 bytes; not modified)."""
        assert buf.is_cuda and buf.is_contiguous(), "need a contiguous device tensor"
        out = ctypes.c_double()
        nbytes = buf.numel() * buf.element_size()
        self.check(self.lib.stwr_ctx_read_rate(self.h, ctypes.c_void_p(buf.data_ptr()), nbytes, reps,
                                               ctypes.byref(out)))
        return float(out.value)

    def error(self) -> str:
        return self.lib.stwr_last_error(self.h).decode()

    def check(self, rc):
        if rc != STWR_OK:
            raise StwrError(rc, self.error())

    def close(self):
        if self.h:
            self.lib.stwr_ctx_destroy(self.h)
            self.h = None


class Problem:
    """One space-time problem held by the library (all calls mirror stwr.h)."""

    def __init__(self, ctx: Context, prob, opts: SolverOpts | None = None):
        self.ctx, self.lib = ctx, ctx.lib
        self.prob = prob
        self.opts = opts or default_opts()
        d, self._keep = make_desc(prob)
        h = ctypes.c_void_p()
        ctx.check(self.lib.stwr_problem_create(ctx.h, ctypes.byref(d), ctypes.byref(self.opts),
                                               ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.stwr_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self, level=0):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self.ctx.check(self.lib.stwr_problem_sizes(self.h, level, ctypes.byref(a), ctypes.byref(b),
                                                   ctypes.byref(c)))
        return a.value, b.value, c.value

    def patch_sizes(self, level=0) -> np.ndarray:
        """Spatial DoFs of every patch of a level."""
        nb = np.zeros(self.sizes(level)[2], dtype=np.int32)
        self.ctx.check(self.lib.stwr_patch_sizes(self.h, level, nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return nb

    def time_chunks(self, level=0) -> int:
        c = ctypes.c_int32()
        self.ctx.check(self.lib.stwr_level_time_chunks(self.h, level, ctypes.byref(c)))
        return c.value

    def vec(self, level=0):
        import torch
        return torch.zeros(self.sizes(level)[0], dtype=torch.float64, device=f"cuda:{self.ctx.device}")

    def set_opts(self, opts):
        self.ctx.check(self.lib.stwr_set_opts(self.h, ctypes.byref(opts)))
        self.opts = opts

    def nonlinear_residual(self, U, F):
        self.ctx.check(self.lib.stwr_nonlinear_residual(self.h, _ptr(U), _ptr(F)))

    def linear_rhs(self, b):
        """b = -F(0); the heat equation's right-hand side."""
        self.ctx.check(self.lib.stwr_linear_rhs(self.h, _ptr(b)))

    def velocity_l2_error(self, U) -> float:
        err = ctypes.c_double()
        self.ctx.check(self.lib.stwr_velocity_l2_error(self.h, _ptr(U), ctypes.byref(err)))
        return err.value

    def full_length(self) -> int:
        M = self.prob.mesh_n
        return (2 * (2 * M + 1) ** 2 + (M + 1) ** 2) * self.prob.n_slabs * (self.prob.q + 1)

    def expand(self, U, full=None):
        """Full nodal vector (ux, uy at every P2 node, p at every vertex)."""
        import torch
        if full is None:
            full = torch.empty(self.full_length(), dtype=torch.float64, device=U.device)
        self.ctx.check(self.lib.stwr_expand(self.h, _ptr(U), _ptr(full)))
        return full

    def assemble(self, U):
        self.ctx.check(self.lib.stwr_assemble(self.h, _ptr(U)))

    def get_operator(self, level=0, values=True):
        nnz = ctypes.c_int64()
        self.ctx.check(self.lib.stwr_get_operator(self.h, level, ctypes.byref(nnz), None, None, None, None))
        n_st, nf, _ = self.sizes(level)
        N, NQ = self.prob.n_slabs, self.prob.q + 1
        rp = np.zeros(nf + 1, dtype=np.int32)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value * N * NQ * NQ) if values else None
        mass = np.zeros(nnz.value) if values else None
        c = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        self.ctx.check(self.lib.stwr_get_operator(self.h, level, ctypes.byref(nnz), c(rp), c(col),
                                                  c(val), c(mass)))
        return rp, col, val, mass

    def apply(self, level, x, y):
        self.ctx.check(self.lib.stwr_apply(self.h, level, _ptr(x), _ptr(y)))

    def residual(self, level, b, x, r):
        self.ctx.check(self.lib.stwr_residual(self.h, level, _ptr(b), _ptr(x), _ptr(r)))

    def patch_factor(self, level, prec=FP64):
        self.ctx.check(self.lib.stwr_patch_factor(self.h, level, prec))

    def patch_apply(self, level, r, z):
        self.ctx.check(self.lib.stwr_patch_apply(self.h, level, _ptr(r), _ptr(z)))

    def patch_apply_noalloc(self, level, r, z):
        self.ctx.check(self.lib.stwr_patch_apply_noalloc(self.h, level, _ptr(r), _ptr(z)))

    def eig_estimate(self, level):
        lam = ctypes.c_double()
        self.ctx.check(self.lib.stwr_eig_estimate(self.h, level, ctypes.byref(lam)))
        return lam.value

    def relax(self, level, b, x, n_steps, a, bnd):
        self.ctx.check(self.lib.stwr_relax(self.h, level, _ptr(b), _ptr(x), n_steps, a, bnd))

    def restrict(self, fine_level, rf, rc):
        self.ctx.check(self.lib.stwr_restrict(self.h, fine_level, _ptr(rf), _ptr(rc)))

    def prolong_add(self, fine_level, ec, xf):
        self.ctx.check(self.lib.stwr_prolong_add(self.h, fine_level, _ptr(ec), _ptr(xf)))

    def coarse_solve(self, b, x):
        self.ctx.check(self.lib.stwr_coarse_solve(self.h, _ptr(b), _ptr(x)))

    def setup_smoothers(self):
        self.ctx.check(self.lib.stwr_setup_smoothers(self.h))

    def vcycle(self, b, x):
        self.ctx.check(self.lib.stwr_vcycle(self.h, _ptr(b), _ptr(x)))

    def project_pressure(self, level, x):
        self.ctx.check(self.lib.stwr_project_pressure(self.h, level, _ptr(x)))

    def fgmres(self, b, x, allow_unconverged=False):
        st = Stats()
        rc = self.lib.stwr_fgmres(self.h, _ptr(b), _ptr(x), ctypes.byref(st))
        if rc != STWR_OK and not (allow_unconverged and rc == -7):
            self.ctx.check(rc)
        return st.as_dict()

    def newton_solve(self, U, allow_unconverged=False):
        st = Stats()
        rc = self.lib.stwr_newton_solve(self.h, _ptr(U), ctypes.byref(st))
        if rc != STWR_OK and not (allow_unconverged and rc == -7):
            self.ctx.check(rc)
        return st.as_dict()


class Server:
    """Continuous-batching solve server (stwr_server_*): n_slots workers with
    their own HIP streams, FIFO admission by HBM budget."""

    def __init__(self, device: int = 0, n_slots: int = 4, hbm_budget: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        rc = self.lib.stwr_server_create(device, n_slots, hbm_budget, ctypes.byref(h))
        if rc != STWR_OK:
            raise StwrError(rc, "stwr_server_create failed")
        self.h = h
        self._keep = {}

    def submit(self, prob, opts: SolverOpts | None = None, want_solution: bool = True) -> int:
        d, keep = make_desc(prob)
        opts = opts or default_opts()
        out = np.zeros(problem_n_st(prob)) if want_solution else None
        rid = ctypes.c_int64()
        rc = self.lib.stwr_server_submit(self.h, ctypes.byref(d), ctypes.byref(opts),
                                         None if out is None else out.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(rid))
        if rc != STWR_OK:
            raise StwrError(rc, "stwr_server_submit failed")
        self._keep[rid.value] = out
        return rid.value

    def poll(self, max_results: int = 256):
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        rc = self.lib.stwr_server_poll(self.h, buf, max_results, ctypes.byref(n))
        if rc != STWR_OK:
            raise StwrError(rc, "stwr_server_poll failed")
        out = []
        for i in range(n.value):
            d = buf[i].as_dict()
            d["solution"] = self._keep.pop(d["id"], None)
            out.append(d)
        return out

    def wait(self, timeout_s: float = 600.0) -> bool:
        return self.lib.stwr_server_wait(self.h, timeout_s) == STWR_OK

    def now(self) -> float:
        t = ctypes.c_double()
        self.lib.stwr_server_now(self.h, ctypes.byref(t))
        return t.value

    def close(self):
        if self.h:
            self.lib.stwr_server_destroy(self.h)
            self.h = None


class Batch:
    """Batched solves on one context (stwr_batch_*): problems advance together,
    their patch factorizations and sweeps in shared persistent launches."""

    INFO = ("steps", "graph_captures", "vcycles", "sweep_launches", "factor_launches", "sweep_tile_q0",
            "sweep_tile_q1", "factor_tile_small1", "factor_tile_small2", "factor_tile_big2", "live")

    def __init__(self, ctx: Context, use_graph: bool = True):
        self.ctx, self.lib = ctx, ctx.lib
        h = ctypes.c_void_p()
        ctx.check(self.lib.stwr_batch_create(ctx.h, 1 if use_graph else 0, ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def add(self, prob, opts: SolverOpts | None = None, want_solution: bool = True) -> int:
        """Create the problem in the batch; raises StwrError (STWR_ERR_BUDGET
        when it does not fit the context's budget)."""
        d, keep = make_desc(prob)
        opts = opts or default_opts()
        out = np.zeros(problem_n_st(prob)) if want_solution else None
        rid = ctypes.c_int64()
        self.ctx.check(self.lib.stwr_batch_add(self.h, ctypes.byref(d), ctypes.byref(opts),
                                               None if out is None else out.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(rid)))
        self._keep[rid.value] = out
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int32()
        self.ctx.check(self.lib.stwr_batch_step(self.h, ctypes.byref(n)))
        return n.value

    def poll(self, max_results: int = 256):
        buf = (Result * max_results)()
        n = ctypes.c_int32()
        self.ctx.check(self.lib.stwr_batch_poll(self.h, buf, max_results, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            d = buf[i].as_dict()
            d["solution"] = self._keep.pop(d["id"], None)
            out.append(d)
        return out

    def run(self, max_steps: int = 1_000_000):
        """Step until every problem has finished; returns all results."""
        res = []
        for _ in range(max_steps):
            live = self.step()
            res += self.poll()
            if live == 0:
                break
        return res + self.poll()

    def info(self) -> dict:
        out = np.zeros(len(self.INFO), dtype=np.int64)
        self.ctx.check(self.lib.stwr_batch_info(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return dict(zip(self.INFO, (int(v) for v in out)))

    def close(self):
        if self.h:
            self.lib.stwr_batch_destroy(self.h)
            self.h = None
