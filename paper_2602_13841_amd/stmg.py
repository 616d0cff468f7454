"""Thin ctypes binding of libstmg.so (argument marshalling only).

Every numerical step runs in the HIP library; this module checks tensor
shapes, dtypes and devices and passes raw device pointers and the current
torch stream.  There is no fallback: if the library is missing the import of
the binding fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstmg.so")

STMG_F64 = 0
STMG_F32 = 1
STMG_F32_BF16 = 2   # batched factorizations: BF16 operands of the FP32 trailing updates
STMG_F32_F16 = 3    # same with FP16 operands
# return codes (include/stmg.h)
STMG_OK, STMG_EINVAL, STMG_ENOMEM, STMG_EHIP, STMG_ESTATE, STMG_ENONFINITE, STMG_NOT_CONVERGED = 0, -1, -2, -3, -4, -5, 1


class StmgError(RuntimeError):
    pass


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells", ctypes.c_int * 3), ("vertices", ctypes.c_void_p),
                ("r", ctypes.c_int), ("k", ctypes.c_int), ("nu", ctypes.c_double), ("tau", ctypes.c_double),
                ("dirichlet_faces", ctypes.c_uint), ("gamma1", ctypes.c_double), ("gamma2", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("n_q", ctypes.c_int), ("max_levels", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("vanka_omega", ctypes.c_double), ("prec_mg", ctypes.c_int),
                ("newton_rtol", ctypes.c_double), ("newton_atol", ctypes.c_double), ("newton_maxit", ctypes.c_int),
                ("ew_eta0", ctypes.c_double), ("ew_c", ctypes.c_double), ("ew_theta", ctypes.c_double),
                ("ew_eta_min", ctypes.c_double), ("ew_eta_max", ctypes.c_double),
                ("ls_lambda0", ctypes.c_double), ("ls_c", ctypes.c_double), ("ls_tau", ctypes.c_double),
                ("ls_alpha_min", ctypes.c_double), ("ls_window", ctypes.c_int), ("ls_max_backtracks", ctypes.c_int),
                ("rb_theta_N", ctypes.c_double), ("rb_theta_L", ctypes.c_double), ("rb_kappa_abs", ctypes.c_double),
                ("rb_stag_theta", ctypes.c_double), ("rb_stag_s", ctypes.c_int),
                ("fgmres_maxit", ctypes.c_int), ("vanka_weighting", ctypes.c_int),
                ("vanka_time_decoupled", ctypes.c_int),
                ("use_graphs", ctypes.c_int),
                ("time_coarsening", ctypes.c_int),
                ("vanka_factor_bf16", ctypes.c_int),
                ("vanka_diagonal", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("fgmres_its_total", ctypes.c_int),
                ("fgmres_its", ctypes.c_int * 64), ("rebuilds", ctypes.c_int), ("backtracks", ctypes.c_int),
                ("res0_M", ctypes.c_double), ("res_M", ctypes.c_double), ("wall_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("prob", Problem), ("arrival_s", ctypes.c_double), ("v_prev", ctypes.c_void_p),
                ("rhs", ctypes.c_void_p), ("u_init", ctypes.c_void_p), ("u_out", ctypes.c_void_p)]


class RequestResult(ctypes.Structure):
    _fields_ = [("start_s", ctypes.c_double), ("end_s", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("rc", ctypes.c_int), ("footprint", ctypes.c_size_t), ("stats", Stats),
                ("reused_context", ctypes.c_int)]


_lib = None

# exported symbols and their argument types
_SIGS = {
    "stmg_default_options": (None, [ctypes.c_void_p]),
    "stmg_footprint_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_workspace_used": (ctypes.c_size_t, [ctypes.c_void_p]),
    "stmg_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "stmg_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "stmg_set_coefficients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
    "stmg_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_set_slab_data": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_jacobian_vmult": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "stmg_jacobian_vmult_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_int]),
    "stmg_mass_vmult": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_num_levels": (ctypes.c_int, [ctypes.c_void_p]),
    "stmg_level_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_level_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "stmg_smoother_rebuild": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_level_jacobian_vmult": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "stmg_vanka_smooth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int]),
    "stmg_vcycle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_prolongate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "stmg_restrict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "stmg_fgmres": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_newton_gmres_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_march": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p]),
    "stmg_serve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_timing_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "stmg_timing_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "stmg_timing_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_level_patch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "stmg_batched_lu": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_batched_lu_config": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "stmg_batched_lu_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "stmg_batched_lu_solve": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise StmgError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if not hasattr(L, name):
                raise StmgError(f"{LIB_PATH} does not export {name}; rebuild the library")
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def default_options(**overrides) -> Options:
    o = Options()
    lib().stmg_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_problem(dim, n, r, k, nu, tau, vertices=None, dirichlet_faces=None, gamma1=10.0, gamma2=10.0):
    """Problem structure; returns (struct, keep-alive vertex array)."""
    import numpy as np
    n = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n,) * dim))
    p = Problem()
    p.dim = dim
    for a in range(3):
        p.n_cells[a] = n[a] if a < len(n) else 1
    vert = None
    if vertices is not None:
        vert = np.ascontiguousarray(vertices, dtype=np.float64)
        p.vertices = vert.ctypes.data
    p.r, p.k, p.nu, p.tau = r, k, nu, tau
    p.dirichlet_faces = (1 << (2 * dim)) - 1 if dirichlet_faces is None else dirichlet_faces
    p.gamma1, p.gamma2 = gamma1, gamma2
    return p, vert


def footprint_bytes(problem: Problem, options: Options | None = None) -> int:
    o = options if options is not None else default_options()
    return int(lib().stmg_footprint_bytes(ctypes.byref(problem), ctypes.byref(o)))


def _host_i64(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.int64)


STMG_NOALLOC_MAX_BATCH = 65536


def batched_lu(A, a_off, m_of, piv, p_off, info=None, prec=None, noalloc=False, config=None):
    """Factor a batch of row-major matrices of mixed sizes in place (device
    tensors A (float64/float32) and piv (int32); host offsets and sizes).
    prec: None (from the dtype of A), or STMG_F32_BF16 / STMG_F32_F16 for
    float32 A with 16-bit operands in the trailing-update MFMA.  noalloc:
    call stmg_batched_lu_noalloc (metadata staged in the library's fixed
    per-device array, batch <= STMG_NOALLOC_MAX_BATCH).  config: (wg_per_cu,
    [nb per size class], threads) for stmg_batched_lu_config (wg_per_cu 0 =
    one launch per size class; threads 256 or 512, default 256)."""
    import numpy as np
    ao, po = _host_i64(a_off), _host_i64(p_off)
    mo = np.ascontiguousarray(m_of, dtype=np.int32)
    if prec is None:
        prec = STMG_F64 if A.dtype == torch.float64 else STMG_F32
    elif (prec == STMG_F64) != (A.dtype == torch.float64):
        raise StmgError("prec does not match the dtype of A")
    ip = _ptr(info) if info is not None else None
    if config is not None:
        nbc = np.ascontiguousarray(config[1] if config[0] else [16] * 5, dtype=np.int32)
        threads = int(config[2]) if len(config) > 2 else 256
        rc = lib().stmg_batched_lu_config(prec, _ptr(A), ao.ctypes.data, mo.ctypes.data, len(mo), _ptr(piv),
                                          po.ctypes.data, ip, int(config[0]), threads, nbc.ctypes.data,
                                          _stream_ptr())
    else:
        f = lib().stmg_batched_lu_noalloc if noalloc else lib().stmg_batched_lu
        rc = f(prec, _ptr(A), ao.ctypes.data, mo.ctypes.data, len(mo), _ptr(piv), po.ctypes.data, ip,
               _stream_ptr())
    if rc != 0:
        raise StmgError(f"stmg_batched_lu{'_noalloc' if noalloc else ''} failed ({rc})")


def batched_lu_solve(LU, a_off, m_of, piv, p_off, b, b_off):
    """Solve with the factors of batched_lu; b (device) is overwritten."""
    import numpy as np
    ao, po, bo = _host_i64(a_off), _host_i64(p_off), _host_i64(b_off)
    mo = np.ascontiguousarray(m_of, dtype=np.int32)
    prec = STMG_F64 if LU.dtype == torch.float64 else STMG_F32
    rc = lib().stmg_batched_lu_solve(prec, _ptr(LU), ao.ctypes.data, mo.ctypes.data, len(mo), _ptr(piv),
                                     po.ctypes.data, _ptr(b), bo.ctypes.data, _stream_ptr())
    if rc != 0:
        raise StmgError(f"stmg_batched_lu_solve failed ({rc})")


def serve(requests, options: Options | None = None, slots: int = 4, hbm_budget: int = 0):
    """Run a request stream through the library's serving loop.

    requests: list of dicts with keys dim, n, r, k, nu, tau, arrival_s and
    optional vertices, dirichlet_faces, v_prev (numpy, one time node),
    rhs (numpy, slab).  Returns (solutions, results, wall_s)."""
    import numpy as np
    o = options if options is not None else default_options()
    nreq = len(requests)
    arr = (Request * nreq)()
    keep, outs = [], []
    for i, q in enumerate(requests):
        p, vert = make_problem(q["dim"], q["n"], q["r"], q["k"], q["nu"], q["tau"], q.get("vertices"),
                               q.get("dirichlet_faces"))
        keep.append(vert)
        arr[i].prob = p
        arr[i].arrival_s = float(q.get("arrival_s", 0.0))
        for key in ("v_prev", "rhs", "u_init"):
            v = q.get(key)
            if v is not None:
                v = np.ascontiguousarray(v, dtype=np.float64)
                keep.append(v)
                setattr(arr[i], key, v.ctypes.data)
        from . import inputs as _I
        N = _I.sizes(q["dim"], q["n"], q["r"], q["k"])[2]
        out = np.zeros(N)
        outs.append(out)
        arr[i].u_out = out.ctypes.data
    res = (RequestResult * nreq)()
    wall = ctypes.c_double()
    rc = lib().stmg_serve(arr, nreq, ctypes.byref(o), slots, hbm_budget, res, ctypes.byref(wall))
    if rc < 0:
        raise StmgError(f"stmg_serve failed ({rc})")
    return outs, list(res), wall.value


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One slab of the space-time discretization on the current GPU."""

    def __init__(self, dim, n, r, k, nu, tau, vertices=None, dirichlet_faces=None, gamma1=10.0, gamma2=10.0,
                 options: Options | None = None, **opt_overrides):
        p, self._vert = make_problem(dim, n, r, k, nu, tau, vertices, dirichlet_faces, gamma1, gamma2)
        self.problem = p
        self.options = options if options is not None else default_options(**opt_overrides)
        # the whole device memory of the context: one torch buffer of the
        # footprint (torch stays the only allocator); kept alive with the context
        self.footprint = footprint_bytes(p, self.options)
        if self.footprint == 0:
            raise StmgError("stmg_footprint_bytes rejected the problem or options")
        self._workspace = torch.empty(self.footprint, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        rc = lib().stmg_create(ctypes.byref(p), ctypes.byref(self.options), _ptr(self._workspace), self.footprint,
                               _stream_ptr(), ctypes.byref(h))
        if rc != 0:
            raise StmgError(f"stmg_create failed with code {rc}")
        self._h = h
        nt, nv, npr = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        self._check(lib().stmg_sizes(h, ctypes.byref(nt), ctypes.byref(nv), ctypes.byref(npr)))
        self.N, self.Nv, self.Np = nt.value, nv.value, npr.value
        self.dim, self.r, self.k = dim, r, k

    def _check(self, rc):
        if rc < 0:
            msg = lib().stmg_last_error(self._h)
            raise StmgError(f"stmg call failed ({rc}): {msg.decode() if msg else ''}")
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().stmg_destroy(self._h)
            self._h = None
        self._workspace = None

    def workspace_used(self):
        """Bytes of the workspace the context laid out."""
        return int(lib().stmg_workspace_used(self._h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, dtype, n=None, name="vector"):
        n = self.N if n is None else n
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise StmgError(f"{name} must be a device tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
            raise StmgError(f"{name}: expected contiguous {dtype} with {n} entries, got {t.dtype} {tuple(t.shape)}")
        return _ptr(t)

    @staticmethod
    def _prec(dtype):
        if dtype == torch.float64:
            return STMG_F64
        if dtype == torch.float32:
            return STMG_F32
        raise StmgError("dtype must be float64 or float32")

    # ---- slab data and operators ----------------------------------------
    def set_slab_data(self, rhs=None, v_prev=None):
        pr = self._vec(rhs, torch.float64, name="rhs") if rhs is not None else None
        pv = self._vec(v_prev, torch.float64, self.Nv // (self.k + 1), "v_prev") if v_prev is not None else None
        self._check(lib().stmg_set_slab_data(self._h, pr, pv))

    def residual(self, u, out=None):
        out = torch.empty_like(u) if out is None else out
        self._check(lib().stmg_residual(self._h, self._vec(u, torch.float64, name="u"),
                                        self._vec(out, torch.float64, name="r")))
        return out

    def jacobian_vmult(self, u_state, x, out=None):
        out = torch.empty_like(x) if out is None else out
        dt = x.dtype
        self._check(lib().stmg_jacobian_vmult(self._h, self._prec(dt), self._vec(u_state, dt, name="u_state"),
                                              self._vec(x, dt, name="x"), self._vec(out, dt, name="y")))
        return out

    def jacobian_vmult_batched(self, u_state, x, out=None):
        nvec = x.shape[0]
        out = torch.empty_like(x) if out is None else out
        dt = x.dtype
        if x.shape != (nvec, self.N) or not x.is_contiguous():
            raise StmgError("x must be (nvec, N) contiguous")
        self._check(lib().stmg_jacobian_vmult_batched(self._h, self._prec(dt), self._vec(u_state, dt, name="u_state"),
                                                      _ptr(x), _ptr(out), nvec))
        return out

    # ---- multigrid hierarchy, smoother, Krylov, Newton ----------------------
    @property
    def mg_dtype(self):
        return torch.float64 if self.options.prec_mg == STMG_F64 else torch.float32

    def num_levels(self):
        return lib().stmg_num_levels(self._h)

    def level_info(self, level):
        k, r, n, N = ctypes.c_int(), ctypes.c_int(), (ctypes.c_int * 3)(), ctypes.c_longlong()
        self._check(lib().stmg_level_info(self._h, level, ctypes.byref(k), ctypes.byref(r), n, ctypes.byref(N)))
        return k.value, r.value, tuple(n[: self.dim]), N.value

    def set_state(self, u):
        self._check(lib().stmg_set_state(self._h, self._vec(u, torch.float64, name="u_state")))

    def level_state(self, level):
        N = self.level_info(level)[3]
        out = torch.empty(N, dtype=torch.float64, device=torch.device("cuda"))
        self._check(lib().stmg_level_state(self._h, level, _ptr(out)))
        return out

    def smoother_rebuild(self, u):
        self._check(lib().stmg_smoother_rebuild(self._h, self._vec(u, torch.float64, name="u_state")))

    def level_jacobian_vmult(self, level, x, out=None):
        N = self.level_info(level)[3]
        out = torch.empty_like(x) if out is None else out
        self._check(lib().stmg_level_jacobian_vmult(self._h, level, self._prec(x.dtype), self._vec(x, x.dtype, N, "x"),
                                                    self._vec(out, x.dtype, N, "y")))
        return out

    def level_patch(self, level, cell):
        """The full space-time surrogate patch of one cell (m x m, row-major,
        multigrid precision) after smoother_rebuild."""
        k, r, n, _ = self.level_info(level)
        from math import comb
        m = (k + 1) * (self.dim * (r + 2) ** self.dim + comb(r + self.dim, self.dim))
        out = torch.empty(m * m, dtype=self.mg_dtype, device="cuda")
        self._check(lib().stmg_level_patch(self._h, level, cell, self.options.prec_mg, _ptr(out)))
        return out.view(m, m)

    def vanka_smooth(self, level, r, d, sweeps=1):
        N = self.level_info(level)[3]
        self._check(lib().stmg_vanka_smooth(self._h, level, self._prec(r.dtype), self._vec(r, r.dtype, N, "r"),
                                            self._vec(d, r.dtype, N, "d"), sweeps))
        return d

    def vcycle(self, r, out=None):
        out = torch.empty_like(r) if out is None else out
        self._check(lib().stmg_vcycle(self._h, self._prec(r.dtype), self._vec(r, r.dtype, name="r"),
                                      self._vec(out, r.dtype, name="d")))
        return out

    def prolongate(self, level, xc, out=None):
        Nf, Nc = self.level_info(level)[3], self.level_info(level + 1)[3]
        out = torch.empty(Nf, dtype=xc.dtype, device=xc.device) if out is None else out
        self._check(lib().stmg_prolongate(self._h, level, self._prec(xc.dtype), self._vec(xc, xc.dtype, Nc, "xc"),
                                          self._vec(out, xc.dtype, Nf, "yf")))
        return out

    def restrict(self, level, xf, out=None):
        Nf, Nc = self.level_info(level)[3], self.level_info(level + 1)[3]
        out = torch.empty(Nc, dtype=xf.dtype, device=xf.device) if out is None else out
        self._check(lib().stmg_restrict(self._h, level, self._prec(xf.dtype), self._vec(xf, xf.dtype, Nf, "xf"),
                                        self._vec(out, xf.dtype, Nc, "yc")))
        return out

    def fgmres(self, u_state, b, rtol, maxit=50):
        x = torch.empty_like(b)
        its = ctypes.c_int()
        hist = (ctypes.c_double * (maxit + 2))()
        rc = self._check(lib().stmg_fgmres(self._h, self._vec(u_state, torch.float64, name="u_state"),
                                           self._vec(b, torch.float64, name="b"), self._vec(x, torch.float64, name="x"),
                                           rtol, maxit, ctypes.byref(its), hist))
        return x, its.value, list(hist[: its.value + 1]), rc == 0

    def newton_solve(self, u):
        st = Stats()
        rc = self._check(lib().stmg_newton_gmres_solve(self._h, self._vec(u, torch.float64, name="u"),
                                                       ctypes.byref(st)))
        return u, st, rc

    def march(self, nslabs, rhs=None, v0=None, u=None):
        """stmg_march over `nslabs` slabs.  rhs: device (nslabs, N) FP64 or
        None; v0: device (Nv1,) or None; u: device (nslabs, N) whose first row
        is slab 0's initial guess (zeros if None).  Returns (u, stats, rc)."""
        N, nv1 = self.N, self.Nv // (self.k + 1)
        if u is None:
            u = torch.zeros((nslabs, N), dtype=torch.float64, device="cuda")
        if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous() or tuple(u.shape) != (nslabs, N):
            raise StmgError(f"u: expected contiguous float64 ({nslabs}, {N}) on the device")
        pr = None
        if rhs is not None:
            if rhs.dtype != torch.float64 or not rhs.is_cuda or not rhs.is_contiguous() or tuple(rhs.shape) != (nslabs, N):
                raise StmgError(f"rhs: expected contiguous float64 ({nslabs}, {N}) on the device")
            pr = _ptr(rhs)
        pv = self._vec(v0, torch.float64, nv1, "v0") if v0 is not None else None
        st = (Stats * max(nslabs, 1))()
        rc = self._check(lib().stmg_march(self._h, nslabs, pr, N, pv, _ptr(u), N, st))
        return u, list(st[:nslabs]), rc

    # ---- kernel timers -----------------------------------------------------
    def timing(self, on: bool = True):
        self._check(lib().stmg_timing_enable(self._h, 1 if on else 0))

    def timing_reset(self):
        self._check(lib().stmg_timing_reset(self._h))

    def timing_get(self, name: str):
        ms, cnt = ctypes.c_double(), ctypes.c_longlong()
        self._check(lib().stmg_timing_get(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def mass_vmult(self, x, out=None):
        out = torch.empty_like(x) if out is None else out
        dt = x.dtype
        self._check(lib().stmg_mass_vmult(self._h, self._prec(dt), self._vec(x, dt, name="x"),
                                          self._vec(out, dt, name="y")))
        return out
