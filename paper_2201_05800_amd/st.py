"""ctypes binding of libstdg.so (include/st.h): the same names, argument
marshalling only.  Device buffers are torch CUDA tensors (float64,
contiguous); streams are torch.cuda.Stream objects or raw hipStream_t ints.
Every compute step runs in the library's HIP kernels; if the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstdg.so")

ST_OK = 0
ST_PENDING = 1
ST_ERR_BAD_ARG = -1
ST_ERR_HIP = -2
ST_ERR_NONFINITE = -3
ST_ERR_NO_CONVERGENCE = -4
ST_ERR_OOM_ADMISSION = -5
ST_ERR_UNSUPPORTED = -6
ST_ERR_NOT_FOUND = -7
ST_ERR_CANCELLED = -8

ST_ADVECTION, ST_ADVDIFF_BR1, ST_BURGERS, ST_EULER, ST_NS_BR1, ST_ADVDIFF_SIPG = 1, 2, 3, 4, 5, 6
ST_K_RESIDUAL, ST_K_JVP, ST_K_GRAD, ST_K_MULTIDOT, ST_K_UPDATE, ST_K_NORMALIZE, ST_K_NEWTON, ST_K_PRECOND = range(8)
KERNEL_CLASSES = ("residual", "jvp", "grad", "multidot", "update", "normalize", "newton", "precond")

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("K", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3)]


class Equation(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("a", ctypes.c_double * 3), ("nu", ctypes.c_double),
                ("gamma", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("omega", ctypes.c_double), ("center", ctypes.c_double * 3), ("bc_value", ctypes.c_double)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_newton", ctypes.c_int), ("cgs_passes", ctypes.c_int),
                ("inner_fp32", ctypes.c_int), ("gmres_rtol", ctypes.c_double), ("timing", ctypes.c_int),
                ("precond", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("gmres_its", ctypes.c_int), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("usec", ctypes.c_double), ("status", ctypes.c_int),
                ("kernel_us", ctypes.c_double * 8), ("kernel_calls", ctypes.c_int * 8),
                ("kernel_bytes", ctypes.c_double * 8)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int), ("device", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", Mesh), ("N", ctypes.c_int), ("Nt", ctypes.c_int), ("eq", Equation),
                ("u_prev", _c_double_p), ("t0", ctypes.c_double), ("dt", ctypes.c_double),
                ("tol", ctypes.c_double), ("opts", SolverOpts)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("u_next", _c_double_p), ("stats", Stats),
                ("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class StError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes) of every entry point declared in include/st.h
_SIGS = [
    ("st_version", ctypes.c_char_p, []),
    ("st_last_error", ctypes.c_char_p, []),
    ("st_default_opts", None, [ctypes.POINTER(SolverOpts)]),
    ("st_lgl", ctypes.c_int, [ctypes.c_int, _c_double_p, _c_double_p, _c_double_p]),
    ("st_create", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.c_int, ctypes.POINTER(Equation),
                                 ctypes.POINTER(ctypes.c_void_p)]),
    ("st_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("st_sizes", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int)]),
    ("st_node_coords", ctypes.c_int, [ctypes.c_void_p, _c_double_p]),
    ("st_residual", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("st_jvp", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    ("st_solve_slab", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(SolverOpts), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.POINTER(Stats), ctypes.c_void_p]),
    ("st_residual_slabs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("st_jvp_slabs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p]),
    ("st_solve_slabs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.POINTER(SolverOpts),
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Stats), ctypes.c_void_p]),
    ("st_error_estimate", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_double_p,
                                         ctypes.c_void_p]),
    ("st_next_dt", ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, _c_double_p]),
    ("st_residual_noalloc", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(Equation), ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("st_server_create", ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]),
    ("st_server_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("st_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    ("st_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Result)]),
    ("st_cancel", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    ("st_server_stats", ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 5),
    ("st_request_footprint", ctypes.c_int64, [ctypes.POINTER(Request)]),
]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        # torch ships its own HIP runtime with the same soname (libamdhip64.so.7)
        # as the system one libstdg links; load torch first so that the process
        # holds exactly one HIP runtime, the one torch's allocations live in
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def symbols():
    return [s[0] for s in _SIGS]


def st_last_error() -> str:
    return lib().st_last_error().decode()


def st_version() -> str:
    return lib().st_version().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise StError(rc, st_last_error())
    return rc


def _dev(t, name="tensor"):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(s):
    if s is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return ctypes.c_void_p(s)
    return ctypes.c_void_p(s.cuda_stream)


def mesh(dim, K, lo, hi, bc=(0, 0, 0)) -> Mesh:
    m = Mesh()
    m.dim = dim
    for a in range(3):
        m.K[a] = int(K[a]) if a < dim else 1
        m.lo[a] = float(lo[a]) if a < dim else 0.0
        m.hi[a] = float(hi[a]) if a < dim else 1.0
        m.bc[a] = int(bc[a]) if a < dim and a < len(bc) else 0
    return m


def equation(kind, a=(0.0, 0.0, 0.0), nu=0.0, gamma=1.4, mu=0.0, prandtl=0.72, omega=0.0,
             center=(0.0, 0.0, 0.0), bc_value=0.0) -> Equation:
    e = Equation()
    e.kind = kind
    for i in range(3):
        e.a[i] = float(a[i]) if i < len(a) else 0.0
        e.center[i] = float(center[i]) if i < len(center) else 0.0
    e.nu, e.gamma, e.mu, e.prandtl = nu, gamma, mu, prandtl
    e.omega = float(omega)
    e.bc_value = float(bc_value)
    return e


def st_default_opts(**over) -> SolverOpts:
    o = SolverOpts()
    lib().st_default_opts(ctypes.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o


def st_lgl(n: int):
    x, w, D = np.zeros(n), np.zeros(n), np.zeros((n, n))
    _check(lib().st_lgl(n, x.ctypes.data_as(_c_double_p), w.ctypes.data_as(_c_double_p),
                        D.ctypes.data_as(_c_double_p)))
    return x, w, D


def st_create(m: Mesh, N: int, Nt: int, eq: Equation) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().st_create(ctypes.byref(m), N, Nt, ctypes.byref(eq), ctypes.byref(h)))
    return h


def st_destroy(h) -> None:
    _check(lib().st_destroy(h))


def st_sizes(h):
    n, ns, nv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
    _check(lib().st_sizes(h, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(nv)))
    return n.value, ns.value, nv.value


def st_node_coords(h, dim: int, ns_per_elem: int) -> np.ndarray:
    n_space = st_sizes(h)[1]
    nv = st_sizes(h)[2]
    E = n_space // (nv * ns_per_elem)
    X = np.zeros((E, dim, ns_per_elem))
    _check(lib().st_node_coords(h, X.ctypes.data_as(_c_double_p)))
    return X


def st_residual(h, U, u_prev, t0, dt, R, stream=None) -> None:
    _check(lib().st_residual(h, _dev(U, "U"), _dev(u_prev, "u_prev"), float(t0), float(dt), _dev(R, "R"),
                             _stream(stream)))


def st_jvp(h, U, t0, dt, v, Jv, inner_fp32=0, stream=None) -> None:
    _check(lib().st_jvp(h, _dev(U, "U"), float(t0), float(dt), _dev(v, "v"), _dev(Jv, "Jv"), int(inner_fp32),
                        _stream(stream)))


def st_residual_noalloc(mesh_, N, Nt, eq, U, u_prev, t0, dt, R, stream=None) -> None:
    _check(lib().st_residual_noalloc(ctypes.byref(mesh_), int(N), int(Nt), ctypes.byref(eq), _dev(U, "U"),
                                     _dev(u_prev, "u_prev"), float(t0), float(dt), _dev(R, "R"), _stream(stream)))


def st_residual_slabs(h, M, U, u_prev, t0, dt, R, stream=None) -> None:
    _check(lib().st_residual_slabs(h, int(M), _dev(U, "U"), _dev(u_prev, "u_prev"), float(t0), float(dt),
                                   _dev(R, "R"), _stream(stream)))


def st_jvp_slabs(h, M, U, t0, dt, v, Jv, inner_fp32=0, stream=None) -> None:
    _check(lib().st_jvp_slabs(h, int(M), _dev(U, "U"), float(t0), float(dt), _dev(v, "v"), _dev(Jv, "Jv"),
                              int(inner_fp32), _stream(stream)))


def st_error_estimate(h, U, u_prev, t0, dt, atol, rtol, stream=None) -> float:
    err = ctypes.c_double(0.0)
    _check(lib().st_error_estimate(h, _dev(U, "U"), _dev(u_prev, "u_prev"), float(t0), float(dt), float(atol),
                                   float(rtol), ctypes.byref(err), _stream(stream)))
    return err.value


def st_next_dt(Nt, dt, err) -> float:
    out = ctypes.c_double(0.0)
    _check(lib().st_next_dt(int(Nt), float(dt), float(err), ctypes.byref(out)))
    return out.value


def st_solve_slab(h, u_prev, t0, dt, tol, opts=None, U_out=None, u_next=None, stream=None, check=True):
    st = Stats()
    rc = lib().st_solve_slab(h, _dev(u_prev, "u_prev"), float(t0), float(dt), float(tol),
                             ctypes.byref(opts) if opts is not None else None, _dev(U_out, "U_out"),
                             _dev(u_next, "u_next"), ctypes.byref(st), _stream(stream))
    return _solve_result(rc, st, check)


def st_solve_slabs(h, M, u_prev, t0, dt, tol, opts=None, U_out=None, u_next=None, stream=None, check=True):
    st = Stats()
    rc = lib().st_solve_slabs(h, int(M), _dev(u_prev, "u_prev"), float(t0), float(dt), float(tol),
                              ctypes.byref(opts) if opts is not None else None, _dev(U_out, "U_out"),
                              _dev(u_next, "u_next"), ctypes.byref(st), _stream(stream))
    return _solve_result(rc, st, check)


def _solve_result(rc, st, check):
    out = dict(rc=rc, newton_its=st.newton_its, gmres_its=st.gmres_its, res0=st.res0, res_final=st.res_final,
               usec=st.usec, status=st.status, kernel_us=list(st.kernel_us), kernel_calls=list(st.kernel_calls),
               kernel_bytes=list(st.kernel_bytes))
    if check:
        _check(rc)
    return out


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
def st_server_create(hbm_budget_bytes: int, max_active: int = 64, device: int = 0):
    o = ServerOpts()
    o.hbm_budget_bytes, o.max_active, o.device = int(hbm_budget_bytes), int(max_active), int(device)
    s = ctypes.c_void_p()
    _check(lib().st_server_create(ctypes.byref(o), ctypes.byref(s)))
    return s


def st_server_destroy(s) -> None:
    _check(lib().st_server_destroy(s))


def request(m: Mesh, N: int, Nt: int, eq: Equation, u_prev: np.ndarray, t0: float, dt: float, tol: float,
            opts: SolverOpts | None = None):
    """Build an st_request_t; keeps a reference to the host array in the result."""
    r = Request()
    r.mesh, r.N, r.Nt, r.eq = m, N, Nt, eq
    arr = np.ascontiguousarray(u_prev, dtype=np.float64)
    r.u_prev = arr.ctypes.data_as(_c_double_p)
    r.t0, r.dt, r.tol = float(t0), float(dt), float(tol)
    r.opts = opts if opts is not None else st_default_opts()
    r._keep = arr
    return r


def st_request_footprint(req: Request) -> int:
    return int(lib().st_request_footprint(ctypes.byref(req)))


def st_submit(s, req: Request) -> int:
    t = ctypes.c_uint64()
    _check(lib().st_submit(s, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def st_poll(s, ticket: int, u_next_out: np.ndarray):
    """Returns (rc, result dict); rc = ST_PENDING while running."""
    res = Result()
    res.u_next = u_next_out.ctypes.data_as(_c_double_p)
    rc = lib().st_poll(s, ctypes.c_uint64(ticket), ctypes.byref(res))
    if rc == ST_ERR_NOT_FOUND:
        _check(rc)
    st = res.stats
    return rc, dict(status=res.status, newton_its=st.newton_its, gmres_its=st.gmres_its, res0=st.res0,
                    res_final=st.res_final, submit_us=res.submit_us, admit_us=res.admit_us,
                    done_us=res.done_us)


def st_cancel(s, ticket: int) -> None:
    _check(lib().st_cancel(s, ctypes.c_uint64(ticket)))


def st_server_stats(s):
    vals = [ctypes.c_int64() for _ in range(5)]
    _check(lib().st_server_stats(s, *[ctypes.byref(v) for v in vals]))
    return dict(zip(("queued", "active", "completed", "ticks", "bytes_in_use"), [v.value for v in vals]))
