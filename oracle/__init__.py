"""CPU FP64 oracle for the space-time DG-SEM slab system (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product package never does.
The arithmetic lives in ``oracle.cpp`` (see its header for the formulations
and the readings of the paper it takes).  Build it with ``build()`` (plain
g++ with OpenMP); nothing here depends on the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ADVECTION, ADVDIFF_BR1, BURGERS, EULER, NS_BR1, ADVDIFF_SIPG = 1, 2, 3, 4, 5, 6
FORM_DG, FORM_RK, FORM_GALERKIN = 0, 1, 2


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("K", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("N", ctypes.c_int),
        ("Nt", ctypes.c_int),
        ("eq", ctypes.c_int),
        ("a", ctypes.c_double * 3),
        ("nu", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("react", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("center", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 3),
        ("bc_value", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("newton_its", ctypes.c_int),
        ("linear_its", ctypes.c_int),
        ("res0", ctypes.c_double),
        ("res_final", ctypes.c_double),
        ("converged", ctypes.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (-O2, OpenMP)."""
    src = os.path.join(HERE, "oracle.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", src, "-o", LIB_PATH]
        subprocess.check_call(cmd)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_nvars.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_slab_size.argtypes = [P]
        L.orc_slab_size.restype = ctypes.c_long
        L.orc_space_size.argtypes = [P]
        L.orc_space_size.restype = ctypes.c_long
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_lgl.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_butcher_from_sbp.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_butcher_appendix_b.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_node_coords.argtypes = [P, dp]
        L.orc_spatial_op.argtypes = [P, dp, dp]
        L.orc_spatial_jvp.argtypes = [P, dp, dp, dp]
        L.orc_num_flux.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
        L.orc_flux.argtypes = [P, ctypes.c_int, dp, dp, dp]
        L.orc_residual.argtypes = [P, ctypes.c_int, dp, dp, ctypes.c_double, dp]
        L.orc_jvp.argtypes = [P, ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.orc_solve.argtypes = [P, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Stats)]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def nvars(eq: int, dim: int) -> int:
    return lib().orc_nvars(eq, dim)


def problem(dim, K, lo, hi, N, Nt, eq, a=(0.0, 0.0, 0.0), nu=0.0, gamma=1.4, mu=0.0,
            prandtl=0.72, react=0.0, omega=0.0, center=(0.0, 0.0, 0.0), bc=(0, 0, 0),
            bc_value=0.0) -> Problem:
    """omega, center: the advection velocity a + omega e_z x (x - center) (2D);
    bc[a]: 0 periodic, 1 Dirichlet with exterior state bc_value."""
    p = Problem()
    p.dim = dim
    for i in range(3):
        p.K[i] = int(K[i]) if i < dim else 1
        p.lo[i] = float(lo[i]) if i < dim else 0.0
        p.hi[i] = float(hi[i]) if i < dim else 1.0
        p.a[i] = float(a[i]) if i < len(a) else 0.0
        p.center[i] = float(center[i]) if i < len(center) else 0.0
        p.bc[i] = int(bc[i]) if i < len(bc) and i < dim else 0
    p.N, p.Nt, p.eq = N, Nt, eq
    p.nu, p.gamma, p.mu, p.prandtl, p.react = nu, gamma, mu, prandtl, react
    p.omega, p.bc_value = float(omega), float(bc_value)
    return p


def slab_size(p) -> int:
    return lib().orc_slab_size(ctypes.byref(p))


def space_size(p) -> int:
    return lib().orc_space_size(ctypes.byref(p))


def set_threads(n: int) -> None:
    lib().orc_set_threads(n)


def get_threads() -> int:
    return lib().orc_get_threads()


def lgl(n: int):
    x, w, D = np.zeros(n), np.zeros(n), np.zeros((n, n))
    lib().orc_lgl(n, _p(x), _p(w), _p(D))
    return x, w, D


def butcher_from_sbp(Nt: int):
    A, b, c = np.zeros((Nt, Nt)), np.zeros(Nt), np.zeros(Nt)
    lib().orc_butcher_from_sbp(Nt, _p(A), _p(b), _p(c))
    return A, b, c


def butcher_appendix_b(Nt: int):
    A, b, c = np.zeros((Nt, Nt)), np.zeros(Nt), np.zeros(Nt)
    if lib().orc_butcher_appendix_b(Nt, _p(A), _p(b), _p(c)) != 0:
        raise ValueError("Appendix B lists Nt = 2, 3, 4 only")
    return A, b, c


def node_coords(p) -> np.ndarray:
    """Physical node coordinates, shape (E, dim, ns)."""
    ns = (p.N + 1) ** p.dim
    E = int(np.prod([p.K[i] for i in range(p.dim)]))
    X = np.zeros((E, p.dim, ns))
    lib().orc_node_coords(ctypes.byref(p), _p(X))
    return X


def spatial_op(p, u) -> np.ndarray:
    u = _c(u)
    F = np.zeros_like(u)
    lib().orc_spatial_op(ctypes.byref(p), _p(u), _p(F))
    return F


def spatial_jvp(p, u, v) -> np.ndarray:
    u, v = _c(u), _c(v)
    J = np.zeros_like(u)
    lib().orc_spatial_jvp(ctypes.byref(p), _p(u), _p(v), _p(J))
    return J


def num_flux(p, axis, uL, uR, qL=None, qR=None) -> np.ndarray:
    uL, uR = _c(uL), _c(uR)
    H = np.zeros_like(uL)
    qLa = _c(qL) if qL is not None else None
    qRa = _c(qR) if qR is not None else None
    lib().orc_num_flux(ctypes.byref(p), axis, _p(uL), _p(uR),
                       _p(qLa) if qLa is not None else None,
                       _p(qRa) if qRa is not None else None, _p(H))
    return H


def flux(p, axis, u, q=None) -> np.ndarray:
    u = _c(u)
    f = np.zeros_like(u)
    qa = _c(q) if q is not None else None
    lib().orc_flux(ctypes.byref(p), axis, _p(u), _p(qa) if qa is not None else None, _p(f))
    return f


def residual(p, U, uprev, dt, form=FORM_DG) -> np.ndarray:
    U, uprev = _c(U), _c(uprev)
    R = np.zeros_like(U)
    lib().orc_residual(ctypes.byref(p), form, _p(U), _p(uprev), float(dt), _p(R))
    return R


def jvp(p, U, dt, V, form=FORM_DG) -> np.ndarray:
    U, V = _c(U), _c(V)
    JV = np.zeros_like(U)
    lib().orc_jvp(ctypes.byref(p), form, _p(U), float(dt), _p(V), _p(JV))
    return JV


def solve(p, uprev, dt, tol=1e-13, form=FORM_DG, max_newton=30, dense_limit=1500):
    """Newton solve of one slab; returns (U, stats dict)."""
    uprev = _c(uprev)
    U = np.zeros(slab_size(p))
    st = Stats()
    rc = lib().orc_solve(ctypes.byref(p), form, _p(uprev), float(dt), float(tol), max_newton,
                         dense_limit, _p(U), ctypes.byref(st))
    return U, dict(rc=rc, newton_its=st.newton_its, linear_its=st.linear_its, res0=st.res0,
                   res_final=st.res_final, converged=bool(st.converged))


def last_time_node(p, U) -> np.ndarray:
    """u^{Nt} = (e_Nt^T (x) I) U, eq. (un), in the spatial layout [E][nv][ns]."""
    nv = nvars(p.eq, p.dim)
    ns = (p.N + 1) ** p.dim
    return np.ascontiguousarray(np.asarray(U).reshape(-1, nv, p.Nt, ns)[:, :, -1, :]).reshape(-1)


# ---------------------------------------------------------------------------
# Embedded error estimate (Sec. "Algorithmic Aspects", adaptive time-stepping;
# eqs. RK_stage_equations and RK_solution).  The embedded solution is to be
# one order below u^{n+1} (order 2 Nt - 2), with the strategy of the Radau IIA
# code the paper cites (Hairer-Wanner IV.8): besides the stage derivatives
# K_l = F(U_l) the embedded formula may use the derivative at the known start
# value, K_0 = F(u^n) (an explicit stage at c = 0), with weight gamma_0:
#     u_hat = u^n + dt (gamma_0 F(u^n) + sum_l b_hat_l K_l).
# Weights taken (reading of the paper; proofs in the pins):
#   Nt = 2: gamma_0 = 0, b_hat = (1, 0)            order 1 = 2 Nt - 3
#   Nt > 2: gamma_0 = b_1, b_hat = (0, b_2 .. b_Nt) order Nt
# i.e. for Nt > 2 the embedded formula is the Lobatto quadrature with the first
# stage derivative replaced by the one at u^n.  Nt = 3 gives order 3 = 2 Nt - 3.
# For Nt = 4 no such formula has order 5: the quadrature conditions up to
# degree 4 on the four distinct nodes fix the summed weight at c = 0 to b_1,
# which leaves only gamma_0, and every gamma_0 != 0 fails the order-5 tree
# conditions (Lobatto IIIC has stage order Nt - 1 = 3, so U_1 - u^n = O(dt^4));
# order 4 is the highest reachable.
# ---------------------------------------------------------------------------
EMBEDDED_ORDER = {2: 1, 3: 3, 4: 4}


def embedded_weights(Nt: int):
    """(A, b, c, gamma0, b_hat): the Appendix B tableau and the embedded
    weights (gamma0 on F(u^n), b_hat on the stage derivatives)."""
    A, b, c = butcher_appendix_b(Nt)
    bh = np.zeros(Nt)
    if Nt == 2:
        gamma0 = 0.0
        bh[0] = 1.0
    else:
        gamma0 = float(b[0])
        bh[1:] = b[1:]
    return A, b, c, gamma0, bh


def stage_derivatives(p, U, uprev):
    """dt K_l from the stage equations, dt K = (A^-1 (x) I)(U - 1 (x) u^n)
    (eq. RK_stage_equations with the Appendix B tableau); shape (E, nv, Nt, ns)."""
    nv = nvars(p.eq, p.dim)
    ns = (p.N + 1) ** p.dim
    A, _, _ = butcher_appendix_b(p.Nt)
    Us = np.asarray(U, dtype=np.float64).reshape(-1, nv, p.Nt, ns)
    un = np.asarray(uprev, dtype=np.float64).reshape(-1, nv, ns)
    return np.einsum("lj,evjs->evls", np.linalg.inv(A), Us - un[:, :, None, :])


def error_estimate(p, U, uprev, dt, atol, rtol):
    """Local error estimate of a solved slab: e = u^{n+1} - u_hat with
    u^{n+1} = u^n + dt sum_l b_l K_l (eq. RK_solution) and u_hat as above,
    formed from the weight differences,
        e = dt sum_l (b_l - b_hat_l) K_l - gamma_0 dt F(u^n),
    (the difference of the two solutions would lose the digits e has below
    |u|).  F is the oracle's spatial operator.  The scalar is the root mean
    square over every spatial node and variable of
    e / (atol + rtol max(|u^n|, |u^{n+1}|)).  Returns (err, e) with e in the
    spatial layout [E][nv][ns]."""
    nv = nvars(p.eq, p.dim)
    ns = (p.N + 1) ** p.dim
    _, b, _, gamma0, bh = embedded_weights(p.Nt)
    un = np.asarray(uprev, dtype=np.float64).reshape(-1, nv, ns)
    hK = stage_derivatives(p, U, uprev)
    # u^{n+1} for the scale: the slab's last time node (eq. un); Lobatto IIIC
    # is stiffly accurate, so it equals u^n + dt sum_l b_l K_l -- up to
    # rounding, which a pure relative scale (atol = 0) magnifies where the
    # state crosses zero
    u1 = last_time_node(p, U).reshape(un.shape)
    e = np.einsum("l,evls->evs", b - bh, hK)
    if gamma0 != 0.0:
        e = e - gamma0 * dt * spatial_op(p, un.ravel()).reshape(un.shape)
    sc = atol + rtol * np.maximum(np.abs(un), np.abs(u1))
    err = float(np.sqrt(np.mean((e / sc) ** 2)))
    return err, e.reshape(-1)


def error_scale_terms(p, U, uprev, dt):
    """The magnitudes the estimate is formed from, per spatial value:
    sum_l |b_l - b_hat_l| |dt K_l| + |gamma_0| |dt F(u^n)|.  Rounding in
    forming e is relative to these, not to |e| (for small steps e is the
    small difference of two stage derivatives)."""
    nv = nvars(p.eq, p.dim)
    ns = (p.N + 1) ** p.dim
    _, b, _, gamma0, bh = embedded_weights(p.Nt)
    un = np.asarray(uprev, dtype=np.float64).reshape(-1, nv, ns)
    s = np.einsum("l,evls->evs", np.abs(b - bh), np.abs(stage_derivatives(p, U, uprev)))
    if gamma0 != 0.0:
        s = s + abs(gamma0) * dt * np.abs(spatial_op(p, un.ravel()).reshape(un.shape))
    return s.reshape(-1)


# ---------------------------------------------------------------------------
# Several time elements in one system (Sec. "Merits": solving for several time
# steps at once; Sec. "Adaptive Mesh Refinement": one system of several
# coupled time elements).  Slab m covers [t0 + m dt, t0 + (m+1) dt]; the
# vector holds the slabs one after another, each in the single-slab layout.
# The upwind trace at tau = -1 of slab m (eq. upwind_flux) is the last time
# node of slab m - 1; slab 0's is u^n.
# ---------------------------------------------------------------------------
def inflow_term(p, w) -> np.ndarray:
    """How the inflow state w enters a slab residual: -(B_tau (x) I) U* with
    B_tau = diag(-1, 0, ..., 0, 1) and U*(tau = -1) = w (eq. DG_in_time) puts
    +w at the first time node and nothing elsewhere."""
    nv = nvars(p.eq, p.dim)
    ns = (p.N + 1) ** p.dim
    out = np.zeros((slab_size(p) // (nv * p.Nt * ns), nv, p.Nt, ns))
    out[:, :, 0, :] = np.asarray(w, dtype=np.float64).reshape(-1, nv, ns)
    return out.reshape(-1)


def residual_slabs(p, U, uprev, dt, M) -> np.ndarray:
    """Residual of M coupled slabs: slab m's residual with its inflow taken
    from the last time node of slab m - 1."""
    Us = np.asarray(U, dtype=np.float64).reshape(M, -1)
    out, inflow = [], np.asarray(uprev, dtype=np.float64)
    for m in range(M):
        out.append(residual(p, Us[m], inflow, dt))
        inflow = last_time_node(p, Us[m])
    return np.concatenate(out)


def jvp_slabs(p, U, dt, V, M) -> np.ndarray:
    """Jacobian of residual_slabs times V: block lower bidiagonal, the slab
    Jacobians on the diagonal and the inflow dependence below them."""
    Us = np.asarray(U, dtype=np.float64).reshape(M, -1)
    Vs = np.asarray(V, dtype=np.float64).reshape(M, -1)
    out = []
    for m in range(M):
        j = jvp(p, Us[m], dt, Vs[m])
        if m > 0:
            j = j + inflow_term(p, last_time_node(p, Vs[m - 1]))
        out.append(j)
    return np.concatenate(out)


def solve_slabs(p, uprev, dt, M, tol=1e-13):
    """Solution of the M-slab system.  The Jacobian is block lower triangular
    and slab m depends on the earlier slabs only through its inflow, so the
    system is solved exactly by forward substitution: one slab solve after
    another, each taking the previous slab's last time node as inflow."""
    out, inflow = [], np.asarray(uprev, dtype=np.float64)
    for _ in range(M):
        U, st = solve(p, inflow, dt, tol=tol)
        if not st["converged"]:
            raise RuntimeError(f"oracle slab solve did not converge: {st}")
        out.append(U)
        inflow = last_time_node(p, U)
    return np.concatenate(out)
