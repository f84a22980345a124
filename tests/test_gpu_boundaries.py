"""GPU parity of Dirichlet boundaries (the boundary convective flux of the
surface integral, Sec. "DG-SEM in Space"; the exterior state g: Rusanov flux
with g, BR1 with u_hat = g and the interior viscous flux, the interior
penalty by Nitsche's terms) for the linear equations and Burgers, against
the oracle: residual, FP64 and FP32-inner JVP of every compiled (dim, N, Nt)
with boundaries on some axes, an element with both ends on the boundary, mid
sizes (tiled and ragged traversals), and slab solves (heat equation with
g = 0, inflow with g != 0, Burgers with inflow and outflow, with and without
the element-block preconditioner).  "Relative" as in gpu_common.rel."""
import sys

import numpy as np
import pytest

from gpu_common import Pair, cfg, check_fp32_jvp, gpu_jvp, gpu_residual, gpu_solve, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ops(orc, P, seed, label):
    U, up, V = P.random(seed)
    for dt in (0.02, 0.3):
        R, Ro = gpu_residual(P, U, up, dt), orc.residual(P.p, U, up, dt)
        J, Jo = gpu_jvp(P, U, V, dt), orc.jvp(P.p, U, dt, V)
        e = (rel(R, Ro), rel(J, Jo))
        check_fp32_jvp(gpu_jvp(P, U, V, dt, 1), Jo, lambda a, b: orc.jvp(P.p, a, dt, b), U, V, label)
        assert e[0] <= TOL and e[1] <= TOL, (label, dt, e)
    return e


@pytest.mark.parametrize("kind", ["adv", "advdiff", "sipg"])
def test_boundary_sweep(orc, kind):
    """Every (dim, N, Nt) with Dirichlet boundaries on some axes, g = 0.3."""
    layouts = {1: ([5], (1,)), 2: ([4, 3], (1, 0)), 3: ([2, 3, 2], (0, 1, 1))}
    for N in range(1, 6):
        for Nt in (2, 3, 4):
            for d in (1, 2, 3):
                if d == 3 and N > 4:
                    continue
                K, bc = layouts[d]
                c = cfg(kind, d, K, N, Nt, nu=0.02, bc=bc, bc_value=0.3)
                P = Pair(c)
                try:
                    e = _ops(orc, P, 10 * N + Nt + d, (kind, d, N, Nt))
                finally:
                    P.close()
        say(kind, "boundary sweep, last", e)


def test_boundary_both_ends_and_mid_sizes(orc):
    """One element between two boundaries (K = 1 on a Dirichlet axis), every
    axis a boundary, and larger meshes (a tiled 2D strip, a ragged one)."""
    cases = [cfg("sipg", 2, [1, 3], 3, 3, nu=0.05, bc=(1, 1), bc_value=-0.4),
             cfg("advdiff", 3, [2, 2, 2], 2, 2, nu=0.05, bc=(1, 1, 1), bc_value=0.2),
             cfg("adv", 2, [1, 1], 4, 4, bc=(1, 1), bc_value=1.1),
             cfg("advdiff", 2, [20, 6], 4, 4, nu=1e-3, bc=(1, 1), bc_value=0.5),
             cfg("sipg", 2, [23, 19], 3, 4, nu=1e-3, bc=(1, 0), bc_value=0.5)]
    for i, c in enumerate(cases):
        P = Pair(c)
        try:
            say("case", i, c["kind"], c["K"], c["bc"], _ops(orc, P, 40 + i, i))
        finally:
            P.close()


@pytest.mark.parametrize("kind", ["advdiff", "sipg"])
@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32inner"])
def test_boundary_slab_solves(orc, kind, fp32):
    """Heat-type problem on [0,1]^2 with g = 0 (sin(pi x) sin(pi y) data and
    a drift), and 1D advection with inflow g = 0.7: GPU solves match the
    oracle within 1e-9."""
    c = cfg(kind, 2, [6, 5], 3, 3, a=(0.3, -0.2), nu=0.05, bc=(1, 1), bc_value=0.0)
    P = Pair(c)
    try:
        X = P.coords()
        up = (np.sin(np.pi * X[:, 0, :]) * np.sin(np.pi * X[:, 1, :])).ravel()
        for k in range(3):
            U, un, s = gpu_solve(P, up, 0.05, 1e-12, inner_fp32=fp32)
            Uo, so = orc.solve(P.p, up, 0.05, tol=1e-13, dense_limit=0)
            e = rel(U, Uo)
            assert e <= 1e-9, (kind, k, e)
            up = un
        say(kind, "heat slabs", e)
    finally:
        P.close()
    c = cfg("adv", 1, [12], 3, 3, a=(1.0,), bc=(1,), bc_value=0.7)
    P = Pair(c)
    try:
        up = np.sin(2 * np.pi * P.coords()[:, 0, :]).ravel()
        U, un, s = gpu_solve(P, up, 1.0 / 24, 1e-12, inner_fp32=fp32)
        Uo, so = orc.solve(P.p, up, 1.0 / 24, tol=1e-13)
        assert rel(U, Uo) <= 1e-9
    finally:
        P.close()


def test_burgers_boundary_operators(orc):
    """Burgers with Dirichlet boundaries (g = 0.3), every compiled (N, Nt):
    residual and JVPs against the oracle; and one element between the two
    boundaries."""
    for N in range(1, 6):
        for Nt in (2, 3, 4):
            for K in (5, 1):
                P = Pair(cfg("burgers", 1, [K], N, Nt, bc=(1,), bc_value=0.3))
                try:
                    e = _ops(orc, P, 100 + 10 * N + Nt + K, ("burgers", K, N, Nt))
                finally:
                    P.close()
    say("burgers boundary sweep, last", e)


@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32inner"])
@pytest.mark.parametrize("precond", [0, 1], ids=["plain", "bjacobi"])
def test_burgers_boundary_slab_solves(orc, fp32, precond):
    """Burgers on [0, 1] with g = 0.5 at both ends (inflow on the left,
    outflow on the right for the positive data): four slabs one after
    another, each matching the oracle's solution within 1e-9."""
    P = Pair(cfg("burgers", 1, [24], 3, 3, bc=(1,), bc_value=0.5))
    try:
        X = P.coords()[:, 0, :]
        up = (0.5 + 0.2 * np.sin(2 * np.pi * X) + 0.1 * np.cos(6 * np.pi * X)).ravel()
        for k in range(4):
            U, un, s = gpu_solve(P, up, 0.01, 1e-12, inner_fp32=fp32, precond=precond)
            Uo, so = orc.solve(P.p, up, 0.01, tol=1e-13, dense_limit=0)
            e = rel(U, Uo)
            assert e <= 1e-9, (k, e)
            up = un
        say(f"burgers boundary slabs fp32={fp32} precond={precond}: {e:.2e}, gmres {s['gmres_its']}")
    finally:
        P.close()


def test_boundary_unsupported_cases():
    from paper_2201_05800_amd import st
    with pytest.raises(st.StError) as ei:
        st.st_create(st.mesh(2, [4, 4], [0, 0], [1, 1], bc=(1, 0)), 2, 3, st.equation(st.ST_EULER, gamma=1.4))
    assert ei.value.code == st.ST_ERR_UNSUPPORTED
    with pytest.raises(st.StError) as ei:
        st.st_create(st.mesh(2, [4, 4], [0, 0], [1, 1], bc=(1, 0)), 2, 3,
                     st.equation(st.ST_ADVDIFF_SIPG, nu=0.01, omega=4.0, center=(0.5, 0.5)))
    assert ei.value.code == st.ST_ERR_UNSUPPORTED
    with pytest.raises(st.StError) as ei:
        st.st_create(st.mesh(2, [4, 4], [0, 0], [1, 1], bc=(2, 0)), 2, 3, st.equation(st.ST_ADVECTION))
    assert ei.value.code == st.ST_ERR_BAD_ARG
