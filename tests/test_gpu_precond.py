"""Element-block Jacobi right preconditioning of the slab GMRES: the
preconditioned solve reaches the oracle's slab solution (the same system, so
the same solution within the slab tolerance) in fewer Arnoldi steps, in FP64
and with FP32-inner JVPs -- the linear equations with their exact element
block, the nonlinear ones with the block of the Jacobian at the mean state;
element blocks above 1024 unknowns reject it, and so does the server for
Euler and Navier-Stokes (it preconditions the scalar equations)."""
import sys

import numpy as np
import pytest

from gpu_common import Pair, cfg, gpu_solve, rel
from paper_2201_05800_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fourier_init(P):
    X = P.coords()
    return inputs.fourier_modes(X, inputs.fourier_params(2, dim=P.c["dim"])).ravel()


CASES = [
    # C2 shape on a smaller periodic box with the same h, dt, N, Nt
    ("advdiff2d-16", cfg("advdiff", 2, [16, 16], 4, 4, hi=[0.25, 0.25], a=(1.0, 0.5), nu=1e-3), 1.0 / 128),
    # ragged sizes, other degrees
    ("advdiff2d-11x7-N3Nt3", cfg("advdiff", 2, [11, 7], 3, 3, a=(1.0, 0.5), nu=1e-3), 1.0 / 40),
    # 1D advection (C1 shape)
    ("adv1d-16", cfg("adv", 1, [16], 3, 3, a=(1.0,)), 1.0 / 32),
    # 3D, 500 unknowns per element (the 8-element-per-block kernel)
    ("advdiff3d-4x3x5-N4Nt4", cfg("advdiff", 3, [4, 3, 5], 4, 4, a=(1.0, 0.5, -0.25), nu=1e-3), 1.0 / 64),
]


@pytest.mark.parametrize("name,c,dt", CASES, ids=[x[0] for x in CASES])
@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32inner"])
def test_preconditioned_solve_matches_oracle(orc, name, c, dt, fp32):
    P = Pair(c)
    try:
        up = fourier_init(P) if c["dim"] > 1 else np.sin(2 * np.pi * P.coords()[:, 0, :]).ravel()
        tol = 1e-11
        say(f"[{name} fp32={fp32}] preconditioned and plain solves, n={P.n}")
        U1, un1, s1 = gpu_solve(P, up, dt, tol, inner_fp32=fp32, precond=1)
        U0, un0, s0 = gpu_solve(P, up, dt, tol, inner_fp32=fp32, precond=0)
        Uo, so = orc.solve(P.p, up, dt, tol=1e-13, dense_limit=0)
        e1, e0 = rel(U1, Uo), rel(U0, Uo)
        say(f"  precond: outer {s1['newton_its']} gmres {s1['gmres_its']} err {e1:.2e};  "
            f"plain: outer {s0['newton_its']} gmres {s0['gmres_its']} err {e0:.2e}")
        assert e1 <= 1e-9 and e0 <= 1e-9
        # the oracle's residual of the preconditioned solution meets the tolerance
        rn = np.linalg.norm(orc.residual(P.p, U1, up, dt))
        assert rn <= 1.01 * tol * max(1.0, s1["res0"])
        assert s1["gmres_its"] * 2 <= s0["gmres_its"], "preconditioning should cut the Arnoldi steps"
        assert np.array_equal(un1, U1.reshape(P.E, P.nv, c["Nt"], P.ns)[:, :, -1, :].ravel())
    finally:
        P.close()


NONLIN = [
    ("burgers1d-48", cfg("burgers", 1, [48], 3, 3), "burgers"),
    ("euler2d-vortex-12", cfg("euler", 2, [12, 12], 3, 3, lo=[-5, -5], hi=[5, 5]), "vortex"),
    ("ns3d-tgv-3-N2Nt2", cfg("ns", 3, [3, 3, 3], 2, 2, lo=[0, 0, 0], hi=[6.283185307179586] * 3, mu=1.0 / 1600),
     "tgv"),
    # the 3D Navier-Stokes workload's element: 5 * 3 * 4^3 = 960 unknowns
    # (row groups of the matrix-core kernel, LDS above 64 KB)
    ("ns3d-tgv-3-N3Nt3", cfg("ns", 3, [3, 3, 3], 3, 3, lo=[0, 0, 0], hi=[6.283185307179586] * 3, mu=1.0 / 1600),
     "tgv"),
    # 5 * 2 * 4^3 = 640 unknowns: three row groups of the large-block kernel
    ("ns3d-tgv-3-N3Nt2", cfg("ns", 3, [3, 3, 3], 3, 2, lo=[0, 0, 0], hi=[6.283185307179586] * 3, mu=1.0 / 1600),
     "tgv"),
    # 960 unknowns, 48 elements: a full group of 32 elements and a ragged one
    ("euler3d-tgv-4x4x3-N3Nt3", cfg("euler", 3, [4, 4, 3], 3, 3, lo=[0, 0, 0], hi=[6.283185307179586] * 3), "tgv"),
]


def nonlin_init(P, kind):
    X = P.coords()
    if kind == "vortex":
        return inputs.isentropic_vortex(X, seed=3).ravel()
    if kind == "burgers":
        return inputs.burgers_smooth(X, inputs.burgers_params(4)).ravel()
    return inputs.taylor_green(X).ravel()


@pytest.mark.parametrize("name,c,init", NONLIN, ids=[x[0] for x in NONLIN])
@pytest.mark.parametrize("fp32", [0, 1], ids=["fp64", "fp32inner"])
def test_preconditioned_nonlinear_solve_matches_oracle(orc, name, c, init, fp32):
    P = Pair(c)
    try:
        up = nonlin_init(P, init)
        h = min((c["hi"][a] - c["lo"][a]) / c["K"][a] for a in range(c["dim"]))
        if init == "vortex":
            lam = inputs.euler_max_speed(up.reshape(P.E, P.nv, P.ns), c["gamma"])
        elif init == "burgers":
            lam = np.abs(up).max()
        else:
            lam = None
        dt = 0.05 if lam is None else inputs.cfl_dt(5.0, h, c["N"], lam)
        tol = 1e-11
        say(f"[{name} fp32={fp32}] preconditioned and plain solves, n={P.n}, dt={dt:.4g}")
        U1, un1, s1 = gpu_solve(P, up, dt, tol, inner_fp32=fp32, precond=1)
        U0, un0, s0 = gpu_solve(P, up, dt, tol, inner_fp32=fp32, precond=0)
        Uo, so = orc.solve(P.p, up, dt, tol=1e-13, dense_limit=0)
        e1, e0 = rel(U1, Uo), rel(U0, Uo)
        say(f"  precond: outer {s1['newton_its']} gmres {s1['gmres_its']} err {e1:.2e};  "
            f"plain: outer {s0['newton_its']} gmres {s0['gmres_its']} err {e0:.2e}")
        assert e1 <= 1e-9 and e0 <= 1e-9
        rn = np.linalg.norm(orc.residual(P.p, U1, up, dt))
        assert rn <= 1.01 * tol * max(1.0, s1["res0"])
        assert s1["gmres_its"] < s0["gmres_its"], "preconditioning should cut the Arnoldi steps"
    finally:
        P.close()


def test_preconditioned_solve_is_deterministic_and_reuses_the_block():
    P = Pair(cfg("advdiff", 2, [16, 16], 4, 4, hi=[0.25, 0.25], a=(1.0, 0.5), nu=1e-3))
    try:
        up = fourier_init(P)
        a = gpu_solve(P, up, 1.0 / 128, 1e-10, precond=1)
        b = gpu_solve(P, up, 1.0 / 128, 1e-10, precond=1)      # block cached for this dt
        c = gpu_solve(P, up, 1.0 / 256, 1e-10, precond=1)      # new dt: block rebuilt
        d = gpu_solve(P, up, 1.0 / 128, 1e-10, precond=1)      # back: rebuilt again
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], d[0])
        assert not np.array_equal(a[0], c[0])
    finally:
        P.close()


def test_nonlinear_block_follows_the_mean_state():
    """The nonlinear block is assembled at the mean of u_prev: a solve on the
    same handle with another mean state rebuilds it, so it runs exactly as on
    a fresh handle (bitwise), and the same mean state reuses it."""
    c = cfg("burgers", 1, [48], 3, 3)
    P, Q = Pair(c), Pair(c)
    try:
        up1 = nonlin_init(P, "burgers")
        up2 = up1 + 0.3
        dt = 0.01
        gpu_solve(P, up1, dt, 1e-11, precond=1)
        a = gpu_solve(P, up2, dt, 1e-11, precond=1)       # new mean: rebuilt
        b = gpu_solve(Q, up2, dt, 1e-11, precond=1)       # fresh handle
        assert np.array_equal(a[0], b[0])
        assert a[2]["gmres_its"] == b[2]["gmres_its"]
        c2 = gpu_solve(P, up2, dt, 1e-11, precond=1)      # same mean: reused
        assert np.array_equal(a[0], c2[0])
    finally:
        P.close()
        Q.close()


def test_adaptive_reorthogonalisation_keeps_cycles_short(orc):
    """Four consecutive preconditioned slabs of the 16x16 advection-diffusion
    box (N = 4, Nt = 4, dt = 1/128): the block Jacobi converges within a
    dozen Arnoldi steps, where the once-projected vector's norm cancels.  The
    adaptive form repeats the projection there (as CGS2 does everywhere), so
    each slab takes one GMRES cycle, like CGS2; every slab matches the
    oracle."""
    P = Pair(cfg("advdiff", 2, [16, 16], 4, 4, a=(1.0, 0.5), nu=1e-3))
    dt = 1.0 / 128
    try:
        u0 = fourier_init(P)
        its = {}
        for cgs in (2, 0):
            u = u0
            its[cgs] = []
            for i in range(4):
                U, un, st = gpu_solve(P, u, dt, 1e-10, precond=1, cgs_passes=cgs)
                its[cgs].append((st["newton_its"], st["gmres_its"]))
                if cgs == 0:
                    Uo, _ = orc.solve(P.p, u, dt, tol=1e-12, dense_limit=4000)
                    e = rel(U, Uo)
                    say(f"adaptive slab {i}: rel err {e:.2e}")
                    assert e <= 1e-9
                u = un
        say("GMRES (outer, steps) per slab:", its)
        for a, b in zip(its[0], its[2]):
            assert a[0] <= b[0] + 1 and a[1] <= 2 * b[1], its
    finally:
        P.close()


def test_preconditioning_rejected_where_unavailable():
    from paper_2201_05800_amd import st
    # an element block of 5 * 2 * 5^3 = 1250 unknowns is above the limit
    P = Pair(cfg("ns", 3, [2, 2, 2], 4, 2, lo=[0, 0, 0], hi=[6.283185307179586] * 3, mu=1.0 / 1600))
    try:
        up = inputs.taylor_green(P.coords()).ravel()
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, up, 0.05, 1e-10, precond=1)
        assert ei.value.code == st.ST_ERR_UNSUPPORTED
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, up, 0.05, 1e-10, precond=2)
        assert ei.value.code == st.ST_ERR_UNSUPPORTED
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, up, 0.05, 1e-10, precond=3)
        assert ei.value.code == st.ST_ERR_BAD_ARG
    finally:
        P.close()
    # the server preconditions the scalar equations only
    srv = st.st_server_create(hbm_budget_bytes=1 << 28, max_active=2)
    try:
        c = cfg("euler", 2, [8, 8], 2, 3)
        d = c["dim"]
        r = st.request(st.mesh(d, c["K"], c["lo"], c["hi"]), c["N"], c["Nt"], st.equation(c["kind"], gamma=1.4),
                       np.ones(64 * 9 * 4), 0.0, 0.01, 1e-10, st.st_default_opts(precond=1))
        with pytest.raises(st.StError) as ei:
            st.st_submit(srv, r)
        assert ei.value.code == st.ST_ERR_UNSUPPORTED
    finally:
        st.st_server_destroy(srv)
