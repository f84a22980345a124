"""GPU parity of the multi-slab system (several coupled time elements in one
system): st_residual_slabs, st_jvp_slabs and st_solve_slabs through the C ABI
against the oracle's residual_slabs, jvp_slabs and solve_slabs.

Bars as for one slab: residual and FP64 JVP within 1e-12 relative, FP32-inner
JVP within the FP32 bound, solved systems within 1e-9 relative.
"""
import sys

import numpy as np
import pytest

from gpu_common import Pair, cfg, check_fp32_jvp, dev, host, rel
from test_gpu_parity import JVP_TOL, RES_TOL, SLAB_TOL, initial
from paper_2201_05800_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def slab_inputs(P, M, seed):
    U, up, V = inputs.random_slab(P.c["kind"], P.c["dim"], P.E * M, P.nv, P.c["Nt"], P.ns, seed)
    return U, up[: P.nsp], V


OPS = [
    ("adv1d", cfg("adv", 1, [7], 3, 3, a=(1.0,))),
    ("advdiff2d", cfg("advdiff", 2, [5, 3], 4, 4, nu=0.01)),
    ("burgers1d", cfg("burgers", 1, [9], 2, 4)),
    ("euler2d", cfg("euler", 2, [3, 4], 3, 3)),
    ("euler3d", cfg("euler", 3, [2, 3, 2], 2, 3)),
    ("ns3d", cfg("ns", 3, [2, 2, 3], 3, 2, mu=0.02)),
    # many blocks per slab, ragged tails
    ("advdiff2d-mid", cfg("advdiff", 2, [23, 19], 4, 4, nu=1e-3)),
    ("euler2d-mid", cfg("euler", 2, [29, 21], 3, 3, lo=[-5, -5], hi=[5, 5])),
]


@pytest.mark.parametrize("name,c", OPS, ids=[o[0] for o in OPS])
@pytest.mark.parametrize("M", [1, 2, 5])
def test_coupled_operator_parity(orc, name, c, M):
    import torch
    P = Pair(c)
    try:
        say("slabs operator", name, "M", M)
        U, up, V = slab_inputs(P, M, seed=70 + M)
        dt = 0.04
        Ud, upd, Vd = dev(U), dev(up), dev(V)
        R = torch.empty_like(Ud)
        P.st.st_residual_slabs(P.h, M, Ud, upd, 0.0, dt, R)
        Ro = orc.residual_slabs(P.p, U, up, dt, M)
        J = torch.empty_like(Vd)
        P.st.st_jvp_slabs(P.h, M, Ud, 0.0, dt, Vd, J, 0)
        Jo = orc.jvp_slabs(P.p, U, dt, V, M)
        J32 = torch.empty_like(Vd)
        P.st.st_jvp_slabs(P.h, M, Ud, 0.0, dt, Vd, J32, 1)
        e = (rel(host(R), Ro), rel(host(J), Jo),
             check_fp32_jvp(host(J32), Jo, lambda a, b: orc.jvp_slabs(P.p, a, dt, b, M), U, V, M)[0])
        say(f"  rel errors residual {e[0]:.2e} jvp {e[1]:.2e} jvp32 {e[2]:.2e}")
        assert e[0] <= RES_TOL and e[1] <= JVP_TOL, e
        if M == 1:
            # the single-slab entry points are the M = 1 system
            R1 = torch.empty_like(Ud)
            P.st.st_residual(P.h, Ud, upd, 0.0, dt, R1)
            J1 = torch.empty_like(Vd)
            P.st.st_jvp(P.h, Ud, 0.0, dt, Vd, J1, 0)
            assert np.array_equal(host(R1), host(R)) and np.array_equal(host(J1), host(J))
    finally:
        P.close()


SOLVES = [
    ("adv1d", cfg("adv", 1, [9], 2, 3, a=(1.0,)), 1.0 / 32, "burgers", 4),
    ("advdiff2d", cfg("advdiff", 2, [12, 10], 4, 4, a=(1.0, 0.5), nu=1e-3), 1.0 / 128, "fourier", 3),
    ("burgers1d", cfg("burgers", 1, [48], 3, 3), 0.01, "burgers", 3),
    ("euler2d-vortex", cfg("euler", 2, [12, 12], 3, 3, lo=[-5, -5], hi=[5, 5]), 0.1, "vortex", 2),
    # the viscous pass per slab (its Q / dQ arrays at the slab's offset)
    ("ns3d-tgv", cfg("ns", 3, [3, 3, 3], 3, 3, lo=[0, 0, 0], hi=[6.283185307179586] * 3, mu=1.0 / 1600), 0.05,
     "tgv", 2),
    ("euler3d-bubble", cfg("euler", 3, [4, 4, 4], 2, 3), 0.05, "bubble", 2),
]


@pytest.mark.parametrize("name,c,dt,init,M", SOLVES, ids=[s[0] for s in SOLVES])
@pytest.mark.parametrize("mode", ["fp64", "fp32inner", "precond", "precond_sweep"])
def test_coupled_solve_parity(orc, name, c, dt, init, M, mode):
    """The coupled M-slab solve against the oracle's slab-by-slab solution
    (precond: element-block Jacobi slab by slab; precond_sweep: the same
    blocks with forward substitution over the slabs)."""
    import torch
    P = Pair(c)
    try:
        up = initial(P, init)
        say("slabs solve", name, mode, "M", M, "dt", dt)
        pc = {"precond": 1, "precond_sweep": 2}.get(mode, 0)
        o = P.st.st_default_opts(inner_fp32=1 if mode == "fp32inner" else 0, precond=pc, max_newton=60)
        U = torch.empty(P.n * M, dtype=torch.float64, device="cuda")
        un = torch.empty(P.nsp, dtype=torch.float64, device="cuda")
        st = P.st.st_solve_slabs(P.h, M, dev(up), 0.0, dt, 1e-12, o, U, un)
        Uo = orc.solve_slabs(P.p, up, dt, M, tol=1e-12)
        e = rel(host(U), Uo)
        eu = rel(host(un), orc.last_time_node(P.p, Uo[-P.n:]))
        say(f"  rel err {e:.2e} (u_next {eu:.2e}), outer {st['newton_its']}, gmres {st['gmres_its']}")
        assert e <= SLAB_TOL and eu <= SLAB_TOL
    finally:
        P.close()


@pytest.mark.parametrize("name,c,dt,init", [
    ("advdiff2d", cfg("advdiff", 2, [12, 10], 4, 4, a=(1.0, 0.5), nu=1e-3), 1.0 / 128, "fourier"),
    ("burgers1d", cfg("burgers", 1, [48], 3, 3), 0.01, "burgers"),
], ids=["advdiff2d", "burgers1d"])
def test_sweep_cuts_iterations(orc, name, c, dt, init):
    """Eight coupled slabs: forward substitution over the slabs takes fewer
    GMRES iterations than the slab-by-slab blocks, and both reach the
    oracle's solution."""
    import torch
    P = Pair(c)
    M = 8
    try:
        up = initial(P, init)
        Uo = orc.solve_slabs(P.p, up, dt, M, tol=1e-12)
        its = {}
        for pc in (1, 2):
            o = P.st.st_default_opts(precond=pc, max_newton=60)
            U = torch.empty(P.n * M, dtype=torch.float64, device="cuda")
            un = torch.empty(P.nsp, dtype=torch.float64, device="cuda")
            st = P.st.st_solve_slabs(P.h, M, dev(up), 0.0, dt, 1e-12, o, U, un)
            its[pc] = st["gmres_its"]
            e = rel(host(U), Uo)
            say(f"sweep {name} precond {pc}: rel err {e:.2e}, outer {st['newton_its']}, gmres {st['gmres_its']}")
            assert e <= SLAB_TOL
        assert its[2] < its[1], its
    finally:
        P.close()


def test_buffers_grow_and_shrink(orc):
    """Solves with M = 4, then 1, then 2 on one handle: every result matches
    the oracle (the buffers are regrown for 4 slabs and then reused)."""
    import torch
    c = cfg("burgers", 1, [16], 3, 3)
    P = Pair(c)
    try:
        up = initial(P, "burgers")
        dt = 0.01
        for M in (4, 1, 2):
            say("grow/shrink M", M)
            U = torch.empty(P.n * M, dtype=torch.float64, device="cuda")
            un = torch.empty(P.nsp, dtype=torch.float64, device="cuda")
            if M == 1:
                P.st.st_solve_slab(P.h, dev(up), 0.0, dt, 1e-12, P.st.st_default_opts(), U, un)
            else:
                P.st.st_solve_slabs(P.h, M, dev(up), 0.0, dt, 1e-12, P.st.st_default_opts(), U, un)
            assert rel(host(U), orc.solve_slabs(P.p, up, dt, M, tol=1e-13)) <= SLAB_TOL
    finally:
        P.close()


def test_slab_count_validation():
    import torch
    P = Pair(cfg("adv", 1, [4], 2, 2, a=(1.0,)))
    try:
        x = torch.zeros(P.n * 2, dtype=torch.float64, device="cuda")
        up = torch.zeros(P.nsp, dtype=torch.float64, device="cuda")
        for M in (0, -1, 65):
            with pytest.raises(P.st.StError) as ei:
                P.st.st_residual_slabs(P.h, M, x, up, 0.0, 0.1, x)
            assert ei.value.code == -1
            with pytest.raises(P.st.StError):
                P.st.st_jvp_slabs(P.h, M, x, 0.0, 0.1, x, x, 0)
            with pytest.raises(P.st.StError):
                P.st.st_solve_slabs(P.h, M, up, 0.0, 0.1, 1e-10)
    finally:
        P.close()
