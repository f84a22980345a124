"""GPU tests of the handle's descriptor reuse: st_residual and st_jvp skip
re-writing an operator descriptor that already holds the same bytes from a
call on the same stream.  Calls that share, change and reallocate those slots
are interleaved on one handle -- residuals and JVPs at other buffers, both
JVP forms, an embedded error estimate (which writes the residual's slots with
a one-time-level operator), a slab solve, a second stream, multi-slab calls
that grow the slab capacity -- and every repeated call must give the first
call's result bit for bit, and the first call must match the oracle.
"""
import sys

import numpy as np
import pytest

from gpu_common import Pair, cfg, dev, host, rel

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = {
    "euler2d": lambda: cfg("euler", 2, [6, 5], 3, 3, lo=[-5.0, -5.0], hi=[5.0, 5.0]),
    "ns3d": lambda: cfg("ns", 3, [3, 3, 2], 2, 3),
    "advdiff2d": lambda: cfg("advdiff", 2, [5, 4], 3, 3),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", list(CASES))
def test_descriptor_reuse(case):
    import torch

    import oracle as orc
    from paper_2201_05800_amd import st
    P = Pair(CASES[case]())
    say(f"descriptor reuse: {case}")
    try:
        dt = 0.02
        U1, up1, V1 = P.random(11)
        U2, up2, V2 = P.random(12)
        dU1, dup1, dV1 = dev(U1), dev(up1), dev(V1)
        dU2, dup2, dV2 = dev(U2), dev(up2), dev(V2)
        out = torch.empty(P.n, dtype=torch.float64, device="cuda")

        def res(U, up):
            st.st_residual(P.h, U, up, 0.0, dt, out)
            return host(out).copy()

        def jvp(U, V, fp32=0):
            st.st_jvp(P.h, U, 0.0, dt, V, out, fp32)
            return host(out).copy()

        R1, J1, J1f = res(dU1, dup1), jvp(dU1, dV1), jvp(dU1, dV1, 1)
        e = (rel(R1, orc.residual(P.p, U1, up1, dt)), rel(J1, orc.jvp(P.p, U1, dt, V1)))
        say(f"  first calls against the oracle: residual {e[0]:.2e} jvp {e[1]:.2e}")
        assert max(e) <= TOL, e

        def same(label, got, want):
            assert np.array_equal(got, want), (case, label, float(np.abs(got - want).max()))

        same("residual again", res(dU1, dup1), R1)
        same("jvp again", jvp(dU1, dV1), J1)
        R2 = res(dU2, dup2)
        assert not np.array_equal(R2, R1)
        same("residual after another residual", res(dU1, dup1), R1)
        same("jvp after the FP32-inner form", (jvp(dU1, dV1, 1), jvp(dU1, dV1))[1], J1)
        same("FP32-inner jvp after the FP64 form", jvp(dU1, dV1, 1), J1f)
        same("jvp after another direction", (jvp(dU1, dV2), jvp(dU1, dV1))[1], J1)

        # the estimate writes the residual's descriptor slots (Nt > 2)
        st.st_error_estimate(P.h, dU1, dup1, 0.0, dt, 1e-6, 1e-6)
        same("residual after an error estimate", res(dU1, dup1), R1)

        # a slab solve (its own descriptor slots, and the state buffers)
        o = st.st_default_opts(restart=20, max_newton=30)
        st.st_solve_slab(P.h, dup1, 0.0, dt, 1e-8, o, check=False)
        same("residual after a solve", res(dU1, dup1), R1)
        same("jvp after a solve", jvp(dU1, dV1), J1)

        # the same call on a second stream
        s2 = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s2):
            st.st_residual(P.h, dU1, dup1, 0.0, dt, out, s2)
        s2.synchronize()
        same("residual on a second stream", host(out).copy(), R1)
        same("residual back on the first stream", res(dU1, dup1), R1)

        # new values behind the same pointers
        dU1.copy_(dU2)
        dup1.copy_(dup2)
        same("residual of changed buffer contents", res(dU1, dup1), R2)
        dU1.copy_(dev(U1))
        dup1.copy_(dev(up1))

        # multi-slab calls that grow the slab capacity (reallocation)
        for M in (2, 4, 2):
            UM = dev(np.concatenate([U1] * M))
            RM = torch.empty(M * P.n, dtype=torch.float64, device="cuda")
            st.st_residual_slabs(P.h, M, UM, dup1, 0.0, dt, RM)
            rm = host(RM)
            want = orc.residual_slabs(P.p, np.concatenate([U1] * M), up1, dt, M)
            assert rel(rm, want) <= TOL, (case, M, rel(rm, want))
            del UM, RM
        same("residual after capacity growth", res(dU1, dup1), R1)
        same("jvp after capacity growth", jvp(dU1, dV1), J1)
    finally:
        P.close()
