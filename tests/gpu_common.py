"""Shared helpers of the GPU tests: one problem description fed to both the
HIP library (through the C ABI binding) and the CPU oracle."""
from __future__ import annotations

import numpy as np

from paper_2201_05800_amd import inputs

KINDS = {"adv": 1, "advdiff": 2, "burgers": 3, "euler": 4, "ns": 5, "sipg": 6}


def cfg(kind, dim, K, N, Nt, lo=None, hi=None, a=(1.0, 0.5, -0.25), nu=0.01, gamma=1.4, mu=0.01, prandtl=0.71,
        omega=0.0, center=(0.0, 0.0, 0.0), bc=(0, 0, 0), bc_value=0.0):
    return dict(kind=KINDS[kind] if isinstance(kind, str) else kind, dim=dim, K=list(K), N=N, Nt=Nt,
                lo=lo or [0.0] * dim, hi=hi or [1.0] * dim, a=a, nu=nu, gamma=gamma, mu=mu, prandtl=prandtl,
                omega=omega, center=center, bc=tuple(bc), bc_value=bc_value)


class Pair:
    """The same slab problem on the GPU (libstdg) and in the oracle."""

    def __init__(self, c):
        import oracle
        from paper_2201_05800_amd import st
        self.c = c
        self.st, self.orc = st, oracle
        d = c["dim"]
        om, ce = c.get("omega", 0.0), c.get("center", (0.0, 0.0, 0.0))
        bc, g = c.get("bc", (0, 0, 0)), c.get("bc_value", 0.0)
        self.p = oracle.problem(d, c["K"], c["lo"], c["hi"], c["N"], c["Nt"], c["kind"], a=c["a"][:d],
                                nu=c["nu"], gamma=c["gamma"], mu=c["mu"], prandtl=c["prandtl"], omega=om,
                                center=ce, bc=bc, bc_value=g)
        self.h = st.st_create(st.mesh(d, c["K"], c["lo"], c["hi"], bc=bc), c["N"], c["Nt"],
                              st.equation(c["kind"], a=c["a"][:d], nu=c["nu"], gamma=c["gamma"], mu=c["mu"],
                                          prandtl=c["prandtl"], omega=om, center=ce, bc_value=g))
        self.n, self.nsp, self.nv = st.st_sizes(self.h)
        self.ns = (c["N"] + 1) ** d
        self.E = int(np.prod(c["K"]))
        assert self.n == oracle.slab_size(self.p)

    def close(self):
        self.st.st_destroy(self.h)

    def random(self, seed):
        return inputs.random_slab(self.c["kind"], self.c["dim"], self.E, self.nv, self.c["Nt"], self.ns, seed)

    def coords(self):
        return self.orc.node_coords(self.p)


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    """The larger of the relative 2-norm error ||a - b|| / ||b|| and the
    element-wise one max|a - b| / max|b|: a bound on it bounds both, so a
    defect confined to a few values cannot hide in the norm of a large
    vector."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    d = a - b
    e2 = np.linalg.norm(d) / (nb if nb > 0 else 1.0)
    emax = (np.abs(d).max() if d.size else 0.0) / (mb if mb > 0 else 1.0)
    return max(e2, emax)


JVP32_NORM_TOL = 2e-5     # relative 2-norm of an FP32-inner JVP against the FP64 oracle


def fp32_elementwise_bound(jvp_fn, U, V, Jo):
    """Element-wise bound for an FP32-inner JVP (FP32 state, FP32 arithmetic
    and accumulation) against the FP64 value Jo = jvp_fn(U, V).  The JVP of
    the nonlinear equations cancels strongly at single nodes, so the bound is
    derived from the conditioning rather than from |Jo|: 64 times the largest
    change of the oracle's JVP when U and V are rounded to FP32 (the input
    rounding alone; FP32 arithmetic over a few dozen terms per value adds a
    similar amount per term), and at least 2e-5 max|Jo|."""
    U32 = np.asarray(U, dtype=np.float32).astype(np.float64)
    V32 = np.asarray(V, dtype=np.float32).astype(np.float64)
    sens = np.abs(jvp_fn(U32, V32) - Jo).max()
    return max(64.0 * sens, JVP32_NORM_TOL * np.abs(Jo).max())


def check_fp32_jvp(J32, Jo, jvp_fn, U, V, label=""):
    """FP32-inner JVP parity: relative 2-norm <= 2e-5 and every value within
    fp32_elementwise_bound.  Returns (2-norm error, max error / bound)."""
    J32, Jo = np.asarray(J32), np.asarray(Jo)
    e2 = np.linalg.norm(J32 - Jo) / max(np.linalg.norm(Jo), 1e-300)
    b = fp32_elementwise_bound(jvp_fn, U, V, Jo)
    em = np.abs(J32 - Jo).max()
    assert e2 <= JVP32_NORM_TOL, (label, e2)
    assert em <= b, (label, em, b)
    return e2, em / b


def gpu_residual(P: Pair, U, up, dt):
    import torch
    Ud, upd = dev(U), dev(up)
    R = torch.empty_like(Ud)
    P.st.st_residual(P.h, Ud, upd, 0.0, dt, R)
    return host(R)


def gpu_jvp(P: Pair, U, V, dt, fp32=0):
    import torch
    Ud, Vd = dev(U), dev(V)
    J = torch.empty_like(Vd)
    P.st.st_jvp(P.h, Ud, 0.0, dt, Vd, J, fp32)
    return host(J)


def gpu_solve(P: Pair, up, dt, tol, **opts):
    import torch
    upd = dev(up)
    U = torch.empty(P.n, dtype=torch.float64, device="cuda")
    un = torch.empty(P.nsp, dtype=torch.float64, device="cuda")
    o = P.st.st_default_opts(**opts)
    stats = P.st.st_solve_slab(P.h, upd, 0.0, dt, tol, o, U, un)
    return host(U), host(un), stats
