"""Shared helpers of the GPU tests: one problem description fed to both the
HIP library (through the C ABI binding) and the CPU oracle."""
from __future__ import annotations

import numpy as np

from paper_2201_05800_amd import inputs

KINDS = {"adv": 1, "advdiff": 2, "burgers": 3, "euler": 4, "ns": 5}


def cfg(kind, dim, K, N, Nt, lo=None, hi=None, a=(1.0, 0.5, -0.25), nu=0.01, gamma=1.4, mu=0.01, prandtl=0.71):
    return dict(kind=KINDS[kind] if isinstance(kind, str) else kind, dim=dim, K=list(K), N=N, Nt=Nt,
                lo=lo or [0.0] * dim, hi=hi or [1.0] * dim, a=a, nu=nu, gamma=gamma, mu=mu, prandtl=prandtl)


class Pair:
    """The same slab problem on the GPU (libstdg) and in the oracle."""

    def __init__(self, c):
        import oracle
        from paper_2201_05800_amd import st
        self.c = c
        self.st, self.orc = st, oracle
        d = c["dim"]
        self.p = oracle.problem(d, c["K"], c["lo"], c["hi"], c["N"], c["Nt"], c["kind"], a=c["a"][:d],
                                nu=c["nu"], gamma=c["gamma"], mu=c["mu"], prandtl=c["prandtl"])
        self.h = st.st_create(st.mesh(d, c["K"], c["lo"], c["hi"]), c["N"], c["Nt"],
                              st.equation(c["kind"], a=c["a"][:d], nu=c["nu"], gamma=c["gamma"], mu=c["mu"],
                                          prandtl=c["prandtl"]))
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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


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
