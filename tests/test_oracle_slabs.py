"""Pins of the oracle's multi-slab system (several coupled time elements in one
system, Sec. "Merits" and Sec. "Adaptive Mesh Refinement").

What fixes it independently of its own code:
* the inflow enters a slab residual exactly as the oracle's slab residual
  depends on u^n (that residual is pinned against the paper elsewhere);
* for the linear equations the coupled residual is affine, so its difference
  quotient is the coupled JVP to rounding (a wrong slab index, node or sign
  in the coupling fails it);
* the coupled Jacobian, assembled column by column, is block lower
  bidiagonal;
* Newton on the coupled system as one system (dense Jacobian, brute force on
  tiny sizes) reaches the forward-substitution solution.
"""
import numpy as np
import pytest

from paper_2201_05800_amd import inputs
from test_oracle_pins import CASES, make


def _inputs(orc, name, M, seed):
    p, E, nv, ns, Nt = make(orc, name)
    U, up, V = inputs.random_slab(p.eq, p.dim, E * M, nv, Nt, ns, seed)
    return p, U, up[: E * nv * ns], V


@pytest.mark.parametrize("name", ["adv1", "advdiff2", "burgers1", "euler2", "ns2"])
def test_inflow_term_is_residual_dependence(orc, name):
    p, U, up, V = _inputs(orc, name, 1, seed=31)
    w = np.asarray(inputs.rng(32).standard_normal(up.size))
    dt = 0.06
    d = orc.residual(p, U, up + w, dt) - orc.residual(p, U, up, dt)
    t = orc.inflow_term(p, w)
    assert np.abs(d - t).max() <= 1e-13 * max(1.0, np.abs(orc.residual(p, U, up, dt)).max())
    # only the first time node sees the inflow
    nv, ns = orc.nvars(p.eq, p.dim), (p.N + 1) ** p.dim
    assert not t.reshape(-1, nv, p.Nt, ns)[:, :, 1:, :].any()


@pytest.mark.parametrize("name", ["adv1", "adv2", "advdiff2"])
@pytest.mark.parametrize("M", [2, 3])
def test_linear_coupled_residual_is_affine(orc, name, M):
    p, U, up, V = _inputs(orc, name, M, seed=40 + M)
    dt = 0.08
    d = orc.residual_slabs(p, U + V, up, dt, M) - orc.residual_slabs(p, U, up, dt, M)
    J = orc.jvp_slabs(p, U, dt, V, M)
    assert np.abs(d - J).max() <= 1e-12 * np.abs(J).max()


@pytest.mark.parametrize("name", ["burgers1", "euler2", "ns2"])
def test_coupled_jvp_central_difference(orc, name):
    M = 3
    p, U, up, V = _inputs(orc, name, M, seed=50)
    dt = 0.05
    e = 1e-5
    fd = (orc.residual_slabs(p, U + e * V, up, dt, M) - orc.residual_slabs(p, U - e * V, up, dt, M)) / (2 * e)
    J = orc.jvp_slabs(p, U, dt, V, M)
    assert np.abs(fd - J).max() < 1e-7 * np.abs(J).max()


@pytest.mark.parametrize("name", ["adv1", "burgers1", "euler1"])
def test_coupled_jacobian_block_lower_bidiagonal(orc, name):
    M = 3
    p, U, up, _ = _inputs(orc, name, M, seed=60)
    n = orc.slab_size(p)
    N = n * M
    J = np.stack([orc.jvp_slabs(p, U, 0.07, np.eye(N)[k], M) for k in range(N)], axis=1)
    for a in range(M):
        for b in range(M):
            blk = J[a * n:(a + 1) * n, b * n:(b + 1) * n]
            if b == a:
                assert np.abs(blk - np.stack([orc.jvp(p, U[a * n:(a + 1) * n], 0.07, np.eye(n)[k])
                                              for k in range(n)], axis=1)).max() == 0.0
            elif b == a - 1:
                # unit weight from the last time node of b to the first of a
                nv, ns = orc.nvars(p.eq, p.dim), (p.N + 1) ** p.dim
                idx = np.arange(n).reshape(-1, nv, p.Nt, ns)
                C = np.zeros((n, n))
                C[idx[:, :, 0, :].ravel(), idx[:, :, -1, :].ravel()] = 1.0
                assert np.array_equal(blk, C)
            else:
                assert not blk.any()


@pytest.mark.parametrize("name", ["adv1", "burgers1", "euler1"])
def test_coupled_newton_reaches_forward_substitution(orc, name):
    """Newton on the whole M-slab system (dense Jacobian from jvp_slabs) from
    1 (x) u^n in every slab ends at the slab-by-slab solution."""
    M = 3
    p, E, nv, ns, Nt = make(orc, name)
    if p.eq == orc.EULER:
        X = orc.node_coords(p)
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * X[:, 0, :])
        up = inputs.euler_conservative(rho, [0.5 + 0 * rho], 1.0 + 0 * rho, 1.4).ravel()
    else:
        _, up, _ = inputs.random_slab(p.eq, p.dim, E, nv, Nt, ns, seed=7)
        if p.eq == orc.BURGERS:
            up = 0.5 + 0.1 * (up - 0.5)
    dt = 0.05
    n = orc.slab_size(p)
    N = n * M
    ref = orc.solve_slabs(p, up, dt, M, tol=1e-14)
    assert np.linalg.norm(orc.residual_slabs(p, ref, up, dt, M)) <= 1e-12 * max(1.0, np.linalg.norm(up))
    U = np.tile(np.repeat(up.reshape(E, nv, 1, ns), Nt, axis=2).ravel(), M)
    for _ in range(30):
        R = orc.residual_slabs(p, U, up, dt, M)
        if np.linalg.norm(R) <= 1e-13 * max(1.0, np.linalg.norm(up)):
            break
        J = np.stack([orc.jvp_slabs(p, U, dt, np.eye(N)[k], M) for k in range(N)], axis=1)
        U = U - np.linalg.solve(J, R)
    assert np.linalg.norm(U - ref) <= 1e-11 * np.linalg.norm(ref)
