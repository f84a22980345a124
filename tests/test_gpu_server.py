"""Serving (continuous batching) on the GPU: every result equals the oracle's
slab solution, is bitwise the same alone and in a mix, and the admission,
cancellation and failure paths behave."""
import sys
import time

import numpy as np
import pytest

from gpu_common import Pair, cfg, gpu_solve, rel
from paper_2201_05800_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_req(st, c, up, dt, tol=1e-11, **o):
    d = c["dim"]
    m = st.mesh(d, c["K"], c["lo"], c["hi"], bc=c.get("bc", (0, 0, 0)))
    eq = st.equation(c["kind"], a=c["a"][:d], nu=c["nu"], gamma=c["gamma"], mu=c["mu"], prandtl=c["prandtl"],
                     bc_value=c.get("bc_value", 0.0))
    return st.request(m, c["N"], c["Nt"], eq, up, 0.0, dt, tol, st.st_default_opts(**o))


def wait_all(st, srv, tickets, sizes, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, nsp in zip(tickets, sizes):
            if t in out:
                continue
            buf = np.zeros(nsp)
            rc, res = st.st_poll(srv, t, buf)
            if rc != st.ST_PENDING:
                out[t] = (rc, buf, res)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out


def burgers_case(K, N, Nt, seed):
    c = cfg("burgers", 1, [K], N, Nt)
    return c


def advdiff_case(K, N, Nt):
    return cfg("advdiff", 2, [K, K], N, Nt, a=(1.0, 0.5), nu=1e-3)


def initial_for(P, kind, seed):
    X = P.coords()
    if kind == "burgers":
        return inputs.burgers_smooth(X, inputs.burgers_params(seed)).ravel()
    return inputs.fourier_modes(X, inputs.fourier_params(seed)).ravel()


def test_alone_vs_mix_bitwise(orc):
    from paper_2201_05800_amd import st
    # (kind, problem, FP32-inner, Gram-Schmidt passes): one, two and the
    # adaptive form (0) mixed in one batch, each request with its own
    cases = [("burgers", burgers_case(40, 3, 3, 1), 0, 1), ("advdiff", advdiff_case(10, 3, 2), 0, 2),
             ("burgers", burgers_case(23, 5, 4, 2), 1, 1), ("advdiff", advdiff_case(8, 4, 4), 1, 2),
             ("burgers", burgers_case(64, 2, 2, 3), 0, 2), ("advdiff", advdiff_case(12, 2, 3), 1, 1),
             ("burgers", burgers_case(7, 2, 3, 4), 1, 2),     # 63 unknowns: element-wise vector paths
             ("advdiff", advdiff_case(9, 3, 3), 0, 0), ("burgers", burgers_case(30, 4, 3, 5), 1, 0)]
    pairs = [Pair(c) for _, c, _, _ in cases]
    try:
        reqs, ups, dts = [], [], []
        for (kind, c, fp32, cgs), P in zip(cases, pairs):
            up = initial_for(P, kind, seed=11)
            h = min((c["hi"][a] - c["lo"][a]) / c["K"][a] for a in range(c["dim"]))
            lam = np.abs(up).max() if kind == "burgers" else np.sqrt(1.25)
            dt = inputs.cfl_dt(5.0, h, c["N"], lam)
            ups.append(up)
            dts.append(dt)
            reqs.append(make_req(st, c, up, dt, inner_fp32=fp32, cgs_passes=cgs))
        srv = st.st_server_create(hbm_budget_bytes=2 << 30, max_active=16)
        try:
            # alone: one at a time
            alone = []
            for r, P in zip(reqs, pairs):
                t = st.st_submit(srv, r)
                (rc, u, res), = wait_all(st, srv, [t], [P.nsp]).values()
                assert rc == st.ST_OK, (rc, res)
                alone.append(u)
            # mix: all at once, in reverse order
            tks = [st.st_submit(srv, r) for r in reversed(reqs)]
            got = wait_all(st, srv, tks, [P.nsp for P in reversed(pairs)])
            mix = [got[t][1] for t in reversed(tks)]
            for i, (a, b) in enumerate(zip(alone, mix)):
                assert got[tks[len(tks) - 1 - i]][0] == st.ST_OK
                assert np.array_equal(a, b), f"request {i} differs alone vs mix"
            stats = st.st_server_stats(srv)
            say("server stats", stats)
        finally:
            st.st_server_destroy(srv)
        # each served result equals the single-slab driver and the oracle
        for (kind, c, fp32, cgs), P, up, dt, u in zip(cases, pairs, ups, dts, alone):
            U1, un1, _ = gpu_solve(P, up, dt, 1e-11, inner_fp32=fp32, cgs_passes=cgs)
            assert np.array_equal(un1, u), "served result differs from st_solve_slab"
            Uo, so = orc.solve(P.p, up, dt, tol=1e-13, dense_limit=0)
            e = rel(u, orc.last_time_node(P.p, Uo))
            say(f"served {kind} K={c['K']} N={c['N']} Nt={c['Nt']} fp32={fp32} cgs={cgs}: "
                f"rel err vs oracle {e:.2e}")
            assert e <= 1e-9
    finally:
        for P in pairs:
            P.close()


def test_served_preconditioned_requests(orc):
    """Element-block Jacobi in the server (scalar equations): preconditioned
    and plain requests of both precisions served together; every result is
    bitwise the single-slab driver's with the same options, matches the
    oracle within 1e-9, and takes fewer Arnoldi steps than unpreconditioned."""
    from paper_2201_05800_amd import st
    cases = [("advdiff", advdiff_case(12, 3, 3), 0, 1), ("burgers", burgers_case(40, 3, 3, 1), 0, 1),
             ("advdiff", advdiff_case(10, 4, 4), 1, 1), ("burgers", burgers_case(23, 5, 2, 2), 1, 1),
             ("advdiff", advdiff_case(9, 2, 2), 0, 0), ("burgers", burgers_case(7, 2, 3, 4), 0, 1)]
    pairs = [Pair(c) for _, c, _, _ in cases]
    try:
        reqs, ups, dts = [], [], []
        for (kind, c, fp32, pc), P in zip(cases, pairs):
            up = initial_for(P, kind, seed=5)
            h = min((c["hi"][a] - c["lo"][a]) / c["K"][a] for a in range(c["dim"]))
            lam = np.abs(up).max() if kind == "burgers" else np.sqrt(1.25)
            dt = inputs.cfl_dt(5.0, h, c["N"], lam)
            ups.append(up)
            dts.append(dt)
            reqs.append(make_req(st, c, up, dt, inner_fp32=fp32, precond=pc))
        srv = st.st_server_create(hbm_budget_bytes=2 << 30, max_active=16)
        try:
            tks = [st.st_submit(srv, r) for r in reqs]
            got = wait_all(st, srv, tks, [P.nsp for P in pairs])
        finally:
            st.st_server_destroy(srv)
        for (kind, c, fp32, pc), P, up, dt, t in zip(cases, pairs, ups, dts, tks):
            rc, u, res = got[t]
            assert rc == st.ST_OK, (kind, rc)
            _, un1, s1 = gpu_solve(P, up, dt, 1e-11, inner_fp32=fp32, precond=pc)
            assert np.array_equal(un1, u), f"served {kind} differs from st_solve_slab (precond={pc})"
            if pc:
                _, _, s0 = gpu_solve(P, up, dt, 1e-11, inner_fp32=fp32, precond=0)
                assert res["gmres_its"] < s0["gmres_its"], (kind, res, s0)
            Uo, so = orc.solve(P.p, up, dt, tol=1e-13, dense_limit=0)
            e = rel(u, orc.last_time_node(P.p, Uo))
            say(f"served {kind} K={c['K']} N={c['N']} Nt={c['Nt']} fp32={fp32} precond={pc}: "
                f"GMRES {res['gmres_its']}, rel err vs oracle {e:.2e}")
            assert e <= 1e-9
    finally:
        for P in pairs:
            P.close()


def test_served_boundary_requests(orc):
    """Requests with Dirichlet boundaries (Burgers and advection-diffusion,
    exterior states 0.5 and 0.2) served together with a periodic one, both
    precisions, with and without the element-block preconditioner: each
    result is bitwise the single-slab driver's and matches the oracle within
    1e-9."""
    from paper_2201_05800_amd import st
    cases = [("burgers", cfg("burgers", 1, [30], 3, 3, bc=(1,), bc_value=0.5), 0, 0),
             ("burgers", cfg("burgers", 1, [17], 4, 2, bc=(1,), bc_value=0.5), 1, 1),
             ("advdiff", cfg("advdiff", 2, [9, 7], 3, 3, a=(1.0, 0.5), nu=1e-3, bc=(1, 0), bc_value=0.2), 0, 1),
             ("advdiff", cfg("advdiff", 2, [6, 6], 2, 4, a=(1.0, 0.5), nu=1e-3, bc=(1, 1), bc_value=0.2), 1, 0),
             ("burgers", burgers_case(20, 3, 3, 6), 0, 1)]
    pairs = [Pair(c) for _, c, _, _ in cases]
    try:
        reqs, ups, dts = [], [], []
        for (kind, c, fp32, pc), P in zip(cases, pairs):
            up = initial_for(P, kind, seed=8)
            if kind == "burgers":
                up = up + 0.4                       # positive data: inflow at the left end
            h = min((c["hi"][a] - c["lo"][a]) / c["K"][a] for a in range(c["dim"]))
            lam = np.abs(up).max() if kind == "burgers" else np.sqrt(1.25)
            dt = inputs.cfl_dt(5.0, h, c["N"], lam)
            ups.append(up)
            dts.append(dt)
            reqs.append(make_req(st, c, up, dt, inner_fp32=fp32, precond=pc))
        srv = st.st_server_create(hbm_budget_bytes=2 << 30, max_active=16)
        try:
            tks = [st.st_submit(srv, r) for r in reqs]
            got = wait_all(st, srv, tks, [P.nsp for P in pairs])
        finally:
            st.st_server_destroy(srv)
        for (kind, c, fp32, pc), P, up, dt, t in zip(cases, pairs, ups, dts, tks):
            rc, u, res = got[t]
            assert rc == st.ST_OK, (kind, rc)
            _, un1, _ = gpu_solve(P, up, dt, 1e-11, inner_fp32=fp32, precond=pc)
            assert np.array_equal(un1, u), f"served {kind} differs from st_solve_slab"
            Uo, so = orc.solve(P.p, up, dt, tol=1e-13, dense_limit=0)
            e = rel(u, orc.last_time_node(P.p, Uo))
            say(f"served {kind} K={c['K']} bc={c['bc']} fp32={fp32} precond={pc}: GMRES {res['gmres_its']}, "
                f"rel err vs oracle {e:.2e}")
            assert e <= 1e-9
    finally:
        for P in pairs:
            P.close()


def test_continuous_batching_overlap(orc):
    """A request submitted while another runs joins the running batch: it is
    admitted before the first one finishes (server timestamps), and both
    results are the same as alone."""
    from paper_2201_05800_amd import st
    c = advdiff_case(64, 4, 4)
    P = Pair(c)
    try:
        up = initial_for(P, "advdiff", 3)
        req = make_req(st, c, up, 1.0 / 128, tol=1e-10)
        srv = st.st_server_create(hbm_budget_bytes=4 << 30, max_active=8)
        try:
            tA = st.st_submit(srv, req)
            t0 = time.time()
            while st.st_server_stats(srv)["active"] < 1:
                assert time.time() - t0 < 30
                time.sleep(0.0005)
            tB = st.st_submit(srv, req)
            max_active = 0
            for _ in range(200):
                max_active = max(max_active, st.st_server_stats(srv)["active"])
                if max_active >= 2:
                    break
                time.sleep(0.0005)
            got = wait_all(st, srv, [tA, tB], [P.nsp] * 2)
            (rcA, uA, rA), (rcB, uB, rB) = got[tA], got[tB]
            assert rcA == st.ST_OK and rcB == st.ST_OK
            assert np.array_equal(uA, uB)
            say("A admit/done", rA["admit_us"], rA["done_us"], "B submit/admit/done", rB["submit_us"],
                rB["admit_us"], rB["done_us"], "max active", max_active)
            assert rB["admit_us"] < rA["done_us"], "B was not admitted while A ran"
            assert max_active >= 2
        finally:
            st.st_server_destroy(srv)
    finally:
        P.close()


def test_admission_budget_and_queueing():
    from paper_2201_05800_amd import st
    c = advdiff_case(16, 3, 3)
    P = Pair(c)
    try:
        up = initial_for(P, "advdiff", 4)
        r = make_req(st, c, up, 1.0 / 64)
        fp = st.st_request_footprint(r)
        # budget below one request: refused at submit
        srv = st.st_server_create(hbm_budget_bytes=max(fp // 2, 1 << 20), max_active=4)
        try:
            with pytest.raises(st.StError) as ei:
                st.st_submit(srv, r)
            assert ei.value.code == st.ST_ERR_OOM_ADMISSION
        finally:
            st.st_server_destroy(srv)
        # budget for exactly one: requests run one at a time, all finish
        srv = st.st_server_create(hbm_budget_bytes=fp + 4096, max_active=4)
        try:
            tks = [st.st_submit(srv, r) for _ in range(3)]
            seen_queue = 0
            for _ in range(20):
                s = st.st_server_stats(srv)
                assert s["active"] <= 1 and s["bytes_in_use"] <= fp + 4096
                seen_queue = max(seen_queue, s["queued"])
                time.sleep(0.001)
            got = wait_all(st, srv, tks, [P.nsp] * 3)
            assert all(v[0] == st.ST_OK for v in got.values())
            assert seen_queue >= 1
        finally:
            st.st_server_destroy(srv)
    finally:
        P.close()


def test_failures_do_not_disturb_others():
    """A non-finite input and a request with too few Newton steps fail with
    their own codes; a healthy request in the same batch completes; a
    cancelled ticket reports cancellation."""
    from paper_2201_05800_amd import st
    c = burgers_case(32, 3, 3, 5)
    P = Pair(c)
    try:
        up = initial_for(P, "burgers", 5)
        bad = up.copy()
        bad[7] = np.nan
        srv = st.st_server_create(hbm_budget_bytes=1 << 30, max_active=8)
        try:
            t_ok = st.st_submit(srv, make_req(st, c, up, 0.02))
            t_nan = st.st_submit(srv, make_req(st, c, bad, 0.02))
            t_lim = st.st_submit(srv, make_req(st, c, up, 0.02, tol=1e-15, max_newton=1))
            t_can = st.st_submit(srv, make_req(st, c, up, 0.02))
            st.st_cancel(srv, t_can)
            got = wait_all(st, srv, [t_ok, t_nan, t_lim, t_can], [P.nsp] * 4)
            assert got[t_ok][0] == st.ST_OK
            assert got[t_nan][0] == st.ST_ERR_NONFINITE
            assert got[t_lim][0] == st.ST_ERR_NO_CONVERGENCE
            assert got[t_can][0] in (st.ST_ERR_CANCELLED, st.ST_OK)
            # the healthy result is the same as alone
            (rc, u_alone, _), = wait_all(st, srv, [st.st_submit(srv, make_req(st, c, up, 0.02))], [P.nsp]).values()
            assert np.array_equal(u_alone, got[t_ok][1])
            with pytest.raises(st.StError):
                st.st_poll(srv, 999999, np.zeros(P.nsp))
        finally:
            st.st_server_destroy(srv)
    finally:
        P.close()


def test_single_slab_nonfinite_and_limits():
    from paper_2201_05800_amd import st
    P = Pair(cfg("euler", 2, [6, 6], 3, 3, lo=[-5, -5], hi=[5, 5]))
    try:
        up = inputs.isentropic_vortex(P.coords(), seed=3).ravel()
        bad = up.copy()
        bad[3] = np.inf
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, bad, 0.05, 1e-10)
        assert ei.value.code == st.ST_ERR_NONFINITE
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, up, 0.05, 1e-15, max_newton=1)
        assert ei.value.code == st.ST_ERR_NO_CONVERGENCE
        with pytest.raises(st.StError) as ei:
            gpu_solve(P, up, -1.0, 1e-10)
        assert ei.value.code == st.ST_ERR_BAD_ARG
    finally:
        P.close()
