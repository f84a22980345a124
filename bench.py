"""Benchmark of the space-time DG-SEM slab path on one MI355X.

Workload (default): 2D advection-diffusion with the BR1 viscous flux,
velocity (1, 0.5), viscosity 1e-3, periodic [0,1]^2, 64 x 64 quads, N = 4,
Nt = 4 (Lobatto IIIC 4 stages), dt = 1/128, initial data a sum of 8 seeded
Fourier modes.  One STEP is one slab solve (Newton-GMRES around the residual
and its JVP, all in HIP kernels): the K timed steps are K consecutive slabs of
that run, each starting from the previous slab's end state.

value = space-time DOF operator evaluations per second: every residual and
every JVP evaluation counts n = 409,600 unknowns.  The JSON line also carries
slab solves/s, per-slab latency p50/p99, the roofline of the dominant kernel
(timed live with HIP events on the solve's stream) and the CPU oracle timed
on a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
TIME_EVERY = 8             # kernel timing on one slab in eight of the timed region

CONFIGS = {
    # 2D advection-diffusion, BR1
    "advdiff2d": dict(workload="2D advection-diffusion BR1, periodic [0,1]^2, 64x64 quads, N=4, Nt=4, dt=1/128",
                      kind=2, dim=2, K=[64, 64], lo=[0.0, 0.0], hi=[1.0, 1.0], N=4, Nt=4, a=(1.0, 0.5),
                      nu=1e-3, dt=1.0 / 128, init="fourier", tol=1e-10),
    # 2D Euler isentropic vortex
    "euler2d": dict(workload="2D Euler isentropic vortex + 1e-3 density noise, periodic [-5,5]^2, 128x128 quads, "
                             "N=3, Nt=3, CFL 5",
                    kind=4, dim=2, K=[128, 128], lo=[-5.0, -5.0], hi=[5.0, 5.0], N=3, Nt=3, gamma=1.4,
                    dt=None, init="vortex", tol=1e-8),
    # 3D Navier-Stokes Taylor-Green vortex
    "ns3d": dict(workload="3D Navier-Stokes Taylor-Green vortex Re=1600 Mach 0.1, periodic [0,2pi]^3, 16^3 hexes, "
                          "N=3, Nt=3, dt=0.05",
                 kind=5, dim=3, K=[16, 16, 16], lo=[0.0] * 3, hi=[2 * math.pi] * 3, N=3, Nt=3, gamma=1.4,
                 mu=1.0 / 1600, prandtl=0.71, dt=0.05, init="tgv", tol=1e-8),
}

# algorithmic bytes per unknown of one launch of each kernel class
#   residual: read U, read u_prev (1/Nt of a vector), write R
#   jvp: linear equations read v, write Jv; nonlinear read U and v, write Jv
#   grad: read the input once, write d values per unknown
#   multidot at Arnoldi index k: read k+1 basis vectors and w
#   update: read k+1 basis vectors, read and write w


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="advdiff2d", choices=sorted(CONFIGS))
    ap.add_argument("--fp32-inner", type=int, default=0)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--cgs-passes", type=int, default=1)
    ap.add_argument("--no-timing", action="store_true", help="run without HIP-event kernel timing")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests in the served-stream sample (0: skip the serving leg)")
    ap.add_argument("--precond-leg", type=int, default=1,
                    help="1: also time the element-block Jacobi preconditioned solves")
    ap.add_argument("--operators", type=int, default=1,
                    help="1: time st_residual / st_jvp on >= 1 GB working sets (0: skip)")
    ap.add_argument("--operator-reps", type=int, default=10)
    ap.add_argument("--precision-split", type=int, default=1,
                    help="solve the first slab in both precision forms after the timed steps (0: skip, so that a "
                         "counter run sees the timed steps' kernels only)")
    ap.add_argument("--slabs-leg", type=int, default=1,
                    help="time M coupled slabs solved as one system against M sequential slab solves")
    ap.add_argument("--bubble-leg", type=int, default=1,
                    help="the 3D Euler bubble (20^3 hexes, Nt=3, dt 0.2 and 0.05 to t=0.6): time per slab, "
                         "iterations and the density L2 error at the end")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) for counter calibration")
    return ap.parse_args()


def initial_state(cfg, X):
    from paper_2201_05800_amd import inputs
    if cfg["init"] == "fourier":
        return inputs.fourier_modes(X, inputs.fourier_params(2))
    if cfg["init"] == "vortex":
        return inputs.isentropic_vortex(X, seed=3)
    if cfg["init"] == "tgv":
        return inputs.taylor_green(X)
    raise ValueError(cfg["init"])


def measured_traffic(config_name, kernel):
    """HBM traffic per launch of `kernel` from the committed rocprofv3 summary
    of this workload, if the kernel source is unchanged since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{config_name}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ": " in line and not line.startswith(("|", "#")):
            k, v = line.strip().split(": ", 1)
            kv[k] = v
    src = os.path.join(ROOT, kv.get("source", ""))
    if not os.path.isfile(src) or "traffic_bytes_per_launch" not in kv:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("source_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(cfg, u0, U, dt, seconds):
    """The oracle's residual evaluation of the same slab on this host's cores,
    repeated for about `seconds` (a bounded sample of the workload)."""
    import numpy as np
    import oracle
    oracle.build()
    p = oracle.problem(cfg["dim"], cfg["K"], cfg["lo"], cfg["hi"], cfg["N"], cfg["Nt"], cfg["kind"],
                       a=cfg.get("a", (0, 0, 0)), nu=cfg.get("nu", 0.0), gamma=cfg.get("gamma", 1.4),
                       mu=cfg.get("mu", 0.0), prandtl=cfg.get("prandtl", 0.72))
    n = U.size
    oracle.residual(p, U, u0, dt)         # warm (page-in, thread start)

    def rate(budget):
        t0 = time.perf_counter()
        evals = 0
        while True:
            oracle.residual(p, U, u0, dt)
            evals += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return evals, el

    evals, el = rate(seconds)
    threads = oracle.get_threads()
    # the same on one host core (a shorter sample), and the host's CPU model
    oracle.set_threads(1)
    try:
        e1, el1 = rate(max(2.0, seconds / 4))
    finally:
        oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=evals * n / el, unit="space-time DOF residual evals/s", cores=threads,
                kind="oracle",
                sample=f"{evals} oracle residual evaluations of one {n}-unknown slab of the same workload "
                       f"({el:.1f} s)",
                one_core_value=e1 * n / el1, cpu_model=model)


def lgl_coords(st, dim, K, lo, hi, N):
    """Physical node coordinates (E, dim, ns) of a periodic box mesh from the
    library's LGL nodes (element-major, x fastest)."""
    import numpy as np
    x, _, _ = st.st_lgl(N + 1)
    n1 = N + 1
    ns = n1 ** dim
    E = int(np.prod(K))
    X = np.zeros((E, dim, ns))
    e = np.arange(E)
    s = np.arange(ns)
    for a in range(dim):
        ea = (e // int(np.prod(K[:a]))) % K[a]
        ia = (s // n1 ** a) % n1
        h = (hi[a] - lo[a]) / K[a]
        X[:, a, :] = lo[a] + h * (ea[:, None] + 0.5 * (1.0 + x[ia][None, :]))
    return X


def served_vs_fp64(st, reqs, served):
    """Every served end-of-slab state against a plain FP64 st_solve_slab of the
    same slab on the same GPU (tolerance 1e-10 on both sides): largest relative
    2-norm difference, over the FP64 and the FP32-inner requests."""
    import numpy as np
    import torch
    worst = {0: 0.0, 1: 0.0}
    for j, (q, r, nsp) in enumerate(reqs):
        h = st.st_create(r.mesh, r.N, r.Nt, r.eq)
        try:
            up = torch.as_tensor(np.ctypeslib.as_array(r.u_prev, shape=(nsp,)).copy()).cuda()
            un = torch.empty(nsp, dtype=torch.float64, device="cuda")
            st.st_solve_slab(h, up, 0.0, r.dt, r.tol, st.st_default_opts(), None, un)
            ref = un.cpu().numpy()
        finally:
            st.st_destroy(h)
        d = float(np.linalg.norm(served[j] - ref) / max(np.linalg.norm(ref), 1e-300))
        f = int(q["inner_fp32"])
        worst[f] = max(worst[f], d)
    return dict(reference="plain FP64 st_solve_slab of the same slab, same GPU",
                max_rel_diff_fp64_requests=worst[0], max_rel_diff_fp32_inner_requests=worst[1])


def serving_bench(n_requests, seed=4, budget_gib=64, max_active=64, load=0.7):
    """Served mix of 1D Burgers and 2D advection-diffusion slab solves (K in
    8..256 per axis, N in 2..5, Nt in 2..4, FP64 / FP32-inner 50/50, CFL 5):
    saturated throughput with every request submitted at once, then latency
    under Poisson arrivals at `load` times that throughput."""
    import numpy as np
    from paper_2201_05800_amd import inputs, st

    def build(stream):
        reqs = []
        for q in stream:
            if q["kind"] == "burgers":
                d, K, lo, hi = 1, [q["K"]], [0.0], [1.0]
                X = lgl_coords(st, d, K, lo, hi, q["N"])
                up = inputs.burgers_smooth(X, inputs.burgers_params(q["seed"])).ravel()
                eq = st.equation(st.ST_BURGERS)
                lam = float(np.abs(up).max())
            else:
                d, K, lo, hi = 2, [q["K"], q["K"]], [0.0, 0.0], [1.0, 1.0]
                X = lgl_coords(st, d, K, lo, hi, q["N"])
                up = inputs.fourier_modes(X, inputs.fourier_params(q["seed"])).ravel()
                eq = st.equation(st.ST_ADVDIFF_BR1, a=(1.0, 0.5), nu=1e-3)
                lam = math.sqrt(1.25)
            dt = inputs.cfl_dt(5.0, 1.0 / q["K"], q["N"], lam)
            r = st.request(st.mesh(d, K, lo, hi), q["N"], q["Nt"], eq, up, 0.0, dt, 1e-10,
                           st.st_default_opts(inner_fp32=int(q["inner_fp32"])))
            reqs.append((q, r, up.size))
        return reqs

    def run(reqs, arrivals):
        srv = st.st_server_create(hbm_budget_bytes=budget_gib << 30, max_active=max_active)
        try:
            tks, done = [], {}
            t0 = time.perf_counter()
            i = 0
            while len(done) < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and arrivals[i] <= now:
                    tks.append((st.st_submit(srv, reqs[i][1]), reqs[i][2], i))
                    i += 1
                for t, nsp, j in tks:
                    if j in done:
                        continue
                    buf = np.empty(nsp)
                    rc, info = st.st_poll(srv, t, buf)
                    if rc != st.ST_PENDING:
                        done[j] = (rc, info, buf)
                time.sleep(0.0002)
            wall = time.perf_counter() - t0
            stats = st.st_server_stats(srv)
        finally:
            st.st_server_destroy(srv)
        lat = np.array([(done[j][1]["done_us"] - done[j][1]["submit_us"]) * 1e-3 for j in range(len(reqs))])
        ok = sum(1 for j in done if done[j][0] == st.ST_OK)
        return wall, lat, ok, stats, {j: done[j][2] for j in done}

    stream = inputs.serving_stream(seed, n_requests, rate=0.0)
    reqs = build(stream)
    unknowns = sum(st.st_request_footprint(r) for _, r, _ in reqs)
    wall_sat, lat_sat, ok_sat, _, served = run(reqs, [0.0] * len(reqs))
    thr = len(reqs) / wall_sat
    accuracy = served_vs_fp64(st, reqs, served)
    # Poisson arrivals at 50 / 70 / 90 % of the saturated throughput, and at
    # a fixed 4096 requests/s (beyond saturation: the queue absorbs it)
    sweep, ok_all, stats_p, lat_p, rate = [], ok_sat, None, None, load * thr
    for frac, fixed in ((0.5, None), (load, None), (0.9, None), (None, 4096.0)):
        r_s = fixed if fixed else frac * thr
        g = np.random.default_rng(seed + 1)
        arr = np.cumsum(g.exponential(1.0 / r_s, size=len(reqs)))
        wall_i, lat_i, ok_i, stats_i, _ = run(reqs, arr)
        ok_all = min(ok_all, ok_i)
        sweep.append(dict(load=frac, rate_per_s=r_s, latency_ms_p50=float(np.percentile(lat_i, 50)),
                          latency_ms_p99=float(np.percentile(lat_i, 99)), solves_per_s=len(reqs) / wall_i, ok=ok_i))
        if frac == load:
            stats_p, lat_p = stats_i, lat_i
    return dict(requests=len(reqs), saturated_solves_per_s=thr, saturated_wall_s=wall_sat,
                poisson_rate_per_s=rate, load=load, latency_ms_p50=float(np.percentile(lat_p, 50)),
                latency_ms_p99=float(np.percentile(lat_p, 99)), latency_ms_p50_saturated=float(np.percentile(lat_sat, 50)),
                latency_ms_p99_saturated=float(np.percentile(lat_sat, 99)), ok=ok_all,
                loads=sweep, ticks=stats_p["ticks"], footprint_bytes_total=unknowns, accuracy=accuracy,
                mix="1D Burgers + 2D advection-diffusion, K 8..256, N 2..5, Nt 2..4, FP64/FP32-inner 50/50, CFL 5")


# Enlarged meshes of the three PDE workloads (same N, Nt, equation and data
# recipe) whose vectors are 400-500 MB, so that one operator call moves about
# 1 GB: beyond the 256 MB Infinity Cache, so the rate is an HBM rate.
OPERATOR_WORKLOADS = {
    "advdiff2d": dict(K=[768, 768], label="2D advection-diffusion BR1, 768x768 quads, N=4, Nt=4"),
    "euler2d": dict(K=[512, 512], label="2D Euler vortex, 512x512 quads on [-5,5]^2, N=3, Nt=3"),
    "ns3d": dict(K=[40, 40, 40], label="3D Navier-Stokes TGV, 40^3 hexes, N=3, Nt=3"),
}


def make_handle(c):
    from paper_2201_05800_amd import st
    d = c["dim"]
    m = st.mesh(d, c["K"], c["lo"], c["hi"])
    eq = st.equation(c["kind"], a=c.get("a", (0, 0, 0)), nu=c.get("nu", 0.0), gamma=c.get("gamma", 1.4),
                     mu=c.get("mu", 0.0), prandtl=c.get("prandtl", 0.72))
    return st.st_create(m, c["N"], c["Nt"], eq)


def multi_slab_bench(c, u0, dt, M, precond):
    """M consecutive slabs from u0: one coupled solve (st_solve_slabs) against
    M sequential st_solve_slab calls, same tolerance; the first call of each
    kind is a warm-up (the coupled one grows the handle's buffers)."""
    import torch
    from paper_2201_05800_amd import st
    h = make_handle(c)
    n, nsp, _ = st.st_sizes(h)
    o = st.st_default_opts(precond=precond, max_newton=100)
    up = torch.as_tensor(u0).cuda()
    Uc = torch.empty(n * M, dtype=torch.float64, device="cuda")
    unc = torch.empty(nsp, dtype=torch.float64, device="cuda")
    Us = torch.empty(n, dtype=torch.float64, device="cuda")
    a, b = torch.empty_like(unc), torch.empty_like(unc)

    def sequential():
        x = up
        its = [0, 0]
        for i in range(M):
            y = a if i % 2 == 0 else b
            r = st.st_solve_slab(h, x, 0.0, dt, c["tol"], o, Us, y)
            its[0] += r["newton_its"]
            its[1] += r["gmres_its"]
            x = y
        return x, its

    st.st_solve_slabs(h, M, up, 0.0, dt, c["tol"], o, Uc, unc)
    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = st.st_solve_slabs(h, M, up, 0.0, dt, c["tol"], o, Uc, unc)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t0
    t0 = time.perf_counter()
    last, its = sequential()
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    diff = float(torch.linalg.norm(unc - last) / torch.linalg.norm(last))
    st.st_destroy(h)
    return dict(slabs=M, unknowns_per_slab=n, precond=precond,
                coupled_ms_per_slab=t_c * 1e3 / M, sequential_ms_per_slab=t_s * 1e3 / M,
                coupled_newton_its=rc["newton_its"], coupled_gmres_its=rc["gmres_its"],
                sequential_newton_its=its[0], sequential_gmres_its=its[1],
                u_next_rel_diff=diff)


def bubble_bench(N=3, dts=(0.2, 0.05), T=0.6):
    """3D Euler smooth bubble on [0,1]^3, 20^3 hexes, Nt=3 (the 4D space-time
    test of the paper's numerical results), element-block Jacobi GMRES, slabs
    solved one after another to t = T; density L2 error at T against the
    exactly advected bubble (LGL quadrature on every element)."""
    import numpy as np
    import torch
    from paper_2201_05800_amd import inputs, st
    c = dict(kind=4, dim=3, K=[20, 20, 20], lo=[0.0] * 3, hi=[1.0] * 3, N=N, Nt=3, gamma=1.4, tol=1e-8)
    h = make_handle(c)
    n, nsp, nv = st.st_sizes(h)
    ns = (N + 1) ** 3
    X = st.st_node_coords(h, 3, ns)
    x, w, _ = st.st_lgl(N + 1)
    W = np.ones(ns)
    for s_ in range(ns):
        for a in range(3):
            W[s_] *= w[(s_ // (N + 1) ** a) % (N + 1)] * 0.5 / 20
    rho_ex = inputs.euler_bubble_3d(X, T)[:, 0, :]
    u0 = inputs.euler_bubble_3d(X, 0.0).ravel()
    o = st.st_default_opts(precond=1, max_newton=50)
    U = torch.empty(n, dtype=torch.float64, device="cuda")
    out = []
    for dt in dts:
        steps = int(round(T / dt))
        u = torch.as_tensor(u0).cuda()
        un = torch.empty_like(u)
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res.append(st.st_solve_slab(h, u, 0.0, dt, c["tol"], o, U, un))
            u, un = un, u
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rho = u.cpu().numpy().reshape(-1, nv, ns)[:, 0, :]
        l2 = float(np.sqrt(np.sum(W[None, :] * (rho - rho_ex) ** 2)))
        out.append(dict(dt=dt, slabs=steps, ms_per_slab=el * 1e3 / steps,
                        newton_its_per_slab=sum(r["newton_its"] for r in res) / steps,
                        gmres_its_per_slab=sum(r["gmres_its"] for r in res) / steps,
                        rho_l2_error_at_t=l2))
        print(f"# bubble dt={dt}: {out[-1]}", file=sys.stderr, flush=True)
    st.st_destroy(h)
    return dict(workload="3D Euler smooth bubble, periodic [0,1]^3, 20^3 hexes, N=%d, Nt=3, to t=0.6, "
                         "element-block Jacobi" % N, unknowns_per_slab=n, runs=out)


def operator_bench(reps, fp32_too=True):
    """st_residual and st_jvp on >= 1 GB working sets, timed with HIP events
    on the calling stream (the whole API call: for Navier-Stokes it includes
    the BR1 gradient passes), and the embedded error estimate of a slab.
    Rates use the algorithmic bytes: residual (2 + 1/Nt) n 8, JVP 24 n
    (linear equations 16 n, FP32-inner 20 n), estimate 3 n_space 8."""
    import numpy as np
    import torch
    from paper_2201_05800_amd import inputs, st
    stream = torch.cuda.current_stream()
    out = []
    for name, ow in OPERATOR_WORKLOADS.items():
        cfg = dict(CONFIGS[name])
        cfg["K"] = ow["K"]
        d = cfg["dim"]
        eq = st.equation(cfg["kind"], a=cfg.get("a", (0, 0, 0)), nu=cfg.get("nu", 0.0), gamma=cfg.get("gamma", 1.4),
                         mu=cfg.get("mu", 0.0), prandtl=cfg.get("prandtl", 0.72))
        h = st.st_create(st.mesh(d, cfg["K"], cfg["lo"], cfg["hi"]), cfg["N"], cfg["Nt"], eq)
        try:
            n, nsp, nv = st.st_sizes(h)
            ns = (cfg["N"] + 1) ** d
            u0 = initial_state(cfg, st.st_node_coords(h, d, ns)).reshape(-1, nv, ns)
            hmin = min((cfg["hi"][a] - cfg["lo"][a]) / cfg["K"][a] for a in range(d))
            dt = cfg["dt"]
            if dt is None:
                dt = inputs.cfl_dt(5.0, hmin, cfg["N"], inputs.euler_max_speed(u0, cfg.get("gamma", 1.4)))
            up = torch.as_tensor(u0.ravel()).cuda()
            # a state near the solution: 1 (x) u^n with 1e-3 relative noise
            U = up.view(-1, nv, 1, ns).expand(-1, nv, cfg["Nt"], ns).contiguous().view(-1)
            g = torch.Generator(device="cuda").manual_seed(7)
            U.mul_(1.0 + 1e-3 * torch.randn(n, generator=g, device="cuda", dtype=torch.float64))
            v = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
            R = torch.empty(n, dtype=torch.float64, device="cuda")
            lin = cfg["kind"] in (st.ST_ADVECTION, st.ST_ADVDIFF_BR1)
            calls = [("st_residual", lambda: st.st_residual(h, U, up, 0.0, dt, R, stream), (2.0 + 1.0 / cfg["Nt"]) * 8)]
            calls.append(("st_jvp", lambda: st.st_jvp(h, U, 0.0, dt, v, R, 0, stream), 16.0 if lin else 24.0))
            if fp32_too:
                calls.append(("st_jvp fp32-inner", lambda: st.st_jvp(h, U, 0.0, dt, v, R, 1, stream),
                              16.0 if lin else 20.0))
            # embedded error estimate: reads U_1, U_Nt and u_prev (3 spatial vectors)
            calls.append(("st_error_estimate", lambda: st.st_error_estimate(h, U, up, 1e-6, 1e-6, stream),
                          24.0 / cfg["Nt"]))
            for op, fn, bpu in calls:
                fn()
                fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(stream)
                for _ in range(reps):
                    fn()
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                gbs = bpu * n / (ms * 1e-3) / 1e9
                out.append(dict(workload=ow["label"], op=op, unknowns=n, ms=round(ms, 4),
                                dof_evals_per_s=n / (ms * 1e-3), algorithmic_GBs=round(gbs, 1),
                                frac=round(gbs / HBM_PEAK_GBS, 4)))
                print(f"# {ow['label']}: {op} {ms:.3f} ms, {gbs:.0f} GB/s", file=sys.stderr, flush=True)
            del U, v, R, up
        finally:
            st.st_destroy(h)
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (a slab, or a multi-slab system, per GPU; splitting one "
              "over several GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2201_05800_amd import inputs, st

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nel * 8, "copy_bytes_written": nel * 8, "launches": 3}))
        return
    cfg = CONFIGS[args.config]
    d = cfg["dim"]
    m = st.mesh(d, cfg["K"], cfg["lo"], cfg["hi"])
    eq = st.equation(cfg["kind"], a=cfg.get("a", (0, 0, 0)), nu=cfg.get("nu", 0.0), gamma=cfg.get("gamma", 1.4),
                     mu=cfg.get("mu", 0.0), prandtl=cfg.get("prandtl", 0.72))
    h = st.st_create(m, cfg["N"], cfg["Nt"], eq)
    n, nsp, nv = st.st_sizes(h)
    ns = (cfg["N"] + 1) ** d
    X = st.st_node_coords(h, d, ns)
    u0 = initial_state(cfg, X)
    dt = cfg["dt"]
    if dt is None:
        hmin = min((cfg["hi"][a] - cfg["lo"][a]) / cfg["K"][a] for a in range(d))
        dt = inputs.cfl_dt(5.0, hmin, cfg["N"], inputs.euler_max_speed(u0, cfg.get("gamma", 1.4)))
    u0 = u0.ravel()

    # HIP-event timing: the warm-up times every kernel class to find the
    # dominant one; in the timed region only that class is timed (two events
    # per launch of it), and only on every TIME_EVERY-th slab: event pairs on
    # every launch of every slab made the slabs 17 % slower (35 % for the
    # preconditioned ones)
    every = sum(1 << c for c in (st.ST_K_RESIDUAL, st.ST_K_JVP, st.ST_K_GRAD, st.ST_K_MULTIDOT, st.ST_K_UPDATE,
                                 st.ST_K_NORMALIZE))
    opts = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=args.fp32_inner,
                              timing=0 if args.no_timing else every)
    stream = torch.cuda.current_stream()
    u = torch.as_tensor(u0).cuda()
    un = torch.empty(nsp, dtype=torch.float64, device="cuda")
    U = torch.empty(n, dtype=torch.float64, device="cuda")

    def step(uin, uout):
        return st.st_solve_slab(h, uin, 0.0, dt, cfg["tol"], opts, U, uout, stream)

    warm = []
    for _ in range(args.warmup):
        warm.append(step(u, un))
        u, un = un, u
    shares_w = [sum(s["kernel_us"][c] for s in warm) for c in range(len(st.KERNEL_CLASSES))]
    dom = max(range(len(shares_w)), key=lambda c: shares_w[c]) if warm else st.ST_K_MULTIDOT
    u.copy_(torch.as_tensor(u0))
    torch.cuda.synchronize()

    lat, stats = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        opts.timing = 0 if args.no_timing or i % TIME_EVERY else 1 << dom
        ts = time.perf_counter()
        s = step(u, un)      # synchronises the stream at its end
        lat.append(time.perf_counter() - ts)
        stats.append(s)
        u, un = un, u
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    op_evals = sum(s["newton_its"] + 1 + s["gmres_its"] for s in stats)
    value = op_evals * n / elapsed
    lat_ms = np.array(lat) * 1e3

    # the other precision form on the first slab, against the form timed
    # (both on this GPU, same tolerance): relative 2-norm difference of U
    def first_slab(fp32):
        o2 = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=fp32)
        Ux = torch.empty(n, dtype=torch.float64, device="cuda")
        st.st_solve_slab(h, torch.as_tensor(u0).cuda(), 0.0, dt, cfg["tol"], o2, Ux, None, stream)
        return Ux.cpu().numpy()
    precision_split = None
    if args.precision_split:
        U64, U32 = first_slab(0), first_slab(1)
        precision_split = dict(slab="the first slab of the workload",
                               fp32_inner_vs_fp64_rel_diff=float(np.linalg.norm(U32 - U64) / np.linalg.norm(U64)))

    # roofline of the dominant kernel: algorithmic bytes (accumulated by the
    # library per kernel class) over the HIP-event time of its launches
    def roof_of(cls, name, bound="hbm"):
        timed = [s for s in stats if s["kernel_calls"][cls] > 0]      # the slabs whose launches were timed
        us = sum(s["kernel_us"][cls] for s in timed)
        calls = sum(s["kernel_calls"][cls] for s in timed)
        by = sum(s["kernel_bytes"][cls] for s in timed)
        ach = by / (us * 1e-6) / 1e9 if us > 0 else 0.0
        return dict(bound=bound, kernel=name, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, avg_launch_us=round(us / max(calls, 1), 3),
                    launches=calls, timed_slabs=len(timed), algorithmic_bytes_per_launch=round(by / max(calls, 1)))

    names = {st.ST_K_RESIDUAL: "k_op (residual)", st.ST_K_JVP: "k_op (JVP)", st.ST_K_GRAD: "k_visc",
             st.ST_K_MULTIDOT: "k_multidot", st.ST_K_UPDATE: "k_update", st.ST_K_NORMALIZE: "k_scale_v0"}
    roof = roof_of(dom, names.get(dom, st.KERNEL_CLASSES[dom]))
    roof["traffic"] = measured_traffic(args.config, roof["kernel"].split(" ")[0])
    warm_total = sum(shares_w) or 1.0
    shares = {st.KERNEL_CLASSES[c]: round(shares_w[c] / warm_total, 4) for c in range(len(shares_w))}

    # element-block Jacobi right preconditioning: the same slabs, solved to
    # the same tolerance (nonlinear equations: the block of the Jacobian at
    # the mean state; element blocks of more than 1024 unknowns are not
    # supported and the leg is skipped)
    precond = None
    nvars = cfg["dim"] + 2 if cfg["kind"] in (st.ST_EULER, st.ST_NS_BR1) else 1
    npe = nvars * cfg["Nt"] * (cfg["N"] + 1) ** cfg["dim"]
    if args.precond_leg and npe > 1024:
        print(f"# preconditioned leg skipped: element block of {npe} unknowns (at most 1024)", file=sys.stderr)
    if args.precond_leg and npe <= 1024:
        opc = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=args.fp32_inner,
                                 precond=1)
        u.copy_(torch.as_tensor(u0))
        step_pc = lambda uin, uout: st.st_solve_slab(h, uin, 0.0, dt, cfg["tol"], opc, U, uout, stream)
        step_pc(u, un)                       # warm-up: assembles and inverts the element block
        u.copy_(torch.as_tensor(u0))
        torch.cuda.synchronize()
        lat_pc, stats_pc = [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            opc.timing = 0 if args.no_timing or i % TIME_EVERY else 1 << st.ST_K_PRECOND
            ts = time.perf_counter()
            stats_pc.append(step_pc(u, un))
            lat_pc.append(time.perf_counter() - ts)
            u, un = un, u
        torch.cuda.synchronize()
        el_pc = time.perf_counter() - t0
        timed_pc = [x for x in stats_pc if x["kernel_calls"][st.ST_K_PRECOND] > 0]
        us = sum(x["kernel_us"][st.ST_K_PRECOND] for x in timed_pc)
        calls = sum(x["kernel_calls"][st.ST_K_PRECOND] for x in timed_pc)
        by = sum(x["kernel_bytes"][st.ST_K_PRECOND] for x in timed_pc)
        precond = dict(
            method="element-block Jacobi, right preconditioning (B^-1 of the element diagonal block of the slab "
                   "Jacobian, the same in every element" +
                   ("" if cfg["kind"] in (st.ST_ADVECTION, st.ST_ADVDIFF_BR1) else ", taken at the mean state") + ")",
            ms_per_step=el_pc * 1e3 / args.steps, slab_solves_per_s=args.steps / el_pc,
            speedup_vs_plain=(elapsed / args.steps) / (el_pc / args.steps),
            latency_ms_p50=float(np.percentile(np.array(lat_pc) * 1e3, 50)),
            latency_ms_p99=float(np.percentile(np.array(lat_pc) * 1e3, 99)),
            newton_its_per_slab=sum(x["newton_its"] for x in stats_pc) / len(stats_pc),
            gmres_its_per_slab=sum(x["gmres_its"] for x in stats_pc) / len(stats_pc),
            dof_evals_per_s=sum(x["newton_its"] + 1 + x["gmres_its"] for x in stats_pc) * n / el_pc,
            precond_kernel=dict(kernel="k_bjacobi", avg_launch_us=round(us / max(calls, 1), 3),
                                achieved_GBs=round(by / (us * 1e-6) / 1e9, 1) if us > 0 else None,
                                achieved_TFLOPs=round(2.0 * npe * n * calls / (us * 1e-6) / 1e12, 2) if us > 0 else None,
                                peak_TFLOPs=78.6, element_block=npe,
                                note="FP64 matrix cores, 2 npe FLOP per unknown; algorithmic bytes: direction in, "
                                     "result out (B^-1, npe^2 doubles, re-read by every block from L2 / MALL)"))
        print(f"# preconditioned: {precond['ms_per_step']:.3f} ms/slab, {precond['gmres_its_per_slab']:.1f} "
              f"GMRES its/slab", file=sys.stderr, flush=True)

    slabs = None
    if args.slabs_leg:
        small = dict(CONFIGS["advdiff2d"], K=[16, 16])
        hs = make_handle(small)
        Xs = st.st_node_coords(hs, 2, (small["N"] + 1) ** 2)
        st.st_destroy(hs)
        u_small = initial_state(small, Xs).ravel()
        slabs = dict(note="M slabs from the same u^n: one coupled Newton-GMRES solve against M sequential "
                          "slab solves, both to the workload's tolerance",
                     workload=[multi_slab_bench(cfg, u0, dt, 4, 0), multi_slab_bench(cfg, u0, dt, 4, 1)],
                     small_16x16=[multi_slab_bench(small, u_small, dt, 8, 0)] +
                                 [multi_slab_bench(small, u_small, dt, M, 1) for M in (4, 8, 16, 32)])
        print(f"# slabs: {slabs}", file=sys.stderr, flush=True)
    bubble = bubble_bench() if args.bubble_leg else None

    serving = serving_bench(args.serve_requests) if args.serve_requests > 0 else None
    operators = operator_bench(args.operator_reps) if args.operators else None

    cpu = None
    if not args.no_cpu_baseline:
        Uh = U.cpu().numpy()
        cpu = cpu_baseline(cfg, u0, Uh, dt, args.cpu_baseline_seconds)

    out = {
        "metric": "space-time DOF residual evals/s + slab solves/s, p50/p99 latency, % HBM peak",
        "value": value,
        "unit": "space-time DOF residual evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not args.fp32_inner else "f64 (f32 inner JVP)",
        "data": "synthetic",
        "config": {"workload": cfg["workload"], "unknowns_per_slab": n, "restart": args.restart,
                   "cgs_passes": args.cgs_passes, "inner_fp32": args.fp32_inner, "tol": cfg["tol"]},
        "slab_solves_per_s": args.steps / elapsed,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "newton_its_per_slab": sum(s["newton_its"] for s in stats) / len(stats),
        "gmres_its_per_slab": sum(s["gmres_its"] for s in stats) / len(stats),
        "operator_evals": op_evals,
        "kernel_time_share_of_timed": shares,
        "precision_split": precision_split,
        # algorithmic bytes of the timed steps per kernel class (the library's
        # per-launch byte model, summed)
        "kernel_bytes_of_timed": {st.KERNEL_CLASSES[c]: sum(s["kernel_bytes"][c] for s in stats)
                                  for c in range(len(st.KERNEL_CLASSES))},
        "roofline": roof,
        "preconditioned": precond,
        "serving": serving,
        "multi_slab": slabs,
        "euler3d_bubble": bubble,
        "operators": operators,
        "cpu_baseline": cpu,
    }
    st.st_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
