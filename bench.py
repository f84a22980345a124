"""Benchmark of the space-time DG-SEM slab path on one MI355X.

Workload (default): the 3D compressible Navier-Stokes Taylor-Green vortex,
Re = 1600, Mach 0.1, periodic [0, 2 pi]^3, 16^3 hexes, N = 3, Nt = 3 (Lobatto
IIIC 3 stages), dt = 0.05, BR1 viscous flux, Rusanov convective flux: 3.9 M
space-time unknowns per slab, a Krylov basis of about 1 GB (beyond the 256 MB
Infinity Cache).  One STEP is one slab solve (Newton-GMRES around the residual
and its JVP, all in HIP kernels): the K timed steps are K consecutive slabs of
that run, each starting from the previous slab's end state.

value = space-time DOF operator evaluations per second during the solves:
every residual and every JVP evaluation counts n unknowns (residual and JVP
rates of the operator calls alone are reported apart).  The JSON line also
carries slab solves/s, per-slab latency p50/p99, the roofline of the dominant
kernel (timed live with HIP events on the solve's stream), the FP32-inner form
against plain FP64 on the 2D Euler vortex and this workload, the 2D
advection-diffusion workload (cache resident) and the CPU oracle timed on a
bounded sample of the same workload on this host.
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
                    dt=None, init="vortex", tol=1e-10),
    # 3D Navier-Stokes Taylor-Green vortex
    "ns3d": dict(workload="3D Navier-Stokes Taylor-Green vortex Re=1600 Mach 0.1, periodic [0,2pi]^3, 16^3 hexes, "
                          "N=3, Nt=3, dt=0.05",
                 kind=5, dim=3, K=[16, 16, 16], lo=[0.0] * 3, hi=[2 * math.pi] * 3, N=3, Nt=3, gamma=1.4,
                 mu=1.0 / 1600, prandtl=0.71, dt=0.05, init="tgv", tol=1e-10),
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="ns3d", choices=sorted(CONFIGS))
    ap.add_argument("--fp32-inner", type=int, default=0)
    ap.add_argument("--cpu-baseline-seconds", type=float, default=8.0,
                    help="seconds per oracle leg (residual, JVP, slab solve of a reduced box)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--cgs-passes", type=int, default=1)
    ap.add_argument("--no-timing", action="store_true", help="run without HIP-event kernel timing")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests in the served stream (0: skip the serving leg)")
    ap.add_argument("--precond-leg", type=int, default=1,
                    help="1: also time the element-block Jacobi preconditioned solves")
    ap.add_argument("--operators", type=int, default=1,
                    help="1: time st_residual / st_jvp on >= 1 GB working sets (0: skip)")
    ap.add_argument("--operator-reps", type=int, default=10)
    ap.add_argument("--forms-leg", type=int, default=1,
                    help="FP64 and FP32-inner solves of the same slabs (2D Euler vortex, 3D Navier-Stokes): time "
                         "per slab and their difference (0: skip, so that a counter run sees the timed steps' "
                         "kernels only)")
    ap.add_argument("--forms-steps", type=int, default=8)
    ap.add_argument("--cache-leg", type=int, default=1,
                    help="the 2D advection-diffusion workload (64x64, vectors of 3.3 MB: cache resident)")
    ap.add_argument("--slabs-leg", type=int, default=1,
                    help="time M coupled slabs solved as one system against M sequential slab solves")
    ap.add_argument("--pulse-leg", type=int, default=1,
                    help="the rotating pulse rows of the paper's advection-diffusion error table")
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


def oracle_problem(cfg):
    import oracle
    return oracle.problem(cfg["dim"], cfg["K"], cfg["lo"], cfg["hi"], cfg["N"], cfg["Nt"], cfg["kind"],
                          a=cfg.get("a", (0, 0, 0)), nu=cfg.get("nu", 0.0), gamma=cfg.get("gamma", 1.4),
                          mu=cfg.get("mu", 0.0), prandtl=cfg.get("prandtl", 0.72))


def cpu_baseline(cfg, u0, U, dt, seconds):
    """The oracle on this host's cores, on bounded samples of the workload:
    its residual and its JVP of the workload's slab, repeated for about
    `seconds` each, and its Newton solve of a reduced box of the workload
    (2 elements per axis in 3D, 4 in 2D, with the workload's spacing, N, Nt,
    dt and state, periodic), repeated for about `seconds`."""
    import numpy as np
    import oracle
    oracle.build()
    p = oracle_problem(cfg)
    n = U.size
    V = np.random.default_rng(11).standard_normal(n)
    oracle.residual(p, U, u0, dt)         # warm (page-in, thread start)

    def rate(fn, budget):
        t0 = time.perf_counter()
        k = 0
        while True:
            fn()
            k += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return k, el

    r_k, r_el = rate(lambda: oracle.residual(p, U, u0, dt), seconds)
    j_k, j_el = rate(lambda: oracle.jvp(p, U, dt, V), seconds)
    # a reduced periodic box: the first 2 elements along each axis (3D) or
    # 4 (2D), with the workload's spacing and state
    d = cfg["dim"]
    cnt = [2 if d == 3 else 4] * d
    h = [(cfg["hi"][a] - cfg["lo"][a]) / cfg["K"][a] for a in range(d)]
    box = dict(cfg, K=cnt, hi=[cfg["lo"][a] + h[a] * cnt[a] for a in range(d)])
    nv = oracle.nvars(cfg["kind"], d)
    ns = (cfg["N"] + 1) ** d
    uf = np.asarray(u0).reshape(-1, nv, ns)
    K = cfg["K"]
    sel = [x + K[0] * (y + (K[1] if d > 1 else 1) * z) for z in range(cnt[2] if d > 2 else 1)
           for y in range(cnt[1] if d > 1 else 1) for x in range(cnt[0])]
    ub = np.ascontiguousarray(uf[np.array(sel)]).ravel()
    pb = oracle_problem(box)
    nb = oracle.slab_size(pb)
    its = []
    s_k, s_el = rate(lambda: its.append(oracle.solve(pb, ub, dt, tol=cfg["tol"], dense_limit=0)[1]), seconds)
    threads = oracle.get_threads()
    # the residual on one host core (a shorter sample), and the host's CPU model
    oracle.set_threads(1)
    try:
        e1, el1 = rate(lambda: oracle.residual(p, U, u0, dt), max(2.0, seconds / 4))
    finally:
        oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=r_k * n / r_el, unit="space-time DOF residual evals/s", cores=threads,
                kind="oracle",
                sample=f"{r_k} oracle residual and {j_k} JVP evaluations of one {n}-unknown slab of the same "
                       f"workload ({r_el:.1f} s, {j_el:.1f} s), and {s_k} Newton-GMRES solves of a "
                       f"{'x'.join(map(str, cnt))}-element box of it ({nb} unknowns, {s_el:.1f} s)",
                jvp_dof_evals_per_s=j_k * n / j_el,
                box_slab_solves_per_s=s_k / s_el, box_unknowns=nb,
                box_gmres_its=float(np.mean([x["linear_its"] for x in its])),
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


def served_vs_fp64(st, reqs, served, sample=256):
    """Served end-of-slab states against a plain FP64, unpreconditioned
    st_solve_slab of the same slab on the same GPU (tolerance 1e-10 on both
    sides): largest relative 2-norm difference, over the FP64 and the
    FP32-inner requests, for every k-th request (at most `sample`)."""
    import numpy as np
    import torch
    worst = {0: 0.0, 1: 0.0}
    step = max(1, len(reqs) // sample)
    for j, (q, r, nsp) in enumerate(reqs):
        if j % step:
            continue
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
    return dict(reference="plain FP64 st_solve_slab of the same slab, same GPU, every %d-th request" % step,
                max_rel_diff_fp64_requests=worst[0], max_rel_diff_fp32_inner_requests=worst[1])


def serving_bench(n_requests, seed=4, budget_gib=64, max_active=64, load=0.7, precond=1):
    """Served mix of 1D Burgers and 2D advection-diffusion slab solves (K in
    8..256 per axis, N in 2..5, Nt in 2..4, FP64 / FP32-inner 50/50, CFL 5,
    element-block Jacobi when `precond`): saturated throughput with every
    request submitted at once, then latency under Poisson arrivals at 50 / 70
    / 90 % of that throughput and at a fixed 4096 requests/s."""
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
                           st.st_default_opts(inner_fp32=int(q["inner_fp32"]), precond=precond))
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
        # algorithmic bytes of the served solves (model): per Arnoldi step
        # the JVP (16 B per unknown, linear; 24 B Burgers, 20 B FP32-inner)
        # and classical Gram-Schmidt at the cycle's mean Arnoldi index
        # ((c + 2) 8 B per unknown for cycles of c steps), per outer
        # iteration a residual and the Newton update
        by = 0.0
        for j in range(len(reqs)):
            q, r, _ = reqs[j]
            info = done[j][1]
            n = r.mesh.K[0] * (r.mesh.K[1] if r.mesh.dim > 1 else 1) * (r.N + 1) ** r.mesh.dim * r.Nt
            its, outer = info["gmres_its"], max(info["newton_its"], 1)
            c = min(30.0, its / outer)
            jb = 16.0 if q["kind"] != "burgers" else (20.0 if q["inner_fp32"] else 24.0)
            by += n * (its * (jb + (c + 2.0) * 8.0) + outer * ((2.0 + 1.0 / r.Nt) * 8.0 + (c + 2.0) * 8.0))
        return wall, lat, ok, stats, {j: done[j][2] for j in done}, by

    stream = inputs.serving_stream(seed, n_requests, rate=0.0)
    reqs = build(stream)
    unknowns = sum(st.st_request_footprint(r) for _, r, _ in reqs)
    wall_sat, lat_sat, ok_sat, _, served, by_sat = run(reqs, [0.0] * len(reqs))
    thr = len(reqs) / wall_sat
    accuracy = served_vs_fp64(st, reqs, served)
    # Poisson arrivals at 50 / 70 / 90 % of the saturated throughput, and at
    # a fixed 4096 requests/s (beyond saturation: the queue absorbs it)
    sweep, ok_all, stats_p, lat_p, rate = [], ok_sat, None, None, load * thr
    for frac, fixed in ((0.5, None), (load, None), (0.9, None), (None, 4096.0)):
        r_s = fixed if fixed else frac * thr
        g = np.random.default_rng(seed + 1)
        arr = np.cumsum(g.exponential(1.0 / r_s, size=len(reqs)))
        wall_i, lat_i, ok_i, stats_i, _, _ = run(reqs, arr)
        ok_all = min(ok_all, ok_i)
        sweep.append(dict(load=frac, rate_per_s=r_s, latency_ms_p50=float(np.percentile(lat_i, 50)),
                          latency_ms_p99=float(np.percentile(lat_i, 99)), solves_per_s=len(reqs) / wall_i, ok=ok_i))
        if frac == load:
            stats_p, lat_p = stats_i, lat_i
    return dict(requests=len(reqs), precond=precond, saturated_solves_per_s=thr, saturated_wall_s=wall_sat,
                saturated_algorithmic_GBs=round(by_sat / wall_sat / 1e9, 1),
                saturated_frac_of_hbm=round(by_sat / wall_sat / 1e9 / HBM_PEAK_GBS, 4),
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


def pulse_table_bench():
    """The rotating pulse of Sec. "Experiments / Advection-Diffusion" (eq.
    advdiffeq, interior penalty, eps = 1e-3, periodic [0,1]^2, dx = dt = 1/N,
    spatial degree Nt - 1) solved slab after slab to t = 1 for the rows of
    Table TableL2Errors: spatial L2 error at t = 1 (LGL quadrature) beside the
    paper's STDG column, and the time of the whole run."""
    import numpy as np
    import torch
    from paper_2201_05800_amd import inputs, st
    paper = {2: [7.28e-2, 4.46e-2, 3.39e-2, 1.84e-2], 3: [4.37e-2, 2.41e-2, 5.38e-3, 5.94e-4],
             4: [2.69e-2, 6.04e-3, 4.93e-4, 9.88e-6]}
    rows = []
    for Nt in (2, 3, 4):
        for N, want in zip((4, 8, 16, 32), paper[Nt]):
            c = dict(kind=st.ST_ADVDIFF_SIPG, dim=2, K=[N, N], lo=[0.0, 0.0], hi=[1.0, 1.0], N=Nt - 1, Nt=Nt,
                     a=(0.0, 0.0), nu=1e-3)
            h = st.st_create(st.mesh(2, c["K"], c["lo"], c["hi"]), Nt - 1, Nt,
                             st.equation(st.ST_ADVDIFF_SIPG, a=(0.0, 0.0), nu=1e-3, omega=4.0, center=(0.5, 0.5)))
            try:
                n, nsp, _ = st.st_sizes(h)
                n1 = Nt
                X = st.st_node_coords(h, 2, n1 * n1)
                u = torch.as_tensor(inputs.rotating_pulse(X, 0.0).ravel()).cuda()
                un = torch.empty_like(u)
                o = st.st_default_opts()
                its = 0
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(N):
                    its += st.st_solve_slab(h, u, 0.0, 1.0 / N, 1e-11, o, None, un)["gmres_its"]
                    u, un = un, u
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                x, w, _ = st.st_lgl(n1)
                W = np.array([w[q % n1] * w[q // n1] for q in range(n1 * n1)]) * (0.5 / N) ** 2
                err = float(np.sqrt(np.sum(W[None, :] * (u.cpu().numpy().reshape(N * N, -1) -
                                                         inputs.rotating_pulse(X, 1.0)) ** 2)))
                rows.append(dict(Nt=Nt, N=N, l2_error=err, paper_stdg=want, ratio=round(err / want, 3),
                                 slabs=N, gmres_its_per_slab=its / N, ms_total=round(el * 1e3, 2)))
            finally:
                st.st_destroy(h)
    print(f"# rotating pulse: {rows}", file=sys.stderr, flush=True)
    return dict(workload="rotating pulse, eq. advdiffeq, interior penalty (eta = 10 p^2), eps = 1e-3, periodic "
                         "[0,1]^2, dx = dt = 1/N, spatial degree Nt - 1, GMRES tol 1e-11", rows=rows)


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
            # embedded error estimate: Nt = 2 reads U_1, U_Nt and u_prev (3
            # spatial vectors); Nt > 2: the spatial operator at u_prev reads
            # and writes one spatial vector, then the estimate reads every
            # time node of U, u_prev and that result (Nt + 4 in all)
            est_bytes = 24.0 / cfg["Nt"] if cfg["Nt"] == 2 else 8.0 * (cfg["Nt"] + 4) / cfg["Nt"]
            calls.append(("st_error_estimate", lambda: st.st_error_estimate(h, U, up, 0.0, dt, 1e-6, 1e-6, stream),
                          est_bytes))
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


class Workload:
    """One slab workload on the GPU: handle, initial state, step size."""

    def __init__(self, name):
        import torch
        from paper_2201_05800_amd import inputs, st
        self.name = name
        self.cfg = cfg = CONFIGS[name]
        d = cfg["dim"]
        self.h = make_handle(cfg)
        self.n, self.nsp, self.nv = st.st_sizes(self.h)
        ns = (cfg["N"] + 1) ** d
        u0 = initial_state(cfg, st.st_node_coords(self.h, d, ns))
        dt = cfg["dt"]
        if dt is None:
            hmin = min((cfg["hi"][a] - cfg["lo"][a]) / cfg["K"][a] for a in range(d))
            dt = inputs.cfl_dt(5.0, hmin, cfg["N"], inputs.euler_max_speed(u0, cfg.get("gamma", 1.4)))
        self.dt = dt
        self.u0 = u0.ravel()
        self.U = torch.empty(self.n, dtype=torch.float64, device="cuda")

    def close(self):
        from paper_2201_05800_amd import st
        st.st_destroy(self.h)


def run_slabs(w, opts, steps, stream, timing_cls=None, every=TIME_EVERY):
    """`steps` consecutive slab solves from w.u0 (the end state of one is the
    next one's u_prev); kernel timing of class `timing_cls` on one slab in
    `every`.  Returns (elapsed s, per-slab latencies s, per-slab stats)."""
    import torch
    from paper_2201_05800_amd import st
    u = torch.as_tensor(w.u0).cuda()
    un = torch.empty(w.nsp, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        opts.timing = 0 if timing_cls is None or i % every else 1 << timing_cls
        ts = time.perf_counter()
        stats.append(st.st_solve_slab(w.h, u, 0.0, w.dt, w.cfg["tol"], opts, w.U, un, stream))  # synchronises
        lat.append(time.perf_counter() - ts)
        u, un = un, u
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, stats


def roof_of(stats, cls, name, bound="hbm"):
    """Algorithmic bytes of kernel class `cls` (accumulated by the library per
    launch) over the HIP-event time of its launches, on the slabs timed."""
    timed = [s for s in stats if s["kernel_calls"][cls] > 0]
    us = sum(s["kernel_us"][cls] for s in timed)
    calls = sum(s["kernel_calls"][cls] for s in timed)
    by = sum(s["kernel_bytes"][cls] for s in timed)
    ach = by / (us * 1e-6) / 1e9 if us > 0 else 0.0
    return dict(bound=bound, kernel=name, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, avg_launch_us=round(us / max(calls, 1), 3),
                launches=calls, timed_slabs=len(timed), algorithmic_bytes_per_launch=round(by / max(calls, 1)))


KERNEL_NAMES = {0: "k_op (residual)", 1: "k_op (JVP)", 2: "k_visc", 3: "k_multidot", 4: "k_update",
                5: "k_scale_v0"}


def timed_solve_leg(w, args, stream, fp32=0, precond=0, steps=None):
    """Warm-up solves timing every kernel class (to find the dominant one),
    then `steps` timed slabs with that class timed on one slab in eight."""
    from paper_2201_05800_amd import st
    steps = steps or args.steps
    every = sum(1 << c for c in (st.ST_K_RESIDUAL, st.ST_K_JVP, st.ST_K_GRAD, st.ST_K_MULTIDOT, st.ST_K_UPDATE,
                                 st.ST_K_NORMALIZE, st.ST_K_PRECOND))
    import torch
    opts = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=fp32, precond=precond)
    o_w = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=fp32, precond=precond,
                             timing=0 if args.no_timing else every)
    warm = []
    u = torch.as_tensor(w.u0).cuda()
    un = torch.empty(w.nsp, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        warm.append(st.st_solve_slab(w.h, u, 0.0, w.dt, w.cfg["tol"], o_w, w.U, un, stream))
        u, un = un, u
    shares_w = [sum(s["kernel_us"][c] for s in warm) for c in range(len(st.KERNEL_CLASSES))]
    dom = max(range(len(shares_w)), key=lambda c: shares_w[c]) if warm and any(shares_w) else st.ST_K_MULTIDOT
    el, lat, stats = run_slabs(w, opts, steps, stream, timing_cls=None if args.no_timing else dom)
    tot = sum(shares_w) or 1.0
    return dict(elapsed=el, lat=lat, stats=stats, dom=dom,
                shares={st.KERNEL_CLASSES[c]: round(shares_w[c] / tot, 4) for c in range(len(shares_w))})


def leg_summary(w, r, steps):
    import numpy as np
    stats, el = r["stats"], r["elapsed"]
    op_evals = sum(s["newton_its"] + 1 + s["gmres_its"] for s in stats)
    lat_ms = np.array(r["lat"]) * 1e3
    return dict(ms_per_slab=el * 1e3 / steps, slab_solves_per_s=steps / el,
                dof_operator_evals_per_s=op_evals * w.n / el,
                latency_ms_p50=float(np.percentile(lat_ms, 50)), latency_ms_p99=float(np.percentile(lat_ms, 99)),
                newton_its_per_slab=sum(s["newton_its"] for s in stats) / len(stats),
                gmres_its_per_slab=sum(s["gmres_its"] for s in stats) / len(stats))


def forms_leg(name, args, stream):
    """Plain FP64 and FP32-inner solves of the same slabs: the FP64 run steps
    from u0; every slab is solved in both forms from the FP64 run's state, each
    timed on its own; the FP32-inner slab is compared with the FP64 one.  The
    same slabs are also solved with the element-block Jacobi in both forms
    (timed on their own, compared with the plain FP64 slab)."""
    import numpy as np
    import torch
    from paper_2201_05800_amd import st
    w = Workload(name)
    try:
        o64 = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes)
        o32 = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=1)
        o64p = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, precond=1)
        o32p = st.st_default_opts(restart=args.restart, cgs_passes=args.cgs_passes, inner_fp32=1, precond=1)
        forms = (o64, o32, o64p, o32p)
        u = torch.as_tensor(w.u0).cuda()
        un = torch.empty(w.nsp, dtype=torch.float64, device="cuda")
        uns = [un] + [torch.empty_like(un) for _ in forms[1:]]
        Us = [w.U] + [torch.empty_like(w.U) for _ in forms[1:]]
        # warm-up of every form (first-call allocations, the block inverse)
        for o, U_, un_ in zip(forms, Us, uns):
            st.st_solve_slab(w.h, u, 0.0, w.dt, w.cfg["tol"], o, U_, un_, stream)
        t = [0.0] * len(forms)
        its = [[] for _ in forms]
        diffs = [[] for _ in forms]
        for _ in range(args.forms_steps):
            for i, (o, U_, un_) in enumerate(zip(forms, Us, uns)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s_ = st.st_solve_slab(w.h, u, 0.0, w.dt, w.cfg["tol"], o, U_, un_, stream)
                t[i] += time.perf_counter() - t0
                its[i].append(s_["gmres_its"])
            for i in range(1, len(forms)):
                diffs[i].append(float(torch.linalg.norm(Us[i] - w.U) / torch.linalg.norm(w.U)))
            u, uns[0] = uns[0], u
        k = args.forms_steps
        ms = [x * 1e3 / k for x in t]
        return dict(workload=w.cfg["workload"], unknowns_per_slab=w.n, slabs=k, tol=w.cfg["tol"],
                    fp64_ms_per_slab=ms[0], fp32_inner_ms_per_slab=ms[1],
                    fp32_inner_speedup=ms[0] / ms[1], fp64_gmres_its_per_slab=float(np.mean(its[0])),
                    fp32_inner_gmres_its_per_slab=float(np.mean(its[1])),
                    fp32_inner_vs_fp64_max_rel_diff=max(diffs[1]),
                    preconditioned=dict(fp64_ms_per_slab=ms[2], fp32_inner_ms_per_slab=ms[3],
                                        fp64_gmres_its_per_slab=float(np.mean(its[2])),
                                        fp32_inner_gmres_its_per_slab=float(np.mean(its[3])),
                                        fp64_vs_plain_max_rel_diff=max(diffs[2]),
                                        fp32_inner_vs_plain_max_rel_diff=max(diffs[3])),
                    note="each slab solved in both forms from the same state; relative 2-norm difference of the "
                         "solved slabs; reduced boxes of these workloads match the oracle within 1e-9 in both "
                         "forms (GPU tests)")
    finally:
        w.close()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (a slab, or a multi-slab system, per GPU; splitting one "
              "over several GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2201_05800_amd import st

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
    stream = torch.cuda.current_stream()
    w = Workload(args.config)
    cfg, n, dt = w.cfg, w.n, w.dt

    # the headline: K consecutive slabs in the selected form (HIP-event timing
    # of the dominant kernel class on one slab in eight: event pairs on every
    # launch of every slab made the slabs up to 35 % slower)
    r = timed_solve_leg(w, args, stream, fp32=args.fp32_inner)
    stats, elapsed = r["stats"], r["elapsed"]
    print(f"# headline: {elapsed * 1e3 / args.steps:.2f} ms/slab", file=sys.stderr, flush=True)
    op_evals = sum(s["newton_its"] + 1 + s["gmres_its"] for s in stats)
    value = op_evals * n / elapsed
    lat_ms = np.array(r["lat"]) * 1e3
    roof = roof_of(stats, r["dom"], KERNEL_NAMES.get(r["dom"], st.KERNEL_CLASSES[r["dom"]]))
    roof["traffic"] = measured_traffic(args.config, roof["kernel"].split(" ")[0])
    # the operator calls alone on this slab (st_residual, st_jvp): rates apart
    U = w.U
    up = torch.as_tensor(w.u0).cuda()
    v = torch.randn(n, generator=torch.Generator(device="cuda").manual_seed(3), device="cuda", dtype=torch.float64)
    R = torch.empty_like(v)
    rates = {}
    for op, fn in (("residual", lambda: st.st_residual(w.h, U, up, 0.0, dt, R, stream)),
                   ("jvp", lambda: st.st_jvp(w.h, U, 0.0, dt, v, R, 0, stream)),
                   ("jvp_fp32_inner", lambda: st.st_jvp(w.h, U, 0.0, dt, v, R, 1, stream))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        rates[op + "_dof_evals_per_s"] = n / (e0.elapsed_time(e1) / 20 * 1e-3)
    del v, R

    # element-block Jacobi right preconditioning: the same slabs, solved to
    # the same tolerance (nonlinear equations: the block of the Jacobian at
    # the mean state; element blocks of more than 1024 unknowns are skipped)
    precond = None
    npe = w.nv * cfg["Nt"] * (cfg["N"] + 1) ** cfg["dim"]
    if args.precond_leg and npe <= 1024:
        rp = timed_solve_leg(w, args, stream, fp32=args.fp32_inner, precond=1)
        timed_pc = [x for x in rp["stats"] if x["kernel_calls"][st.ST_K_PRECOND] > 0]
        us = sum(x["kernel_us"][st.ST_K_PRECOND] for x in timed_pc)
        calls = sum(x["kernel_calls"][st.ST_K_PRECOND] for x in timed_pc)
        by = sum(x["kernel_bytes"][st.ST_K_PRECOND] for x in timed_pc)
        precond = dict(
            method="element-block Jacobi, right preconditioning (B^-1 of the element diagonal block of the slab "
                   "Jacobian, the same in every element" +
                   ("" if cfg["kind"] in (st.ST_ADVECTION, st.ST_ADVDIFF_BR1) else ", taken at the mean state") + ")",
            speedup_vs_plain=elapsed / rp["elapsed"], **leg_summary(w, rp, args.steps),
            precond_kernel=dict(kernel="k_bjacobi_big", avg_launch_us=round(us / max(calls, 1), 3),
                                achieved_GBs=round(by / (us * 1e-6) / 1e9, 1) if us > 0 else None,
                                achieved_TFLOPs=round(2.0 * npe * n * calls / (us * 1e-6) / 1e12, 2) if us > 0 else None,
                                peak_TFLOPs=78.6, element_block=npe,
                                note="FP64 matrix cores, 2 npe FLOP per unknown; algorithmic bytes: direction in, "
                                     "result out (B^-1, npe^2 doubles, re-read by every block from L2 / MALL)"))
        print(f"# preconditioned: {precond['ms_per_slab']:.3f} ms/slab, {precond['gmres_its_per_slab']:.1f} "
              f"GMRES its/slab", file=sys.stderr, flush=True)

    # plain FP64 against FP32-inner on the 2D Euler vortex and this workload
    forms = None
    if args.forms_leg:
        forms = [forms_leg(nm, args, stream) for nm in ("euler2d", "ns3d")]
        print(f"# forms: {forms}", file=sys.stderr, flush=True)

    # the 2D advection-diffusion workload: 3.3 MB vectors, a basis of about
    # 100 MB, inside the 256 MB Infinity Cache (labelled cache resident)
    cache = None
    if args.cache_leg and args.config != "advdiff2d":
        wc = Workload("advdiff2d")
        try:
            rc = timed_solve_leg(wc, args, stream, steps=32)
            cr = roof_of(rc["stats"], rc["dom"], KERNEL_NAMES.get(rc["dom"], st.KERNEL_CLASSES[rc["dom"]]),
                         bound="cache_resident")
            cr["traffic"] = measured_traffic("advdiff2d", cr["kernel"].split(" ")[0])
            cache = dict(workload=wc.cfg["workload"], unknowns_per_slab=wc.n, slabs=32, tol=wc.cfg["tol"],
                         **leg_summary(wc, rc, 32), roofline=cr,
                         note="Krylov basis of about 100 MB: inside the 256 MB Infinity Cache, so the kernel "
                              "rate is not an HBM rate")
            if args.precond_leg:
                rcp = timed_solve_leg(wc, args, stream, precond=1, steps=32)
                cache["preconditioned"] = leg_summary(wc, rcp, 32)
        finally:
            wc.close()
        print(f"# cache resident: {cache['ms_per_slab']:.2f} ms/slab", file=sys.stderr, flush=True)

    slabs = None
    if args.slabs_leg:
        small = dict(CONFIGS["advdiff2d"], K=[16, 16])
        hs = make_handle(small)
        Xs = st.st_node_coords(hs, 2, (small["N"] + 1) ** 2)
        st.st_destroy(hs)
        u_small = initial_state(small, Xs).ravel()
        big = CONFIGS["advdiff2d"]
        hb = make_handle(big)
        u_big = initial_state(big, st.st_node_coords(hb, 2, (big["N"] + 1) ** 2)).ravel()
        st.st_destroy(hb)
        slabs = dict(note="M slabs from the same u^n: one coupled Newton-GMRES solve against M sequential "
                          "slab solves, both to the workload's tolerance",
                     precond="0 none, 1 element-block Jacobi slab by slab, 2 the same blocks with forward "
                             "substitution over the slabs",
                     advdiff2d_64x64=[multi_slab_bench(big, u_big, 1.0 / 128, 4, pc) for pc in (0, 1, 2)] +
                                     [multi_slab_bench(big, u_big, 1.0 / 128, 16, 2)],
                     small_16x16=[multi_slab_bench(small, u_small, 1.0 / 128, 8, 0)] +
                                 [multi_slab_bench(small, u_small, 1.0 / 128, M, pc) for M in (4, 8, 16, 32)
                                  for pc in (1, 2)])
        print(f"# slabs: {slabs}", file=sys.stderr, flush=True)
    bubble = bubble_bench() if args.bubble_leg else None
    pulse = pulse_table_bench() if args.pulse_leg else None

    serving = serving_bench(args.serve_requests) if args.serve_requests > 0 else None
    operators = operator_bench(args.operator_reps) if args.operators else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, w.u0, w.U.cpu().numpy(), dt, args.cpu_baseline_seconds)

    out = {
        "metric": "space-time DOF residual evals/s + slab solves/s, p50/p99 latency, % HBM peak",
        "value": value,
        "unit": "space-time DOF operator evals/s (residual + JVP evaluations during the slab solves)",
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
        "operator_calls_on_this_slab": rates,
        "kernel_time_share_of_warmup": r["shares"],
        # algorithmic bytes of the timed steps per kernel class (the library's
        # per-launch byte model, summed)
        "kernel_bytes_of_timed": {st.KERNEL_CLASSES[c]: sum(s["kernel_bytes"][c] for s in stats)
                                  for c in range(len(st.KERNEL_CLASSES))},
        "roofline": roof,
        "preconditioned": precond,
        "forms": forms,
        "cache_resident_advdiff2d": cache,
        "serving": serving,
        "multi_slab": slabs,
        "euler3d_bubble": bubble,
        "rotating_pulse_table": pulse,
        "operators": operators,
        "cpu_baseline": cpu,
    }
    w.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
