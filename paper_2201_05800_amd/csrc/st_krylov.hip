// st_krylov.hip -- Newton-GMRES vector kernels (FP64), batched over slabs.
//
// GMRES(m) with classical Gram-Schmidt: the k+1 projections of a new Krylov
// vector and its squared norm are one fused multi-dot (one pass over the
// basis); the correction is one fused multi-axpy pass that writes the next
// basis vector already normalised (its norm follows from the projections by
// Pythagoras); an optional second pass (CGS2) repeats both.  Reductions are deterministic and need no atomics:
// a producer kernel writes one row of partial sums per block, and the
// consumer kernel reduces that table in a fixed order -- redundantly in every
// block, so every block holds the same bits.  The Givens update of the
// Hessenberg least-squares problem and the stopping test run redundantly in
// every block of the last correction kernel; block 0 commits them to the
// device state, which no other block of that kernel reads, so the iteration
// never needs the host.
//
// Every kernel takes a table of VecSeg descriptors (one per slab); a slab's
// block count depends only on its own length, so its arithmetic is identical
// alone and in a batch.  The Gram-Schmidt kernels are instantiated per number
// of basis vectors NV = k + 1, with k the host's Arnoldi step index.
#include "st_krylov.hpp"

#include <array>
#include <cstring>
#include <utility>

namespace stdg {

namespace {

constexpr int NPART = MMAX + 2;   // partial slots per block row (multi-dot table)

// descriptor pointers are generic; loads through the global address space
// give global_load instructions (no flat-address waits)
template <class T>
DI __attribute__((address_space(1))) T* gl(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
template <class T>
DI const __attribute__((address_space(1))) T* gl(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

DI double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

DI int find_vseg(const VecSeg* segs, int nseg, int b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int VWAVES = VBLOCK / 64;

// Element-wise sweeps y_i = f(x_i) over one slab's vector: pairs of elements
// per 16-byte access where n is even and both vectors allow it (at most
// VMAXBLK blocks of a slab are resident, and with 8-byte accesses they leave
// the memory pipeline half idle: measured 3.4 against 5.4 TB/s for the FP32
// cast of 50 M values), else one element per access; UNP accesses per thread
// and loop step.  Either way each y_i is f(x_i), bit for bit.
constexpr int UNP = 4;
typedef double v2d __attribute__((ext_vector_type(2)));    // a pair of elements (16 bytes)
typedef float v2f __attribute__((ext_vector_type(2)));
template <class X, class Y, class F>
DI void map_sweep(const X* x, Y* y, int64_t n, int64_t t0, int64_t stride, F f) {
    using X2 = typename std::conditional<sizeof(X) == 8, v2d, v2f>::type;
    using Y2 = typename std::conditional<sizeof(Y) == 8, v2d, v2f>::type;
    const bool pairs = (n & 1) == 0 && ((uintptr_t)x % sizeof(X2)) == 0 && ((uintptr_t)y % sizeof(Y2)) == 0;
    if (pairs) {
        const auto* __restrict__ x2 = gl((const X2*)x);
        auto* __restrict__ y2 = gl((Y2*)y);
        const int64_t np = n >> 1;
        for (int64_t i = t0; i < np; i += UNP * stride) {
            X2 a[UNP];
#pragma unroll
            for (int q = 0; q < UNP; ++q)
                if (i + q * stride < np) a[q] = x2[i + q * stride];
#pragma unroll
            for (int q = 0; q < UNP; ++q)
                if (i + q * stride < np) {
                    Y2 b;
                    b.x = f(a[q].x);
                    b.y = f(a[q].y);
                    store_nt(&y2[i + q * stride], b);
                }
        }
    } else {
        const auto* __restrict__ x1 = gl(x);
        auto* __restrict__ y1 = gl(y);
        for (int64_t i = t0; i < n; i += UNP * stride) {
            X a[UNP];
#pragma unroll
            for (int q = 0; q < UNP; ++q)
                if (i + q * stride < n) a[q] = x1[i + q * stride];
#pragma unroll
            for (int q = 0; q < UNP; ++q)
                if (i + q * stride < n) store_nt(&y1[i + q * stride], f(a[q]));
        }
    }
}

// Block reduction of NV per-thread values; returns with sums in out[0..NV)
// (waves added in a fixed order).  smem: VWAVES * NV doubles.
template <int NV>
DI void block_sums(const double (&acc)[NV], double* smem, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0) smem[wave * NV + i] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int i = threadIdx.x;
        double s = smem[i];
#pragma unroll
        for (int q = 1; q < VWAVES; ++q) s += smem[q * NV + i];
        out[i] = s;
    }
    __syncthreads();
}

// Column sums of a partial table P[b * ld + c] (b < nb <= VMAXBLK, c < NVAL), in
// the same fixed order in every block; result in s_out[0..NVAL).  Every
// thread issues all of its loads before adding (they come from other XCDs).
// s_tmp: VBLOCK doubles.
template <int NVAL>
DI void reduce_table(const __attribute__((address_space(1))) double* P, int ld, int nb, double* s_tmp,
                     double* s_out) {
    constexpr int G = (VBLOCK / NVAL) < 64 ? (VBLOCK / NVAL) : 64;
    constexpr int MAXR = (VMAXBLK + G - 1) / G;
    const int c = threadIdx.x % NVAL, r = threadIdx.x / NVAL;
    double a = 0.0;
    if (r < G) {
        double v[MAXR];
#pragma unroll
        for (int q = 0; q < MAXR; ++q) {
            const int b = r + q * G;
            v[q] = b < nb ? P[(int64_t)b * ld + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < MAXR; ++q) a += v[q];
    }
    s_tmp[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x < NVAL) {
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) s += s_tmp[g * NVAL + threadIdx.x];
        s_out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Elements per thread and loop step of the Gram-Schmidt sweeps: as many as
// keep the basis entries of all of them in registers at two waves per SIMD
// (the launches hold at most two blocks per CU), so that a thread issues its
// loads in few rounds.
template <int NV>
constexpr int sweep_unroll() { return NV <= 13 ? 4 : (NV <= 18 ? 3 : (NV <= 27 ? 2 : 1)); }

// The Gram-Schmidt sweeps move one element (double) or, where n is even
// and the vectors allow 16-byte accesses, a pair of elements (v2d) per
// access: a wave then moves 1 KB per load instruction, which the at most
// VMAXBLK blocks of a slab need to keep HBM busy.  Pairs per thread and loop
// step: two pairs up to 16 basis vectors, one pair up to 27 (about the
// registers of the element sweeps), none (element accesses) beyond, where a
// thread takes one element per step and a pair would double its registers.
template <int NV>
constexpr int sweep_unroll_pairs() { return NV <= 16 ? 2 : (NV <= 27 ? 1 : 0); }
DI double zero_of(double) { return 0.0; }
DI v2d zero_of(v2d) { return v2d{0.0, 0.0}; }
DI double dot_of(double a, double b) { return a * b; }
DI double dot_of(v2d a, v2d b) { return a.x * b.x + a.y * b.y; }
DI void sub_scaled(double& w, double h, double a) { w -= h * a; }
DI void sub_scaled(v2d& w, double h, v2d a) { w.x -= h * a.x; w.y -= h * a.y; }
DI double scaled(double s, double w) { return s * w; }
DI v2d scaled(double s, v2d w) { return v2d{s * w.x, s * w.y}; }

// Basis entries V_i[t + q stride] (i < NV, q < UN) and w[t + q stride], in
// units of E (n of them per vector); zero past the end.  All loads are
// issued before any is used.  NTL: non-temporal loads, for bases larger
// than the Infinity Cache holds (they would only evict each other there).
template <bool NTL, class E>
DI E load_v(const __attribute__((address_space(1))) E* p) {
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}
template <int NV, int UN, bool NTL, class E>
DI void load_group(const __attribute__((address_space(1))) E* V, const __attribute__((address_space(1))) E* w,
                   int64_t n, int64_t t, int64_t stride, E (&a)[UN][NV], E (&wv)[UN]) {
#pragma unroll
    for (int q = 0; q < UN; ++q) {
        const int64_t tq = t + q * stride;
        const bool p = tq < n;
#pragma unroll
        for (int i = 0; i < NV; ++i) a[q][i] = p ? load_v<NTL>(&V[(int64_t)i * n + tq]) : zero_of(E{});
        wv[q] = p ? load_v<NTL>(&w[tq]) : zero_of(E{});
    }
}
// pairs where n is even and the vectors are 16-byte aligned
DI bool use_pairs(int64_t n, const void* V, const void* w) {
    return (n & 1) == 0 && ((uintptr_t)V & 15) == 0 && ((uintptr_t)w & 15) == 0;
}

}  // namespace

// Partial sums of ||R||^2 (one per block) -> part2.
__global__ __launch_bounds__(VBLOCK) void k_rnorm(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double smem[VWAVES];
    __shared__ double s_out[1];
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const auto* __restrict__ R = gl((const double*)sg.R);
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    for (int64_t i = (int64_t)lb * VBLOCK + threadIdx.x; i < sg.n; i += 4 * stride) {
        double r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = i + q * stride < sg.n ? R[i + q * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[0] += r[q] * r[q];
    }
    block_sums<1>(acc, smem, s_out);
    if (threadIdx.x == 0) gl(sg.part2)[lb] = s_out[0];
}

// Start of an outer iteration (one block per slab): ||R|| from the partials,
// the stopping threshold on the first iteration, and the GMRES cycle state
// beta = ||R||, g = beta e1, k = 0, eta_abs = max(eta_rel beta, eta_tgt target).
__global__ __launch_bounds__(VBLOCK) void k_begin(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double s_tmp[VBLOCK];
    __shared__ double s_out[1];
    if (blockIdx.x >= nseg) return;
    const VecSeg& sg = segs[blockIdx.x];
    reduce_table<1>(gl((const double*)sg.part2), 1, sg.nblk, s_tmp, s_out);
    if (threadIdx.x != 0) return;
    GState* st = sg.st;
    const double nr2 = s_out[0];
    const double nr = sqrt(nr2);
    if (st->outer == 0) st->target = sg.tol * (nr > 1.0 ? nr : 1.0);
    st->outer += 1;
    st->rnorm = nr;
    st->beta = nr;
    st->k = 0;
    st->kfinal = 0;
    st->iters = 0;
    st->g[0] = nr;
    const double ea = sg.eta_rel * nr, ef = sg.eta_tgt * st->target;
    st->eta_abs = ea > ef ? ea : ef;
    st->reorth = 0;
    st->nonfinite = !isfinite(nr2);
    int stop = st->nonfinite ? 2 : (nr <= st->target ? 1 : 0);
    if (!stop && sg.dev_stop) {
        const int taken = st->outer - 1;     // Newton updates before this residual
        if (taken >= sg.max_newton) stop = 3;
        else if (taken == 0 || nr < 0.9 * st->best) { st->best = nr; st->stall = 0; }
        else if (++st->stall >= 8) stop = 3;
    }
    st->stop = stop;
    st->done = stop != 0;
}

// V_0 = -R / beta
__global__ __launch_bounds__(VBLOCK) void k_scale_v0(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    if (sg.st->done) return;
    const int lb = blockIdx.x - sg.blk0;
    const double s = -1.0 / sg.st->beta;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    map_sweep((const double*)sg.R, sg.V, sg.n, (int64_t)lb * VBLOCK + threadIdx.x, stride,
              [s](double r) { return s * r; });
}

// Projections V_i . w (i < NV) and w . w of one Gram-Schmidt pass, as one
// row of partial sums per block -> part.  The loads of every thread's first
// elements are in flight before the cycle state is read, except with gate
// set (a pass that usually finds its step finished: the state is read first).
template <int NV, bool NTL>
__global__ __launch_bounds__(VBLOCK) void k_multidot(const VecSeg* __restrict__ segs, int nseg, int gate) {
    __shared__ double smem[VWAVES * (NV + 1)];
    __shared__ double s_out[NV + 1];
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    const GState* st = sg.st;
    double acc[NV + 1];
    // the loads of every thread's first elements are issued before the
    // cycle state is read
    auto sweep = [&](auto e_tag, auto un_tag) -> bool {
        using E = decltype(e_tag);
        constexpr int UN = decltype(un_tag)::value;
        constexpr int W = sizeof(E) / sizeof(double);
        const int64_t n = sg.n / W;
        const auto* __restrict__ V = gl((const E*)sg.V);
        const auto* __restrict__ w = gl((const E*)sg.w);
        int64_t t = (int64_t)lb * VBLOCK + threadIdx.x;
        E a[UN][NV], wv[UN];
        if (gate && (st->done || !st->reorth)) return false;
        load_group<NV, UN, NTL>(V, w, n, t, stride, a, wv);
        if (st->done || st->k != NV - 1) return false;
        auto accumulate = [&](bool first) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                double s = dot_of(a[0][i], wv[0]);
#pragma unroll
                for (int q = 1; q < UN; ++q) s += dot_of(a[q][i], wv[q]);
                acc[i] = first ? s : acc[i] + s;
            }
            double s = dot_of(wv[0], wv[0]);
#pragma unroll
            for (int q = 1; q < UN; ++q) s += dot_of(wv[q], wv[q]);
            acc[NV] = first ? s : acc[NV] + s;
        };
        accumulate(true);
        for (t += UN * stride; t < n; t += UN * stride) {
            load_group<NV, UN, NTL>(V, w, n, t, stride, a, wv);
            accumulate(false);
        }
        return true;
    };
    constexpr int UP = sweep_unroll_pairs<NV>();
    bool run;
    if constexpr (UP > 0) {
        run = use_pairs(sg.n, sg.V, sg.w) ? sweep(v2d{}, std::integral_constant<int, UP>{})
                                          : sweep(double{}, std::integral_constant<int, sweep_unroll<NV>()>{});
    } else {
        run = sweep(double{}, std::integral_constant<int, sweep_unroll<NV>()>{});
    }
    if (!run) return;
    block_sums<NV + 1>(acc, smem, s_out);
    if (threadIdx.x <= NV) gl(sg.part)[(int64_t)lb * NPART + threadIdx.x] = s_out[threadIdx.x];
}

// One Gram-Schmidt correction with h = the column sums of the multi-dot
// table (every block reduces it the same way).
//  * not the last pass: w -= sum_i h_i V_i; block 0 accumulates h into the
//    Arnoldi column (hacc) and, on pass 0, keeps ||w||^2 (breakdown test).
//  * adaptive pass 0 (last = 2): the last pass unless the corrected vector's
//    norm by Pythagoras, h_{k+1,k}^2 = w.w - sum_i h_i^2, falls below
//    REORTH w.w -- then the cancellation would leave the new vector neither
//    normalised nor orthogonal to working precision, so the pass acts as a
//    first pass and the second pass (enqueued always, exiting at once when
//    the step is finished) repeats the projection: selective
//    reorthogonalisation, classical Gram-Schmidt twice where once is not
//    enough.
//  * last pass: the new norm follows from the multi-dot's w.w slot,
//    h_{k+1,k}^2 = w.w - sum_i h_i^2 (the basis is orthonormal), so the
//    Givens rotation of column k, the residual estimate and the stopping test
//    are known before the sweep; unless the cycle ends here the sweep writes
//    V_{k+1} = (w - sum_i h_i V_i) / h_{k+1,k} directly.  Every block
//    computes the same column; block 0 commits it.
// State written by block 0 here (done, k, H, rotations, g[k+1]) is never read
// by another block of this kernel; a block that sees done = 1 set here skips
// a sweep whose result is not needed.  Every thread's first elements are
// loaded while the table is reduced.
// reorthogonalise when ||w - V h||^2 < ||w||^2 / 2: the criterion of Daniel,
// Gragg, Kaufman and Stewart (1976), under which a second classical pass
// restores orthogonality to working precision ("twice is enough")
constexpr double REORTH = 0.5;

template <int NV, class E, int UN, bool NTL>
DI void update_body(const VecSeg& sg, GState* st, int lb, int64_t stride, int pass, int last, double* s_tmp,
                    double* s_h, double* s_col, double* s_cs, double* s_sn, double* s_hacc, double* s_misc) {
    constexpr int k = NV - 1;
    constexpr int W = sizeof(E) / sizeof(double);
    const int64_t n = sg.n;                // elements
    const int64_t ne = n / W;              // units of E
    const auto* __restrict__ V = gl((const E*)sg.V);
    auto* __restrict__ w = gl((E*)sg.w);
    const int ti = threadIdx.x;
    // The cycle state this kernel reads is requested before the vectors:
    // loads complete in order, so waiting for the state then does not wait
    // for the vectors, and the table loads below go out while the vectors
    // are still in flight.
    const auto* sr = gl((const GState*)st);
    // the gated second pass of the adaptive form (last = 3) reads the state
    // before it loads: it usually finds that pass 0 finished the step.  (The
    // flag is written by pass 0's launch only; k and done may change within
    // this launch, where block 0 commits the step.)
    if (last == 3 && (sr->done || !sr->reorth)) return;
    if (last == 3) last = 1;
    const int done = sr->done;
    // g_k, the absolute tolerance and ||w||^2 of pass 0, one per thread
    const double misc_i = !last ? 0.0 : (ti == 0 ? sr->g[k] : (ti == 1 ? sr->eta_abs : (ti == 2 && pass > 0 ? sr->wn0 : 0.0)));
    const double cs_i = (last && ti < k) ? sr->cs[ti] : 0.0;
    const double sn_i = (last && ti < k) ? sr->sn[ti] : 0.0;
    const double hacc_i = (pass > 0 && ti < NV) ? sr->hacc[ti] : 0.0;
    int64_t t = (int64_t)lb * VBLOCK + ti;
    E a[UN][NV], wv[UN];
    load_group<NV, UN, NTL>(V, w, ne, t, stride, a, wv);
    if (done) return;
    if (ti < NV) {
        s_cs[ti] = cs_i;
        s_sn[ti] = sn_i;
        s_hacc[ti] = hacc_i;
    }
    if (ti < 3) s_misc[ti] = misc_i;
    reduce_table<NV + 1>(gl((const double*)sg.part), NPART, sg.nblk, s_tmp, s_h);   // (block barriers)
    double h[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = s_h[i];
    const double ww = s_h[NV];

    double scale = 1.0;                 // 1 / h_{k+1,k} on the last pass
    auto* __restrict__ dst = w;         // where the corrected vector goes (units of E)
    bool fin = last != 0;
    if (last == 2) {
        double hn2 = ww;
#pragma unroll
        for (int i = 0; i < NV; ++i) hn2 -= h[i] * h[i];
        fin = hn2 > REORTH * ww;         // same bits in every block; NaN: the second pass decides
    }
    if (last == 2 && lb == 0 && ti == 0) st->reorth = fin ? 0 : 1;
    if (!fin) {
        if (lb == 0 && ti <= NV) {
            if (ti < NV) st->hacc[ti] = s_hacc[ti] + s_h[ti];
            else if (pass == 0) st->wn0 = ww;
            if (ti == 0) {
                st->kbytes[3] += 8.0 * (double)(NV + 1) * (double)n;   // this pass's multi-dot
                st->kbytes[4] += 8.0 * (double)(NV + 2) * (double)n;   // and correction (w in place)
            }
        }
    } else {
        // Arnoldi column k (earlier passes were committed by earlier kernels)
        double hn2 = ww;
#pragma unroll
        for (int i = 0; i < NV; ++i) hn2 -= h[i] * h[i];
        const double wn0 = pass == 0 ? ww : s_misc[2];
        const bool cancel = !(hn2 > 1e-12 * ww);       // Pythagoras lost to round-off
        const double hn = cancel ? 0.0 : sqrt(hn2);
        if (ti == 0) {
            double col[NV + 1];
            for (int i = 0; i < NV; ++i) col[i] = s_hacc[i] + h[i];
            col[NV] = hn;
            for (int i = 0; i < k; ++i) {
                const double a = col[i], b = col[i + 1];
                col[i] = s_cs[i] * a + s_sn[i] * b;
                col[i + 1] = -s_sn[i] * a + s_cs[i] * b;
            }
            for (int i = 0; i <= NV; ++i) s_col[i] = col[i];
        }
        __syncthreads();
        const double a = s_col[k];
        const double den = sqrt(a * a + hn * hn);
        const double c = den > 0.0 ? a / den : 1.0;
        const double sn = den > 0.0 ? hn / den : 0.0;
        const double gk = s_misc[0];
        const double gk1 = -sn * gk;
        const double res = fabs(gk1);
        const bool nonfin = !isfinite(ww) || !isfinite(res) || !isfinite(den);
        const bool breakdown = cancel || hn <= 1e-14 * sqrt(wn0);
        const bool stop = nonfin || res <= s_misc[1] || breakdown || k + 1 >= sg.m;
        if (lb == 0 && ti == 0) {
            double* H = st->H;
            for (int i = 0; i < k; ++i) H[i * MMAX + k] = s_col[i];
            H[k * MMAX + k] = den;
            st->cs[k] = c;
            st->sn[k] = sn;
            st->g[k + 1] = gk1;       // read by the next step's kernel only
            st->gr[k] = c * gk;
            st->iters += 1;
            st->iters_total += 1;
            st->kbytes[3] += 8.0 * (double)(NV + 1) * (double)n;   // multi-dot: V_0..V_k and w
            st->kbytes[4] += 8.0 * (double)(NV + 2) * (double)n;   // update: V_0..V_k, w, V_{k+1}
            if (nonfin) {
                st->nonfinite = 1;
                st->done = 1;
                st->kfinal = k;          // drop the broken column
            } else if (stop) {
                st->done = 1;
                st->kfinal = k + 1;
            } else {
                st->k = k + 1;
            }
        }
        if (stop) return;
        scale = 1.0 / hn;
        dst = gl((E*)(sg.V + (int64_t)(k + 1) * n));
    }
    auto correct = [&]() {
#pragma unroll
        for (int q = 0; q < UN; ++q) {
#pragma unroll
            for (int i = 0; i < NV; ++i) sub_scaled(wv[q], h[i], a[q][i]);
            if (t + q * stride < ne) store_nt(&dst[t + q * stride], scaled(scale, wv[q]));
        }
    };
    correct();
    for (t += UN * stride; t < ne; t += UN * stride) {
        load_group<NV, UN, NTL>(V, w, ne, t, stride, a, wv);
        correct();
    }
}

template <int NV, bool NTL>
__global__ __launch_bounds__(VBLOCK) void k_update(const VecSeg* __restrict__ segs, int nseg, int pass,
                                                   int last) {
    __shared__ double s_tmp[VBLOCK];
    __shared__ double s_h[NV + 1];
    __shared__ double s_col[NV + 1];
    __shared__ double s_cs[NV], s_sn[NV], s_hacc[NV];     // Givens rotations and the Arnoldi column so far
    __shared__ double s_misc[3];                          // g_k, eta_abs, ||w||^2 of pass 0
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    GState* st = sg.st;
    const int lb = blockIdx.x - sg.blk0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    constexpr int UP = sweep_unroll_pairs<NV>();
    if constexpr (UP > 0) {
        if (use_pairs(n, sg.V, sg.w)) {
            update_body<NV, v2d, UP, NTL>(sg, st, lb, stride, pass, last, s_tmp, s_h, s_col, s_cs, s_sn, s_hacc,
                                     s_misc);
            return;
        }
    }
    update_body<NV, double, sweep_unroll<NV>(), NTL>(sg, st, lb, stride, pass, last, s_tmp, s_h, s_col, s_cs, s_sn,
                                                s_hacc, s_misc);
}

// y = H(0:kf, 0:kf)^-1 gr(0:kf) by back substitution; one block per segment
// (the triangle is staged in LDS by the whole block first).
__global__ __launch_bounds__(BLOCK) void k_finish(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double sH[MMAX * MMAX];
    __shared__ double sg[MMAX];
    if (blockIdx.x >= nseg) return;
    GState* st = segs[blockIdx.x].st;
    const int kf = st->kfinal;
    // all loads in flight at once (the state was written from another XCD)
    double v[MMAX * MMAX / BLOCK];
#pragma unroll
    for (int q = 0; q < MMAX * MMAX / BLOCK; ++q) {
        const int i = threadIdx.x + q * BLOCK;
        v[q] = i < kf * MMAX ? st->H[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < MMAX * MMAX / BLOCK; ++q) sH[threadIdx.x + q * BLOCK] = v[q];
    if (threadIdx.x < kf) sg[threadIdx.x] = st->gr[threadIdx.x];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double y[MMAX];
    for (int i = kf - 1; i >= 0; --i) {
        double s = sg[i];
        for (int j = i + 1; j < kf; ++j) s -= sH[i * MMAX + j] * y[j];
        y[i] = s / sH[i * MMAX + i];
    }
    for (int i = 0; i < kf; ++i) st->y[i] = y[i];
}

// U += sum_{i < kfinal} y_i V_i
__global__ __launch_bounds__(VBLOCK) void k_update_u(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double s_y[MMAX];
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const GState* st = sg.st;
    const int kf = st->kfinal;
    if (kf == 0) return;
    if (threadIdx.x < MMAX) s_y[threadIdx.x] = threadIdx.x < kf ? st->y[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = blockIdx.x - sg.blk0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    const auto* __restrict__ V = gl((const double*)sg.V);
    auto* __restrict__ U = gl(sg.U);
    for (int64_t t = (int64_t)lb * VBLOCK + threadIdx.x; t < n; t += stride) {
        double u = U[t];
        // groups of 8 independent loads; indices past kf re-read V_{kf-1} with weight 0
        for (int i0 = 0; i0 < kf; i0 += 8) {
            double a[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = i0 + j < kf ? i0 + j : kf - 1;
                a[j] = V[(int64_t)i * n + t];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) u += s_y[i0 + j < MMAX ? i0 + j : MMAX - 1] * (i0 + j < kf ? a[j] : 0.0);
        }
        U[t] = u;
    }
}

// U = 1 (x) u_prev (initial guess of the Newton iteration)
__global__ __launch_bounds__(VBLOCK) void k_init_guess(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t blkn = (int64_t)sg.nt * sg.ns;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    for (int64_t i = (int64_t)lb * VBLOCK + threadIdx.x; i < sg.n; i += stride) {
        const int64_t ev = i / blkn;
        const int64_t s = i % sg.ns;
        sg.U[i] = sg.uprev[ev * sg.ns + s];
    }
}

// u_next = (e_Nt^T (x) I) U (eq. (un))
__global__ __launch_bounds__(VBLOCK) void k_extract_last(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t nsp = sg.n / sg.nt;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    for (int64_t i = (int64_t)lb * VBLOCK + threadIdx.x; i < nsp; i += stride) {
        const int64_t ev = i / sg.ns;
        const int64_t s = i % sg.ns;
        sg.unext[i] = sg.U[(ev * sg.nt + (sg.nt - 1)) * sg.ns + s];
    }
}

// U32 = fl(U)
__global__ __launch_bounds__(VBLOCK) void k_cast32(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    map_sweep((const double*)sg.U, sg.U32, sg.n, (int64_t)lb * VBLOCK + threadIdx.x, stride,
              [](double u) { return (float)u; });
}

// Embedded error estimate (Sec. "Algorithmic Aspects", adaptive time-stepping;
// eqs. RK_stage_equations, RK_solution, SBP_to_RK).  The embedded solution
// u_hat = u^n + dt (gamma_0 F(u^n) + sum_l b_hat_l K_l) has
//   Nt = 2: gamma_0 = 0, b_hat = (1, 0): b - b_hat is minus the first row of
//           A, so the first stage equation gives e = -(U_1 - u^n);
//   Nt > 2: gamma_0 = b_1, b_hat = (0, b_2, ..): e = b_1 dt (K_1 - F(u^n)),
//           with b_1 dt K_1 = w_1 (D_tau (U - 1 u^n))_1 + (U_1 - u^n) from
//           A^-1 = 2 (D_tau + M_tau^-1 e_1 e_1^T), and b_1 dt F(u^n) the first
//           time node of fs.
// Partial sums of the squared scaled values per block.
__global__ __launch_bounds__(VBLOCK) void k_errest(EstArgs a) {
    __shared__ double smem[VWAVES];
    __shared__ double s_out[1];
    const auto* __restrict__ U = gl(a.U);
    const auto* __restrict__ up = gl(a.up);
    const auto* __restrict__ fs = gl(a.fs);
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)a.nblk * VBLOCK;
    const bool narrow = a.nsp <= 0xffffffffLL;     // 32-bit division suffices
    for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < a.nsp; i += stride) {
        const int64_t ev = narrow ? (int64_t)((uint32_t)i / (uint32_t)a.ns) : i / a.ns;
        const int64_t s = i - ev * a.ns;
        const int64_t base = ev * a.nt * a.ns + s;
        const double u1 = U[base];                               // first time node
        const double uN = U[base + (int64_t)(a.nt - 1) * a.ns];  // u^{n+1}
        const double un = up[i];
        double e;
        if (a.nt == 2) {
            e = un - u1;
        } else {
            double k1 = a.c[0] * (u1 - un);
            for (int j = 1; j < a.nt; ++j) k1 += a.c[j] * (U[base + (int64_t)j * a.ns] - un);
            e = (k1 + (u1 - un)) - a.fsw * fs[i];
        }
        const double sc = a.atol + a.rtol * fmax(fabs(un), fabs(uN));
        const double r = e / sc;
        acc[0] += r * r;
    }
    block_sums<1>(acc, smem, s_out);
    if (threadIdx.x == 0) gl(a.part)[blockIdx.x] = s_out[0];
}
// the partial sums in a fixed order, then the root mean square
__global__ __launch_bounds__(VBLOCK) void k_errest_final(EstArgs a) {
    __shared__ double s_tmp[VBLOCK];
    __shared__ double s_out[1];
    reduce_table<1>(gl((const double*)a.part), 1, a.nblk, s_tmp, s_out);
    if (threadIdx.x == 0) gl(a.out)[0] = sqrt(s_out[0] / (double)a.nsp);
}

// out_m(first time node) += in_{m-1}(last time node), m = 1 .. slabs - 1
__global__ __launch_bounds__(VBLOCK) void k_couple(CoupleArgs a) {
    if (a.skip && *gl(a.skip)) return;
    const int64_t k = a.kp ? (int64_t)*gl(a.kp) : 0;
    const auto* __restrict__ in = gl(a.in0 + k * a.ld);
    auto* __restrict__ out = gl(a.out);
    const int64_t total = (int64_t)(a.slabs - 1) * a.nsp;
    const int64_t blk = (int64_t)a.nt * a.ns;
    for (int64_t i = (int64_t)blockIdx.x * VBLOCK + threadIdx.x; i < total; i += (int64_t)a.nblk * VBLOCK) {
        const int64_t m = i / a.nsp;                    // source slab
        const int64_t r = i - m * a.nsp;
        const int64_t ev = r / a.ns;                    // (element, variable)
        const int64_t s = r - ev * a.ns;
        out[(m + 1) * a.n + ev * blk + s] += in[m * a.n + ev * blk + (a.nt - 1) * a.ns + s];
    }
}

// Descriptor uploads in stream order: the descriptor (or a 2 KB chunk of
// it) is the kernel's first argument, so it sits at the start of the
// kernel-argument segment, and the threads copy its 8-byte words in parallel
// (one thread copying a 3 KB operator descriptor took about 8 us).
template <class S>
__global__ void k_put_desc(S v, S* dst) {
    static_assert(sizeof(S) % 8 == 0, "descriptor of whole 8-byte words");
    (void)v;
    const auto* src = (const __attribute__((address_space(4))) uint64_t*)__builtin_amdgcn_kernarg_segment_ptr();
    auto* d = (__attribute__((address_space(1))) uint64_t*)dst;
    for (int i = threadIdx.x; i < (int)(sizeof(S) / 8); i += blockDim.x) d[i] = src[i];
}
struct DescChunk {
    uint64_t w[256];
};
__global__ void k_put_chunk(DescChunk v, uint64_t* dst, int nw) {
    (void)v;
    const auto* src = (const __attribute__((address_space(4))) uint64_t*)__builtin_amdgcn_kernarg_segment_ptr();
    auto* d = (__attribute__((address_space(1))) uint64_t*)dst;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) d[i] = src[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define LAUNCH_V(K, G, ...) launch_k(K, dim3(G), dim3(VBLOCK), st, __VA_ARGS__)

LaunchTiming& launch_timing() {
    static thread_local LaunchTiming lt;
    return lt;
}

namespace {
template <int NV, bool NTL>
void md_launch(const VecSeg* s, int nseg, int G, int gate, hipStream_t st) {
    LAUNCH_V((k_multidot<NV, NTL>), G, s, nseg, gate);
}
template <int NV, bool NTL>
void up_launch(const VecSeg* s, int nseg, int G, int pl, hipStream_t st) {
    LAUNCH_V((k_update<NV, NTL>), G, s, nseg, pl >> 2, pl & 3);
}
using VLaunch = void (*)(const VecSeg*, int, int, int, hipStream_t);
template <bool NTL, int... I>
constexpr std::array<VLaunch, sizeof...(I)> md_table(std::integer_sequence<int, I...>) {
    return {&md_launch<I + 1, NTL>...};
}
template <bool NTL, int... I>
constexpr std::array<VLaunch, sizeof...(I)> up_table(std::integer_sequence<int, I...>) {
    return {&up_launch<I + 1, NTL>...};
}
}  // namespace

void vk_rnorm(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_rnorm, G, s, nseg); }
void vk_begin(const VecSeg* s, int nseg, hipStream_t st) { LAUNCH_V(k_begin, nseg, s, nseg); }
void vk_scale_v0(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_scale_v0, G, s, nseg); }
void vk_multidot(const VecSeg* s, int nseg, int G, int k, hipStream_t st, int gate, int stream) {
    static const auto tbl = md_table<false>(std::make_integer_sequence<int, MMAX>{});
    static const auto tbl_nt = md_table<true>(std::make_integer_sequence<int, MMAX>{});
    (stream ? tbl_nt : tbl)[k](s, nseg, G, gate, st);
}
void vk_update(const VecSeg* s, int nseg, int G, int pass, int last, int k, hipStream_t st, int stream) {
    static const auto tbl = up_table<false>(std::make_integer_sequence<int, MMAX>{});
    static const auto tbl_nt = up_table<true>(std::make_integer_sequence<int, MMAX>{});
    (stream ? tbl_nt : tbl)[k](s, nseg, G, (pass << 2) | (last & 3), st);
}
void gs_pass_plan(int passes, int p, int* last, int* gate) {
    // passes 1: CGS1; 2: CGS2; 0: adaptive (pass 0 decides whether pass 1 runs)
    if (passes == 0) {
        *last = p == 0 ? 2 : 3;
        *gate = p == 1;
    } else {
        *last = p == passes - 1 ? 1 : 0;
        *gate = 0;
    }
}
void vk_finish(const VecSeg* s, int nseg, hipStream_t st) {
    launch_k(k_finish, dim3(nseg), dim3(BLOCK), st, s, nseg);
}
void vk_update_u(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_update_u, G, s, nseg); }
void vk_init_guess(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_init_guess, G, s, nseg); }
void vk_extract_last(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_extract_last, G, s, nseg); }
void vk_cast32(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_cast32, G, s, nseg); }
void vk_error_estimate(const EstArgs& a, hipStream_t st) {
    LAUNCH_V(k_errest, a.nblk, a);
    LAUNCH_V(k_errest_final, 1, a);
}
void vk_couple(const CoupleArgs& a, hipStream_t st) {
    if (a.slabs > 1) LAUNCH_V(k_couple, a.nblk, a);
}
void put_opseg(OpSeg* dst, const OpSeg& v, hipStream_t st) {
    static_assert(sizeof(OpSeg) % 8 == 0, "descriptor of whole 8-byte words");
    constexpr int NW = (int)(sizeof(OpSeg) / 8);
    const auto* src = reinterpret_cast<const uint64_t*>(&v);
    for (int w0 = 0; w0 < NW; w0 += 256) {
        DescChunk c;
        const int nw = NW - w0 < 256 ? NW - w0 : 256;
        std::memcpy(c.w, src + w0, sizeof(uint64_t) * nw);
        launch_k(k_put_chunk, dim3(1), dim3(256), st, c, reinterpret_cast<uint64_t*>(dst) + w0, nw);
    }
}
void put_vecseg(VecSeg* dst, const VecSeg& v, hipStream_t st) {
    launch_k(k_put_desc<VecSeg>, dim3(1), dim3(64), st, v, dst);
}

}  // namespace stdg
