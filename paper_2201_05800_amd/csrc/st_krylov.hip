// st_krylov.hip -- Newton-GMRES vector kernels (FP64), batched over slabs.
//
// GMRES(m) with classical Gram-Schmidt: the k+1 projections of the new
// Krylov vector are one fused multi-dot (one pass over the basis), the
// correction is one multi-axpy pass; an optional second pass (CGS2) repeats
// both.  Reductions are two-stage and deterministic: fixed per-block chunks,
// block partials, and a final reduction in fixed order by the last block to
// finish (device-scope ticket).  The Givens update of the Hessenberg least
// squares problem and the stopping test run in that last block, so the
// iteration never needs the host.  Every kernel takes a table of VecSeg
// descriptors (one per slab); a slab's block count depends only on its own
// length, so its arithmetic is identical alone and in a batch.
#include "st_krylov.hpp"

namespace stdg {

namespace {

constexpr int NPART = MMAX + 2;   // partial slots per block

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

// Reduce nval per-thread values over the block; thread i < nval of the
// block returns the block sum of value i in `out` (others unspecified).
template <int NMAX>
DI void block_sums(const double (&acc)[NMAX], int nval, double* smem /* [4][NMAX] */, double& out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
        if (i < nval) {
            double s = wave_sum(acc[i]);
            if (lane == 0) smem[wave * NMAX + i] = s;
        }
    }
    __syncthreads();
    out = 0.0;
    if (threadIdx.x < nval) {
        const int i = threadIdx.x;
        out = smem[i] + smem[NMAX + i] + smem[2 * NMAX + i] + smem[3 * NMAX + i];
    }
}

// Publish the block partials; returns true in the last block of the segment
// to arrive (which then sees every partial).
DI bool arrive_last(const VecSeg& sg, int lb, int nval, double bsum, bool* s_last) {
    if (threadIdx.x < nval) sg.part[(int64_t)lb * NPART + threadIdx.x] = bsum;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(&sg.st->ticket, 1u);
        *s_last = (t == (unsigned)sg.nblk - 1);
    }
    __syncthreads();
    if (*s_last) __threadfence();
    return *s_last;
}

// Fixed-order sum of partial slot i over the segment's blocks.
DI double final_sum(const VecSeg& sg, int i) {
    double s = 0.0;
    for (int b = 0; b < sg.nblk; ++b) s += sg.part[(int64_t)b * NPART + i];
    return s;
}

}  // namespace

// ||R||_2 and the start of a GMRES cycle: beta = ||R||, g = beta e1, k = 0,
// eta_abs = max(eta_rel beta, eta_floor).
__global__ __launch_bounds__(BLOCK) void k_norm_begin(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double smem[4 * 1];
    __shared__ bool s_last;
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < sg.n; i += stride) {
        const double r = sg.R[i];
        acc[0] += r * r;
    }
    double bs;
    block_sums<1>(acc, 1, smem, bs);
    if (!arrive_last(sg, lb, 1, bs, &s_last)) return;
    if (threadIdx.x == 0) {
        GState* st = sg.st;
        const double nr2 = final_sum(sg, 0);
        const double nr = sqrt(nr2);
        st->ticket = 0;
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
        st->nonfinite = !isfinite(nr2);
        st->done = (nr <= st->target) || st->nonfinite;
    }
}

// V_0 = -R / beta
__global__ __launch_bounds__(BLOCK) void k_scale_v0(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    if (sg.st->done) return;
    const int lb = blockIdx.x - sg.blk0;
    const double s = -1.0 / sg.st->beta;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < sg.n; i += stride) sg.V[i] = s * sg.R[i];
}

// Projections hp_i = V_i . w (i <= k) of one Gram-Schmidt pass; pass 0 also
// takes ||w||^2 before orthogonalisation (for the breakdown test).
__global__ __launch_bounds__(BLOCK) void k_multidot(const VecSeg* __restrict__ segs, int nseg, int pass) {
    __shared__ double smem[4 * NPART];
    __shared__ bool s_last;
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    GState* st = sg.st;
    if (st->done) return;
    const int k = st->k;
    const int nval = k + 2;
    const int lb = blockIdx.x - sg.blk0;
    double acc[NPART];
#pragma unroll
    for (int i = 0; i < NPART; ++i) acc[i] = 0.0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t t = (int64_t)lb * BLOCK + threadIdx.x; t < n; t += stride) {
        const double wv = sg.w[t];
#pragma unroll
        for (int i = 0; i < MMAX; ++i)
            if (i <= k) acc[i] += sg.V[(int64_t)i * n + t] * wv;
        acc[MMAX] += wv * wv;
    }
    // move the w.w slot next to the projections
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
        if (i == k + 1) acc[i] = acc[MMAX];
    double bs;
    block_sums<NPART>(acc, nval, smem, bs);
    if (!arrive_last(sg, lb, nval, bs, &s_last)) return;
    if (threadIdx.x < nval) {
        const int i = threadIdx.x;
        const double s = final_sum(sg, i);
        if (i <= k) {
            st->hp[i] = s;
            st->hacc[i] = (pass == 0 ? 0.0 : st->hacc[i]) + s;
        } else if (pass == 0) {
            st->wn0 = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) st->ticket = 0;
}

// w -= sum_i hp_i V_i; on the last pass the last block also finishes the
// Arnoldi column: h_{k+1,k} = ||w||, Givens rotations, residual estimate,
// stopping test, and 1/h_{k+1,k} for the normalisation.
__global__ __launch_bounds__(BLOCK) void k_update(const VecSeg* __restrict__ segs, int nseg, int last) {
    __shared__ double smem[4 * 1];
    __shared__ bool s_last;
    __shared__ double s_h[MMAX];
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    GState* st = sg.st;
    if (st->done) return;
    const int k = st->k;
    if (threadIdx.x < MMAX) s_h[threadIdx.x] = threadIdx.x <= k ? st->hp[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = blockIdx.x - sg.blk0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    double acc[1] = {0.0};
    for (int64_t t = (int64_t)lb * BLOCK + threadIdx.x; t < n; t += stride) {
        double wv = sg.w[t];
#pragma unroll
        for (int i = 0; i < MMAX; ++i)
            if (i <= k) wv -= s_h[i] * sg.V[(int64_t)i * n + t];
        sg.w[t] = wv;
        acc[0] += wv * wv;
    }
    double bs;
    block_sums<1>(acc, 1, smem, bs);
    if (!arrive_last(sg, lb, 1, bs, &s_last)) return;
    if (threadIdx.x != 0) return;
    st->ticket = 0;
    if (!last) return;
    const int m = sg.m;
    const double w2 = final_sum(sg, 0);
    const double hn = sqrt(w2);
    double* H = st->H;
    for (int i = 0; i <= k; ++i) H[i * MMAX + k] = st->hacc[i];
    H[(k + 1) * MMAX + k] = hn;
    for (int i = 0; i < k; ++i) {
        const double a = H[i * MMAX + k], b = H[(i + 1) * MMAX + k];
        H[i * MMAX + k] = st->cs[i] * a + st->sn[i] * b;
        H[(i + 1) * MMAX + k] = -st->sn[i] * a + st->cs[i] * b;
    }
    const double a = H[k * MMAX + k], b = hn;
    const double den = sqrt(a * a + b * b);
    const double c = den > 0.0 ? a / den : 1.0;
    const double s = den > 0.0 ? b / den : 0.0;
    st->cs[k] = c;
    st->sn[k] = s;
    H[k * MMAX + k] = den;
    H[(k + 1) * MMAX + k] = 0.0;
    const double gk = st->g[k];
    st->g[k + 1] = -s * gk;
    st->g[k] = c * gk;
    st->iters += 1;
    st->iters_total += 1;
    const double res = fabs(st->g[k + 1]);
    const bool nonfin = !isfinite(hn) || !isfinite(res) || !isfinite(den);
    const bool breakdown = hn <= 1e-14 * sqrt(st->wn0);
    if (nonfin) {
        st->nonfinite = 1;
        st->done = 1;
        st->kfinal = k;          // drop the broken column
    } else if (res <= st->eta_abs || breakdown || k + 1 >= m) {
        st->done = 1;
        st->kfinal = k + 1;
    } else {
        st->k = k + 1;
        st->inv = 1.0 / hn;
    }
}

// V_{k} = w / h_{k,k-1} (k already advanced by k_update)
__global__ __launch_bounds__(BLOCK) void k_normalize(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const GState* st = sg.st;
    if (st->done) return;
    const int lb = blockIdx.x - sg.blk0;
    const double s = st->inv;
    double* __restrict__ vk = sg.V + (int64_t)st->k * sg.n;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < sg.n; i += stride) vk[i] = s * sg.w[i];
}

// y = H(0:kf, 0:kf)^-1 g(0:kf) by back substitution; one block per segment.
__global__ void k_finish(const VecSeg* __restrict__ segs, int nseg) {
    if (blockIdx.x >= nseg || threadIdx.x != 0) return;
    GState* st = segs[blockIdx.x].st;
    const int kf = st->kfinal;
    for (int i = kf - 1; i >= 0; --i) {
        double s = st->g[i];
        for (int j = i + 1; j < kf; ++j) s -= st->H[i * MMAX + j] * st->y[j];
        st->y[i] = s / st->H[i * MMAX + i];
    }
}

// U += sum_{i < kfinal} y_i V_i
__global__ __launch_bounds__(BLOCK) void k_update_u(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double s_y[MMAX];
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const GState* st = sg.st;
    const int kf = st->kfinal;
    if (kf == 0) return;
    if (threadIdx.x < MMAX) s_y[threadIdx.x] = threadIdx.x < kf ? st->y[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = blockIdx.x - sg.blk0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t t = (int64_t)lb * BLOCK + threadIdx.x; t < n; t += stride) {
        double u = sg.U[t];
#pragma unroll
        for (int i = 0; i < MMAX; ++i)
            if (i < kf) u += s_y[i] * sg.V[(int64_t)i * n + t];
        sg.U[t] = u;
    }
}

// U = 1 (x) u_prev (initial guess of the Newton iteration)
__global__ __launch_bounds__(BLOCK) void k_init_guess(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t blkn = (int64_t)sg.nt * sg.ns;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < sg.n; i += stride) {
        const int64_t ev = i / blkn;
        const int64_t s = i % sg.ns;
        sg.U[i] = sg.uprev[ev * sg.ns + s];
    }
}

// u_next = (e_Nt^T (x) I) U (eq. (un))
__global__ __launch_bounds__(BLOCK) void k_extract_last(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t nsp = sg.n / sg.nt;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < nsp; i += stride) {
        const int64_t ev = i / sg.ns;
        const int64_t s = i % sg.ns;
        sg.unext[i] = sg.U[(ev * sg.nt + (sg.nt - 1)) * sg.ns + s];
    }
}

// U32 = fl(U)
__global__ __launch_bounds__(BLOCK) void k_cast32(const VecSeg* __restrict__ segs, int nseg) {
    const VecSeg& sg = segs[find_vseg(segs, nseg, blockIdx.x)];
    const int lb = blockIdx.x - sg.blk0;
    const int64_t stride = (int64_t)sg.nblk * BLOCK;
    for (int64_t i = (int64_t)lb * BLOCK + threadIdx.x; i < sg.n; i += stride) sg.U32[i] = (float)sg.U[i];
}

__global__ void k_put_opseg(OpSeg* dst, OpSeg v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }
__global__ void k_put_vecseg(VecSeg* dst, VecSeg v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define LAUNCH_V(K, G, ...) hipLaunchKernelGGL(K, dim3(G), dim3(BLOCK), 0, st, __VA_ARGS__)

void vk_norm_begin(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_norm_begin, G, s, nseg); }
void vk_scale_v0(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_scale_v0, G, s, nseg); }
void vk_multidot(const VecSeg* s, int nseg, int G, int pass, hipStream_t st) { LAUNCH_V(k_multidot, G, s, nseg, pass); }
void vk_update(const VecSeg* s, int nseg, int G, int last, hipStream_t st) { LAUNCH_V(k_update, G, s, nseg, last); }
void vk_normalize(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_normalize, G, s, nseg); }
void vk_finish(const VecSeg* s, int nseg, hipStream_t st) {
    hipLaunchKernelGGL(k_finish, dim3(nseg), dim3(64), 0, st, s, nseg);
}
void vk_update_u(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_update_u, G, s, nseg); }
void vk_init_guess(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_init_guess, G, s, nseg); }
void vk_extract_last(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_extract_last, G, s, nseg); }
void vk_cast32(const VecSeg* s, int nseg, int G, hipStream_t st) { LAUNCH_V(k_cast32, G, s, nseg); }
void put_opseg(OpSeg* dst, const OpSeg& v, hipStream_t st) {
    hipLaunchKernelGGL(k_put_opseg, dim3(1), dim3(64), 0, st, dst, v);
}
void put_vecseg(VecSeg* dst, const VecSeg& v, hipStream_t st) {
    hipLaunchKernelGGL(k_put_vecseg, dim3(1), dim3(64), 0, st, dst, v);
}

}  // namespace stdg
