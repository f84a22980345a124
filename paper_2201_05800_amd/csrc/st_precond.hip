// st_precond.hip -- element-block Jacobi preconditioner for the slab GMRES of
// the linear equations (right preconditioning).
//
// For advection and advection-diffusion on the uniform periodic mesh the
// slab Jacobian (eq. (Jacobian_ST)) is the same operator in every element:
// its diagonal block B (the coupling of an element's space-time unknowns to
// themselves, through the DG time discretisation, the volume terms and the
// element's own share of its face fluxes) is one npe x npe matrix.  GMRES
// then solves (J B^-1) y = -R and the Newton update is B^-1 (V y).  The
// host assembles B once per (handle, dt) by applying the operator kernel to
// unit vectors on a 3^d-element copy of the mesh, and inverts it (partial
// pivoting); the kernels here apply B^-1 to every element of a vector.
#include "st_krylov.hpp"

namespace stdg {

namespace {
template <class T>
DI __attribute__((address_space(1))) T* gp(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
template <class T>
DI const __attribute__((address_space(1))) T* gp(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <class Seg>
DI int find_pseg(const Seg* segs, int nseg, int b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}
constexpr int PC_BLOCK = 256;               // threads: 4 groups of 64
constexpr int PC_NPE_LARGE = 192;           // above: 8 elements per block (LDS)
}  // namespace

int pc_eb(int npe) { return npe <= PC_NPE_LARGE ? 16 : 8; }
int pc_blocks(int E, int npe) { return (E + pc_eb(npe) - 1) / pc_eb(npe); }

// out_e (+)= B^-1 in_e for PC_EB elements per block.  The block's inputs are
// staged in LDS transposed (unknown-major, element-fastest); wavefront g of
// the block takes elements [g PC_EG, (g+1) PC_EG) and, lane by lane, the rows
// of B^-1 (read column by column from L2, coalesced across the lanes).
template <int PC_EB>
__global__ __launch_bounds__(PC_BLOCK) void k_bjacobi(const PcSeg* __restrict__ segs, int nseg) {
    constexpr int PC_EG = PC_EB / 4;        // elements per wavefront
    extern __shared__ double tileT[];       // [npe][PC_EB]
    const PcSeg& sg = segs[find_pseg(segs, nseg, blockIdx.x)];
    if (sg.skip && *(const __attribute__((address_space(1))) int*)sg.skip) return;
    const int npe = sg.npe;
    const int e0 = (blockIdx.x - sg.blk0) * PC_EB;
    const int ne = min(PC_EB, sg.E - e0);
    const double* inb = static_cast<const double*>(sg.in.base);
    if (sg.in.kp) inb += (int64_t)(*(const __attribute__((address_space(1))) int*)sg.in.kp + sg.in.koff) * sg.in.ld;
    const auto* __restrict__ in = gp(inb) + (int64_t)e0 * npe;
    for (int t = threadIdx.x; t < PC_EB * npe; t += PC_BLOCK) {
        const int e = t / npe, j = t - e * npe;          // coalesced over the block's contiguous inputs
        tileT[j * PC_EB + e] = e < ne ? in[t] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const auto* __restrict__ B = gp(sg.binvT);
    auto* __restrict__ out = gp(sg.out) + (int64_t)e0 * npe;
    for (int r = lane; r < npe; r += 64) {
        double acc[PC_EG];
#pragma unroll
        for (int q = 0; q < PC_EG; ++q) acc[q] = 0.0;
#pragma unroll 4
        for (int j = 0; j < npe; ++j) {
            const double b = B[(int64_t)j * npe + r];
            const double* tv = tileT + j * PC_EB + g * PC_EG;
#pragma unroll
            for (int q = 0; q < PC_EG; ++q) acc[q] += b * tv[q];
        }
#pragma unroll
        for (int q = 0; q < PC_EG; ++q) {
            const int e = g * PC_EG + q;
            if (e < ne) {
                const int64_t i = (int64_t)e * npe + r;
                out[i] = sg.accumulate ? out[i] + acc[q] : acc[q];
            }
        }
    }
}

// w = sum_{i < kfinal} y_i V_i (the Krylov combination the preconditioned
// Newton update maps through B^-1)
__global__ __launch_bounds__(VBLOCK) void k_combine(const VecSeg* __restrict__ segs, int nseg) {
    __shared__ double s_y[MMAX];
    const VecSeg& sg = segs[find_pseg(segs, nseg, blockIdx.x)];
    const GState* st = sg.st;
    const int kf = st->kfinal;                  // 0: w = 0 (no update)
    if (threadIdx.x < MMAX) s_y[threadIdx.x] = threadIdx.x < kf ? st->y[threadIdx.x] : 0.0;
    __syncthreads();
    const int lb = blockIdx.x - sg.blk0;
    const int64_t n = sg.n;
    const int64_t stride = (int64_t)sg.nblk * VBLOCK;
    const auto* __restrict__ V = gp((const double*)sg.V);
    auto* __restrict__ w = gp(sg.w);
    for (int64_t t = (int64_t)lb * VBLOCK + threadIdx.x; t < n; t += stride) {
        double u = 0.0;
        for (int i0 = 0; i0 < kf; i0 += 8) {
            double a[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = V[(int64_t)(i0 + j < kf ? i0 + j : kf - 1) * n + t];
#pragma unroll
            for (int j = 0; j < 8; ++j) u += s_y[i0 + j < MMAX ? i0 + j : MMAX - 1] * (i0 + j < kf ? a[j] : 0.0);
        }
        w[t] = u;
    }
}

__global__ void k_set_units(double* x, int64_t ld, int count) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < count) x[(int64_t)c * ld + c] = 1.0;
}

__global__ void k_put_pcseg(PcSeg* dst, PcSeg v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }

void pc_apply(const PcSeg* s, int nseg, int G, int npe, hipStream_t st) {
    const int eb = pc_eb(npe);
    const size_t shm = sizeof(double) * (size_t)eb * npe;
    if (eb == 16) launch_ks(k_bjacobi<16>, dim3(G), dim3(PC_BLOCK), shm, st, s, nseg);
    else launch_ks(k_bjacobi<8>, dim3(G), dim3(PC_BLOCK), shm, st, s, nseg);
}
void pc_combine(const VecSeg* s, int nseg, int G, hipStream_t st) {
    launch_k(k_combine, dim3(G), dim3(VBLOCK), st, s, nseg);
}
void pc_set_units(double* x, int64_t ld, int count, hipStream_t st) {
    launch_k(k_set_units, dim3((count + 63) / 64), dim3(64), st, x, ld, count);
}
void put_pcseg(PcSeg* dst, const PcSeg& v, hipStream_t st) {
    launch_k(k_put_pcseg, dim3(1), dim3(64), st, dst, v);
}

}  // namespace stdg
