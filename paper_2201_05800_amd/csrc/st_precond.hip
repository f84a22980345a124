// st_precond.hip -- element-block Jacobi preconditioner for the slab GMRES
// (right preconditioning).
//
// One npe x npe matrix B serves every element: for advection and
// advection-diffusion on the uniform periodic mesh the slab Jacobian (eq.
// (Jacobian_ST)) is the same operator in every element, and B is its exact
// diagonal block (the coupling of an element's space-time unknowns to
// themselves, through the DG time discretisation, the volume terms and the
// element's own share of its face fluxes); for the nonlinear equations B is
// that block of the Jacobian at a constant reference state.  GMRES then
// solves (J B^-1) y = -R and the Newton update is B^-1 (V y).  The host
// assembles B once per (handle, dt) by applying the JVP kernels to unit
// vectors on a 3^d-element copy of the mesh, and inverts it (partial
// pivoting); the kernels here apply B^-1 to every element of a vector.
#include "st_krylov.hpp"

#include <algorithm>

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
constexpr int PC_BLOCK = 256;               // 4 wavefronts
constexpr int PC_EB = 16;                   // elements per block (the MFMA column count)
// k_bjacobi_big (blocks above 128 unknowns)
constexpr int PB_EB = 32;                   // elements per block: two MFMA column sets
constexpr int PB_KCB = 4;                   // column steps per A-operand chunk
constexpr int PB_KP = 6 * PB_KCB;           // column steps per staged part (three chunk pairs)
constexpr int PB_SQ = PB_EB * 4 * PB_KP / PC_BLOCK;   // staged words per thread and part
typedef double v4d __attribute__((ext_vector_type(4)));
// a flag or index in device memory, zero for a null pointer (branch free: the
// pointer is selected, then always loaded); every lane reads the same word
__device__ const int pc_zero = 0;
DI int pc_index(const int* p) {
    return __builtin_amdgcn_readfirstlane(*(const __attribute__((address_space(1))) int*)(p ? p : &pc_zero));
}
}  // namespace

// the small-block kernel (k_bjacobi_ks) runs one 16-row tile of B^-1 per block
static bool pc_small(int npe) {
    const int KS = (npe + 3) / 4, T = (npe + 15) / 16;
    return T <= 8 && (KS + 3) / 4 <= 8;
}
// row tiles per wavefront of k_bjacobi_big for T row tiles: 3 where one row
// group of 12 holds them all (fewer idle tiles than a group of 16), else 4
// (larger blocks keep groups of 16 tiles: four of them at npe = 960, so
// that each XCD streams a quarter of B^-1)
static int pb_tile_width(int T) { return T <= 12 ? 3 : 4; }
int pc_blocks(int E, int npe) {
    const int T = (npe + 15) / 16;
    if (pc_small(npe)) return (E + PC_EB - 1) / PC_EB * T;      // one block per (elements, row tile)
    const int GT = 4 * pb_tile_width(T);
    return (E + PB_EB - 1) / PB_EB * ((T + GT - 1) / GT);       // per (elements, row group)
}

// out_e (+)= B^-1 in_e for every element, as dense products on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: A 16x4 with A[i][k] in lane i + 16k,
// B 4x16 with B[k][j] in lane j + 16k, D 16x16 with D[i][j] in lane
// j + 16 (i mod 4), register i div 4).  B^-1 comes packed per (16-row tile,
// 4-column step) in that A-operand lane order (zero padded), so each operand
// is one coalesced load; the elements' inputs are staged in LDS in B-operand
// order.
// Blocks above 128 unknowns (at most 1024): one GPU block per (32 elements,
// group of PB_GT = 4 PB_TW row tiles; PB_TW 3 for blocks of at most 192
// unknowns, else 4: pb_tile_width).  Every A operand (16 rows x 4 columns
// of B^-1, streamed from the caches) feeds two products, one per half of the
// 32 elements, and every B operand from LDS feeds the PB_TW row tiles of its
// wavefront.  The elements' inputs are staged in parts of PB_KP column steps,
// double buffered (48 KB of LDS, two blocks per CU): the next part's loads
// are in flight while the current part is multiplied, and the A operands run
// one chunk ahead across the parts.  A part is straight-line code: loads take
// clamped indices rather than branches, the column steps run on to a whole
// number of parts (zero inputs there), the last part loads a next part it
// never stores, and row tiles past the last one multiply and are not stored.
// Consecutive blocks take consecutive row groups of the same elements;
// workgroups go round-robin over the 8 XCDs, so where the number of row
// groups divides 8 (4 for npe from 769 to 1024) each XCD streams the same
// rows of B^-1 (a quarter of it, 1.8 MB at npe = 960), which then stay in its
// L2.  The group accumulates in registers (the column steps in order) and
// writes its rows back through LDS.
template <int PB_TW>
__global__ __launch_bounds__(PC_BLOCK, 2) void k_bjacobi_big(const PcSeg* __restrict__ segs, int nseg) {
    constexpr int PB_GT = 4 * PB_TW;         // row tiles per block (row group)
    extern __shared__ double sm[];           // two buffers of [PB_KP][2][64] B operands
    constexpr int BW = PB_EB * 4 * PB_KP;    // words of one buffer
    const PcSeg& sg = segs[find_pseg(segs, nseg, blockIdx.x)];
    const int skip = pc_index(sg.skip);
    const int kin = pc_index(sg.in.kp);
    if (skip) return;
    const int npe = sg.npe;
    const int KS = (npe + 3) >> 2, T = (npe + 15) >> 4;
    const int NG = (T + PB_GT - 1) / PB_GT;  // row groups
    const int b = blockIdx.x - sg.blk0;
    const int eg = b / NG;
    const int g0 = (b - eg * NG) * PB_GT;    // first row tile of this block's group
    const int e0 = eg * PB_EB;
    const int ne = min(PB_EB, sg.E - e0);
    const double* inb = static_cast<const double*>(sg.in.base);
    if (sg.in.kp) inb += (int64_t)(kin + sg.in.koff) * sg.in.ld;
    const auto* __restrict__ in = gp(inb) + (int64_t)e0 * npe;
    auto* __restrict__ out = gp(sg.out) + (int64_t)e0 * npe;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const auto* __restrict__ A = gp(sg.binvT);
    // A operands of column steps [ks0, ks0 + PB_KCB) (clamped: past KS they
    // are loaded and meet zero inputs or are never used)
    auto load_chunk = [&](int ks0, double (&a)[PB_KCB][PB_TW]) {
#pragma unroll
        for (int c = 0; c < PB_KCB; ++c)
#pragma unroll
            for (int q = 0; q < PB_TW; ++q) {
                const int ks = min(ks0 + c, KS - 1), rt = min(g0 + wave + 4 * q, T - 1);
                a[c][q] = A[((int64_t)rt * KS + ks) * 64 + lane];
            }
    };
    v4d acc[PB_TW][2];
    // the products of column steps [ks0, ks0 + PB_KCB), kr steps into the part
    auto mul_chunk = [&](const double* buf, int kr, const double (&a)[PB_KCB][PB_TW]) {
#pragma unroll
        for (int c = 0; c < PB_KCB; ++c) {
            const double b0 = buf[((kr + c) * 2 + 0) * 64 + lane];
            const double b1 = buf[((kr + c) * 2 + 1) * 64 + lane];
#pragma unroll
            for (int q = 0; q < PB_TW; ++q) {
                acc[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][q], b0, acc[q][0], 0, 0, 0);
                acc[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][q], b1, acc[q][1], 0, 0, 0);
            }
        }
    };
    // column steps [kb, kb + PB_KP) of the block's elements in B-operand
    // order, buffer word w = ((ks - kb) 2 + half) 64 + lane, lane = j + 16
    // (col mod 4): thread t + q PC_BLOCK holds word t + q PC_BLOCK; zeros past
    // npe and past the last element (selected when the words are stored, so
    // that nothing waits for the loads before then)
    double st[PB_SQ];
    unsigned okm = 0;
    auto stage_load = [&](int kb) {
        okm = 0;
#pragma unroll
        for (int q = 0; q < PB_SQ; ++q) {
            const int t = threadIdx.x + q * PC_BLOCK;
            const int l = t & 63, j = ((t >> 6) & 1) * 16 + (l & 15);
            const int c = 4 * (kb + (t >> 7)) + (l >> 4);
            const bool ok = j < ne && c < npe;
            st[q] = in[ok ? (int64_t)j * npe + c : 0];
            okm |= (ok ? 1u : 0u) << q;
        }
    };
    auto stage_store = [&](double* buf) {
#pragma unroll
        for (int q = 0; q < PB_SQ; ++q) buf[threadIdx.x + q * PC_BLOCK] = (okm >> q) & 1u ? st[q] : 0.0;
    };
    double a0[PB_KCB][PB_TW], a1[PB_KCB][PB_TW];
#pragma unroll
    for (int q = 0; q < PB_TW; ++q) acc[q][0] = acc[q][1] = v4d{0.0, 0.0, 0.0, 0.0};
    load_chunk(0, a0);
    stage_load(0);
    stage_store(sm);
    __syncthreads();
    for (int kb = 0, p = 0; kb < KS; kb += PB_KP, ++p) {
        const double* buf = sm + (p & 1) * BW;
        // three chunk pairs; the next part's inputs are requested after the
        // first A chunk, so that the products wait for them only from the
        // second pair on
#pragma unroll
        for (int pr = 0; pr < PB_KP / (2 * PB_KCB); ++pr) {
            const int ks0 = kb + 2 * PB_KCB * pr;
            load_chunk(ks0 + PB_KCB, a1);
            if (pr == 0) stage_load(kb + PB_KP);
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(buf, 2 * PB_KCB * pr, a0);
            load_chunk(ks0 + 2 * PB_KCB, a0);  // after the last pair: the next part's first chunk
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(buf, 2 * PB_KCB * pr + PB_KCB, a1);
        }
        if (kb + PB_KP < KS) {
            // the other buffer was last read in the previous part, before
            // the barrier that ended it
            stage_store(sm + ((p + 1) & 1) * BW);
            __syncthreads();
        }
    }
    // The group's tiles go back through LDS, one half of the elements at a
    // time, so that consecutive threads store consecutive rows of an element
    // (whole cache lines; stored from the MFMA layout directly, each
    // instruction would write 32-byte pieces of 16 elements).  Tile rt holds
    // element 16 h + (lane & 15) at rows 16 rt + (lane >> 4) + 4 r; LDS word
    // (j, local row) at j SR + row - 16 g0 with an odd stride SR.
    constexpr int SR = 16 * PB_GT + 1;
    static_assert(16 * SR <= 2 * PB_EB * 4 * PB_KP, "the result tile fits the part buffers");
    __syncthreads();                          // every wave is done with the part buffers
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < PB_TW; ++q) {
            const int rl = (wave + 4 * q) * 16 + (lane >> 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm[(lane & 15) * SR + rl + 4 * r] = acc[q][h][r];
        }
        __syncthreads();
        const int row0 = g0 * 16;
        for (int t = threadIdx.x; t < 16 * 16 * PB_GT; t += PC_BLOCK) {
            const int jj = t / (16 * PB_GT), rl = t - jj * (16 * PB_GT);
            const int j = 16 * h + jj, row = row0 + rl;
            if (j < ne && row < npe) {
                double z = sm[jj * SR + rl];
                if (sg.accumulate) z += out[(int64_t)j * npe + row];
                store_nt(&out[(int64_t)j * npe + row], z);
            }
        }
        __syncthreads();                      // the LDS tile is read before the next half overwrites it
    }
}

// Small blocks (npe <= 128, at most 8 row tiles): one block per (16
// elements, 16-row tile of B^-1), so that a slab of a few thousand elements
// still gives every CU several blocks; the 4 wavefronts split the column
// steps of the tile (short dependent chains on the matrix cores), with their
// A operands loaded in one go, and the four partial products are added in a
// fixed order through LDS.
__global__ __launch_bounds__(PC_BLOCK) void k_bjacobi_ks(const PcSeg* __restrict__ segs, int nseg) {
    extern __shared__ double sm[];           // [KS * 64] B operands, then partials [4][16][17]
    const PcSeg& sg = segs[find_pseg(segs, nseg, blockIdx.x)];
    // the skip flag, the Arnoldi index behind the input pointer and the
    // block's A operands are requested together, before the flag is tested
    const int skip = pc_index(sg.skip);
    const int kin = pc_index(sg.in.kp);
    const int npe = sg.npe;
    const int KS = (npe + 3) >> 2, T = (npe + 15) >> 4;
    const int KW = (KS + 3) >> 2;            // column steps per wavefront (<= 8)
    const int b = blockIdx.x - sg.blk0;
    const int eg = b / T, rt = b - eg * T;   // element group, row tile
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const auto* __restrict__ A = gp(sg.binvT);
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int ks = wave * KW + c;
        a[c] = (c < KW && ks < KS) ? A[((int64_t)rt * KS + ks) * 64 + lane] : 0.0;
    }
    if (skip) return;
    const int e0 = eg * PC_EB;
    const int ne = min(PC_EB, sg.E - e0);
    const double* inb = static_cast<const double*>(sg.in.base);
    if (sg.in.kp) inb += (int64_t)(kin + sg.in.koff) * sg.in.ld;
    const auto* __restrict__ in = gp(inb) + (int64_t)e0 * npe;
    // the block's inputs, every load issued before the first is used
    // (element-fastest thread order: consecutive lanes write consecutive LDS
    // words, B-operand order); columns past npe and elements past the end
    // stage zeros, so no LDS clearing pass is needed
    constexpr int NIN = PC_EB * 128 / PC_BLOCK;
    double v[NIN];
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
        const int t = threadIdx.x + q * PC_BLOCK;
        const int j = t & (PC_EB - 1), c = t >> 4;
        v[q] = (j < ne && c < npe) ? in[(int64_t)j * npe + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NIN; ++q) {
        const int t = threadIdx.x + q * PC_BLOCK;
        const int j = t & (PC_EB - 1), c = t >> 4;
        if (c < 4 * KS) sm[(c >> 2) * 64 + j + 16 * (c & 3)] = v[q];
    }
    __syncthreads();
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    double bo[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int ks = wave * KW + c;
        bo[c] = (c < KW && ks < KS) ? sm[ks * 64 + lane] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (c < KW) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], bo[c], acc, 0, 0, 0);
    __syncthreads();                         // B operands consumed: reuse sm for the partials
    constexpr int NR = 17;                   // odd row stride: no LDS bank conflicts across j
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = (lane >> 4) + 4 * r, j = lane & 15;
        sm[(wave * 16 + j) * NR + row] = acc[r];
    }
    __syncthreads();
    // the tile's rows of the block's elements: 16 x 16 values
    auto* __restrict__ out = gp(sg.out) + (int64_t)e0 * npe;
    const int j = threadIdx.x >> 4, r = threadIdx.x & 15, row = rt * 16 + r;
    if (j < ne && row < npe) {
        double z = sm[j * NR + r];
        z += sm[(16 + j) * NR + r];
        z += sm[(32 + j) * NR + r];
        z += sm[(48 + j) * NR + r];
        const int64_t t = (int64_t)j * npe + row;
        if (sg.accumulate) z += out[t];
        store_nt(&out[t], z);
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
        store_nt(&w[t], u);
    }
}

// Forward substitution over the M slabs of a coupled system.  Slab m's
// inflow term -(U_1 - u^n) (eq. DG_in_time) takes u^n from slab m-1's last
// time node, so the coupled Jacobian is blockdiag(J_m) + L, with L the unit
// coupling of slab m's first time node to slab m-1's last.  The
// preconditioner P = blockdiag(B) + L (B the element block of each J_m) is
// solved exactly, element by element: with y = B^-1 r of every slab already
// computed (pc_apply),
//   z_0 = y_0,   z_m = y_m - C l_{m-1}  (m >= 1),   l_m = z_m at the last time node,
// C = the columns of B^-1 at the first time node (npe x nl, nl = nv ns).
// One wavefront per element, the slabs in sequence; C staged in LDS when
// CL.  acc null: z overwrites y in slabs 1..M-1; acc set: acc += z in every
// slab (the Newton update) and y is left as it is.
template <bool CL>
__global__ __launch_bounds__(PC_BLOCK) void k_slab_sweep(SweepArgs a) {
    extern __shared__ double sm[];           // [CL ? npe nl : 0] C, then [4 waves][2][nl] l
    if (pc_index(a.skip)) return;
    const int npe = a.npe, nl = a.nl, nt = a.nt, ns = a.ns;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int e = blockIdx.x * (PC_BLOCK / 64) + wave;
    const bool active = e < a.E;
    const double* Cp = a.C;
    if constexpr (CL) {
        for (int t = threadIdx.x; t < npe * nl; t += PC_BLOCK) sm[t] = gp(a.C)[t];
        Cp = sm;
    }
    double* lb = sm + (CL ? npe * nl : 0) + wave * 2 * nl;
    for (int m = 0; m < a.M; ++m) {
        __syncthreads();                     // l_{m-1} written (and C staged)
        if (!active) continue;
        const int64_t off = (int64_t)m * a.n + (int64_t)e * npe;
        auto* __restrict__ ym = gp(a.y) + off;
        const double* lprev = lb + ((m + 1) & 1) * nl;
        double* lnext = lb + (m & 1) * nl;
        for (int row = lane; row < npe; row += 64) {
            double z = ym[row];
            if (m > 0) {
                const double* Cr = Cp + (int64_t)row * nl;
                for (int k = 0; k < nl; ++k) z -= Cr[k] * lprev[k];
            }
            // row = (v nt + j) ns + s
            const int vj = row / ns, s = row - vj * ns, v = vj / nt, j = vj - v * nt;
            if (j == nt - 1) lnext[v * ns + s] = z;
            if (a.acc) gp(a.acc)[off + row] += z;
            else if (m > 0) ym[row] = z;
        }
    }
}

__global__ void k_set_units(double* x, int64_t ld, int count) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < count) x[(int64_t)c * ld + c] = 1.0;
}

__global__ void k_put_pcseg(PcSeg* dst, PcSeg v) { if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v; }

// dynamic LDS of the block Jacobi kernels for element blocks of npe unknowns
static size_t bjacobi_lds(int npe) {
    const int KS = (npe + 3) / 4;
    if (pc_small(npe)) return sizeof(double) * std::max<size_t>(64 * (size_t)KS, 4 * 16 * 17);   // k_bjacobi_ks
    return sizeof(double) * 2 * PB_EB * 4 * PB_KP;                                             // two part buffers
}

hipError_t pc_prepare(int npe) {
    if (npe < 1 || npe > PC_NPE_MAX) return hipErrorInvalidValue;
    return bjacobi_lds(npe) <= 64 * 1024 ? hipSuccess : hipErrorInvalidValue;
}

void pc_apply(const PcSeg* s, int nseg, int G, int npe, hipStream_t st) {
    const int T = (npe + 15) / 16;
    const size_t shm = bjacobi_lds(npe);
    if (pc_small(npe))
        launch_ks(k_bjacobi_ks, dim3(G), dim3(PC_BLOCK), shm, st, s, nseg);
    else if (pb_tile_width(T) == 3)
        launch_ks(k_bjacobi_big<3>, dim3(G), dim3(PC_BLOCK), shm, st, s, nseg);
    else
        launch_ks(k_bjacobi_big<4>, dim3(G), dim3(PC_BLOCK), shm, st, s, nseg);
}
// C in LDS up to this many bytes (several blocks per CU still fit)
constexpr size_t SWEEP_C_LDS = 48 * 1024;
static size_t sweep_lds(const SweepArgs& a, bool cl) {
    return sizeof(double) * ((cl ? (size_t)a.npe * a.nl : 0) + (size_t)(PC_BLOCK / 64) * 2 * a.nl);
}
void pc_sweep(const SweepArgs& a, hipStream_t st) {
    const bool cl = sizeof(double) * (size_t)a.npe * a.nl <= SWEEP_C_LDS;
    const dim3 G((a.E + PC_BLOCK / 64 - 1) / (PC_BLOCK / 64));
    if (cl) launch_ks(k_slab_sweep<true>, G, dim3(PC_BLOCK), sweep_lds(a, true), st, a);
    else launch_ks(k_slab_sweep<false>, G, dim3(PC_BLOCK), sweep_lds(a, false), st, a);
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

namespace stdg {
// Operand order of the block Jacobi kernels: for row tile rt (16 rows) and column step ks
// (4 columns), 64 values in lane order, lane l holding
// (B^-1)[16 rt + l mod 16][4 ks + l div 16], zero outside npe x npe.
std::vector<double> pc_pack(const std::vector<double>& binv, int npe) {
    const int KS = (npe + 3) / 4, T = (npe + 15) / 16;
    std::vector<double> a((size_t)T * KS * 64, 0.0);
    for (int rt = 0; rt < T; ++rt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l) {
                const int row = rt * 16 + (l & 15), col = ks * 4 + (l >> 4);
                if (row < npe && col < npe) a[((size_t)rt * KS + ks) * 64 + l] = binv[(size_t)row * npe + col];
            }
    return a;
}

// C of k_slab_sweep from the packed B^-1: C[row][v ns + s] = (B^-1)[row][(v nt + 0) ns + s].
std::vector<double> pc_inflow_columns(const std::vector<double>& packed, int npe, int nv, int nt, int ns) {
    const int KS = (npe + 3) / 4, nl = nv * ns;
    std::vector<double> c((size_t)npe * nl);
    for (int row = 0; row < npe; ++row)
        for (int v = 0; v < nv; ++v)
            for (int s = 0; s < ns; ++s) {
                const int col = v * nt * ns + s;
                c[(size_t)row * nl + v * ns + s] =
                    packed[((size_t)(row / 16) * KS + col / 4) * 64 + (row % 16) + 16 * (col % 4)];
            }
    return c;
}
}  // namespace stdg
