// st_ops_impl.hpp -- slab operator kernels: residual, Jacobian-vector
// product and the Navier-Stokes viscous pass, for one (equation, dim, N+1,
// Nt); pointwise physics of eq. (general) without source (convective flux,
// its largest wave speed for the Rusanov flux, viscous flux from the BR1
// lifted gradient of the conservative variables).
//
// Thread mapping: for the systems one thread per space-time node (element,
// time node, spatial node), so a thread holds one state of R variables; for
// the scalar equations one thread per spatial node holds all Nt time nodes
// (TPT time nodes per thread, tpt_of below).  A block holds
// EPB consecutive elements, chosen so that the block is a whole number of
// wavefronts with few idle lanes.  The kernel runs in phases separated by
// block barriers:
//   0. the block's states (and, for a JVP, the direction) go to an LDS tile;
//   1. every thread evaluates the total flux along all d axes at its node
//      (primitive variables computed once) and stages it in LDS;
//   2. volume term: the sum-factorised D contraction along each axis
//      (eq. (elementint) in strong form);
//   3. surface term on compacted threads: one thread per face point
//      (element, axis, side, time node, face node) computes the Rusanov
//      flux with the neighbour's trace (eq. (flux:llf)) and leaves H - f in
//      the LDS slot of the face node, so no lane idles while face nodes work;
//   4. each node adds the lifted surface terms of its faces and the DG
//      time discretisation (eq. (DG_in_time)): the time derivative reads the
//      other time nodes of the same spatial node from the tile.
// Neighbour traces are read from global memory (L2 resident: the logical
// block order is remapped so that each XCD sweeps one contiguous range).
#pragma once
#include "st_krylov.hpp"
#include <type_traits>

namespace stdg {

// Logical block of a physical block: workgroups are dispatched round-robin
// over the 8 XCDs, so physical block i runs on XCD i % 8.  Logical blocks
// [x*q + min(x, r), ...) go to XCD x: each XCD sweeps a contiguous range.
DI int xcd_remap(int i, int G) {
    const int x = i & 7, j = i >> 3;
    const int q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + j;
}

// compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1
template <int B, int E, class F>
DI void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class Seg>
DI int find_seg(const Seg* segs, int nseg, int L) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].blk0 <= L) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Device pointer of a descriptor entry, in the global address space (so that
// accesses compile to global_load/global_store rather than flat ones).
template <class P>
using gptr = __attribute__((address_space(1))) P*;

// A flag or index in device memory; a null pointer reads as zero.  Branch
// free (the pointer is selected, then always loaded), so that a kernel
// issues the loads of all its descriptor indirections together.
static __device__ const int k_zero_index = 0;
DI int load_index(const int* p) { return *(gptr<const int>)(p ? p : &k_zero_index); }

template <class P>
DI gptr<P> resolve(const DynPtr& d) {
    const P* b = static_cast<const P*>(d.base);
    b += (int64_t)(load_index(d.kp) + d.koff) * d.ld;       // kp null: koff = 0
    return (gptr<P>)const_cast<P*>(b);
}

// ---------------------------------------------------------------------------
// block shape: EPB elements of NPE = N1^D * NT space-time nodes per block
// ---------------------------------------------------------------------------
constexpr int best_epb(int npe) {
    int best = 1, bnum = 0, bden = 1;
    for (int e = 1; e * npe <= 512; ++e) {
        const int b = e * npe, bs = (b + 63) / 64 * 64;
        if (b * bden > bnum * bs) { best = e; bnum = b; bden = bs; }   // strictly better lane use
    }
    return best;
}

// LDS pitch of one element's NPE nodes in the operator kernels' tiles
// (padding measured: bank conflicts fall, run time does not)
constexpr int lds_pitch(int npe) { return npe; }

// Time nodes per thread: the scalar equations keep all Nt time nodes of a
// spatial node in one thread (few registers, index work shared by Nt
// nodes); the systems take one space-time node per thread (registers).
__host__ __device__ constexpr int tpt_of(int eq, int nt) { return nvars_of(eq, 1) == 1 ? nt : 1; }

template <int D, int N1, int NT, int TPT>
struct Shape {
    static constexpr int NS = ipow(N1, D);            // spatial nodes per element
    static constexpr int NPE = NS * NT;               // space-time nodes per element
    static constexpr int NF = ipow(N1, D - 1);        // nodes per face
    static constexpr int NJ = NT / TPT;               // time groups per spatial node
    static constexpr int NTH = NS * NJ;               // threads per element
    static constexpr int EPB = best_epb(NTH);         // elements per block
    static constexpr int B = EPB * NTH;               // threads with nodes
    static constexpr int BS = (B + 63) / 64 * 64;     // block size
    static constexpr int NN = EPB * NPE;              // nodes per block
    static constexpr int NFP = EPB * D * 2 * NJ * NF; // face points per block (TPT time nodes each)
};

template <int B, int E>
constexpr int ipow_c = ipow(B, E);
template <int N1, int A>
DI int coord(int s) { return (int)(((unsigned)s / (unsigned)ipow_c<N1, A>) % (unsigned)N1); }

// Element coordinates of element e (x fastest) with the descriptor's
// invariant-divisor constants; element indices fit 31 bits (checked when the
// problem is made).
struct ECoord {
    int c[3];
};
DI unsigned fdiv(unsigned n, unsigned m, int sh) {
    // sh = 31 only for the divisor 1 (m = 2^31); otherwise the high word of
    // the product, shifted by sh - 32
    return sh == 31 ? n : __umulhi(n, m) >> (sh - 32);
}
DI ECoord ecoord(const OpSeg& sg, int e) {
    ECoord x;
    const unsigned t = fdiv((unsigned)e, sg.dm[0], sg.ds[0]);
    x.c[0] = e - (int)t * sg.K[0];
    const unsigned z = fdiv(t, sg.dm[1], sg.ds[1]);
    x.c[1] = (int)t - (int)z * sg.K[1];
    x.c[2] = (int)z;
    return x;
}
// Element across the face of element e (coordinates x) along axis a (periodic).
// The mesh sizes are read as uniform values first, so that a lane-varying
// axis selects among registers (not among descriptor addresses).
DI int neighbour(const OpSeg& sg, int e, const ECoord& x, int a, bool right) {
    const int K0 = __builtin_amdgcn_readfirstlane(sg.K[0]);
    const int K1 = __builtin_amdgcn_readfirstlane(sg.K[1]);
    const int K2 = __builtin_amdgcn_readfirstlane(sg.K[2]);
    const int es = a == 0 ? 1 : (a == 1 ? K0 : K0 * K1);
    const int ca = a == 0 ? x.c[0] : (a == 1 ? x.c[1] : x.c[2]);
    const int K = a == 0 ? K0 : (a == 1 ? K1 : K2);
    const int step = right ? (ca + 1 == K ? 1 - K : 1) : (ca == 0 ? K - 1 : -1);
    return e + step * es;
}

// First element of block b of a segment: lexicographic (tx = 0), or the
// tiled traversal -- tiles of tx x ty elements (tile rows x-fastest), each
// tile a column swept through z, row by row, EPB consecutive x-elements per
// block.  Uniform per block (scalar arithmetic).
template <int EPB>
DI int block_elem0(const OpSeg& sg, int b) {
    if (sg.tx == 0) return b * EPB;
    // divisions by the descriptor's invariant divisors (tk, with tm/ts)
    const int t = (int)fdiv((unsigned)b, sg.tm[0], sg.ts[0]);      // tile
    int rem = b - t * sg.tk[0];
    const int z = (int)fdiv((unsigned)rem, sg.tm[1], sg.ts[1]);    // layer of the tile
    rem -= z * sg.tk[1];
    const int yi = (int)fdiv((unsigned)rem, sg.tm[2], sg.ts[2]);   // row of the layer
    const int xb = rem - yi * sg.tk[2];
    const int tyi = (int)fdiv((unsigned)t, sg.tm[3], sg.ts[3]);
    const int txi = t - tyi * sg.tk[3];
    const int x = txi * sg.tx + xb * EPB, y = tyi * sg.ty + yi;
    return x + sg.K[0] * (y + sg.K[1] * z);
}

// Spatial node on face (axis a, side) with face index f (the other axes in
// increasing order, the first one fastest), for a runtime axis.
template <int D, int N1>
DI int face_node_rt(int a, int f, bool right) {
    const int ia = right ? N1 - 1 : 0;
    if constexpr (D == 1) {
        return ia;
    } else if constexpr (D == 2) {
        return a == 0 ? ia + f * N1 : f + ia * N1;
    } else {
        const int f1 = (int)((unsigned)f % N1), f2 = (int)((unsigned)f / N1);
        return a == 0 ? ia + f1 * N1 + f2 * N1 * N1 : (a == 1 ? f1 + ia * N1 + f2 * N1 * N1 : f1 + f2 * N1 + ia * N1 * N1);
    }
}
template <int N1>
DI int stride_rt(int a) { return a == 0 ? 1 : (a == 1 ? N1 : N1 * N1); }

// ---------------------------------------------------------------------------
// pointwise physics with the primitive variables shared by all axes
// ---------------------------------------------------------------------------
template <int EQ, int D, class T>
struct Flux {
    using S = typename BaseOf<T>::type;
    static constexpr int R = nvars_of(EQ, D);
    static constexpr bool GAS = (EQ == EQ_EULER || EQ == EQ_NS);

    struct Prim {
        T inv;        // 1 / rho
        T vel[D];
        T p;
    };
    SDI Prim prim(const T* u, const EqParams& P) {
        Prim w;
        if constexpr (GAS) {
            w.inv = recip_(u[0]);
            T mv = make_state<T>(S(0), S(0));
#pragma unroll
            for (int b = 0; b < D; ++b) {
                w.vel[b] = u[1 + b] * w.inv;
                mv = b == 0 ? u[1] * w.vel[0] : mv + u[1 + b] * w.vel[b];
            }
            w.p = (S(P.gamma) - S(1)) * (u[D + 1] - S(0.5) * mv);
        }
        return w;
    }

    // convective flux along axis a
    SDI void conv(int a, const T* u, const Prim& w, T* f, const EqParams& P) {
        if constexpr (EQ == EQ_ADV || EQ == EQ_ADVDIFF) {
            f[0] = u[0] * S(P.a[a]);
        } else if constexpr (EQ == EQ_BURGERS) {
            f[0] = S(0.5) * (u[0] * u[0]);
        } else {
            const T va = w.vel[a];
            f[0] = u[1 + a];
#pragma unroll
            for (int b = 0; b < D; ++b) f[1 + b] = u[1 + b] * va;
            f[1 + a] = f[1 + a] + w.p;
            f[D + 1] = (u[D + 1] + w.p) * va;
        }
    }

    // largest characteristic speed along axis a (w: the primitives of u)
    SDI T speed(int a, const T* u, const Prim& w, const EqParams& P) {
        if constexpr (EQ == EQ_ADV || EQ == EQ_ADVDIFF) {
            return make_state<T>(S(fabs(P.a[a])), S(0));
        } else if constexpr (EQ == EQ_BURGERS) {
            return absval(u[0]);
        } else {
            const T c = sqrt_(S(P.gamma) * w.p * w.inv);
            return absval(w.vel[a]) + c;
        }
    }

    // Navier-Stokes viscous quantities from the conservative gradient
    // qb[v] = d u_v / d x_b, one axis b at a time: velocity gradient
    // gv[b][c] = d v_c / d x_b, temperature gradient (T = p / rho), and at
    // the end the divergence.  Tm = p / rho and v2 = |v|^2 from visc_pre.
    struct Visc {
        T gv[D][D];
        T gT[D];
        T div;
        T Tm, v2;
    };
    SDI void visc_pre(const Prim& w, Visc& z) {
        if constexpr (EQ == EQ_NS) {
            z.Tm = w.p * w.inv;
            z.v2 = w.vel[0] * w.vel[0];
#pragma unroll
            for (int b = 1; b < D; ++b) z.v2 = z.v2 + w.vel[b] * w.vel[b];
        }
    }
    SDI void visc_axis(int b, const Prim& w, const T* qb, Visc& z, const EqParams& P) {
        if constexpr (EQ == EQ_NS) {
            const S gm1 = S(P.gamma) - S(1);
            const T gr = qb[0];
            T vgm = w.vel[0] * qb[1];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                z.gv[b][c] = (qb[1 + c] - w.vel[c] * gr) * w.inv;
                if (c > 0) vgm = vgm + w.vel[c] * qb[1 + c];
            }
            const T gp = gm1 * (qb[D + 1] - vgm + S(0.5) * (z.v2 * gr));
            z.gT[b] = (gp - z.Tm * gr) * w.inv;
        }
    }
    SDI void visc_div(Visc& z) {
        if constexpr (EQ == EQ_NS) {
            z.div = z.gv[0][0];
#pragma unroll
            for (int c = 1; c < D; ++c) z.div = z.div + z.gv[c][c];
        }
    }
    // subtract the viscous flux along axis a from f (total flux = Fc - Fv)
    SDI void sub_visc(int a, const Prim& w, const Visc& z, T* f, const EqParams& P) {
        if constexpr (EQ == EQ_NS) {
            const S mu = S(P.mu);
            T work = make_state<T>(S(0), S(0));
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T tau = mu * (z.gv[a][c] + z.gv[c][a]);
                if (c == a) tau = tau - (S(2) / S(3)) * mu * z.div;
                f[1 + c] = f[1 + c] - tau;
                work = c == 0 ? tau * w.vel[0] : work + tau * w.vel[c];
            }
            f[D + 1] = f[D + 1] - (work + S(P.kappa) * z.gT[a]);
        }
    }
};

// Index of spatial node (coordinates ic) on a face normal to axis a: the
// other axes in increasing order, the first one fastest.
template <int D, int N1>
DI int face_index(int a, const int* ic) {
    if constexpr (D == 1) return 0;
    else if constexpr (D == 2) return a == 0 ? ic[1] : ic[0];
    else return a == 0 ? ic[1] + N1 * ic[2] : ic[0] + N1 * (a == 1 ? ic[2] : ic[1]);
}

// Offset of (axis a, side, variable v >= 1, time node j, face node f) in an
// element's viscous face traces (vtrace_per_elem values per element).
template <int D, int N1, int NT>
DI int vtrace_at(int a, int side, int v, int j, int f) {
    constexpr int NF = ipow(N1, D - 1);
    return ((a * 2 + side) * (D + 1) + v - 1) * (NT * NF) + j * NF + f;
}

// BR1 viscous state of the Navier-Stokes equations at one node of an element
// tile: the lifted gradient of the conservative variables along each axis b
// (strong form),
//   q_b = (2/h_b) [ sum_k D_{i_b,k} u_k + M^-1 B (u_hat - u) ],  u_hat = {u},
// for the node's time level (no viscous flux in time), folded at once into
// the velocity and temperature gradients of Flux::Visc.
//   tile: [plane][v][node] with pitch NL, the value plane then (JVP) the
//         tangent plane; nd: the node's tile index, s its spatial node;
//   sD:   the LGL differentiation matrix (LDS copy);
//   u, w: the node's state and its primitives;
//   nb(b, right, un): the neighbour's state across the face of axis b at the
//         matching node (called on face nodes only; interior lifts vanish);
//   zs:   PARK only: [row][node] with pitch NL, D D + D rows, where the
//         gradients are parked axis by axis and reloaded, so that fewer
//         registers are live while the next axes are differentiated: the
//         values (residual), the tangents (JVP; their values stay in
//         registers, which keeps the JVP pass's LDS at the residual's).
template <int D, int N1, class CT, class T, class F, bool JVP, bool PARK, class NB>
DI void br1_visc(const CT* tile, const CT* sD, CT* zs, int NL, int nd, int s, const T* u,
                 const typename F::Prim& w, const OpSeg& sg, NB&& nb, typename F::Visc& z) {
    constexpr int R = D + 2;
    constexpr int NZ = D * D + D;
    CT keep[JVP ? NZ : 1];                      // JVP: the parked rows' values
    const CT iw0 = CT(sg.iw0);
    F::visc_pre(w, z);
    static_for<0, D>([&](auto B_) {
        constexpr int b = decltype(B_)::value;
        constexpr int stride = ipow(N1, b);
        const int ib = coord<N1, b>(s);
        T un[R];
        if (ib == 0 || ib == N1 - 1) {
            nb(b, ib == N1 - 1, un);
        } else {
#pragma unroll
            for (int v = 0; v < R; ++v) un[v] = u[v];
        }
        CT Drow[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) Drow[k] = sD[ib * N1 + k];
        const CT J = CT(sg.rh[b]);
        const CT lw = ib == N1 - 1 ? iw0 : (ib == 0 ? -iw0 : CT(0));
        T qb[R];
#pragma unroll
        for (int v = 0; v < R; ++v) {
            const CT* ln = tile + v * NL + nd - ib * stride;
            CT gv = Drow[0] * ln[0];
#pragma unroll
            for (int k = 1; k < N1; ++k) gv += Drow[k] * ln[k * stride];
            T g;
            if constexpr (JVP) {
                const CT* lt = ln + R * NL;
                CT gt = Drow[0] * lt[0];
#pragma unroll
                for (int k = 1; k < N1; ++k) gt += Drow[k] * lt[k * stride];
                g = make_state<T>(gv, gt);
            } else {
                g = gv;
            }
            g = g + lw * (CT(0.5) * (u[v] + un[v]) - u[v]);
            qb[v] = J * g;
        }
        F::visc_axis(b, w, qb, z, sg.P);
        if constexpr (PARK) {
            auto park = [&](int row, const T& x) {
                if constexpr (JVP) {
                    keep[row] = value(x);
                    zs[row * NL + nd] = part(x);
                } else {
                    zs[row * NL + nd] = value(x);
                }
            };
#pragma unroll
            for (int c = 0; c < D; ++c) park(b * D + c, z.gv[b][c]);
            park(D * D + b, z.gT[b]);
        }
    });
    if constexpr (PARK) {
        // reload (the asm keeps the compiler from carrying the parked parts
        // in registers across the axes instead)
        __asm__ volatile("" ::: "memory");
        auto ld = [&](int row) {
            if constexpr (JVP) return make_state<T>(keep[row], zs[row * NL + nd]);
            else return make_state<T>(zs[row * NL + nd], CT(0));
        };
#pragma unroll
        for (int b = 0; b < D; ++b) {
#pragma unroll
            for (int c = 0; c < D; ++c) z.gv[b][c] = ld(b * D + c);
            z.gT[b] = ld(D * D + b);
        }
    }
    F::visc_div(z);
}

// ---------------------------------------------------------------------------
// Residual / JVP kernel of the nonlinear equations (the linear ones use
// k_lin below).
//   JVP = false: out = R(U) with u_prev (null = 0); CT compute type, UT storage
//                type of U.
//   JVP = true : out = J(U) v by dual numbers (U of type UT, v double).
// Navier-Stokes: the convective part as for Euler; the viscous pass (k_visc)
// has left the viscous terms of the element's own residual (added at the
// end) and its face traces of -Fv, from which the face points add the
// neighbour's half of the BR1 flux.
// BND (Burgers): Dirichlet boundaries on the axes with bc[a] = 1; a face on
// the domain boundary takes the exterior state g (constant: no tangent) in
// place of the neighbour's state in its Rusanov flux.
// ---------------------------------------------------------------------------
template <int EQ, int D, int N1, int NT, class CT, class UT, bool JVP, bool BND = false>
__global__ __launch_bounds__((Shape<D, N1, NT, tpt_of(EQ, NT)>::BS)) void k_op(const OpSeg* __restrict__ segs,
                                                                               int nseg, int G) {
    constexpr int TPT = tpt_of(EQ, NT);
    using SH = Shape<D, N1, NT, TPT>;
    using T = typename std::conditional<JVP, Dual<CT>, CT>::type;
    using F = Flux<EQ, D, T>;
    constexpr int R = nvars_of(EQ, D);
    constexpr int NS = SH::NS, NPE = SH::NPE, NF = SH::NF, NJ = SH::NJ, NTH = SH::NTH;
    constexpr int EPB = SH::EPB, B = SH::B, BS = SH::BS, NFP = SH::NFP;
    static_assert(!linear_eq(EQ), "the linear equations use k_lin");
    static_assert(!BND || EQ == EQ_BURGERS, "Dirichlet boundaries of the nonlinear equations: Burgers");
    constexpr bool NSV = EQ == EQ_NS;
    constexpr int TS = JVP ? 2 : 1;
    constexpr int PL = JVP ? R : 0;             // tile plane of the stored part
    constexpr int EV = R * NPE;                  // values of one element
    constexpr int LP = lds_pitch(NPE);           // LDS pitch of one element's nodes
    constexpr int NL = EPB * LP;                 // LDS plane: the block's nodes of one variable
    // NS: the viscous pass's output per element, and where its traces start
    constexpr int PE = NSV ? visc_per_elem(D, N1, NT) : 0, VRS = NSV ? visc_vr_per_elem(D, N1, NT) : 0;
    __shared__ CT tile[TS * R * NL];             // [plane][v][node]: value, then tangent
    __shared__ CT buf[D * R * NL];               // [a][v][node]: flux along a, then H - f
    __shared__ CT sD[N1 * N1], sDt[NT * NT], swt[NT];

    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    // the skip flag and the Arnoldi indices behind the pointers: one round
    // of loads before the segment is skipped or its data is read
    const int skip = load_index(sg.skip);
    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<double> __restrict__ Vp = JVP ? resolve<double>(sg.V) : nullptr;
    // NS: the viscous pass's output (its tangent for a JVP)
    const gptr<CT> __restrict__ Qp = NSV ? resolve<CT>(sg.Q) : nullptr;
    const gptr<double> __restrict__ out = resolve<double>(sg.out);
    if (skip) return;
    const EqParams& P = sg.P;
    const int tid = threadIdx.x;
    const int el = (int)((unsigned)tid / NTH);
    const int jt = (int)((unsigned)(tid - el * NTH) / NS);   // time group
    const int s = tid - el * NTH - jt * NS;                  // spatial node
    const int e0 = block_elem0<EPB>(sg, L - sg.blk0);
    const int e = e0 + el;
    const bool active = (tid < B) && (e < sg.E);
    const int nd0 = el * LP + jt * TPT * NS + s;             // block node of time node jt*TPT
    const int r0 = jt * TPT * NS + s;                        // element node of time node jt*TPT
    int ic[D];                                               // coordinates of the spatial node
    static_for<0, D>([&](auto A) { ic[decltype(A)::value] = coord<N1, decltype(A)::value>(s); });
    const CT iw0 = CT(sg.iw0);                               // M^-1 B weight of the end nodes
    const gptr<const double> __restrict__ upv = (gptr<const double>)sg.uprev;

    // state of element node rr (= j * NS + s) of element ee
    auto load_state = [&](int ee, int rr, T* u) {
        const gptr<UT> Ue = Up + (int64_t)ee * EV;
#pragma unroll
        for (int v = 0; v < R; ++v) {
            if constexpr (JVP) u[v] = make_state<T>(CT(Ue[v * NPE + rr]), CT((Vp + (int64_t)ee * EV)[v * NPE + rr]));
            else u[v] = CT(Ue[v * NPE + rr]);
        }
    };
    // add to the stored part of x (the value for a residual, the tangent for a JVP)
    auto add_part = [](T& x, CT g) {
        if constexpr (JVP) x.d += g;
        else x += g;
    };
    // -Fv of element ee from its face traces at offset o (variable 1; the
    // density's viscous flux is zero)
    auto load_trace = [&](int ee, int o, CT* g) {
        const gptr<CT> Qe = Qp + (int64_t)ee * PE + VRS;
        g[0] = CT(0);
#pragma unroll
        for (int v = 1; v < R; ++v) g[v] = Qe[o + (v - 1) * (NT * NF)];
    };

    // Face points: (axis a, element, side, time group, face node), axis-major
    // so that a wavefront mostly works on one axis.
    struct FPI {
        int a, pel, to0, rn0, en, stride;
        int tq;                  // NS: the neighbour's face-trace offset (its face on the other side)
        bool right, ok, local;   // local: the neighbour is one of the block's elements (state from the tile)
        bool bnd;                // BND: the face is on a Dirichlet boundary (exterior state)
    };
    auto fp_info = [&](int p) {
        FPI fi;
        constexpr int PER_AX = EPB * 2 * NJ * NF;
        fi.a = (int)((unsigned)p / PER_AX);
        int rem = p - fi.a * PER_AX;
        fi.pel = (int)((unsigned)rem / (2 * NJ * NF));
        rem -= fi.pel * (2 * NJ * NF);
        fi.right = rem >= NJ * NF;
        rem -= fi.right ? NJ * NF : 0;
        const int jg = (int)((unsigned)rem / NF);
        const int f = rem - jg * NF;
        const int ep = e0 + fi.pel;
        fi.ok = p < NFP && ep < sg.E;
        fi.stride = stride_rt<N1>(fi.a);
        const int so = face_node_rt<D, N1>(fi.a, f, fi.right);
        fi.rn0 = jg * TPT * NS + so + (fi.right ? -(N1 - 1) : (N1 - 1)) * fi.stride;   // neighbour's node
        fi.to0 = fi.pel * LP + jg * TPT * NS + so;                                     // own block node
        const ECoord xe = ecoord(sg, fi.ok ? ep : 0);
        fi.en = fi.ok ? neighbour(sg, ep, xe, fi.a, fi.right) : 0;
        fi.bnd = false;
        if constexpr (BND) {
            const int ca = fi.a == 0 ? xe.c[0] : (fi.a == 1 ? xe.c[1] : xe.c[2]);
            fi.bnd = fi.ok && sg.bc[fi.a] && (fi.right ? ca == sg.K[fi.a] - 1 : ca == 0);
        }
        fi.local = fi.ok && !fi.bnd && fi.en >= e0 && fi.en < e0 + EPB;
        fi.tq = NSV ? vtrace_at<D, N1, NT>(fi.a, fi.right ? 0 : 1, 1, jg * TPT, f) : 0;
        return fi;
    };
    // neighbour data of a face point: its state (and NS: its -Fv along the
    // face axis)
    struct FPD {
        T un[TPT][R];
        CT gn[NSV ? TPT : 1][NSV ? R : 1];
    };
    auto fp_load = [&](const FPI& fi, FPD& d) {
        if (!fi.ok || fi.bnd) return;
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj) {
            if (!fi.local) load_state(fi.en, fi.rn0 + jj * NS, d.un[jj]);
            if constexpr (NSV) load_trace(fi.en, fi.tq + jj * NF, d.gn[jj]);
        }
    };
    auto fp_compute = [&](const FPI& fi, const FPD& d) {
        if (!fi.ok) return;
        static_for<0, D>([&](auto A) {
            constexpr int ax = decltype(A)::value;
            if (ax != fi.a) return;
            const bool right = fi.right;
            {
#pragma unroll
                for (int jj = 0; jj < TPT; ++jj) {
                    const int to = fi.to0 + jj * NS;
                    T uo[R], fn[R];
#pragma unroll
                    for (int v = 0; v < R; ++v) {
                        if constexpr (JVP) uo[v] = make_state<T>(tile[v * NL + to], tile[(R + v) * NL + to]);
                        else uo[v] = tile[v * NL + to];
                    }
                    T unl[R];
                    if (fi.local) {
                        // the neighbour's state from the tile (after the first barrier)
                        const int tn = (fi.en - e0) * LP + fi.rn0 + jj * NS;
#pragma unroll
                        for (int v = 0; v < R; ++v) {
                            if constexpr (JVP) unl[v] = make_state<T>(tile[v * NL + tn], tile[(R + v) * NL + tn]);
                            else unl[v] = tile[v * NL + tn];
                        }
                    } else if (BND && fi.bnd) {
#pragma unroll
                        for (int v = 0; v < R; ++v) unl[v] = make_state<T>(CT(sg.bcg), CT(0));
                    } else {
#pragma unroll
                        for (int v = 0; v < R; ++v) unl[v] = d.un[jj][v];
                    }
                    const T* un = unl;
                    const typename F::Prim w = F::prim(un, P);
                    F::conv(ax, un, w, fn, P);
                    if constexpr (NSV) {
#pragma unroll
                        for (int v = 0; v < R; ++v) add_part(fn[v], d.gn[jj][v]);
                    }
                    const T lo = F::speed(ax, uo, F::prim(uo, P), P), ln = F::speed(ax, un, w, P);
                    const T lam = right ? larger(lo, ln) : larger(ln, lo);
#pragma unroll
                    for (int v = 0; v < R; ++v) {
                        const T jump = right ? uo[v] - un[v] : un[v] - uo[v];      // u_L - u_R
                        const CT pen = part((CT(0.5) * lam) * jump);
                        CT& slot = buf[(ax * R + v) * NL + to];
                        slot = CT(0.5) * (part(fn[v]) - slot) + pen;
                    }
                }
            }
        });
    };

    // (0) every global load of the block issued at once: the tables, own
    //     states (and NS: own -Fv), the data of this thread's first face
    //     point; then the tables and the tile to
    //     LDS (the tables were requested first, so waiting for them does not
    //     wait for the rest)
    const CT tD = CT(sg.Dx[tid < N1 * N1 ? tid : 0]);
    const CT tDt = CT(sg.Dt[tid < NT * NT ? tid : 0]);
    const CT twt = CT(sg.wt[tid < NT ? tid : 0]);
    T u[TPT][R];
    CT vr[NSV ? R : 1];                                   // NS: own viscous residual terms (v >= 1)
    if (active) {
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj) load_state(e, r0 + jj * NS, u[jj]);
        if constexpr (NSV) {
            static_assert(TPT == 1, "Navier-Stokes takes one space-time node per thread");
            const gptr<CT> Qe = Qp + (int64_t)e * PE;
#pragma unroll
            for (int v = 1; v < R; ++v) vr[v] = Qe[(v - 1) * NPE + r0];
        }
    } else {
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj)
#pragma unroll
            for (int v = 0; v < R; ++v) u[jj][v] = make_state<T>(CT(1), CT(0));
    }
    const FPI fi0 = fp_info(tid);
    FPD fd0;
    fp_load(fi0, fd0);
    if (tid < N1 * N1) sD[tid] = tD;
    if (tid < NT * NT) sDt[tid] = tDt;
    if (tid < NT) swt[tid] = twt;
    if (active) {
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj)
#pragma unroll
            for (int v = 0; v < R; ++v) {
                tile[v * NL + nd0 + jj * NS] = value(u[jj][v]);
                if constexpr (JVP) tile[(R + v) * NL + nd0 + jj * NS] = part(u[jj][v]);
            }
    }

    // (1) total flux along every axis at the own nodes -> buf (NS: the
    //     convective part; the viscous terms come from the viscous pass)
    if (active) {
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj) {
            const typename F::Prim w = F::prim(u[jj], P);
            static_for<0, D>([&](auto A) {
                constexpr int a = decltype(A)::value;
                T f[R];
                F::conv(a, u[jj], w, f, P);
#pragma unroll
                for (int v = 0; v < R; ++v) buf[(a * R + v) * NL + nd0 + jj * NS] = part(f[v]);
            });
        }
    }
    __syncthreads();

    // (2) volume term -(2/h_a) sum_k D_{ia,k} f_k along each axis
    CT acc[TPT][R];
#pragma unroll
    for (int jj = 0; jj < TPT; ++jj)
#pragma unroll
        for (int v = 0; v < R; ++v) acc[jj][v] = CT(0);
    if (active) {
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int stride = ipow(N1, a);
            const int ia = ic[a];
            CT Drow[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) Drow[k] = sD[ia * N1 + k];
            const CT J = CT(sg.rh[a]);
#pragma unroll
            for (int jj = 0; jj < TPT; ++jj)
#pragma unroll
                for (int v = 0; v < R; ++v) {
                    const CT* ln = buf + (a * R + v) * NL + nd0 + jj * NS - ia * stride;
                    CT sum = Drow[0] * ln[0];
#pragma unroll
                    for (int k = 1; k < N1; ++k) sum += Drow[k] * ln[k * stride];
                    acc[jj][v] -= J * sum;
                }
        });
    }
    __syncthreads();

    // (3) face points: H - f into the flux slot of the face node.  The slot
    // of (axis, face node) belongs to exactly one face point.
    fp_compute(fi0, fd0);
    for (int p = tid + BS; p < NFP; p += BS) {
        const FPI fi = fp_info(p);
        FPD fd;
        fp_load(fi, fd);
        fp_compute(fi, fd);
    }
    __syncthreads();

    // (4) lifted surface terms and DG in time:
    //   R_j = w_j (dt/2 F_j - (D_tau U)_j) - delta_{j1} (u^1 - u^n)
    if (active) {
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            const int ia = ic[a];
            if (ia == 0 || ia == N1 - 1) {
                const CT wl = ia == N1 - 1 ? CT(sg.rh[a]) * iw0 : -(CT(sg.rh[a]) * iw0);
#pragma unroll
                for (int jj = 0; jj < TPT; ++jj)
#pragma unroll
                    for (int v = 0; v < R; ++v) acc[jj][v] -= wl * buf[(a * R + v) * NL + nd0 + jj * NS];
            }
        });
        if constexpr (NSV)
#pragma unroll
            for (int v = 1; v < R; ++v) acc[0][v] += vr[v];
        const CT hdt = CT(0.5 * sg.dt);
        const gptr<double> oe = out + (int64_t)e * EV + r0;
#pragma unroll
        for (int jj = 0; jj < TPT; ++jj) {
            const int j = jt * TPT + jj;
#pragma unroll
            for (int v = 0; v < R; ++v) {
                // the stored part at time node k of this spatial node
                auto tv = [&](int k) -> CT {
                    if constexpr (TPT == NT) return part(u[k][v]);
                    else return tile[(PL + v) * NL + el * LP + k * NS + s];
                };
                CT dtu = sDt[j * NT] * tv(0);
#pragma unroll
                for (int k = 1; k < NT; ++k) dtu += sDt[j * NT + k] * tv(k);
                CT res = swt[j] * (hdt * acc[jj][v] - dtu);
                if (j == 0) {
                    const CT up = (!JVP && upv) ? CT(upv[(int64_t)e * (R * NS) + v * NS + s]) : CT(0);
                    res -= tv(0) - up;
                }
                store_nt(&oe[v * NPE + jj * NS], double(res));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Residual kernel of the linear scalar equations (advection; advection-
// diffusion with BR1).  Along every axis the spatial operator of a line of
// n1 nodes is the descriptor's line operator: A on the own line, HL/HR on the
// two neighbours' face values, and on the two end rows FL/FR on the
// neighbours' lines -- k_op's fluxes, lifted gradient and face terms folded
// into small matrices, so a node needs n1 + 2 values per axis and no flux
// staging.  One thread per spatial node holds all Nt time nodes.  Phases:
//   0. every global load issued: own values, on end nodes the neighbours'
//      face values, the neighbour line of this thread's first face point;
//      own values and face values to LDS;
//   1. every node: A and HL/HR along every axis (into registers); face
//      points (axis, element, side, face node): FL/FR on the neighbour's
//      line, into LDS;
//   2. end nodes add their face-point terms; DG in time (eq. DG_in_time);
//      store.
// The JVP of these equations is this kernel on v with u_prev = 0.
// ROT (2D): the rotating velocity b = a + omega e_z x (x - center); b_a is
// the same at every node of a line along axis a (it depends on the other
// coordinate only), so the line operator is Av + b_a Ac + |b_a| Ad, with the
// three parts in the descriptor and b_a formed per line.  FL / FR (the
// neighbour's interior nodes) come from the viscous part only: the advection
// flux sees the neighbour's face value alone.
// BND: Dirichlet boundaries on the axes with bc[a] = 1.  The line of an
// element at a boundary takes its own-line matrix A_L / A_R / A_LR from the
// descriptor, the exterior state g in place of the neighbour's face value
// (with its own coefficient), and no neighbour line (FL / FR) on that side.
// ---------------------------------------------------------------------------
template <int EQ, int D, int N1, int NT, class CT, class UT, bool ROT = false, bool BND = false>
__global__ __launch_bounds__((Shape<D, N1, NT, NT>::BS)) void k_lin(const OpSeg* __restrict__ segs, int nseg, int G) {
    using SH = Shape<D, N1, NT, NT>;
    constexpr int NS = SH::NS, NPE = SH::NPE, NF = SH::NF;
    constexpr int EPB = SH::EPB, B = SH::B, BS = SH::BS;
    constexpr int N = N1 - 1;
    constexpr int LP = lds_pitch(NPE), NL = EPB * LP;
    constexpr int PER_AX = EPB * 2 * NF;            // face points per axis
    constexpr int NFP = D * PER_AX;                 // (axis, element, side, face node)
    constexpr int NH = NFP * NT;                    // face-point values, all time nodes
    constexpr int LA = N1 * N1 + 4 * N1;            // line-operator entries per axis (per part)
    constexpr int NP = ROT ? 3 : 1;                 // parts per axis
    static_assert(!ROT || (D == 2 && N1 <= ROT_MAX_N1), "rotating velocity: 2D, n1 <= 5");
    static_assert(!(ROT && BND), "rotating velocity with boundaries is not built");
    constexpr int LB = 3 * N1 * N1 + 4 * N1;         // boundary variants per axis
    constexpr int NTAB = D * NP * LA + (BND ? D * LB : 0);
    constexpr int NQ = (NTAB + BS - 1) / BS;
    __shared__ CT tile[NL];                         // [element][time][spatial node]
    __shared__ CT halo[NH];                         // [face point][j]: neighbour's face value
    __shared__ CT fsum[NH];                         // [face point][j]: FL/FR term
    __shared__ CT sL[NTAB], sDt[NT * NT], swt[NT];

    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    const int skip = load_index(sg.skip);
    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<double> __restrict__ out = resolve<double>(sg.out);
    if (skip) return;
    const gptr<const double> __restrict__ upv = (gptr<const double>)sg.uprev;
    const int tid = threadIdx.x;
    const int el = (int)((unsigned)tid / NS);
    const int s = tid - el * NS;
    const int e0 = block_elem0<EPB>(sg, L - sg.blk0);
    const int e = e0 + el;
    const bool active = (tid < B) && (e < sg.E);
    int ic[D];                                      // coordinates of the spatial node
    static_for<0, D>([&](auto A) { ic[decltype(A)::value] = coord<N1, decltype(A)::value>(s); });
    // face index of the node's line along axis a: the other coordinates,
    // in increasing axis order, the first fastest
    auto face_of = [&](int a) -> int {
        if constexpr (D == 1) return 0;
        else if constexpr (D == 2) return a == 0 ? ic[1] : ic[0];
        else return a == 0 ? ic[1] + N1 * ic[2] : (a == 1 ? ic[0] + N1 * ic[2] : ic[0] + N1 * ic[1]);
    };
    auto fpi = [&](int a, int pel, int side, int f) { return ((a * EPB + pel) * 2 + side) * NF + f; };

    // face point p = ((a * EPB + pel) * 2 + side) * NF + f: the neighbour
    // across face (a, side) of element e0 + pel, and its line at face index f
    // from the face inwards
    struct FPI {
        int a, side, rn, step, en;
        bool ok, local;      // local: the neighbour is one of the block's elements (read from the tile)
        bool bnd;            // the face is a Dirichlet boundary: no neighbour line
    };
    auto fp_info = [&](int p) {
        FPI fi;
        fi.a = (int)((unsigned)p / PER_AX);
        int rem = p - fi.a * PER_AX;
        const int pel = (int)((unsigned)rem / (2 * NF));
        rem -= pel * (2 * NF);
        fi.side = rem >= NF ? 1 : 0;
        const int f = rem - fi.side * NF;
        const int ep = e0 + pel;
        fi.ok = p < NFP && ep < sg.E;
        const bool right = fi.side == 1;
        const int stride = stride_rt<N1>(fi.a);
        fi.rn = face_node_rt<D, N1>(fi.a, f, right) + (right ? -N : N) * stride;   // neighbour's face node
        fi.step = right ? stride : -stride;
        const ECoord xe = ecoord(sg, fi.ok ? ep : 0);
        fi.bnd = false;
        if constexpr (BND) {
            const int ca = fi.a == 0 ? xe.c[0] : (fi.a == 1 ? xe.c[1] : xe.c[2]);
            fi.bnd = fi.ok && sg.bc[fi.a] && (right ? ca == sg.K[fi.a] - 1 : ca == 0);
        }
        fi.en = fi.ok ? neighbour(sg, ep, xe, fi.a, right) : 0;
        fi.local = fi.ok && !fi.bnd && fi.en >= e0 && fi.en < e0 + EPB;
        return fi;
    };
    auto fp_load = [&](const FPI& fi, CT (&nl)[NT][N]) {
        if (!fi.ok || fi.local || fi.bnd) return;
        const gptr<UT> lb = Up + (int64_t)fi.en * NPE + fi.rn;
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int m = 1; m <= N; ++m) nl[j][m - 1] = CT(lb[j * NS + m * fi.step]);
    };
    auto fp_compute = [&](int p, const FPI& fi, const CT (&nl)[NT][N]) {
        if (!fi.ok) return;
        if (fi.bnd) {
#pragma unroll
            for (int j = 0; j < NT; ++j) fsum[p * NT + j] = CT(0);
            return;
        }
        const CT* Fs = sL + fi.a * NP * LA + N1 * N1 + 2 * N1 + fi.side * N1;   // FL or FR (viscous part)
        if (fi.local) {
            // the neighbour's line from the tile (after the first barrier)
            const CT* ln = tile + (fi.en - e0) * LP + fi.rn;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                CT c = Fs[1] * ln[j * NS + fi.step];
#pragma unroll
                for (int m = 2; m <= N; ++m) c += Fs[m] * ln[j * NS + m * fi.step];
                fsum[p * NT + j] = c;
            }
            return;
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            CT c = Fs[1] * nl[j][0];
#pragma unroll
            for (int m = 2; m <= N; ++m) c += Fs[m] * nl[j][m - 1];
            fsum[p * NT + j] = c;
        }
    };

    // (0) the tables (requested first), own values, the neighbours' face
    //     values of end nodes, the first face point's neighbour line
    CT tL[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int t = tid + q * BS;
        if constexpr (ROT) {
            tL[q] = CT(sg.lin[t < NTAB ? t : 0]);        // packed parts
        } else {
            constexpr int NI = D * LA;                   // interior operators first, then the boundary ones
            if (t < NI) {
                const int a = (int)((unsigned)t / LA);
                tL[q] = CT(sg.lin[a * LIN_AXIS + (t - a * LA)]);
            } else {
                const int tb = t < NTAB ? t - NI : 0;
                const int a = (int)((unsigned)tb / LB);
                tL[q] = CT(sg.linb[a * LB + (tb - a * LB)]);
            }
        }
    }
    const CT tDt = CT(sg.Dt[tid < NT * NT ? tid : 0]);
    const CT twt = CT(sg.wt[tid < NT ? tid : 0]);
    CT u[NT];
    CT unb[D][NT];
    const ECoord ex = ecoord(sg, active ? e : 0);
    // Dirichlet boundary of the element on axis a, lower (1) and upper (2) end
    auto bside = [&](int a) -> int {
        if constexpr (!BND) return 0;
        if (!sg.bc[a]) return 0;
        const int ca = a == 0 ? ex.c[0] : (a == 1 ? ex.c[1] : ex.c[2]);
        return (ca == 0 ? 1 : 0) | (ca == sg.K[a] - 1 ? 2 : 0);
    };
    if (active) {
        const gptr<UT> Ue = Up + (int64_t)e * NPE + s;
#pragma unroll
        for (int j = 0; j < NT; ++j) u[j] = CT(Ue[j * NS]);
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int stride = ipow_c<N1, a>;
            const int ia = ic[a];
            if (ia == 0 || ia == N) {
                const bool right = ia == N;
                if (bside(a) & (right ? 2 : 1)) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) unb[a][j] = CT(sg.bcg);      // the exterior state
                } else {
                    const gptr<UT> Un = Up + (int64_t)neighbour(sg, e, ex, a, right) * NPE + s + ((right ? 0 : N) - ia) * stride;
#pragma unroll
                    for (int j = 0; j < NT; ++j) unb[a][j] = CT(Un[j * NS]);
                }
            }
        });
    }
    const FPI fi0 = fp_info(tid);
    CT nl0[NT][N];
    fp_load(fi0, nl0);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (tid + q * BS < NTAB) sL[tid + q * BS] = tL[q];
    if (tid < NT * NT) sDt[tid] = tDt;
    if (tid < NT) swt[tid] = twt;
    if (active) {
#pragma unroll
        for (int j = 0; j < NT; ++j) tile[el * LP + j * NS + s] = u[j];
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            const int ia = ic[a];
            if (ia == 0 || ia == N) {
                const int h = fpi(a, el, ia == N ? 1 : 0, face_of(a)) * NT;
#pragma unroll
                for (int j = 0; j < NT; ++j) halo[h + j] = unb[a][j];
            }
        });
    }
    __syncthreads();

    // (1) A and HL/HR along every axis; then the face points
    CT acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = CT(0);
    if (active) {
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int stride = ipow_c<N1, a>;
            const int ia = ic[a];
            const CT* La = sL + a * NP * LA;
            CT Ar[N1];
            CT hl, hr;
            if constexpr (ROT) {
                // b_a of this line: axis 0 depends on y, axis 1 on x
                const int ob = 1 - a;
                const int eb = ecoord(sg, e).c[ob];
                const double xo = sg.lo[ob] + (2.0 / sg.rh[ob]) * (eb + 0.5 * (1.0 + sg.xi[ic[ob]]));
                const double bd = a == 0 ? sg.P.a[0] - sg.omega * (xo - sg.center[1])
                                         : sg.P.a[1] + sg.omega * (xo - sg.center[0]);
                const CT b = CT(bd), ab = CT(fabs(bd));
                const CT* Lc = La + LA;
                const CT* Ld = La + 2 * LA;
#pragma unroll
                for (int k = 0; k < N1; ++k) Ar[k] = La[ia * N1 + k] + b * Lc[ia * N1 + k] + ab * Ld[ia * N1 + k];
                hl = La[N1 * N1 + ia] + b * Lc[N1 * N1 + ia] + ab * Ld[N1 * N1 + ia];
                hr = La[N1 * N1 + N1 + ia] + b * Lc[N1 * N1 + N1 + ia] + ab * Ld[N1 * N1 + N1 + ia];
            } else {
                const int bs = bside(a);
                if (BND && bs) {
                    // the element's own-line matrix at the boundary, and the
                    // coefficient of the exterior state on the boundary side(s)
                    const CT* Lb = sL + D * LA + a * LB;
                    const CT* Ab = Lb + (bs == 3 ? 2 : bs - 1) * N1 * N1;
                    const CT* gc = Lb + 3 * N1 * N1;
#pragma unroll
                    for (int k = 0; k < N1; ++k) Ar[k] = Ab[ia * N1 + k];
                    hl = bs == 1 ? gc[ia] : (bs == 3 ? gc[2 * N1 + ia] : La[N1 * N1 + ia]);
                    hr = bs == 2 ? gc[N1 + ia] : (bs == 3 ? gc[3 * N1 + ia] : La[N1 * N1 + N1 + ia]);
                } else {
#pragma unroll
                    for (int k = 0; k < N1; ++k) Ar[k] = La[ia * N1 + k];
                    hl = La[N1 * N1 + ia];
                    hr = La[N1 * N1 + N1 + ia];
                }
            }
            const int f = face_of(a);
            const CT* hL = halo + fpi(a, el, 0, f) * NT;
            const CT* hR = halo + fpi(a, el, 1, f) * NT;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const CT* ln = tile + el * LP + j * NS + s - ia * stride;
                CT sum = Ar[0] * ln[0];
#pragma unroll
                for (int k = 1; k < N1; ++k) sum += Ar[k] * ln[k * stride];
                sum += hl * hL[j];
                sum += hr * hR[j];
                acc[j] += sum;
            }
        });
    }
    fp_compute(tid, fi0, nl0);
    for (int p = tid + BS; p < NFP; p += BS) {
        const FPI fi = fp_info(p);
        CT nl[NT][N];
        fp_load(fi, nl);
        fp_compute(p, fi, nl);
    }
    __syncthreads();

    // (2) end rows: the face-point terms; DG in time
    //   R_j = w_j (dt/2 F_j - (D_tau U)_j) - delta_{j1} (u^1 - u^n)
    if (active) {
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            const int ia = ic[a];
            if (ia == 0 || ia == N) {
                const CT* fs = fsum + fpi(a, el, ia == N ? 1 : 0, face_of(a)) * NT;
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[j] += fs[j];
            }
        });
        const CT hdt = CT(0.5 * sg.dt);
        const gptr<double> oe = out + (int64_t)e * NPE + s;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            CT dtu = sDt[j * NT] * u[0];
#pragma unroll
            for (int k = 1; k < NT; ++k) dtu += sDt[j * NT + k] * u[k];
            CT res = swt[j] * (hdt * acc[j] - dtu);
            if (j == 0) {
                const CT up = upv ? CT(upv[(int64_t)e * NS + s]) : CT(0);
                res -= u[0] - up;
            }
            store_nt(&oe[j * NS], double(res));
        }
    }
}

// ---------------------------------------------------------------------------
// Navier-Stokes viscous pass.  Every node computes its BR1 viscous state
// (br1_visc) and from it g_a = -Fv_a(u, q), the viscous part of the total
// flux along each axis a.  The pass writes, per element (layout of
// visc_per_elem):
//   * the viscous terms of the element's own residual, in k_op's units
//     (before the DG time terms): the volume term -(2/h_a) sum_k D_{ia,k} g_a,k
//     over the axes, and on face nodes the own half of the BR1 face flux
//     {g} - g = (g_nb - g) / 2, lifted: + (1/2) (2/h_a) M^-1 B g;
//   * the face traces of g_a along the face axis (corner and edge nodes on
//     every face they lie on), from which the neighbours add the other half.
// k_op then treats Navier-Stokes like Euler, plus these two reads.
// JVP = true: the tangent at (U, v) by dual numbers (U of type UT, v
// double).  Output of type CT.  Same block shape as k_op.
// ---------------------------------------------------------------------------
// At least two waves per SIMD are asked for; the pass keeps within that by
// parking the viscous state in LDS (br1_visc).
template <int D, int N1, int NT, class CT, class UT, bool JVP>
__global__ __attribute__((amdgpu_waves_per_eu(2))) __launch_bounds__((Shape<D, N1, NT, 1>::BS)) void k_visc(const OpSeg* __restrict__ segs, int nseg, int G) {
    using SH = Shape<D, N1, NT, 1>;
    using T = typename std::conditional<JVP, Dual<CT>, CT>::type;
    using F = Flux<EQ_NS, D, T>;
    constexpr int R = D + 2;
    constexpr int NS = SH::NS, NPE = SH::NPE, EPB = SH::EPB, B = SH::B;
    constexpr int EV = R * NPE;
    constexpr int PE = visc_per_elem(D, N1, NT), VRS = visc_vr_per_elem(D, N1, NT);
    constexpr int TS = JVP ? 2 : 1;
    __shared__ CT tile[TS * R * B];             // [plane][v][node]
    constexpr int NZ = D * D + D;               // = D (R - 1): also the rows of g staged below
    __shared__ CT zs[NZ * B];                   // parked viscous state, then g [a][v - 1][node]
    __shared__ CT sD[N1 * N1];
    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    const int skip = load_index(sg.skip);
    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<double> __restrict__ Vp = JVP ? resolve<double>(sg.V) : nullptr;
    const gptr<CT> __restrict__ Qp = resolve<CT>(sg.out);
    if (skip) return;
    const EqParams& P = sg.P;
    const int tid = threadIdx.x;
    const int el = (int)((unsigned)tid / NPE);
    const int r = tid - el * NPE;
    const int j = (int)((unsigned)r / NS);
    const int s = r - j * NS;
    const int e0 = block_elem0<EPB>(sg, L - sg.blk0);
    const int e = e0 + el;
    const bool active = (tid < B) && (e < sg.E);
    auto load_state = [&](int ee, int rr, T* u) {
        const gptr<UT> Ue = Up + (int64_t)ee * EV;
#pragma unroll
        for (int v = 0; v < R; ++v) {
            if constexpr (JVP) u[v] = make_state<T>(CT(Ue[v * NPE + rr]), CT((Vp + (int64_t)ee * EV)[v * NPE + rr]));
            else u[v] = CT(Ue[v * NPE + rr]);
        }
    };

    const CT tD = CT(sg.Dx[tid < N1 * N1 ? tid : 0]);
    T u[R];
    if (active) load_state(e, r, u);
    if (tid < N1 * N1) sD[tid] = tD;
    if (active) {
#pragma unroll
        for (int v = 0; v < R; ++v) {
            tile[v * B + tid] = value(u[v]);
            if constexpr (JVP) tile[(R + v) * B + tid] = part(u[v]);
        }
    }
    __syncthreads();
    int ic[D];
    static_for<0, D>([&](auto A) { ic[decltype(A)::value] = coord<N1, decltype(A)::value>(s); });
    const gptr<CT> Qe = Qp + (int64_t)e * PE;
    const CT iw0 = CT(sg.iw0);
    CT vr[R];                                   // the node's own viscous residual terms (v >= 1)
    if (active) {
        const ECoord x = ecoord(sg, e);
        const typename F::Prim w = F::prim(u, P);
        typename F::Visc z;
        br1_visc<D, N1, CT, T, F, JVP, true>(tile, sD, zs, B, tid, s, u, w, sg,
                                             [&](int b, bool right, T* un) {
                                                 const int stride = b == 0 ? 1 : (b == 1 ? N1 : N1 * N1);
                                                 load_state(neighbour(sg, e, x, b, right),
                                                            r + ((right ? 0 : N1 - 1) - ic[b]) * stride, un);
                                             },
                                             z);
#pragma unroll
        for (int v = 1; v < R; ++v) vr[v] = CT(0);
        // g along every axis: staged for the volume term (this thread's
        // column of zs only, which its own reload above has consumed), on
        // face nodes stored as traces and lifted into the own half
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            T f[R];
#pragma unroll
            for (int v = 0; v < R; ++v) f[v] = make_state<T>(CT(0), CT(0));
            F::sub_visc(a, w, z, f, P);
#pragma unroll
            for (int v = 1; v < R; ++v) zs[(a * (R - 1) + v - 1) * B + tid] = part(f[v]);
            const int ia = ic[a];
            if (ia == 0 || ia == N1 - 1) {
                const int o = VRS + vtrace_at<D, N1, NT>(a, ia == 0 ? 0 : 1, 1, j, face_index<D, N1>(a, ic));
                const CT wl = ia == N1 - 1 ? CT(sg.rh[a]) * iw0 : -(CT(sg.rh[a]) * iw0);
#pragma unroll
                for (int v = 1; v < R; ++v) {
                    store_nt(&Qe[o + (v - 1) * (NT * ipow(N1, D - 1))], part(f[v]));
                    vr[v] += CT(0.5) * wl * part(f[v]);
                }
            }
        });
    }
    __syncthreads();
    if (!active) return;
    // volume term -(2/h_a) sum_k D_{ia,k} g_a,k
    static_for<0, D>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int stride = ipow(N1, a);
        const int ia = ic[a];
        CT Drow[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) Drow[k] = sD[ia * N1 + k];
        const CT J = CT(sg.rh[a]);
#pragma unroll
        for (int v = 1; v < R; ++v) {
            const CT* ln = zs + (a * (R - 1) + v - 1) * B + tid - ia * stride;
            CT sum = Drow[0] * ln[0];
#pragma unroll
            for (int k = 1; k < N1; ++k) sum += Drow[k] * ln[k * stride];
            vr[v] -= J * sum;
        }
    });
#pragma unroll
    for (int v = 1; v < R; ++v) store_nt(&Qe[(v - 1) * NPE + r], vr[v]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int EQ, int D, int N1, int NT, class CT, class UT, bool JVP, bool BND = false>
void launch_op(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_op<EQ, D, N1, NT, CT, UT, JVP, BND>, dim3(G), dim3(Shape<D, N1, NT, tpt_of(EQ, NT)>::BS), st, segs,
             nseg, G);
}
template <int EQ, int D, int N1, int NT, class CT, class UT, bool ROT = false, bool BND = false>
void launch_lin(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_lin<EQ, D, N1, NT, CT, UT, ROT, BND>, dim3(G), dim3(Shape<D, N1, NT, NT>::BS), st, segs, nseg, G);
}
template <int D, int N1, int NT, class CT, class UT, bool JVP>
void launch_visc(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_visc<D, N1, NT, CT, UT, JVP>, dim3(G), dim3(Shape<D, N1, NT, 1>::BS), st, segs, nseg, G);
}

template <int EQ, int D, int N1, int NT>
OpTable make_table() {
    OpTable t{};
    t.eq = EQ; t.dim = D; t.n1 = N1; t.nt = NT; t.epb = Shape<D, N1, NT, tpt_of(EQ, NT)>::EPB;
    if constexpr (linear_eq(EQ)) {
        t.res64 = launch_lin<EQ, D, N1, NT, double, double>;
        t.lin32 = launch_lin<EQ, D, N1, NT, float, double>;
        if constexpr (D == 2 && N1 <= ROT_MAX_N1) {
            t.res64_rot = launch_lin<EQ, D, N1, NT, double, double, true>;
            t.lin32_rot = launch_lin<EQ, D, N1, NT, float, double, true>;
        }
        t.res64_bnd = launch_lin<EQ, D, N1, NT, double, double, false, true>;
        t.lin32_bnd = launch_lin<EQ, D, N1, NT, float, double, false, true>;
    } else {
        t.res64 = launch_op<EQ, D, N1, NT, double, double, false>;
        t.jvp64 = launch_op<EQ, D, N1, NT, double, double, true>;
        t.jvp32 = launch_op<EQ, D, N1, NT, float, float, true>;
        if constexpr (EQ == EQ_BURGERS) {
            t.res64_bnd = launch_op<EQ, D, N1, NT, double, double, false, true>;
            t.jvp64_bnd = launch_op<EQ, D, N1, NT, double, double, true, true>;
            t.jvp32_bnd = launch_op<EQ, D, N1, NT, float, float, true, true>;
        }
    }
    if constexpr (EQ == EQ_NS) {
        t.visc_res64 = launch_visc<D, N1, NT, double, double, false>;
        t.visc_jvp64 = launch_visc<D, N1, NT, double, double, true>;
        t.visc_jvp32 = launch_visc<D, N1, NT, float, float, true>;
    }
    return t;
}

// The spatial operator at one time level: the residual kernels instantiated
// for a single time node, run with the time derivative off and unit weight,
// give (dt/2) F(u) (the inflow term vanishes when u_prev is the state
// itself).  Only the FP64 residual entries are filled.
template <int EQ, int D, int N1>
OpTable make_spatial_table() {
    OpTable t{};
    t.eq = EQ; t.dim = D; t.n1 = N1; t.nt = 1; t.epb = Shape<D, N1, 1, 1>::EPB;
    if constexpr (linear_eq(EQ)) {
        t.res64 = launch_lin<EQ, D, N1, 1, double, double>;
        if constexpr (D == 2 && N1 <= ROT_MAX_N1) t.res64_rot = launch_lin<EQ, D, N1, 1, double, double, true>;
        t.res64_bnd = launch_lin<EQ, D, N1, 1, double, double, false, true>;
    } else {
        t.res64 = launch_op<EQ, D, N1, 1, double, double, false>;
        if constexpr (EQ == EQ_BURGERS) t.res64_bnd = launch_op<EQ, D, N1, 1, double, double, false, true>;
    }
    if constexpr (EQ == EQ_NS) t.visc_res64 = launch_visc<D, N1, 1, double, double, false>;
    return t;
}

}  // namespace stdg
