// st_ops_impl.hpp -- slab operator kernels: residual, Jacobian-vector
// product and BR1 lifted gradient, for one (equation, dim, N+1, Nt).
//
// Thread mapping: one thread per (element, spatial node); the thread keeps
// all Nt time nodes and all variables of its node in registers, so the time
// derivative and the upwind coupling of the time element (eq. (DG_in_time))
// are thread-local.  A block holds EPB = 256 / ns consecutive elements; the
// per-axis flux values of the block are staged in LDS for the
// sum-factorised D contractions along each space axis.  Interface traces of
// neighbouring elements are read from global memory (L2 resident: the
// logical block order is remapped so that each XCD sweeps one contiguous
// range of elements).
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

template <class P>
DI gptr<P> resolve(const DynPtr& d) {
    const P* b = static_cast<const P*>(d.base);
    if (d.kp) b += (int64_t)(*d.kp + d.koff) * d.ld;
    return (gptr<P>)const_cast<P*>(b);
}

template <int D> DI int node_coord(int s, int n1, int a) {
    return a == 0 ? s % n1 : (a == 1 ? (s / n1) % n1 : s / (n1 * n1));
}

// numerical flux along +e_a between left state L and right state R:
// Rusanov convective part (eq. (flux:llf)) minus the central BR1 viscous part
template <int EQ, int D, class T>
DI void num_flux(int a, const T* uL, const T* uR, const T* qL, const T* qR, T* H, const EqParams& P) {
    using Ph = Phys<EQ, D, T>;
    using S = typename BaseOf<T>::type;
    constexpr int R = Ph::R;
    T fL[R], fR[R];
    Ph::conv(a, uL, fL, P);
    Ph::conv(a, uR, fR, P);
    T lam = larger(Ph::speed(a, uL, P), Ph::speed(a, uR, P));
#pragma unroll
    for (int v = 0; v < R; ++v) H[v] = S(0.5) * (fL[v] + fR[v]) + (S(0.5) * lam) * (uL[v] - uR[v]);
    if constexpr (viscous_eq(EQ)) {
        T gL[R], gR[R];
        Ph::visc(a, uL, qL, gL, P);
        Ph::visc(a, uR, qR, gR, P);
#pragma unroll
        for (int v = 0; v < R; ++v) H[v] = H[v] - S(0.5) * (gL[v] + gR[v]);
    }
}

template <int EQ, int D, class T>
DI void total_flux(int a, const T* u, const T* q, T* f, const EqParams& P) {
    using Ph = Phys<EQ, D, T>;
    Ph::conv(a, u, f, P);
    if constexpr (viscous_eq(EQ)) {
        constexpr int R = Ph::R;
        T g[R];
        Ph::visc(a, u, q, g, P);
#pragma unroll
        for (int v = 0; v < R; ++v) f[v] = f[v] - g[v];
    }
}

// ---------------------------------------------------------------------------
// Residual / JVP kernel.
//   JVP = false: out = R(U) with u_prev (null = 0); CT compute type, UT storage
//                type of U.  With U := v and u_prev = 0 this is also the JVP of
//                the linear equations.
//   JVP = true : out = J(U) v by dual numbers (U of type UT, v double).
// ---------------------------------------------------------------------------
template <int EQ, int D, int N1, int NT, class CT, class UT, bool JVP>
__global__ __launch_bounds__(BLOCK) void k_op(const OpSeg* __restrict__ segs, int nseg, int G) {
    using T = typename std::conditional<JVP, Dual<CT>, CT>::type;
    constexpr int R = nvars_of(EQ, D);
    constexpr int NS = ipow(N1, D);
    constexpr int EPB = BLOCK / NS > 0 ? BLOCK / NS : 1;
    constexpr bool VISC = viscous_eq(EQ);
    __shared__ CT buf[EPB * NT * R * NS];

    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    if (sg.skip && *sg.skip) return;
    const EqParams& P = sg.P;
    const int tid = threadIdx.x;
    const int el = tid / NS;
    const int s = tid - el * NS;
    const int64_t e = (int64_t)(L - sg.blk0) * EPB + el;
    const bool active = (el < EPB) && (e < sg.E);

    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<double> __restrict__ Vp = JVP ? resolve<double>(sg.V) : nullptr;
    const gptr<CT> __restrict__ Qp = VISC ? resolve<CT>(sg.Q) : nullptr;
    const gptr<CT> __restrict__ dQp = (VISC && JVP) ? resolve<CT>(sg.dQ) : nullptr;
    const gptr<double> __restrict__ out = resolve<double>(sg.out);
    const gptr<const double> __restrict__ upv = (gptr<const double>)sg.uprev;

    const int ec[3] = {(int)(e % sg.K[0]), (int)((e / sg.K[0]) % sg.K[1]), (int)(e / ((int64_t)sg.K[0] * sg.K[1]))};
    const int64_t es[3] = {1, sg.K[0], (int64_t)sg.K[0] * sg.K[1]};

    T u[NT][R];
    CT acc[NT][R];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int v = 0; v < R; ++v) {
            acc[j][v] = CT(0);
            if (active) {
                const int64_t idx = ((e * R + v) * NT + j) * NS + s;
                u[j][v] = make_state<T>(CT(Up[idx]), JVP ? CT(Vp[idx]) : CT(0));
            } else {
                u[j][v] = make_state<T>(CT(1), CT(0));
            }
        }

    auto load_q = [&](gptr<CT> base, gptr<CT> dbase, int64_t ee, int ss, int j, T* q) {
#pragma unroll
        for (int b = 0; b < D; ++b)
#pragma unroll
            for (int v = 0; v < R; ++v) {
                const int64_t idx = (((ee * D + b) * R + v) * NT + j) * NS + ss;
                q[b * R + v] = make_state<T>(base[idx], JVP ? dbase[idx] : CT(0));
            }
    };

    static_for<0, D>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int stride = ipow(N1, a);
        const int ia = node_coord<D>(s, N1, a);
        // (1) total flux along a at the own node, every time node -> LDS
        if (active) {
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                T q[VISC ? D * R : 1];
                if constexpr (VISC) load_q(Qp, dQp, e, s, j, q);
                T f[R];
                total_flux<EQ, D, T>(a, u[j], q, f, P);
#pragma unroll
                for (int v = 0; v < R; ++v) buf[((el * NT + j) * R + v) * NS + s] = part(f[v]);
            }
        }
        __syncthreads();
        if (active) {
            const CT J = CT(sg.rh[a]);
            // (2) volume term -(2/h_a) sum_k D_{ia,k} f_k along the line
            CT Drow[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) Drow[k] = CT(sg.Dx[ia * N1 + k]);
            const int s0 = s - ia * stride;
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int v = 0; v < R; ++v) {
                    const CT* line = buf + ((el * NT + j) * R + v) * NS + s0;
                    CT sum = Drow[0] * line[0];
#pragma unroll
                    for (int k = 1; k < N1; ++k) sum += Drow[k] * line[k * stride];
                    acc[j][v] -= J * sum;
                }
            // (3) interface term -(2/h_a) M^-1 B (H - f) on the face nodes
            if (ia == 0 || ia == N1 - 1) {
                const int side = (ia == N1 - 1) ? 1 : -1;
                const int ca = ec[a] + side;
                const int cw = ca < 0 ? ca + sg.K[a] : (ca >= sg.K[a] ? ca - sg.K[a] : ca);
                const int64_t en = e + (int64_t)(cw - ec[a]) * es[a];
                const int sn = s + ((side > 0 ? 0 : N1 - 1) - ia) * stride;
                const CT wl = J / CT(sg.wx[0]);
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    T un[R];
#pragma unroll
                    for (int v = 0; v < R; ++v) {
                        const int64_t idx = ((en * R + v) * NT + j) * NS + sn;
                        un[v] = make_state<T>(CT(Up[idx]), JVP ? CT(Vp[idx]) : CT(0));
                    }
                    T qo[VISC ? D * R : 1], qn[VISC ? D * R : 1];
                    if constexpr (VISC) {
                        load_q(Qp, dQp, e, s, j, qo);
                        load_q(Qp, dQp, en, sn, j, qn);
                    }
                    T H[R];
                    if (side > 0) num_flux<EQ, D, T>(a, u[j], un, qo, qn, H, P);
                    else          num_flux<EQ, D, T>(a, un, u[j], qn, qo, H, P);
#pragma unroll
                    for (int v = 0; v < R; ++v) {
                        const CT fo = buf[((el * NT + j) * R + v) * NS + s];
                        const CT d = part(H[v]) - fo;
                        acc[j][v] -= (side > 0 ? wl : -wl) * d;
                    }
                }
            }
        }
        __syncthreads();
    });

    // (4) DG in time: R_j = w_j (dt/2 F_j - (D_tau U)_j) - delta_{j1} (u^1 - u^n)
    if (active) {
        const CT hdt = CT(0.5 * sg.dt);
#pragma unroll
        for (int v = 0; v < R; ++v) {
            CT up = CT(0);
            if (!JVP && upv) up = CT(upv[(e * R + v) * NS + s]);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                CT dtu = CT(sg.Dt[j * NT]) * part(u[0][v]);
#pragma unroll
                for (int k = 1; k < NT; ++k) dtu += CT(sg.Dt[j * NT + k]) * part(u[k][v]);
                CT r = CT(sg.wt[j]) * (hdt * acc[j][v] - dtu);
                if (j == 0) r -= part(u[0][v]) - up;
                out[((e * R + v) * NT + j) * NS + s] = double(r);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// BR1 lifted gradient of the conservative variables (strong form):
//   q_b = (2/h_b) [ sum_k D_{i_b,k} u_k + M^-1 B (u_hat - u) ],  u_hat = {u},
// for every time node (no viscous flux in time).  Output layout
//   Q[((e * D + b) * R + v) * Nt + j) * ns + s], type CT.
// ---------------------------------------------------------------------------
template <int D, int N1, int NT, int R, class CT, class UT>
__global__ __launch_bounds__(BLOCK) void k_grad(const OpSeg* __restrict__ segs, int nseg, int G) {
    constexpr int NS = ipow(N1, D);
    constexpr int EPB = BLOCK / NS > 0 ? BLOCK / NS : 1;
    __shared__ CT buf[EPB * NT * R * NS];
    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    if (sg.skip && *sg.skip) return;
    const int tid = threadIdx.x;
    const int el = tid / NS;
    const int s = tid - el * NS;
    const int64_t e = (int64_t)(L - sg.blk0) * EPB + el;
    const bool active = (el < EPB) && (e < sg.E);
    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<CT> __restrict__ Qp = resolve<CT>(sg.out);
    const int ec[3] = {(int)(e % sg.K[0]), (int)((e / sg.K[0]) % sg.K[1]), (int)(e / ((int64_t)sg.K[0] * sg.K[1]))};
    const int64_t es[3] = {1, sg.K[0], (int64_t)sg.K[0] * sg.K[1]};

    if (active) {
#pragma unroll
        for (int v = 0; v < R; ++v)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                buf[((el * NT + j) * R + v) * NS + s] = CT(Up[((e * R + v) * NT + j) * NS + s]);
    }
    __syncthreads();
    if (!active) return;
    static_for<0, D>([&](auto B) {
        constexpr int b = decltype(B)::value;
        constexpr int stride = ipow(N1, b);
        const int ib = node_coord<D>(s, N1, b);
        const int s0 = s - ib * stride;
        const CT J = CT(sg.rh[b]);
        CT Drow[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) Drow[k] = CT(sg.Dx[ib * N1 + k]);
        const bool face = (ib == 0 || ib == N1 - 1);
        const int side = (ib == N1 - 1) ? 1 : -1;
        int64_t en = e;
        int sn = s;
        if (face) {
            const int ca = ec[b] + side;
            const int cw = ca < 0 ? ca + sg.K[b] : (ca >= sg.K[b] ? ca - sg.K[b] : ca);
            en = e + (int64_t)(cw - ec[b]) * es[b];
            sn = s + ((side > 0 ? 0 : N1 - 1) - ib) * stride;
        }
        const CT wl = CT(1) / CT(sg.wx[0]);
#pragma unroll
        for (int v = 0; v < R; ++v)
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const CT* line = buf + ((el * NT + j) * R + v) * NS + s0;
                CT g = Drow[0] * line[0];
#pragma unroll
                for (int k = 1; k < N1; ++k) g += Drow[k] * line[k * stride];
                if (face) {
                    const CT uo = line[ib * stride];
                    const CT un = CT(Up[((en * R + v) * NT + j) * NS + sn]);
                    const CT uh = CT(0.5) * (uo + un);
                    g += (side > 0 ? wl : -wl) * (uh - uo);
                }
                Qp[(((e * D + b) * R + v) * NT + j) * NS + s] = J * g;
            }
    });
}

// ---------------------------------------------------------------------------
// Advection-diffusion with the BR1 viscous flux in a single kernel.
// Fv = nu grad u, so the central viscous flux through a face needs only the
// neighbour's NORMAL lifted derivative at the face node, which depends on the
// neighbour's line of nodes normal to the face and on this element's face
// value.  Each face thread reads that line (L2) together with its own state,
// so the lifted gradient never goes through HBM.  Same arithmetic as k_grad
// followed by k_op; JVP of this linear operator = the operator applied to v
// with u_prev = 0.
// ---------------------------------------------------------------------------
template <int D, int N1, int NT, class CT, class UT>
__global__ __launch_bounds__(BLOCK) void k_advdiff(const OpSeg* __restrict__ segs, int nseg, int G) {
    constexpr int NS = ipow(N1, D);
    constexpr int EPB = BLOCK / NS > 0 ? BLOCK / NS : 1;
    __shared__ CT tile[EPB * NT * NS];
    __shared__ CT fl[EPB * NT * NS];

    const int L = xcd_remap(blockIdx.x, G);
    const OpSeg& sg = segs[find_seg(segs, nseg, L)];
    if (sg.skip && *sg.skip) return;
    const EqParams& P = sg.P;
    const int tid = threadIdx.x;
    const int el = tid / NS;
    const int s = tid - el * NS;
    const int64_t e = (int64_t)(L - sg.blk0) * EPB + el;
    const bool active = (el < EPB) && (e < sg.E);
    const gptr<UT> __restrict__ Up = resolve<UT>(sg.U);
    const gptr<double> __restrict__ out = resolve<double>(sg.out);
    const gptr<const double> __restrict__ upv = (gptr<const double>)sg.uprev;
    const int ec[3] = {(int)(e % sg.K[0]), (int)((e / sg.K[0]) % sg.K[1]), (int)(e / ((int64_t)sg.K[0] * sg.K[1]))};
    const int64_t es[3] = {1, sg.K[0], (int64_t)sg.K[0] * sg.K[1]};
    const CT nu = CT(P.nu);
    const CT w0 = CT(sg.wx[0]);

    // own values and, on every face axis, the neighbour's line normal to it
    CT u[NT];
    CT line[D][N1][NT];
    int side[D];
#pragma unroll
    for (int a = 0; a < D; ++a) side[a] = 0;
    if (active) {
#pragma unroll
        for (int j = 0; j < NT; ++j) u[j] = CT(Up[(e * NT + j) * NS + s]);
        static_for<0, D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int stride = ipow(N1, a);
            const int ia = node_coord<D>(s, N1, a);
            if (ia == 0 || ia == N1 - 1) {
                side[a] = (ia == N1 - 1) ? 1 : -1;
                const int ca = ec[a] + side[a];
                const int cw = ca < 0 ? ca + sg.K[a] : (ca >= sg.K[a] ? ca - sg.K[a] : ca);
                const int64_t en = e + (int64_t)(cw - ec[a]) * es[a];
                const int s0 = s - ia * stride;
#pragma unroll
                for (int k = 0; k < N1; ++k)
#pragma unroll
                    for (int j = 0; j < NT; ++j) line[a][k][j] = CT(Up[(en * NT + j) * NS + s0 + k * stride]);
            }
        });
#pragma unroll
        for (int j = 0; j < NT; ++j) tile[(el * NT + j) * NS + s] = u[j];
    } else {
#pragma unroll
        for (int j = 0; j < NT; ++j) u[j] = CT(0);
    }
    __syncthreads();

    // own lifted gradient q[b][j] (central u-hat on faces)
    CT q[D][NT];
    if (active) {
        static_for<0, D>([&](auto B) {
            constexpr int b = decltype(B)::value;
            constexpr int stride = ipow(N1, b);
            const int ib = node_coord<D>(s, N1, b);
            const int s0 = s - ib * stride;
            CT Drow[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) Drow[k] = CT(sg.Dx[ib * N1 + k]);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const CT* ln = tile + (el * NT + j) * NS + s0;
                CT g = Drow[0] * ln[0];
#pragma unroll
                for (int k = 1; k < N1; ++k) g += Drow[k] * ln[k * stride];
                if (side[b] != 0) {
                    const CT un = side[b] > 0 ? line[b][0][j] : line[b][N1 - 1][j];
                    const CT uh = CT(0.5) * (u[j] + un);
                    g += (side[b] > 0 ? CT(1) : CT(-1)) / w0 * (uh - u[j]);
                }
                q[b][j] = CT(sg.rh[b]) * g;
            }
        });
    }

    CT acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = CT(0);
    static_for<0, D>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int stride = ipow(N1, a);
        const int ia = node_coord<D>(s, N1, a);
        const CT av = CT(P.a[a]);
        if (active) {
#pragma unroll
            for (int j = 0; j < NT; ++j) fl[(el * NT + j) * NS + s] = u[j] * av - q[a][j] * nu;
        }
        __syncthreads();
        if (active) {
            const CT J = CT(sg.rh[a]);
            CT Drow[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) Drow[k] = CT(sg.Dx[ia * N1 + k]);
            const int s0 = s - ia * stride;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const CT* ln = fl + (el * NT + j) * NS + s0;
                CT sum = Drow[0] * ln[0];
#pragma unroll
                for (int k = 1; k < N1; ++k) sum += Drow[k] * ln[k * stride];
                acc[j] -= J * sum;
            }
            if (side[a] != 0) {
                // neighbour's normal derivative at its face node: its D row at
                // that node plus its own lift with the same u-hat
                const int inb = side[a] > 0 ? 0 : N1 - 1;
                CT Dn[N1];
#pragma unroll
                for (int k = 0; k < N1; ++k) Dn[k] = CT(sg.Dx[inb * N1 + k]);
                const CT lam = CT(fabs(P.a[a]));
                const CT wl = J / w0;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const CT un = side[a] > 0 ? line[a][0][j] : line[a][N1 - 1][j];
                    CT gn = Dn[0] * line[a][0][j];
#pragma unroll
                    for (int k = 1; k < N1; ++k) gn += Dn[k] * line[a][k][j];
                    const CT uh = CT(0.5) * (un + u[j]);
                    gn += (side[a] > 0 ? CT(-1) : CT(1)) / w0 * (uh - un);
                    const CT qn = J * gn;
                    const CT uL = side[a] > 0 ? u[j] : un, uR = side[a] > 0 ? un : u[j];
                    const CT qL = side[a] > 0 ? q[a][j] : qn, qR = side[a] > 0 ? qn : q[a][j];
                    const CT fL = uL * av, fR = uR * av;
                    CT H = CT(0.5) * (fL + fR) + (CT(0.5) * lam) * (uL - uR);
                    H = H - CT(0.5) * (qL * nu + qR * nu);
                    const CT fo = fl[(el * NT + j) * NS + s];
                    acc[j] -= (side[a] > 0 ? wl : -wl) * (H - fo);
                }
            }
        }
        __syncthreads();
    });

    if (active) {
        const CT hdt = CT(0.5 * sg.dt);
        const CT up = upv ? CT(upv[e * NS + s]) : CT(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            CT dtu = CT(sg.Dt[j * NT]) * u[0];
#pragma unroll
            for (int k = 1; k < NT; ++k) dtu += CT(sg.Dt[j * NT + k]) * u[k];
            CT r = CT(sg.wt[j]) * (hdt * acc[j] - dtu);
            if (j == 0) r -= u[0] - up;
            out[(e * NT + j) * NS + s] = double(r);
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int D, int N1>
constexpr int op_epb() {
    return BLOCK / ipow(N1, D) > 0 ? BLOCK / ipow(N1, D) : 1;
}

template <int EQ, int D, int N1, int NT, class CT, class UT, bool JVP>
void launch_op(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_op<EQ, D, N1, NT, CT, UT, JVP>, dim3(G), dim3(BLOCK), st, segs, nseg, G);
}
template <int D, int N1, int NT, class CT, class UT>
void launch_advdiff(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_advdiff<D, N1, NT, CT, UT>, dim3(G), dim3(BLOCK), st, segs, nseg, G);
}
template <int D, int N1, int NT, int R, class CT, class UT>
void launch_grad(const OpSeg* segs, int nseg, int G, hipStream_t st) {
    launch_k(k_grad<D, N1, NT, R, CT, UT>, dim3(G), dim3(BLOCK), st, segs, nseg, G);
}

template <int EQ, int D, int N1, int NT>
OpTable make_table() {
    constexpr int R = nvars_of(EQ, D);
    OpTable t{};
    t.eq = EQ; t.dim = D; t.n1 = N1; t.nt = NT; t.epb = op_epb<D, N1>();
    if constexpr (EQ == EQ_ADVDIFF) {
        // single-kernel BR1: no gradient pass, no gradient buffers
        t.res64 = launch_advdiff<D, N1, NT, double, double>;
        t.lin32 = launch_advdiff<D, N1, NT, float, double>;
        return t;
    }
    t.res64 = launch_op<EQ, D, N1, NT, double, double, false>;
    if constexpr (linear_eq(EQ)) {
        t.lin32 = launch_op<EQ, D, N1, NT, float, double, false>;
    } else {
        t.jvp64 = launch_op<EQ, D, N1, NT, double, double, true>;
        t.jvp32 = launch_op<EQ, D, N1, NT, float, float, true>;
    }
    if constexpr (viscous_eq(EQ)) {
        t.grad64 = launch_grad<D, N1, NT, R, double, double>;
        t.grad32 = launch_grad<D, N1, NT, R, float, float>;
        t.grad64to32 = launch_grad<D, N1, NT, R, float, double>;
    }
    return t;
}

}  // namespace stdg
