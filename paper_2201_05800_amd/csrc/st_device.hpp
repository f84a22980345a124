// st_device.hpp -- device-side types of the space-time DG-SEM slab kernels
// (gfx950): kernel timing hook, forward-mode dual numbers (the pointwise
// physics in st_ops_impl.hpp is templated on the scalar, so the same code
// gives residuals in double / float and exact Jacobian-vector products in
// Dual<double> / Dual<float>), equation parameters, launch descriptors and
// the device-resident GMRES state.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stdg {

// Optional per-launch timing: when a start/stop event pair is armed, the next
// kernel launched through launch_k records them at its own start and end
// (hipExtLaunchKernelGGL), the same interval a kernel trace reports.
struct LaunchTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
LaunchTiming& launch_timing();   // thread-local

template <class K, class... A>
void launch_ks(K kernel, dim3 grid, dim3 block, size_t shm, hipStream_t st, A... args) {
    LaunchTiming& lt = launch_timing();
    if (lt.start) {
        hipEvent_t e0 = lt.start, e1 = lt.stop;
        lt.start = lt.stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, e0, e1, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    }
}
template <class K, class... A>
void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t st, A... args) {
    launch_ks(kernel, grid, block, 0, st, args...);
}

constexpr int MMAX = 32;           // largest GMRES restart length
constexpr int BLOCK = 256;         // threads per block of the operator kernels
constexpr int VBLOCK = 256;        // threads per block of the Krylov vector kernels
constexpr int VMAXBLK = 512;       // most blocks of one slab in a Krylov vector launch

enum EqKind { EQ_ADV = 1, EQ_ADVDIFF = 2, EQ_BURGERS = 3, EQ_EULER = 4, EQ_NS = 5, EQ_ADVDIFF_SIPG = 6 };

__host__ __device__ constexpr int nvars_of(int eq, int dim) {
    return (eq == EQ_EULER || eq == EQ_NS) ? dim + 2 : 1;
}
__host__ __device__ constexpr bool viscous_eq(int eq) { return eq == EQ_ADVDIFF || eq == EQ_NS || eq == EQ_ADVDIFF_SIPG; }
__host__ __device__ constexpr bool linear_eq(int eq) { return eq == EQ_ADV || eq == EQ_ADVDIFF || eq == EQ_ADVDIFF_SIPG; }
__host__ __device__ __forceinline__ constexpr int ipow(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Output of the Navier-Stokes viscous pass, per element, for the d + 1
// variables after the density (whose viscous flux is zero):
//   [0, visc_vr_per_elem): the viscous terms of the element's own residual,
//      [v - 1][time node][spatial node];
//   then the face traces: on each of the 2d faces the viscous part of the
//      face-normal total flux, -Fv_a, at every face node and time node,
//      [axis][side (0 left, 1 right)][v - 1][time node][face node], the face
//      node index running over the other axes in increasing order, the
//      first fastest.
__host__ __device__ constexpr int visc_vr_per_elem(int dim, int n1, int nt) {
    return (dim + 1) * nt * ipow(n1, dim);
}
__host__ __device__ constexpr int visc_per_elem(int dim, int n1, int nt) {
    return visc_vr_per_elem(dim, n1, nt) + 2 * dim * (dim + 1) * nt * ipow(n1, dim - 1);
}

// ---------------------------------------------------------------------------
// forward-mode dual numbers  x + x' eps,  eps^2 = 0
// ---------------------------------------------------------------------------
template <class S>
struct Dual {
    S v, d;
};
template <class T> struct BaseOf { using type = T; };
template <class S> struct BaseOf<Dual<S>> { using type = S; };

#define SDI static __device__ __forceinline__
#define DI __device__ __forceinline__

// Stores of vectors that later kernels read: non-temporal, so that they go
// on to HBM instead of staying dirty in the caches, where the next kernel's
// reads of other data would pay for writing them back (measured: a 31.5 MB
// vector written with plain stores adds 10 us to the following 540 MB
// read sweep, written non-temporally 1 us, at the same cost to the writer).
template <class P, class T>
DI void store_nt(P* p, T v) { __builtin_nontemporal_store(v, p); }

template <class S> DI Dual<S> operator+(Dual<S> a, Dual<S> b) { return {a.v + b.v, a.d + b.d}; }
template <class S> DI Dual<S> operator-(Dual<S> a, Dual<S> b) { return {a.v - b.v, a.d - b.d}; }
template <class S> DI Dual<S> operator-(Dual<S> a) { return {-a.v, -a.d}; }
template <class S> DI Dual<S> operator*(Dual<S> a, Dual<S> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class S> DI Dual<S> operator/(Dual<S> a, Dual<S> b) {
    S r = S(1) / b.v;
    S q = a.v * r;
    return {q, (a.d - q * b.d) * r};
}
template <class S> DI Dual<S> operator+(Dual<S> a, S b) { return {a.v + b, a.d}; }
template <class S> DI Dual<S> operator+(S a, Dual<S> b) { return {a + b.v, b.d}; }
template <class S> DI Dual<S> operator-(Dual<S> a, S b) { return {a.v - b, a.d}; }
template <class S> DI Dual<S> operator-(S a, Dual<S> b) { return {a - b.v, -b.d}; }
template <class S> DI Dual<S> operator*(Dual<S> a, S b) { return {a.v * b, a.d * b}; }
template <class S> DI Dual<S> operator*(S a, Dual<S> b) { return {a * b.v, a * b.d}; }
template <class S> DI Dual<S> operator/(Dual<S> a, S b) { S r = S(1) / b; return {a.v * r, a.d * r}; }
template <class S> DI Dual<S> operator/(S a, Dual<S> b) {
    S r = S(1) / b.v;
    S q = a * r;
    return {q, -(q * b.d) * r};
}

// 1/x: the hardware reciprocal estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each step squares the relative error; the result is
// within a few ulp of 1/x for normal x, and non-finite for x = 0 or NaN).
DI double recip_(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
DI float recip_(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}
template <class S> DI Dual<S> recip_(Dual<S> a) {
    const S r = recip_(a.v);
    return {r, -(a.d * r) * r};
}

DI double sqrt_(double x) { return sqrt(x); }
DI float sqrt_(float x) { return sqrtf(x); }
template <class S> DI Dual<S> sqrt_(Dual<S> a) {
    S s = sqrt_(a.v);
    return {s, a.d * (S(0.5) * recip_(s))};
}
DI double value(double x) { return x; }
DI float value(float x) { return x; }
template <class S> DI S value(Dual<S> x) { return x.v; }
// |x| with derivative sign(x), sign(0) = +1
template <class T> DI T absval(T x) { return value(x) >= 0 ? x : -x; }
// max(a, b); a tie selects a
template <class T> DI T larger(T a, T b) { return value(a) >= value(b) ? a : b; }

// the part of a result that the caller stores: the value for residuals,
// the tangent for Jacobian-vector products
DI double part(double x) { return x; }
DI float part(float x) { return x; }
template <class S> DI S part(Dual<S> x) { return x.d; }

template <class T> DI T make_state(typename BaseOf<T>::type u, typename BaseOf<T>::type v);
template <> DI double make_state<double>(double u, double) { return u; }
template <> DI float make_state<float>(float u, float) { return u; }
template <> DI Dual<double> make_state<Dual<double>>(double u, double v) { return {u, v}; }
template <> DI Dual<float> make_state<Dual<float>>(float u, float v) { return {u, v}; }

// ---------------------------------------------------------------------------
// equation parameters (by value in kernel arguments)
// ---------------------------------------------------------------------------
struct EqParams {
    double a[3];
    double nu;
    double gamma;
    double mu;
    double kappa;   // mu gamma / ((gamma - 1) Pr), gas constant 1
};

// ---------------------------------------------------------------------------
// launch descriptors
// ---------------------------------------------------------------------------
// GMRES state of one slab solve (device resident).
struct GState {
    int k;          // index of the newest basis vector; this step builds k+1
    int done;       // cycle finished (converged, breakdown, m steps, non-finite)
    int kfinal;     // basis vectors used in the update when done
    int iters;      // Arnoldi steps in the current cycle
    int iters_total;// Arnoldi steps over the whole solve
    int outer;      // outer (Newton) iterations started
    int nonfinite;  // a NaN/Inf was met
    unsigned ticket;// last-block-done counter of the running reduction
    int reorth;     // adaptive Gram-Schmidt: the step's second pass is needed
                    // (set by pass 0, read by the gated pass-1 kernels)
    int stall;      // outer iterations since ||R|| last fell below 0.9 best
    int stop;       // outer iteration stops: 1 converged, 2 non-finite, 3 the
                    // Newton-step limit or no progress (VecSeg.dev_stop)
    double target;  // outer stopping threshold tol * max(1, ||R(U0)||)
    double beta;    // ||r0|| of the cycle
    double eta_abs; // absolute inner tolerance of the cycle
    double rnorm;   // ||R(U)|| at the cycle start
    double wn0;     // ||w||^2 before orthogonalisation
    double inv;     // 1 / h_{k+1,k} for the normalisation
    double best;    // smallest ||R|| of the progress test
    double kbytes[8];  // algorithmic bytes of the Krylov kernels that did work
    double hacc[MMAX + 1];
    double hp[MMAX + 1];
    double H[(MMAX + 1) * MMAX];
    double cs[MMAX], sn[MMAX];
    double g[MMAX + 1];  // g[k]: unrotated right-hand side entry carried to step k
    double gr[MMAX];     // rotated right-hand side of the least-squares problem
    double y[MMAX];
};

// A device pointer that may follow the Arnoldi index: base + (*kp + koff) * ld.
struct DynPtr {
    const void* base;
    int64_t ld;
    const int* kp;
    int koff;
};

// entries per axis of the linear line operator: n1^2 + 4 n1 for n1 <= 8
constexpr int LIN_AXIS = 8 * 8 + 4 * 8;
// rotating velocity (2D): the line operator of each axis in three parts
// (viscous, central advection per unit velocity, Rusanov dissipation per
// unit speed), packed with stride n1^2 + 4 n1, for n1 <= ROT_MAX_N1
constexpr int ROT_MAX_N1 = 5;
// Dirichlet boundaries (linear equations): per axis the own-line operators of
// an element at the lower, the upper and both boundaries (n1^2 each), and the
// exterior state's coefficients gL (lower), gR (upper), gL and gR of the
// element at both boundaries (n1 each), packed with stride 3 n1^2 + 4 n1
constexpr int LINB_AXIS = 3 * 8 * 8 + 4 * 8;

// One slab instance inside an operator launch.
struct OpSeg {
    DynPtr U;            // state (double or float)
    DynPtr V;            // direction (JVP only), double
    const double* uprev; // previous-slab state (residual), may be null = 0
    DynPtr Q;            // NS: -Fv along every axis from the viscous pass (its
                         // tangent for a JVP)
    DynPtr dQ;           // unused
    DynPtr out;          // double output
    const int* skip;     // skip the segment when *skip != 0 (may be null)
    int K[3];
    int E;
    unsigned dm[2];      // e / K[a] = (e * dm[a]) >> ds[a] for e < 2^31 (a = 0, 1)
    int ds[2];
    int tx, ty;          // block traversal tiles (elements; tx = 0: lexicographic)
    int tk[4];           // traversal divisors: blocks per tile, per tile layer,
                         // per tile row; tiles along x
    unsigned tm[4];      // n / tk[i] = (n * tm[i]) >> ts[i] for n < 2^31
    int ts[4];
    double rh[3];        // 2 / h_a
    double iw0;          // 1 / wx[0]: M^-1 B weight of the end nodes
    double dt;
    int blk0;            // first logical block
    int nblk;
    EqParams P;          // equation parameters
    // LGL tables: Dx[j * n1 + k] = l_k'(x_j) in space, Dt likewise in time
    double Dx[64];
    double wx[8];
    double Dt[16];
    double wt[4];
    // Linear equations: the spatial operator along one axis as a map of a
    // line of n1 nodes and the neighbours' lines across its two end faces,
    // per axis a at lin[a * LIN_AXIS]: A[i * n1 + k] (own line), HL[i] and
    // HR[i] (the neighbours' face values), FL[m] and FR[m] (the left and the
    // right neighbour's node at distance m >= 1 from its face, end rows only).
    // Rotating velocity: part p of axis a at lin[(a * 3 + p) * (n1^2 + 4 n1)]
    // with the same sub-layout (p = 0 viscous, 1 central per unit b_a,
    // 2 dissipation per unit |b_a|).
    double lin[3 * LIN_AXIS];
    // rotating velocity b = a + omega e_z x (x - center) (2D)
    double lo[2];
    double xi[8];        // LGL nodes on [-1, 1]
    double omega;
    double center[2];
    // Dirichlet boundaries: axes with bc[a] = 1, the exterior state (0 in a
    // JVP: the linear part only), the boundary line operators
    int bc[3];
    double bcg;
    double linb[3 * LINB_AXIS];
};

// One slab instance inside a vector (Krylov) launch.
struct VecSeg {
    double* V;       // basis, (m+1) vectors of n
    double* w;       // Arnoldi work vector
    double* R;       // residual
    double* U;       // state
    int64_t n;
    GState* st;
    double* part;    // per-block partials of the multi-dot, nblk * (MMAX + 2)
    double* part2;   // per-block partial norms, nblk
    double eta_rel;  // inner forcing: eta_abs = max(eta_rel ||R||, eta_tgt * target)
    double eta_tgt;
    double tol;      // outer tolerance (relative to max(1, ||R(U0)||))
    int m;           // restart length
    const double* uprev;  // previous-slab state (initial guess)
    double* unext;   // end-of-slab state output
    float* U32;      // FP32 copy of U (FP32-inner JVPs)
    int nt;          // temporal nodes
    int ns;          // spatial nodes per element
    int blk0;
    int nblk;
    // 1: k_begin also stops the outer iteration after max_newton Newton
    // updates, and after 8 outer iterations in a row that do not bring ||R||
    // below 0.9 times its smallest value so far (the solver's own tests, so
    // that work enqueued before the host has read them exits at once); 0:
    // only on convergence and non-finite values
    int dev_stop;
    int max_newton;
};

// One slab inside an element-block Jacobi launch: out_e = B^-1 in_e for every
// element e (the element's npe consecutive values), or out_e += B^-1 in_e.
// Forward substitution over the slabs of a coupled system (k_slab_sweep).
struct SweepArgs {
    const double* C;      // npe x nl: the first-time-node columns of B^-1 (row-major)
    double* y;            // B^-1 r of every slab (slab m at m n); overwritten by z unless acc
    double* acc;          // null, or acc += z in every slab
    const int* skip;      // skip when *skip != 0 (may be null)
    int64_t n;            // unknowns per slab
    int npe, nl, nt, ns;  // unknowns per element, nv ns, Nt, spatial nodes per element
    int E, M;             // elements per slab, slabs
};

struct PcSeg {
    DynPtr in;            // input vector (may follow the Arnoldi index)
    double* out;
    const double* binvT;  // B^-1 packed by pc_pack (matrix-core operand order)
    const int* skip;      // skip the segment when *skip != 0 (may be null)
    int npe;              // unknowns per element
    int E;                // elements
    int accumulate;       // 1: out += B^-1 in
    int blk0;
    int nblk;
};

// blocks of one slab in a vector launch: about 2 elements per thread, at
// most VMAXBLK blocks; larger slabs loop (grid stride).  Consumers
// reduce the per-block partial tables redundantly in every block, so the
// block count is kept at what the bandwidth needs.
__host__ __device__ inline int vec_blocks(int64_t n) {
    int64_t b = (n + 2 * VBLOCK - 1) / (2 * VBLOCK);
    if (b < 1) b = 1;
    if (b > VMAXBLK) b = VMAXBLK;
    return (int)b;
}

}  // namespace stdg
