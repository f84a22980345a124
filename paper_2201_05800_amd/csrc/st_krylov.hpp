// st_krylov.hpp -- host launchers of the Newton-GMRES vector kernels and of
// the slab operator tables.
#pragma once
#include "st_device.hpp"
#include <vector>

namespace stdg {

constexpr int NPART_SLOTS = MMAX + 2;   // per-block partial slots of the multi-dot table

void vk_rnorm(const VecSeg* s, int nseg, int G, hipStream_t st);      // partial ||R||^2
void vk_begin(const VecSeg* s, int nseg, hipStream_t st);             // ||R||, cycle state
void vk_scale_v0(const VecSeg* s, int nseg, int G, hipStream_t st);
// k: the Arnoldi step index (0 .. m-1), the same for every slab of the launch;
// gate: read the cycle state before loading (a pass that usually exits);
// stream: non-temporal basis loads (gs_stream)
void vk_multidot(const VecSeg* s, int nseg, int G, int k, hipStream_t st, int gate, int stream);
// pass: Gram-Schmidt pass index; last: 1 the final pass (writes V_{k+1}
// normalised), 0 not, 2 the final pass unless the new vector's norm cancels
// (then the next pass is), 3 that next pass (exits unless pass 0 asked for it)
void vk_update(const VecSeg* s, int nseg, int G, int pass, int last, int k, hipStream_t st, int stream);
// Whether the Gram-Schmidt sweeps of a launch load the basis non-temporally:
// where the Krylov bases of the launch (basis_bytes in all) exceed what the
// 256 MB Infinity Cache could hold, caching them only makes the vectors evict
// each other (3D Navier-Stokes slab, 976 MB of basis: 5 % less time per
// slab with non-temporal loads; 2D advection-diffusion slab, 102 MB: 4 %
// more).  The arithmetic, and so every result, is the same either way.
constexpr int64_t GS_STREAM_BYTES = (int64_t)192 << 20;
inline int gs_stream(int64_t basis_bytes) { return basis_bytes > GS_STREAM_BYTES ? 1 : 0; }
// last / gate of pass p for a cgs_passes option (0 adaptive, 1, 2)
void gs_pass_plan(int passes, int p, int* last, int* gate);
void vk_finish(const VecSeg* s, int nseg, hipStream_t st);
void vk_update_u(const VecSeg* s, int nseg, int G, hipStream_t st);
void vk_init_guess(const VecSeg* s, int nseg, int G, hipStream_t st);
void vk_extract_last(const VecSeg* s, int nseg, int G, hipStream_t st);
void vk_cast32(const VecSeg* s, int nseg, int G, hipStream_t st);
// embedded error estimate of a solved slab: err = rms over the nsp spatial
// values of e / (atol + rtol max(|u^n|, |u^{n+1}|)) with
//   nt = 2: e = -(U_1 - u^n)
//   nt > 2: e = sum_j c_j (U_j - u^n) + (U_1 - u^n) - fs_1
// (c_j = w_1 D_tau[0][j]; fs: slab vector whose first time node holds
// (w_1 dt / 2) F(u^n)); part: nblk partial sums, out: the estimate (device)
struct EstArgs {
    const double* U;
    const double* up;
    const double* fs;     // (dt / 2) F(u_prev), a spatial vector (Nt > 2)
    double fsw;           // its weight w_1
    double* part;
    double* out;
    int64_t nsp;          // E nv ns spatial values
    int nt, ns, nblk;
    double atol, rtol;
    double c[4];
};
void vk_error_estimate(const EstArgs& a, hipStream_t st);
// Coupling of consecutive slabs of a multi-slab system: slab m >= 1 takes
// the last time node of slab m - 1, (e_Nt^T (x) I) U_{m-1}, as its upwind
// inflow u^n, which enters the first time node of the slab residual with
// unit weight (the residual is affine in u^n).  out_m += that node of in_{m-1}
// for m = 1 .. slabs - 1; in is in0 + ld * (*kp) when kp is set (the Arnoldi
// direction), else in0.  Applied to the residual of the slabs with no inflow
// beyond slab 0, and to the JVP of the decoupled slabs, it gives those of
// the coupled system.
struct CoupleArgs {
    const double* in0;
    const int* kp;        // may be null
    int64_t ld;
    double* out;
    const int* skip;      // skip when *skip != 0 (may be null)
    int64_t n;            // unknowns per slab
    int64_t nsp;          // spatial values per slab (E nv ns)
    int slabs, nt, ns, nblk;
};
void vk_couple(const CoupleArgs& a, hipStream_t st);
// element-block Jacobi (st_precond.hip): elements per block, launch, and
// w = sum_{i < kfinal} y_i V_i for the preconditioned Newton update
constexpr int PC_NPE_MAX = 1024;    // largest element block (unknowns per element)
int pc_blocks(int E, int npe);
// launch set-up for blocks of npe unknowns (LDS above 64 KB)
hipError_t pc_prepare(int npe);
// B^-1 (row-major, npe x npe) packed as the kernel's matrix-core operand
std::vector<double> pc_pack(const std::vector<double>& binv, int npe);
// every segment of one launch has the same npe
void pc_apply(const PcSeg* s, int nseg, int G, int npe, hipStream_t st);
void pc_combine(const VecSeg* s, int nseg, int G, hipStream_t st);
// forward substitution over the slabs of a coupled system (k_slab_sweep)
void pc_sweep(const SweepArgs& a, hipStream_t st);
// the first-time-node columns of B^-1 (npe x nv ns, row-major) from its packed form
std::vector<double> pc_inflow_columns(const std::vector<double>& packed, int npe, int nv, int nt, int ns);
void pc_set_units(double* x, int64_t ld, int count, hipStream_t st);
void put_pcseg(PcSeg* dst, const PcSeg& v, hipStream_t st);
void put_opseg(OpSeg* dst, const OpSeg& v, hipStream_t st);
void put_vecseg(VecSeg* dst, const VecSeg& v, hipStream_t st);

using OpLaunch = void (*)(const OpSeg*, int, int, hipStream_t);

// Kernels of one (equation, dim, N+1, Nt).
struct OpTable {
    int eq, dim, n1, nt, epb;
    int rot;             // 1: the rotating-velocity entry (res64 / lin32 are the ROT kernels)
    int bnd;             // 1: the Dirichlet-boundary entry (res64 / lin32 are the BND kernels)
    OpLaunch res64;      // residual, FP64
    OpLaunch lin32;      // linear equations: R(v) with u_prev = 0 in FP32 (FP32-inner JVP)
    OpLaunch jvp64;      // nonlinear JVP, FP64
    OpLaunch jvp32;      // nonlinear JVP, FP32 state and arithmetic
    // Navier-Stokes viscous pass (BR1 gradient, then -Fv along every axis):
    OpLaunch visc_res64; // of U (double), for the residual
    OpLaunch visc_jvp64; // its tangent at (U, v), double
    OpLaunch visc_jvp32; // its tangent at (U32, v), float
    // linear equations in 2D, n1 <= 5: the rotating-velocity variants of
    // res64 / lin32 (line operator in three parts, b_a per line)
    OpLaunch res64_rot;
    OpLaunch lin32_rot;
    // the Dirichlet-boundary variants of res64 / lin32 (linear equations) and
    // of res64 / jvp64 / jvp32 (Burgers)
    OpLaunch res64_bnd;
    OpLaunch lin32_bnd;
    OpLaunch jvp64_bnd;
    OpLaunch jvp32_bnd;
};

void register_ops_adv(std::vector<OpTable>& t);
void register_ops_advdiff(std::vector<OpTable>& t);
void register_ops_burgers(std::vector<OpTable>& t);
void register_ops_euler(std::vector<OpTable>& t);
void register_ops_ns(std::vector<OpTable>& t);

}  // namespace stdg
