// st_noalloc.hip -- st_residual_noalloc: the slab residual of st_residual for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  It takes the problem
// itself instead of a handle, and every device buffer its kernels need beyond
// the caller's inputs and outputs -- the launch descriptors and, for
// Navier-Stokes, the output of the BR1 viscous pass -- from one
// file-scope device array of fixed size.  The kernels are st_residual's.
#include "st_engine.hpp"

#include <cmath>
#include <cstring>
#include <mutex>

using namespace stdg;

// Each device holds its own copy of this array from the time the library is
// loaded there until the process ends.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[ST_NOALLOC_SCRATCH_BYTES];

namespace {

// Layout of the static scratch array: two operator descriptors (viscous pass,
// operator), then the Navier-Stokes viscous pass's output (visc_len values).
constexpr size_t SCRATCH_BYTES = (size_t)ST_NOALLOC_SCRATCH_BYTES;
constexpr size_t DESC_SLOT = 16384;
constexpr size_t Q_OFFSET = 2 * DESC_SLOT;
static_assert(sizeof(OpSeg) <= DESC_SLOT, "descriptor slot too small");

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// The scratch array's device address on the current device (looked up once
// per device, with that device current).
int scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(ST_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(ST_ERR_UNSUPPORTED, "st_residual_noalloc: device index");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(ST_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return ST_OK;
}

}  // namespace

extern "C" {

int st_residual_noalloc(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, const double* U,
                        const double* u_prev, double t0, double dt, double* R, void* stream) {
    (void)t0;
    if (!U || !u_prev || !R) return set_error(ST_ERR_BAD_ARG, "st_residual_noalloc: null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ST_ERR_BAD_ARG, "st_residual_noalloc: dt must be positive");
    Problem pb;
    int rc = make_problem(mesh, N, Nt, eq, pb);
    if (rc != ST_OK) return rc;
    const bool visc = grad_pass(pb);
    const size_t qbytes = visc ? sizeof(double) * (size_t)visc_len(pb) : 0;
    if (Q_OFFSET + qbytes > SCRATCH_BYTES)
        return set_error(ST_ERR_BAD_ARG, "st_residual_noalloc: the viscous pass's output (" + std::to_string(qbytes) +
                                             " bytes) exceeds the static scratch (" +
                                             std::to_string(SCRATCH_BYTES - Q_OFFSET) + " bytes)");
    void* base = nullptr;
    rc = scratch_ptr(&base);
    if (rc != ST_OK) return rc;
    char* sp = (char*)base;
    OpSeg* dv = (OpSeg*)sp;
    OpSeg* dop = (OpSeg*)(sp + DESC_SLOT);
    double* Q = (double*)(sp + Q_OFFSET);
    hipStream_t st = (hipStream_t)stream;
    const OpSeg b = base_opseg(pb, dt);
    if (visc) {
        OpSeg g = b;
        visc_tiles(g, pb);
        g.U = dptr(U);
        g.out = dptr(Q);
        put_opseg(dv, g, st);
    }
    OpSeg s = b;
    if (visc) s.Q = dptr(Q);
    s.U = dptr(U);
    s.uprev = u_prev;
    s.out = dptr(R);
    put_opseg(dop, s, st);
    const int G = op_blocks(pb);
    if (visc) pb.ops->visc_res64(dv, 1, G, st);
    pb.ops->res64(dop, 1, G, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ST_ERR_HIP, std::string("st_residual_noalloc: ") + hipGetErrorString(e));
    return ST_OK;
}

}  // extern "C"
