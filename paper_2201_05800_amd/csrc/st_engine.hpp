// st_engine.hpp -- host-side problem description shared by the engine and
// the serving scheduler.
#pragma once
#include "../../include/st.h"
#include "st_krylov.hpp"

#include <string>
#include <vector>

namespace stdg {

struct Problem {
    st_mesh_t mesh;
    st_equation_t eq;
    int N, Nt, n1, nv, ns;
    int K[3];
    double h[3];
    int64_t E, n, nsp;
    const OpTable* ops;
    EqParams P;
    double Dx[64], wx[8], xi[8], Dt[16], wt[4];
};

// the operator needs the viscous pass first (Navier-Stokes BR1)
inline bool grad_pass(const Problem& pb) { return pb.ops->visc_res64 != nullptr; }

// values of the Navier-Stokes viscous pass's output for one slab
inline int64_t visc_len(const Problem& pb) { return pb.E * visc_per_elem(pb.mesh.dim, pb.n1, pb.Nt); }

inline int op_blocks(const Problem& pb) {
    return (int)((pb.E + pb.ops->epb - 1) / pb.ops->epb);
}

int set_error(int code, const std::string& msg);
void lgl_tables(int n, double* x, double* w, double* D);
const OpTable* find_table(int eq, int dim, int n1, int nt, bool rot = false, bool bnd = false);
int make_problem(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, Problem& pb);
OpSeg base_opseg(const Problem& pb, double dt);
// the viscous pass's block traversal (narrower 3D columns than the operator's)
void visc_tiles(OpSeg& s, const Problem& pb);
DynPtr dptr(const void* p);
// B^-1 of a scalar equation's element block (host only), packed for the
// matrix-core kernel; up_host: u_prev on the host (Burgers' mean state)
int scalar_block_inverse(const Problem& pb, const double* up_host, double dt, std::vector<double>& packed);
DynPtr dptr_k(const void* base, int64_t ld, const int* kp);

}  // namespace stdg
