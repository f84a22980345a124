/*
 * oracle.h -- CPU FP64 oracle for the space-time DG-SEM slab system.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference that
 * the GPU path is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, includes or calls anything here, and nothing here includes the
 * product's headers.
 *
 * Source: Versbach, Linders, Kloefkorn, Birken, "Theoretical and Practical
 * Aspects of Space-Time DG-SEM Implementations" (arXiv 2201.05800).
 *
 * Three formulations of one slab (one time element [t_n, t_n + dt] times the
 * whole spatial mesh, periodic unless bc[] says otherwise) are implemented:
 *   ORC_FORM_DG       DG-SEM in time, strong form in space: the slab system
 *                     eq. (DG_vs_RK:DG) written as R = RHS - LHS, whose
 *                     Jacobian is exactly eq. (Jacobian_ST).
 *   ORC_FORM_RK       method of lines with Lobatto IIIC, eq. (DG_vs_RK:RK):
 *                     R_RK = U - 1 (x) u^n - dt (A (x) I) F(U), with A typed in
 *                     from the Butcher tableaux of Appendix B.
 *   ORC_FORM_GALERKIN the space-time Galerkin weak form, eqs. (stconvDiscr),
 *                     (stelementint), (stsurfaceint), evaluated with literal
 *                     LGL quadrature over (d+1)-dimensional basis functions.
 *
 * Exact relations between them (checked by the tests):
 *   R     = -((M_tau D_tau + e1 e1^T) (x) I) R_RK
 *   R_Gal = (I_tau (x) M_xi^phys) R
 *
 * Layout of every slab vector (length E * nv * Nt * ns, ns = (N+1)^dim):
 *   index = ((e * nv + v) * Nt + j) * ns + s,
 *   e = ex + Kx * (ey + Ky * ez), s = ix + n1 * (iy + n1 * iz).
 * Spatial vectors (u^n, u at one time level): index = (e * nv + v) * ns + s.
 *
 * All pointers are host pointers owned by the caller.
 */
#ifndef ORACLE_H
#define ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_ADVECTION = 1,      /* u_t + a . grad u = 0                          */
    ORC_ADVDIFF_BR1 = 2,    /* u_t + a . grad u - nu lap u = 0, BR1 viscous  */
    ORC_BURGERS = 3,        /* u_t + (u^2/2)_x = 0, d = 1                    */
    ORC_EULER = 4,          /* compressible Euler, r = d + 2                 */
    ORC_NS_BR1 = 5,         /* compressible Navier-Stokes, BR1 viscous       */
    ORC_ADVDIFF_SIPG = 6    /* u_t + div(b u) - nu lap u = 0, symmetric      */
                            /* interior penalty (eta = 10 p^2)               */
};

enum { ORC_FORM_DG = 0, ORC_FORM_RK = 1, ORC_FORM_GALERKIN = 2 };

typedef struct {
    int dim;            /* 1, 2 or 3                                          */
    int K[3];           /* elements per axis (periodic on every axis)         */
    double lo[3];       /* domain lower corner                                */
    double hi[3];       /* domain upper corner                                */
    int N;              /* spatial polynomial degree (N+1 LGL nodes per axis) */
    int Nt;             /* temporal LGL nodes (degree Nt-1)                   */
    int eq;             /* ORC_* equation kind                                */
    double a[3];        /* advection velocity                                 */
    double nu;          /* diffusivity (advection-diffusion)                  */
    double gamma;       /* ratio of specific heats (Euler / NS)               */
    double mu;          /* dynamic viscosity (NS)                             */
    double prandtl;     /* Prandtl number (NS)                                */
    double react;       /* linear source S(u) = react * u (0 on the hot path) */
    /* advection velocity field of the scalar equations: b(x) = a + omega
     * e_z x (x - center) in 2D (a rotation about `center`; omega = 0 elsewhere) */
    double omega;
    double center[3];
    /* boundaries per axis: 0 periodic, 1 Dirichlet with the exterior state
     * bc_value (scalar equations only) */
    int bc[3];
    double bc_value;
} orc_problem;

typedef struct {
    int newton_its;
    int linear_its;     /* GMRES iterations summed over Newton steps (0 if direct) */
    double res0;
    double res_final;
    int converged;
} orc_stats;

int  orc_nvars(int eq, int dim);
long orc_slab_size(const orc_problem* p);
long orc_space_size(const orc_problem* p);

void orc_set_threads(int n);
int  orc_get_threads(void);

/* LGL nodes x[n], weights w[n] and differentiation matrix D[n*n],
 * D[j*n+k] = l_k'(x_j), from the Lagrange basis definition. */
void orc_lgl(int n, double* x, double* w, double* D);
/* Butcher tableau from the SBP matrices, eq. (SBP_to_RK). */
void orc_butcher_from_sbp(int Nt, double* A, double* b, double* c);
/* Butcher tableau typed in from Appendix B (Nt = 2, 3, 4); returns -1 otherwise. */
int  orc_butcher_appendix_b(int Nt, double* A, double* b, double* c);

/* Physical coordinates of every spatial node: X[(e * dim + a) * ns + s]. */
void orc_node_coords(const orc_problem* p, double* X);

/* F = M^-1 L_h(u) at one time level, eq. (ode). */
void orc_spatial_op(const orc_problem* p, const double* u, double* F);
/* Pointwise flux check: numerical flux along axis `axis` between uL, uR
 * (and BR1 gradients qL, qR laid out [dim][nv], may be NULL for inviscid). */
void orc_num_flux(const orc_problem* p, int axis, const double* uL, const double* uR,
                  const double* qL, const double* qR, double* H);
/* Physical flux along axis, f_a(u) - fv_a(u, q). */
void orc_flux(const orc_problem* p, int axis, const double* u, const double* q, double* f);

/* Slab residual in one of the three forms. */
void orc_residual(const orc_problem* p, int form, const double* U, const double* uprev,
                  double dt, double* R);
/* Exact Jacobian-vector product (forward-mode dual numbers), form DG or RK. */
void orc_jvp(const orc_problem* p, int form, const double* U, double dt, const double* V,
             double* JV);
/* Jacobian of F = M^-1 L_h at u applied to v (spatial level). */
void orc_spatial_jvp(const orc_problem* p, const double* u, const double* v, double* Jv);

/* Newton solve of one slab from U0 = 1 (x) u^n.  Linear solves are dense LU
 * when the slab has at most `dense_limit` unknowns, else restarted GMRES with
 * modified Gram-Schmidt.  Stops when ||R|| <= tol * max(1, ||R(U0)||). */
int  orc_solve(const orc_problem* p, int form, const double* uprev, double dt, double tol,
               int max_newton, int dense_limit, double* U, orc_stats* st);

#ifdef __cplusplus
}
#endif
#endif
