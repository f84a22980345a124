/*
 * st.h -- C ABI of the MI355X space-time DG-SEM slab library (libstdg.so).
 *
 * Method: Versbach, Linders, Kloefkorn, Birken, "Theoretical and Practical
 * Aspects of Space-Time DG-SEM Implementations" (arXiv 2201.05800).
 *
 * One SLAB is one time element [t0, t0 + dt] of a periodic Cartesian spatial
 * mesh (Sec. "Space-Time DG-SEM": the upwind flux in time decouples the time
 * elements, so each is a stand-alone system).  The unknowns are the nodal
 * values at the tensor LGL nodes of every space-time element, N + 1 nodes per
 * space axis and Nt nodes in time (degree Nt - 1, the Remark after eq.
 * (stsurfaceint)).  The library evaluates the slab residual, its exact
 * Jacobian-vector product, and solves the slab system by Newton-GMRES; every
 * step runs in hand-written HIP kernels for gfx950.
 *
 * CONVENTIONS
 *   Pointers named U, R, v, Jv, u_prev, U_out, u_next are DEVICE pointers to
 *   FP64 arrays owned by the caller (e.g. torch CUDA tensors); the library
 *   keeps none of them after the call returns.  `stream` is a hipStream_t
 *   (NULL = default stream); every call is asynchronous on that stream
 *   unless stated otherwise.
 *
 *   Slab vector layout (length n = E * nv * Nt * ns):
 *       index = ((e * nv + var) * Nt + j) * ns + s
 *   e = ex + Kx * (ey + Ky * ez) (element, x fastest), j = time node,
 *   s = ix + n1 * (iy + n1 * iz) (spatial node, x fastest), n1 = N + 1,
 *   ns = n1^dim.  This is a permutation of the coefficient vector
 *   (u^1, ..., u^Nt) of eq. (StCoeff); node order does not change the
 *   solution (Sec. "Algorithmic Aspects").
 *   Spatial vectors (u_prev, u_next): index = (e * nv + var) * ns + s.
 *
 *   Return codes: ST_OK (0) or a negative ST_ERR_*; st_last_error() gives a
 *   thread-local message.  No C++ exception crosses this boundary.
 */
#ifndef ST_H
#define ST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ST_OK 0
#define ST_PENDING 1
#define ST_ERR_BAD_ARG (-1)        /* invalid handle, size, pointer or option  */
#define ST_ERR_HIP (-2)            /* a HIP runtime call failed               */
#define ST_ERR_NONFINITE (-3)      /* NaN/Inf in an input or in a residual    */
#define ST_ERR_NO_CONVERGENCE (-4) /* Newton/GMRES limit reached              */
#define ST_ERR_OOM_ADMISSION (-5)  /* request larger than the server's budget */
#define ST_ERR_UNSUPPORTED (-6)    /* (eq, dim, N, Nt) not compiled in, or an  */
                                   /* option not available for it             */
#define ST_ERR_NOT_FOUND (-7)      /* unknown ticket                          */

#define ST_MAX_SLABS 64            /* slabs of one multi-slab system           */
#define ST_ERR_CANCELLED (-8)      /* ticket cancelled before completion      */

/* Cartesian mesh, cf. cartesianDomain(lower, upper, counts) in Sec.
 * "DG-SEM in Space".  Axes are periodic unless bc[a] = 1: then both ends of
 * axis a are Dirichlet boundaries with the exterior state bc_value of the
 * equation (the boundary convective flux of the surface integral): the
 * scalar linear equations with a constant velocity, and Burgers; the other
 * equations return ST_ERR_UNSUPPORTED from st_create. */
typedef struct {
    int dim;          /* 1, 2 or 3 */
    int K[3];         /* elements per axis (unused axes: 1) */
    double lo[3];     /* lower corner */
    double hi[3];     /* upper corner */
    int bc[3];        /* 0: periodic (default), 1: Dirichlet */
} st_mesh_t;

/* u_t + div(Fc(u) - Fv(u, grad u)) = 0, eq. (general) without source. */
typedef enum {
    ST_ADVECTION = 1,   /* Fc = a u; Rusanov = upwind                       */
    ST_ADVDIFF_BR1 = 2, /* Fc = a u, Fv = nu grad u; BR1 viscous flux        */
    ST_BURGERS = 3,     /* Fc = u^2 / 2, dim = 1                             */
    ST_EULER = 4,       /* compressible Euler, Sec. "Euler Equations"        */
    ST_NS_BR1 = 5,      /* compressible Navier-Stokes (constant mu, Stokes   */
                        /* hypothesis, T = p / rho, Fourier heat flux), BR1  */
    ST_ADVDIFF_SIPG = 6 /* Fc = b u, Fv = nu grad u; the paper's symmetric   */
                        /* interior penalty flux, eta = 10 N^2 (Sec. "DG-SEM */
                        /* in Space")                                        */
} st_eq_kind_t;

typedef struct {
    int kind;         /* st_eq_kind_t */
    double a[3];      /* advection velocity (ADVECTION, ADVDIFF_BR1) */
    double nu;        /* diffusivity (ADVDIFF_BR1) */
    double gamma;     /* ratio of specific heats (EULER, NS_BR1) */
    double mu;        /* dynamic viscosity (NS_BR1) */
    double prandtl;   /* Prandtl number (NS_BR1) */
    /* ADVECTION, ADVDIFF_BR1, ADVDIFF_SIPG in 2D with N <= 4: the velocity
     * field b(x) = a + omega e_z x (x - center), a rotation about `center`
     * (the rotating pulse of Sec. "Experiments / Advection-Diffusion",
     * eq. (advdiffeq)); omega = 0: the constant velocity a.  The flux b(x_i) u_i
     * is interpolated at the nodes; b is divergence free and its normal
     * component is continuous across every face, the periodic seams included. */
    double omega;
    double center[3];
    /* exterior state g of Dirichlet boundaries (st_mesh_t.bc): the Rusanov
     * flux with g, BR1 with u_hat = g and the interior viscous flux, the
     * interior penalty by Nitsche's terms */
    double bc_value;
} st_equation_t;

/* Newton-GMRES options (the paper names Newton-GMRES, Sec. "Euler
 * Equations"; everything below is this library's choice). */
typedef struct {
    int restart;       /* GMRES restart length m, 1..32 (default 30)            */
    int max_newton;    /* outer iterations; each is one residual evaluation and */
                       /* one GMRES cycle of at most m steps (default 60)       */
    int cgs_passes;    /* classical Gram-Schmidt passes: 1 or 2 (default 1), or */
                       /* 0 adaptive: one pass, and a second one in the steps   */
                       /* where the new vector's norm falls below 1/sqrt(2) of  */
                       /* the projected vector's (selective reorthogonalisation)*/
    int inner_fp32;    /* 1: JVPs in FP32 (state, math, accumulation); the      */
                       /* residual, Arnoldi and update stay FP64                */
    double gmres_rtol; /* minimum inner forcing term eta (default 1e-3; raised  */
                       /* to 1e-5 at least when inner_fp32)                     */
    int timing;        /* bit mask of ST_K_* kernel classes to time with HIP    */
                       /* events on the solve's stream (0 = none); an event    */
                       /* pair per launch slows launch-bound solves (17 % for  */
                       /* a 409,600-unknown slab with one class timed)          */
    int precond;       /* 0: none (default); 1: element-block Jacobi, right     */
                       /* preconditioning (element blocks of at most 1024       */
                       /* unknowns, nv Nt (N+1)^d); 2: for coupled slabs        */
                       /* (st_solve_slabs) the same blocks plus forward         */
                       /* substitution over the slabs; as 1 for a single slab;  */
                       /* the server takes 0 and 1                              */
} st_solver_opts_t;

/* Kernel classes of the slab solve (bits of st_solver_opts_t.timing and
 * indices of st_stats_t.kernel_us / kernel_calls). */
enum {
    ST_K_RESIDUAL = 0,  /* residual operator kernel                          */
    ST_K_JVP = 1,       /* Jacobian-vector product operator kernel           */
    ST_K_GRAD = 2,      /* Navier-Stokes viscous pass (BR1 gradient, Fv)     */
    ST_K_MULTIDOT = 3,  /* Gram-Schmidt projections (fused multi-dot)        */
    ST_K_UPDATE = 4,    /* Gram-Schmidt correction + Givens + normalisation  */
    ST_K_NORMALIZE = 5, /* first Krylov vector V_0 = -R / ||R||              */
    ST_K_NEWTON = 6,    /* Newton update U += V y, residual norm, setup      */
    ST_K_PRECOND = 7,   /* element-block Jacobi applications                 */
    ST_K_COUNT = 8
};

typedef struct {
    int newton_its;    /* outer iterations done */
    int gmres_its;     /* Arnoldi steps summed over all cycles */
    double res0;       /* ||R(U0)||_2, U0 = 1 (x) u_prev */
    double res_final;  /* ||R(U)||_2 at return */
    double usec;       /* wall time of the call (host clock, includes syncs) */
    int status;        /* ST_OK or ST_ERR_NO_CONVERGENCE / ST_ERR_NONFINITE */
    double kernel_us[8];  /* summed event time per timed kernel class */
    int kernel_calls[8];  /* timed launches per kernel class          */
    double kernel_bytes[8];  /* algorithmic bytes moved per kernel class (launches  */
                             /* that did work; viscous pass: input + output)        */
} st_stats_t;

typedef struct st_ctx* st_handle_t;
typedef struct st_srv* st_server_t;

/* Library version string. */
const char* st_version(void);
/* Thread-local text of the last error. */
const char* st_last_error(void);

/* Default solver options. */
void st_default_opts(st_solver_opts_t* opts);

/* Host-side LGL nodes x[n], weights w[n] and differentiation matrix
 * D[j * n + k] = l_k'(x_j) (Sec. "DG-SEM in Space"; eq. (DG_in_time) for the
 * temporal D_tau).  n in 2..8.  No GPU needed. */
int st_lgl(int n, double* x, double* w, double* D);

/* Create a handle for one (mesh, N, Nt, equation).  N in 1..5 (1..4 for
 * dim 3; 1..4 for EULER / NS_BR1), Nt in 2..4.  Allocates device workspace
 * on the current device.  Returns ST_ERR_UNSUPPORTED for combinations that
 * are not compiled in.  The calls of one handle share its workspace and its
 * launch descriptors (which a call rewrites only where they differ from what
 * the previous call on the same stream left): calls on one stream follow
 * stream order; calls of one handle on different streams or threads must
 * not overlap (synchronise between them). */
int st_create(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, st_handle_t* out);
int st_destroy(st_handle_t h);

/* Sizes: n_slab = E * nv * Nt * ns unknowns, n_space = E * nv * ns, nv. */
int st_sizes(st_handle_t h, int64_t* n_slab, int64_t* n_space, int* nv);

/* Host: physical coordinates of the spatial nodes, X[(e * dim + a) * ns + s]. */
int st_node_coords(st_handle_t h, double* X);

/* Slab residual (eq. (DG_vs_RK:DG) as right side minus left side):
 *   R = (D_tau^T M_tau (x) I) U - (B_tau (x) I) U* + dt/2 (M_tau (x) I) F(U),
 * upwind U* = (u_prev, 0, ..., 0, u^Nt) (eq. (upwind_flux)), F = M^-1 L_h the
 * DG-SEM spatial operator (Rusanov convective flux, BR1 viscous flux).  Its
 * Jacobian is exactly eq. (Jacobian_ST).  t0 is accepted for the ABI's
 * completeness; the supported equations are autonomous. */
int st_residual(st_handle_t h, const double* U, const double* u_prev, double t0, double dt,
                double* R, void* stream);

/* Jv = dR/dU (U) v, eq. (Jacobian_ST), exact linearisation (active branch of
 * the Rusanov max, d|x|/dx = sign(x), sign(0) = +1).  inner_fp32 = 1
 * evaluates it with FP32 state, arithmetic and accumulation (v read as FP64
 * and rounded, Jv written as FP64). */
int st_jvp(st_handle_t h, const double* U, double t0, double dt, const double* v, double* Jv,
           int inner_fp32, void* stream);

/* Solve R(U) = 0 for one slab by Newton-GMRES from U0 = 1 (x) u_prev; stops
 * when ||R(U)||_2 <= tol * max(1, ||R(U0)||_2).  Writes the whole slab
 * U_out (may be NULL) and the end-of-slab state u_next = (e_Nt^T (x) I) U
 * (eq. (un); may be NULL).  Synchronises `stream` once per outer iteration.
 * On ST_ERR_NO_CONVERGENCE the last iterate is written and stats filled.
 * opts->precond = 1 right-preconditions GMRES with the inverse of an element
 * diagonal block of eq. (Jacobian_ST), the same in every element: for the
 * linear equations the exact block of the uniform periodic mesh; for the
 * nonlinear ones the block of the Jacobian at the constant state u_bar, the
 * quadrature-weighted mean of u_prev (conserved on the periodic mesh, so the
 * same for every slab of a run).  Assembled with the JVP kernels and
 * inverted on the host on the first preconditioned solve with a given dt
 * (a copy of u_prev to the host for u_bar; device memory npe^2 doubles,
 * npe = nv Nt (N+1)^d <= 1024, else ST_ERR_UNSUPPORTED); the solution is that
 * of the unpreconditioned system. */
int st_solve_slab(st_handle_t h, const double* u_prev, double t0, double dt, double tol,
                  const st_solver_opts_t* opts, double* U_out, double* u_next, st_stats_t* stats,
                  void* stream);

/* Several consecutive slabs as one system (the space-time mesh with M
 * elements in time; Sec. "Merits" notes that solving for several time steps
 * at once opens parallelism in time, and Sec. "Adaptive Mesh Refinement" sets
 * up such a system of coupled time elements).  Slab m covers
 * [t0 + m dt, t0 + (m+1) dt]; vectors hold the M slabs one after another, each
 * in the layout of a single slab (M n_slab doubles).  Slab 0 takes u_prev as
 * its upwind inflow, slab m >= 1 the last time node of slab m - 1, so the
 * residual of slab m is st_residual's with u_prev = (e_Nt^T (x) I) U_{m-1},
 * and the Jacobian is block lower bidiagonal: diagonal blocks those of
 * eq. (Jacobian_ST), below them the inflow coupling (unit weight at the first
 * time node).  Its exact solution is that of M sequential slab solves.
 * 1 <= M <= ST_MAX_SLABS, else ST_ERR_BAD_ARG.  The handle's buffers grow to
 * hold M slabs on first use (waits for the device). */
int st_residual_slabs(st_handle_t h, int M, const double* U, const double* u_prev, double t0,
                      double dt, double* R, void* stream);
int st_jvp_slabs(st_handle_t h, int M, const double* U, double t0, double dt, const double* v,
                 double* Jv, int inner_fp32, void* stream);
/* Newton-GMRES on the coupled system of M slabs, as st_solve_slab (same
 * options, preconditioner block in every element of every slab, stopping
 * test on the 2-norm of the whole residual); U_out receives M n_slab values,
 * u_next the end state of the last slab.  opts->precond = 1 applies the
 * element blocks slab by slab (block Jacobi, the inflow coupling left out);
 * opts->precond = 2 solves the block lower bidiagonal system with those
 * blocks on the diagonal and the exact inflow coupling below it, by forward
 * substitution over the slabs, element by element:
 *   z_0 = B^-1 r_0,   z_m = B^-1 (r_m - (e_1 (x) I)(e_Nt^T (x) I) z_{m-1}),
 * so that the preconditioned operator differs from the identity only by the
 * couplings between neighbouring elements (and, for the nonlinear
 * equations, by the frozen mean state); device memory: npe nv (N+1)^d more
 * doubles. */
int st_solve_slabs(st_handle_t h, int M, const double* u_prev, double t0, double dt, double tol,
                   const st_solver_opts_t* opts, double* U_out, double* u_next, st_stats_t* stats,
                   void* stream);

/* The slab residual of st_residual without a handle and without allocating:
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * problem is given as to st_create; U, u_prev, R as to st_residual (device,
 * caller-owned).  Every other device buffer its kernels use -- the launch
 * descriptors and, for ST_NS_BR1, the output of the viscous pass ((dim + 1)
 * Nt (N+1)^(dim-1) (N + 1 + 2 dim) doubles per element) -- lives in one
 * static device array of ST_NOALLOC_SCRATCH_BYTES, which each GPU the
 * library runs on holds until the process ends.  A Navier-Stokes slab whose
 * viscous-pass output does not fit (the array less 32 KiB of descriptors) is
 * rejected with ST_ERR_BAD_ARG; the other equations have no size limit here.  Calls that overlap on one GPU (other
 * streams, other threads) share the array and race; calls on one stream are
 * ordered.  Asynchronous on `stream`; no hipMalloc/hipFree, no host-device
 * copy, no memset (every value of the array that a kernel reads was written
 * by the call before, in stream order).  The first call on a device looks up
 * the array's address there (hipGetSymbolAddress). */
#define ST_NOALLOC_SCRATCH_BYTES (16u << 20)
int st_residual_noalloc(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, const double* U,
                        const double* u_prev, double t0, double dt, double* R, void* stream);

/* Local error estimate of a solved slab by an embedded solution (Sec.
 * "Algorithmic Aspects", adaptive time-stepping; eqs. (RK_stage_equations),
 * (RK_solution), with the tableau of eq. (SBP_to_RK)).  The embedded solution
 * is one order below u^{n+1} where that is reachable, built as in the Radau
 * IIA strategy the paper cites: besides the stage derivatives K_l it may use
 * F(u_prev), the spatial operator at the known start value,
 *   u_hat = u_prev + dt (gamma_0 F(u_prev) + sum_l b_hat_l K_l),
 * with (gamma_0, b_hat) = (0; 1, 0) for Nt = 2 (order 1) and
 * (b_1; 0, b_2, .., b_Nt) for Nt = 3, 4 (order 3 and 4; no formula of this
 * kind has order 5 for Nt = 4).  The stage derivatives follow from the stage
 * values, dt K = (A^-1 (x) I)(U - 1 (x) u_prev) with
 * A^-1 = 2 (D_tau + M_tau^-1 e_1 e_1^T) (eq. SBP_to_RK), so
 *   Nt = 2:  e = u^{n+1} - u_hat = -(U_1 - u_prev),
 *   Nt > 2:  e = w_1 (D_tau (U - 1 (x) u_prev))_1 + (U_1 - u_prev)
 *                - (w_1 dt / 2) F(u_prev)                    (w_1 = 2 b_1),
 * which at a solved slab is b_1 dt (F(U_1) - F(u_prev)).  F(u_prev) is one
 * evaluation of the spatial operator at one time level (the residual
 * kernels instantiated for a single time node).
 * *err (host) = sqrt(mean over the n_space values of
 * (e / (atol + rtol max(|u_prev|, |u^{n+1}|)))^2).  U: device, slab layout;
 * u_prev: device, spatial layout; dt > 0 the slab's step (t0 is accepted;
 * every supported equation is autonomous).  atol, rtol >= 0, atol + rtol > 0,
 * else ST_ERR_BAD_ARG.  Synchronises `stream` (the value is copied to the
 * host); the first call allocates about 4 KB of device memory, and for
 * Nt > 2 one spatial vector (Navier-Stokes: plus its viscous pass's output
 * at one time level), kept by the handle. */
int st_error_estimate(st_handle_t h, const double* U, const double* u_prev, double t0, double dt, double atol,
                      double rtol, double* err, void* stream);

/* Host only: the next step size of the embedded pair above, whose estimate
 * scales like dt^(q+1) with q = 1, 3, 4 the embedded order for Nt = 2, 3, 4:
 * dt_next = dt min(5, max(0.2, 0.9 err^(-1/(q+1)))) (5 when err = 0); a step
 * is accepted when err <= 1.  Nt in 2..4, dt > 0, err >= 0, else
 * ST_ERR_BAD_ARG.  No GPU needed. */
int st_next_dt(int Nt, double dt, double err, double* dt_next);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent slab solves.
 * A server owns one HIP stream and a scheduler thread.  Requests are admitted
 * while their device footprint fits the HBM budget and a slot is free; every
 * scheduler tick advances each admitted request by one outer iteration, with
 * the operator kernels grouped per (equation, dim, N, Nt, precision) and the
 * Krylov kernels batched over all requests.  Each request's arithmetic does
 * not depend on what else is in the batch (per-request reductions in a fixed
 * order), so a result is bitwise the same alone and in a mix.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t hbm_budget_bytes;  /* device memory the server may hold for requests */
    int max_active;            /* admitted requests at most (slots)              */
    int device;                /* HIP device ordinal                              */
} st_server_opts_t;

typedef struct {
    st_mesh_t mesh;
    int N, Nt;
    st_equation_t eq;
    const double* u_prev;      /* HOST pointer, n_space doubles, copied at submit */
    double t0, dt, tol;
    st_solver_opts_t opts;
} st_request_t;

typedef struct {
    int status;                /* ST_OK, ST_ERR_NO_CONVERGENCE, ST_ERR_NONFINITE ... */
    double* u_next;            /* HOST buffer of n_space doubles supplied by caller */
    st_stats_t stats;
    double submit_us, admit_us, done_us;   /* server clock (microseconds)  */
} st_result_t;

int st_server_create(const st_server_opts_t* opts, st_server_t* out);
/* Stops the scheduler thread (pending requests are cancelled) and frees all. */
int st_server_destroy(st_server_t s);
/* Copies *req (and u_prev) and enqueues it; never blocks on the GPU.
 * ST_ERR_OOM_ADMISSION if the request alone exceeds the budget. */
int st_submit(st_server_t s, const st_request_t* req, uint64_t* ticket);
/* Non-blocking: ST_PENDING while queued or running; otherwise the final
 * status, with u_next copied into out->u_next and the ticket released. */
int st_poll(st_server_t s, uint64_t ticket, st_result_t* out);
/* Cancel a queued or running request (its slot is freed at the next tick). */
int st_cancel(st_server_t s, uint64_t ticket);
/* Counters: queued, active, completed, ticks, bytes in use. */
int st_server_stats(st_server_t s, int64_t* queued, int64_t* active, int64_t* completed,
                    int64_t* ticks, int64_t* bytes_in_use);
/* Device bytes a request would hold while admitted. */
int64_t st_request_footprint(const st_request_t* req);

#ifdef __cplusplus
}
#endif
#endif
