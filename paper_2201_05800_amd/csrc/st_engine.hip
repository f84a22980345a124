// st_engine.hip -- host side of libstdg: handles, LGL tables, the residual
// and JVP entry points, and the Newton-GMRES slab driver.
#include "st_engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace stdg {

thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// ---------------------------------------------------------------------------
// LGL nodes, weights and differentiation matrix.
// Nodes: Newton iteration on (x P_p - P_{p-1}) / ((p+1) P_p), whose roots are
// -1, +1 and the zeros of P_p' (starting from the Chebyshev-Gauss-Lobatto
// points).  Weights 2 / (p (p+1) P_p(x)^2).  D from barycentric weights:
// D_jk = (b_k / b_j) / (x_j - x_k), D_jj = -sum_{k != j} D_jk.
// ---------------------------------------------------------------------------
void lgl_tables(int n, double* x, double* w, double* D) {
    const int p = n - 1;
    std::vector<double> xs(n), xo(n), P(n * (p + 1));
    for (int i = 0; i < n; ++i) xs[i] = std::cos(M_PI * i / p);
    for (int it = 0; it < 200; ++it) {
        double dmax = 0.0;
        for (int i = 0; i < n; ++i) {
            double pm = 1.0, pc = xs[i];
            for (int k = 2; k <= p; ++k) {
                double pn = ((2 * k - 1) * xs[i] * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pn;
            }
            if (p == 1) { pm = 1.0; pc = xs[i]; }
            double xn = xs[i] - (xs[i] * pc - pm) / ((p + 1) * pc);
            dmax = std::max(dmax, std::fabs(xn - xs[i]));
            xs[i] = xn;
        }
        if (dmax < 1e-16) break;
    }
    for (int i = 0; i < n; ++i) x[i] = -xs[i];   // ascending
    for (int i = 0; i < n; ++i) {
        double pm = 1.0, pc = x[i];
        for (int k = 2; k <= p; ++k) {
            double pn = ((2 * k - 1) * x[i] * pc - (k - 1) * pm) / k;
            pm = pc;
            pc = pn;
        }
        w[i] = 2.0 / (p * (p + 1.0) * pc * pc);
    }
    std::vector<double> b(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) b[j] /= (x[j] - x[k]);
    for (int j = 0; j < n; ++j) {
        double diag = 0.0;
        for (int k = 0; k < n; ++k) {
            if (k == j) continue;
            double v = (b[k] / b[j]) / (x[j] - x[k]);
            D[j * n + k] = v;
            diag -= v;
        }
        D[j * n + j] = diag;
    }
}

// Kernel tables by (equation, dim, n1, nt) and velocity kind.  The interior
// penalty variant of advection-diffusion runs the same line-operator kernels
// as BR1 (only the host-built line operator differs); the rotating-velocity
// entries carry the three-part kernels of the linear equations.
const OpTable* find_table(int eq, int dim, int n1, int nt, bool rot, bool bnd) {
    static std::vector<OpTable> tables;
    static std::once_flag once;
    std::call_once(once, [] {
        register_ops_adv(tables);
        register_ops_advdiff(tables);
        register_ops_burgers(tables);
        register_ops_euler(tables);
        register_ops_ns(tables);
        const size_t n0 = tables.size();
        for (size_t i = 0; i < n0; ++i) {
            if (tables[i].res64_rot) {
                OpTable t = tables[i];
                t.res64 = t.res64_rot;
                t.lin32 = t.lin32_rot;
                t.rot = 1;
                tables.push_back(t);
            }
            if (tables[i].res64_bnd) {
                OpTable t = tables[i];
                t.res64 = t.res64_bnd;
                t.lin32 = t.lin32_bnd;
                t.jvp64 = t.jvp64_bnd;
                t.jvp32 = t.jvp32_bnd;
                t.bnd = 1;
                tables.push_back(t);
            }
        }
    });
    const int keq = eq == EQ_ADVDIFF_SIPG ? EQ_ADVDIFF : eq;
    for (const auto& t : tables)
        if (t.eq == keq && t.dim == dim && t.n1 == n1 && t.nt == nt && (t.rot != 0) == rot && (t.bnd != 0) == bnd)
            return &t;
    return nullptr;
}

// ---------------------------------------------------------------------------
// problem description
// ---------------------------------------------------------------------------
int make_problem(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, Problem& pb) {
    if (!mesh || !eq) return set_error(ST_ERR_BAD_ARG, "null mesh or equation");
    const int d = mesh->dim;
    if (d < 1 || d > 3) return set_error(ST_ERR_BAD_ARG, "dim must be 1, 2 or 3");
    if (eq->kind < ST_ADVECTION || eq->kind > ST_ADVDIFF_SIPG) return set_error(ST_ERR_BAD_ARG, "unknown equation kind");
    if (eq->kind == ST_BURGERS && d != 1) return set_error(ST_ERR_UNSUPPORTED, "Burgers is one-dimensional");
    if (N < 1 || Nt < 2) return set_error(ST_ERR_BAD_ARG, "need N >= 1 and Nt >= 2");
    pb.mesh = *mesh;
    pb.eq = *eq;
    pb.N = N;
    pb.Nt = Nt;
    pb.n1 = N + 1;
    pb.nv = nvars_of(eq->kind, d);
    pb.ns = 1;
    for (int a = 0; a < d; ++a) pb.ns *= pb.n1;
    pb.E = 1;
    for (int a = 0; a < 3; ++a) {
        int K = a < d ? mesh->K[a] : 1;
        if (K < 1) return set_error(ST_ERR_BAD_ARG, "element counts must be >= 1");
        double L = a < d ? mesh->hi[a] - mesh->lo[a] : 1.0;
        if (!(L > 0.0)) return set_error(ST_ERR_BAD_ARG, "hi must exceed lo on every axis");
        pb.K[a] = K;
        pb.h[a] = L / K;
        pb.E *= K;
    }
    if (pb.E > (int64_t)1 << 30) return set_error(ST_ERR_BAD_ARG, "too many elements");
    pb.n = pb.E * pb.nv * Nt * pb.ns;
    pb.nsp = pb.E * pb.nv * pb.ns;
    const bool rot = eq->omega != 0.0;
    if (!std::isfinite(eq->omega)) return set_error(ST_ERR_BAD_ARG, "omega must be finite");
    if (rot && (!linear_eq(eq->kind) || d != 2 || pb.n1 > ROT_MAX_N1))
        return set_error(ST_ERR_UNSUPPORTED, "a rotating velocity needs a linear equation in 2D with N <= 4");
    bool bnd = false;
    for (int a = 0; a < 3; ++a) {
        const int b = a < d ? mesh->bc[a] : 0;
        if (b != 0 && b != 1) return set_error(ST_ERR_BAD_ARG, "bc must be 0 (periodic) or 1 (Dirichlet)");
        pb.mesh.bc[a] = b;
        bnd = bnd || b == 1;
    }
    if (bnd && (!(linear_eq(eq->kind) || eq->kind == ST_BURGERS) || rot))
        return set_error(ST_ERR_UNSUPPORTED,
                         "Dirichlet boundaries: the linear equations with a constant velocity, and Burgers");
    if (bnd && !std::isfinite(eq->bc_value)) return set_error(ST_ERR_BAD_ARG, "bc_value must be finite");
    pb.ops = find_table(eq->kind, d, pb.n1, Nt, rot, bnd);
    if (!pb.ops)
        return set_error(ST_ERR_UNSUPPORTED, "(equation, dim, N, Nt) = (" + std::to_string(eq->kind) + ", " +
                                                 std::to_string(d) + ", " + std::to_string(N) + ", " +
                                                 std::to_string(Nt) + ") is not compiled in");
    if ((eq->kind == ST_EULER || eq->kind == ST_NS_BR1) && !(eq->gamma > 1.0))
        return set_error(ST_ERR_BAD_ARG, "gamma must exceed 1");
    if (eq->kind == ST_NS_BR1 && !(eq->prandtl > 0.0)) return set_error(ST_ERR_BAD_ARG, "Prandtl must be > 0");
    for (int a = 0; a < 3; ++a) pb.P.a[a] = eq->a[a];
    pb.P.nu = eq->nu;
    pb.P.gamma = eq->gamma;
    pb.P.mu = eq->mu;
    pb.P.kappa = eq->kind == ST_NS_BR1 ? eq->mu * eq->gamma / ((eq->gamma - 1.0) * eq->prandtl) : 0.0;
    std::vector<double> x(8), w(8), Dm(64);
    lgl_tables(pb.n1, x.data(), w.data(), Dm.data());
    std::memcpy(pb.Dx, Dm.data(), sizeof(double) * pb.n1 * pb.n1);
    std::memcpy(pb.wx, w.data(), sizeof(double) * pb.n1);
    std::memcpy(pb.xi, x.data(), sizeof(double) * pb.n1);
    lgl_tables(Nt, x.data(), w.data(), Dm.data());
    std::memcpy(pb.Dt, Dm.data(), sizeof(double) * Nt * Nt);
    std::memcpy(pb.wt, w.data(), sizeof(double) * Nt);
    return ST_OK;
}

// division by an invariant integer (Granlund-Montgomery): with 2^k >= d and
// M = ceil(2^(31+k) / d), floor(n / d) = (n M) >> (31 + k) for 0 <= n < 2^31
static void div_magic(int d, unsigned& m, int& sh) {
    int k = 0;
    while (((uint64_t)1 << k) < (uint64_t)d) ++k;
    m = (unsigned)((((uint64_t)1 << (31 + k)) + (uint64_t)d - 1) / (uint64_t)d);
    sh = 31 + k;
}

// Spatial operator of a linear equation (advection, advection-diffusion with
// BR1 or with the symmetric interior penalty) along axis a, restricted to one
// line of n1 nodes: the contribution F_i at node i of the line is linear in
// the line's values u, the left neighbour's line uL and the right one's uR
// (eqs. elementint, surfaceint in strong form, flux:llf).  Evaluated here for
// the unit vectors, it gives F = A u + BL uL + BR uR; BL is nonzero only in
// its last column (the neighbour's face value enters every node through the
// lift) and its first row (the face flux needs the neighbour's normal
// derivative), BR likewise in its first column and last row (checked).
//   advection: -(2/h) D (a u), Rusanov {a u} + lambda/2 (u_L - u_R) at the
//              faces, lifted by -(2/h) M^-1 B (H - f);
//   BR1:       lifted gradient with u_hat = {u}, central {nu q};
//   SIPG:      the symmetric interior penalty form, sigma = eta nu / h,
//              eta = 10 N^2, on the line with J = 2/h:
//              -nu J^2 M^-1 D^T M D u, and per face the consistency term
//              nu {u'} (end row), the symmetry term nu/2 J^2 M^-1 D^T e (jump)
//              (every row), the penalty -sigma J/w (jump) (end row).
// `av` is the velocity, `lam` the Rusanov wave speed, `nu` the diffusivity.
// The line operator as a function of the line u, the neighbours' lines uL,
// uR and, at a Dirichlet boundary (bl: lower end, br: upper end), the
// exterior state gv in place of that neighbour: the Rusanov flux with gv,
// BR1 with u_hat = gv and the own viscous flux, SIPG by Nitsche's terms
// (the face terms with the own derivative instead of the average, gv instead
// of the neighbour's face value, the symmetry term at full weight).
static void line_apply(const Problem& pb, int a, double av, double lam, double nu, const double* u,
                       const double* uL, const double* uR, bool bl, bool br, double gv, double* acc) {
    const int n1 = pb.n1, N = n1 - 1;
    const double J = 2.0 / pb.h[a];
    const bool sipg = pb.eq.kind == ST_ADVDIFF_SIPG;
    const double eta = pb.N > 0 ? 10.0 * pb.N * pb.N : 1.0;
    const double sig = eta * nu / pb.h[a];
    const double iw0 = 1.0 / pb.wx[0];
    const double* D = pb.Dx;
    const double* w = pb.wx;
    const double uLf = bl ? gv : uL[N], uRf = br ? gv : uR[0];     // the states across the two faces
    double g[8], f[8];
    if (!sipg) {
        for (int i = 0; i < n1; ++i) {
            g[i] = 0.0;
            for (int k = 0; k < n1; ++k) g[i] += D[i * n1 + k] * u[k];
        }
        g[0] += -iw0 * ((bl ? gv : 0.5 * (u[0] + uL[N])) - u[0]);
        g[N] += iw0 * ((br ? gv : 0.5 * (u[N] + uR[0])) - u[N]);
        for (int i = 0; i < n1; ++i) f[i] = u[i] * av - (J * g[i]) * nu;
    } else {
        for (int i = 0; i < n1; ++i) f[i] = u[i] * av;
    }
    for (int i = 0; i < n1; ++i) {
        double sv = 0.0;
        for (int k = 0; k < n1; ++k) sv += D[i * n1 + k] * f[k];
        acc[i] = -J * sv;
    }
    // upper face: Rusanov with u_L = u_N, u_R = uR_0 (BR1: and the
    // neighbour's lifted-gradient flux; at a boundary the own one)
    double fnr = uRf * av;
    if (!sipg) {
        if (br) {
            fnr -= (J * g[N]) * nu;
        } else {
            double gn = 0.0;
            for (int k = 0; k < n1; ++k) gn += D[k] * uR[k];
            gn += -iw0 * (0.5 * (uR[0] + u[N]) - uR[0]);
            fnr -= (J * gn) * nu;
        }
    }
    acc[N] -= J * iw0 * (0.5 * (fnr - f[N]) + 0.5 * lam * (u[N] - uRf));
    // lower face: u_L = uL_N, u_R = u_0
    double fnl = uLf * av;
    if (!sipg) {
        if (bl) {
            fnl -= (J * g[0]) * nu;
        } else {
            double gn = 0.0;
            for (int k = 0; k < n1; ++k) gn += D[N * n1 + k] * uL[k];
            gn += iw0 * (0.5 * (uL[N] + u[0]) - uL[N]);
            fnl -= (J * gn) * nu;
        }
    }
    acc[0] += J * iw0 * (0.5 * (fnl - f[0]) + 0.5 * lam * (uLf - u[0]));
    if (sipg && nu != 0.0) {
        double du[8];
        for (int q = 0; q < n1; ++q) {
            du[q] = 0.0;
            for (int k = 0; k < n1; ++k) du[q] += D[q * n1 + k] * u[k];
        }
        double dR = 0.0, dL = 0.0;   // the neighbours' derivatives at the shared faces
        for (int k = 0; k < n1; ++k) {
            dR += br ? 0.0 : D[k] * uR[k];
            dL += bl ? 0.0 : D[N * n1 + k] * uL[k];
        }
        const double avR = br ? J * du[N] : 0.5 * J * (du[N] + dR);
        const double avL = bl ? J * du[0] : 0.5 * J * (du[0] + dL);
        const double sR = br ? 1.0 : 0.5, sL = bl ? 1.0 : 0.5;
        const double jR = u[N] - uRf, jL = uLf - u[0];
        for (int i = 0; i < n1; ++i) {
            double vol = 0.0;
            for (int q = 0; q < n1; ++q) vol += w[q] * D[q * n1 + i] * du[q];
            acc[i] += -nu * J * J * vol / w[i] + nu * J * J * (sR * D[N * n1 + i] * jR + sL * D[i] * jL) / w[i];
        }
        acc[N] += nu * (J / w[N]) * avR - sig * (J / w[N]) * jR;
        acc[0] += -nu * (J / w[0]) * avL + sig * (J / w[0]) * jL;
    }
}

// Spatial operator of a linear equation (advection, advection-diffusion with
// BR1 or with the symmetric interior penalty) along axis a, restricted to one
// line of n1 nodes: the contribution F_i at node i of the line is linear in
// the line's values u, the left neighbour's line uL and the right one's uR
// (eqs. elementint, surfaceint in strong form, flux:llf).  Evaluated here for
// the unit vectors, it gives F = A u + BL uL + BR uR; BL is nonzero only in
// its last column (the neighbour's face value enters every node through the
// lift) and its first row (the face flux needs the neighbour's normal
// derivative), BR likewise in its first column and last row (checked).
//   advection: -(2/h) D (a u), Rusanov {a u} + lambda/2 (u_L - u_R) at the
//              faces, lifted by -(2/h) M^-1 B (H - f);
//   BR1:       lifted gradient with u_hat = {u}, central {nu q};
//   SIPG:      the symmetric interior penalty form, sigma = eta nu / h,
//              eta = 10 N^2, on the line with J = 2/h:
//              -nu J^2 M^-1 D^T M D u, and per face the consistency term
//              nu {u'} (end row), the symmetry term nu/2 J^2 M^-1 D^T e (jump)
//              (every row), the penalty -sigma J/w (jump) (end row).
// `av` is the velocity, `lam` the Rusanov wave speed, `nu` the diffusivity.
// bnd (may be null): the Dirichlet variants, A_L, A_R, A_LR (own line, the
// element at the lower / upper / both boundaries) and the exterior state's
// coefficients gL_L, gR_R, gL_LR, gR_LR.
static void line_operator_parts(const Problem& pb, int a, double av, double lam, double nu, double* out,
                                double* bnd = nullptr) {
    const int n1 = pb.n1, N = n1 - 1;
    auto apply = [&](const double* u, const double* uL, const double* uR, double* acc) {
        line_apply(pb, a, av, lam, nu, u, uL, uR, false, false, 0.0, acc);
    };
    double M[3][8][8];   // [input line][row i][column k]
    for (int which = 0; which < 3; ++which)
        for (int k = 0; k < n1; ++k) {
            double in[3][8] = {};
            in[which][k] = 1.0;
            double acc[8];
            apply(in[0], in[1], in[2], acc);
            for (int i = 0; i < n1; ++i) M[which][i][k] = acc[i];
        }
    // the kernel keeps only the last column and first row of BL (first
    // column and last row of BR): anything else would be lost
    for (int i = 0; i < n1; ++i)
        for (int k = 0; k < n1; ++k) {
            if (!(k == N || i == 0) && M[1][i][k] != 0.0) std::abort();
            if (!(k == 0 || i == N) && M[2][i][k] != 0.0) std::abort();
        }
    double* A = out;
    double* HL = A + n1 * n1;
    double* HR = HL + n1;
    double* FL = HR + n1;
    double* FR = FL + n1;
    for (int i = 0; i < n1; ++i)
        for (int k = 0; k < n1; ++k) A[i * n1 + k] = M[0][i][k];
    for (int i = 0; i < n1; ++i) {
        HL[i] = M[1][i][N];
        HR[i] = M[2][i][0];
    }
    FL[0] = FR[0] = 0.0;
    for (int m = 1; m < n1; ++m) {
        FL[m] = M[1][0][N - m];   // row 0: left neighbour's node at distance m from its face
        FR[m] = M[2][N][m];       // row N: right neighbour's node at distance m
    }
    if (!bnd) return;
    // Dirichlet variants: own-line matrices with the neighbour across a
    // boundary replaced by the exterior state (g = 0), and the response to
    // g = 1 (the other neighbour's contributions HL/HR, FL/FR are unchanged)
    const double zero[8] = {};
    for (int var = 0; var < 3; ++var) {
        const bool bl = var != 1, br = var != 0;
        double* Av = bnd + var * n1 * n1;
        for (int k = 0; k < n1; ++k) {
            double in[8] = {};
            in[k] = 1.0;
            double acc[8];
            line_apply(pb, a, av, lam, nu, in, zero, zero, bl, br, 0.0, acc);
            for (int i = 0; i < n1; ++i) Av[i * n1 + k] = acc[i];
        }
    }
    double* gc = bnd + 3 * n1 * n1;       // gL_L, gR_R, gL_LR (both ends), gR_LR = 0
    double acc[8];
    line_apply(pb, a, av, lam, nu, zero, zero, zero, true, false, 1.0, acc);
    for (int i = 0; i < n1; ++i) gc[i] = acc[i];
    line_apply(pb, a, av, lam, nu, zero, zero, zero, false, true, 1.0, acc);
    for (int i = 0; i < n1; ++i) gc[n1 + i] = acc[i];
    line_apply(pb, a, av, lam, nu, zero, zero, zero, true, true, 1.0, acc);
    for (int i = 0; i < n1; ++i) {
        gc[2 * n1 + i] = acc[i];
        gc[3 * n1 + i] = 0.0;
    }
}

// The line operators of the descriptor: constant velocity, one per axis at
// stride LIN_AXIS; rotating velocity (2D), three parts per axis (viscous,
// central advection per unit velocity, dissipation per unit speed) packed
// at stride n1^2 + 4 n1.
static void line_operators(const Problem& pb, double* lin, double* linb) {
    const double nu = pb.eq.kind == ST_ADVECTION ? 0.0 : pb.P.nu;
    if (!pb.ops->rot) {
        const int LB = 3 * pb.n1 * pb.n1 + 4 * pb.n1;
        for (int a = 0; a < pb.mesh.dim; ++a) {
            const double av = pb.P.a[a];
            line_operator_parts(pb, a, av, std::fabs(av), nu, lin + a * LIN_AXIS,
                                pb.mesh.bc[a] ? linb + a * LB : nullptr);
        }
        return;
    }
    const int LA = pb.n1 * pb.n1 + 4 * pb.n1;
    for (int a = 0; a < pb.mesh.dim; ++a) {
        line_operator_parts(pb, a, 0.0, 0.0, nu, lin + (a * 3 + 0) * LA);
        line_operator_parts(pb, a, 1.0, 0.0, 0.0, lin + (a * 3 + 1) * LA);
        line_operator_parts(pb, a, 0.0, 1.0, 0.0, lin + (a * 3 + 2) * LA);
    }
}

// Block traversal: columns of tx x ty elements swept through z, each column
// row by row, so that a face neighbour is met again within a few rows of the
// column (L2 reuse of halo traces) rather than a whole plane of the mesh
// later.  tx is a multiple of the elements per block and divides K0, ty
// divides K1; 2D takes whole-height strips 64 elements wide, 3D columns of
// about want3d x want3d elements (measured best: about 10 x 10 for the
// operator kernels, 4 x 4 for the viscous pass).  Lexicographic when K0 is
// not a multiple of the block width.
static void set_tiles(OpSeg& s, const Problem& pb, int want3d) {
    const int epb = pb.ops->epb;
    s.tx = 0;
    s.ty = 0;
    if (pb.mesh.dim >= 2 && pb.K[0] % epb == 0) {
        const int want_x = pb.mesh.dim == 2 ? 64 : want3d, want_y = pb.mesh.dim == 2 ? pb.K[1] : want3d;
        int tx = epb;
        for (int c = epb; c <= pb.K[0] && c <= std::max(want_x, epb); c += epb)
            if (pb.K[0] % c == 0) tx = c;
        int ty = 1;
        for (int c = 1; c <= pb.K[1] && c <= want_y; ++c)
            if (pb.K[1] % c == 0) ty = c;
        s.tx = tx;
        s.ty = ty;
        const int bx = tx / epb;
        s.tk[2] = bx;                         // blocks per tile row
        s.tk[1] = bx * ty;                    // per tile layer
        s.tk[0] = bx * ty * pb.K[2];          // per tile
        s.tk[3] = pb.K[0] / tx;               // tiles along x
        for (int i = 0; i < 4; ++i) div_magic(s.tk[i], s.tm[i], s.ts[i]);
    }
}

void visc_tiles(OpSeg& s, const Problem& pb) { set_tiles(s, pb, 4); }

OpSeg base_opseg(const Problem& pb, double dt) {
    OpSeg s;
    std::memset(&s, 0, sizeof(s));
    for (int a = 0; a < 3; ++a) {
        s.K[a] = pb.K[a];
        s.rh[a] = 2.0 / pb.h[a];
    }
    s.E = (int)pb.E;
    for (int a = 0; a < 2; ++a) div_magic(pb.K[a], s.dm[a], s.ds[a]);
    set_tiles(s, pb, 12);
    s.iw0 = 1.0 / pb.wx[0];
    if (linear_eq(pb.eq.kind)) line_operators(pb, s.lin, s.linb);
    for (int a = 0; a < 3; ++a) s.bc[a] = a < pb.mesh.dim ? pb.mesh.bc[a] : 0;
    s.bcg = pb.eq.bc_value;
    for (int a = 0; a < 2; ++a) {
        s.lo[a] = pb.mesh.lo[a];
        s.center[a] = pb.eq.center[a];
    }
    std::memcpy(s.xi, pb.xi, sizeof(s.xi));
    s.omega = pb.eq.omega;
    s.P = pb.P;
    s.dt = dt;
    s.blk0 = 0;
    s.nblk = op_blocks(pb);
    std::memcpy(s.Dx, pb.Dx, sizeof(s.Dx));
    std::memcpy(s.wx, pb.wx, sizeof(s.wx));
    std::memcpy(s.Dt, pb.Dt, sizeof(s.Dt));
    std::memcpy(s.wt, pb.wt, sizeof(s.wt));
    return s;
}

DynPtr dptr(const void* p) { return DynPtr{p, 0, nullptr, 0}; }
DynPtr dptr_k(const void* base, int64_t ld, const int* kp) { return DynPtr{base, ld, kp, 0}; }

}  // namespace stdg

using namespace stdg;

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct st_ctx {
    Problem pb;
    int device = 0;
    OpSeg* d_op = nullptr;      // 8 operator descriptor slots
    VecSeg* d_vs = nullptr;     // 1 vector descriptor slot
    GState* d_st = nullptr;
    double* d_part = nullptr;
    double* Q = nullptr;        // NS: -Fv of U along every axis (residual)
    double* dQ = nullptr;       // NS: its tangent in the JVP direction
    float* U32 = nullptr;
    float* dQ32 = nullptr;
    double* V = nullptr;        // Krylov basis (m vectors)
    double* w = nullptr;
    double* R = nullptr;
    double* U = nullptr;
    int m_alloc = 0;
    GState* h_st = nullptr;     // pinned host mirror of the state header
    hipEvent_t ev_state = nullptr;  // recorded after each copy of the header
    std::vector<void*> allocs;
    // element-block Jacobi: B^-1 packed for the matrix cores, the dt it was
    // assembled for, the preconditioned direction z, 3 descriptor slots;
    // pc_C: the first-time-node columns of B^-1 (forward substitution over
    // the slabs of a coupled system)
    double* binvT = nullptr;
    double* pc_C = nullptr;
    double pc_dt = 0.0;
    std::vector<double> pc_ubar;   // nonlinear: the mean state it was assembled at
    double* pz = nullptr;
    PcSeg* d_pc = nullptr;
    // embedded error estimate: partial sums + result; for Nt > 2 the spatial
    // operator at u_prev (a spatial vector) and, for Navier-Stokes, the
    // viscous pass's output at one time level
    double* d_est = nullptr;
    double* est_f = nullptr;
    double* est_q = nullptr;
    // vector buffers (V, w, R, U, pz, Q, dQ, U32, dQ32, d_part) hold `cap`
    // consecutive slabs; the solve's descriptors: 4 cap operator segments
    // (residual viscous pass, residual, JVP viscous pass, JVP) and cap + 2
    // vector segments (Krylov, per-slab initial guess, extraction)
    int cap = 1;
    OpSeg* d_opm = nullptr;
    VecSeg* d_vsm = nullptr;

    // Host copies of the operator descriptors last written to the slots of
    // d_op and d_opm, each with the stream that wrote it.  A descriptor is
    // about 10 KB, written by five launches; a call that would write the
    // same bytes to a slot on the same stream skips them, since stream order
    // has already put those bytes there (repeated st_residual / st_jvp calls
    // on the same buffers: 25-70 us less per call).  Every write to those
    // slots goes through put_op; reallocating d_opm clears the copies.
    struct OpCopy {
        const OpSeg* dst;
        hipStream_t st;
        OpSeg v;
    };
    std::vector<OpCopy> op_copies;
    void put_op(OpSeg* dst, const OpSeg& v, hipStream_t st) {
        for (auto& c : op_copies) {
            if (c.dst != dst) continue;
            if (c.st == st && std::memcmp(&c.v, &v, sizeof(OpSeg)) == 0) return;
            put_opseg(dst, v, st);
            c.st = st;
            c.v = v;
            return;
        }
        put_opseg(dst, v, st);
        op_copies.push_back(OpCopy{dst, st, v});
    }

    // optional HIP-event timing of kernel classes (st_solver_opts_t.timing)
    struct Timer {
        int mask = 0;
        std::vector<hipEvent_t> pool;
        std::vector<std::pair<int, size_t>> marks;   // (class, first event)
        size_t used = 0;
        void reset(int m) { mask = m; marks.clear(); used = 0; }
        // time `launch` if its class is selected: a single kernel is timed by
        // its own start/end (ext launch), several kernels by stream events
        template <class F>
        void run(int cls, hipStream_t st, F&& launch, bool single = true) {
            if (!((mask >> cls) & 1)) { launch(); return; }
            while (pool.size() < used + 2) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) { launch(); return; }
                pool.push_back(e);
            }
            if (single) {
                launch_timing() = LaunchTiming{pool[used], pool[used + 1]};
                launch();
                launch_timing() = LaunchTiming{};
            } else {
                (void)hipEventRecord(pool[used], st);
                launch();
                (void)hipEventRecord(pool[used + 1], st);
            }
            marks.push_back({cls, used});
            used += 2;
        }
        void collect(st_stats_t* s) {
            for (int c = 0; c < ST_K_COUNT; ++c) { s->kernel_us[c] = 0.0; s->kernel_calls[c] = 0; }
            for (auto& mk : marks) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, pool[mk.second], pool[mk.second + 1]) == hipSuccess) {
                    s->kernel_us[mk.first] += 1000.0 * ms;
                    s->kernel_calls[mk.first] += 1;
                }
            }
        }
    } timer;

    template <class T>
    int alloc(T** p, size_t count) {
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void**)p, count * sizeof(T));
        if (e != hipSuccess) return set_error(ST_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(*p);
        return ST_OK;
    }
    void release(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    ~st_ctx() {
        for (hipEvent_t e : timer.pool) (void)hipEventDestroy(e);
        for (void* p : allocs) (void)hipFree(p);
        if (h_st) (void)hipHostFree(h_st);
        if (ev_state) (void)hipEventDestroy(ev_state);
    }
};

#define CHK(x)                                  \
    do {                                        \
        int rc_ = (x);                          \
        if (rc_ != ST_OK) return rc_;           \
    } while (0)
#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return set_error(ST_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Vector buffers for M consecutive slabs.  Growing waits for the device and
// drops the buffers' contents (and the Krylov basis size).
static int ensure_cap(st_ctx* h, int M) {
    const Problem& pb = h->pb;
    if (M <= h->cap && h->d_opm) return ST_OK;
    const int c = std::max(M, h->cap);
    HIPCHK(hipDeviceSynchronize());
    for (void* p : {(void*)h->V, (void*)h->w, (void*)h->R, (void*)h->U, (void*)h->pz, (void*)h->Q, (void*)h->dQ,
                    (void*)h->U32, (void*)h->dQ32, (void*)h->d_part, (void*)h->d_opm, (void*)h->d_vsm})
        h->release(p);
    h->V = h->w = h->R = h->U = h->pz = h->Q = h->dQ = h->d_part = nullptr;
    h->U32 = h->dQ32 = nullptr;
    h->d_opm = nullptr;
    h->op_copies.clear();
    h->d_vsm = nullptr;
    h->m_alloc = 0;
    h->cap = c;
    const size_t n = (size_t)pb.n * c;
    CHK(h->alloc(&h->d_part, (size_t)vec_blocks((int64_t)n) * (NPART_SLOTS + 1)));
    CHK(h->alloc(&h->d_opm, (size_t)4 * c));
    CHK(h->alloc(&h->d_vsm, (size_t)c + 2));
    if (grad_pass(pb)) {
        CHK(h->alloc(&h->Q, (size_t)visc_len(pb) * c));
        CHK(h->alloc(&h->dQ, (size_t)visc_len(pb) * c));
    }
    return ST_OK;
}

static int ensure_fp32(st_ctx* h) {
    const Problem& pb = h->pb;
    if (h->U32) return ST_OK;
    const size_t n = (size_t)pb.n * h->cap;
    CHK(h->alloc(&h->U32, n));
    if (grad_pass(pb)) CHK(h->alloc(&h->dQ32, (size_t)visc_len(pb) * h->cap));
    return ST_OK;
}

static int ensure_solve(st_ctx* h, int m) {
    const Problem& pb = h->pb;
    if (h->m_alloc >= m && h->V) return ST_OK;
    const size_t n = (size_t)pb.n * h->cap;
    // grow: drop the old basis
    h->release(h->V);
    h->V = nullptr;
    CHK(h->alloc(&h->V, n * m));
    if (!h->w) {
        CHK(h->alloc(&h->w, n));
        CHK(h->alloc(&h->R, n));
        CHK(h->alloc(&h->U, n));
    }
    h->m_alloc = m;
    return ST_OK;
}

// In-place inverse of the row-major n x n matrix A by Gauss-Jordan
// elimination with partial pivoting; false if a pivot vanishes.
static bool invert_dense(std::vector<double>& A, int n) {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
        const double piv = A[(size_t)p * n + c];
        if (!(std::fabs(piv) > 0.0) || !std::isfinite(piv)) return false;
        if (p != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)p * n + k], A[(size_t)c * n + k]);
                std::swap(I[(size_t)p * n + k], I[(size_t)c * n + k]);
            }
        const double ip = 1.0 / piv;
        // columns < c of A are already unit columns: row operations start at c
        for (int k = c; k < n; ++k) A[(size_t)c * n + k] *= ip;
        for (int k = 0; k < n; ++k) I[(size_t)c * n + k] *= ip;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
            for (int k = 0; k < n; ++k) I[(size_t)r * n + k] -= f * I[(size_t)c * n + k];
        }
    }
    A.swap(I);
    return true;
}

// Element diagonal block of the slab Jacobian of the scalar equations,
// assembled on the host.  The own-element part of the spatial operator is the
// Kronecker sum of the own-line operators A_a of line_operator_parts (the
// neighbours' lines excluded), sum_a I (x) .. (x) A_a (x) .. (x) I, so with
// the DG time discretisation (eq. DG_in_time; its Jacobian, eq. Jacobian_ST,
// in this library's node order [j][s]):
//   B[(j,s),(k,s')] = (-w_j Dtau[j][k] - delta_j0 delta_k0) delta_ss'
//                     + (dt/2) w_j delta_jk A_elem[s][s'].
// Burgers: the Jacobian at the constant state u_bar, which is the advection
// operator with velocity u_bar and Rusanov speed |u_bar| (the jump term of
// the linearised wave speed vanishes at a constant state).
static std::vector<double> scalar_block(const Problem& pb, double dt, double ubar) {
    const int d = pb.mesh.dim, n1 = pb.n1, ns = pb.ns, Nt = pb.Nt, npe = Nt * ns;
    const bool burgers = pb.eq.kind == ST_BURGERS;
    const double nu = (pb.eq.kind == ST_ADVECTION || burgers) ? 0.0 : pb.P.nu;
    std::vector<double> Aa((size_t)3 * LIN_AXIS);
    for (int a = 0; a < d; ++a) {
        const double av = burgers ? ubar : pb.P.a[a];
        line_operator_parts(pb, a, av, std::fabs(av), nu, Aa.data() + a * LIN_AXIS);
    }
    std::vector<double> Ael((size_t)ns * ns, 0.0);
    for (int s = 0; s < ns; ++s)
        for (int t = 0; t < ns; ++t)
            for (int a = 0, st = 1; a < d; ++a, st *= n1) {
                bool same = true;
                for (int b = 0, sb = 1; b < d; ++b, sb *= n1)
                    if (b != a && (s / sb) % n1 != (t / sb) % n1) same = false;
                if (same) Ael[(size_t)s * ns + t] += Aa[a * LIN_AXIS + ((s / st) % n1) * n1 + (t / st) % n1];
            }
    std::vector<double> B((size_t)npe * npe, 0.0);
    for (int j = 0; j < Nt; ++j)
        for (int k = 0; k < Nt; ++k) {
            const double tjk = -pb.wt[j] * pb.Dt[j * Nt + k] - (j == 0 && k == 0 ? 1.0 : 0.0);
            for (int s = 0; s < ns; ++s) {
                B[(size_t)(j * ns + s) * npe + k * ns + s] += tjk;
                if (j == k)
                    for (int t = 0; t < ns; ++t)
                        B[(size_t)(j * ns + s) * npe + k * ns + t] += 0.5 * dt * pb.wt[j] * Ael[(size_t)s * ns + t];
            }
        }
    return B;
}

// Mean state u_bar of u_prev (quadrature-weighted, per variable) and the
// largest |u_prev| per variable, from host data [E][nv][ns].
static void mean_state(const Problem& pb, const double* up, std::vector<double>& ubar, std::vector<double>& amax) {
    const int d = pb.mesh.dim;
    std::vector<double> W(pb.ns);
    for (int sn = 0; sn < pb.ns; ++sn) {
        W[sn] = 1.0;
        for (int a = 0, q = sn; a < d; ++a, q /= pb.n1) W[sn] *= pb.wx[q % pb.n1];
    }
    ubar.assign(pb.nv, 0.0);
    amax.assign(pb.nv, 0.0);
    double wsum = 0.0;
    for (int sn = 0; sn < pb.ns; ++sn) wsum += W[sn];
    for (int64_t e = 0; e < pb.E; ++e)
        for (int v = 0; v < pb.nv; ++v) {
            const double* ue = up + (e * pb.nv + v) * pb.ns;
            double t = 0.0;
            for (int sn = 0; sn < pb.ns; ++sn) {
                t += W[sn] * ue[sn];
                amax[v] = std::max(amax[v], std::fabs(ue[sn]));
            }
            ubar[v] += t;
        }
    for (int v = 0; v < pb.nv; ++v) ubar[v] /= wsum * (double)pb.E;
}

namespace stdg {
// B^-1 of the scalar equations packed for the matrix-core kernel (host only;
// u_prev on the host, used for Burgers' mean state).  ST_ERR_UNSUPPORTED for
// a singular block, a rotating velocity or an element block above the limit.
int scalar_block_inverse(const Problem& pb, const double* up_host, double dt, std::vector<double>& packed) {
    const int npe = (int)(pb.nv * pb.Nt * pb.ns);
    if (npe > PC_NPE_MAX) return set_error(ST_ERR_UNSUPPORTED, "element block larger than the preconditioner supports");
    if (pb.ops->rot)
        return set_error(ST_ERR_UNSUPPORTED, "element-block Jacobi needs the same block in every element "
                                             "(not so with a rotating velocity)");
    double ubar = 0.0;
    if (pb.eq.kind == ST_BURGERS) {
        std::vector<double> ub, am;
        mean_state(pb, up_host, ub, am);
        ubar = ub[0];
        if (!std::isfinite(ubar)) return set_error(ST_ERR_BAD_ARG, "preconditioner setup: u_prev is not finite");
    }
    std::vector<double> B = scalar_block(pb, dt, ubar);
    if (!invert_dense(B, npe)) return set_error(ST_ERR_UNSUPPORTED, "element block of the Jacobian is singular");
    packed = pc_pack(B, npe);
    return ST_OK;
}
}  // namespace stdg

// Element diagonal block B of the slab Jacobian and its inverse, for this
// handle's (mesh spacing, N, Nt, equation) and dt.  The scalar equations
// assemble B on the host (scalar_block).  Euler and Navier-Stokes read B off
// the JVP applied to the npe unit vectors of element 0 of a periodic 3^d-element mesh
// with the same spacing (so the element's neighbours are distinct elements
// and B excludes their coupling).  Linear equations: the Jacobian is the same
// in every element.  Nonlinear equations: the Jacobian at the constant state
// u_bar, the quadrature-weighted mean of u_prev (the mean of the conserved
// variables, which the scheme conserves on the periodic mesh, so every slab
// of a run has the same u_bar up to round-off); a frozen-coefficient
// approximation of every element's block.  The inverse is kept per handle
// for its dt (and u_bar), and rebuilt when either changes.
static int upload_block_inverse(st_ctx* h, const std::vector<double>& packed) {
    const Problem& pb = h->pb;
    const int npe = (int)(pb.nv * pb.Nt * pb.ns);
    const std::vector<double> C = pc_inflow_columns(packed, npe, pb.nv, pb.Nt, pb.ns);
    if (!h->binvT) {
        CHK(h->alloc(&h->binvT, packed.size()));
        CHK(h->alloc(&h->pc_C, C.size()));
        CHK(h->alloc(&h->d_pc, 3));
    }
    HIPCHK(hipMemcpy(h->binvT, packed.data(), sizeof(double) * packed.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->pc_C, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice));
    return ST_OK;
}

static int ensure_precond(st_ctx* h, const double* u_prev, double dt, hipStream_t st) {
    const Problem& pb = h->pb;
    const bool lin = linear_eq(pb.eq.kind);
    const int npe = (int)(pb.nv * pb.Nt * pb.ns);
    if (npe > PC_NPE_MAX) return set_error(ST_ERR_UNSUPPORTED, "element block larger than the preconditioner supports");
    if (pb.ops->rot)
        return set_error(ST_ERR_UNSUPPORTED, "element-block Jacobi needs the same block in every element "
                                             "(not so with a rotating velocity)");
    if (!h->pz) CHK(h->alloc(&h->pz, (size_t)pb.n * h->cap));
    const int d = pb.mesh.dim;
    // nonlinear: the reference state u_bar, the quadrature-weighted mean of
    // u_prev (the block is rebuilt when it moves beyond round-off)
    std::vector<double> ubar, up;
    if (!lin) {
        const int64_t nprev = pb.E * pb.nv * pb.ns;
        up.resize((size_t)nprev);
        HIPCHK(hipMemcpyAsync(up.data(), u_prev, sizeof(double) * nprev, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::vector<double> amax;
        mean_state(pb, up.data(), ubar, amax);
        bool same = h->binvT && h->pc_dt == dt && (int)h->pc_ubar.size() == pb.nv;
        for (int v = 0; v < pb.nv; ++v) {
            if (!std::isfinite(ubar[v])) return set_error(ST_ERR_BAD_ARG, "preconditioner setup: u_prev is not finite");
            if (same && std::fabs(ubar[v] - h->pc_ubar[v]) > 1e-12 * std::max(amax[v], 1e-300)) same = false;
        }
        if (same) return ST_OK;
    } else if (h->binvT && h->pc_dt == dt) {
        return ST_OK;
    }
    if (pb.nv == 1) {
        // scalar equations: the block assembled on the host
        std::vector<double> packed;
        CHK(scalar_block_inverse(pb, up.data(), dt, packed));
        if (pc_prepare(npe) != hipSuccess)
            return set_error(ST_ERR_UNSUPPORTED, "element block needs more LDS than the device grants");
        CHK(upload_block_inverse(h, packed));
        h->pc_dt = dt;
        h->pc_ubar = ubar;
        return ST_OK;
    }
    if (pc_prepare(npe) != hipSuccess)
        return set_error(ST_ERR_UNSUPPORTED, "element block needs more LDS than the device grants");
    st_mesh_t m3 = pb.mesh;
    for (int a = 0; a < 3; ++a) {
        m3.K[a] = a < pb.mesh.dim ? 3 : 1;
        m3.lo[a] = 0.0;
        m3.hi[a] = a < pb.mesh.dim ? 3.0 * pb.h[a] : 1.0;
    }
    Problem pp;
    CHK(make_problem(&m3, pb.N, pb.Nt, &pb.eq, pp));
    const int Gp = op_blocks(pp);
    const int64_t np = pp.n, nq = visc_len(pp);
    const bool visc = grad_pass(pb);
    double *din = nullptr, *dout = nullptr, *dstate = nullptr, *dq = nullptr;
    OpSeg* dsegs = nullptr;
    auto cleanup = [&] {
        if (din) (void)hipFree(din);
        if (dout) (void)hipFree(dout);
        if (dstate) (void)hipFree(dstate);
        if (dq) (void)hipFree(dq);
        if (dsegs) (void)hipFree(dsegs);
    };
    // nonlinear: the reference state u_bar at every node of the probe mesh
    std::vector<double> ref;
    if (!lin) {
        ref.resize((size_t)np);
        const int epe = pb.nv * pb.Nt * pb.ns;   // values of one element, [v][j][s]
        for (int64_t i = 0; i < np; ++i) ref[(size_t)i] = ubar[(i % epe) / (pb.Nt * pb.ns)];
    }
    std::vector<OpSeg> segs(npe), gsegs(visc ? npe : 0);
    for (int c = 0; c < npe; ++c) {
        OpSeg s = base_opseg(pp, dt);
        s.blk0 = c * Gp;
        s.nblk = Gp;
        segs[c] = s;
    }
    if (hipMalloc((void**)&din, sizeof(double) * np * npe) != hipSuccess ||
        hipMalloc((void**)&dout, sizeof(double) * np * npe) != hipSuccess ||
        hipMalloc((void**)&dsegs, sizeof(OpSeg) * npe * (visc ? 2 : 1)) != hipSuccess ||
        (!lin && hipMalloc((void**)&dstate, sizeof(double) * np) != hipSuccess) ||
        (visc && hipMalloc((void**)&dq, sizeof(double) * nq * npe) != hipSuccess)) {
        cleanup();
        return set_error(ST_ERR_HIP, "preconditioner setup: device allocation failed");
    }
    for (int c = 0; c < npe; ++c) {
        const DynPtr unit = dptr(din + (size_t)c * np);
        segs[c].uprev = nullptr;
        segs[c].out = dptr(dout + (size_t)c * np);
        if (lin) {
            segs[c].U = unit;                      // R(v) with u_prev = 0 is J v
        } else {
            segs[c].U = dptr(dstate);
            segs[c].V = unit;
            if (visc) {
                OpSeg g = segs[c];
                visc_tiles(g, pp);
                g.out = dptr(dq + (size_t)c * nq);
                gsegs[c] = g;
                segs[c].Q = dptr(dq + (size_t)c * nq);
            }
        }
    }
    std::vector<double> B((size_t)npe * npe);
    hipError_t e = hipMemcpyAsync(dsegs, segs.data(), sizeof(OpSeg) * npe, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && visc)
        e = hipMemcpyAsync(dsegs + npe, gsegs.data(), sizeof(OpSeg) * npe, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !lin)
        e = hipMemcpyAsync(dstate, ref.data(), sizeof(double) * np, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(din, 0, sizeof(double) * np * npe, st);
    if (e == hipSuccess) {
        pc_set_units(din, np, npe, st);           // unit vector c at unknown c of element 0
        if (lin) {
            pb.ops->res64(dsegs, npe, npe * Gp, st);
        } else {
            if (visc) pb.ops->visc_jvp64(dsegs + npe, npe, npe * Gp, st);
            pb.ops->jvp64(dsegs, npe, npe * Gp, st);
        }
        e = hipGetLastError();
    }
    // element 0's block of every response: column c of B
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(B.data(), sizeof(double) * npe, dout, sizeof(double) * np, sizeof(double) * npe, npe,
                             hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return set_error(ST_ERR_HIP, std::string("preconditioner setup: ") + hipGetErrorString(e));
    // the copy holds B^T (row c = response to unit c); transpose to row-major B
    std::vector<double> Bm((size_t)npe * npe);
    for (int i = 0; i < npe; ++i)
        for (int c = 0; c < npe; ++c) Bm[(size_t)i * npe + c] = B[(size_t)c * npe + i];
    if (!invert_dense(Bm, npe)) return set_error(ST_ERR_UNSUPPORTED, "element block of the Jacobian is singular");
    // B^-1 in the kernel's matrix-core operand order
    const std::vector<double> packed = pc_pack(Bm, npe);
    CHK(upload_block_inverse(h, packed));
    h->pc_dt = dt;
    h->pc_ubar = ubar;
    return ST_OK;
}

namespace stdg {
void setup_residual(st_ctx* h, int M, const double* U, const double* u_prev, double* R, double dt, OpSeg* dv,
                    OpSeg* dop, hipStream_t st, bool time_terms = true);
CoupleArgs couple_args(const Problem& pb, int M, const double* in0, const int* kp, int64_t ld, double* out,
                       const int* skip);
void launch_residual(st_ctx* h, int M, const OpSeg* dv, const OpSeg* dop, const CoupleArgs& cp, hipStream_t st);
}  // namespace stdg

extern "C" {

const char* st_version(void) { return "stdg 0.1 (gfx950)"; }
const char* st_last_error(void) { return g_last_error.c_str(); }

void st_default_opts(st_solver_opts_t* o) {
    if (!o) return;
    o->restart = 30;
    o->max_newton = 60;
    o->cgs_passes = 1;
    o->inner_fp32 = 0;
    o->gmres_rtol = 1e-3;
    o->timing = 0;
    o->precond = 0;
}

int st_lgl(int n, double* x, double* w, double* D) {
    if (n < 2 || n > 8 || !x || !w || !D) return set_error(ST_ERR_BAD_ARG, "st_lgl: n in 2..8, non-null outputs");
    lgl_tables(n, x, w, D);
    return ST_OK;
}

int st_create(const st_mesh_t* mesh, int N, int Nt, const st_equation_t* eq, st_handle_t* out) {
    if (!out) return set_error(ST_ERR_BAD_ARG, "null output handle");
    *out = nullptr;
    st_ctx* h = new st_ctx();
    int rc = make_problem(mesh, N, Nt, eq, h->pb);
    if (rc != ST_OK) { delete h; return rc; }
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) { delete h; return set_error(ST_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)); }
    if ((rc = h->alloc(&h->d_op, 8)) != ST_OK ||
        (rc = h->alloc(&h->d_vs, 1)) != ST_OK ||
        (rc = h->alloc(&h->d_st, 1)) != ST_OK ||
        (rc = ensure_cap(h, 1)) != ST_OK) {
        delete h;
        return rc;
    }
    e = hipHostMalloc((void**)&h->h_st, sizeof(GState), hipHostMallocDefault);
    if (e != hipSuccess) { delete h; return set_error(ST_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e)); }
    e = hipEventCreateWithFlags(&h->ev_state, hipEventDisableTiming);
    if (e != hipSuccess) { delete h; return set_error(ST_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e)); }
    *out = h;
    return ST_OK;
}

int st_destroy(st_handle_t h) {
    if (!h) return set_error(ST_ERR_BAD_ARG, "null handle");
    (void)hipDeviceSynchronize();
    delete h;
    return ST_OK;
}

int st_sizes(st_handle_t h, int64_t* n_slab, int64_t* n_space, int* nv) {
    if (!h) return set_error(ST_ERR_BAD_ARG, "null handle");
    if (n_slab) *n_slab = h->pb.n;
    if (n_space) *n_space = h->pb.nsp;
    if (nv) *nv = h->pb.nv;
    return ST_OK;
}

int st_node_coords(st_handle_t h, double* X) {
    if (!h || !X) return set_error(ST_ERR_BAD_ARG, "null argument");
    const Problem& pb = h->pb;
    const int d = pb.mesh.dim, n1 = pb.n1;
    for (int64_t e = 0; e < pb.E; ++e) {
        const int64_t ec[3] = {e % pb.K[0], (e / pb.K[0]) % pb.K[1], e / ((int64_t)pb.K[0] * pb.K[1])};
        for (int a = 0; a < d; ++a)
            for (int s = 0; s < pb.ns; ++s) {
                const int ia = a == 0 ? s % n1 : (a == 1 ? (s / n1) % n1 : s / (n1 * n1));
                X[(e * d + a) * pb.ns + s] = pb.mesh.lo[a] + pb.h[a] * (ec[a] + 0.5 * (1.0 + pb.xi[ia]));
            }
    }
    return ST_OK;
}

int st_residual(st_handle_t h, const double* U, const double* u_prev, double t0, double dt, double* R,
                void* stream) {
    return st_residual_slabs(h, 1, U, u_prev, t0, dt, R, stream);
}

int st_residual_slabs(st_handle_t h, int M, const double* U, const double* u_prev, double t0, double dt, double* R,
                      void* stream) {
    (void)t0;
    if (!h || !U || !u_prev || !R) return set_error(ST_ERR_BAD_ARG, "st_residual: null argument");
    if (M < 1 || M > ST_MAX_SLABS) return set_error(ST_ERR_BAD_ARG, "st_residual_slabs: slabs must be in 1..64");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ST_ERR_BAD_ARG, "st_residual: dt must be positive");
    CHK(ensure_cap(h, M));
    const Problem& pb = h->pb;
    hipStream_t st = (hipStream_t)stream;
    OpSeg* dv = M == 1 ? h->d_op + 0 : h->d_opm;
    OpSeg* dop = M == 1 ? h->d_op + 1 : h->d_opm + M;
    h->timer.reset(0);
    setup_residual(h, M, U, u_prev, R, dt, dv, dop, st);
    launch_residual(h, M, dv, dop, couple_args(pb, M, U, nullptr, 0, R, nullptr), st);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

}  // extern "C"

namespace stdg {

// Descriptors of M consecutive slabs: segment m covers blocks [m G, (m+1) G)
// of one launch; `make(m, seg)` fills slab m's pointers.
template <class F>
static void put_slab_segs(st_ctx* h, OpSeg* dst, int M, const OpSeg& proto, hipStream_t st, F&& make) {
    for (int m = 0; m < M; ++m) {
        OpSeg s = proto;
        s.blk0 = m * proto.nblk;
        make(m, s);
        h->put_op(dst + m, s, st);
    }
}

// Residual of M consecutive slabs at U, in two halves: upload the
// descriptors (viscous pass to dv[0..M), operator to dop[0..M)) and launch.
// Slab 0 takes u_prev as inflow, the others none: the coupling kernel adds
// theirs.  time_terms = false zeroes D_tau in the descriptor: the kernels then
// return w_j (dt/2) F(U_j) - delta_j1 (U_1 - u_prev), the spatial operator at
// every time node (exactly, where U_1 = u_prev).
void setup_residual(st_ctx* h, int M, const double* U, const double* u_prev, double* R, double dt, OpSeg* dv,
                    OpSeg* dop, hipStream_t st, bool time_terms) {
    const Problem& pb = h->pb;
    const int64_t n = pb.n, nq = visc_len(pb);
    OpSeg base = base_opseg(pb, dt);
    if (!time_terms) std::memset(base.Dt, 0, sizeof(base.Dt));
    if (grad_pass(pb)) {
        OpSeg g = base;
        visc_tiles(g, pb);
        put_slab_segs(h, dv, M, g, st, [&](int m, OpSeg& x) {
            x.U = dptr(U + m * n);
            x.out = dptr(h->Q + m * nq);
        });
    }
    put_slab_segs(h, dop, M, base, st, [&](int m, OpSeg& x) {
        if (grad_pass(pb)) x.Q = dptr(h->Q + m * nq);
        x.U = dptr(U + m * n);
        x.uprev = m == 0 ? u_prev : nullptr;
        x.out = dptr(R + m * n);
    });
}

CoupleArgs couple_args(const Problem& pb, int M, const double* in0, const int* kp, int64_t ld, double* out,
                       const int* skip) {
    CoupleArgs a;
    a.in0 = in0;
    a.kp = kp;
    a.ld = ld;
    a.out = out;
    a.skip = skip;
    a.n = pb.n;
    a.nsp = pb.nsp;
    a.slabs = M;
    a.nt = pb.Nt;
    a.ns = pb.ns;
    a.nblk = vec_blocks((int64_t)(M > 1 ? M - 1 : 1) * pb.nsp);
    return a;
}

void launch_residual(st_ctx* h, int M, const OpSeg* dv, const OpSeg* dop, const CoupleArgs& cp, hipStream_t st) {
    const Problem& pb = h->pb;
    const int G = M * op_blocks(pb);
    auto& T = h->timer;
    if (grad_pass(pb)) T.run(ST_K_GRAD, st, [&] { pb.ops->visc_res64(dv, M, G, st); });
    T.run(ST_K_RESIDUAL, st, [&] { pb.ops->res64(dop, M, G, st); });
    if (M > 1) T.run(ST_K_RESIDUAL, st, [&] { vk_couple(cp, st); });
}

// Jv of M consecutive slabs (decoupled; the coupling kernel completes it),
// in two halves: upload the descriptors and launch the kernels.  U: double
// state (U32 must hold the FP32 copy when inner_fp32 and the equation is
// nonlinear).  The direction of slab m is dir + m n, moved by ld * (*kp)
// when kp is set (the Arnoldi index).  NS: the viscous pass writes the
// tangent of -Fv at (U, v) to dQ (dQ32), which the JVP kernel reads.
void setup_jvp(st_ctx* h, int M, const double* U, const double* dir, const int* kp, int64_t ld, double* out,
               const int* skip, bool fp32, double dt, OpSeg* dv, OpSeg* dop, hipStream_t st) {
    const Problem& pb = h->pb;
    const int kind = pb.eq.kind;
    const int64_t n = pb.n, nq = visc_len(pb);
    OpSeg base = base_opseg(pb, dt);
    base.skip = skip;
    auto dirp = [&](int m) { return DynPtr{dir + m * n, ld, kp, 0}; };
    auto state = [&](int m) { return dptr(fp32 ? (const void*)(h->U32 + m * n) : (const void*)(U + m * n)); };
    auto dq = [&](int m) { return dptr(fp32 ? (void*)(h->dQ32 + m * nq) : (void*)(h->dQ + m * nq)); };
    if (grad_pass(pb)) {
        OpSeg g = base;
        visc_tiles(g, pb);
        put_slab_segs(h, dv, M, g, st, [&](int m, OpSeg& x) {
            x.U = state(m);
            x.V = dirp(m);
            x.out = dq(m);
        });
    }
    put_slab_segs(h, dop, M, base, st, [&](int m, OpSeg& x) {
        x.out = dptr(out + m * n);
        if (linear_eq(kind)) {
            // J v = R(v) with u_prev = 0 and no exterior state (the linear part)
            x.U = dirp(m);
            x.uprev = nullptr;
            x.bcg = 0.0;
        } else {
            x.U = state(m);
            x.V = dirp(m);
            if (grad_pass(pb)) x.Q = dq(m);
        }
    });
}

void launch_jvp(st_ctx* h, int M, bool fp32, const OpSeg* dv, const OpSeg* dop, const CoupleArgs& cp,
                hipStream_t st) {
    const Problem& pb = h->pb;
    const int G = M * op_blocks(pb);
    const int kind = pb.eq.kind;
    if (grad_pass(pb))
        h->timer.run(ST_K_GRAD, st, [&] { (fp32 ? pb.ops->visc_jvp32 : pb.ops->visc_jvp64)(dv, M, G, st); });
    h->timer.run(ST_K_JVP, st, [&] {
        if (linear_eq(kind)) (fp32 ? pb.ops->lin32 : pb.ops->res64)(dop, M, G, st);
        else (fp32 ? pb.ops->jvp32 : pb.ops->jvp64)(dop, M, G, st);
    });
    if (M > 1) h->timer.run(ST_K_JVP, st, [&] { vk_couple(cp, st); });
}

// FP32 copy of U for FP32-inner JVPs of the nonlinear equations (uses the
// vector slot for the cast).
void enqueue_jvp_prepare(st_ctx* h, int M, const double* U, bool fp32, hipStream_t st) {
    const Problem& pb = h->pb;
    if (linear_eq(pb.eq.kind) || !fp32) return;
    VecSeg v;
    std::memset(&v, 0, sizeof(v));
    v.U = const_cast<double*>(U);
    v.U32 = h->U32;
    v.n = pb.n * M;
    v.nblk = vec_blocks(v.n);
    v.st = h->d_st;
    put_vecseg(h->d_vs, v, st);
    vk_cast32(h->d_vs, 1, v.nblk, st);
}

}  // namespace stdg

extern "C" {

int st_jvp(st_handle_t h, const double* U, double t0, double dt, const double* v, double* Jv, int inner_fp32,
           void* stream) {
    return st_jvp_slabs(h, 1, U, t0, dt, v, Jv, inner_fp32, stream);
}

int st_jvp_slabs(st_handle_t h, int M, const double* U, double t0, double dt, const double* v, double* Jv,
                 int inner_fp32, void* stream) {
    (void)t0;
    if (!h || !v || !Jv) return set_error(ST_ERR_BAD_ARG, "st_jvp: null argument");
    if (M < 1 || M > ST_MAX_SLABS) return set_error(ST_ERR_BAD_ARG, "st_jvp_slabs: slabs must be in 1..64");
    if (!linear_eq(h->pb.eq.kind) && !U) return set_error(ST_ERR_BAD_ARG, "st_jvp: null state");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ST_ERR_BAD_ARG, "st_jvp: dt must be positive");
    hipStream_t st = (hipStream_t)stream;
    const bool fp32 = inner_fp32 != 0;
    CHK(ensure_cap(h, M));
    if (fp32) CHK(ensure_fp32(h));
    OpSeg* dv = M == 1 ? h->d_op + 3 : h->d_opm + 2 * M;
    OpSeg* dop = M == 1 ? h->d_op + 4 : h->d_opm + 3 * M;
    h->timer.reset(0);
    enqueue_jvp_prepare(h, M, U, fp32, st);
    setup_jvp(h, M, U, v, nullptr, 0, Jv, nullptr, fp32, dt, dv, dop, st);
    launch_jvp(h, M, fp32, dv, dop, couple_args(h->pb, M, v, nullptr, 0, Jv, nullptr), st);
    HIPCHK(hipGetLastError());
    return ST_OK;
}

int st_error_estimate(st_handle_t h, const double* U, const double* u_prev, double t0, double dt, double atol,
                      double rtol, double* err, void* stream) {
    (void)t0;
    if (!h || !U || !u_prev || !err) return set_error(ST_ERR_BAD_ARG, "st_error_estimate: null argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ST_ERR_BAD_ARG, "st_error_estimate: dt must be positive");
    if (!(atol >= 0.0) || !(rtol >= 0.0) || !(atol + rtol > 0.0))
        return set_error(ST_ERR_BAD_ARG, "st_error_estimate: need atol, rtol >= 0 and atol + rtol > 0");
    const Problem& pb = h->pb;
    hipStream_t st = (hipStream_t)stream;
    if (!h->d_est) CHK(h->alloc(&h->d_est, (size_t)VMAXBLK + 1));
    EstArgs a;
    std::memset(&a, 0, sizeof(a));
    if (pb.Nt > 2) {
        // (dt / 2) F(u_prev) in est_f: the residual kernels for one time
        // level with the time derivative off and unit weight, at u_prev with
        // u_prev as its own inflow (that term is then exactly zero)
        Problem p1 = pb;
        p1.Nt = 1;
        p1.n = pb.nsp;
        p1.ops = find_table(pb.eq.kind, pb.mesh.dim, pb.n1, 1, pb.ops->rot != 0, pb.ops->bnd != 0);
        if (!p1.ops) return set_error(ST_ERR_UNSUPPORTED, "st_error_estimate: no one-time-level operator");
        p1.wt[0] = 1.0;
        p1.Dt[0] = 0.0;
        if (!h->est_f) CHK(h->alloc(&h->est_f, (size_t)pb.nsp));
        if (grad_pass(p1) && !h->est_q) CHK(h->alloc(&h->est_q, (size_t)visc_len(p1)));
        const OpSeg b = base_opseg(p1, dt);
        if (grad_pass(p1)) {
            OpSeg g = b;
            visc_tiles(g, p1);
            g.U = dptr(u_prev);
            g.out = dptr(h->est_q);
            h->put_op(h->d_op + 0, g, st);
        }
        OpSeg x = b;
        if (grad_pass(p1)) x.Q = dptr(h->est_q);
        x.U = dptr(u_prev);
        x.uprev = u_prev;
        x.out = dptr(h->est_f);
        h->put_op(h->d_op + 1, x, st);
        const int G = op_blocks(p1);
        if (grad_pass(p1)) p1.ops->visc_res64(h->d_op + 0, 1, G, st);
        p1.ops->res64(h->d_op + 1, 1, G, st);
        for (int j = 0; j < pb.Nt; ++j) a.c[j] = pb.wt[0] * pb.Dt[j];   // w_1 D_tau[0][j]
        a.fs = h->est_f;
        a.fsw = pb.wt[0];
    }
    a.U = U;
    a.up = u_prev;
    a.part = h->d_est + 1;
    a.out = h->d_est;
    a.nsp = pb.nsp;
    a.nt = pb.Nt;
    a.ns = pb.ns;
    a.nblk = vec_blocks(pb.nsp);
    a.atol = atol;
    a.rtol = rtol;
    vk_error_estimate(a, st);
    HIPCHK(hipMemcpyAsync(err, h->d_est, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ST_OK;
}

int st_next_dt(int Nt, double dt, double err, double* dt_next) {
    if (!dt_next || Nt < 2 || Nt > 4 || !(dt > 0.0) || !(err >= 0.0))
        return set_error(ST_ERR_BAD_ARG, "st_next_dt: need Nt in 2..4, dt > 0, err >= 0 and an output");
    // step-size control of the embedded pair of st_error_estimate: its
    // estimate is of the embedded order q (1, 3, 4 for Nt = 2, 3, 4), so it
    // scales like dt^(q+1); safety factor 0.9, growth in [0.2, 5]
    constexpr double fac = 0.9, facmin = 0.2, facmax = 5.0;
    const int q = Nt == 2 ? 1 : Nt;
    double f = err > 0.0 ? fac * std::pow(1.0 / err, 1.0 / (q + 1)) : facmax;
    if (!std::isfinite(f)) f = facmin;
    f = std::min(facmax, std::max(facmin, f));
    *dt_next = dt * f;
    return ST_OK;
}

int st_solve_slab(st_handle_t h, const double* u_prev, double t0, double dt, double tol,
                  const st_solver_opts_t* opts_in, double* U_out, double* u_next, st_stats_t* stats,
                  void* stream) {
    return st_solve_slabs(h, 1, u_prev, t0, dt, tol, opts_in, U_out, u_next, stats, stream);
}

int st_solve_slabs(st_handle_t h, int M, const double* u_prev, double t0, double dt, double tol,
                   const st_solver_opts_t* opts_in, double* U_out, double* u_next, st_stats_t* stats,
                   void* stream) {
    (void)t0;
    auto t_start = std::chrono::steady_clock::now();
    if (!h || !u_prev) return set_error(ST_ERR_BAD_ARG, "st_solve_slab: null argument");
    if (M < 1 || M > ST_MAX_SLABS) return set_error(ST_ERR_BAD_ARG, "st_solve_slabs: slabs must be in 1..64");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(ST_ERR_BAD_ARG, "st_solve_slab: dt must be positive");
    if (!(tol > 0.0)) return set_error(ST_ERR_BAD_ARG, "st_solve_slab: tol must be positive");
    st_solver_opts_t o;
    st_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.restart < 1 || o.restart > MMAX) return set_error(ST_ERR_BAD_ARG, "restart must be in 1..32");
    if (o.cgs_passes < 0 || o.cgs_passes > 2) return set_error(ST_ERR_BAD_ARG, "cgs_passes must be 0, 1 or 2");
    if (o.max_newton < 1) return set_error(ST_ERR_BAD_ARG, "max_newton must be >= 1");
    if (o.precond < 0 || o.precond > 2) return set_error(ST_ERR_BAD_ARG, "precond must be 0, 1 or 2");
    const Problem& pb = h->pb;
    const bool fp32 = o.inner_fp32 != 0;
    const int m = o.restart;
    CHK(ensure_cap(h, M));
    CHK(ensure_solve(h, m));
    if (fp32) CHK(ensure_fp32(h));
    hipStream_t st = (hipStream_t)stream;
    const bool pc = o.precond >= 1;
    const bool sweep = o.precond == 2 && M > 1;   // forward substitution over the slabs
    if (pc) CHK(ensure_precond(h, u_prev, dt, st));
    const int kind = pb.eq.kind;
    const int64_t nM = pb.n * M;             // unknowns of the (multi-slab) system
    const int gstream = gs_stream((int64_t)(m + 1) * nM * 8);   // the Krylov basis beyond the Infinity Cache

    // forcing: linear equations solve each cycle as far as the outer tolerance
    double eta_rel = linear_eq(kind) ? 0.0 : std::max(o.gmres_rtol, 0.0);
    if (fp32) eta_rel = std::max(eta_rel, 1e-5);

    VecSeg vs;
    std::memset(&vs, 0, sizeof(vs));
    vs.V = h->V;
    vs.w = h->w;
    vs.R = h->R;
    vs.U = h->U;
    vs.n = nM;
    vs.st = h->d_st;
    vs.part = h->d_part;
    vs.part2 = h->d_part + (size_t)vec_blocks(nM) * NPART_SLOTS;
    vs.eta_rel = eta_rel;
    vs.eta_tgt = 0.5;
    vs.tol = tol;
    vs.m = m;
    vs.uprev = u_prev;
    vs.unext = u_next;
    vs.U32 = h->U32;
    vs.nt = pb.Nt;
    vs.ns = pb.ns;
    vs.blk0 = 0;
    vs.nblk = vec_blocks(nM);
    vs.dev_stop = 1;
    vs.max_newton = o.max_newton;
    const int Gv = vs.nblk;
    h->timer.reset(o.timing);
    HIPCHK(hipMemsetAsync(h->d_st, 0, sizeof(GState), st));
    VecSeg* dvs = h->d_vsm;                  // [0]: the system, [1, M]: per-slab guess, [M + 1]: extraction
    put_vecseg(dvs, vs, st);
    // initial guess 1 (x) u_prev in every slab
    const int Gs = vec_blocks(pb.n);
    for (int sl = 0; sl < M; ++sl) {
        VecSeg g = vs;
        g.U = h->U + sl * pb.n;
        g.n = pb.n;
        g.blk0 = sl * Gs;
        g.nblk = Gs;
        put_vecseg(dvs + 1 + sl, g, st);
    }
    vk_init_guess(dvs + 1, M, M * Gs, st);

    // residual descriptors, fixed for the whole solve
    OpSeg* d_rv = h->d_opm;
    OpSeg* d_rop = h->d_opm + M;
    setup_residual(h, M, h->U, u_prev, h->R, dt, d_rv, d_rop, st);
    const CoupleArgs cp_res = couple_args(pb, M, h->U, nullptr, 0, h->R, nullptr);

    // JVP descriptors: the direction V_k follows the device Arnoldi index;
    // the whole segment is skipped once the cycle is done
    const int* kp = &h->d_st->k;
    const int* skip = &h->d_st->done;
    OpSeg* d_jv = h->d_opm + 2 * M;
    OpSeg* d_jop = h->d_opm + 3 * M;
    // right preconditioning: the JVP takes z = B^-1 V_k, formed per step
    const double* dir = pc ? h->pz : h->V;
    const int* dkp = pc ? nullptr : kp;
    const int64_t dld = pc ? 0 : nM;
    setup_jvp(h, M, h->U, dir, dkp, dld, h->w, skip, fp32, dt, d_jv, d_jop, st);
    const CoupleArgs cp_jvp = couple_args(pb, M, dir, dkp, dld, h->w, skip);
    const int npe = (int)(pb.nv * pb.Nt * pb.ns);
    const int64_t Eall = pb.E * M;           // element blocks of all slabs (B^-1 is the same in each)
    const int Gpc = pc ? pc_blocks((int)Eall, npe) : 0;
    if (pc) {
        PcSeg a;
        std::memset(&a, 0, sizeof(a));
        a.in = dptr_k(h->V, nM, kp);
        a.out = h->pz;
        a.binvT = h->binvT;
        a.skip = skip;
        a.npe = npe;
        a.E = (int)Eall;
        a.accumulate = 0;
        a.blk0 = 0;
        a.nblk = Gpc;
        put_pcseg(h->d_pc + 0, a, st);
        PcSeg u = a;                     // Newton update: U += B^-1 (V y), V y staged in w
        u.in = dptr(h->w);
        u.out = h->U;
        u.skip = nullptr;
        u.accumulate = 1;
        put_pcseg(h->d_pc + 1, u, st);
        PcSeg y = u;                     // coupled slabs: B^-1 (V y) to pz, then the sweep adds P^-1 (V y) to U
        y.out = h->pz;
        y.accumulate = 0;
        put_pcseg(h->d_pc + 2, y, st);
    }
    SweepArgs sw_dir, sw_upd;
    std::memset(&sw_dir, 0, sizeof(sw_dir));
    sw_dir.C = h->pc_C;
    sw_dir.y = h->pz;
    sw_dir.skip = skip;
    sw_dir.n = pb.n;
    sw_dir.npe = npe;
    sw_dir.nl = pb.nv * pb.ns;
    sw_dir.nt = pb.Nt;
    sw_dir.ns = pb.ns;
    sw_dir.E = (int)pb.E;
    sw_dir.M = M;
    sw_upd = sw_dir;
    sw_upd.acc = h->U;
    sw_upd.skip = nullptr;

    int status = ST_ERR_NO_CONVERGENCE;
    int outer = 0;
    double r0 = 0.0, rn = 0.0, best = INFINITY;
    int stall = 0;
    auto& T = h->timer;
    // one Arnoldi step (every kernel of it exits at once when the cycle is done)
    auto arnoldi_step = [&](int k) {
        if (pc) T.run(ST_K_PRECOND, st, [&] { pc_apply(h->d_pc + 0, 1, Gpc, npe, st); });
        if (sweep) T.run(ST_K_PRECOND, st, [&] { pc_sweep(sw_dir, st); });
        launch_jvp(h, M, fp32, d_jv, d_jop, cp_jvp, st);
        const int npass = o.cgs_passes == 0 ? 2 : o.cgs_passes;
        for (int p = 0; p < npass; ++p) {
            int lastp = 0, gate = 0;
            gs_pass_plan(o.cgs_passes, p, &lastp, &gate);
            T.run(ST_K_MULTIDOT, st, [&] { vk_multidot(dvs, 1, Gv, k, st, gate, gstream); });
            T.run(ST_K_UPDATE, st, [&] { vk_update(dvs, 1, Gv, p, lastp, k, st, gstream); });
        }
    };
    // Steps of each cycle enqueued before the host reads the outer iteration's
    // state: the GPU runs them while the host waits for the state, decides and
    // enqueues the rest.  k_begin takes the same stopping decisions as the host
    // below (VecSeg.dev_stop), so when the iteration stops they exit at once.
    const int kpre = std::min(m, 2);
    for (;;) {
        launch_residual(h, M, d_rv, d_rop, cp_res, st);
        T.run(ST_K_NEWTON, st, [&] {
            vk_rnorm(dvs, 1, Gv, st);
            vk_begin(dvs, 1, st);
        }, false);
        HIPCHK(hipMemcpyAsync(h->h_st, h->d_st, offsetof(GState, hacc), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(h->ev_state, st));
        // Jacobian base point of FP32-inner JVPs: the FP32 copy of U
        if (fp32 && !linear_eq(kind)) T.run(ST_K_NEWTON, st, [&] { vk_cast32(dvs, 1, Gv, st); });
        T.run(ST_K_NORMALIZE, st, [&] { vk_scale_v0(dvs, 1, Gv, st); });
        for (int k = 0; k < kpre; ++k) arnoldi_step(k);
        HIPCHK(hipEventSynchronize(h->ev_state));
        const GState& hs = *h->h_st;
        rn = hs.rnorm;
        if (outer == 0) r0 = rn;
        bool more = false;
        if (hs.nonfinite) status = ST_ERR_NONFINITE;
        else if (rn <= hs.target) status = ST_OK;
        else if (outer >= o.max_newton) {}
        else if (rn < 0.9 * best) { best = rn; stall = 0; more = true; }
        else more = ++stall < 8;          // no progress over 8 outer iterations: stop
        if (more == (hs.stop != 0))
            return set_error(ST_ERR_HIP, "st_solve_slab: device and host stopping tests disagree");
        if (!more) break;
        ++outer;
        for (int k = kpre; k < m; ++k) arnoldi_step(k);
        T.run(ST_K_NEWTON, st, [&] {
            vk_finish(dvs, 1, st);
            if (sweep) {
                pc_combine(dvs, 1, Gv, st);
                pc_apply(h->d_pc + 2, 1, Gpc, npe, st);
                pc_sweep(sw_upd, st);
            } else if (pc) {
                pc_combine(dvs, 1, Gv, st);
                pc_apply(h->d_pc + 1, 1, Gpc, npe, st);
            } else {
                vk_update_u(dvs, 1, Gv, st);
            }
        }, false);
        HIPCHK(hipGetLastError());
    }
    if (u_next) {
        // u_next = (e_Nt^T (x) I) U of the last slab
        VecSeg x = vs;
        x.U = h->U + (M - 1) * pb.n;
        x.n = pb.n;
        x.nblk = Gs;
        put_vecseg(dvs + M + 1, x, st);
        vk_extract_last(dvs + M + 1, 1, Gs, st);
    }
    if (U_out) HIPCHK(hipMemcpyAsync(U_out, h->U, sizeof(double) * nM, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(h->h_st, h->d_st, offsetof(GState, hacc), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
        h->timer.collect(stats);
        // algorithmic bytes: operator kernels from launch counts, Krylov
        // kernels accumulated on the device
        const double n8 = 8.0 * (double)nM;
        const int its = h->h_st->iters_total;
        const bool visc = grad_pass(pb), lin = linear_eq(kind);
        for (int c = 0; c < ST_K_COUNT; ++c) stats->kernel_bytes[c] = 0.0;
        // coupling of M slabs: 3 (M - 1) spatial vectors of a slab per launch
        const double cpl = 24.0 * (double)(M - 1) * (double)pb.nsp;
        stats->kernel_bytes[ST_K_RESIDUAL] = (outer + 1) * (2.0 * n8 + 8.0 * (double)pb.nsp + cpl);
        const double jvp_b = lin ? 2.0 * n8 : (fp32 ? 2.5 : 3.0) * n8;   // [U,] v in, Jv out
        stats->kernel_bytes[ST_K_JVP] = its * (jvp_b + cpl);
        if (visc) {
            // viscous pass: residual reads U and writes its output (the
            // viscous terms of the own residual, the face traces); JVP reads U
            // and v and writes the output's tangent
            const double tr = 8.0 * (double)visc_len(pb) * M;
            stats->kernel_bytes[ST_K_GRAD] =
                (outer + 1) * (n8 + tr) + its * ((fp32 ? 1.5 : 2.0) * n8 + (fp32 ? 0.5 : 1.0) * tr);
        }
        // direction in, z out; the sweep over coupled slabs: y in, z out (slabs 1..M-1)
        if (pc) stats->kernel_bytes[ST_K_PRECOND] = (its + outer) * 2.0 * n8;
        if (sweep) stats->kernel_bytes[ST_K_PRECOND] += its * (n8 + 8.0 * (double)pb.n * (M - 1));
        // accumulated per Gram-Schmidt pass that did work
        stats->kernel_bytes[ST_K_MULTIDOT] = h->h_st->kbytes[3];
        stats->kernel_bytes[ST_K_UPDATE] = h->h_st->kbytes[4];
        stats->newton_its = outer;
        stats->gmres_its = h->h_st->iters_total;
        stats->res0 = r0;
        stats->res_final = rn;
        stats->status = status;
        stats->usec = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (status == ST_ERR_NONFINITE) return set_error(status, "non-finite residual or Krylov quantity");
    if (status != ST_OK)
        return set_error(status, "no convergence: ||R|| = " + std::to_string(rn) + " after " +
                                     std::to_string(outer) + " outer iterations");
    return ST_OK;
}

}  // extern "C"
