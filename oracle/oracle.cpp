/*
 * oracle.cpp -- CPU FP64 oracle for the space-time DG-SEM slab system.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, slow and written to be
 * checked against the paper by eye: no sum factorisation, no fusion, every
 * derivative is taken from the Lagrange basis definition, every flux is
 * re-evaluated where it is used.  Exact Jacobian-vector products come from
 * forward-mode dual numbers pushed through the very same residual code.
 *
 * Readings of the paper that this file takes (one line each):
 *  - time map t = t_n + dt/2 (1 + tau): the factor is dt/2 (Sec. "Space-Time
 *    DG-SEM"; the 2/dt printed in eq. (DGSEM_time_component) is a misprint,
 *    eq. (DG_in_time) has dt/2).
 *  - reference element [-1,1] per axis, metric factor 2/h_a.
 *  - Rusanov flux eq. (flux:llf) with jump [[u]] = n.(u_E - u_N): along +e_a
 *    with left state L and right state R, H = {f} + lambda/2 (u_L - u_R),
 *    lambda = max(lambda(u_L), lambda(u_R)) pointwise; ties pick u_L.
 *    lambda: advection |a_a|, Burgers |u|, Euler/NS |v_a| + c.
 *  - viscous terms by BR1 (central u-hat = {u} in the lifted gradient of the
 *    conservative variables, central {F_v}), no diffusion in time (the
 *    space-time viscous flux has a zero time column, Sec. "Space-Time DG-SEM").
 *  - derivative of |x| is sign(x) with sign(0) = +1; of max(a,b) the active
 *    branch with the tie rule above.
 *  - Euler pressure p = (gamma-1)(E - |m|^2/(2 rho)) (ideal gas).
 *  - Navier-Stokes: constant mu, Stokes hypothesis, gas constant 1 so that
 *    T = p/rho, heat conductivity kappa = mu gamma / ((gamma-1) Pr).
 *  - symmetric interior penalty (ORC_ADVDIFF_SIPG; the paper's flux, Sec.
 *    "DG-SEM in Space", whose printed formula and code are garbled): the
 *    standard SIPG bilinear form
 *      a(u, psi) = sum_K int nu grad u . grad psi - sum_F int nu {grad u}.[[psi]]
 *                - sum_F int nu {grad psi}.[[u]] + sum_F int sigma [[u]].[[psi]],
 *    [[u]] = n_K u_K + n_N u_N, sigma = eta nu / h_F, eta = 10 p^2 (p the
 *    spatial degree, 1 for p = 0) and h_F = cell volume / facet area = h_a,
 *    all integrals by the LGL rule; the spatial operator is M^-1 of minus it.
 *  - advection velocity b(x) = a + omega e_z x (x - center) (2D rotation); the
 *    flux b(x_i) u_i is interpolated at the nodes like every other flux.
 *  - Dirichlet boundaries (bc = 1, scalar equations): exterior state g =
 *    bc_value; convective flux Rusanov(u, g); BR1 u_hat = g with the interior
 *    viscous flux; SIPG by Nitsche's terms, the interior-face terms with the
 *    averages replaced by the interior values and u_N by g.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Scalars: double, and a dual number a + b eps (eps^2 = 0) for exact JVPs.
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }

inline double value(double a) { return a; }
inline double value(Dual a) { return a.v; }
inline double sqrt_(double a) { return std::sqrt(a); }
inline Dual sqrt_(Dual a) { return sqrt(a); }
template <class T> inline T absval(T a) { return value(a) >= 0.0 ? a : T(0.0) - a; }
// max with the tie rule: equal values pick the first argument.
template <class T> inline T larger(T a, T b) { return value(a) >= value(b) ? a : b; }

// ---------------------------------------------------------------------------
// One-dimensional Legendre-Gauss-Lobatto nodes, weights, Lagrange basis.
// ---------------------------------------------------------------------------
// Legendre P_p(x) and P_p'(x) by the three-term recurrence.
void legendre(int p, double x, double& P, double& dP) {
    if (p == 0) { P = 1.0; dP = 0.0; return; }
    double Pm = 1.0, Pc = x, dPm = 0.0, dPc = 1.0;
    for (int k = 1; k < p; ++k) {
        double Pn = ((2 * k + 1) * x * Pc - k * Pm) / (k + 1);
        double dPn = dPm + (2 * k + 1) * Pc;
        Pm = Pc; Pc = Pn; dPm = dPc; dPc = dPn;
    }
    P = Pc; dP = dPc;
}

// n LGL nodes: -1, the roots of P'_{n-1}, +1.  Weights 2/(p(p+1) P_p(x_i)^2).
void lgl(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0); w.assign(n, 0.0);
    if (n == 1) { x[0] = 0.0; w[0] = 2.0; return; }
    const int p = n - 1;
    x[0] = -1.0; x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double xi = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, xi, P, dP);
            // Legendre ODE: (1-x^2) P'' = 2x P' - p(p+1) P
            double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
            double dx = dP / d2P;
            xi -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        x[i] = xi;
    }
    std::sort(x.begin(), x.end());
    for (int i = 0; i < n; ++i) {
        double P, dP;
        legendre(p, x[i], P, dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
}

// Lagrange basis polynomial l_i(x) and its derivative, from the product form.
double lagrange(const std::vector<double>& X, int i, double x) {
    double r = 1.0;
    for (size_t k = 0; k < X.size(); ++k)
        if ((int)k != i) r *= (x - X[k]) / (X[i] - X[k]);
    return r;
}
double lagrange_deriv(const std::vector<double>& X, int i, double x) {
    double s = 0.0;
    for (size_t m = 0; m < X.size(); ++m) {
        if ((int)m == i) continue;
        double t = 1.0 / (X[i] - X[m]);
        for (size_t k = 0; k < X.size(); ++k)
            if ((int)k != i && k != m) t *= (x - X[k]) / (X[i] - X[k]);
        s += t;
    }
    return s;
}

// Dense square inverse by Gauss-Jordan with partial pivoting (small n only).
bool invert(int n, std::vector<double> A, std::vector<double>& Ainv) {
    Ainv.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        for (int k = 0; k < n; ++k) {
            std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(Ainv[c * n + k], Ainv[piv * n + k]);
        }
        double d = A[c * n + c];
        for (int k = 0; k < n; ++k) { A[c * n + k] /= d; Ainv[c * n + k] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                Ainv[r * n + k] -= f * Ainv[c * n + k];
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// Problem set-up: mesh geometry, node sets, matrices.
// ---------------------------------------------------------------------------
struct Setup {
    orc_problem P;
    int d, n1, ns, nv, Nt, E;
    int K[3];
    double h[3];
    int estride[3], nstride[3];
    std::vector<double> xi, wi, D;     // spatial LGL nodes, weights, D[j*n1+k] = l_k'(xi_j)
    std::vector<double> tau, om, Dt;   // temporal LGL nodes, weights, D_tau
    bool viscous;                      // BR1 lifted gradient (advection-diffusion BR1, NS)
    bool sipg;                         // symmetric interior penalty viscous terms
    double eta;                        // SIPG penalty 10 p^2

    explicit Setup(const orc_problem* p) {
        P = *p;
        d = p->dim; n1 = p->N + 1; Nt = p->Nt;
        nv = orc_nvars(p->eq, d);
        ns = 1; for (int a = 0; a < d; ++a) ns *= n1;
        E = 1;
        for (int a = 0; a < 3; ++a) {
            K[a] = a < d ? p->K[a] : 1;
            h[a] = a < d ? (p->hi[a] - p->lo[a]) / p->K[a] : 1.0;
        }
        for (int a = 0; a < d; ++a) E *= K[a];
        estride[0] = 1; estride[1] = K[0]; estride[2] = K[0] * K[1];
        nstride[0] = 1; nstride[1] = n1; nstride[2] = n1 * n1;
        lgl(n1, xi, wi);
        lgl(Nt, tau, om);
        D.resize(n1 * n1);
        for (int j = 0; j < n1; ++j)
            for (int k = 0; k < n1; ++k) D[j * n1 + k] = lagrange_deriv(xi, k, xi[j]);
        Dt.resize(Nt * Nt);
        for (int j = 0; j < Nt; ++j)
            for (int k = 0; k < Nt; ++k) Dt[j * Nt + k] = lagrange_deriv(tau, k, tau[j]);
        viscous = (p->eq == ORC_ADVDIFF_BR1 || p->eq == ORC_NS_BR1);
        sipg = p->eq == ORC_ADVDIFF_SIPG;
        eta = p->N > 0 ? 10.0 * p->N * p->N : 1.0;
    }
    int ecoord(int e, int a) const { return (e / estride[a]) % K[a]; }
    // element across the face of e along axis a (dir = +-1); -1 on a
    // Dirichlet boundary
    int neighbor(int e, int a, int dir) const {
        int c = ecoord(e, a);
        if (P.bc[a] == 1 && (c + dir < 0 || c + dir >= K[a])) return -1;
        int cn = (c + dir + K[a]) % K[a];
        return e + (cn - c) * estride[a];
    }
    // physical coordinate a of spatial node s of element e
    double coord(int e, int s, int a) const {
        return P.lo[a] + h[a] * (ecoord(e, a) + 0.5 * (1.0 + xi[ncoord(s, a)]));
    }
    // advection velocity b_a at node s of element e (scalar equations)
    double vel(int e, int s, int a) const {
        double b = P.a[a];
        if (d == 2 && P.omega != 0.0) {
            if (a == 0) b -= P.omega * (coord(e, s, 1) - P.center[1]);
            if (a == 1) b += P.omega * (coord(e, s, 0) - P.center[0]);
        }
        return b;
    }
    int ncoord(int s, int a) const { return (s / nstride[a]) % n1; }
    int node_with(int s, int a, int i) const { return s + (i - ncoord(s, a)) * nstride[a]; }
    // physical LGL weight of spatial node s: prod_a (h_a/2) w_{i_a}
    double wphys(int s) const {
        double w = 1.0;
        for (int a = 0; a < d; ++a) w *= 0.5 * h[a] * wi[ncoord(s, a)];
        return w;
    }
    long slab_size() const { return (long)E * nv * Nt * ns; }
    long space_size() const { return (long)E * nv * ns; }
};

// ---------------------------------------------------------------------------
// Pointwise physics (eq. (general) with S = react * u).
// ---------------------------------------------------------------------------
// Convective flux along axis a; ba is the advection velocity b_a at the
// point (scalar linear equations).
template <class T>
void conv_flux(const Setup& S, int a, const T* u, T* f, double ba) {
    const orc_problem& P = S.P;
    switch (P.eq) {
    case ORC_ADVECTION:
    case ORC_ADVDIFF_BR1:
    case ORC_ADVDIFF_SIPG:
        f[0] = ba * u[0];
        break;
    case ORC_BURGERS:
        f[0] = 0.5 * u[0] * u[0];
        break;
    default: {  // Euler flux f_a, Sec. "Euler Equations"
        const int d = S.d;
        T rho = u[0];
        T vel[3];
        for (int b = 0; b < d; ++b) vel[b] = u[1 + b] / rho;
        T mm = 0.0;
        for (int b = 0; b < d; ++b) mm += u[1 + b] * vel[b];
        T p = (P.gamma - 1.0) * (u[d + 1] - 0.5 * mm);
        f[0] = u[1 + a];
        for (int b = 0; b < d; ++b) f[1 + b] = u[1 + a] * vel[b] + (a == b ? p : T(0.0));
        f[d + 1] = (u[d + 1] + p) * vel[a];
    }
    }
}

// Largest wave speed along axis a (ba as in conv_flux).
template <class T>
T wave_speed(const Setup& S, int a, const T* u, double ba) {
    const orc_problem& P = S.P;
    switch (P.eq) {
    case ORC_ADVECTION:
    case ORC_ADVDIFF_BR1:
    case ORC_ADVDIFF_SIPG:
        return T(std::fabs(ba));
    case ORC_BURGERS:
        return absval(u[0]);
    default: {
        const int d = S.d;
        T rho = u[0];
        T mm = 0.0;
        for (int b = 0; b < d; ++b) mm += u[1 + b] * u[1 + b] / rho;
        T p = (P.gamma - 1.0) * (u[d + 1] - 0.5 * mm);
        T c = sqrt_(P.gamma * p / rho);
        return absval(u[1 + a] / rho) + c;
    }
    }
}

// Viscous flux along axis a from the state u and the gradient q[b*nv + v]
// = d u_v / d x_b of the conservative variables.
template <class T>
void visc_flux(const Setup& S, int a, const T* u, const T* q, T* f) {
    const orc_problem& P = S.P;
    const int d = S.d, nv = S.nv;
    if (P.eq == ORC_ADVDIFF_BR1) { f[0] = P.nu * q[a * nv]; return; }
    if (P.eq != ORC_NS_BR1) { for (int v = 0; v < nv; ++v) f[v] = 0.0; return; }
    const double g = P.gamma;
    T rho = u[0];
    T vel[3];
    for (int b = 0; b < d; ++b) vel[b] = u[1 + b] / rho;
    T mm = 0.0;
    for (int b = 0; b < d; ++b) mm += u[1 + b] * vel[b];
    T p = (g - 1.0) * (u[d + 1] - 0.5 * mm);
    T Temp = p / rho;
    // chain rule: grad v_c = (grad m_c - v_c grad rho)/rho,
    // grad p = (g-1)(grad E - v . grad m + |v|^2/2 grad rho), grad T = (grad p - T grad rho)/rho
    T gv[3][3];   // gv[b][c] = d v_c / d x_b
    T gT[3];
    for (int b = 0; b < d; ++b) {
        T grho = q[b * nv + 0];
        T vgm = 0.0, v2 = 0.0;
        for (int c = 0; c < d; ++c) {
            gv[b][c] = (q[b * nv + 1 + c] - vel[c] * grho) / rho;
            vgm += vel[c] * q[b * nv + 1 + c];
            v2 += vel[c] * vel[c];
        }
        T gp = (g - 1.0) * (q[b * nv + d + 1] - vgm + 0.5 * v2 * grho);
        gT[b] = (gp - Temp * grho) / rho;
    }
    T div = 0.0;
    for (int c = 0; c < d; ++c) div += gv[c][c];
    const double mu = P.mu;
    const double kappa = mu * g / ((g - 1.0) * P.prandtl);
    f[0] = 0.0;
    T work = 0.0;
    for (int c = 0; c < d; ++c) {
        // tau_{ac} = mu (d_a v_c + d_c v_a) - 2/3 mu delta_ac div v
        T tau = mu * (gv[a][c] + gv[c][a]) - (a == c ? (2.0 / 3.0) * mu * div : T(0.0));
        f[1 + c] = tau;
        work += tau * vel[c];
    }
    f[d + 1] = work + kappa * gT[a];
}

// Total physical flux f_a(u) - fv_a(u, q) (BR1 equations; for SIPG the
// convective flux only: its viscous terms are assembled by sipg_terms).
template <class T>
void total_flux(const Setup& S, int a, const T* u, const T* q, T* f, double ba) {
    conv_flux(S, a, u, f, ba);
    if (S.viscous) {
        T fv[8];
        visc_flux(S, a, u, q, fv);
        for (int v = 0; v < S.nv; ++v) f[v] = f[v] - fv[v];
    }
}

// Numerical flux along +e_a between left state L and right state R:
// Rusanov for the convective part, central average for the viscous part.
template <class T>
void num_flux(const Setup& S, int a, const T* uL, const T* uR, const T* qL, const T* qR, T* H, double ba) {
    const int nv = S.nv;
    T fL[8], fR[8];
    conv_flux(S, a, uL, fL, ba);
    conv_flux(S, a, uR, fR, ba);
    T lam = larger(wave_speed(S, a, uL, ba), wave_speed(S, a, uR, ba));
    for (int v = 0; v < nv; ++v) H[v] = 0.5 * (fL[v] + fR[v]) + 0.5 * lam * (uL[v] - uR[v]);
    if (S.viscous) {
        T gL[8], gR[8];
        visc_flux(S, a, uL, qL, gL);
        visc_flux(S, a, uR, qR, gR);
        for (int v = 0; v < nv; ++v) H[v] = H[v] - 0.5 * (gL[v] + gR[v]);
    }
}

// ---------------------------------------------------------------------------
// Strong-form spatial operator F = M^-1 L_h(u) (eq. (ode)), DG-SEM in space
// with collocated LGL quadrature (Sec. "DG-SEM in Space").
// u, F: spatial vectors [E][nv][ns].
// ---------------------------------------------------------------------------
// BR1 lifted gradient q[((e*d + b)*nv + v)*ns + s] = d u_v / d x_b.
template <class T>
void lifted_gradient(const Setup& S, const T* u, T* q) {
    const int d = S.d, nv = S.nv, ns = S.ns, n1 = S.n1;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e) {
        for (int b = 0; b < d; ++b) {
            const double J = 2.0 / S.h[b];
            for (int v = 0; v < nv; ++v) {
                const T* ue = u + ((long)e * nv + v) * ns;
                for (int s = 0; s < ns; ++s) {
                    int i = S.ncoord(s, b);
                    T g = 0.0;
                    for (int k = 0; k < n1; ++k) g += S.D[i * n1 + k] * ue[S.node_with(s, b, k)];
                    if (i == n1 - 1) {
                        int en = S.neighbor(e, b, +1);
                        T uhat = T(S.P.bc_value);     // Dirichlet boundary: u_hat = g
                        if (en >= 0) uhat = 0.5 * (ue[s] + u[((long)en * nv + v) * ns + S.node_with(s, b, 0)]);
                        g += (uhat - ue[s]) / S.wi[n1 - 1];
                    }
                    if (i == 0) {
                        int en = S.neighbor(e, b, -1);
                        T uhat = T(S.P.bc_value);
                        if (en >= 0) uhat = 0.5 * (u[((long)en * nv + v) * ns + S.node_with(s, b, n1 - 1)] + ue[s]);
                        g -= (uhat - ue[s]) / S.wi[0];
                    }
                    q[(((long)e * d + b) * nv + v) * ns + s] = J * g;
                }
            }
        }
    }
}

template <class T>
void gather_node(const Setup& S, const T* u, const T* q, int e, int s, T* un, T* qn) {
    for (int v = 0; v < S.nv; ++v) un[v] = u[((long)e * S.nv + v) * S.ns + s];
    if (q)
        for (int b = 0; b < S.d; ++b)
            for (int v = 0; v < S.nv; ++v)
                qn[b * S.nv + v] = q[(((long)e * S.d + b) * S.nv + v) * S.ns + s];
}

// SIPG viscous terms, F += -M^-1 a(u, .) with the bilinear form of the
// header (scalar equation).  Along each axis a the element's nodal basis is
// l_{i_a}(x_a) times the others, so every term acts on lines of n1 nodes:
// with J = 2/h_a and the line's values u_k (k = 0..N), for node i of the line
//   volume:      -nu J^2 (1/w_i) sum_q w_q D_qi (D u)_q        (= -M^-1 int nu u' psi_i')
//   right face:  consistency +nu (J/w_N) {u'} [i = N],
//                symmetry    +nu s J^2 (D_Ni / w_i) (u_N - u_R),
//                penalty     -(eta nu/h_a) (J/w_N) (u_N - u_R) [i = N],
//   left face:   consistency -nu (J/w_0) {u'} [i = 0],
//                symmetry    +nu s J^2 (D_0i / w_i) (u_L - u_0),
//                penalty     -(eta nu/h_a) (J/w_0) (u_0 - u_L) [i = 0],
// where u' = J D u is the normal derivative, {u'} its average over the two
// elements (s = 1/2) -- on a Dirichlet boundary the interior value, s = 1
// and the exterior state g in place of u_R / u_L.
template <class T>
void sipg_terms(const Setup& S, const T* u, T* F) {
    const int d = S.d, ns = S.ns, n1 = S.n1, N = n1 - 1;
    const double nu = S.P.nu;
    const T g = T(S.P.bc_value);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e) {
        const T* ue = u + (long)e * ns;
        for (int s = 0; s < ns; ++s) {
            T acc = 0.0;
            for (int a = 0; a < d; ++a) {
                const double J = 2.0 / S.h[a];
                const double sig = S.eta * nu / S.h[a];
                const int i = S.ncoord(s, a);
                // the line through s along a, and its derivative
                T ul[8], du[8];
                for (int k = 0; k < n1; ++k) ul[k] = ue[S.node_with(s, a, k)];
                for (int q = 0; q < n1; ++q) {
                    du[q] = 0.0;
                    for (int k = 0; k < n1; ++k) du[q] += S.D[q * n1 + k] * ul[k];
                }
                T vol = 0.0;
                for (int q = 0; q < n1; ++q) vol += S.wi[q] * S.D[q * n1 + i] * du[q];
                acc -= nu * J * J * vol / S.wi[i];
                // right face of the element
                {
                    const int en = S.neighbor(e, a, +1);
                    T ext, dav;
                    double sc;
                    if (en >= 0) {
                        const T* un = u + (long)en * ns;
                        T dn = 0.0;
                        for (int k = 0; k < n1; ++k) dn += S.D[0 * n1 + k] * un[S.node_with(s, a, k)];
                        ext = un[S.node_with(s, a, 0)];
                        dav = 0.5 * J * (du[N] + dn);
                        sc = 0.5;
                    } else {
                        ext = g;
                        dav = J * du[N];
                        sc = 1.0;
                    }
                    const T jump = ul[N] - ext;
                    if (i == N) acc += nu * (J / S.wi[N]) * dav - sig * (J / S.wi[N]) * jump;
                    acc += nu * sc * J * J * (S.D[N * n1 + i] / S.wi[i]) * jump;
                }
                // left face
                {
                    const int en = S.neighbor(e, a, -1);
                    T ext, dav;
                    double sc;
                    if (en >= 0) {
                        const T* un = u + (long)en * ns;
                        T dn = 0.0;
                        for (int k = 0; k < n1; ++k) dn += S.D[N * n1 + k] * un[S.node_with(s, a, k)];
                        ext = un[S.node_with(s, a, N)];
                        dav = 0.5 * J * (du[0] + dn);
                        sc = 0.5;
                    } else {
                        ext = g;
                        dav = J * du[0];
                        sc = 1.0;
                    }
                    const T jump = ext - ul[0];     // (u_L - u_0)
                    if (i == 0) acc += -nu * (J / S.wi[0]) * dav + sig * (J / S.wi[0]) * jump;
                    acc += nu * sc * J * J * (S.D[0 * n1 + i] / S.wi[i]) * jump;
                }
            }
            F[(long)e * ns + s] += acc;
        }
    }
}

template <class T>
void spatial_op(const Setup& S, const T* u, T* F) {
    const int d = S.d, nv = S.nv, ns = S.ns, n1 = S.n1;
    std::vector<T> qbuf;
    const T* q = nullptr;
    if (S.viscous) {
        qbuf.resize((size_t)S.E * d * nv * ns);
        lifted_gradient(S, u, qbuf.data());
        q = qbuf.data();
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e) {
        for (int s = 0; s < ns; ++s) {
            T acc[8], ui[8], qi[24], uk[8], qk[24], f[8], fo[8], un[8], qn[24], H[8];
            for (int v = 0; v < nv; ++v) acc[v] = 0.0;
            gather_node(S, u, q, e, s, ui, qi);
            for (int a = 0; a < d; ++a) {
                const double J = 2.0 / S.h[a];
                const int i = S.ncoord(s, a);
                // volume term: -(2/h_a) sum_k D_ik f_a(u_k)
                for (int k = 0; k < n1; ++k) {
                    const int sk = S.node_with(s, a, k);
                    gather_node(S, u, q, e, sk, uk, qk);
                    total_flux(S, a, uk, qk, f, S.vel(e, sk, a));
                    for (int v = 0; v < nv; ++v) acc[v] -= J * S.D[i * n1 + k] * f[v];
                }
                const double ba = S.vel(e, s, a);
                total_flux(S, a, ui, qi, fo, ba);
                // surface terms: -(2/h_a) M^-1 B (H - f); on a Dirichlet
                // boundary the exterior state g (its gradient: the interior one)
                if (i == n1 - 1) {
                    int en = S.neighbor(e, a, +1);
                    if (en >= 0) {
                        gather_node(S, u, q, en, S.node_with(s, a, 0), un, qn);
                    } else {
                        for (int v = 0; v < nv; ++v) un[v] = T(S.P.bc_value);
                        for (int c = 0; c < d * nv; ++c) qn[c] = qi[c];
                    }
                    num_flux(S, a, ui, un, qi, qn, H, ba);
                    for (int v = 0; v < nv; ++v) acc[v] -= J * (H[v] - fo[v]) / S.wi[n1 - 1];
                }
                if (i == 0) {
                    int en = S.neighbor(e, a, -1);
                    if (en >= 0) {
                        gather_node(S, u, q, en, S.node_with(s, a, n1 - 1), un, qn);
                    } else {
                        for (int v = 0; v < nv; ++v) un[v] = T(S.P.bc_value);
                        for (int c = 0; c < d * nv; ++c) qn[c] = qi[c];
                    }
                    num_flux(S, a, un, ui, qn, qi, H, ba);
                    for (int v = 0; v < nv; ++v) acc[v] += J * (H[v] - fo[v]) / S.wi[0];
                }
            }
            for (int v = 0; v < nv; ++v) {
                acc[v] += S.P.react * ui[v];
                F[((long)e * nv + v) * ns + s] = acc[v];
            }
        }
    }
    if (S.sipg) sipg_terms(S, u, F);
}

// Apply F at every time node of a slab vector.
template <class T>
void spatial_op_slab(const Setup& S, const T* U, T* FU) {
    const int nv = S.nv, ns = S.ns, Nt = S.Nt;
    std::vector<T> u((size_t)S.E * nv * ns), F((size_t)S.E * nv * ns);
    for (int j = 0; j < Nt; ++j) {
        for (int e = 0; e < S.E; ++e)
            for (int v = 0; v < nv; ++v)
                for (int s = 0; s < ns; ++s)
                    u[((long)e * nv + v) * ns + s] = U[(((long)e * nv + v) * Nt + j) * ns + s];
        spatial_op(S, u.data(), F.data());
        for (int e = 0; e < S.E; ++e)
            for (int v = 0; v < nv; ++v)
                for (int s = 0; s < ns; ++s)
                    FU[(((long)e * nv + v) * Nt + j) * ns + s] = F[((long)e * nv + v) * ns + s];
    }
}

// ---------------------------------------------------------------------------
// Slab residuals.
// ---------------------------------------------------------------------------
// DG-SEM in time, eq. (DG_vs_RK:DG) as R = RHS - LHS:
//   R = (D_tau^T M_tau (x) I) U - (B_tau (x) I) U* + dt/2 (M_tau (x) I) F(U),
// with the upwind flux U* = (u^n, 0, ..., 0, u^Nt), eq. (upwind_flux).
template <class T>
void residual_dg(const Setup& S, const T* U, const T* uprev, double dt, T* R) {
    const int nv = S.nv, ns = S.ns, Nt = S.Nt;
    std::vector<T> FU(S.slab_size());
    spatial_op_slab(S, U, FU.data());
#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e)
        for (int v = 0; v < nv; ++v)
            for (int s = 0; s < ns; ++s) {
                const long base = ((long)e * nv + v) * Nt * ns + s;
                for (int j = 0; j < Nt; ++j) {
                    T r = 0.0;
                    // (D^T M)_{jk} = D_{kj} w_k
                    for (int k = 0; k < Nt; ++k) r += S.Dt[k * Nt + j] * S.om[k] * U[base + (long)k * ns];
                    // -(B U*)_j:  B = diag(-1, 0, ..., 0, 1)
                    if (j == 0) r += uprev[((long)e * nv + v) * ns + s];
                    if (j == Nt - 1) r -= U[base + (long)(Nt - 1) * ns];
                    r += 0.5 * dt * S.om[j] * FU[base + (long)j * ns];
                    R[base + (long)j * ns] = r;
                }
            }
}

// Butcher tableaux of Lobatto IIIC, Appendix B.
bool appendix_b(int Nt, double* A, double* b, double* c) {
    const double r5 = std::sqrt(5.0);
    if (Nt == 2) {
        const double a[4] = {0.5, -0.5, 0.5, 0.5};
        std::memcpy(A, a, sizeof a);
        b[0] = b[1] = 0.5;
        c[0] = 0.0; c[1] = 1.0;
        return true;
    }
    if (Nt == 3) {
        const double a[9] = {1.0 / 6, -1.0 / 3, 1.0 / 6,
                             1.0 / 6, 5.0 / 12, -1.0 / 12,
                             1.0 / 6, 2.0 / 3, 1.0 / 6};
        std::memcpy(A, a, sizeof a);
        b[0] = 1.0 / 6; b[1] = 2.0 / 3; b[2] = 1.0 / 6;
        c[0] = 0.0; c[1] = 0.5; c[2] = 1.0;
        return true;
    }
    if (Nt == 4) {
        const double a[16] = {1.0 / 12, -r5 / 12, r5 / 12, -1.0 / 12,
                              1.0 / 12, 0.25, (10 - 7 * r5) / 60, r5 / 60,
                              1.0 / 12, (10 + 7 * r5) / 60, 0.25, -r5 / 60,
                              1.0 / 12, 5.0 / 12, 5.0 / 12, 1.0 / 12};
        std::memcpy(A, a, sizeof a);
        b[0] = 1.0 / 12; b[1] = 5.0 / 12; b[2] = 5.0 / 12; b[3] = 1.0 / 12;
        c[0] = 0.0; c[1] = 0.5 - r5 / 10; c[2] = 0.5 + r5 / 10; c[3] = 1.0;
        return true;
    }
    return false;
}

// Lobatto IIIC stage equations, eqs. (RK_stage_equations), (DG_vs_RK:RK):
//   R_RK = U - 1 (x) u^n - dt (A (x) I) F(U).
template <class T>
void residual_rk(const Setup& S, const T* U, const T* uprev, double dt, T* R) {
    const int nv = S.nv, ns = S.ns, Nt = S.Nt;
    double A[16], b[4], c[4];
    if (!appendix_b(Nt, A, b, c)) std::abort();
    std::vector<T> FU(S.slab_size());
    spatial_op_slab(S, U, FU.data());
#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e)
        for (int v = 0; v < nv; ++v)
            for (int s = 0; s < ns; ++s) {
                const long base = ((long)e * nv + v) * Nt * ns + s;
                for (int j = 0; j < Nt; ++j) {
                    T r = U[base + (long)j * ns] - uprev[((long)e * nv + v) * ns + s];
                    for (int k = 0; k < Nt; ++k) r -= dt * A[j * Nt + k] * FU[base + (long)k * ns];
                    R[base + (long)j * ns] = r;
                }
            }
}

// Space-time Galerkin form, eqs. (stconvDiscr)-(stsurfaceint), with the
// space-time fluxes [F_c, u], [F_v, 0] and numerical fluxes [H_c, u*], [H_v, 0]
// (Sec. "Space-Time DG-SEM"):
//   <L(u), psi_J> = sum_q W_q ( F(u_q) . grad_x psi_J(q) + u_q d_t psi_J(q) + S(u_q) psi_J(q) )
//                 - sum over element faces of  W_f (H . n) psi_J(f),
// with every integral taken by the tensor LGL rule of the (d+1)-cube and every
// basis value/derivative evaluated from the Lagrange product formula.
void residual_galerkin(const Setup& S, const double* U, const double* uprev, double dt, double* R) {
    const int d = S.d, nv = S.nv, ns = S.ns, n1 = S.n1, Nt = S.Nt;
    const int nst = ns * Nt;   // space-time nodes per element; index J = j*ns + s
    // Basis tables: L[i][q] = l_i(x_q), DL[i][q] = l_i'(x_q), ends l_i(-1), l_i(+1).
    std::vector<double> L(n1 * n1), DL(n1 * n1), Lm(n1), Lp(n1);
    for (int i = 0; i < n1; ++i) {
        for (int q = 0; q < n1; ++q) {
            L[i * n1 + q] = lagrange(S.xi, i, S.xi[q]);
            DL[i * n1 + q] = lagrange_deriv(S.xi, i, S.xi[q]);
        }
        Lm[i] = lagrange(S.xi, i, -1.0);
        Lp[i] = lagrange(S.xi, i, 1.0);
    }
    std::vector<double> Lt(Nt * Nt), DLt(Nt * Nt), Ltm(Nt), Ltp(Nt);
    for (int i = 0; i < Nt; ++i) {
        for (int q = 0; q < Nt; ++q) {
            Lt[i * Nt + q] = lagrange(S.tau, i, S.tau[q]);
            DLt[i * Nt + q] = lagrange_deriv(S.tau, i, S.tau[q]);
        }
        Ltm[i] = lagrange(S.tau, i, -1.0);
        Ltp[i] = lagrange(S.tau, i, 1.0);
    }
    auto uat = [&](int e, int v, int j, int s) -> double {
        return U[(((long)e * nv + v) * Nt + j) * ns + s];
    };
    // value of the spatial basis phi_{sJ} at node sq (tensor product of L tables)
    auto phi = [&](int sJ, int sq) {
        double r = 1.0;
        for (int a = 0; a < d; ++a) r *= L[S.ncoord(sJ, a) * n1 + S.ncoord(sq, a)];
        return r;
    };
    auto dphi = [&](int sJ, int sq, int a) {  // d phi / d x_a at node sq (physical)
        double r = 2.0 / S.h[a];
        for (int b = 0; b < d; ++b)
            r *= (b == a ? DL : L)[S.ncoord(sJ, b) * n1 + S.ncoord(sq, b)];
        return r;
    };

    // BR1 weak gradient, per time node (no viscous term in time):
    //   (M q_a)_J = - sum_q W_q u_q d_a phi_J(q) + sum_{faces normal to a} W_f u_hat n_a phi_J(f)
    std::vector<double> qg;
    if (S.viscous) {
        qg.assign((size_t)S.E * Nt * d * nv * ns, 0.0);   // [e][j][b][v][s]
#pragma omp parallel for schedule(static)
        for (int e = 0; e < S.E; ++e)
            for (int j = 0; j < Nt; ++j)
                for (int b = 0; b < d; ++b)
                    for (int v = 0; v < nv; ++v)
                        for (int sJ = 0; sJ < ns; ++sJ) {
                            double rhs = 0.0, mass = 0.0;
                            for (int sq = 0; sq < ns; ++sq) {
                                double W = S.wphys(sq);
                                rhs -= W * uat(e, v, j, sq) * dphi(sJ, sq, b);
                                mass += W * phi(sJ, sq) * phi(sJ, sq);
                            }
                            for (int side = 0; side < 2; ++side) {
                                const int iface = side ? n1 - 1 : 0;
                                const double nrm = side ? 1.0 : -1.0;
                                int en = S.neighbor(e, b, side ? +1 : -1);
                                for (int sf = 0; sf < ns; ++sf) {
                                    if (S.ncoord(sf, b) != iface) continue;
                                    double Wf = 1.0, ph = 1.0;
                                    for (int c = 0; c < d; ++c) {
                                        if (c == b) {
                                            ph *= (side ? Lp : Lm)[S.ncoord(sJ, c)];
                                        } else {
                                            Wf *= 0.5 * S.h[c] * S.wi[S.ncoord(sf, c)];
                                            ph *= L[S.ncoord(sJ, c) * n1 + S.ncoord(sf, c)];
                                        }
                                    }
                                    double uo = uat(e, v, j, sf);
                                    // Dirichlet boundary: u_hat = g
                                    double uh = S.P.bc_value;
                                    if (en >= 0) uh = 0.5 * (uo + uat(en, v, j, S.node_with(sf, b, n1 - 1 - iface)));
                                    rhs += Wf * uh * nrm * ph;
                                }
                            }
                            qg[((((long)e * Nt + j) * d + b) * nv + v) * ns + sJ] = rhs / mass;
                        }
    }
    auto gather = [&](int e, int j, int s, double* un, double* qn) {
        for (int v = 0; v < nv; ++v) un[v] = uat(e, v, j, s);
        if (S.viscous)
            for (int b = 0; b < d; ++b)
                for (int v = 0; v < nv; ++v)
                    qn[b * nv + v] = qg[((((long)e * Nt + j) * d + b) * nv + v) * ns + s];
    };
    // SIPG: derivative along a of the element's polynomial (scalar) at node s
    auto broken_grad = [&](int e, int j, int s, int a) {
        double g = 0.0;
        for (int sp = 0; sp < ns; ++sp) g += uat(e, 0, j, sp) * dphi(sp, s, a);
        return g;
    };

#pragma omp parallel for schedule(static)
    for (int e = 0; e < S.E; ++e) {
        std::vector<double> res((size_t)nv * nst, 0.0);
        double uq[8], qq[24], f[8], un[8], qn[24], H[8];
        // volume integral
        for (int jq = 0; jq < Nt; ++jq)
            for (int sq = 0; sq < ns; ++sq) {
                const double W = 0.5 * dt * S.om[jq] * S.wphys(sq);
                gather(e, jq, sq, uq, qq);
                double fl[3][8];
                for (int a = 0; a < d; ++a) {
                    total_flux(S, a, uq, qq, fl[a], S.vel(e, sq, a));
                    if (S.sipg) fl[a][0] -= S.P.nu * broken_grad(e, jq, sq, a);   // F_v = nu grad u
                }
                for (int jJ = 0; jJ < Nt; ++jJ)
                    for (int sJ = 0; sJ < ns; ++sJ) {
                        const double pt = Lt[jJ * Nt + jq];
                        const double ph = phi(sJ, sq);
                        const double dpt = (2.0 / dt) * DLt[jJ * Nt + jq];
                        for (int v = 0; v < nv; ++v) {
                            double t = uq[v] * ph * dpt + S.P.react * uq[v] * ph * pt;
                            for (int a = 0; a < d; ++a) t += fl[a][v] * dphi(sJ, sq, a) * pt;
                            res[(size_t)v * nst + jJ * ns + sJ] += W * t;
                        }
                    }
            }
        // spatial faces
        for (int a = 0; a < d; ++a)
            for (int side = 0; side < 2; ++side) {
                const int iface = side ? n1 - 1 : 0;
                const double nrm = side ? 1.0 : -1.0;
                const int en = S.neighbor(e, a, side ? +1 : -1);
                for (int jq = 0; jq < Nt; ++jq)
                    for (int sf = 0; sf < ns; ++sf) {
                        if (S.ncoord(sf, a) != iface) continue;
                        double Wf = 0.5 * dt * S.om[jq];
                        for (int c = 0; c < d; ++c)
                            if (c != a) Wf *= 0.5 * S.h[c] * S.wi[S.ncoord(sf, c)];
                        gather(e, jq, sf, uq, qq);
                        const int sfn = S.node_with(sf, a, n1 - 1 - iface);
                        if (en >= 0) {
                            gather(en, jq, sfn, un, qn);
                        } else {     // Dirichlet boundary: exterior state g, interior gradient
                            for (int v = 0; v < nv; ++v) un[v] = S.P.bc_value;
                            for (int c = 0; c < d * nv; ++c) qn[c] = qq[c];
                        }
                        const double ba = S.vel(e, sf, a);
                        if (side) num_flux(S, a, uq, un, qq, qn, H, ba);
                        else      num_flux(S, a, un, uq, qn, qq, H, ba);
                        // SIPG: {grad u}.n, the jump u_K - u_N and the penalty
                        double dav = 0.0, jmp = 0.0, sym = 0.0;
                        if (S.sipg) {
                            const double dK = broken_grad(e, jq, sf, a);
                            dav = en >= 0 ? 0.5 * (dK + broken_grad(en, jq, sfn, a)) : dK;
                            jmp = uq[0] - un[0];
                            sym = en >= 0 ? 0.5 : 1.0;
                        }
                        const double sig = S.eta * S.P.nu / S.h[a];
                        for (int jJ = 0; jJ < Nt; ++jJ)
                            for (int sJ = 0; sJ < ns; ++sJ) {
                                double ph = Lt[jJ * Nt + jq];
                                for (int c = 0; c < d; ++c)
                                    ph *= (c == a) ? (side ? Lp : Lm)[S.ncoord(sJ, c)]
                                                   : L[S.ncoord(sJ, c) * n1 + S.ncoord(sf, c)];
                                for (int v = 0; v < nv; ++v)
                                    res[(size_t)v * nst + jJ * ns + sJ] -= Wf * nrm * H[v] * ph;
                                if (S.sipg) {
                                    // -a(u, psi): + nu {u'} n psi + nu {psi'} n (u_K - u_N) - sigma (u_K - u_N) psi
                                    const double dps = Lt[jJ * Nt + jq] * dphi(sJ, sf, a);
                                    res[(size_t)jJ * ns + sJ] += Wf * (S.P.nu * nrm * dav * ph +
                                                                       S.P.nu * sym * nrm * dps * jmp - sig * jmp * ph);
                                }
                            }
                    }
            }
        // temporal faces: top uses the interior trace u^Nt, bottom the previous slab u^n
        for (int sf = 0; sf < ns; ++sf) {
            const double Wf = S.wphys(sf);
            for (int jJ = 0; jJ < Nt; ++jJ)
                for (int sJ = 0; sJ < ns; ++sJ) {
                    const double ph = phi(sJ, sf);
                    for (int v = 0; v < nv; ++v) {
                        double top = uat(e, v, Nt - 1, sf);
                        double bot = uprev[((long)e * nv + v) * ns + sf];
                        res[(size_t)v * nst + jJ * ns + sJ] -=
                            Wf * ph * (top * Ltp[jJ] - bot * Ltm[jJ]);
                    }
                }
        }
        for (int v = 0; v < nv; ++v)
            for (int jJ = 0; jJ < Nt; ++jJ)
                for (int sJ = 0; sJ < ns; ++sJ)
                    R[(((long)e * nv + v) * Nt + jJ) * ns + sJ] = res[(size_t)v * nst + jJ * ns + sJ];
    }
}

// ---------------------------------------------------------------------------
// Jacobian-vector products by forward-mode dual numbers.
// ---------------------------------------------------------------------------
void jvp(const Setup& S, int form, const double* U, double dt, const double* V, double* JV) {
    const long n = S.slab_size(), m = S.space_size();
    std::vector<Dual> Ud(n), Rd(n), up(m);
    for (long i = 0; i < n; ++i) Ud[i] = Dual(U[i], V[i]);
    for (long i = 0; i < m; ++i) up[i] = Dual(0.0, 0.0);   // u^n is data, not an unknown
    if (form == ORC_FORM_RK) residual_rk(S, Ud.data(), up.data(), dt, Rd.data());
    else residual_dg(S, Ud.data(), up.data(), dt, Rd.data());
    for (long i = 0; i < n; ++i) JV[i] = Rd[i].d;
}

void residual_any(const Setup& S, int form, const double* U, const double* uprev, double dt, double* R) {
    if (form == ORC_FORM_RK) residual_rk(S, U, uprev, dt, R);
    else if (form == ORC_FORM_GALERKIN) residual_galerkin(S, U, uprev, dt, R);
    else residual_dg(S, U, uprev, dt, R);
}

double norm2(const std::vector<double>& x) {
    double s = 0.0;
    for (double v : x) s += v * v;
    return std::sqrt(s);
}

// Dense LU with partial pivoting, solves A x = b in place (A row-major n x n).
bool lu_solve(int n, std::vector<double>& A, std::vector<double>& b) {
    std::vector<int> piv(n);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
        if (A[(size_t)p * n + c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[(size_t)c * n + k], A[(size_t)p * n + k]);
            std::swap(b[c], b[p]);
        }
        const double inv = 1.0 / A[(size_t)c * n + c];
#pragma omp parallel for schedule(static)
        for (int r = c + 1; r < n; ++r) {
            double f = A[(size_t)r * n + c] * inv;
            if (f == 0.0) continue;
            A[(size_t)r * n + c] = f;
            for (int k = c + 1; k < n; ++k) A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[(size_t)r * n + k] * b[k];
        b[r] = s / A[(size_t)r * n + r];
    }
    return true;
}

// Restarted GMRES(m) with modified Gram-Schmidt and Givens rotations,
// zero initial guess, stops at ||b - A x|| <= rtol ||b||.
template <class Op>
int gmres_mgs(long n, Op apply, const std::vector<double>& b, std::vector<double>& x, double rtol,
              int m, int maxit) {
    x.assign(n, 0.0);
    const double bn = norm2(b);
    if (bn == 0.0) return 0;
    std::vector<std::vector<double>> V(m + 1, std::vector<double>(n));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), w(n), r(n);
    int total = 0;
    while (total < maxit) {
        apply(x.data(), w.data());
        for (long i = 0; i < n; ++i) r[i] = b[i] - w[i];
        double beta = norm2(r);
        if (beta <= rtol * bn) break;
        for (long i = 0; i < n; ++i) V[0][i] = r[i] / beta;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (; k < m && total < maxit; ++k, ++total) {
            apply(V[k].data(), w.data());
            for (int i = 0; i <= k; ++i) {   // modified Gram-Schmidt
                double h = 0.0;
                for (long t = 0; t < n; ++t) h += w[t] * V[i][t];
                H[(size_t)i * m + k] = h;
                for (long t = 0; t < n; ++t) w[t] -= h * V[i][t];
            }
            double hn = norm2(w);
            H[(size_t)(k + 1) * m + k] = hn;
            if (hn > 0.0)
                for (long t = 0; t < n; ++t) V[k + 1][t] = w[t] / hn;
            for (int i = 0; i < k; ++i) {
                double a = H[(size_t)i * m + k], c = H[(size_t)(i + 1) * m + k];
                H[(size_t)i * m + k] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)k * m + k], c = H[(size_t)(k + 1) * m + k];
            double den = std::sqrt(a * a + c * c);
            cs[k] = a / den; sn[k] = c / den;
            H[(size_t)k * m + k] = den;
            H[(size_t)(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (std::fabs(g[k + 1]) <= rtol * bn || hn == 0.0) { ++k; ++total; break; }
        }
        // back-substitution and update
        std::vector<double> y(k);
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[(size_t)i * m + j] * y[j];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (long t = 0; t < n; ++t) x[t] += y[i] * V[i][t];
    }
    return total;
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

int orc_nvars(int eq, int dim) {
    return (eq == ORC_EULER || eq == ORC_NS_BR1) ? dim + 2 : 1;
}
long orc_slab_size(const orc_problem* p) { return Setup(p).slab_size(); }
long orc_space_size(const orc_problem* p) { return Setup(p).space_size(); }

void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_lgl(int n, double* x, double* w, double* D) {
    std::vector<double> X, W;
    lgl(n, X, W);
    for (int i = 0; i < n; ++i) { x[i] = X[i]; w[i] = W[i]; }
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) D[j * n + k] = lagrange_deriv(X, k, X[j]);
}

void orc_butcher_from_sbp(int Nt, double* A, double* b, double* c) {
    // A = 1/2 (D_tau + M_tau^-1 e1 e1^T)^-1, b = 1/2 M_tau 1, c = (1 + tau)/2
    std::vector<double> X, W, M(Nt * Nt), Minv;
    lgl(Nt, X, W);
    for (int j = 0; j < Nt; ++j)
        for (int k = 0; k < Nt; ++k) M[j * Nt + k] = lagrange_deriv(X, k, X[j]);
    M[0] += 1.0 / W[0];
    invert(Nt, M, Minv);
    for (int i = 0; i < Nt * Nt; ++i) A[i] = 0.5 * Minv[i];
    for (int i = 0; i < Nt; ++i) { b[i] = 0.5 * W[i]; c[i] = 0.5 * (1.0 + X[i]); }
}

int orc_butcher_appendix_b(int Nt, double* A, double* b, double* c) {
    return appendix_b(Nt, A, b, c) ? 0 : -1;
}

void orc_node_coords(const orc_problem* p, double* X) {
    Setup S(p);
    for (int e = 0; e < S.E; ++e)
        for (int a = 0; a < S.d; ++a)
            for (int s = 0; s < S.ns; ++s) X[((long)e * S.d + a) * S.ns + s] = S.coord(e, s, a);
}

void orc_spatial_op(const orc_problem* p, const double* u, double* F) {
    Setup S(p);
    spatial_op(S, u, F);
}

void orc_spatial_jvp(const orc_problem* p, const double* u, const double* v, double* Jv) {
    Setup S(p);
    const long m = S.space_size();
    std::vector<Dual> ud(m), Fd(m);
    for (long i = 0; i < m; ++i) ud[i] = Dual(u[i], v[i]);
    spatial_op(S, ud.data(), Fd.data());
    for (long i = 0; i < m; ++i) Jv[i] = Fd[i].d;
}

void orc_num_flux(const orc_problem* p, int axis, const double* uL, const double* uR,
                  const double* qL, const double* qR, double* H) {
    Setup S(p);
    double z[24] = {0};
    num_flux(S, axis, uL, uR, qL ? qL : z, qR ? qR : z, H, p->a[axis]);
}

void orc_flux(const orc_problem* p, int axis, const double* u, const double* q, double* f) {
    Setup S(p);
    double z[24] = {0};
    total_flux(S, axis, u, q ? q : z, f, p->a[axis]);
}

void orc_residual(const orc_problem* p, int form, const double* U, const double* uprev, double dt,
                  double* R) {
    Setup S(p);
    residual_any(S, form, U, uprev, dt, R);
}

void orc_jvp(const orc_problem* p, int form, const double* U, double dt, const double* V, double* JV) {
    Setup S(p);
    jvp(S, form, U, dt, V, JV);
}

int orc_solve(const orc_problem* p, int form, const double* uprev, double dt, double tol,
              int max_newton, int dense_limit, double* Uout, orc_stats* st) {
    Setup S(p);
    if (form == ORC_FORM_GALERKIN) form = ORC_FORM_DG;   // same solution set, cheaper residual
    const long n = S.slab_size();
    const int nv = S.nv, ns = S.ns, Nt = S.Nt;
    std::vector<double> U(n), R(n), dU(n), rhs(n);
    for (int e = 0; e < S.E; ++e)      // U0 = 1 (x) u^n
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < Nt; ++j)
                for (int s = 0; s < ns; ++s)
                    U[(((long)e * nv + v) * Nt + j) * ns + s] = uprev[((long)e * nv + v) * ns + s];
    residual_any(S, form, U.data(), uprev, dt, R.data());
    const double r0 = norm2(R);
    double rn = r0;
    int it = 0, lin = 0;
    const double target = tol * std::max(1.0, r0);
    while (rn > target && it < max_newton) {
        for (long i = 0; i < n; ++i) rhs[i] = -R[i];
        if (n <= dense_limit) {
            std::vector<double> J((size_t)n * n), col(n), ev(n, 0.0);
            for (long c = 0; c < n; ++c) {
                ev[c] = 1.0;
                jvp(S, form, U.data(), dt, ev.data(), col.data());
                ev[c] = 0.0;
                for (long r = 0; r < n; ++r) J[(size_t)r * n + c] = col[r];
            }
            if (!lu_solve((int)n, J, rhs)) break;
            dU = rhs;
        } else {
            auto op = [&](const double* x, double* y) { jvp(S, form, U.data(), dt, x, y); };
            double rt = std::max(1e-14, std::min(1e-10, 0.1 * target / rn));
            lin += gmres_mgs(n, op, rhs, dU, rt, 60, 20000);
        }
        for (long i = 0; i < n; ++i) U[i] += dU[i];
        residual_any(S, form, U.data(), uprev, dt, R.data());
        rn = norm2(R);
        ++it;
    }
    std::memcpy(Uout, U.data(), sizeof(double) * n);
    if (st) {
        st->newton_its = it; st->linear_its = lin; st->res0 = r0; st->res_final = rn;
        st->converged = rn <= target;
    }
    return rn <= target ? 0 : 1;
}

}  // extern "C"
