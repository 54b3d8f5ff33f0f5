// Serial FP64 CPU oracle of the implicit LSKUM iteration with modified LU-SGS.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// HIP library is checked against; the library never links, loads or calls it.
// It shares no code with the HIP path.  Only tests, the smoke check and the
// benchmark's CPU-baseline leg may use it.
//
// Every function follows the paper (Verma, Mamidi, Nemili, "GPU Accelerated
// Implicit Kinetic Meshfree Method based on Modified LU-SGS", 2024) in its
// order and notation; the cited section/equation/algorithm is given at each
// function.  Where the paper is silent, the reading used is stated as
// "Reading:" and applies to the HIP path as well.
//
// Build: g++ -O2 -ffp-contract=off -fno-fast-math -fopenmp -std=c++17 -shared -fPIC
//
// Threads: the per-point loops (and, in the sweeps, the points of one colour)
// are split over OpenMP threads.  Every point writes only its own outputs
// from inputs no other iteration of the same loop writes, and the sums over
// points (residual norm, forces) stay serial, so results are bitwise the same
// for any thread count (tested).
//
// Conventions
//   U = (rho, rho u1, rho u2, rho E), E total specific energy (eq. 2; the
//   energy flux (p + rho e) u1 and Listing 1's pressure make e total energy).
//   Point types: 0 wall, 1 interior, 2 outer.  Frame: unit tangent (tx, ty);
//   the normal n = (-ty, tx) points into the fluid.  Interior/outer: t = (1,0).
//   Colours are 0-based (the paper's colour k is our k-1).
//
// Pins (tests/test_oracle_*.py): split fluxes against quadrature of the
// half-range Maxwellian moments and G+ + G- = G (eq. 2); tangents against
// central differences and, summed over the halves, against the complex-step
// derivative of the unsplit flux (eq. 2); LS weights reproduce linear fields;
// the inner iterations keep exact quadratic derivatives; uniform flow gives
// R == 0; the sweeps equal a dense (D+U)^-1 D (D+L)^-1 (-R) solve; colouring
// validity; the Anandhanarayanan diagonal in closed form at rest and at a
// supersonic split velocity (eq. 34-35); forces of a linear wall pressure by
// the divergence theorem (sign and projection), zero lift at zero incidence
// and positive lift at positive incidence; the kinetic far field: uniform flow
// a fixed point, the ghost's flux difference exactly, its diagonal in closed
// form.
// Parity unpinned (no external value exists): the boundary treatment, the
// time step rule, the residual norm and the tolerance anchor are readings,
// pinned only by invariants.

#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Forward-mode algorithmic differentiation (the paper's tangent mode, done by
// operator overloading instead of source transformation).  v is the value,
// d the derivative along the seed direction.
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
inline Dual operator+(double a, Dual b) { return Dual(a) + b; }
inline Dual operator+(Dual a, double b) { return a + Dual(b); }
inline Dual operator-(double a, Dual b) { return Dual(a) - b; }
inline Dual operator-(Dual a, double b) { return a - Dual(b); }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
inline Dual sqrt(Dual a) {
    double s = std::sqrt(a.v);
    return {s, a.d / (2.0 * s)};
}
inline Dual exp(Dual a) {
    double e = std::exp(a.v);
    return {e, e * a.d};
}
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline Dual erf(Dual a) {
    return {std::erf(a.v), 2.0 / std::sqrt(kPi) * std::exp(-a.v * a.v) * a.d};
}
using std::erf;
using std::exp;
using std::log;
using std::sqrt;

template <class T>
struct Prim {
    T rho, u1, u2, p;
};

// Primitive variables from the conserved vector (eq. 2; pressure as in
// Listing 1 with gamma - 1 general).
template <class T>
Prim<T> prim_from_U(const T U[4], double gamma) {
    Prim<T> w;
    w.rho = U[0];
    w.u1 = U[1] / U[0];
    w.u2 = U[2] / U[0];
    w.p = (gamma - 1.0) * (U[3] - 0.5 * w.rho * (w.u1 * w.u1 + w.u2 * w.u2));
    return w;
}

template <class T>
void U_from_prim(const Prim<T>& w, double gamma, T U[4]) {
    U[0] = w.rho;
    U[1] = w.rho * w.u1;
    U[2] = w.rho * w.u2;
    U[3] = w.p / (gamma - 1.0) + 0.5 * w.rho * (w.u1 * w.u1 + w.u2 * w.u2);
}

// Kinetic split flux along unit direction d = (dx, dy), sign s = +1 / -1:
// the half-range moment  <Psi, v_d F>  over v_d > 0 (s = +1) or v_d < 0
// (s = -1) of the Maxwellian F and moment vector Psi of eq. (3)-(4), i.e. the
// split fluxes of the KFVS equations (eq. 5-6).  With beta = rho/(2p),
// S = u_d sqrt(beta), A = (1 + s erf S)/2 and B = exp(-S^2)/(2 sqrt(pi beta)):
//   mass     rho (u_d A + s B)
//   momentum p A d + u * mass
//   energy   (rho E + p) u_d A + s (rho E + p/2) B
// (Section 2, eq. 3-6; the closed form is not printed in the paper and is
// pinned against numerical quadrature of the moments in the tests.)
template <class T>
void split_flux(const Prim<T>& w, double dx, double dy, int s, double gamma, T G[4]) {
    T beta = w.rho / (2.0 * w.p);
    T ud = w.u1 * dx + w.u2 * dy;
    T S = ud * sqrt(beta);
    T A = 0.5 * (1.0 + (double)s * erf(S));
    T B = exp(-(S * S)) / (2.0 * sqrt(kPi * beta));
    T rhoE = w.p / (gamma - 1.0) + 0.5 * w.rho * (w.u1 * w.u1 + w.u2 * w.u2);
    T mass = w.rho * (ud * A + (double)s * B);
    G[0] = mass;
    G[1] = w.p * A * dx + w.u1 * mass;
    G[2] = w.p * A * dy + w.u2 * mass;
    G[3] = (rhoE + w.p) * ud * A + (double)s * (rhoE + 0.5 * w.p) * B;
}

// q-variables (eq. 14).
template <class T>
void q_from_prim(const Prim<T>& w, double gamma, T q[4]) {
    T beta = w.rho / (2.0 * w.p);
    q[0] = log(w.rho) + log(beta) / (gamma - 1.0) - beta * (w.u1 * w.u1 + w.u2 * w.u2);
    q[1] = 2.0 * beta * w.u1;
    q[2] = 2.0 * beta * w.u2;
    q[3] = -2.0 * beta;
}

// Inverse of eq. (14): beta = -q4/2, u = (q2, q3)/(2 beta),
// rho = exp(q1 + beta |u|^2 - ln(beta)/(gamma - 1)), p = rho/(2 beta).
template <class T>
Prim<T> prim_from_q(const T q[4], double gamma) {
    Prim<T> w;
    T beta = -0.5 * q[3];
    w.u1 = q[1] / (2.0 * beta);
    w.u2 = q[2] / (2.0 * beta);
    w.rho = exp(q[0] + beta * (w.u1 * w.u1 + w.u2 * w.u2) - log(beta) / (gamma - 1.0));
    w.p = w.rho / (2.0 * beta);
    return w;
}

struct Cloud {
    int64_t n;
    const double *x, *y, *tx, *ty;
    const int8_t* type;
    const int32_t *off, *idx;
    const int32_t* colour;
    int32_t ncolour;
};

struct Params {
    double gamma, cfl, mach, aoa_deg;
    int32_t inner_iters, jvp_mode;  // jvp_mode 0 exact tangent, 1 flux difference
    int32_t limiter;                // 0 none (the paper), 1 Venkatakrishnan on q~
    double limiter_k;
    int32_t variant;                // 0 Anandhanarayanan et al., 1 Manish et al.
    int32_t order;                  // 0 colour order (Algorithm 6), 1 wall first (Algorithm 5)
    int32_t farfield;               // 0 outer points held at the free stream, 1 kinetic far field
};

enum { OK = 0, ERR_ARG = -1, ERR_CONN = -2, ERR_DEGEN = -3, ERR_COLOUR = -4, ERR_NONPHYS = -5 };

// One split stencil of a point: direction d, transverse e, sign s.
// Reading: the wall uses its own (t, n) frame: splits t+, t-, n- (the fluid
// side, dn > 0); interior points use x+, x-, y+, y-; outer points are
// Dirichlet, or, with the kinetic far field, use their own (t, n) frame (n out
// of the domain): splits t+, t-, n+ (the inner side, dn < 0), the n- half
// coming from the free stream (see far_field_term).
struct Split {
    double dx, dy, ex, ey;
    int s;
};

int splits_of(const Cloud& c, int64_t p, Split out[4], bool farfield) {
    if (c.type[p] == 2 && !farfield) return 0;
    if (c.type[p] == 0 || c.type[p] == 2) {
        double tx = c.tx[p], ty = c.ty[p];
        double nx = -ty, ny = tx;
        out[0] = {tx, ty, nx, ny, +1};
        out[1] = {tx, ty, nx, ny, -1};
        out[2] = {nx, ny, tx, ty, c.type[p] == 0 ? -1 : +1};
        return 3;
    }
    out[0] = {1.0, 0.0, 0.0, 1.0, +1};
    out[1] = {1.0, 0.0, 0.0, 1.0, -1};
    out[2] = {0.0, 1.0, 1.0, 0.0, +1};
    out[3] = {0.0, 1.0, 1.0, 0.0, -1};
    return 4;
}

// Least-squares weights of one split stencil (eq. 11, eq. 13; eq. 20-24 use
// the same weights for the first-order implicit operator).  The member set is
// N_k = { i : s * da_i < 0 } with da = (r_i - r_0).d, db = (r_i - r_0).e, and
// d/da f ~ sum_i w_i (f_i - f_0),  w_i = (S_bb da_i - S_ab db_i) / det.
// Reading: neighbours with da_i == 0 belong to neither half; a half with fewer
// than two members or det <= 1e-12 S_aa S_bb is degenerate and contributes 0.
struct Stencil {
    std::vector<int32_t> nb;
    std::vector<double> w;
    double ls1 = 0.0;  // LS_k(1) = sum of the weights (eq. 31)
    bool degenerate = false;
};

Stencil split_stencil(const Cloud& c, int64_t p, const Split& k) {
    Stencil st;
    double saa = 0, sbb = 0, sab = 0;
    std::vector<double> da, db;
    for (int32_t e = c.off[p]; e < c.off[p + 1]; ++e) {
        int32_t i = c.idx[e];
        double rx = c.x[i] - c.x[p], ry = c.y[i] - c.y[p];
        double a = rx * k.dx + ry * k.dy;
        double b = rx * k.ex + ry * k.ey;
        if (!((double)k.s * a < 0.0)) continue;
        st.nb.push_back(i);
        da.push_back(a);
        db.push_back(b);
        saa += a * a;
        sbb += b * b;
        sab += a * b;
    }
    double det = saa * sbb - sab * sab;
    if (st.nb.size() < 2 || !(det > 1e-12 * saa * sbb)) {
        st.degenerate = true;
        st.nb.clear();
        return st;
    }
    for (size_t j = 0; j < st.nb.size(); ++j) {
        double wj = (sbb * da[j] - sab * db[j]) / det;
        st.w.push_back(wj);
        st.ls1 += wj;
    }
    return st;
}

void project_out_normal(const Cloud& c, int64_t p, double v[4]) {
    double nx = -c.ty[p], ny = c.tx[p];
    double mn = v[1] * nx + v[2] * ny;
    v[1] -= mn * nx;
    v[2] -= mn * ny;
}

// Free stream (reading): rho = 1, p = 1/gamma (unit speed of sound),
// velocity M (cos a, sin a).  Wall points keep rho and p and only the
// tangential part of the velocity.
void free_stream(const Cloud& c, const Params& P, double* U) {
    double a = P.aoa_deg * kPi / 180.0;
    for (int64_t p = 0; p < c.n; ++p) {
        Prim<double> w{1.0, P.mach * std::cos(a), P.mach * std::sin(a), 1.0 / P.gamma};
        if (c.type[p] == 0) {
            double tx = c.tx[p], ty = c.ty[p];
            double ut = w.u1 * tx + w.u2 * ty;
            w.u1 = ut * tx;
            w.u2 = ut * ty;
        }
        double Up[4];
        U_from_prim(w, P.gamma, Up);
        for (int v = 0; v < 4; ++v) U[v * c.n + p] = Up[v];
    }
}

// q_variables(): eq. (14) at every point (Algorithm 1).
int q_variables(const Cloud& c, const Params& P, const double* U, double* q) {
    int st = OK;
#pragma omp parallel for reduction(min : st)
    for (int64_t p = 0; p < c.n; ++p) {
        double Up[4] = {U[p], U[c.n + p], U[2 * c.n + p], U[3 * c.n + p]};
        Prim<double> w = prim_from_U(Up, P.gamma);
        if (!(w.rho > 0.0) || !(w.p > 0.0)) st = ERR_NONPHYS;
        double qp[4];
        q_from_prim(w, P.gamma, qp);
        for (int v = 0; v < 4; ++v) q[v * c.n + p] = qp[v];
    }
    return st;
}

// One least-squares pass for q_x, q_y over the full stencil (eq. 16).
// With qx_in == nullptr it is the first-order pass (dq_i = q_i - q_0);
// otherwise the defect-corrected right-hand side
//   dq~_i = dq_i - 1/2 (dx_i (qx_i - qx_0) + dy_i (qy_i - qy_0))
// uses the previous pass's derivatives (eq. 8-10, 15-16).
// Reading: the inner iterations are Jacobi sweeps over all points.
int q_grad_pass(const Cloud& c, const double* q, const double* qx_in, const double* qy_in,
                double* qx_out, double* qy_out) {
    int st = OK;
#pragma omp parallel for reduction(min : st)
    for (int64_t p = 0; p < c.n; ++p) {
        double sxx = 0, syy = 0, sxy = 0;
        double bx[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0};
        for (int32_t e = c.off[p]; e < c.off[p + 1]; ++e) {
            int32_t i = c.idx[e];
            double dx = c.x[i] - c.x[p], dy = c.y[i] - c.y[p];
            sxx += dx * dx;
            syy += dy * dy;
            sxy += dx * dy;
            for (int v = 0; v < 4; ++v) {
                double dq = q[v * c.n + i] - q[v * c.n + p];
                if (qx_in) {
                    dq = dq - 0.5 * (dx * (qx_in[v * c.n + i] - qx_in[v * c.n + p]) +
                                     dy * (qy_in[v * c.n + i] - qy_in[v * c.n + p]));
                }
                bx[v] += dx * dq;
                by[v] += dy * dq;
            }
        }
        double det = sxx * syy - sxy * sxy;
        if (!(det > 1e-12 * sxx * syy)) {
            st = ERR_DEGEN;
            continue;
        }
        for (int v = 0; v < 4; ++v) {
            qx_out[v * c.n + p] = (syy * bx[v] - sxy * by[v]) / det;
            qy_out[v * c.n + p] = (sxx * by[v] - sxy * bx[v]) / det;
        }
    }
    return st;
}

// q_derivatives(): first-order pass, then m inner iterations (eq. 16).
int q_derivatives(const Cloud& c, const Params& P, const double* q, double* qx, double* qy) {
    int st = q_grad_pass(c, q, nullptr, nullptr, qx, qy);
    if (st) return st;
    std::vector<double> tx(4 * c.n), ty(4 * c.n);
    for (int it = 0; it < P.inner_iters; ++it) {
        st = q_grad_pass(c, q, qx, qy, tx.data(), ty.data());
        if (st) return st;
        std::memcpy(qx, tx.data(), sizeof(double) * 4 * c.n);
        std::memcpy(qy, ty.data(), sizeof(double) * 4 * c.n);
    }
    return OK;
}

// Optional limiter on the q~ reconstruction (not part of the paper, which
// describes none; an addition for transonic robustness).  Venkatakrishnan's
// limiter (AIAA 93-0880 / J. Comput. Phys. 1995): for point p and component v,
// with dmax = max_i q_i - q_p, dmin = min_i q_i - q_p over the full stencil,
// each reconstruction increment d2 = -1/2 (dx_i qx_p + dy_i qy_p) toward a
// neighbour direction gets
//   phi_i = [(d1^2 + eps^2) d2 + 2 d2^2 d1] / [d2 (d1^2 + 2 d2^2 + d1 d2 + eps^2)]
// with d1 = dmax (d2 > 0) or dmin (d2 < 0), phi_i = 1 for d2 = 0, and
// phi_p = min(1, min_i phi_i); eps^2 = (K h)^3 with h the nearest-neighbour
// distance.  The residual then uses phi_p * (qx_p, qy_p).
void limit_gradients(const Cloud& c, const Params& P, const double* q, double* qx, double* qy) {
    std::vector<double> phi(4 * c.n, 1.0);
#pragma omp parallel for
    for (int64_t p = 0; p < c.n; ++p) {
        double rmin = INFINITY;
        double dmax[4] = {0, 0, 0, 0}, dmin[4] = {0, 0, 0, 0};
        for (int32_t e = c.off[p]; e < c.off[p + 1]; ++e) {
            int32_t i = c.idx[e];
            double dx = c.x[i] - c.x[p], dy = c.y[i] - c.y[p];
            double r = std::sqrt(dx * dx + dy * dy);
            if (r < rmin) rmin = r;
            for (int v = 0; v < 4; ++v) {
                double d = q[v * c.n + i] - q[v * c.n + p];
                if (d > dmax[v]) dmax[v] = d;
                if (d < dmin[v]) dmin[v] = d;
            }
        }
        double kh = P.limiter_k * rmin;
        double eps2 = kh * kh * kh;
        for (int v = 0; v < 4; ++v) {
            double ph = 1.0;
            for (int32_t e = c.off[p]; e < c.off[p + 1]; ++e) {
                int32_t i = c.idx[e];
                double dx = c.x[i] - c.x[p], dy = c.y[i] - c.y[p];
                double d2 = -0.5 * (dx * qx[v * c.n + p] + dy * qy[v * c.n + p]);
                if (d2 == 0.0) continue;
                double d1 = d2 > 0.0 ? dmax[v] : dmin[v];
                double num = (d1 * d1 + eps2) * d2 + 2.0 * d2 * d2 * d1;
                double den = d2 * (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2);
                double f = num / den;
                if (f < ph) ph = f;
            }
            phi[v * c.n + p] = ph < 0.0 ? 0.0 : ph;
        }
    }
    for (int64_t k = 0; k < 4 * c.n; ++k) {
        qx[k] *= phi[k];
        qy[k] *= phi[k];
    }
}

// Distance from point p to its nearest neighbour.
double nearest_distance(const Cloud& c, int64_t p) {
    double rmin = INFINITY;
    for (int32_t e = c.off[p]; e < c.off[p + 1]; ++e) {
        int32_t i = c.idx[e];
        double r = std::sqrt((c.x[i] - c.x[p]) * (c.x[i] - c.x[p]) +
                             (c.y[i] - c.y[p]) * (c.y[i] - c.y[p]));
        if (r < rmin) rmin = r;
    }
    return rmin;
}

// q-variables of the free stream (the state outer points start from).
void free_stream_q(const Params& P, double q[4]) {
    double a = P.aoa_deg * kPi / 180.0;
    Prim<double> w{1.0, P.mach * std::cos(a), P.mach * std::sin(a), 1.0 / P.gamma};
    double U[4];
    U_from_prim(w, P.gamma, U);
    q_from_prim(prim_from_U(U, P.gamma), P.gamma, q);
}

// Kinetic far field (reading; the paper holds no outer boundary treatment).
// At an outer point with outward normal n, the molecules entering the domain
// (v_n < 0) are those of the free stream: the n- split derivative of the
// point is the one-sided difference to a ghost point one nearest-neighbour
// distance h outside that carries the free stream,
//   (G_n-(q_inf) - G_n-(q_0)) / h,
// with the point's own (unreconstructed) q-variables.  The splits t+, t-
// and n+ of the point's own stencil supply the rest of its residual.
void far_field_term(const Cloud& c, const Params& P, int64_t p, const double* q, double F[4]) {
    double nx = -c.ty[p], ny = c.tx[p];
    double h = nearest_distance(c, p);
    double qinf[4], q0[4], Gi[4], G0[4];
    free_stream_q(P, qinf);
    for (int v = 0; v < 4; ++v) q0[v] = q[v * c.n + p];
    split_flux(prim_from_q(qinf, P.gamma), nx, ny, -1, P.gamma, Gi);
    split_flux(prim_from_q(q0, P.gamma), nx, ny, -1, P.gamma, G0);
    for (int v = 0; v < 4; ++v) F[v] = (Gi[v] - G0[v]) / h;
}

// flux_residual(): R_0 = sum over the point's split stencils k of
//   sum_{i in N_k} w_i [ G_k(q~_i) - G_k(q~_0^(i)) ]            (eq. 11, 15)
// with q~_i = q_i - 1/2 (dx_i qx_i + dy_i qy_i) and
//      q~_0^(i) = q_0 - 1/2 (dx_i qx_0 + dy_i qy_0).
// Reading: at wall points the normal-momentum component of R is removed;
// outer points carry R = 0.  A q~ with q~_4 >= 0 (beta <= 0) is non-physical.
int flux_residual(const Cloud& c, const Params& P, const double* q, const double* qx,
                  const double* qy, double* R, int64_t* degenerate_count) {
    int st = OK;
    int64_t ndeg = 0;
#pragma omp parallel for reduction(min : st) reduction(+ : ndeg)
    for (int64_t p = 0; p < c.n; ++p) {
        double Rp[4] = {0, 0, 0, 0};
        Split sp[4];
        int ns = splits_of(c, p, sp, P.farfield != 0);
        for (int k = 0; k < ns; ++k) {
            Stencil stn = split_stencil(c, p, sp[k]);
            if (stn.degenerate) {
                ++ndeg;
                continue;
            }
            for (size_t j = 0; j < stn.nb.size(); ++j) {
                int32_t i = stn.nb[j];
                double dx = c.x[i] - c.x[p], dy = c.y[i] - c.y[p];
                double qti[4], qt0[4];
                for (int v = 0; v < 4; ++v) {
                    qti[v] = q[v * c.n + i] - 0.5 * (dx * qx[v * c.n + i] + dy * qy[v * c.n + i]);
                    qt0[v] = q[v * c.n + p] - 0.5 * (dx * qx[v * c.n + p] + dy * qy[v * c.n + p]);
                }
                if (!(qti[3] < 0.0) || !(qt0[3] < 0.0)) {
                    st = ERR_NONPHYS;
                    continue;
                }
                Prim<double> wi = prim_from_q(qti, P.gamma);
                Prim<double> w0 = prim_from_q(qt0, P.gamma);
                double Gi[4], G0[4];
                split_flux(wi, sp[k].dx, sp[k].dy, sp[k].s, P.gamma, Gi);
                split_flux(w0, sp[k].dx, sp[k].dy, sp[k].s, P.gamma, G0);
                for (int v = 0; v < 4; ++v) Rp[v] += stn.w[j] * (Gi[v] - G0[v]);
            }
        }
        if (c.type[p] == 2 && P.farfield) {
            double Fg[4];
            far_field_term(c, P, p, q, Fg);
            for (int v = 0; v < 4; ++v) Rp[v] += Fg[v];
        }
        if (c.type[p] == 0) project_out_normal(c, p, Rp);
        for (int v = 0; v < 4; ++v) R[v * c.n + p] = Rp[v];
    }
    if (degenerate_count) *degenerate_count = ndeg;
    return st;
}

// Split-flux Jacobian-vector product A_k(U) dU.
//   jvp_mode 0: exact, by forward-mode AD of the split flux (Section 3, the
//               paper's modified LU-SGS; Listings 2-3 show the same technique
//               for the unsplit flux);
//   jvp_mode 1: flux difference G_k(U + dU) - G_k(U) (eq. 28).
void flux_jvp(const double U[4], const double dU[4], const Split& k, const Params& P,
              double J[4]) {
    if (P.jvp_mode == 1) {
        double Ua[4], Ga[4], Gb[4];
        for (int v = 0; v < 4; ++v) Ua[v] = U[v] + dU[v];
        split_flux(prim_from_U(Ua, P.gamma), k.dx, k.dy, k.s, P.gamma, Ga);
        split_flux(prim_from_U(U, P.gamma), k.dx, k.dy, k.s, P.gamma, Gb);
        for (int v = 0; v < 4; ++v) J[v] = Ga[v] - Gb[v];
        return;
    }
    Dual Ud[4], G[4];
    for (int v = 0; v < 4; ++v) Ud[v] = Dual(U[v], dU[v]);
    split_flux(prim_from_U(Ud, P.gamma), k.dx, k.dy, k.s, P.gamma, G);
    for (int v = 0; v < 4; ++v) J[v] = G[v].d;
}

// Unsplit Euler flux along unit direction d (eq. 2):
//   (rho u_d, p d + rho u u_d, (rho E + p) u_d).
template <class T>
void unsplit_flux(const Prim<T>& w, double dx, double dy, double gamma, T G[4]) {
    T ud = w.u1 * dx + w.u2 * dy;
    T rhoE = w.p / (gamma - 1.0) + 0.5 * w.rho * (w.u1 * w.u1 + w.u2 * w.u2);
    G[0] = w.rho * ud;
    G[1] = w.p * dx + w.rho * w.u1 * ud;
    G[2] = w.p * dy + w.rho * w.u2 * ud;
    G[3] = (rhoE + w.p) * ud;
}

// Unsplit flux Jacobian product A_d(U) dU: exact by forward-mode AD
// (jvp_mode 0) or the flux difference G_d(U + dU) - G_d(U) (jvp_mode 1), the
// same two treatments as the split products.
void unsplit_jvp(const double U[4], const double dU[4], double dx, double dy, const Params& P,
                 double J[4]) {
    if (P.jvp_mode == 1) {
        double Ua[4], Ga[4], Gb[4];
        for (int v = 0; v < 4; ++v) Ua[v] = U[v] + dU[v];
        unsplit_flux(prim_from_U(Ua, P.gamma), dx, dy, P.gamma, Ga);
        unsplit_flux(prim_from_U(U, P.gamma), dx, dy, P.gamma, Gb);
        for (int v = 0; v < 4; ++v) J[v] = Ga[v] - Gb[v];
        return;
    }
    Dual Ud[4], G[4];
    for (int v = 0; v < 4; ++v) Ud[v] = Dual(U[v], dU[v]);
    unsplit_flux(prim_from_U(Ud, P.gamma), dx, dy, P.gamma, G);
    for (int v = 0; v < 4; ++v) J[v] = G[v].d;
}

// Local time step and scalar diagonal.
// Reading (time step, not given in the paper):
//   dt_0 = CFL * min_i |r_i - r_0| / (|u_0| + a_0).
// Anandhanarayanan et al. (eq. 25 with eq. 34-35): the split Jacobians are
// replaced by +-rho(A^+-) I with rho(A+) = max(u_d + a, 0), rho(A-) =
// max(a - u_d, 0), so D_0 = 1/dt_0 - sum_k s_k LS_k(1) rho(A_k^{s_k}).
// Manish et al. (eq. 29-33): A^+- = (A +- rho(A) I)/2 with rho(A) = |u_d| + a;
// the rho part gives the scalar D_0 = 1/dt_0 - sum_k s_k LS_k(1) rho(A_k)/2 and
// the A part the term S of manish_source.
void timestep_diag(const Cloud& c, const Params& P, const double* U, double* dt, double* D) {
#pragma omp parallel for
    for (int64_t p = 0; p < c.n; ++p) {
        double Up[4] = {U[p], U[c.n + p], U[2 * c.n + p], U[3 * c.n + p]};
        Prim<double> w = prim_from_U(Up, P.gamma);
        double a = std::sqrt(P.gamma * w.p / w.rho);
        double umag = std::sqrt(w.u1 * w.u1 + w.u2 * w.u2);
        double rmin = nearest_distance(c, p);
        double dtp = P.cfl * rmin / (umag + a);
        double Dp = 1.0 / dtp;
        Split sp[4];
        int ns = splits_of(c, p, sp, P.farfield != 0);
        for (int k = 0; k < ns; ++k) {
            Stencil stn = split_stencil(c, p, sp[k]);
            double ud = w.u1 * sp[k].dx + w.u2 * sp[k].dy;
            if (P.variant == 1) {
                Dp -= (double)sp[k].s * stn.ls1 * 0.5 * (std::fabs(ud) + a);
                continue;
            }
            double rad = (double)sp[k].s * ud + a;
            if (rad < 0.0) rad = 0.0;
            Dp -= (double)sp[k].s * stn.ls1 * rad;
        }
        if (c.type[p] == 2 && P.farfield && P.variant == 0) {
            // the far-field ghost: an n- split with the single weight 1/h, LS(1) = 1/h,
            // and the ghost's increment zero (the free stream is fixed)
            double un = -w.u1 * c.ty[p] + w.u2 * c.tx[p];
            double rad = a - un;
            if (rad < 0.0) rad = 0.0;
            Dp += rad / rmin;
        }
        dt[p] = dtp;
        D[p] = Dp;
    }
}

// The term S of Manish et al. (eq. 33, kept on the explicit side, eq. 36-38):
//   S_0 = -1/2 sum_k LS_k(1) (A_{d_k}(U_0) dU_0),
// the unsplit Jacobian of each split's direction at the point's own state.
// Reading: S is evaluated with the increment of the previous iteration
// (dU_prev; zero at the first iteration), the only increment known when the
// forward sweep's right-hand side R - S is formed.  On a symmetric stencil
// LS_k+(1) = -LS_k-(1) and S vanishes.
void manish_source(const Cloud& c, const Params& P, const double* U, const double* dU_prev,
                   double* S) {
#pragma omp parallel for
    for (int64_t p = 0; p < c.n; ++p) {
        double Sp[4] = {0, 0, 0, 0};
        Split sp[4];
        int ns = splits_of(c, p, sp, P.farfield != 0);
        double Up[4] = {U[p], U[c.n + p], U[2 * c.n + p], U[3 * c.n + p]};
        double dUp[4] = {0, 0, 0, 0};
        if (dU_prev)
            for (int v = 0; v < 4; ++v) dUp[v] = dU_prev[v * c.n + p];
        for (int k = 0; k < ns; ++k) {
            Stencil stn = split_stencil(c, p, sp[k]);
            double J[4];
            unsplit_jvp(Up, dUp, sp[k].dx, sp[k].dy, P, J);
            for (int v = 0; v < 4; ++v) Sp[v] -= 0.5 * stn.ls1 * J[v];
        }
        for (int v = 0; v < 4; ++v) S[v * c.n + p] = Sp[v];
    }
}

// LUSGS(): forward and backward sweeps of eq. (27) in colour order
// (Algorithm 6): colours ascending for the forward sweep, descending for the
// backward sweep; within a colour the points are independent.  Order 1 is
// Algorithm 5 (wall points first; see the end of the function).
//   forward:  dU*_0 = -( R_0 + sum_k sum_{i in N_k, col(i) < col(0)} w_i A_k(U_i) dU*_i ) / D_0
//   backward: dU_0  = dU*_0 - ( sum_k sum_{i in N_k, col(i) > col(0)} w_i A_k(U_i) dU_i ) / D_0
// The products A_k(U_i) dU_i are the split-flux Jacobian products at the
// neighbour's state in the point's split direction (eq. 20-24, 27).
// dU* and dU share the array dU.  Reading: wall points drop the
// normal-momentum component of their increment, outer points keep 0.
void lusgs(const Cloud& c, const Params& P, const double* U, const double* R, const double* D,
           double* dU) {
    std::vector<std::vector<int64_t>> by_colour(c.ncolour);
    for (int64_t p = 0; p < c.n; ++p) by_colour[c.colour[p]].push_back(p);
    for (int64_t i = 0; i < 4 * c.n; ++i) dU[i] = 0.0;

    auto sweep_point = [&](int64_t p, bool forward) {
        if (c.type[p] == 2 && !P.farfield) {
            for (int v = 0; v < 4; ++v) dU[v * c.n + p] = 0.0;
            return;
        }
        double acc[4] = {0, 0, 0, 0};
        if (forward)
            for (int v = 0; v < 4; ++v) acc[v] = R[v * c.n + p];
        Split sp[4];
        int ns = splits_of(c, p, sp, P.farfield != 0);
        for (int k = 0; k < ns; ++k) {
            Stencil stn = split_stencil(c, p, sp[k]);
            for (size_t j = 0; j < stn.nb.size(); ++j) {
                int32_t i = stn.nb[j];
                bool take = forward ? (c.colour[i] < c.colour[p]) : (c.colour[i] > c.colour[p]);
                if (!take) continue;
                double Ui[4] = {U[i], U[c.n + i], U[2 * c.n + i], U[3 * c.n + i]};
                double dUi[4] = {dU[i], dU[c.n + i], dU[2 * c.n + i], dU[3 * c.n + i]};
                double J[4];
                flux_jvp(Ui, dUi, sp[k], P, J);
                for (int v = 0; v < 4; ++v) acc[v] += stn.w[j] * J[v];
            }
        }
        double out[4];
        for (int v = 0; v < 4; ++v) {
            if (forward)
                out[v] = -acc[v] / D[p];
            else
                out[v] = dU[v * c.n + p] - acc[v] / D[p];
        }
        if (c.type[p] == 0) project_out_normal(c, p, out);
        for (int v = 0; v < 4; ++v) dU[v * c.n + p] = out[v];
    };
    // the points of one colour share no edge: they are swept in parallel
    auto sweep_colour = [&](int col, bool forward, int g) {
        const std::vector<int64_t>& pts = by_colour[col];
        const int64_t m = (int64_t)pts.size();
#pragma omp parallel for
        for (int64_t j = 0; j < m; ++j)
            if (g < 0 || c.type[pts[j]] == g) sweep_point(pts[j], forward);
    };
    if (P.order == 0) {
        for (int col = 0; col < c.ncolour; ++col) sweep_colour(col, true, -1);
        for (int col = c.ncolour - 1; col >= 0; --col) sweep_colour(col, false, -1);
        return;
    }
    // Algorithm 5: the same per-point sweeps, grouped into wall, interior and
    // outer points; each sweep visits the groups in that order, the colours
    // ascending (forward) or descending (backward) within a group.  A point
    // still sums over its lower- (upper-) colour neighbours and reads whatever
    // the shared increment array holds for them at that moment.
    const int8_t groups[3] = {0, 1, 2};
    for (int8_t g : groups)
        for (int col = 0; col < c.ncolour; ++col) sweep_colour(col, true, g);
    for (int8_t g : groups)
        for (int col = c.ncolour - 1; col >= 0; --col) sweep_colour(col, false, g);
}

// state_update(): U <- U + dU (Section 3, definition of dU).
int state_update(const Cloud& c, const Params& P, double* U, const double* dU) {
    int st = OK;
#pragma omp parallel for reduction(min : st)
    for (int64_t p = 0; p < c.n; ++p) {
        for (int v = 0; v < 4; ++v) U[v * c.n + p] += dU[v * c.n + p];
        double Up[4] = {U[p], U[c.n + p], U[2 * c.n + p], U[3 * c.n + p]};
        Prim<double> w = prim_from_U(Up, P.gamma);
        if (!(w.rho > 0.0) || !(w.p > 0.0)) st = ERR_NONPHYS;
    }
    return st;
}

// Reading: res = sqrt(sum over non-outer points of R_rho^2) / (number of
// non-outer points) -- the paper reports a "density residual".
double residual_norm(const Cloud& c, const double* R) {
    double s = 0.0;
    int64_t na = 0;
    for (int64_t p = 0; p < c.n; ++p) {
        if (c.type[p] == 2) continue;
        s += R[p] * R[p];
        ++na;
    }
    return na ? std::sqrt(s) / (double)na : 0.0;
}

}  // namespace

// ===========================================================================
// C ABI (host pointers only).  Arrays of point fields are SoA [4][n].
// ===========================================================================
extern "C" {

typedef struct {
    int64_t n;
    const double *x, *y, *tx, *ty;
    const int8_t* type;
    const int32_t *off, *idx;
    const int32_t* colour;
    int32_t ncolour;
} ora_cloud;

typedef struct {
    double gamma, cfl, mach, aoa_deg;
    int32_t inner_iters, jvp_mode;
    int32_t limiter, variant;
    double limiter_k;
    int32_t order, farfield;
} ora_params;

static Cloud to_cloud(const ora_cloud* c) {
    return Cloud{c->n, c->x, c->y, c->tx, c->ty, c->type, c->off, c->idx, c->colour, c->ncolour};
}
static Params to_params(const ora_params* p) {
    return Params{p->gamma,    p->cfl,     p->mach,      p->aoa_deg, p->inner_iters,
                  p->jvp_mode, p->limiter, p->limiter_k, p->variant, p->order,
                  p->farfield};
}

// Point colouring, Algorithm 4: colour(first point) = first colour; then for
// every point i in storage order and every neighbour p of i in CSR order, an
// uncoloured p takes the smallest colour not used by its own neighbours.
// Reading: a point never reached this way (isolated) takes the smallest
// colour absent from its neighbours, in storage order afterwards.
// Returns the number of colours (colours are 0-based), or < 0 on error.
int32_t ora_colour(int64_t n, const int32_t* off, const int32_t* idx, int32_t* colour) {
    if (n <= 0) return 0;
    for (int64_t i = 0; i < n; ++i) colour[i] = -1;
    auto smallest_free = [&](int64_t p) {
        std::vector<char> used;
        for (int32_t e = off[p]; e < off[p + 1]; ++e) {
            int32_t c = colour[idx[e]];
            if (c >= 0) {
                if ((size_t)c >= used.size()) used.resize(c + 1, 0);
                used[c] = 1;
            }
        }
        int32_t k = 0;
        while ((size_t)k < used.size() && used[k]) ++k;
        return k;
    };
    colour[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            int32_t p = idx[e];
            if (colour[p] < 0) colour[p] = smallest_free(p);
        }
    for (int64_t i = 0; i < n; ++i)
        if (colour[i] < 0) colour[i] = smallest_free(i);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i)
        if (colour[i] + 1 > nc) nc = colour[i] + 1;
    return nc;
}

// Number of OpenMP threads of the oracle's loops (n >= 1), and the current one.
void ora_set_threads(int32_t n) {
    if (n >= 1) omp_set_num_threads(n);
}
int32_t ora_threads(void) { return (int32_t)omp_get_max_threads(); }

void ora_split_flux(const double* U, double dx, double dy, int32_t s, double gamma, double* G) {
    split_flux(prim_from_U(U, gamma), dx, dy, s, gamma, G);
}

void ora_flux_jvp(const double* U, const double* dU, double dx, double dy, int32_t s,
                  const ora_params* prm, double* J) {
    Split k{dx, dy, -dy, dx, s};
    flux_jvp(U, dU, k, to_params(prm), J);
}

void ora_q_from_U(int64_t n, const double* U, double gamma, double* q) {
    for (int64_t p = 0; p < n; ++p) {
        double Up[4] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]};
        double qp[4];
        q_from_prim(prim_from_U(Up, gamma), gamma, qp);
        for (int v = 0; v < 4; ++v) q[v * n + p] = qp[v];
    }
}

void ora_U_from_q(int64_t n, const double* q, double gamma, double* U) {
    for (int64_t p = 0; p < n; ++p) {
        double qp[4] = {q[p], q[n + p], q[2 * n + p], q[3 * n + p]};
        double Up[4];
        U_from_prim(prim_from_q(qp, gamma), gamma, Up);
        for (int v = 0; v < 4; ++v) U[v * n + p] = Up[v];
    }
}

// Split stencil of point p (split index k in the point's own order: wall
// t+, t-, n-; interior x+, x-, y+, y-; with farfield != 0, outer t+, t-, n+).  Writes up to cap members and weights;
// returns the member count (0 for degenerate), or -1 if k is not a split.
int32_t ora_split_weights(const ora_cloud* oc, int64_t p, int32_t k, int32_t cap, int32_t* nb,
                          double* w, double* ls1, int32_t farfield) {
    Cloud c = to_cloud(oc);
    Split sp[4];
    int ns = splits_of(c, p, sp, farfield != 0);
    if (k < 0 || k >= ns) return -1;
    Stencil st = split_stencil(c, p, sp[k]);
    *ls1 = st.ls1;
    int32_t m = (int32_t)st.nb.size();
    for (int32_t j = 0; j < m && j < cap; ++j) {
        nb[j] = st.nb[j];
        w[j] = st.w[j];
    }
    return m;
}

// Split directions of point p: writes (dx, dy, s) triples, returns the count.
int32_t ora_split_dirs(const ora_cloud* oc, int64_t p, double* out, int32_t farfield) {
    Cloud c = to_cloud(oc);
    Split sp[4];
    int ns = splits_of(c, p, sp, farfield != 0);
    for (int k = 0; k < ns; ++k) {
        out[3 * k] = sp[k].dx;
        out[3 * k + 1] = sp[k].dy;
        out[3 * k + 2] = sp[k].s;
    }
    return ns;
}

void ora_free_stream(const ora_cloud* oc, const ora_params* prm, double* U) {
    free_stream(to_cloud(oc), to_params(prm), U);
}

int32_t ora_q_grad_pass(const ora_cloud* oc, const double* q, const double* qx_in,
                        const double* qy_in, double* qx_out, double* qy_out) {
    return q_grad_pass(to_cloud(oc), q, qx_in, qy_in, qx_out, qy_out);
}

int32_t ora_q_derivatives(const ora_cloud* oc, const ora_params* prm, const double* q, double* qx,
                          double* qy) {
    return q_derivatives(to_cloud(oc), to_params(prm), q, qx, qy);
}

// Residual of state U: q_variables, q_derivatives, flux_residual.
int32_t ora_residual(const ora_cloud* oc, const ora_params* prm, const double* U, double* R,
                     double* res, int64_t* degenerate) {
    Cloud c = to_cloud(oc);
    Params P = to_params(prm);
    std::vector<double> q(4 * c.n), qx(4 * c.n), qy(4 * c.n);
    int st = q_variables(c, P, U, q.data());
    if (st) return st;
    st = q_derivatives(c, P, q.data(), qx.data(), qy.data());
    if (st) return st;
    if (P.limiter) limit_gradients(c, P, q.data(), qx.data(), qy.data());
    st = flux_residual(c, P, q.data(), qx.data(), qy.data(), R, degenerate);
    if (res) *res = residual_norm(c, R);
    return st;
}

// Limited gradients (Venkatakrishnan) of given q, q_x, q_y, in place.
void ora_limit_gradients(const ora_cloud* oc, const ora_params* prm, const double* q, double* qx,
                         double* qy) {
    limit_gradients(to_cloud(oc), to_params(prm), q, qx, qy);
}

// Residual from given q, q_x, q_y (flux_residual alone).
int32_t ora_flux_residual(const ora_cloud* oc, const ora_params* prm, const double* q,
                          const double* qx, const double* qy, double* R) {
    return flux_residual(to_cloud(oc), to_params(prm), q, qx, qy, R, nullptr);
}

void ora_timestep_diag(const ora_cloud* oc, const ora_params* prm, const double* U, double* dt,
                       double* D) {
    timestep_diag(to_cloud(oc), to_params(prm), U, dt, D);
}

void ora_lusgs(const ora_cloud* oc, const ora_params* prm, const double* U, const double* R,
               const double* D, double* dU) {
    lusgs(to_cloud(oc), to_params(prm), U, R, D, dU);
}

double ora_residual_norm(const ora_cloud* oc, const double* R) {
    return residual_norm(to_cloud(oc), R);
}

void ora_unsplit_jvp(const double* U, const double* dU, double dx, double dy,
                     const ora_params* prm, double* J) {
    unsplit_jvp(U, dU, dx, dy, to_params(prm), J);
}

void ora_manish_source(const ora_cloud* oc, const ora_params* prm, const double* U,
                       const double* dU_prev, double* S) {
    manish_source(to_cloud(oc), to_params(prm), U, dU_prev, S);
}

// One implicit iteration (body of Algorithm 1): q_variables, q_derivatives,
// flux_residual, LUSGS, state_update.  U is updated in place; R (optional)
// receives this iteration's residual and *res its norm.  dU_io (optional): on
// entry the previous iteration's increment (read by the Manish variant's S;
// NULL = zero), on exit this iteration's increment.  Returns 0, or
// ERR_NONPHYS (-5) / ERR_DEGEN (-3).
int32_t ora_iteration(const ora_cloud* oc, const ora_params* prm, double* U, double* R_out,
                      double* dU_io, double* res) {
    Cloud c = to_cloud(oc);
    Params P = to_params(prm);
    std::vector<double> R(4 * c.n), dU(4 * c.n), dt(c.n), D(c.n);
    int st = ora_residual(oc, prm, U, R.data(), res, nullptr);
    if (st) return st;
    timestep_diag(c, P, U, dt.data(), D.data());
    std::vector<double> rhs(R);
    if (P.variant == 1) {
        // forward-sweep right-hand side R - S (eq. 38)
        std::vector<double> S(4 * c.n);
        manish_source(c, P, U, dU_io, S.data());
        for (int64_t i = 0; i < 4 * c.n; ++i) rhs[i] = R[i] - S[i];
    }
    lusgs(c, P, U, rhs.data(), D.data(), dU.data());
    st = state_update(c, P, U, dU.data());
    if (R_out) std::memcpy(R_out, R.data(), sizeof(double) * 4 * c.n);
    if (dU_io) std::memcpy(dU_io, dU.data(), sizeof(double) * 4 * c.n);
    return st;
}

// One explicit iteration (the paper's explicit LSKUM solver, Section 5): the
// semi-discrete equation dU/dt = -R (eq. 19 without the implicit operator) with
// the first-order forward difference in time, U <- U - dt R, dt the same local
// time step as the implicit scheme (the CFL number is the caller's).  Outer
// points keep the free stream (R = 0); wall points keep tangency (R has no
// normal-momentum component).  Returns 0, ERR_NONPHYS or ERR_DEGEN.
int32_t ora_explicit_iteration(const ora_cloud* oc, const ora_params* prm, double* U,
                               double* R_out, double* res) {
    Cloud c = to_cloud(oc);
    Params P = to_params(prm);
    std::vector<double> R(4 * c.n), dt(c.n), D(c.n);
    int st = ora_residual(oc, prm, U, R.data(), res, nullptr);
    if (st) return st;
    timestep_diag(c, P, U, dt.data(), D.data());
    std::vector<double> dU(4 * c.n);
#pragma omp parallel for
    for (int64_t p = 0; p < c.n; ++p)
        for (int v = 0; v < 4; ++v) dU[v * c.n + p] = -dt[p] * R[v * c.n + p];
    st = state_update(c, P, U, dU.data());
    if (R_out) std::memcpy(R_out, R.data(), sizeof(double) * 4 * c.n);
    return st;
}

// Runs up to max_iters iterations from U, stopping when res <= tol_abs.
// history (optional, max_iters entries) receives res per iteration.
// Returns the number of iterations run, or a negative status.
int32_t ora_solve(const ora_cloud* oc, const ora_params* prm, double* U, int32_t max_iters,
                  double tol_abs, double* history) {
    std::vector<double> dU(4 * oc->n, 0.0);  // increment carried between iterations
    for (int32_t it = 0; it < max_iters; ++it) {
        double res = 0.0;
        int32_t st = ora_iteration(oc, prm, U, nullptr, dU.data(), &res);
        if (history) history[it] = res;
        if (st) return st;
        if (res <= tol_abs) return it + 1;
    }
    return max_iters;
}

// Lift and drag coefficients (reading; the paper reports CL/CD without the
// rule).  Wall points, in storage order, form one closed polygon; on each
// edge the pressure is the mean of its end points and the force is
// -(p_mid - p_inf) |e| n_out, n_out the edge normal pointing out of the body.
// CL = (Fy cos a - Fx sin a)/q_inf, CD = (Fx cos a + Fy sin a)/q_inf with
// q_inf = rho_inf |V_inf|^2 / 2 and unit chord.
int32_t ora_forces(const ora_cloud* oc, const ora_params* prm, const double* U, double* cl,
                   double* cd) {
    Cloud c = to_cloud(oc);
    std::vector<int64_t> wall;
    for (int64_t p = 0; p < c.n; ++p)
        if (c.type[p] == 0) wall.push_back(p);
    size_t m = wall.size();
    if (m < 3) return ERR_ARG;
    double area2 = 0.0;
    for (size_t j = 0; j < m; ++j) {
        int64_t a = wall[j], b = wall[(j + 1) % m];
        area2 += c.x[a] * c.y[b] - c.x[b] * c.y[a];
    }
    double orient = area2 > 0.0 ? 1.0 : -1.0;  // +1 counter-clockwise
    double pinf = 1.0 / prm->gamma;
    double fx = 0.0, fy = 0.0;
    for (size_t j = 0; j < m; ++j) {
        int64_t a = wall[j], b = wall[(j + 1) % m];
        double Ua[4] = {U[a], U[c.n + a], U[2 * c.n + a], U[3 * c.n + a]};
        double Ub[4] = {U[b], U[c.n + b], U[2 * c.n + b], U[3 * c.n + b]};
        double pa = prim_from_U(Ua, prm->gamma).p, pb = prim_from_U(Ub, prm->gamma).p;
        double pm = 0.5 * (pa + pb) - pinf;
        double ex = c.x[b] - c.x[a], ey = c.y[b] - c.y[a];
        // outward normal times length: right normal for a counter-clockwise polygon
        double nx = orient * ey, ny = -orient * ex;
        fx -= pm * nx;
        fy -= pm * ny;
    }
    double al = prm->aoa_deg * kPi / 180.0;
    double qinf = 0.5 * prm->mach * prm->mach;
    *cl = (fy * std::cos(al) - fx * std::sin(al)) / qinf;
    *cd = (fx * std::cos(al) + fy * std::sin(al)) / qinf;
    return OK;
}

}  // extern "C"
