// Device kernels of the MI355X implicit LSKUM solver (gfx950, wave64).
//
// One iteration (Section 4, Algorithm 3, with the colour sweeps of
// Algorithms 6-7):
//   k_qgrad<...>   x (1 + m)        q-derivatives, eq. (16): first-order pass and
//                                   m inner passes; the optional limiter is
//                                   applied in the last pass
//   k_residual<...>                 LSKUM residual eq. (11), (15); local time
//                                   step and scalar diagonal eq. (25), (34)-(35);
//                                   per-point linearisation data for the sweeps
//   k_norm_partial, k_norm_comp     density residual norm per component and the
//                                   convergence test
//   k_sweep<...>   x C colours      forward sweep, eq. (27) first line
//   k_sweep<...>   x C colours      backward sweep, eq. (27) second line
//   k_update                        U += dU and the q-variables of eq. (14)
//
// Mapping: LANES consecutive lanes share a point and split its neighbour
// loop, combining partial sums with cross-lane shuffles in a fixed order;
// points of a block are contiguous (storage order, or colour order in the
// sweeps); block ids are remapped so that consecutive point ranges stay on one
// XCD (each XCD has its own L2).  All per-point sums run in CSR neighbour
// order.  The per-point 4x4 algebra is not a dense contraction, so no matrix
// cores are used.
#include "lskum_internal.h"
#include "lskum_math.h"

#include <cmath>

namespace lskum {

namespace {

constexpr int kBlock = 256;
constexpr double kInvSqrtPi = 0.56418958354775628694807945156077;
constexpr int8_t kWall = 0, kInterior = 1, kOuter = 2;

// Frame points (wall, and outer points under the kinetic far field) split
// their stencil along the tangent t and the normal n = (-t_y, t_x): t+, t-
// and one normal half -- the fluid side (dn > 0, the n- split) at a wall, the
// inner side (dn < 0, the n+ split) at an outer point, whose normal points
// out of the domain.
__device__ __forceinline__ bool in_normal_split(int8_t ty, double dn) {
    return ty == kWall ? dn > 0.0 : dn < 0.0;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Give XCD x the
// contiguous range of logical blocks [x*per + min(x, rem), ...) so that
// neighbouring point ranges share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, r = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + r;
}

// A point takes part in an iteration while its component is active.
__device__ __forceinline__ bool live(const int32_t* __restrict__ comp,
                                     const int32_t* __restrict__ active, int64_t p) {
    return active[comp ? comp[p] : 0] != 0;
}

// Projections onto a wall frame, evaluated without contraction so that split
// membership (the sign of da) is decided exactly as a plain multiply-add would.
__device__ __forceinline__ double dot_nc(double ax, double ay, double bx, double by) {
#pragma clang fp contract(off)
    double r = ax * bx;
    double s = ay * by;
    return r + s;
}

struct Prim {
    double rho, u1, u2, p, sb, isb, rhoE;  // sb = sqrt(beta), isb = 1/sqrt(beta)
};

// Primitive state of a (reconstructed) q vector, eq. (14) inverted:
// beta = -q4/2, u = (q2, q3)/(2 beta), rho = exp(q1 + beta |u|^2) beta^(-1/(gamma-1)),
// p = rho/(2 beta).  Division free: with r = 1/sqrt(beta), 1/(2 beta) = r^2/2 and,
// for gamma = 1.4, beta^(-5/2) = r^5.
__device__ __forceinline__ Prim prim_from_q(const D4& q, double inv_gm1, bool g14) {
    Prim w;
    const double beta = -0.5 * q.w;
    const double r = rsqrt(beta);
    const double i2b = 0.5 * r * r;
    w.u1 = q.y * i2b;
    w.u2 = q.z * i2b;
    const double usq = w.u1 * w.u1 + w.u2 * w.u2;
    const double e = exp_fast(q.x + beta * usq);
    const double r2 = r * r;
    w.rho = g14 ? e * (r2 * r2 * r) : e * exp(-inv_gm1 * log(beta));
    w.p = w.rho * i2b;
    w.sb = beta * r;
    w.isb = r;
    w.rhoE = w.p * inv_gm1 + 0.5 * w.rho * usq;
    return w;
}

// Kinetic split flux G_d^sg of a primitive state (half-range moments of the
// Maxwellian, eq. 3-6): DIR 0 = x, 1 = y, 2 = unit direction (dx, dy).
template <int DIR>
__device__ __forceinline__ void split_flux(const Prim& w, double dx, double dy, double sg,
                                           double inv_gm1, double G[4]) {
    (void)inv_gm1;
    const double ud = DIR == 0 ? w.u1 : (DIR == 1 ? w.u2 : w.u1 * dx + w.u2 * dy);
    const double S = ud * w.sb;
    const double A = 0.5 * (1.0 + sg * erf_fast(S));
    const double B = exp_fast(-(S * S)) * (0.5 * kInvSqrtPi) * w.isb;
    const double mass = w.rho * (ud * A + sg * B);
    const double pA = w.p * A;
    G[0] = mass;
    if (DIR == 0) {
        G[1] = pA + w.u1 * mass;
        G[2] = w.u2 * mass;
    } else if (DIR == 1) {
        G[1] = w.u1 * mass;
        G[2] = pA + w.u2 * mass;
    } else {
        G[1] = pA * dx + w.u1 * mass;
        G[2] = pA * dy + w.u2 * mass;
    }
    G[3] = (w.rhoE + w.p) * ud * A + sg * (w.rhoE + 0.5 * w.p) * B;
}

template <int DIR>
__device__ __forceinline__ void acc_split_diff(const Prim& wi, const Prim& w0, double dx, double dy,
                                               double sg, double wgt, double inv_gm1, double R[4]) {
    double Gi[4], G0[4];
    split_flux<DIR>(wi, dx, dy, sg, inv_gm1, Gi);
    split_flux<DIR>(w0, dx, dy, sg, inv_gm1, G0);
#pragma unroll
    for (int v = 0; v < 4; ++v) R[v] += wgt * (Gi[v] - G0[v]);
}

// ---------------------------------------------------------------------------
// Geometry precompute (once per cloud).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_precompute(int64_t n, const D2* __restrict__ xy,
                                                       const D2* __restrict__ frame,
                                                       const int8_t* __restrict__ type,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ idx,
                                                       PointGeom* __restrict__ geom,
                                                       unsigned long long* __restrict__ counts) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const D2 r0 = xy[p];
    const int8_t ty = type[p];
    const D2 t = frame[p];
    double sxx = 0, syy = 0, sxy = 0, rmin2 = INFINITY;
    // split sums: a = split direction, b = transverse
    double saa[4] = {0, 0, 0, 0}, sbb[4] = {0, 0, 0, 0}, sab[4] = {0, 0, 0, 0};
    int cnt[4] = {0, 0, 0, 0};
    const int32_t e0 = off[p], e1 = off[p + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const D2 ri = xy[idx[e]];
        const double dx = ri.x - r0.x, dy = ri.y - r0.y;
        sxx += dx * dx;
        syy += dy * dy;
        sxy += dx * dy;
        const double d2 = dx * dx + dy * dy;
        rmin2 = d2 < rmin2 ? d2 : rmin2;
        if (ty != kInterior) {
            const double ds = dot_nc(dx, dy, t.x, t.y);
            const double dn = dot_nc(dx, dy, -t.y, t.x);
            if (ds != 0.0) {
                const int k = ds < 0.0 ? 0 : 1;
                saa[k] += ds * ds; sbb[k] += dn * dn; sab[k] += ds * dn; ++cnt[k];
            }
            if (in_normal_split(ty, dn)) {
                saa[2] += dn * dn; sbb[2] += ds * ds; sab[2] += ds * dn; ++cnt[2];
            }
        } else {
            if (dx != 0.0) {
                const int k = dx < 0.0 ? 0 : 1;
                saa[k] += dx * dx; sbb[k] += dy * dy; sab[k] += dx * dy; ++cnt[k];
            }
            if (dy != 0.0) {
                const int k = dy < 0.0 ? 2 : 3;
                saa[k] += dy * dy; sbb[k] += dx * dx; sab[k] += dx * dy; ++cnt[k];
            }
        }
    }
    PointGeom g;
    const double det = sxx * syy - sxy * sxy;
    if (!(det > 1e-12 * sxx * syy)) {
        atomicAdd(&counts[0], 1ull);  // singular full stencil
        g.lsq = {0, 0, 0, sqrt(rmin2)};
    } else {
        g.lsq = {syy / det, -sxy / det, sxx / det, sqrt(rmin2)};
    }
    const int nsplit = ty == kInterior ? 4 : 3;
    double cb[4] = {0, 0, 0, 0}, cab[4] = {0, 0, 0, 0};
    for (int k = 0; k < nsplit; ++k) {
        const double dk = saa[k] * sbb[k] - sab[k] * sab[k];
        if (cnt[k] < 2 || !(dk > 1e-12 * saa[k] * sbb[k])) {
            // degenerate half stencil: contributes 0 (counted for the points
            // that always take part; outer splits only with the far field)
            if (ty != kOuter) atomicAdd(&counts[1], 1ull);
            continue;
        }
        cb[k] = sbb[k] / dk;
        cab[k] = -sab[k] / dk;
    }
    // LS_k(1): the weight sums, with the weights exactly as the kernels form them
    double ls1[4] = {0, 0, 0, 0};
    {
        for (int32_t e = e0; e < e1; ++e) {
            const D2 ri = xy[idx[e]];
            const double dx = ri.x - r0.x, dy = ri.y - r0.y;
            if (ty != kInterior) {
                const double ds = dot_nc(dx, dy, t.x, t.y);
                const double dn = dot_nc(dx, dy, -t.y, t.x);
                if (ds != 0.0) {
                    const int k = ds < 0.0 ? 0 : 1;
                    ls1[k] += cb[k] * ds + cab[k] * dn;
                }
                if (in_normal_split(ty, dn)) ls1[2] += cb[2] * dn + cab[2] * ds;
            } else {
                if (dx != 0.0) {
                    const int k = dx < 0.0 ? 0 : 1;
                    ls1[k] += cb[k] * dx + cab[k] * dy;
                }
                if (dy != 0.0) {
                    const int k = dy < 0.0 ? 2 : 3;
                    ls1[k] += cb[k] * dy + cab[k] * dx;
                }
            }
        }
    }
    for (int k = 0; k < 4; ++k) g.split[k] = {cb[k], cab[k]};
    g.ls1 = {ls1[0], ls1[1], ls1[2], ls1[3]};
    geom[p] = g;
}

// Free stream: rho 1, p 1/gamma, velocity M (cos a, sin a); wall points keep
// the tangential velocity only.
__global__ void __launch_bounds__(kBlock) k_free_stream(int64_t n, const int8_t* __restrict__ type,
                                                        const D2* __restrict__ frame, double gamma,
                                                        const int32_t* __restrict__ comp,
                                                        const double* __restrict__ vinf,
                                                        D4* __restrict__ U) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int k = comp ? comp[p] : 0;
    double u1 = vinf[2 * k], u2 = vinf[2 * k + 1];
    if (type[p] == kWall) {
        const D2 t = frame[p];
        const double ut = u1 * t.x + u2 * t.y;
        u1 = ut * t.x;
        u2 = ut * t.y;
    }
    const double rho = 1.0, pr = 1.0 / gamma;
    U[p] = {rho, rho * u1, rho * u2, pr / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2)};
}

// q-variables of eq. (14) from U.
__device__ __forceinline__ D4 q_of_U(const D4& u, double gamma, double inv_gm1, bool& bad) {
    const double rho = u.x;
    const double irho = 1.0 / rho;
    const double u1 = u.y * irho, u2 = u.z * irho;
    const double usq = u1 * u1 + u2 * u2;
    const double p = (gamma - 1.0) * (u.w - 0.5 * rho * usq);
    bad = !(rho > 0.0) || !(p > 0.0);
    const double beta = 0.5 * rho / p;
    return {log(rho) + inv_gm1 * log(beta) - beta * usq, 2.0 * beta * u1, 2.0 * beta * u2,
            -2.0 * beta};
}

__global__ void __launch_bounds__(kBlock) k_q_from_U(int64_t n, double gamma,
                                                     const D4* __restrict__ U, D4* __restrict__ q,
                                                     int32_t* __restrict__ flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    bool bad;
    q[p] = q_of_U(U[p], gamma, 1.0 / (gamma - 1.0), bad);
    if (bad) flags[0] = 1;
}

// ---------------------------------------------------------------------------
// q-derivatives (eq. 16): first-order pass and Jacobi inner passes, with the
// optional limiter fused into the last pass.
//
// Venkatakrishnan's limiter on the q~ reconstruction (an addition: the paper
// names no limiter).  Per point and component, phi = min over neighbours of
//   (d1^2 + eps^2 + 2 d1 d2) / (d1^2 + 2 d2^2 + d1 d2 + eps^2),
// d2 = -(dx qx + dy qy)/2 the reconstruction increment toward the neighbour,
// d1 the largest (d2 > 0) or smallest (d2 < 0) neighbour difference,
// eps^2 = (K h)^3 with h the nearest-neighbour distance, and phi <= 1.
// With A = d1^2 + eps^2 and d1 d2 >= 0 the ratio is >= 1 for |d2| <= |d1|/2
// and falls with |d2| beyond (its derivative in d2 > 0 has the sign of
// d1 A - 4 A d2 - 4 d1 d2^2 <= 0 there; d2 < 0 is the mirror image), so
// min(1, ratio) is non-increasing in |d2| on each side: the minimum over the
// neighbours is the ratio at the largest positive and the most negative d2.
// The walk therefore only keeps the extremes of dx qx + dy qy, and the ratio
// is formed twice per component.  The limited derivatives phi * (qx, qy) go
// to qxl, qyl; the unlimited ones of that pass to qx_out, qy_out only when
// those are given (a query of the derivatives: the residual reads qxl, qyl).
//
// LANES consecutive lanes share one point and split its neighbours; the LS
// right-hand sides, the neighbour extrema and the limiter minimum are
// combined with cross-lane shuffles.
// ---------------------------------------------------------------------------
template <int LANES>
__device__ __forceinline__ double lane_sum(double v) {
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The limiter factor of one component from the walk's extremes tlo <= 0 <=
// thi of dx qx + dy qy (d2 = -t/2): the ratio at d2 = -tlo/2 with d1 = dmax
// and at d2 = -thi/2 with d1 = dmin, and 1.
__device__ __forceinline__ double venkat_phi(double tlo, double thi, double dmax, double dmin,
                                             double eps2) {
    double phi = 1.0;
    if (tlo < 0.0) {
        const double d2 = -0.5 * tlo, d1 = dmax;
        const double nu = d1 * d1 + eps2 + 2.0 * d1 * d2;
        const double de = d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2;
        phi = fmin(phi, nu / de);
    }
    if (thi > 0.0) {
        const double d2 = -0.5 * thi, d1 = dmin;
        const double nu = d1 * d1 + eps2 + 2.0 * d1 * d2;
        const double de = d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2;
        phi = fmin(phi, nu / de);
    }
    return fmax(phi, 0.0);
}

// Neighbour data of the q-derivative sums: position, q and (defect
// correction passes) the current derivatives.
struct QNbr {
    D2 r;
    D4 q, gx, gy;
};

template <bool INNER>
__device__ __forceinline__ QNbr load_qnbr(int32_t i, const D2* __restrict__ xy,
                                          const D4* __restrict__ q, const D4* __restrict__ qx,
                                          const D4* __restrict__ qy) {
    QNbr nb{xy[i], q[i], {}, {}};
    if (INNER) {
        nb.gx = qx[i];
        nb.gy = qy[i];
    }
    return nb;
}

constexpr int kDxyCache = 8;  // limiter: LDS slots per thread for neighbour offsets

// Four workgroups per CU: the limited pass fits 128 VGPRs (four wavefronts
// per SIMD), which measured faster than three wavefronts without the bound.
template <bool INNER, bool LIMIT, int LANES>
__global__ void __launch_bounds__(kBlock, 4) k_qgrad(
    int64_t n, double K, const D2* __restrict__ xy, const int32_t* __restrict__ off,
    const int32_t* __restrict__ idx, const PointGeom* __restrict__ geom,
    const int32_t* __restrict__ comp, const int32_t* __restrict__ active,
    const D4* __restrict__ q, const D4* __restrict__ qx_in, const D4* __restrict__ qy_in,
    D4* __restrict__ qx_out, D4* __restrict__ qy_out, D4* __restrict__ qxl,
    D4* __restrict__ qyl) {
    const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t p = gt / LANES;
    const int lane = (int)(gt % LANES);
    if (p >= n || !live(comp, active, p)) return;  // uniform over the lanes of a point
    const D2 r0 = xy[p];
    const D4 q0 = q[p];
    const double qv[4] = {q0.x, q0.y, q0.z, q0.w};
    D4 gx0{}, gy0{};
    if (INNER) {
        gx0 = qx_in[p];
        gy0 = qy_in[p];
    }
    double bx[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0};
    double dmax[4] = {0, 0, 0, 0}, dmin[4] = {0, 0, 0, 0};
    // both neighbour walks are software-pipelined: indices two entries ahead,
    // neighbour data one entry ahead of the one being used; past the end the
    // last entry is re-read (in bounds) and not used
    // with the limiter, a lane keeps the offsets of its first kDxyCache
    // entries in LDS for the second walk
    __shared__ D2 dxy_cache[LIMIT ? kDxyCache * kBlock : 1];
    const int32_t e0 = off[p], e1 = off[p + 1], last = e1 - 1;
    if (e0 + lane < e1) {
        int32_t e = e0 + lane;
        int32_t i_next = idx[min(e + LANES, last)];
        QNbr cur = load_qnbr<INNER>(idx[e], xy, q, qx_in, qy_in);
        for (int k = 0; e < e1; e += LANES, ++k) {
            const int32_t i_after = idx[min(e + 2 * LANES, last)];
            const QNbr nxt = load_qnbr<INNER>(i_next, xy, q, qx_in, qy_in);
            const double dx = cur.r.x - r0.x, dy = cur.r.y - r0.y;
            if (LIMIT && k < kDxyCache) dxy_cache[k * kBlock + threadIdx.x] = {dx, dy};
            const D4 qi = cur.q;
            double dq[4] = {qi.x - qv[0], qi.y - qv[1], qi.z - qv[2], qi.w - qv[3]};
            if (LIMIT) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dmax[v] = fmax(dmax[v], dq[v]);
                    dmin[v] = fmin(dmin[v], dq[v]);
                }
            }
            if (INNER) {
                const D4 gxi = cur.gx, gyi = cur.gy;
                dq[0] -= 0.5 * (dx * (gxi.x - gx0.x) + dy * (gyi.x - gy0.x));
                dq[1] -= 0.5 * (dx * (gxi.y - gx0.y) + dy * (gyi.y - gy0.y));
                dq[2] -= 0.5 * (dx * (gxi.z - gx0.z) + dy * (gyi.z - gy0.z));
                dq[3] -= 0.5 * (dx * (gxi.w - gx0.w) + dy * (gyi.w - gy0.w));
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                bx[v] += dx * dq[v];
                by[v] += dy * dq[v];
            }
            cur = nxt;
            i_next = i_after;
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bx[v] = lane_sum<LANES>(bx[v]);
        by[v] = lane_sum<LANES>(by[v]);
    }
    const PointGeom& G = geom[p];
    const D4 L = G.lsq;
    double gx[4], gy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        gx[v] = L.x * bx[v] + L.y * by[v];
        gy[v] = L.y * bx[v] + L.z * by[v];
    }
    if (lane == 0 && (!LIMIT || qx_out)) {  // the limited pass writes them on request only
        qx_out[p] = {gx[0], gx[1], gx[2], gx[3]};
        qy_out[p] = {gy[0], gy[1], gy[2], gy[3]};
    }
    if (!LIMIT) return;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
            dmax[v] = fmax(dmax[v], __shfl_xor(dmax[v], o, 64));
            dmin[v] = fmin(dmin[v], __shfl_xor(dmin[v], o, 64));
        }
    const double kh = K * L.w;
    const double eps2 = kh * kh * kh;
    double tlo[4] = {0, 0, 0, 0}, thi[4] = {0, 0, 0, 0};  // extremes of dx qx + dy qy
    int k = 0;
    for (int32_t e = e0 + lane; e < e1; e += LANES, ++k) {
        double dx, dy;
        if (k < kDxyCache) {  // written by this thread in the first walk
            const D2 d = dxy_cache[k * kBlock + threadIdx.x];
            dx = d.x;
            dy = d.y;
        } else {
            const D2 ri = xy[idx[e]];
            dx = ri.x - r0.x;
            dy = ri.y - r0.y;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double t = dx * gx[v] + dy * gy[v];
            tlo[v] = fmin(tlo[v], t);
            thi[v] = fmax(thi[v], t);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
            tlo[v] = fmin(tlo[v], __shfl_xor(tlo[v], o, 64));
            thi[v] = fmax(thi[v], __shfl_xor(thi[v], o, 64));
        }
    if (lane == 0) {
        double phi[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) phi[v] = venkat_phi(tlo[v], thi[v], dmax[v], dmin[v], eps2);
        qxl[p] = {phi[0] * gx[0], phi[1] * gx[1], phi[2] * gx[2], phi[3] * gx[3]};
        qyl[p] = {phi[0] * gy[0], phi[1] * gy[1], phi[2] * gy[2], phi[3] * gy[3]};
    }
}

// The same q-derivative pass with the neighbour gathers staged in LDS.  Tile
// b holds the points tile_pts[b kQTile ...] (-1 past its end: kQTile
// consecutive points, or a block of kQTileJ points by kQTileK rows of a cloud
// stored row by row); the host lists the union of their neighbours
// (tile_idx[tile_off[b] ...], sorted) and gives every CSR entry its
// neighbour's position in that list (lnbr).  The block
// first copies position, q (and the current derivatives) of the listed
// points into LDS -- runs of consecutive indices, so mostly coalesced --
// then every neighbour read of the sums comes from LDS: a point's 24
// neighbour records are shared with the tile's other points instead of being
// gathered 24 times from the caches.  Four lanes per point, each summing
// its neighbours in the order of k_qgrad<INNER, LIMIT, 4>; the compiler may
// contract the products differently, so the two forms can differ in the
// last bits.
static_assert(kQTile * 4 == kBlock, "a q-derivative tile is one point per four lanes");
constexpr int kLnPre = 8;  // list positions per lane held in registers (a whole stencil of <= 32)

template <bool INNER, bool LIMIT>
__global__ void __launch_bounds__(kBlock, 4) k_qgrad_tiled(
    double K, const D2* __restrict__ xy, const int32_t* __restrict__ off,
    const int32_t* __restrict__ tile_pts, const uint16_t* __restrict__ lnbr,
    const int32_t* __restrict__ tile_off,
    const int32_t* __restrict__ tile_idx, int32_t hmax, const PointGeom* __restrict__ geom,
    const int32_t* __restrict__ comp, const int32_t* __restrict__ active,
    const D4* __restrict__ q, const D4* __restrict__ qx_in, const D4* __restrict__ qy_in,
    D4* __restrict__ qx_out, D4* __restrict__ qy_out, D4* __restrict__ qxl,
    D4* __restrict__ qyl) {
    // one double array per field component (structure of arrays): the lanes
    // of a wave read consecutive list positions, so 8-byte reads fall in
    // distinct banks, where 32-byte records would put lanes four records
    // apart into the same bank
    extern __shared__ double smem[];
    double* s_x = smem;
    double* s_y = s_x + hmax;
    double* s_q = s_y + hmax;                  // 4 components
    double* s_g = s_q + 4 * hmax;              // 8 components (x then y derivatives)
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    // the point's own data and its first list positions are requested before
    // the staging, so their latency overlaps it
    const int64_t p = tile_pts[(int64_t)tile * kQTile + threadIdx.x / 4];
    const int lane = threadIdx.x % 4;
    const bool inb = p >= 0;
    D2 r0{};
    D4 q0{}, gx0{}, gy0{}, L{};
    int32_t e0 = 0, e1 = 0;
    if (inb) {
        r0 = xy[p];
        q0 = q[p];
        e0 = off[p];
        e1 = off[p + 1];
        L = geom[p].lsq;
        if (INNER) {
            gx0 = qx_in[p];
            gy0 = qy_in[p];
        }
    }
    int lpre[kLnPre];
#pragma unroll
    for (int k = 0; k < kLnPre; ++k) {
        const int32_t e = e0 + lane + 4 * k;
        lpre[k] = e < e1 ? lnbr[e] : 0;
    }
    const int32_t h0 = tile_off[tile], nh = tile_off[tile + 1] - h0;
    for (int32_t k = threadIdx.x; k < nh; k += kBlock) {
        const int32_t i = tile_idx[h0 + k];
        const D2 r = xy[i];
        const D4 qi = q[i];
        s_x[k] = r.x;
        s_y[k] = r.y;
        s_q[k] = qi.x;
        s_q[hmax + k] = qi.y;
        s_q[2 * hmax + k] = qi.z;
        s_q[3 * hmax + k] = qi.w;
        if (INNER) {
            const D4 gx = qx_in[i], gy = qy_in[i];
            s_g[k] = gx.x;
            s_g[hmax + k] = gx.y;
            s_g[2 * hmax + k] = gx.z;
            s_g[3 * hmax + k] = gx.w;
            s_g[4 * hmax + k] = gy.x;
            s_g[5 * hmax + k] = gy.y;
            s_g[6 * hmax + k] = gy.z;
            s_g[7 * hmax + k] = gy.w;
        }
    }
    __syncthreads();
    if (!inb || !live(comp, active, p)) return;  // uniform over the lanes of a point
    const double qv[4] = {q0.x, q0.y, q0.z, q0.w};
    double bx[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0};
    double dmax[4] = {0, 0, 0, 0}, dmin[4] = {0, 0, 0, 0};
    // a lane takes entries e0 + lane, e0 + lane + 4, ... in order: the first
    // kLnPre from registers, any further ones from memory
    auto first_walk = [&](int li) {
        const double dx = s_x[li] - r0.x, dy = s_y[li] - r0.y;
        const D4 qi = {s_q[li], s_q[hmax + li], s_q[2 * hmax + li], s_q[3 * hmax + li]};
        double dq[4] = {qi.x - qv[0], qi.y - qv[1], qi.z - qv[2], qi.w - qv[3]};
        if (LIMIT) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dmax[v] = fmax(dmax[v], dq[v]);
                dmin[v] = fmin(dmin[v], dq[v]);
            }
        }
        if (INNER) {
            const D4 gxi = {s_g[li], s_g[hmax + li], s_g[2 * hmax + li], s_g[3 * hmax + li]};
            const D4 gyi = {s_g[4 * hmax + li], s_g[5 * hmax + li], s_g[6 * hmax + li],
                            s_g[7 * hmax + li]};
            dq[0] -= 0.5 * (dx * (gxi.x - gx0.x) + dy * (gyi.x - gy0.x));
            dq[1] -= 0.5 * (dx * (gxi.y - gx0.y) + dy * (gyi.y - gy0.y));
            dq[2] -= 0.5 * (dx * (gxi.z - gx0.z) + dy * (gyi.z - gy0.z));
            dq[3] -= 0.5 * (dx * (gxi.w - gx0.w) + dy * (gyi.w - gy0.w));
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            bx[v] += dx * dq[v];
            by[v] += dy * dq[v];
        }
    };
#pragma unroll
    for (int k = 0; k < kLnPre; ++k)
        if (e0 + lane + 4 * k < e1) first_walk(lpre[k]);
    for (int32_t e = e0 + lane + 4 * kLnPre; e < e1; e += 4) first_walk(lnbr[e]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bx[v] = lane_sum<4>(bx[v]);
        by[v] = lane_sum<4>(by[v]);
    }
    double gx[4], gy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        gx[v] = L.x * bx[v] + L.y * by[v];
        gy[v] = L.y * bx[v] + L.z * by[v];
    }
    if (lane == 0 && (!LIMIT || qx_out)) {  // the limited pass writes them on request only
        qx_out[p] = {gx[0], gx[1], gx[2], gx[3]};
        qy_out[p] = {gy[0], gy[1], gy[2], gy[3]};
    }
    if (!LIMIT) return;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = 2; o > 0; o >>= 1) {
            dmax[v] = fmax(dmax[v], __shfl_xor(dmax[v], o, 64));
            dmin[v] = fmin(dmin[v], __shfl_xor(dmin[v], o, 64));
        }
    const double kh = K * L.w;
    const double eps2 = kh * kh * kh;
    double tlo[4] = {0, 0, 0, 0}, thi[4] = {0, 0, 0, 0};  // extremes of dx qx + dy qy
    auto second_walk = [&](int li) {
        const double dx = s_x[li] - r0.x, dy = s_y[li] - r0.y;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double t = dx * gx[v] + dy * gy[v];
            tlo[v] = fmin(tlo[v], t);
            thi[v] = fmax(thi[v], t);
        }
    };
#pragma unroll
    for (int k = 0; k < kLnPre; ++k)
        if (e0 + lane + 4 * k < e1) second_walk(lpre[k]);
    for (int32_t e = e0 + lane + 4 * kLnPre; e < e1; e += 4) second_walk(lnbr[e]);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = 2; o > 0; o >>= 1) {
            tlo[v] = fmin(tlo[v], __shfl_xor(tlo[v], o, 64));
            thi[v] = fmax(thi[v], __shfl_xor(thi[v], o, 64));
        }
    if (lane == 0) {
        double phi[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) phi[v] = venkat_phi(tlo[v], thi[v], dmax[v], dmin[v], eps2);
        qxl[p] = {phi[0] * gx[0], phi[1] * gx[1], phi[2] * gx[2], phi[3] * gx[3]};
        qyl[p] = {phi[0] * gy[0], phi[1] * gy[1], phi[2] * gy[2], phi[3] * gy[3]};
    }
}

// Unsplit Euler flux Jacobian product A_d(U) dU along unit direction d
// (eq. 2 differentiated by hand): with u_d' = ((dm . d) - u_d drho)/rho and
// p' = (gamma-1)(dE - u . dm + |u|^2 drho / 2),
//   (dm . d, dm u_d + m u_d' + p' d, (dE + p') u_d + (E + p) u_d');
// FD = true: the flux difference G_d(U + dU) - G_d(U) instead.
template <bool FD>
__device__ __forceinline__ void unsplit_jvp(const D4& u, const double dv[4], double dx, double dy,
                                            double gm1, double J[4]) {
    if (FD) {
        const double a0 = u.x + dv[0], a1 = u.y + dv[1], a2 = u.z + dv[2], a3 = u.w + dv[3];
        const double ua = (a1 * dx + a2 * dy) / a0, ub = (u.y * dx + u.z * dy) / u.x;
        const double pa = gm1 * (a3 - 0.5 * (a1 * a1 + a2 * a2) / a0);
        const double pb = gm1 * (u.w - 0.5 * (u.y * u.y + u.z * u.z) / u.x);
        J[0] = (a1 * dx + a2 * dy) - (u.y * dx + u.z * dy);
        J[1] = (a1 * ua + pa * dx) - (u.y * ub + pb * dx);
        J[2] = (a2 * ua + pa * dy) - (u.z * ub + pb * dy);
        J[3] = (a3 + pa) * ua - (u.w + pb) * ub;
        return;
    }
    const double irho = 1.0 / u.x, u1 = u.y * irho, u2 = u.z * irho;
    const double ud = u1 * dx + u2 * dy;
    const double p = gm1 * (u.w - 0.5 * u.x * (u1 * u1 + u2 * u2));
    const double dmd = dv[1] * dx + dv[2] * dy;
    const double udd = (dmd - ud * dv[0]) * irho;
    const double pd = gm1 * (dv[3] - (u1 * dv[1] + u2 * dv[2]) + 0.5 * (u1 * u1 + u2 * u2) * dv[0]);
    J[0] = dmd;
    J[1] = dv[1] * ud + u.y * udd + pd * dx;
    J[2] = dv[2] * ud + u.z * udd + pd * dy;
    J[3] = (dv[3] + pd) * ud + (u.w + p) * udd;
}

// Neighbour data of one stencil pair of the residual.
struct Nbr {
    D2 r;
    D4 q, gx, gy;
};

__device__ __forceinline__ Nbr load_nbr(int32_t i, const D2* __restrict__ xy,
                                        const D4* __restrict__ q, const D4* __restrict__ qx,
                                        const D4* __restrict__ qy) {
    return {xy[i], q[i], qx[i], qy[i]};
}

// One (point, neighbour) pair of the residual sum (eq. 11): the q~
// reconstructions at both ends (eq. 15), their primitive states and the split
// flux differences of every split the neighbour lies in (x+-/y+- at interior
// points, t+-/n- at a wall), weighted by the point's split coefficients.
__device__ __forceinline__ void residual_pair(int8_t ty, const D2& t, const D2& r0, const D4& q0,
                                              const D4& gx0, const D4& gy0, const D2& c0,
                                              const D2& c1, const D2& c2, const D2& c3,
                                              const Nbr& nb, double inv_gm1, bool g14,
                                              double Rp[4], int& bad) {
    const double dx = nb.r.x - r0.x, dy = nb.r.y - r0.y;
    const D4 qi = nb.q, gxi = nb.gx, gyi = nb.gy;
    const D4 qti = {qi.x - 0.5 * (dx * gxi.x + dy * gyi.x), qi.y - 0.5 * (dx * gxi.y + dy * gyi.y),
                    qi.z - 0.5 * (dx * gxi.z + dy * gyi.z), qi.w - 0.5 * (dx * gxi.w + dy * gyi.w)};
    const D4 qt0 = {q0.x - 0.5 * (dx * gx0.x + dy * gy0.x), q0.y - 0.5 * (dx * gx0.y + dy * gy0.y),
                    q0.z - 0.5 * (dx * gx0.z + dy * gy0.z), q0.w - 0.5 * (dx * gx0.w + dy * gy0.w)};
    if (ty != kInterior) {  // wall, or an outer point under the kinetic far field
        const double ds = dot_nc(dx, dy, t.x, t.y);
        const double dn = dot_nc(dx, dy, -t.y, t.x);
        const bool in_t = ds != 0.0, in_n = in_normal_split(ty, dn);
        if (!in_t && !in_n) return;
        bad |= !(qti.w < 0.0) || !(qt0.w < 0.0);
        const Prim wi = prim_from_q(qti, inv_gm1, g14);
        const Prim w0 = prim_from_q(qt0, inv_gm1, g14);
        if (in_t) {
            const D2 c = ds < 0.0 ? c0 : c1;
            const double sg = ds < 0.0 ? 1.0 : -1.0;
            acc_split_diff<2>(wi, w0, t.x, t.y, sg, c.x * ds + c.y * dn, inv_gm1, Rp);
        }
        if (in_n)
            acc_split_diff<2>(wi, w0, -t.y, t.x, ty == kWall ? -1.0 : 1.0, c2.x * dn + c2.y * ds,
                              inv_gm1, Rp);
        return;
    }
    const bool in_x = dx != 0.0, in_y = dy != 0.0;
    if (!in_x && !in_y) return;
    bad |= !(qti.w < 0.0) || !(qt0.w < 0.0);
    const Prim wi = prim_from_q(qti, inv_gm1, g14);
    const Prim w0 = prim_from_q(qt0, inv_gm1, g14);
    if (in_x) {
        const D2 c = dx < 0.0 ? c0 : c1;
        const double sg = dx < 0.0 ? 1.0 : -1.0;
        acc_split_diff<0>(wi, w0, 1.0, 0.0, sg, c.x * dx + c.y * dy, inv_gm1, Rp);
    }
    if (in_y) {
        const D2 c = dy < 0.0 ? c2 : c3;
        const double sg = dy < 0.0 ? 1.0 : -1.0;
        acc_split_diff<1>(wi, w0, 0.0, 1.0, sg, c.x * dy + c.y * dx, inv_gm1, Rp);
    }
}

// ---------------------------------------------------------------------------
// Residual (eq. 11 with the q~ reconstruction of eq. 15), local time step,
// scalar diagonal (eq. 25, 34-35) and the sweep linearisation data.
// ---------------------------------------------------------------------------
// LANES consecutive lanes share one point: each takes every LANES-th
// neighbour, the four residual sums are combined with cross-lane shuffles and
// the first lane finishes the point.
template <bool MIXED, int LANES>
__global__ void __launch_bounds__(kBlock) k_residual(
    int64_t n, double gamma, const double* __restrict__ cfl, const D2* __restrict__ xy,
    const D2* __restrict__ frame,
    const int8_t* __restrict__ type, const int32_t* __restrict__ off,
    const int32_t* __restrict__ idx, const PointGeom* __restrict__ geom,
    const int32_t* __restrict__ comp, const int32_t* __restrict__ active,
    const D4* __restrict__ U, const D4* __restrict__ q, const D4* __restrict__ qx,
    const D4* __restrict__ qy, D4* __restrict__ R, double* __restrict__ Dg,
    D4* __restrict__ jv0, D4* __restrict__ jv2, F4* __restrict__ jv0f, F4* __restrict__ jv2f,
    float* __restrict__ Df,
    double* __restrict__ rr_out, int32_t* __restrict__ flags, int variant, int fd,
    D4* dUio, F4* dUfio, D4* __restrict__ Rs, const int32_t* __restrict__ colour, int sweep0,
    int farfield, const double* __restrict__ vinf) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t gt = (int64_t)lb * blockDim.x + threadIdx.x;
    const int64_t p = gt / LANES;
    const int lane = (int)(gt % LANES);
    const double inv_gm1 = 1.0 / (gamma - 1.0);
    const bool g14 = gamma == 1.4;
    if (p < n && live(comp, active, p)) {
        const int8_t ty = type[p];
        const D2 r0 = xy[p];
        const D2 t = frame[p];
        double Rp[4] = {0, 0, 0, 0};
        int bad = 0;
        // outer points take part only under the kinetic far field
        const bool part = ty != kOuter || farfield;
        if (part) {
            const D4 q0 = q[p], gx0 = qx[p], gy0 = qy[p];
            const PointGeom& G = geom[p];
            const D2 c0 = G.split[0], c1 = G.split[1], c2 = G.split[2], c3 = G.split[3];
            const int32_t e1 = off[p + 1];
            int32_t e = off[p] + lane;
            if (e < e1) {
                // software pipeline: neighbour indices two entries ahead and
                // neighbour data one entry ahead of the pair being computed;
                // past the end the last entry is re-read (in bounds), unused
                const int32_t last = e1 - 1;
                int32_t i_next = idx[min(e + LANES, last)];
                Nbr cur = load_nbr(idx[e], xy, q, qx, qy);
                for (; e < e1; e += LANES) {
                    const int32_t i_after = idx[min(e + 2 * LANES, last)];
                    const Nbr nxt = load_nbr(i_next, xy, q, qx, qy);
                    residual_pair(ty, t, r0, q0, gx0, gy0, c0, c1, c2, c3, cur, inv_gm1, g14, Rp,
                                  bad);
                    cur = nxt;
                    i_next = i_after;
                }
            }
        }
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) Rp[v] += __shfl_xor(Rp[v], o, 64);
            bad |= __shfl_xor(bad, o, 64);
        }
        if (lane == 0) {
            if (ty == kWall) {  // drop the normal-momentum component
                const double nx = -t.y, ny = t.x;
                const double mn = Rp[1] * nx + Rp[2] * ny;
                Rp[1] -= mn * nx;
                Rp[2] -= mn * ny;
            }
            if (ty == kOuter && farfield) {
                // kinetic far field: the n- half (molecules entering the domain)
                // from a free-stream ghost one nearest-neighbour distance outside,
                // (G_n-(U_inf) - G_n-(U_0)) / h with the point's own q
                const int k = comp ? comp[p] : 0;
                const double v1 = vinf[2 * k], v2 = vinf[2 * k + 1];
                Prim wf;
                wf.rho = 1.0;
                wf.u1 = v1;
                wf.u2 = v2;
                wf.p = 1.0 / gamma;
                wf.sb = sqrt(0.5 * gamma);
                wf.isb = 1.0 / wf.sb;
                wf.rhoE = wf.p * inv_gm1 + 0.5 * (v1 * v1 + v2 * v2);
                const Prim w0 = prim_from_q(q[p], inv_gm1, g14);
                double Gf[4], G0[4];
                split_flux<2>(wf, -t.y, t.x, -1.0, inv_gm1, Gf);
                split_flux<2>(w0, -t.y, t.x, -1.0, inv_gm1, G0);
                const double ih = 1.0 / geom[p].lsq.w;
#pragma unroll
                for (int v = 0; v < 4; ++v) Rp[v] += (Gf[v] - G0[v]) * ih;
            }
            rr_out[p] = ty != kOuter ? Rp[0] * Rp[0] : 0.0;
            R[p] = {Rp[0], Rp[1], Rp[2], Rp[3]};

            // linearisation data at the current state, local time step, diagonal
            const D4 u = U[p];
            const double rho = u.x, irho = 1.0 / rho;
            const double u1 = u.y * irho, u2 = u.z * irho;
            const double usq = u1 * u1 + u2 * u2;
            const double pr = (gamma - 1.0) * (u.w - 0.5 * rho * usq);
            const double beta = 0.5 * rho / pr;
            const double sb = sqrt(beta);
            const double sx = u1 * sb, sy = u2 * sb;
            const D4 j0 = {rho, u1, u2, pr};
            const D4 j2 = {erf_fast(sx), exp_fast(-(sx * sx)), erf_fast(sy), exp_fast(-(sy * sy))};
            const double a = sqrt(gamma * pr / rho);
            const PointGeom& G = geom[p];
            const double dt = cfl[comp ? comp[p] : 0] * G.lsq.w / (sqrt(usq) + a);
            double Dp = 1.0 / dt;
            if (variant == 0) {
                // Anandhanarayanan et al.: split Jacobians -> +-rho(A+-) I (eq. 34-35)
                if (ty == kWall) {
                    const double ut = u1 * t.x + u2 * t.y, un = -u1 * t.y + u2 * t.x;
                    Dp -= G.ls1.x * fmax(ut + a, 0.0);
                    Dp += G.ls1.y * fmax(a - ut, 0.0);
                    Dp += G.ls1.z * fmax(a - un, 0.0);
                } else if (ty != kOuter) {
                    Dp -= G.ls1.x * fmax(u1 + a, 0.0);
                    Dp += G.ls1.y * fmax(a - u1, 0.0);
                    Dp -= G.ls1.z * fmax(u2 + a, 0.0);
                    Dp += G.ls1.w * fmax(a - u2, 0.0);
                } else if (farfield) {
                    // t+, t-, n+ of the stencil and the ghost's n- half, whose
                    // single weight is 1/h (its increment is zero)
                    const double ut = u1 * t.x + u2 * t.y, un = -u1 * t.y + u2 * t.x;
                    Dp -= G.ls1.x * fmax(ut + a, 0.0);
                    Dp += G.ls1.y * fmax(a - ut, 0.0);
                    Dp -= G.ls1.z * fmax(un + a, 0.0);
                    Dp += fmax(a - un, 0.0) / G.lsq.w;
                }
            } else {
                // Manish et al.: A+- = (A +- rho(A) I)/2, rho(A) = |u_d| + a (eq. 29-33); the
                // A part, S_0 = -1/2 sum_k LS_k(1) A_k dU_0, is taken with the previous
                // iteration's increment onto the forward right-hand side R - S (eq. 36-38)
                double dv[4] = {0, 0, 0, 0};
                if (MIXED) {
                    const F4 d = dUfio[p];
                    dv[0] = d.x; dv[1] = d.y; dv[2] = d.z; dv[3] = d.w;
                } else {
                    const D4 d = dUio[p];
                    dv[0] = d.x; dv[1] = d.y; dv[2] = d.z; dv[3] = d.w;
                }
                double Sv[4] = {0, 0, 0, 0}, Ja[4], Jb[4];
                double ca = 0.0, cb = 0.0;
                if (ty == kWall) {
                    const double ut = u1 * t.x + u2 * t.y, un = -u1 * t.y + u2 * t.x;
                    Dp -= 0.5 * (fabs(ut) + a) * (G.ls1.x - G.ls1.y);
                    Dp += 0.5 * (fabs(un) + a) * G.ls1.z;
                    if (fd) {
                        unsplit_jvp<true>(u, dv, t.x, t.y, gamma - 1.0, Ja);
                        unsplit_jvp<true>(u, dv, -t.y, t.x, gamma - 1.0, Jb);
                    } else {
                        unsplit_jvp<false>(u, dv, t.x, t.y, gamma - 1.0, Ja);
                        unsplit_jvp<false>(u, dv, -t.y, t.x, gamma - 1.0, Jb);
                    }
                    ca = G.ls1.x + G.ls1.y;
                    cb = G.ls1.z;
                } else if (ty == kOuter && farfield) {
                    const double ut = u1 * t.x + u2 * t.y, un = -u1 * t.y + u2 * t.x;
                    Dp -= 0.5 * (fabs(ut) + a) * (G.ls1.x - G.ls1.y);
                    Dp -= 0.5 * (fabs(un) + a) * G.ls1.z;
                    if (fd) {
                        unsplit_jvp<true>(u, dv, t.x, t.y, gamma - 1.0, Ja);
                        unsplit_jvp<true>(u, dv, -t.y, t.x, gamma - 1.0, Jb);
                    } else {
                        unsplit_jvp<false>(u, dv, t.x, t.y, gamma - 1.0, Ja);
                        unsplit_jvp<false>(u, dv, -t.y, t.x, gamma - 1.0, Jb);
                    }
                    ca = G.ls1.x + G.ls1.y;
                    cb = G.ls1.z;
                } else if (ty != kOuter) {
                    Dp -= 0.5 * (fabs(u1) + a) * (G.ls1.x - G.ls1.y);
                    Dp -= 0.5 * (fabs(u2) + a) * (G.ls1.z - G.ls1.w);
                    if (fd) {
                        unsplit_jvp<true>(u, dv, 1.0, 0.0, gamma - 1.0, Ja);
                        unsplit_jvp<true>(u, dv, 0.0, 1.0, gamma - 1.0, Jb);
                    } else {
                        unsplit_jvp<false>(u, dv, 1.0, 0.0, gamma - 1.0, Ja);
                        unsplit_jvp<false>(u, dv, 0.0, 1.0, gamma - 1.0, Jb);
                    }
                    ca = G.ls1.x + G.ls1.y;
                    cb = G.ls1.z + G.ls1.w;
                }
                if (part)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Sv[v] = -0.5 * (ca * Ja[v] + cb * Jb[v]);
                Rs[p] = {Rp[0] - Sv[0], Rp[1] - Sv[1], Rp[2] - Sv[2], Rp[3] - Sv[3]};
                if (sweep0)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Sv[v] = Rp[v] - Sv[v];
            }
            if (MIXED) {
                jv0f[p] = {(float)j0.x, (float)j0.y, (float)j0.z, (float)j0.w};
                jv2f[p] = {(float)j2.x, (float)j2.y, (float)j2.z, (float)j2.w};
                Df[p] = (float)Dp;
            } else {
                jv0[p] = j0;
                jv2[p] = j2;
                Dg[p] = Dp;
            }
            // the forward sweep's first colour phase: its points have no lower
            // neighbours, dU* = -R / D (R - S for the Manish variant), in the
            // sweep precision and with the sweep kernel's arithmetic
            if (sweep0 && colour[p] == 0) {
                double rs[4] = {Rp[0], Rp[1], Rp[2], Rp[3]};
                if (variant != 0) {
                    const D4 r2 = Rs[p];
                    rs[0] = r2.x; rs[1] = r2.y; rs[2] = r2.z; rs[3] = r2.w;
                }
                if (MIXED) {
                    float o[4] = {0.f, 0.f, 0.f, 0.f};
                    if (part) {
                        const float iD = 1.0f / (float)Dp;
#pragma unroll
                        for (int v = 0; v < 4; ++v) o[v] = -((float)rs[v] + 0.0f) * iD;
                        if (ty == kWall) {
                            const float nx = (float)(-t.y), ny = (float)t.x;
                            const float mn = o[1] * nx + o[2] * ny;
                            o[1] -= mn * nx;
                            o[2] -= mn * ny;
                        }
                    }
                    dUfio[p] = {o[0], o[1], o[2], o[3]};
                } else {
                    double o[4] = {0, 0, 0, 0};
                    if (part) {
                        const double iD = 1.0 / Dp;
#pragma unroll
                        for (int v = 0; v < 4; ++v) o[v] = -(rs[v] + 0.0) * iD;
                        if (ty == kWall) {
                            const double nx = -t.y, ny = t.x;
                            const double mn = o[1] * nx + o[2] * ny;
                            o[1] -= mn * nx;
                            o[2] -= mn * ny;
                        }
                    }
                    dUio[p] = {o[0], o[1], o[2], o[3]};
                }
            }
            if (bad || !(rho > 0.0) || !(pr > 0.0)) flags[0] = 1;
        }
    }
}

// Residual norm of each component in two deterministic stages: one block
// per reduction chunk sums R_rho^2 over the chunk's points, then one thread
// wavefront per component adds its chunks: res = sqrt(sum) / (non-outer count).
// A component whose norm is not finite is retired as failed; one that reaches
// tol_abs (> 0) is retired as converged.
__global__ void __launch_bounds__(kBlock) k_norm_partial(const double* __restrict__ rr,
                                                         const int32_t* __restrict__ chunk_start,
                                                         const int32_t* __restrict__ chunk_comp,
                                                         const int32_t* __restrict__ active,
                                                         double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    const int c = blockIdx.x;
    if (!active[chunk_comp[c]]) return;  // uniform over the block
    double s = 0.0;
    // unrolled so that the loads are issued together; the additions keep their order
#pragma unroll 4
    for (int64_t p = chunk_start[c] + threadIdx.x; p < chunk_start[c + 1]; p += blockDim.x)
        s += rr[p];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w];
        partial[c] = t;
    }
}

__global__ void __launch_bounds__(64) k_norm_comp(const double* __restrict__ partial,
                                                  const int32_t* __restrict__ comp_chunk_off,
                                                  const double* __restrict__ inv_active,
                                                  const double* __restrict__ tol_abs,
                                                  int32_t* __restrict__ active,
                                                  int32_t* __restrict__ status,
                                                  int32_t* __restrict__ iters,
                                                  double* __restrict__ res_last,
                                                  double* __restrict__ out) {
    const int k = blockIdx.x;  // one wavefront per component
    if (!active[k]) return;
    double t = 0.0;
    // unrolled so that the loads are issued together; the additions keep their order
#pragma unroll 8
    for (int c = comp_chunk_off[k] + threadIdx.x; c < comp_chunk_off[k + 1]; c += 64) t += partial[c];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (threadIdx.x != 0) return;
    const double res = sqrt(t) * inv_active[k];
    out[k] = res;
    res_last[k] = res;
    iters[k] += 1;
    if (!(res <= 1e300)) {
        status[k] = -1;
        active[k] = 0;
    } else if (tol_abs[k] > 0.0 && res <= tol_abs[k]) {
        status[k] = 1;
        active[k] = 0;
    }
}

__global__ void k_reset_components(int ncomp, int32_t* __restrict__ active,
                                   int32_t* __restrict__ status, int32_t* __restrict__ iters) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncomp) return;
    active[k] = 1;
    status[k] = 0;
    iters[k] = 0;
}

// ---------------------------------------------------------------------------
// Split-flux Jacobian-vector products for the sweeps.
// ---------------------------------------------------------------------------
template <class T>
struct Lin {  // linearisation data of one neighbour
    T rho, u1, u2, p, sb, beta, irho, ip;
};

// Tangent of the split flux along unit direction (dx, dy) with sign sg,
// given erf(S) and exp(-S^2) at the linearisation state.  Hand-written
// forward-mode derivative of the closed-form split flux (the paper's exact
// Jacobian-vector product): with rho', u', p' from dU,
//   beta' = (rho' - 2 beta p')/(2p),  S' = u_d' sqrt(beta) + u_d beta'/(2 sqrt(beta)),
//   A' = sg exp(-S^2) S'/sqrt(pi),    B' = B (-2 S S' - beta'/(2 beta)),
// and the product rule on each flux component.
template <class T>
__device__ __forceinline__ void jvp_exact(const Lin<T>& L, T er, T g, T dx, T dy, T sg,
                                          const T dU[4], T gm1, T inv_gm1, T J[4]) {
    const T rd = dU[0];
    const T u1d = (dU[1] - L.u1 * rd) * L.irho;
    const T u2d = (dU[2] - L.u2 * rd) * L.irho;
    const T usq = L.u1 * L.u1 + L.u2 * L.u2;
    const T pd = gm1 * (dU[3] - T(0.5) * rd * usq - L.rho * (L.u1 * u1d + L.u2 * u2d));
    const T bd = (rd - T(2) * L.beta * pd) * (T(0.5) * L.ip);
    const T ud = L.u1 * dx + L.u2 * dy;
    const T udd = u1d * dx + u2d * dy;
    const T ib = T(2) * L.p * L.irho;  // 1/beta = 2p/rho, without a division
    const T isb = L.sb * ib;           // 1/sqrt(beta)
    const T S = ud * L.sb;
    const T Sd = udd * L.sb + T(0.5) * ud * bd * isb;
    const T A = T(0.5) * (T(1) + sg * er);
    const T Ad = sg * g * Sd * T(kInvSqrtPi);
    const T B = g * T(0.5 * kInvSqrtPi) * isb;
    const T Bd = B * (T(-2) * S * Sd - T(0.5) * bd * ib);
    const T F = ud * A + sg * B;
    const T Fd = udd * A + ud * Ad + sg * Bd;
    const T rhoE = L.p * inv_gm1 + T(0.5) * L.rho * usq;
    const T J0 = rd * F + L.rho * Fd;
    const T mass = L.rho * F;
    const T pAd = pd * A + L.p * Ad;
    J[0] = J0;
    J[1] = pAd * dx + u1d * mass + L.u1 * J0;
    J[2] = pAd * dy + u2d * mass + L.u2 * J0;
    J[3] = (dU[3] + pd) * ud * A + (rhoE + L.p) * (udd * A + ud * Ad) +
           sg * ((dU[3] + T(0.5) * pd) * B + (rhoE + T(0.5) * L.p) * Bd);
}

// Split flux from the linearisation data (value only, used by the
// flux-difference products).
__device__ __forceinline__ void flux_lin(const Lin<double>& L, double er, double g, double dx,
                                         double dy, double sg, double inv_gm1, double G[4]) {
    const double ud = L.u1 * dx + L.u2 * dy;
    const double A = 0.5 * (1.0 + sg * er);
    const double B = g * (0.5 * kInvSqrtPi) / L.sb;
    const double rhoE = L.p * inv_gm1 + 0.5 * L.rho * (L.u1 * L.u1 + L.u2 * L.u2);
    const double mass = L.rho * (ud * A + sg * B);
    G[0] = mass;
    G[1] = L.p * A * dx + L.u1 * mass;
    G[2] = L.p * A * dy + L.u2 * mass;
    G[3] = (rhoE + L.p) * ud * A + sg * (rhoE + 0.5 * L.p) * B;
}

// Flux difference G(U + dU) - G(U) of eq. (28).
__device__ __forceinline__ void jvp_fluxdiff(const Lin<double>& L, double er, double g, const D4& u,
                                             double dx, double dy, double sg, const double dU[4],
                                             double gamma, double inv_gm1, double J[4]) {
    const double a0 = u.x + dU[0], a1 = u.y + dU[1], a2 = u.z + dU[2], a3 = u.w + dU[3];
    Lin<double> W;
    W.rho = a0;
    W.irho = 1.0 / a0;
    W.u1 = a1 * W.irho;
    W.u2 = a2 * W.irho;
    W.p = (gamma - 1.0) * (a3 - 0.5 * W.rho * (W.u1 * W.u1 + W.u2 * W.u2));
    W.beta = 0.5 * W.rho / W.p;
    W.sb = sqrt(W.beta);
    const double S = (W.u1 * dx + W.u2 * dy) * W.sb;
    double Ga[4], Gb[4];
    flux_lin(W, erf_fast(S), exp_fast(-(S * S)), dx, dy, sg, inv_gm1, Ga);
    flux_lin(L, er, g, dx, dy, sg, inv_gm1, Gb);
#pragma unroll
    for (int v = 0; v < 4; ++v) J[v] = Ga[v] - Gb[v];
}

// The linearisation data of neighbour i from its (rho, u1, u2, p) record: the
// derived quantities are formed here rather than read, which halves the bytes
// a sweep gathers per neighbour for them.
// One reciprocal, of rho p, gives both 1/rho and 1/p; the fp32 sweeps use
// the hardware reciprocal and square root (about 1 ulp).
template <class T>
__device__ __forceinline__ Lin<T> load_lin(const Vec4<T>* jv0, int32_t i) {
    const Vec4<T> a = jv0[i];
    T r, sb;
    if constexpr (std::is_same_v<T, float>) {
        r = __builtin_amdgcn_rcpf(a.x * a.w);
    } else {
        r = T(1) / (a.x * a.w);
    }
    const T irho = a.w * r, ip = a.x * r;
    const T beta = T(0.5) * a.x * ip;
    if constexpr (std::is_same_v<T, float>) {
        sb = __builtin_amdgcn_sqrtf(beta);
    } else {
        sb = sqrt(beta);
    }
    return Lin<T>{a.x, a.y, a.z, a.w, sb, beta, irho, ip};
}

// Split weights and bits of the sweep-list entries of the colour-sorted point
// q (thread per q): for interior points the x split (a) and y split (b) the
// neighbour falls in; for frame points the t split (a) and the normal split
// (b): n- on the fluid side of a wall point, n+ on the inner side of an outer
// point (used under the kinetic far field) -- membership and weights exactly
// as the residual forms them.
__global__ void __launch_bounds__(kBlock) k_sweep_weights(int64_t n,
                                                          const int32_t* __restrict__ col_perm,
                                                          const D2* __restrict__ xy,
                                                          const D2* __restrict__ frame,
                                                          const int8_t* __restrict__ type,
                                                          const PointGeom* __restrict__ geom,
                                                          const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ idx,
                                                          D2* __restrict__ w,
                                                          F2* __restrict__ wf,
                                                          uint8_t* __restrict__ code) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int32_t p = col_perm[q];
    const int8_t ty = type[p];
    const D2 r0 = xy[p], t = frame[p];
    const PointGeom& G = geom[p];
    for (int32_t e = off[q]; e < off[q + 1]; ++e) {
        const D2 ri = xy[idx[e]];
        const double dx = ri.x - r0.x, dy = ri.y - r0.y;
        uint8_t cd = 0;
        double wa = 0.0, wb = 0.0;
        if (ty != kInterior) {
            const double ds = dot_nc(dx, dy, t.x, t.y);
            const double dn = dot_nc(dx, dy, -t.y, t.x);
            cd |= kSwWall;
            if (ds != 0.0) {
                const D2 cc = ds < 0.0 ? G.split[0] : G.split[1];
                cd |= kSwA | (ds < 0.0 ? kSwNegA : 0);
                wa = cc.x * ds + cc.y * dn;
            }
            if (in_normal_split(ty, dn)) {
                cd |= kSwB | (dn < 0.0 ? kSwNegB : 0);
                wb = G.split[2].x * dn + G.split[2].y * ds;
            }
        } else {
            if (dx != 0.0) {
                const D2 cc = dx < 0.0 ? G.split[0] : G.split[1];
                cd |= kSwA | (dx < 0.0 ? kSwNegA : 0);
                wa = cc.x * dx + cc.y * dy;
            }
            if (dy != 0.0) {
                const D2 cc = dy < 0.0 ? G.split[2] : G.split[3];
                cd |= kSwB | (dy < 0.0 ? kSwNegB : 0);
                wb = cc.x * dy + cc.y * dx;
            }
        }
        w[e] = {wa, wb};
        wf[e] = {(float)wa, (float)wb};
        code[e] = cd;
    }
}

// Contribution sum_k w_i^k A_k(U_i) dU_i of neighbour i to point p's sweep
// sum (eq. 22-27) from the entry's weights and split bits: interior points
// use the x and y split the neighbour falls in, frame points the t split and
// the normal split (n- at a wall, n+ at a far-field outer point) in the frame
// t of point p.
template <class T, int MODE>
__device__ __forceinline__ void sweep_contrib(uint8_t cd, const D2* __restrict__ frame, int32_t p,
                                              const W2<T>& w, int32_t i,
                                              const Vec4<T>* __restrict__ jv0,
                                              const Vec4<T>* __restrict__ jv2,
                                              const D4* __restrict__ U,
                                              const Vec4<T>* __restrict__ dU, double gamma,
                                              T acc[4]) {
    const T gm1 = T(gamma - 1.0), inv_gm1 = T(1.0 / (gamma - 1.0));
    const Vec4<T> di = dU[i];
    const T dv[4] = {di.x, di.y, di.z, di.w};
    const Lin<T> L = load_lin(jv0, i);
    const Vec4<T> k2 = jv2[i];  // interior entries only; loaded with the rest
    T J[4];
    if (cd & kSwWall) {
        // wall-frame directions: erf/exp at the neighbour state are formed here
        const D2 t = frame[p];
        if (cd & kSwA) {
            const double sg = (cd & kSwNegA) ? 1.0 : -1.0;
            if constexpr (MODE == 1) {
                const double S = (L.u1 * t.x + L.u2 * t.y) * L.sb;
                jvp_fluxdiff(L, erf_fast(S), exp_fast(-(S * S)), U[i], t.x, t.y, sg, dv, gamma,
                             1.0 / (gamma - 1.0), J);
            } else {
                const T S = (L.u1 * T(t.x) + L.u2 * T(t.y)) * L.sb;
                jvp_exact<T>(L, erf_k(S), exp_k(-(S * S)), T(t.x), T(t.y), T(sg), dv, gm1, inv_gm1, J);
            }
            const T wa = T(w.x);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += wa * J[v];
        }
        if (cd & kSwB) {
            const double sg = (cd & kSwNegB) ? 1.0 : -1.0;
            if constexpr (MODE == 1) {
                const double S = (-L.u1 * t.y + L.u2 * t.x) * L.sb;
                jvp_fluxdiff(L, erf_fast(S), exp_fast(-(S * S)), U[i], -t.y, t.x, sg, dv, gamma,
                             1.0 / (gamma - 1.0), J);
            } else {
                const T S = (-L.u1 * T(t.y) + L.u2 * T(t.x)) * L.sb;
                jvp_exact<T>(L, erf_k(S), exp_k(-(S * S)), T(-t.y), T(t.x), T(sg), dv, gm1, inv_gm1, J);
            }
            const T wb = T(w.y);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += wb * J[v];
        }
        return;
    }
    if (cd & kSwA) {
        const T sg = (cd & kSwNegA) ? T(1) : T(-1);
        if constexpr (MODE == 1)
            jvp_fluxdiff(L, k2.x, k2.y, U[i], 1.0, 0.0, sg, dv, gamma, 1.0 / (gamma - 1.0), J);
        else
            jvp_exact<T>(L, k2.x, k2.y, T(1), T(0), sg, dv, gm1, inv_gm1, J);
        const T wa = T(w.x);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += wa * J[v];
    }
    if (cd & kSwB) {
        const T sg = (cd & kSwNegB) ? T(1) : T(-1);
        if constexpr (MODE == 1)
            jvp_fluxdiff(L, k2.z, k2.w, U[i], 0.0, 1.0, sg, dv, gamma, 1.0 / (gamma - 1.0), J);
        else
            jvp_exact<T>(L, k2.z, k2.w, T(0), T(1), sg, dv, gm1, inv_gm1, J);
        const T wb = T(w.y);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += wb * J[v];
    }
}

// One colour phase of a sweep (eq. 27).  FWD: dU*_0 = -(R_0 + sum_lower w A dU*) / D_0;
// backward: dU_0 = dU*_0 - (sum_upper w A dU) / D_0.  MODE 0 exact tangent,
// 1 flux difference.  T is the arithmetic of the products and increments.
// LANES consecutive lanes share one point: each walks every LANES-th entry of
// the point's lower (forward) or upper (backward) list, and the partial sums
// are combined with cross-lane shuffles.  The phase's points are the
// colour-sorted positions [start, start + count) and their lists one
// contiguous block.
template <class T, bool FWD, int MODE, int LANES>
__global__ void __launch_bounds__(kBlock, 5) k_sweep(
    int32_t start, int32_t count, const int32_t* __restrict__ col_perm,
    const D2* __restrict__ frame, const int8_t* __restrict__ type,
    const int32_t* __restrict__ loff, const int32_t* __restrict__ lidx,
    const W2<T>* __restrict__ lw, const uint8_t* __restrict__ lcode,
    const int32_t* __restrict__ comp, const int32_t* __restrict__ active,
    const Vec4<T>* __restrict__ jv0, const Vec4<T>* __restrict__ jv2,
    const D4* __restrict__ U, const D4* __restrict__ R,
    const T* __restrict__ Dg, Vec4<T>* __restrict__ dU, double gamma, int farfield) {
    const int gt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int pt = gt / LANES, lane = gt % LANES;
    if (pt >= count) return;  // uniform over the lanes of a point
    // A phase is short and latency-bound, so its loads are ordered to form as
    // few dependent levels as possible: q-indexed offsets and permutation;
    // then the point's own record and the list entries together; then the
    // neighbours' data.  Nothing waits on the point type before the list walk
    // (an outer point's products are formed and discarded).
    const int32_t q = start + pt;
    const int32_t p = col_perm[q];
    const int32_t e0 = loff[q], e1 = loff[q + 1];
    if (comp && !active[comp[p]]) return;  // retired component of a batch (uniform per point)
    if (!comp && !active[0]) return;
    // the lane's first list entry, requested before the point's own record
    int32_t e = e0 + lane;
    uint8_t cd = 0;
    W2<T> w = {T(0), T(0)};
    int32_t i = 0;
    if (e < e1) {
        cd = lcode[e];
        w = lw[e];
        i = lidx[e];
    }
    T acc[4] = {T(0), T(0), T(0), T(0)};
    while (e < e1) {
        // the next entry is requested before this one's neighbour data is used;
        // past the end the last entry is re-read (in bounds) and not used
        const int32_t en = e + LANES;
        const int32_t ec = en < e1 ? en : e1 - 1;
        const uint8_t cdn = lcode[ec];
        const W2<T> wn = lw[ec];
        const int32_t in = lidx[ec];
        sweep_contrib<T, MODE>(cd, frame, p, w, i, jv0, jv2, U, dU, gamma, acc);
        cd = cdn;
        w = wn;
        i = in;
        e = en;
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] += __shfl_xor(acc[v], o, 64);
    if (lane != 0) return;
    // the point's own data is read after the walk, by the one lane that uses
    // it: held through the walk it cost every lane ten registers
    const int8_t ty = type[p];
    const T dg = Dg[p];
    Vec4<T> own;
    if (FWD) {
        const D4 r = R[p];
        own = {T(r.x), T(r.y), T(r.z), T(r.w)};
    } else {
        own = dU[p];
    }
    if (ty == kOuter && !farfield) {
        if (FWD) dU[p] = {T(0), T(0), T(0), T(0)};
        return;
    }
    const T iD = T(1) / dg;
    T out[4];
    if (FWD) {
        out[0] = -(own.x + acc[0]) * iD;
        out[1] = -(own.y + acc[1]) * iD;
        out[2] = -(own.z + acc[2]) * iD;
        out[3] = -(own.w + acc[3]) * iD;
    } else {
        out[0] = own.x - acc[0] * iD;
        out[1] = own.y - acc[1] * iD;
        out[2] = own.z - acc[2] * iD;
        out[3] = own.w - acc[3] * iD;
    }
    if (ty == kWall) {
        const D2 t = frame[p];
        const T nx = T(-t.y), ny = T(t.x);
        const T mn = out[1] * nx + out[2] * ny;
        out[1] -= mn * nx;
        out[2] -= mn * ny;
    }
    dU[p] = {out[0], out[1], out[2], out[3]};
}

// U += dU (Section 3) and the q-variables of the new state (eq. 14).
template <class T>
__global__ void __launch_bounds__(kBlock) k_update(int64_t n, double gamma, D4* __restrict__ U,
                                                   const Vec4<T>* __restrict__ dU,
                                                   const int32_t* __restrict__ comp,
                                                   const int32_t* __restrict__ active,
                                                   D4* __restrict__ q, int32_t* __restrict__ flags) {
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= n || !live(comp, active, p)) return;
    D4 u = U[p];
    const Vec4<T> d = dU[p];
    u.x += (double)d.x;
    u.y += (double)d.y;
    u.z += (double)d.z;
    u.w += (double)d.w;
    U[p] = u;
    bool bad;
    q[p] = q_of_U(u, gamma, 1.0 / (gamma - 1.0), bad);
    if (bad) flags[0] = 1;
}

// Explicit iteration (the paper's explicit LSKUM solver): U <- U - dt R with
// the implicit scheme's local time step dt = CFL rmin / (|u| + a) at the
// current state, then the next q-variables.  Outer points keep their state
// unless the kinetic far field gives them a residual.
__global__ void __launch_bounds__(kBlock) k_explicit_update(
    int64_t n, double gamma, const double* __restrict__ cfl, const int8_t* __restrict__ type,
    const PointGeom* __restrict__ geom, const int32_t* __restrict__ comp,
    const int32_t* __restrict__ active, const D4* __restrict__ R, D4* __restrict__ U,
    D4* __restrict__ q, int32_t* __restrict__ flags, int farfield) {
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= n || !live(comp, active, p) || (type[p] == kOuter && !farfield)) return;
    D4 u = U[p];
    const double rho = u.x, irho = 1.0 / rho;
    const double u1 = u.y * irho, u2 = u.z * irho;
    const double usq = u1 * u1 + u2 * u2;
    const double pr = (gamma - 1.0) * (u.w - 0.5 * rho * usq);
    const double a = sqrt(gamma * pr / rho);
    const double dt = cfl[comp ? comp[p] : 0] * geom[p].lsq.w / (sqrt(usq) + a);
    const D4 r = R[p];
    u.x -= dt * r.x;
    u.y -= dt * r.y;
    u.z -= dt * r.z;
    u.w -= dt * r.w;
    U[p] = u;
    bool bad;
    q[p] = q_of_U(u, gamma, 1.0 / (gamma - 1.0), bad);
    if (bad) flags[0] = 1;
}

// Pressure force on the closed wall polygon of each component (one block per
// component): sum over edges (a, b) of -(p_mid - p_inf) * |e| * (edge normal
// pointing out of the body), orient = +1 for a counter-clockwise polygon.
__global__ void __launch_bounds__(kBlock) k_forces(const int32_t* __restrict__ wall,
                                                   const int32_t* __restrict__ wall_off,
                                                   const double* __restrict__ orient_k,
                                                   const D2* __restrict__ xy, const D4* __restrict__ U,
                                                   double gamma, double* __restrict__ out) {
    __shared__ double rx[kBlock / 64], ry[kBlock / 64];
    const int k = blockIdx.x;
    const int64_t w0 = wall_off[k], m = wall_off[k + 1] - w0;
    const double orient = orient_k[k];
    double fx = 0.0, fy = 0.0;
    const double pinf = 1.0 / gamma;
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
        const int32_t a = wall[w0 + j], b = wall[w0 + (j + 1 == m ? 0 : j + 1)];
        const D4 ua = U[a], ub = U[b];
        const double pa = (gamma - 1.0) * (ua.w - 0.5 * (ua.y * ua.y + ua.z * ua.z) / ua.x);
        const double pb = (gamma - 1.0) * (ub.w - 0.5 * (ub.y * ub.y + ub.z * ub.z) / ub.x);
        const double pm = 0.5 * (pa + pb) - pinf;
        const D2 ra = xy[a], rb = xy[b];
        const double ex = rb.x - ra.x, ey = rb.y - ra.y;
        fx -= pm * (orient * ey);
        fy -= pm * (-orient * ex);
    }
    for (int o = 32; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, 64);
        fy += __shfl_xor(fy, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        rx[threadIdx.x >> 6] = fx;
        ry[threadIdx.x >> 6] = fy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sx = 0, sy = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            sx += rx[w];
            sy += ry[w];
        }
        out[2 * k] = sx;
        out[2 * k + 1] = sy;
    }
}

__global__ void __launch_bounds__(kBlock) k_soa_to_aos(const double* __restrict__ soa,
                                                       D4* __restrict__ aos, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    aos[p] = {soa[p], soa[n + p], soa[2 * n + p], soa[3 * n + p]};
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_aos_to_soa(const Vec4<T>* __restrict__ aos,
                                                       double* __restrict__ soa, int64_t n) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const Vec4<T> v = aos[p];
    soa[p] = (double)v.x;
    soa[n + p] = (double)v.y;
    soa[2 * n + p] = (double)v.z;
    soa[3 * n + p] = (double)v.w;
}

__global__ void k_clear_flags(int32_t* flags) {
    if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_precompute(Cloud& c, hipStream_t st) {
    unsigned long long* d_cnt = nullptr;
    hipError_t e = hipMalloc((void**)&d_cnt, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    unsigned long long h[2] = {0, 0};
    e = hipMemsetAsync(d_cnt, 0, 2 * sizeof(unsigned long long), st);
    if (e == hipSuccess && c.n > 0) {
        hipLaunchKernelGGL(k_precompute, dim3(grid_for(c.n)), dim3(kBlock), 0, st, c.n, c.xy,
                           c.frame, c.type, c.off, c.idx, c.geom, d_cnt);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, d_cnt, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_cnt);
    if (e != hipSuccess) return e;
    c.n_degenerate = (int64_t)h[1];
    if (h[0]) return hipErrorInvalidValue;  // singular full stencil, reported by the caller
    return hipSuccess;
}

hipError_t launch_sweep_weights(Cloud& c, hipStream_t st) {
    if (c.n > 0) {
        hipLaunchKernelGGL(k_sweep_weights, dim3(grid_for(c.n)), dim3(kBlock), 0, st, c.n,
                           c.col_perm, c.xy, c.frame, c.type, c.geom, c.lo_off, c.lo_idx, c.lo_w,
                           c.lo_wf, c.lo_code);
        hipLaunchKernelGGL(k_sweep_weights, dim3(grid_for(c.n)), dim3(kBlock), 0, st, c.n,
                           c.col_perm, c.xy, c.frame, c.type, c.geom, c.up_off, c.up_idx, c.up_w,
                           c.up_wf, c.up_code);
    }
    return hipGetLastError();
}

hipError_t launch_free_stream(State& s) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_free_stream, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n, c.type,
                       c.frame, s.prm.gamma, c.comp, s.vinf, s.U);
    return hipGetLastError();
}

hipError_t launch_q_from_U(State& s) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_q_from_U, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n,
                       s.prm.gamma, s.U, s.q, s.flags);
    return hipGetLastError();
}

template <int LANES>
static void qgrad_lanes(State& s, bool keep) {
    const Cloud& c = *s.cloud;
    const dim3 g(grid_for(c.n * LANES)), b(kBlock);
    const double K = s.prm.limiter_k;
    const int m = s.prm.inner_iters;
    const bool lim = s.prm.limiter != 0;
    // pass 0 (first order), then m inner passes; the limiter rides on the last
    if (m == 0 && lim)
        hipLaunchKernelGGL((k_qgrad<false, true, LANES>), g, b, 0, s.stream, c.n, K, c.xy, c.off,
                           c.idx, c.geom, c.comp, s.active, s.q, nullptr, nullptr,
                           keep ? s.qx[0] : nullptr, keep ? s.qy[0] : nullptr, s.qxl, s.qyl);
    else
        hipLaunchKernelGGL((k_qgrad<false, false, LANES>), g, b, 0, s.stream, c.n, K, c.xy, c.off,
                           c.idx, c.geom, c.comp, s.active, s.q, nullptr, nullptr, s.qx[0],
                           s.qy[0], nullptr, nullptr);
    int cur = 0;
    for (int it = 0; it < m; ++it) {
        if (it == m - 1 && lim)
            hipLaunchKernelGGL((k_qgrad<true, true, LANES>), g, b, 0, s.stream, c.n, K, c.xy,
                               c.off, c.idx, c.geom, c.comp, s.active, s.q, s.qx[cur], s.qy[cur],
                               keep ? s.qx[1 - cur] : nullptr, keep ? s.qy[1 - cur] : nullptr,
                               s.qxl, s.qyl);
        else
            hipLaunchKernelGGL((k_qgrad<true, false, LANES>), g, b, 0, s.stream, c.n, K, c.xy,
                               c.off, c.idx, c.geom, c.comp, s.active, s.q, s.qx[cur], s.qy[cur],
                               s.qx[1 - cur], s.qy[1 - cur], nullptr, nullptr);
        cur = 1 - cur;
    }
    s.qsel = cur;
}

// Tiled passes (LDS-staged neighbours): block = tile, dynamic LDS sized by
// the cloud's largest tile neighbour list.
static void qgrad_tiled(State& s, bool keep) {
    const Cloud& c = *s.cloud;
    const dim3 g((unsigned)c.ntile), b(kBlock);
    const double K = s.prm.limiter_k;
    const int m = s.prm.inner_iters;
    const bool lim = s.prm.limiter != 0;
    const size_t lds0 = (size_t)c.tile_hmax * 6 * sizeof(double);
    const size_t lds1 = (size_t)c.tile_hmax * 14 * sizeof(double);
    if (m == 0 && lim)
        hipLaunchKernelGGL((k_qgrad_tiled<false, true>), g, b, lds0, s.stream, K, c.xy, c.off,
                           c.tile_pts, c.lnbr, c.tile_off, c.tile_idx, c.tile_hmax, c.geom,
                           c.comp, s.active, s.q, nullptr, nullptr, keep ? s.qx[0] : nullptr,
                           keep ? s.qy[0] : nullptr, s.qxl, s.qyl);
    else
        hipLaunchKernelGGL((k_qgrad_tiled<false, false>), g, b, lds0, s.stream, K, c.xy, c.off,
                           c.tile_pts, c.lnbr, c.tile_off, c.tile_idx, c.tile_hmax, c.geom,
                           c.comp, s.active, s.q, nullptr, nullptr, s.qx[0], s.qy[0], nullptr,
                           nullptr);
    int cur = 0;
    for (int it = 0; it < m; ++it) {
        if (it == m - 1 && lim)
            hipLaunchKernelGGL((k_qgrad_tiled<true, true>), g, b, lds1, s.stream, K, c.xy, c.off,
                               c.tile_pts, c.lnbr, c.tile_off, c.tile_idx, c.tile_hmax, c.geom,
                               c.comp, s.active, s.q, s.qx[cur], s.qy[cur],
                               keep ? s.qx[1 - cur] : nullptr, keep ? s.qy[1 - cur] : nullptr,
                               s.qxl, s.qyl);
        else
            hipLaunchKernelGGL((k_qgrad_tiled<true, false>), g, b, lds1, s.stream, K, c.xy, c.off,
                               c.tile_pts, c.lnbr, c.tile_off, c.tile_idx, c.tile_hmax, c.geom,
                               c.comp, s.active, s.q, s.qx[cur], s.qy[cur], s.qx[1 - cur],
                               s.qy[1 - cur], nullptr, nullptr);
        cur = 1 - cur;
    }
    s.qsel = cur;
}

hipError_t launch_q_derivatives(State& s, bool keep_unlimited) {
    if (s.qgrad_tiled && s.cloud->ntile > 0) {
        qgrad_tiled(s, keep_unlimited);
        return hipGetLastError();
    }
    switch (s.qgrad_lanes) {
        case 1: qgrad_lanes<1>(s, keep_unlimited); break;
        case 2: qgrad_lanes<2>(s, keep_unlimited); break;
        case 8: qgrad_lanes<8>(s, keep_unlimited); break;
        default: qgrad_lanes<4>(s, keep_unlimited); break;
    }
    return hipGetLastError();
}

// In colour order the first forward phase (no lower neighbours) is done by the
// residual kernel and the first backward phase (no upper neighbours: dU = dU*)
// is skipped.
static int fused_first_colour(const State& s) { return s.prm.order == 0 && s.prm.scheme == 0; }

template <bool MIXED, int LANES>
static void residual_lanes(State& s, bool in_step) {
    const Cloud& c = *s.cloud;
    const unsigned nb = grid_for(c.n * LANES);
    hipLaunchKernelGGL((k_residual<MIXED, LANES>), dim3(nb), dim3(kBlock), 0, s.stream, c.n,
                       s.prm.gamma, s.cfl, c.xy, c.frame, c.type, c.off, c.idx, c.geom, c.comp,
                       s.active, s.U, s.q, s.prm.limiter ? s.qxl : s.qx[s.qsel],
                       s.prm.limiter ? s.qyl : s.qy[s.qsel], s.R, s.D, s.jv0, s.jv2, s.jv0f,
                       s.jv2f, s.Df, s.rr, s.flags, s.prm.variant,
                       s.prm.jvp_mode, s.dU, s.dUf, s.Rs, c.colour,
                       in_step && fused_first_colour(s), s.prm.farfield, s.vinf);
}

template <bool MIXED>
static void residual_t(State& s, bool in_step) {
    switch (s.residual_lanes) {
        case 1: residual_lanes<MIXED, 1>(s, in_step); break;
        case 2: residual_lanes<MIXED, 2>(s, in_step); break;
        case 8: residual_lanes<MIXED, 8>(s, in_step); break;
        default: residual_lanes<MIXED, 4>(s, in_step); break;
    }
}

hipError_t launch_residual(State& s, int slot, bool in_step) {
    (void)slot;
    if (s.prm.precision == 1)
        residual_t<true>(s, in_step);
    else
        residual_t<false>(s, in_step);
    return hipGetLastError();
}

hipError_t launch_norm(State& s, int slot) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_norm_partial, dim3(c.nchunk), dim3(kBlock), 0, s.stream, s.rr,
                       c.chunk_start, c.chunk_comp, s.active, s.partial);
    hipLaunchKernelGGL(k_norm_comp, dim3(c.ncomp), dim3(64), 0, s.stream, s.partial,
                       c.comp_chunk_off, c.comp_inv_active, s.tol_abs, s.active, s.status, s.iters,
                       s.res_last, s.res_hist + (size_t)slot * c.ncomp);
    return hipGetLastError();
}

hipError_t launch_reset_components(State& s) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_reset_components, dim3((c.ncomp + 63) / 64), dim3(64), 0, s.stream,
                       c.ncomp, s.active, s.status, s.iters);
    return hipGetLastError();
}

// The phases of a sweep as ranges of the colour-sorted points: one per
// colour (Algorithm 6), or per (point type, colour) with wall, interior and
// outer points in turn (Algorithm 5); colours ascending forward, descending
// backward.
static std::vector<std::pair<int32_t, int32_t>> sweep_phases(const State& s, bool forward) {
    const Cloud& c = *s.cloud;
    std::vector<std::pair<int32_t, int32_t>> ph;
    const int C = c.ncolour;
    if (s.prm.order == 0) {
        for (int k = fused_first_colour(s) ? 1 : 0; k < C; ++k) {
            const int col = forward ? k : C - 1 - k;
            ph.emplace_back(c.h_col_off[col], c.h_col_off[col + 1] - c.h_col_off[col]);
        }
        return ph;
    }
    for (int g = 0; g < 3; ++g)
        for (int k = 0; k < C; ++k) {
            const int col = forward ? k : C - 1 - k;
            const int32_t a = c.h_grp_off[3 * col + g], b = c.h_grp_off[3 * col + g + 1];
            ph.emplace_back(a, b - a);
        }
    return ph;
}

// The sweep-list weights in the sweep arithmetic's precision.
template <class T>
static const W2<T>* list_weights(const D2* w, const F2* wf) {
    if constexpr (std::is_same_v<T, float>) return wf;
    else return w;
}

template <class T, int MODE, int LANES>
static void sweep_lanes(State& s, bool forward, const Vec4<T>* jv0, const Vec4<T>* jv2,
                        const T* Dg, Vec4<T>* dU) {
    const Cloud& c = *s.cloud;
    for (const auto& [start, cnt] : sweep_phases(s, forward)) {
        if (!cnt) continue;
        const dim3 g(grid_for((int64_t)cnt * LANES)), b(kBlock);
        if (forward)
            hipLaunchKernelGGL((k_sweep<T, true, MODE, LANES>), g, b, 0, s.stream, start, cnt,
                               c.col_perm, c.frame, c.type, c.lo_off, c.lo_idx,
                               list_weights<T>(c.lo_w, c.lo_wf), c.lo_code, c.comp, s.active,
                               jv0, jv2, s.U, s.prm.variant ? s.Rs : s.R, Dg, dU,
                               s.prm.gamma, s.prm.farfield);
        else
            hipLaunchKernelGGL((k_sweep<T, false, MODE, LANES>), g, b, 0, s.stream, start, cnt,
                               c.col_perm, c.frame, c.type, c.up_off, c.up_idx,
                               list_weights<T>(c.up_w, c.up_wf), c.up_code, c.comp, s.active,
                               jv0, jv2, s.U, s.R, Dg, dU, s.prm.gamma, s.prm.farfield);
    }
}

template <class T, int MODE>
static void sweep_t(State& s, bool forward, const Vec4<T>* jv0, const Vec4<T>* jv2,
                    const T* Dg, Vec4<T>* dU) {
    switch (s.sweep_lanes) {
        case 1: sweep_lanes<T, MODE, 1>(s, forward, jv0, jv2, Dg, dU); break;
        case 2: sweep_lanes<T, MODE, 2>(s, forward, jv0, jv2, Dg, dU); break;
        case 8: sweep_lanes<T, MODE, 8>(s, forward, jv0, jv2, Dg, dU); break;
        case 16: sweep_lanes<T, MODE, 16>(s, forward, jv0, jv2, Dg, dU); break;
        default: sweep_lanes<T, MODE, 4>(s, forward, jv0, jv2, Dg, dU); break;
    }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_zero4(int64_t n, Vec4<T>* __restrict__ v) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) v[p] = {T(0), T(0), T(0), T(0)};
}

hipError_t launch_sweep_dir(State& s, bool forward) {
    const Cloud& c = *s.cloud;
    // Algorithm 5 reads increments of points not yet visited in the forward
    // sweep: they start the sweep at zero (a kernel, so that graphs replay it)
    if (forward && s.prm.order == 1) {
        if (s.prm.precision == 1)
            hipLaunchKernelGGL(k_zero4<float>, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n,
                               s.dUf);
        else
            hipLaunchKernelGGL(k_zero4<double>, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream,
                               c.n, s.dU);
    }
    if (s.prm.precision == 1)
        sweep_t<float, 0>(s, forward, s.jv0f, s.jv2f, s.Df, s.dUf);
    else if (s.prm.jvp_mode == 1)
        sweep_t<double, 1>(s, forward, s.jv0, s.jv2, s.D, s.dU);
    else
        sweep_t<double, 0>(s, forward, s.jv0, s.jv2, s.D, s.dU);
    return hipGetLastError();
}

hipError_t launch_sweeps(State& s) {
    hipError_t e = launch_sweep_dir(s, true);
    if (e != hipSuccess) return e;
    return launch_sweep_dir(s, false);
}

hipError_t launch_explicit_update(State& s) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_explicit_update, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n,
                       s.prm.gamma, s.cfl, c.type, c.geom, c.comp, s.active, s.R, s.U, s.q,
                       s.flags, s.prm.farfield);
    return hipGetLastError();
}

hipError_t launch_update(State& s) {
    const Cloud& c = *s.cloud;
    if (s.prm.precision == 1)
        hipLaunchKernelGGL(k_update<float>, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n,
                           s.prm.gamma, s.U, s.dUf, c.comp, s.active, s.q, s.flags);
    else
        hipLaunchKernelGGL(k_update<double>, dim3(grid_for(c.n)), dim3(kBlock), 0, s.stream, c.n,
                           s.prm.gamma, s.U, s.dU, c.comp, s.active, s.q, s.flags);
    return hipGetLastError();
}

hipError_t launch_forces(State& s) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_forces, dim3(c.ncomp), dim3(kBlock), 0, s.stream, c.wall_list,
                       c.wall_off, c.comp_orient, c.xy, s.U, s.prm.gamma, s.fsum);
    return hipGetLastError();
}

hipError_t launch_soa_to_aos(const double* soa, D4* aos, int64_t n, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_soa_to_aos, dim3(grid_for(n)), dim3(kBlock), 0, st, soa, aos, n);
    return hipGetLastError();
}

hipError_t launch_aos_to_soa(const D4* aos, double* soa, int64_t n, hipStream_t st) {
    if (n)
        hipLaunchKernelGGL(k_aos_to_soa<double>, dim3(grid_for(n)), dim3(kBlock), 0, st, aos, soa, n);
    return hipGetLastError();
}

hipError_t launch_aosf_to_soa(const F4* aos, double* soa, int64_t n, hipStream_t st) {
    if (n)
        hipLaunchKernelGGL(k_aos_to_soa<float>, dim3(grid_for(n)), dim3(kBlock), 0, st, aos, soa, n);
    return hipGetLastError();
}

hipError_t launch_clear_flags(int32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, st, flags);
    return hipGetLastError();
}

__global__ void k_fill(int n, double v, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = v;
}

hipError_t launch_fill(double* p, int n, double v, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, n, v, p);
    return hipGetLastError();
}

__global__ void k_residual_out(const double* __restrict__ res, const int32_t* __restrict__ flags,
                               double* __restrict__ out) {
    if (threadIdx.x == 0) {
        out[0] = res[0];
        out[1] = flags[0] ? 1.0 : 0.0;
    }
}

hipError_t launch_residual_out(const double* res, const int32_t* flags, double* out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_residual_out, dim3(1), dim3(64), 0, st, res, flags, out);
    return hipGetLastError();
}

__global__ void k_copy_flag(const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
    if (threadIdx.x == 0) dst[0] = src[0];
}

hipError_t launch_copy_flag(const int32_t* src, int32_t* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_flag, dim3(1), dim3(64), 0, st, src, dst);
    return hipGetLastError();
}

hipError_t reset_cfl(State& s) {
    const int nc = s.cloud->ncomp;
    hipLaunchKernelGGL(k_fill, dim3((nc + 255) / 256), dim3(256), 0, s.stream, nc, s.prm.cfl,
                       s.cfl);
    return hipGetLastError();
}

hipError_t clear_increment(State& s, int64_t p0, int64_t n) {
    if (n <= 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(s.dU + p0, 0, n * sizeof(D4), s.stream);
    if (e == hipSuccess) e = hipMemsetAsync(s.dUf + p0, 0, n * sizeof(F4), s.stream);
    return e;
}

}  // namespace lskum
