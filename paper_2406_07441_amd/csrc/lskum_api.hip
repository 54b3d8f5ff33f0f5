// Host side of the MI355X LSKUM library: the C ABI of include/lskum.h.
//
// Cloud creation validates the CSR, colours the points (Algorithm 4) and
// uploads geometry; a state owns the device work arrays of one flow
// condition.  lskum_solve captures check_every iterations in one HIP graph
// and replays it, reading back only the residual norms between replays.
#include "../../include/lskum.h"
#include "lskum_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

struct lskum_cloud {
    lskum::Cloud c;
};
struct lskum_state {
    lskum::State s;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? LSKUM_ERR_OOM : LSKUM_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

void free_cloud(lskum::Cloud& c) {
    (void)hipFree(c.xy);
    (void)hipFree(c.frame);
    (void)hipFree(c.type);
    (void)hipFree(c.off);
    (void)hipFree(c.idx);
    (void)hipFree(c.colour);
    (void)hipFree(c.col_perm);
    (void)hipFree(c.wall_list);
    (void)hipFree(c.geom);
    (void)hipFree(c.lo_off);
    (void)hipFree(c.lo_idx);
    (void)hipFree(c.up_off);
    (void)hipFree(c.up_idx);
    c = lskum::Cloud{};
}

// Greedy point colouring of Algorithm 4.  Colours are 0-based.  The first
// point takes colour 0; each point i in storage order visits its neighbours
// in CSR order and gives every uncoloured one the smallest colour not used
// among that neighbour's own neighbours.  Points never reached (no edges)
// are coloured the same way afterwards, in storage order.
int32_t greedy_colouring(int64_t n, const int32_t* off, const int32_t* idx,
                         std::vector<int32_t>& col) {
    col.assign(n, -1);
    if (n == 0) return 0;
    std::vector<int64_t> stamp;  // stamp[k] == p  <=>  colour k is taken near p
    auto assign = [&](int64_t p) {
        for (int32_t e = off[p]; e < off[p + 1]; ++e) {
            const int32_t k = col[idx[e]];
            if (k < 0) continue;
            if ((size_t)k >= stamp.size()) stamp.resize(k + 1, -1);
            stamp[k] = p;
        }
        int32_t k = 0;
        while ((size_t)k < stamp.size() && stamp[k] == p) ++k;
        col[p] = k;
    };
    col[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = off[i]; e < off[i + 1]; ++e)
            if (col[idx[e]] < 0) assign(idx[e]);
    for (int64_t i = 0; i < n; ++i)
        if (col[i] < 0) assign(i);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i) nc = std::max(nc, col[i] + 1);
    return nc;
}

// CSR checks: offsets monotone, indices in range, no self edge, symmetric.
int validate_csr(int64_t n, const int32_t* off, const int32_t* idx) {
    if (off[0] != 0) return fail(LSKUM_ERR_CONNECTIVITY, "nbr_off[0] must be 0");
    for (int64_t p = 0; p < n; ++p)
        if (off[p + 1] < off[p]) return fail(LSKUM_ERR_CONNECTIVITY, "nbr_off not monotone");
    const int64_t nnz = off[n];
    std::vector<int64_t> indeg(n + 1, 0);
    for (int64_t p = 0; p < n; ++p)
        for (int32_t e = off[p]; e < off[p + 1]; ++e) {
            const int32_t i = idx[e];
            if (i < 0 || i >= n)
                return fail(LSKUM_ERR_CONNECTIVITY, "neighbour index out of range at point " +
                                                        std::to_string(p));
            if (i == p)
                return fail(LSKUM_ERR_CONNECTIVITY, "self edge at point " + std::to_string(p));
            ++indeg[i + 1];
        }
    for (int64_t p = 0; p < n; ++p) indeg[p + 1] += indeg[p];
    std::vector<int32_t> tr(nnz);
    std::vector<int64_t> pos(indeg.begin(), indeg.end() - 1);
    for (int64_t p = 0; p < n; ++p)
        for (int32_t e = off[p]; e < off[p + 1]; ++e) tr[pos[idx[e]]++] = (int32_t)p;
    std::vector<int32_t> a, b;
    for (int64_t p = 0; p < n; ++p) {
        if (indeg[p + 1] - indeg[p] != off[p + 1] - off[p])
            return fail(LSKUM_ERR_CONNECTIVITY, "connectivity not symmetric at point " +
                                                    std::to_string(p));
        a.assign(idx + off[p], idx + off[p + 1]);
        b.assign(tr.begin() + indeg[p], tr.begin() + indeg[p + 1]);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b)
            return fail(LSKUM_ERR_CONNECTIVITY, "connectivity not symmetric at point " +
                                                    std::to_string(p));
        if (std::adjacent_find(a.begin(), a.end()) != a.end())
            return fail(LSKUM_ERR_CONNECTIVITY, "duplicate neighbour at point " +
                                                    std::to_string(p));
    }
    return LSKUM_OK;
}

void free_state(lskum::State& s) {
    if (s.graph) (void)hipGraphExecDestroy(s.graph);
    if (s.have_events)
        for (hipEvent_t ev : s.ev) (void)hipEventDestroy(ev);
    void* ptrs[] = {s.U,   s.q,    s.qx[0], s.qx[1], s.qy[0], s.qy[1], s.R,    s.dU,
                    s.jv0, s.jv1,  s.jv2,   s.D,     s.jv0f,  s.jv1f,  s.jv2f, s.dUf,
                    s.Df,  s.partial, s.res_hist, s.flags};
    for (void* p : ptrs) (void)hipFree(p);
    if (s.own_stream && s.stream) (void)hipStreamDestroy(s.stream);
}

int check_params(const lskum_params* p) {
    if (!p) return fail(LSKUM_ERR_ARG, "params is NULL");
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || p->inner_iters < 0 || p->inner_iters > 64 ||
        (p->jvp_mode != 0 && p->jvp_mode != 1) || (p->precision != 0 && p->precision != 1) ||
        p->check_every < 1 || p->check_every > 4096 || p->max_iters < 0 || !(p->tol_rel >= 0.0))
        return fail(LSKUM_ERR_ARG, "invalid lskum_params");
    auto lanes_ok = [](int l) { return l == 0 || l == 1 || l == 2 || l == 4 || l == 8; };
    if (!lanes_ok(p->sweep_lanes) || !lanes_ok(p->residual_lanes) || p->reserved != 0)
        return fail(LSKUM_ERR_ARG, "lanes must be 0, 1, 2, 4 or 8 and reserved 0");
    if (p->precision == 1 && p->jvp_mode == 1)
        return fail(LSKUM_ERR_ARG, "mixed precision supports the exact Jacobian products only");
    return LSKUM_OK;
}

lskum::Params to_params(const lskum_params* p) {
    return lskum::Params{p->gamma,       p->cfl,         p->inner_iters, p->jvp_mode,
                         p->precision,   p->check_every, p->tol_rel,     p->max_iters,
                         p->sweep_lanes, p->residual_lanes};
}

// Lanes per point: the caller's choice, else 8 for the latency-bound sweeps
// and 2 for the compute-bound residual (measured best on the 163,840-point
// transonic cloud, FP64 and mixed).
void apply_lanes(lskum::State& s) {
    s.sweep_lanes = s.prm.sweep_lanes ? s.prm.sweep_lanes : 8;
    s.residual_lanes = s.prm.residual_lanes ? s.prm.residual_lanes : 2;
}

int read_flags(lskum::State& s, int32_t* h) {
    HIPCHK(hipMemcpyAsync(h, s.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    return LSKUM_OK;
}

// Enqueues one iteration; the residual norm goes to res_hist[slot].
int enqueue_step(lskum::State& s, int slot) {
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, slot));
    HIPCHK(lskum::launch_norm(s, slot));
    HIPCHK(lskum::launch_sweeps(s));
    HIPCHK(lskum::launch_update(s));
    s.have_dU = true;
    return LSKUM_OK;
}

int copy_field_out(lskum::State& s, const lskum::D4* src, double* dst, int on_device) {
    const int64_t n = s.cloud->n;
    if (on_device) {
        HIPCHK(lskum::launch_aos_to_soa(src, dst, n, s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
        return LSKUM_OK;
    }
    std::vector<lskum::D4> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), src, n * sizeof(lskum::D4), hipMemcpyDeviceToHost, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    for (int64_t p = 0; p < n; ++p) {
        dst[p] = h[p].x;
        dst[n + p] = h[p].y;
        dst[2 * n + p] = h[p].z;
        dst[3 * n + p] = h[p].w;
    }
    return LSKUM_OK;
}

}  // namespace

extern "C" {

const char* lskum_last_error(void) { return g_err.c_str(); }

void lskum_default_params(lskum_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1.4;
    p->cfl = 100.0;
    p->inner_iters = 1;
    p->jvp_mode = LSKUM_JVP_EXACT;
    p->precision = LSKUM_FP64;
    p->check_every = 10;
    p->tol_rel = 1e-8;
    p->max_iters = 20000;
}

int lskum_cloud_create(int64_t n, const double* x, const double* y, const int8_t* type,
                       const double* tx, const double* ty, const int32_t* nbr_off,
                       const int32_t* nbr_idx, const int32_t* colour, lskum_cloud** out) {
    g_err.clear();
    if (!out) return fail(LSKUM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n <= 0 || n >= (int64_t)1 << 31) return fail(LSKUM_ERR_ARG, "n out of range");
    if (!x || !y || !type || !nbr_off || !nbr_idx) return fail(LSKUM_ERR_ARG, "NULL array");
    int64_t nwall = 0, nact = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (type[p] < 0 || type[p] > 2) return fail(LSKUM_ERR_ARG, "invalid point type");
        nwall += type[p] == 0;
        nact += type[p] != 2;
        if (!std::isfinite(x[p]) || !std::isfinite(y[p]))
            return fail(LSKUM_ERR_ARG, "non-finite coordinate");
    }
    if (nwall && (!tx || !ty)) return fail(LSKUM_ERR_ARG, "wall points need a frame");
    int st = validate_csr(n, nbr_off, nbr_idx);
    if (st) return st;
    const int64_t nnz = nbr_off[n];

    lskum_cloud* cl = new (std::nothrow) lskum_cloud();
    if (!cl) return fail(LSKUM_ERR_OOM, "host allocation");
    lskum::Cloud& c = cl->c;
    c.n = n;
    c.nnz = nnz;
    c.n_wall = nwall;
    c.n_active = nact;
    (void)hipGetDevice(&c.device);

    // colours
    if (colour) {
        c.h_colour.assign(colour, colour + n);
        int32_t nc = 0;
        for (int64_t p = 0; p < n; ++p) {
            if (colour[p] < 0) {
                delete cl;
                return fail(LSKUM_ERR_COLOURING, "negative colour");
            }
            nc = std::max(nc, colour[p] + 1);
            for (int32_t e = nbr_off[p]; e < nbr_off[p + 1]; ++e)
                if (colour[nbr_idx[e]] == colour[p]) {
                    delete cl;
                    return fail(LSKUM_ERR_COLOURING, "edge inside a colour at point " +
                                                         std::to_string(p));
                }
        }
        c.ncolour = nc;
    } else {
        c.ncolour = greedy_colouring(n, nbr_off, nbr_idx, c.h_colour);
    }
    c.h_col_off.assign(c.ncolour + 1, 0);
    for (int64_t p = 0; p < n; ++p) ++c.h_col_off[c.h_colour[p] + 1];
    for (int32_t k = 0; k < c.ncolour; ++k) c.h_col_off[k + 1] += c.h_col_off[k];
    std::vector<int32_t> perm(n), fill(c.h_col_off.begin(), c.h_col_off.end() - 1);
    for (int64_t p = 0; p < n; ++p) perm[fill[c.h_colour[p]]++] = (int32_t)p;

    // wall polygon (storage order) and its orientation
    std::vector<int32_t> wall;
    wall.reserve(nwall);
    for (int64_t p = 0; p < n; ++p)
        if (type[p] == 0) wall.push_back((int32_t)p);
    double area2 = 0.0;
    for (size_t j = 0; j < wall.size(); ++j) {
        const int32_t a = wall[j], b = wall[(j + 1) % wall.size()];
        area2 += x[a] * y[b] - x[b] * y[a];
    }
    c.wall_orient = area2 >= 0.0 ? 1.0 : -1.0;

    // lower/upper colour neighbour lists (CSR order kept)
    std::vector<int32_t> lo_off(n + 1, 0), up_off(n + 1, 0), lo_idx, up_idx;
    lo_idx.reserve(nnz / 2 + 1);
    up_idx.reserve(nnz / 2 + 1);
    for (int64_t p = 0; p < n; ++p) {
        for (int32_t e = nbr_off[p]; e < nbr_off[p + 1]; ++e) {
            const int32_t i = nbr_idx[e];
            if (c.h_colour[i] < c.h_colour[p]) lo_idx.push_back(i);
            else up_idx.push_back(i);
        }
        lo_off[p + 1] = (int32_t)lo_idx.size();
        up_off[p + 1] = (int32_t)up_idx.size();
    }

    std::vector<lskum::D2> hxy(n), hfr(n);
    for (int64_t p = 0; p < n; ++p) {
        hxy[p] = {x[p], y[p]};
        if (type[p] == 0) {
            const double nrm = std::hypot(tx[p], ty[p]);
            if (!(std::fabs(nrm - 1.0) < 1e-6)) {
                delete cl;
                return fail(LSKUM_ERR_ARG, "wall tangent is not a unit vector");
            }
            hfr[p] = {tx[p], ty[p]};
        } else {
            hfr[p] = {1.0, 0.0};
        }
    }

    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    chk(dalloc(&c.xy, n));
    chk(dalloc(&c.frame, n));
    chk(dalloc(&c.type, n));
    chk(dalloc(&c.off, n + 1));
    chk(dalloc(&c.idx, nnz));
    chk(dalloc(&c.colour, n));
    chk(dalloc(&c.col_perm, n));
    chk(dalloc(&c.wall_list, wall.size()));
    chk(dalloc(&c.geom, n));
    chk(dalloc(&c.lo_off, n + 1));
    chk(dalloc(&c.up_off, n + 1));
    chk(dalloc(&c.lo_idx, lo_idx.size()));
    chk(dalloc(&c.up_idx, up_idx.size()));
    if (e == hipSuccess) {
        chk(hipMemcpy(c.xy, hxy.data(), n * sizeof(lskum::D2), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.frame, hfr.data(), n * sizeof(lskum::D2), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.type, type, n, hipMemcpyHostToDevice));
        chk(hipMemcpy(c.off, nbr_off, (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.idx, nbr_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.colour, c.h_colour.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.col_perm, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.lo_off, lo_off.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c.up_off, up_off.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
        if (!lo_idx.empty())
            chk(hipMemcpy(c.lo_idx, lo_idx.data(), lo_idx.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        if (!up_idx.empty())
            chk(hipMemcpy(c.up_idx, up_idx.data(), up_idx.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        if (!wall.empty())
            chk(hipMemcpy(c.wall_list, wall.data(), wall.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    }
    if (e == hipSuccess) {
        hipError_t pe = lskum::launch_precompute(c, nullptr);
        if (pe == hipErrorInvalidValue) {
            free_cloud(c);
            delete cl;
            return fail(LSKUM_ERR_DEGENERATE, "a point's full stencil has a singular LS matrix");
        }
        chk(pe);
    }
    if (e != hipSuccess) {
        int r = hip_fail(e, "lskum_cloud_create");
        free_cloud(c);
        delete cl;
        return r;
    }
    *out = cl;
    return LSKUM_OK;
}

int lskum_cloud_info(const lskum_cloud* cl, int64_t* n, int64_t* nnz, int32_t* n_colours,
                     int64_t* n_degenerate) {
    if (!cl) return fail(LSKUM_ERR_ARG, "cloud is NULL");
    if (n) *n = cl->c.n;
    if (nnz) *nnz = cl->c.nnz;
    if (n_colours) *n_colours = cl->c.ncolour;
    if (n_degenerate) *n_degenerate = cl->c.n_degenerate;
    return LSKUM_OK;
}

int lskum_cloud_colours(const lskum_cloud* cl, int32_t* colour_out) {
    if (!cl || !colour_out) return fail(LSKUM_ERR_ARG, "NULL argument");
    std::memcpy(colour_out, cl->c.h_colour.data(), cl->c.n * sizeof(int32_t));
    return LSKUM_OK;
}

void lskum_cloud_destroy(lskum_cloud* cl) {
    if (!cl) return;
    free_cloud(cl->c);
    delete cl;
}

int lskum_state_create(const lskum_cloud* cl, double mach, double aoa_deg,
                       const lskum_params* prm, void* hip_stream, lskum_state** out) {
    g_err.clear();
    if (!cl || !out) return fail(LSKUM_ERR_ARG, "NULL argument");
    *out = nullptr;
    int st = check_params(prm);
    if (st) return st;
    if (!(mach > 0.0) || !std::isfinite(aoa_deg)) return fail(LSKUM_ERR_ARG, "invalid flow condition");
    lskum_state* so = new (std::nothrow) lskum_state();
    if (!so) return fail(LSKUM_ERR_OOM, "host allocation");
    lskum::State& s = so->s;
    s.cloud = &cl->c;
    s.prm = to_params(prm);
    apply_lanes(s);
    s.mach = mach;
    s.aoa_deg = aoa_deg;
    s.stream = (hipStream_t)hip_stream;
    if (!s.stream) {
        // a private stream of default priority: graph capture needs a non-legacy stream
        hipError_t se = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (se != hipSuccess) {
            delete so;
            return hip_fail(se, "hipStreamCreateWithFlags");
        }
        s.own_stream = true;
    }
    const int64_t n = cl->c.n;
    s.partial_cap = (int)((n + 255) / 256) * 8 + 2;  // residual blocks at 8 lanes per point
    s.res_cap = 4096;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    chk(dalloc(&s.U, n));
    chk(dalloc(&s.q, n));
    for (int k = 0; k < 2; ++k) {
        chk(dalloc(&s.qx[k], n));
        chk(dalloc(&s.qy[k], n));
    }
    chk(dalloc(&s.R, n));
    chk(dalloc(&s.dU, n));
    chk(dalloc(&s.jv0, n));
    chk(dalloc(&s.jv1, n));
    chk(dalloc(&s.jv2, n));
    chk(dalloc(&s.D, n));
    chk(dalloc(&s.jv0f, n));
    chk(dalloc(&s.jv1f, n));
    chk(dalloc(&s.jv2f, n));
    chk(dalloc(&s.dUf, n));
    chk(dalloc(&s.Df, n));
    chk(dalloc(&s.partial, s.partial_cap));
    chk(dalloc(&s.res_hist, s.res_cap));
    chk(dalloc(&s.flags, 4));
    if (e == hipSuccess) chk(lskum::launch_clear_flags(s.flags, s.stream));
    if (e == hipSuccess) chk(lskum::launch_free_stream(s));
    if (e == hipSuccess) chk(lskum::launch_q_from_U(s));
    if (e != hipSuccess) {
        int r = hip_fail(e, "lskum_state_create");
        free_state(s);
        delete so;
        return r;
    }
    // residual of the free-stream state: the anchor of the relative tolerance
    if (int r = lskum_residual(so, nullptr, 0, &s.res_fs)) {
        free_state(s);
        delete so;
        return r;
    }
    *out = so;
    return LSKUM_OK;
}

void lskum_state_destroy(lskum_state* so) {
    if (!so) return;
    (void)hipStreamSynchronize(so->s.stream);
    free_state(so->s);
    delete so;
}

int lskum_state_set_params(lskum_state* so, const lskum_params* prm) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    int st = check_params(prm);
    if (st) return st;
    lskum::State& s = so->s;
    const lskum::Params np = to_params(prm);
    // the captured iteration depends on everything but the stopping rule
    const bool same_kernels = np.gamma == s.prm.gamma && np.cfl == s.prm.cfl &&
                              np.inner_iters == s.prm.inner_iters &&
                              np.jvp_mode == s.prm.jvp_mode && np.precision == s.prm.precision;
    if (s.graph && !same_kernels) {
        (void)hipGraphExecDestroy(s.graph);
        s.graph = nullptr;
    }
    const bool same_lanes = np.sweep_lanes == s.prm.sweep_lanes &&
                            np.residual_lanes == s.prm.residual_lanes;
    if (s.graph && !same_lanes) {
        (void)hipGraphExecDestroy(s.graph);
        s.graph = nullptr;
    }
    if (np.precision != s.prm.precision) s.have_dU = false;
    s.prm = np;
    apply_lanes(s);
    return LSKUM_OK;
}

int lskum_state_set_U(lskum_state* so, const double* U, int on_device) {
    if (!so || !U) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    const int64_t n = s.cloud->n;
    if (on_device) {
        HIPCHK(lskum::launch_soa_to_aos(U, s.U, n, s.stream));
    } else {
        std::vector<lskum::D4> h(n);
        for (int64_t p = 0; p < n; ++p) h[p] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]};
        HIPCHK(hipMemcpyAsync(s.U, h.data(), n * sizeof(lskum::D4), hipMemcpyHostToDevice,
                              s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
    }
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_q_from_U(s));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    s.have_dU = false;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "state has rho <= 0 or p <= 0");
    return LSKUM_OK;
}

int lskum_state_get_U(lskum_state* so, double* U, int on_device) {
    if (!so || !U) return fail(LSKUM_ERR_ARG, "NULL argument");
    return copy_field_out(so->s, so->s.U, U, on_device);
}

int lskum_state_get_dU(lskum_state* so, double* dU, int on_device) {
    if (!so || !dU) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    if (!s.have_dU) return fail(LSKUM_ERR_ARG, "no step has been taken");
    if (s.prm.precision == 1) {
        const int64_t n = s.cloud->n;
        if (on_device) {
            HIPCHK(lskum::launch_aosf_to_soa(s.dUf, dU, n, s.stream));
            HIPCHK(hipStreamSynchronize(s.stream));
            return LSKUM_OK;
        }
        std::vector<lskum::F4> h(n);
        HIPCHK(hipMemcpyAsync(h.data(), s.dUf, n * sizeof(lskum::F4), hipMemcpyDeviceToHost,
                              s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
        for (int64_t p = 0; p < n; ++p) {
            dU[p] = h[p].x;
            dU[n + p] = h[p].y;
            dU[2 * n + p] = h[p].z;
            dU[3 * n + p] = h[p].w;
        }
        return LSKUM_OK;
    }
    return copy_field_out(s, s.dU, dU, on_device);
}

int lskum_q_derivatives(lskum_state* so, double* qx, double* qy, int on_device) {
    if (!so || !qx || !qy) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    HIPCHK(lskum::launch_q_derivatives(s));
    if (int r = copy_field_out(s, s.qx[s.qsel], qx, on_device)) return r;
    return copy_field_out(s, s.qy[s.qsel], qy, on_device);
}

int lskum_residual(lskum_state* so, double* R, int on_device, double* res) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    lskum::State& s = so->s;
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(lskum::launch_norm(s, 0));
    if (R)
        if (int r = copy_field_out(s, s.R, R, on_device)) return r;
    double hres = 0.0;
    HIPCHK(hipMemcpyAsync(&hres, s.res_hist, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    if (res) *res = hres;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical reconstructed state (beta <= 0)");
    return LSKUM_OK;
}

int lskum_lusgs_step(lskum_state* so, double* res) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    lskum::State& s = so->s;
    if (res) HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    if (int r = enqueue_step(s, 0)) return r;
    if (!res) return LSKUM_OK;
    HIPCHK(hipMemcpyAsync(res, s.res_hist, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical state in the step");
    return LSKUM_OK;
}

int lskum_step_timed(lskum_state* so, double* ms) {
    if (!so || !ms) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    if (!s.have_events) {
        for (hipEvent_t& ev : s.ev) HIPCHK(hipEventCreate(&ev));
        s.have_events = true;
    }
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(hipEventRecord(s.ev[0], s.stream));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(hipEventRecord(s.ev[1], s.stream));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(hipEventRecord(s.ev[2], s.stream));
    HIPCHK(lskum::launch_norm(s, 0));
    HIPCHK(hipEventRecord(s.ev[3], s.stream));
    HIPCHK(lskum::launch_sweep_dir(s, true));
    HIPCHK(hipEventRecord(s.ev[4], s.stream));
    HIPCHK(lskum::launch_sweep_dir(s, false));
    HIPCHK(hipEventRecord(s.ev[5], s.stream));
    HIPCHK(lskum::launch_update(s));
    HIPCHK(hipEventRecord(s.ev[6], s.stream));
    HIPCHK(hipEventSynchronize(s.ev[6]));
    s.have_dU = true;
    for (int k = 0; k < 6; ++k) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, s.ev[k], s.ev[k + 1]));
        ms[k] = t;
    }
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical state in the step");
    return LSKUM_OK;
}

int lskum_solve(lskum_state* so, lskum_report* rep) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    lskum::State& s = so->s;
    const int K = std::min(s.prm.check_every, s.res_cap);
    const double tol = s.prm.tol_rel * s.res_fs;
    lskum_report r{};
    r.res_fs = s.res_fs;
    r.status = LSKUM_OK;
    if (!s.graph || s.graph_iters != K) {
        if (s.graph) (void)hipGraphExecDestroy(s.graph);
        s.graph = nullptr;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
        int cap = LSKUM_OK;
        for (int j = 0; j < K && cap == LSKUM_OK; ++j) cap = enqueue_step(s, j);
        hipError_t ce = hipStreamEndCapture(s.stream, &g);
        if (cap) return cap;
        HIPCHK(ce);
        hipError_t ie = hipGraphInstantiate(&s.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ie);
        s.graph_iters = K;
    }
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    std::vector<double> hist(K);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    bool conv = false;
    while (it < s.prm.max_iters) {
        int32_t f = 0;
        int done;
        if (it + K <= s.prm.max_iters) {
            HIPCHK(hipGraphLaunch(s.graph, s.stream));
            done = K;
        } else {
            done = s.prm.max_iters - it;
            for (int j = 0; j < done; ++j)
                if (int e = enqueue_step(s, j)) return e;
        }
        HIPCHK(hipMemcpyAsync(hist.data(), s.res_hist, done * sizeof(double),
                              hipMemcpyDeviceToHost, s.stream));
        HIPCHK(hipMemcpyAsync(&f, s.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
        if (it == 0) r.res_first = hist[0];
        it += done;
        r.res_final = hist[done - 1];
        if (f) {
            r.status = LSKUM_ERR_NONPHYSICAL;
            break;
        }
        if (!std::isfinite(r.res_final)) {
            r.status = LSKUM_ERR_NONPHYSICAL;
            break;
        }
        for (int j = 0; j < done; ++j)
            if (hist[j] <= tol) conv = true;
        if (conv) break;
    }
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    r.iters = it;
    s.have_dU = true;
    if (r.status == LSKUM_OK && !conv) r.status = LSKUM_ERR_NOT_CONVERGED;
    if (r.status != LSKUM_ERR_NONPHYSICAL) {
        double cl = 0, cd = 0;
        if (s.cloud->n_wall >= 3 && lskum_forces(so, &cl, &cd) == LSKUM_OK) {
            r.cl = cl;
            r.cd = cd;
        }
    }
    if (rep) *rep = r;
    if (r.status == LSKUM_ERR_NOT_CONVERGED)
        return fail(LSKUM_ERR_NOT_CONVERGED, "max_iters reached");
    if (r.status == LSKUM_ERR_NONPHYSICAL) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical state");
    return LSKUM_OK;
}

int lskum_forces(lskum_state* so, double* cl, double* cd) {
    if (!so || !cl || !cd) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    if (s.cloud->n_wall < 3) return fail(LSKUM_ERR_ARG, "cloud has fewer than 3 wall points");
    // partial[] is free between steps; use its first two slots for the sum
    HIPCHK(lskum::launch_forces(s, s.partial));
    double f[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(f, s.partial, sizeof(f), hipMemcpyDeviceToHost, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    const double a = s.aoa_deg * 3.14159265358979323846 / 180.0;
    const double qinf = 0.5 * s.mach * s.mach;
    *cl = (f[1] * std::cos(a) - f[0] * std::sin(a)) / qinf;
    *cd = (f[0] * std::cos(a) + f[1] * std::sin(a)) / qinf;
    return LSKUM_OK;
}

}  // extern "C"
