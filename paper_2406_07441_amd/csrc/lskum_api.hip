// Host side of the MI355X LSKUM library: the C ABI of include/lskum.h.
//
// Cloud creation validates the CSR, colours the points (Algorithm 4) and
// uploads geometry; a state owns the device work arrays of one flow
// condition.  A batch is a state over the disjoint union of one copy of a
// cloud per flow condition ("components"): every kernel of an iteration --
// including each colour phase of the sweeps -- is then one launch over all
// conditions, and converged conditions retire on the device.  lskum_solve and
// lskum_batch_solve capture check_every iterations in one HIP graph and replay
// it, reading back only a few bytes of bookkeeping between replays.
#include "../../include/lskum.h"
#include "lskum_internal.h"
#include "lskum_tiles.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

constexpr double kPi = 3.14159265358979323846;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? LSKUM_ERR_OOM : LSKUM_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                      \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

template <class T>
hipError_t upload(T* dst, const T* src, size_t count) {
    if (count == 0) return hipSuccess;
    return hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice);
}

void free_cloud(lskum::Cloud& c) {
    void* ptrs[] = {c.xy,     c.frame,     c.type,   c.off,      c.idx,      c.colour,
                    c.col_perm, c.wall_list, c.geom, c.lo_off,   c.lo_idx,   c.up_off,
                    c.up_idx, c.lo_w,      c.up_w,     c.lo_code,  c.up_code,  c.comp,
                    c.lo_wf, c.up_wf,
                    c.comp_off, c.wall_off, c.comp_inv_active,
                    c.comp_orient, c.chunk_start, c.chunk_comp, c.comp_chunk_off,
                    c.tile_pts, c.tile_off, c.tile_idx, c.lnbr};
    for (void* p : ptrs) (void)hipFree(p);
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

// Device upload of a (possibly multi-component) cloud whose host arrays are
// filled in c.h_*: colour permutation, lower/upper colour neighbour lists,
// wall list, per-component tables, then the geometry precompute kernel.
int upload_cloud(lskum::Cloud& c) {
    const int64_t n = c.n, nnz = c.nnz;
    c.ncolour = 0;
    for (int64_t p = 0; p < n; ++p) c.ncolour = std::max(c.ncolour, c.h_colour[p] + 1);
    // colour-sorted points, by point type (wall, interior, outer) within a
    // colour and by index within that: colour c, type g occupies
    // [h_grp_off[3c + g], h_grp_off[3c + g + 1])
    c.h_grp_off.assign(3 * (size_t)c.ncolour + 1, 0);
    for (int64_t p = 0; p < n; ++p) ++c.h_grp_off[3 * c.h_colour[p] + c.h_type[p] + 1];
    for (size_t k = 0; k + 1 < c.h_grp_off.size(); ++k) c.h_grp_off[k + 1] += c.h_grp_off[k];
    c.h_col_off.assign(c.ncolour + 1, 0);
    for (int32_t k = 0; k <= c.ncolour; ++k) c.h_col_off[k] = c.h_grp_off[3 * k];
    std::vector<int32_t> perm(n), fill(c.h_grp_off.begin(), c.h_grp_off.end() - 1);
    for (int64_t p = 0; p < n; ++p) perm[fill[3 * c.h_colour[p] + c.h_type[p]]++] = (int32_t)p;

    // sweep lists in colour-sorted point order
    std::vector<int32_t> lo_off(n + 1, 0), up_off(n + 1, 0), lo_idx, up_idx;
    lo_idx.reserve(nnz / 2 + 1);
    up_idx.reserve(nnz / 2 + 1);
    for (int64_t q = 0; q < n; ++q) {
        const int32_t p = perm[q];
        for (int32_t e = c.h_off[p]; e < c.h_off[p + 1]; ++e) {
            const int32_t i = c.h_idx[e];
            if (c.h_colour[i] < c.h_colour[p]) lo_idx.push_back(i);
            else up_idx.push_back(i);
        }
        lo_off[q + 1] = (int32_t)lo_idx.size();
        up_off[q + 1] = (int32_t)up_idx.size();
    }

    // wall list per component (storage order) and polygon orientation
    std::vector<int32_t> wall;
    std::vector<int32_t> comp_off32(c.ncomp + 1), wall_off32(c.ncomp + 1);
    c.h_wall_off.assign(c.ncomp + 1, 0);
    c.h_comp_orient.assign(c.ncomp, 1.0);
    c.h_comp_active.assign(c.ncomp, 0);
    c.h_comp_inv_active.assign(c.ncomp, 0.0);
    for (int32_t k = 0; k < c.ncomp; ++k) {
        const size_t w0 = wall.size();
        int64_t act = 0;
        for (int64_t p = c.h_comp_off[k]; p < c.h_comp_off[k + 1]; ++p) {
            if (c.h_type[p] == 0) wall.push_back((int32_t)p);
            act += c.h_type[p] != 2;
        }
        double area2 = 0.0;
        const size_t m = wall.size() - w0;
        for (size_t j = 0; j < m; ++j) {
            const int32_t a = wall[w0 + j], b = wall[w0 + (j + 1) % m];
            area2 += c.h_x[a] * c.h_y[b] - c.h_x[b] * c.h_y[a];
        }
        c.h_comp_orient[k] = area2 >= 0.0 ? 1.0 : -1.0;
        c.h_wall_off[k + 1] = (int64_t)wall.size();
        c.h_comp_active[k] = act;
        c.h_comp_inv_active[k] = act ? 1.0 / (double)act : 0.0;
    }
    for (int32_t k = 0; k <= c.ncomp; ++k) {
        comp_off32[k] = (int32_t)c.h_comp_off[k];
        wall_off32[k] = (int32_t)c.h_wall_off[k];
    }
    c.n_wall = (int64_t)wall.size();
    c.wall_orient = c.h_comp_orient[0];
    c.n_active = 0;
    for (int64_t a : c.h_comp_active) c.n_active += a;

    // wall and outer points keep their frame; outer points use it with the
    // kinetic far field only, which needs a unit tangent at every one of them
    // q-derivative tiles: runs of consecutive points or blocks of rows,
    // whichever stages fewer points
    lskum::TileSet tiles =
        lskum::build_tiles(n, c.h_off.data(), c.h_idx.data(), c.h_comp_off, lskum::kQTile,
                           lskum::kQTileJ, lskum::kQTileK, lskum::kQTileMax);
    c.ntile = (int32_t)tiles.ntile;
    c.tile_hmax = tiles.hmax;

    std::vector<lskum::D2> hxy(n), hfr(n);
    c.outer_frames = true;
    for (int64_t p = 0; p < n; ++p) {
        hxy[p] = {c.h_x[p], c.h_y[p]};
        hfr[p] = {1.0, 0.0};
        if (c.h_type[p] == 0) {
            hfr[p] = {c.h_tx[p], c.h_ty[p]};
        } else if (c.h_type[p] == 2) {
            if (std::fabs(std::hypot(c.h_tx[p], c.h_ty[p]) - 1.0) < 1e-6)
                hfr[p] = {c.h_tx[p], c.h_ty[p]};
            else
                c.outer_frames = false;
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
    if (c.ntile) {
        chk(dalloc(&c.tile_pts, tiles.pts.size()));
        chk(dalloc(&c.tile_off, tiles.off.size()));
        chk(dalloc(&c.tile_idx, std::max<size_t>(1, tiles.list.size())));
        chk(dalloc(&c.lnbr, std::max<size_t>(1, tiles.lnbr.size())));
    }
    chk(dalloc(&c.lo_off, n + 1));
    chk(dalloc(&c.up_off, n + 1));
    chk(dalloc(&c.lo_idx, lo_idx.size()));
    chk(dalloc(&c.up_idx, up_idx.size()));
    chk(dalloc(&c.lo_w, lo_idx.size()));
    chk(dalloc(&c.up_w, up_idx.size()));
    chk(dalloc(&c.lo_wf, lo_idx.size()));
    chk(dalloc(&c.up_wf, up_idx.size()));
    chk(dalloc(&c.lo_code, lo_idx.size()));
    chk(dalloc(&c.up_code, up_idx.size()));
    chk(dalloc(&c.comp_off, c.ncomp + 1));
    chk(dalloc(&c.wall_off, c.ncomp + 1));
    chk(dalloc(&c.comp_inv_active, c.ncomp));
    chk(dalloc(&c.comp_orient, c.ncomp));
    // reduction chunks of at most 1024 points, never straddling components
    constexpr int64_t kChunk = 1024;
    std::vector<int32_t> chunk_start, chunk_comp, comp_chunk_off(c.ncomp + 1, 0);
    for (int32_t k = 0; k < c.ncomp; ++k) {
        for (int64_t p = c.h_comp_off[k]; p < c.h_comp_off[k + 1]; p += kChunk) {
            chunk_start.push_back((int32_t)p);
            chunk_comp.push_back(k);
        }
        comp_chunk_off[k + 1] = (int32_t)chunk_comp.size();
    }
    chunk_start.push_back((int32_t)n);
    c.nchunk = (int32_t)chunk_comp.size();
    chk(dalloc(&c.chunk_start, chunk_start.size()));
    chk(dalloc(&c.chunk_comp, chunk_comp.size()));
    chk(dalloc(&c.comp_chunk_off, comp_chunk_off.size()));
    std::vector<int32_t> comp;
    if (c.ncomp > 1) {
        comp.resize(n);
        for (int32_t k = 0; k < c.ncomp; ++k)
            for (int64_t p = c.h_comp_off[k]; p < c.h_comp_off[k + 1]; ++p) comp[p] = k;
        chk(dalloc(&c.comp, n));
    }
    if (e == hipSuccess) {
        chk(upload(c.xy, hxy.data(), n));
        chk(upload(c.frame, hfr.data(), n));
        chk(upload(c.type, c.h_type.data(), n));
        chk(upload(c.off, c.h_off.data(), n + 1));
        chk(upload(c.idx, c.h_idx.data(), nnz));
        chk(upload(c.colour, c.h_colour.data(), n));
        chk(upload(c.col_perm, perm.data(), n));
        if (c.ntile) {
            chk(upload(c.tile_pts, tiles.pts.data(), tiles.pts.size()));
            chk(upload(c.tile_off, tiles.off.data(), tiles.off.size()));
            chk(upload(c.tile_idx, tiles.list.data(), tiles.list.size()));
            chk(upload(c.lnbr, tiles.lnbr.data(), tiles.lnbr.size()));
        }
        chk(upload(c.lo_off, lo_off.data(), n + 1));
        chk(upload(c.up_off, up_off.data(), n + 1));
        chk(upload(c.lo_idx, lo_idx.data(), lo_idx.size()));
        chk(upload(c.up_idx, up_idx.data(), up_idx.size()));
        chk(upload(c.wall_list, wall.data(), wall.size()));
        chk(upload(c.comp_off, comp_off32.data(), c.ncomp + 1));
        chk(upload(c.wall_off, wall_off32.data(), c.ncomp + 1));
        chk(upload(c.comp_inv_active, c.h_comp_inv_active.data(), c.ncomp));
        chk(upload(c.comp_orient, c.h_comp_orient.data(), c.ncomp));
        if (c.comp) chk(upload(c.comp, comp.data(), n));
        chk(upload(c.chunk_start, chunk_start.data(), chunk_start.size()));
        chk(upload(c.chunk_comp, chunk_comp.data(), chunk_comp.size()));
        chk(upload(c.comp_chunk_off, comp_chunk_off.data(), comp_chunk_off.size()));
    }
    if (e == hipSuccess) {
        hipError_t pe = lskum::launch_precompute(c, nullptr);
        if (pe == hipErrorInvalidValue)
            return fail(LSKUM_ERR_DEGENERATE, "a point's full stencil has a singular LS matrix");
        chk(pe);
    }
    if (e == hipSuccess) {
        chk(lskum::launch_sweep_weights(c, nullptr));
        if (e == hipSuccess) chk(hipStreamSynchronize(nullptr));
    }
    if (e != hipSuccess) return hip_fail(e, "cloud upload");
    return LSKUM_OK;
}

void free_state(lskum::State& s) {
    if (s.graph) (void)hipGraphExecDestroy(s.graph);
    if (s.have_events)
        for (hipEvent_t ev : s.ev) (void)hipEventDestroy(ev);
    void* ptrs[] = {s.U,    s.q,      s.qx[0], s.qx[1],  s.qy[0],   s.qy[1],    s.qxl, s.Rs,
                    s.qyl,  s.R,      s.dU,    s.jv0,    s.jv2,      s.D,
                    s.jv0f, s.jv2f,  s.dUf,    s.Df,      s.rr,       s.fsum, s.partial,
                    s.res_hist, s.flags, s.active, s.status, s.iters, s.res_last, s.tol_abs, s.cfl,
                    s.vinf};
    for (void* p : ptrs) (void)hipFree(p);
    if (s.own_stream && s.stream) (void)hipStreamDestroy(s.stream);
    s = lskum::State{};
}

constexpr const char* kNoOuterFrame =
    "the kinetic far field needs a unit tangent (tx, ty) at every outer point";

int check_params(const lskum_params* p) {
    if (!p) return fail(LSKUM_ERR_ARG, "params is NULL");
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || p->inner_iters < 0 || p->inner_iters > 64 ||
        (p->jvp_mode != 0 && p->jvp_mode != 1) || (p->precision != 0 && p->precision != 1) ||
        p->check_every < 1 || p->check_every > 4096 || p->max_iters < 0 || !(p->tol_rel >= 0.0))
        return fail(LSKUM_ERR_ARG, "invalid lskum_params");
    auto lanes_ok = [](int l) { return l == 0 || l == 1 || l == 2 || l == 4 || l == 8; };
    if (!(lanes_ok(p->sweep_lanes) || p->sweep_lanes == 16) || !lanes_ok(p->residual_lanes))
        return fail(LSKUM_ERR_ARG, "lanes must be 0, 1, 2, 4 or 8 (16 for the sweeps)");
    if ((p->limiter != 0 && p->limiter != 1) || !(p->limiter_k > 0.0))
        return fail(LSKUM_ERR_ARG, "limiter must be 0 or 1 with limiter_k > 0");
    if (p->order != 0 && p->order != 1)
        return fail(LSKUM_ERR_ARG, "order must be LSKUM_ORDER_COLOUR or LSKUM_ORDER_WALL_FIRST");
    if (p->scheme != 0 && p->scheme != 1)
        return fail(LSKUM_ERR_ARG, "scheme must be LSKUM_IMPLICIT or LSKUM_EXPLICIT");
    if (p->variant != 0 && p->variant != 1)
        return fail(LSKUM_ERR_ARG, "variant must be LSKUM_ANANDH or LSKUM_MANISH");
    if (p->precision == 1 && p->jvp_mode == 1)
        return fail(LSKUM_ERR_ARG, "mixed precision supports the exact Jacobian products only");
    if (!lanes_ok(p->qgrad_lanes))
        return fail(LSKUM_ERR_ARG, "qgrad_lanes must be 0, 1, 2, 4 or 8");
    if (p->farfield != 0 && p->farfield != 1)
        return fail(LSKUM_ERR_ARG,
                    "farfield must be LSKUM_FARFIELD_DIRICHLET or LSKUM_FARFIELD_KINETIC");
    return LSKUM_OK;
}

lskum::Params to_params(const lskum_params* p) {
    return lskum::Params{p->gamma,       p->cfl,            p->inner_iters, p->jvp_mode,
                         p->precision,   p->check_every,    p->tol_rel,     p->max_iters,
                         p->sweep_lanes, p->residual_lanes, p->limiter,     p->limiter_k,
                         p->variant,     p->scheme,         p->order,       p->farfield,
                         p->qgrad_lanes};
}

// Lanes per point: the caller's choice, else 8 for the latency-bound sweeps
// and 2 for the compute-bound residual (measured best on the 163,840-point
// transonic cloud, FP64 and mixed).
void apply_lanes(lskum::State& s) {
    s.sweep_lanes = s.prm.sweep_lanes ? s.prm.sweep_lanes : 8;
    s.residual_lanes = s.prm.residual_lanes ? s.prm.residual_lanes : 2;
    s.qgrad_tiled = s.prm.qgrad_lanes == 0;
    s.qgrad_lanes = s.prm.qgrad_lanes ? s.prm.qgrad_lanes : 4;
}

int read_flags(lskum::State& s, int32_t* h) {
    HIPCHK(hipMemcpyAsync(h, s.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    return LSKUM_OK;
}

// Enqueues one iteration; component residual norms go to res_hist[slot][k].
int enqueue_step(lskum::State& s, int slot) {
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, slot, true));
    HIPCHK(lskum::launch_norm(s, slot));
    if (s.prm.scheme == 1) {
        HIPCHK(lskum::launch_explicit_update(s));
        s.have_dU = false;
        return LSKUM_OK;
    }
    HIPCHK(lskum::launch_sweeps(s));
    HIPCHK(lskum::launch_update(s));
    s.have_dU = true;
    return LSKUM_OK;
}

// Sets the per-component retirement tolerances (0 disables retirement).
int set_tolerances(lskum::State& s, bool on) {
    const int nc = s.cloud->ncomp;
    std::vector<double> tol(nc, 0.0);
    if (on)
        for (int k = 0; k < nc; ++k) tol[k] = s.prm.tol_rel * s.h_res_fs[k];
    HIPCHK(hipMemcpyAsync(s.tol_abs, tol.data(), nc * sizeof(double), hipMemcpyHostToDevice,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    return LSKUM_OK;
}

int copy_field_out(lskum::State& s, const lskum::D4* src, int64_t p0, int64_t n, double* dst,
                   int on_device) {
    if (on_device) {
        HIPCHK(lskum::launch_aos_to_soa(src + p0, dst, n, s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
        return LSKUM_OK;
    }
    std::vector<lskum::D4> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), src + p0, n * sizeof(lskum::D4), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    for (int64_t p = 0; p < n; ++p) {
        dst[p] = h[p].x;
        dst[n + p] = h[p].y;
        dst[2 * n + p] = h[p].z;
        dst[3 * n + p] = h[p].w;
    }
    return LSKUM_OK;
}

// Allocates and initialises the device arrays of a state over cloud c with
// per-component flow conditions; U starts at the free stream.
int init_state(lskum::State& s, const lskum::Cloud& c, const lskum_params* prm,
               const std::vector<double>& mach, const std::vector<double>& aoa,
               void* hip_stream) {
    s.cloud = &c;
    s.prm = to_params(prm);
    apply_lanes(s);
    s.h_mach = mach;
    s.h_aoa = aoa;
    s.mach = mach[0];
    s.aoa_deg = aoa[0];
    s.stream = (hipStream_t)hip_stream;
    if (!s.stream) {
        // a private stream of default priority: graph capture needs a non-legacy stream
        HIPCHK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
        s.own_stream = true;
    }
    const int64_t n = c.n;
    const int nc = c.ncomp;
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
    chk(dalloc(&s.qxl, n));
    chk(dalloc(&s.qyl, n));
    chk(dalloc(&s.R, n));
    chk(dalloc(&s.Rs, n));
    chk(dalloc(&s.dU, n));
    chk(dalloc(&s.jv0, n));
    chk(dalloc(&s.jv2, n));
    chk(dalloc(&s.D, n));
    chk(dalloc(&s.jv0f, n));
    chk(dalloc(&s.jv2f, n));
    chk(dalloc(&s.dUf, n));
    chk(dalloc(&s.Df, n));
    chk(dalloc(&s.rr, n));
    chk(dalloc(&s.fsum, 2 * nc));
    chk(dalloc(&s.partial, c.nchunk));
    chk(dalloc(&s.res_hist, (size_t)s.res_cap * nc));
    chk(dalloc(&s.flags, 4));
    chk(dalloc(&s.active, nc));
    chk(dalloc(&s.status, nc));
    chk(dalloc(&s.iters, nc));
    chk(dalloc(&s.res_last, nc));
    chk(dalloc(&s.tol_abs, nc));
    chk(dalloc(&s.cfl, nc));
    chk(dalloc(&s.vinf, 2 * nc));
    if (e != hipSuccess) return hip_fail(e, "state allocation");
    std::vector<double> vinf(2 * nc), zero(nc, 0.0);
    for (int k = 0; k < nc; ++k) {
        const double a = aoa[k] * kPi / 180.0;
        vinf[2 * k] = mach[k] * std::cos(a);
        vinf[2 * k + 1] = mach[k] * std::sin(a);
    }
    HIPCHK(hipMemcpyAsync(s.vinf, vinf.data(), 2 * nc * sizeof(double), hipMemcpyHostToDevice,
                          s.stream));
    HIPCHK(hipMemcpyAsync(s.tol_abs, zero.data(), nc * sizeof(double), hipMemcpyHostToDevice,
                          s.stream));
    HIPCHK(lskum::reset_cfl(s));
    s.h_cfl.assign(nc, s.prm.cfl);
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_free_stream(s));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(lskum::clear_increment(s, 0, n));
    // residual norms of the free-stream state: the anchors of the relative tolerance
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(lskum::launch_norm(s, 0));
    s.h_res_fs.assign(nc, 0.0);
    HIPCHK(hipMemcpyAsync(s.h_res_fs.data(), s.res_hist, nc * sizeof(double),
                          hipMemcpyDeviceToHost, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(hipStreamSynchronize(s.stream));
    s.res_fs = s.h_res_fs[0];
    return LSKUM_OK;
}

// Host-side bookkeeping of a graph-replayed solve over all components.
struct SolveOut {
    std::vector<int32_t> status, iters;
    std::vector<double> res_last, seconds;
    double total = 0.0;
    int iters_run = 0;
    bool any_flag = false;
};

// One window step of the CFL control after `done` more iterations, from the
// components' last residuals `rl` and activity `act`; uploads changed CFL
// numbers (they take effect from the next iteration on).
int cfl_control_step(lskum::State& s, lskum::CflControl& ctl, int done,
                     const std::vector<double>& rl, const std::vector<int32_t>& act) {
    const int nc = (int)rl.size();
    for (int k = 0; k < nc; ++k)
        if (act[k] && rl[k] < ctl.best_cur[k]) ctl.best_cur[k] = rl[k];
    ctl.since += done;
    if (ctl.since < ctl.window) return LSKUM_OK;
    bool changed = false;
    for (int k = 0; k < nc; ++k) {
        if (!act[k] || ctl.best_cur[k] < ctl.best_prev[k]) continue;  // progress
        const double c = std::max(ctl.cfl_min, s.h_cfl[k] * ctl.factor);
        if (c < s.h_cfl[k]) {
            s.h_cfl[k] = c;
            ++ctl.cuts[k];
            changed = true;
        }
    }
    ctl.best_prev = ctl.best_cur;
    ctl.best_cur.assign(nc, HUGE_VAL);
    ctl.since = 0;
    if (changed) {
        HIPCHK(hipMemcpyAsync(s.cfl, s.h_cfl.data(), nc * sizeof(double), hipMemcpyHostToDevice,
                              s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
    }
    return LSKUM_OK;
}

int run_solve(lskum::State& s, SolveOut& out, lskum::CflControl* ctl = nullptr) {
    const int nc = s.cloud->ncomp;
    if (ctl && ctl->window <= 0) ctl = nullptr;
    std::vector<double> rl(ctl ? nc : 0);
    const int K = std::min(s.prm.check_every, s.res_cap);
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
    if (int r = set_tolerances(s, true)) return r;
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(hipStreamSynchronize(s.stream));
    out.status.assign(nc, 0);
    out.iters.assign(nc, 0);
    out.res_last.assign(nc, 0.0);
    out.seconds.assign(nc, 0.0);
    std::vector<int32_t> act(nc, 1);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    while (it < s.prm.max_iters) {
        int32_t f = 0;
        int done = K;
        if (it + K <= s.prm.max_iters) {
            HIPCHK(hipGraphLaunch(s.graph, s.stream));
        } else {
            done = s.prm.max_iters - it;
            for (int j = 0; j < done; ++j)
                if (int e = enqueue_step(s, j)) return e;
        }
        it += done;
        HIPCHK(hipMemcpyAsync(act.data(), s.active, nc * sizeof(int32_t), hipMemcpyDeviceToHost,
                              s.stream));
        HIPCHK(hipMemcpyAsync(&f, s.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream));
        if (ctl)
            HIPCHK(hipMemcpyAsync(rl.data(), s.res_last, nc * sizeof(double),
                                  hipMemcpyDeviceToHost, s.stream));
        HIPCHK(hipStreamSynchronize(s.stream));
        if (ctl)
            if (int r = cfl_control_step(s, *ctl, done, rl, act)) return r;
        const double now =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        int live = 0;
        for (int k = 0; k < nc; ++k) {
            if (act[k]) ++live;
            else if (out.seconds[k] == 0.0) out.seconds[k] = now;
        }
        if (f) out.any_flag = true;
        if (!live) break;
    }
    s.have_dU = true;
    out.iters_run = it;
    out.total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nc; ++k)
        if (out.seconds[k] == 0.0) out.seconds[k] = out.total;
    HIPCHK(hipMemcpyAsync(out.status.data(), s.status, nc * sizeof(int32_t), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipMemcpyAsync(out.iters.data(), s.iters, nc * sizeof(int32_t), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipMemcpyAsync(out.res_last.data(), s.res_last, nc * sizeof(double),
                          hipMemcpyDeviceToHost, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    if (int r = set_tolerances(s, false)) return r;
    HIPCHK(lskum::launch_reset_components(s));
    return LSKUM_OK;
}

int forces_all(lskum::State& s, std::vector<double>& cl, std::vector<double>& cd) {
    const lskum::Cloud& c = *s.cloud;
    const int nc = c.ncomp;
    HIPCHK(lskum::launch_forces(s));
    std::vector<double> f(2 * nc);
    HIPCHK(hipMemcpyAsync(f.data(), s.fsum, 2 * nc * sizeof(double), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    cl.assign(nc, 0.0);
    cd.assign(nc, 0.0);
    for (int k = 0; k < nc; ++k) {
        if (c.h_wall_off[k + 1] - c.h_wall_off[k] < 3) continue;
        const double a = s.h_aoa[k] * kPi / 180.0;
        const double qinf = 0.5 * s.h_mach[k] * s.h_mach[k];
        cl[k] = (f[2 * k + 1] * std::cos(a) - f[2 * k] * std::sin(a)) / qinf;
        cd[k] = (f[2 * k] * std::cos(a) + f[2 * k + 1] * std::sin(a)) / qinf;
    }
    return LSKUM_OK;
}

void fill_report(lskum_report& r, const lskum::State& s, const SolveOut& o, int k) {
    r.iters = o.iters[k];
    r.res_fs = s.h_res_fs[k];
    r.res_final = o.res_last[k];
    r.seconds = o.seconds[k];
    r.status = o.status[k] == 1
                   ? LSKUM_OK
                   : (o.status[k] == -1 ? LSKUM_ERR_NONPHYSICAL : LSKUM_ERR_NOT_CONVERGED);
}

}  // namespace

int lskum::api_error(int code, const std::string& msg) { return fail(code, msg); }

int lskum::api_check_params(const lskum_params* p) { return check_params(p); }

lskum::Params lskum::api_params(const lskum_params* p) { return to_params(p); }

void lskum::api_clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// Residual without allocation: lskum_residual_noalloc works in `scratch`, a
// file-scope device array that every GPU holds once, for the life of the
// process.  Its device address is taken with hipGetSymbolAddress on the first
// call on each device (the array's name is only a host-side handle); calls on
// one device share it, so overlapping calls race.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// bytes per point of the scratch layout below, and the fixed part
constexpr size_t kNoallocPerPoint = 11 * sizeof(lskum::D4) + 2 * sizeof(double);
constexpr size_t kNoallocFixed = (size_t)1 << 20;

int scratch_ptr(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(LSKUM_ERR_ARG, "device index out of range");
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "scratch symbol address");
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return LSKUM_OK;
}

// carves 256-byte aligned arrays out of a byte range
struct Carver {
    unsigned char* p;
    template <class T>
    T* take(size_t count) {
        T* r = reinterpret_cast<T*>(p);
        p += (count * sizeof(T) + 255) & ~(size_t)255;
        return r;
    }
};

}  // namespace

extern "C" {

const char* lskum_last_error(void) { return g_err.c_str(); }

#ifndef LSKUM_BUILD_HASH
#define LSKUM_BUILD_HASH "unknown"
#endif
const char* lskum_build_hash(void) { return LSKUM_BUILD_HASH; }

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
    p->limiter = 0;
    p->limiter_k = 5.0;
    p->variant = LSKUM_ANANDH;
    p->scheme = LSKUM_IMPLICIT;
    p->order = LSKUM_ORDER_COLOUR;
    p->farfield = LSKUM_FARFIELD_DIRICHLET;
}

int lskum_cloud_create(int64_t n, const double* x, const double* y, const int8_t* type,
                       const double* tx, const double* ty, const int32_t* nbr_off,
                       const int32_t* nbr_idx, const int32_t* colour, lskum_cloud** out) {
    g_err.clear();
    if (!out) return fail(LSKUM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n <= 0 || n >= (int64_t)1 << 31) return fail(LSKUM_ERR_ARG, "n out of range");
    if (!x || !y || !type || !nbr_off || !nbr_idx) return fail(LSKUM_ERR_ARG, "NULL array");
    int64_t nwall = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (type[p] < 0 || type[p] > 2) return fail(LSKUM_ERR_ARG, "invalid point type");
        nwall += type[p] == 0;
        if (!std::isfinite(x[p]) || !std::isfinite(y[p]))
            return fail(LSKUM_ERR_ARG, "non-finite coordinate");
    }
    if (nwall && (!tx || !ty)) return fail(LSKUM_ERR_ARG, "wall points need a frame");
    for (int64_t p = 0; p < n && nwall; ++p)
        if (type[p] == 0 && !(std::fabs(std::hypot(tx[p], ty[p]) - 1.0) < 1e-6))
            return fail(LSKUM_ERR_ARG, "wall tangent is not a unit vector");
    int st = validate_csr(n, nbr_off, nbr_idx);
    if (st) return st;
    const int64_t nnz = nbr_off[n];

    lskum_cloud* cl = new (std::nothrow) lskum_cloud();
    if (!cl) return fail(LSKUM_ERR_OOM, "host allocation");
    lskum::Cloud& c = cl->c;
    c.n = n;
    c.nnz = nnz;
    (void)hipGetDevice(&c.device);
    if (colour) {
        for (int64_t p = 0; p < n; ++p) {
            if (colour[p] < 0) {
                delete cl;
                return fail(LSKUM_ERR_COLOURING, "negative colour");
            }
            for (int32_t e = nbr_off[p]; e < nbr_off[p + 1]; ++e)
                if (colour[nbr_idx[e]] == colour[p]) {
                    delete cl;
                    return fail(LSKUM_ERR_COLOURING, "edge inside a colour at point " +
                                                         std::to_string(p));
                }
        }
        c.h_colour.assign(colour, colour + n);
    } else {
        greedy_colouring(n, nbr_off, nbr_idx, c.h_colour);
    }
    c.h_x.assign(x, x + n);
    c.h_y.assign(y, y + n);
    c.h_type.assign(type, type + n);
    c.h_tx.assign(n, 1.0);
    c.h_ty.assign(n, 0.0);
    if (tx && ty) {
        c.h_tx.assign(tx, tx + n);
        c.h_ty.assign(ty, ty + n);
    }
    c.h_off.assign(nbr_off, nbr_off + n + 1);
    c.h_idx.assign(nbr_idx, nbr_idx + nnz);
    c.ncomp = 1;
    c.h_comp_off = {0, n};
    if (int r = upload_cloud(c)) {
        free_cloud(c);
        delete cl;
        return r;
    }
    if (!tx || !ty) {  // no frames given: outer points have none either
        for (int64_t p = 0; p < n; ++p) c.outer_frames &= type[p] != 2;
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
    if (prm->farfield && !cl->c.outer_frames) return fail(LSKUM_ERR_ARG, kNoOuterFrame);
    if (!(mach > 0.0) || !std::isfinite(aoa_deg)) return fail(LSKUM_ERR_ARG, "invalid flow condition");
    lskum_state* so = new (std::nothrow) lskum_state();
    if (!so) return fail(LSKUM_ERR_OOM, "host allocation");
    if (int r = init_state(so->s, cl->c, prm, {mach}, {aoa_deg}, hip_stream)) {
        free_state(so->s);
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
    if (prm->farfield && !s.cloud->outer_frames) return fail(LSKUM_ERR_ARG, kNoOuterFrame);
    const lskum::Params np = to_params(prm);
    // the captured iteration depends on everything but the stopping rule
    const bool same_kernels = np.gamma == s.prm.gamma &&
                              np.inner_iters == s.prm.inner_iters &&
                              np.jvp_mode == s.prm.jvp_mode && np.precision == s.prm.precision &&
                              np.limiter == s.prm.limiter && np.limiter_k == s.prm.limiter_k &&
                              np.sweep_lanes == s.prm.sweep_lanes &&
                              np.residual_lanes == s.prm.residual_lanes &&
                              np.variant == s.prm.variant && np.scheme == s.prm.scheme &&
                              np.order == s.prm.order && np.farfield == s.prm.farfield &&
                              np.qgrad_lanes == s.prm.qgrad_lanes;
    if (s.graph && !same_kernels) {
        (void)hipGraphExecDestroy(s.graph);
        s.graph = nullptr;
    }
    if (np.precision != s.prm.precision) {
        // the lagged increment of the Manish variant lives in the sweep precision's array
        s.have_dU = false;
        HIPCHK(lskum::clear_increment(s, 0, s.cloud->n));
    }
    const bool new_cfl = np.cfl != s.prm.cfl;
    s.prm = np;
    apply_lanes(s);
    if (new_cfl) {  // per-condition values give way to the new one
        HIPCHK(lskum::reset_cfl(s));
        s.h_cfl.assign(s.cloud->ncomp, s.prm.cfl);
    }
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
    HIPCHK(lskum::clear_increment(s, 0, n));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    s.have_dU = false;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "state has rho <= 0 or p <= 0");
    return LSKUM_OK;
}

int lskum_state_get_U(lskum_state* so, double* U, int on_device) {
    if (!so || !U) return fail(LSKUM_ERR_ARG, "NULL argument");
    return copy_field_out(so->s, so->s.U, 0, so->s.cloud->n, U, on_device);
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
    return copy_field_out(s, s.dU, 0, s.cloud->n, dU, on_device);
}

int lskum_q_derivatives(lskum_state* so, double* qx, double* qy, int on_device) {
    if (!so || !qx || !qy) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_q_derivatives(s, true));
    if (int r = copy_field_out(s, s.qx[s.qsel], 0, s.cloud->n, qx, on_device)) return r;
    return copy_field_out(s, s.qy[s.qsel], 0, s.cloud->n, qy, on_device);
}

int lskum_residual(lskum_state* so, double* R, int on_device, double* res) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    lskum::State& s = so->s;
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(lskum::launch_norm(s, 0));
    if (R)
        if (int r = copy_field_out(s, s.R, 0, s.cloud->n, R, on_device)) return r;
    double hres = 0.0;
    HIPCHK(hipMemcpyAsync(&hres, s.res_hist, sizeof(double), hipMemcpyDeviceToHost, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    if (res) *res = hres;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical reconstructed state (beta <= 0)");
    return LSKUM_OK;
}

int64_t lskum_residual_noalloc_max_points(void) {
    return (int64_t)((kScratchBytes - kNoallocFixed) / kNoallocPerPoint) - 256;
}

int lskum_residual_noalloc(const lskum_cloud* cl, double mach, double aoa_deg,
                           const lskum_params* prm, const double* U, double* R, double* res,
                           void* hip_stream) {
    g_err.clear();
    if (!cl || !U || !res) return fail(LSKUM_ERR_ARG, "NULL argument");
    if (int st = check_params(prm)) return st;
    if (!(mach > 0.0) || !std::isfinite(aoa_deg)) return fail(LSKUM_ERR_ARG, "invalid flow condition");
    const lskum::Cloud& c = cl->c;
    if (prm->farfield && !c.outer_frames) return fail(LSKUM_ERR_ARG, kNoOuterFrame);
    if (c.n > lskum_residual_noalloc_max_points())
        return fail(LSKUM_ERR_ARG, "cloud has " + std::to_string(c.n) +
                                       " points, more than the allocation-free residual's "
                                       "scratch holds (" +
                                       std::to_string(lskum_residual_noalloc_max_points()) + ")");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != c.device) return fail(LSKUM_ERR_ARG, "the cloud lives on another device");
    unsigned char* base = nullptr;
    if (int r = scratch_ptr(dev, &base)) return r;

    // a state whose every array lies in scratch: fp64 arithmetic, the
    // Anandhanarayanan variant (R does not depend on either)
    lskum::State s;
    s.cloud = &c;
    s.prm = to_params(prm);
    s.prm.precision = 0;
    s.prm.variant = 0;
    s.prm.scheme = 0;
    apply_lanes(s);
    s.stream = (hipStream_t)hip_stream;
    const int64_t n = c.n;
    const int nc = c.ncomp;
    Carver cv{base};
    s.U = cv.take<lskum::D4>(n);
    s.q = cv.take<lskum::D4>(n);
    for (int k = 0; k < 2; ++k) {
        s.qx[k] = cv.take<lskum::D4>(n);
        s.qy[k] = cv.take<lskum::D4>(n);
    }
    s.qxl = cv.take<lskum::D4>(n);
    s.qyl = cv.take<lskum::D4>(n);
    s.R = cv.take<lskum::D4>(n);
    s.jv0 = cv.take<lskum::D4>(n);
    s.jv2 = cv.take<lskum::D4>(n);
    s.D = cv.take<double>(n);
    s.rr = cv.take<double>(n);
    s.partial = cv.take<double>(c.nchunk);
    s.res_hist = cv.take<double>(nc);
    s.res_last = cv.take<double>(nc);
    s.tol_abs = cv.take<double>(nc);
    s.cfl = cv.take<double>(nc);
    s.vinf = cv.take<double>(2 * nc);
    s.flags = cv.take<int32_t>(4);
    s.active = cv.take<int32_t>(nc);
    s.status = cv.take<int32_t>(nc);
    s.iters = cv.take<int32_t>(nc);
    if ((size_t)(cv.p - base) > kScratchBytes)
        return fail(LSKUM_ERR_ARG, "cloud too large for the allocation-free residual");
    const double a = aoa_deg * kPi / 180.0;
    // per-condition values by fill kernels (no memset and no host copy)
    HIPCHK(lskum::launch_fill(s.cfl, nc, s.prm.cfl, s.stream));
    HIPCHK(lskum::launch_fill(s.tol_abs, nc, 0.0, s.stream));
    for (int k = 0; k < nc; ++k) {
        HIPCHK(lskum::launch_fill(s.vinf + 2 * k, 1, mach * std::cos(a), s.stream));
        HIPCHK(lskum::launch_fill(s.vinf + 2 * k + 1, 1, mach * std::sin(a), s.stream));
    }
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_soa_to_aos(U, s.U, n, s.stream));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(lskum::launch_norm(s, 0));
    if (R) HIPCHK(lskum::launch_aos_to_soa(s.R, R, n, s.stream));
    HIPCHK(lskum::launch_residual_out(s.res_hist, s.flags, res, s.stream));
    return LSKUM_OK;
}

int lskum_lusgs_step(lskum_state* so, double* res) {
    if (!so) return fail(LSKUM_ERR_ARG, "state is NULL");
    lskum::State& s = so->s;
    HIPCHK(lskum::launch_reset_components(s));
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
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(hipEventRecord(s.ev[0], s.stream));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(hipEventRecord(s.ev[1], s.stream));
    HIPCHK(lskum::launch_residual(s, 0, true));
    HIPCHK(hipEventRecord(s.ev[2], s.stream));
    HIPCHK(lskum::launch_norm(s, 0));
    HIPCHK(hipEventRecord(s.ev[3], s.stream));
    const bool expl = s.prm.scheme == 1;
    if (!expl) HIPCHK(lskum::launch_sweep_dir(s, true));
    HIPCHK(hipEventRecord(s.ev[4], s.stream));
    if (!expl) HIPCHK(lskum::launch_sweep_dir(s, false));
    HIPCHK(hipEventRecord(s.ev[5], s.stream));
    HIPCHK(expl ? lskum::launch_explicit_update(s) : lskum::launch_update(s));
    HIPCHK(hipEventRecord(s.ev[6], s.stream));
    HIPCHK(hipEventSynchronize(s.ev[6]));
    s.have_dU = !expl;
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
    SolveOut o;
    if (int r = run_solve(s, o)) return r;
    lskum_report r{};
    fill_report(r, s, o, 0);
    r.seconds = o.total;
    if (o.any_flag && r.status == LSKUM_ERR_NOT_CONVERGED) r.status = LSKUM_ERR_NONPHYSICAL;
    // the residual of the first iteration of this solve
    HIPCHK(hipMemcpyAsync(&r.res_first, s.res_hist, sizeof(double), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    if (r.status != LSKUM_ERR_NONPHYSICAL && s.cloud->n_wall >= 3) {
        std::vector<double> cl, cd;
        if (forces_all(s, cl, cd) == LSKUM_OK) {
            r.cl = cl[0];
            r.cd = cd[0];
        }
    }
    if (rep) *rep = r;
    if (r.status == LSKUM_ERR_NOT_CONVERGED) return fail(LSKUM_ERR_NOT_CONVERGED, "max_iters reached");
    if (r.status == LSKUM_ERR_NONPHYSICAL) return fail(LSKUM_ERR_NONPHYSICAL, "non-physical state");
    return LSKUM_OK;
}

int lskum_forces(lskum_state* so, double* cl, double* cd) {
    if (!so || !cl || !cd) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = so->s;
    if (s.cloud->n_wall < 3) return fail(LSKUM_ERR_ARG, "cloud has fewer than 3 wall points");
    std::vector<double> l, d;
    if (int r = forces_all(s, l, d)) return r;
    *cl = l[0];
    *cd = d[0];
    return LSKUM_OK;
}

// ---------------------------------------------------------------------------
// Batches of flow conditions.
// ---------------------------------------------------------------------------
int lskum_batch_create(int32_t n_clouds, const lskum_cloud* const* clouds, int32_t n_cond,
                       const int32_t* cond_cloud, const double* mach, const double* aoa_deg,
                       const lskum_params* prm, void* hip_stream, lskum_batch** out) {
    g_err.clear();
    if (!out || !clouds || !cond_cloud || !mach || !aoa_deg)
        return fail(LSKUM_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (n_clouds < 1 || n_cond < 1) return fail(LSKUM_ERR_ARG, "need at least one cloud and condition");
    if (int st = check_params(prm)) return st;
    int64_t n = 0, nnz = 0;
    for (int32_t k = 0; k < n_cond; ++k) {
        if (cond_cloud[k] < 0 || cond_cloud[k] >= n_clouds || !clouds[cond_cloud[k]])
            return fail(LSKUM_ERR_ARG, "condition refers to an invalid cloud");
        if (!(mach[k] > 0.0) || !std::isfinite(aoa_deg[k]))
            return fail(LSKUM_ERR_ARG, "invalid flow condition");
        if (prm->farfield && !clouds[cond_cloud[k]]->c.outer_frames)
            return fail(LSKUM_ERR_ARG, kNoOuterFrame);
        n += clouds[cond_cloud[k]]->c.n;
        nnz += clouds[cond_cloud[k]]->c.nnz;
    }
    if (n >= (int64_t)1 << 31 || nnz >= (int64_t)1 << 31)
        return fail(LSKUM_ERR_ARG, "batch too large for 32-bit indices");
    lskum_batch* b = new (std::nothrow) lskum_batch();
    if (!b) return fail(LSKUM_ERR_OOM, "host allocation");
    lskum::Cloud& c = b->c;
    c.n = n;
    c.nnz = nnz;
    c.ncomp = n_cond;
    (void)hipGetDevice(&c.device);
    c.h_x.reserve(n);
    c.h_y.reserve(n);
    c.h_tx.reserve(n);
    c.h_ty.reserve(n);
    c.h_type.reserve(n);
    c.h_colour.reserve(n);
    c.h_off.reserve(n + 1);
    c.h_idx.reserve(nnz);
    c.h_off.push_back(0);
    c.h_comp_off.assign(1, 0);
    for (int32_t k = 0; k < n_cond; ++k) {
        const lskum::Cloud& s = clouds[cond_cloud[k]]->c;
        const int32_t base = (int32_t)c.h_x.size();
        const int32_t ebase = (int32_t)c.h_idx.size();
        c.h_x.insert(c.h_x.end(), s.h_x.begin(), s.h_x.end());
        c.h_y.insert(c.h_y.end(), s.h_y.begin(), s.h_y.end());
        c.h_tx.insert(c.h_tx.end(), s.h_tx.begin(), s.h_tx.end());
        c.h_ty.insert(c.h_ty.end(), s.h_ty.begin(), s.h_ty.end());
        c.h_type.insert(c.h_type.end(), s.h_type.begin(), s.h_type.end());
        c.h_colour.insert(c.h_colour.end(), s.h_colour.begin(), s.h_colour.end());
        for (int64_t p = 0; p < s.n; ++p) c.h_off.push_back(ebase + s.h_off[p + 1]);
        for (int32_t i : s.h_idx) c.h_idx.push_back(base + i);
        c.h_comp_off.push_back((int64_t)c.h_x.size());
    }
    b->cond_cloud.assign(cond_cloud, cond_cloud + n_cond);
    if (int r = upload_cloud(c)) {
        free_cloud(c);
        delete b;
        return r;
    }
    for (int32_t k = 0; k < n_cond; ++k) c.outer_frames &= clouds[cond_cloud[k]]->c.outer_frames;
    std::vector<double> m(mach, mach + n_cond), a(aoa_deg, aoa_deg + n_cond);
    if (int r = init_state(b->s, c, prm, m, a, hip_stream)) {
        free_state(b->s);
        free_cloud(c);
        delete b;
        return r;
    }
    *out = b;
    return LSKUM_OK;
}

int lskum_batch_info(const lskum_batch* b, int64_t* n_points, int64_t* nnz, int32_t* n_colours) {
    if (!b) return fail(LSKUM_ERR_ARG, "batch is NULL");
    if (n_points) *n_points = b->c.n;
    if (nnz) *nnz = b->c.nnz;
    if (n_colours) *n_colours = b->c.ncolour;
    return LSKUM_OK;
}

int lskum_batch_set_params(lskum_batch* b, const lskum_params* prm) {
    if (!b) return fail(LSKUM_ERR_ARG, "batch is NULL");
    lskum_state tmp;
    std::swap(tmp.s, b->s);
    int r = lskum_state_set_params(&tmp, prm);
    std::swap(tmp.s, b->s);
    return r;
}

int lskum_batch_set_cfl(lskum_batch* b, const double* cfl) {
    if (!b || !cfl) return fail(LSKUM_ERR_ARG, "NULL argument");
    lskum::State& s = b->s;
    const int nc = b->c.ncomp;
    for (int k = 0; k < nc; ++k)
        if (!(cfl[k] > 0.0) || !std::isfinite(cfl[k]))
            return fail(LSKUM_ERR_ARG, "cfl must be finite and > 0");
    HIPCHK(hipMemcpyAsync(s.cfl, cfl, nc * sizeof(double), hipMemcpyHostToDevice, s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    s.h_cfl.assign(cfl, cfl + nc);
    return LSKUM_OK;
}

int lskum_batch_get_cfl(const lskum_batch* b, double* cfl) {
    if (!b || !cfl) return fail(LSKUM_ERR_ARG, "NULL argument");
    std::copy(b->s.h_cfl.begin(), b->s.h_cfl.end(), cfl);
    return LSKUM_OK;
}

int lskum_batch_set_cfl_control(lskum_batch* b, int32_t window, double factor, double cfl_min) {
    if (!b) return fail(LSKUM_ERR_ARG, "batch is NULL");
    if (window < 0 || (window > 0 && (!(factor > 0.0) || !(factor < 1.0) || !(cfl_min > 0.0) ||
                                      !std::isfinite(cfl_min))))
        return fail(LSKUM_ERR_ARG, "need window >= 0, and 0 < factor < 1, cfl_min > 0");
    const int nc = b->c.ncomp;
    lskum::CflControl& c = b->ctl;
    c.window = window;
    c.factor = factor;
    c.cfl_min = cfl_min;
    c.since = 0;
    c.best_prev.assign(nc, HUGE_VAL);
    c.best_cur.assign(nc, HUGE_VAL);
    c.cuts.assign(nc, 0);
    return LSKUM_OK;
}

int lskum_batch_solve(lskum_batch* b, lskum_report* reps, double* seconds_total) {
    if (!b) return fail(LSKUM_ERR_ARG, "batch is NULL");
    lskum::State& s = b->s;
    SolveOut o;
    if (int r = run_solve(s, o, &b->ctl)) return r;
    std::vector<double> cl, cd;
    const bool have_forces = forces_all(s, cl, cd) == LSKUM_OK;
    const int nc = b->c.ncomp;
    int worst = LSKUM_OK;
    for (int k = 0; k < nc; ++k) {
        lskum_report r{};
        fill_report(r, s, o, k);
        if (have_forces) {
            r.cl = cl[k];
            r.cd = cd[k];
        }
        if (reps) reps[k] = r;
        if (r.status != LSKUM_OK && worst == LSKUM_OK) worst = r.status;
    }
    if (seconds_total) *seconds_total = o.total;
    if (worst != LSKUM_OK) return fail(worst, "some conditions did not converge");
    return LSKUM_OK;
}

int lskum_batch_step_timed(lskum_batch* b, double* ms) {
    if (!b) return fail(LSKUM_ERR_ARG, "batch is NULL");
    lskum_state tmp;
    std::swap(tmp.s, b->s);
    int r = lskum_step_timed(&tmp, ms);
    std::swap(tmp.s, b->s);
    return r;
}

int lskum_batch_get_U(lskum_batch* b, int32_t cond, double* U, int on_device) {
    if (!b || !U) return fail(LSKUM_ERR_ARG, "NULL argument");
    if (cond < 0 || cond >= b->c.ncomp) return fail(LSKUM_ERR_ARG, "condition out of range");
    const int64_t p0 = b->c.h_comp_off[cond], n = b->c.h_comp_off[cond + 1] - p0;
    return copy_field_out(b->s, b->s.U, p0, n, U, on_device);
}

int lskum_batch_set_U(lskum_batch* b, int32_t cond, const double* U, int on_device) {
    if (!b || !U) return fail(LSKUM_ERR_ARG, "NULL argument");
    if (cond < 0 || cond >= b->c.ncomp) return fail(LSKUM_ERR_ARG, "condition out of range");
    lskum::State& s = b->s;
    const int64_t p0 = b->c.h_comp_off[cond], n = b->c.h_comp_off[cond + 1] - p0;
    if (on_device) {
        HIPCHK(lskum::launch_soa_to_aos(U, s.U + p0, n, s.stream));
    } else {
        std::vector<lskum::D4> h(n);
        for (int64_t p = 0; p < n; ++p) h[p] = {U[p], U[n + p], U[2 * n + p], U[3 * n + p]};
        HIPCHK(hipMemcpyAsync(s.U + p0, h.data(), n * sizeof(lskum::D4), hipMemcpyHostToDevice,
                              s.stream));
    }
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(lskum::clear_increment(s, p0, n));
    int32_t f = 0;
    if (int r = read_flags(s, &f)) return r;
    if (f) return fail(LSKUM_ERR_NONPHYSICAL, "state has rho <= 0 or p <= 0");
    return LSKUM_OK;
}

// Times each candidate lane count (1, 2, 4, 8 lanes per point; 16 for the sweeps) for the sweep
// and the residual kernels on the batch itself and keeps the fastest of each.
// The batch's state is saved before and restored after the trial steps.
int lskum_batch_autotune(lskum_batch* b, int32_t iters, int32_t* sweep_lanes,
                         int32_t* residual_lanes, int32_t* qgrad_lanes) {
    if (!b || iters < 1) return fail(LSKUM_ERR_ARG, "invalid argument");
    lskum::State& s = b->s;
    std::vector<lskum::D4> saved(b->c.n);
    HIPCHK(hipMemcpyAsync(saved.data(), s.U, b->c.n * sizeof(lskum::D4), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    const lskum::Params keep = s.prm;
    // candidate k: sweep lanes cands[k], residual and direct q-derivative
    // lanes cands[k] (k < 4); the LDS-tiled q-derivative form is a sixth
    // candidate of its own
    const int cands[5] = {1, 2, 4, 8, 16};
    double best_sw = 1e300, best_rs = 1e300, best_qg = 1e300;
    int bsw = 8, brs = 2, bqg = 0;
    lskum_state tmp;
    std::swap(tmp.s, b->s);
    int rc = LSKUM_OK;
    for (int li = 0; li < 6 && rc == LSKUM_OK; ++li) {
        const bool tiles = li == 5;
        if (tiles && b->c.ntile == 0) break;
        tmp.s.prm.sweep_lanes = li < 5 ? cands[li] : bsw;
        tmp.s.prm.residual_lanes = li < 4 ? cands[li] : brs;
        tmp.s.prm.qgrad_lanes = tiles ? 0 : (li < 4 ? cands[li] : 4);
        apply_lanes(tmp.s);
        double ms[6], sw = 0, rs = 0, qg = 0;
        for (int it = 0; it < iters + 1 && rc == LSKUM_OK; ++it) {
            rc = lskum_step_timed(&tmp, ms);
            if (it == 0) continue;  // warm-up
            qg += ms[0];
            rs += ms[1];
            sw += ms[3] + ms[4];
        }
        if (li < 5 && sw < best_sw) {
            best_sw = sw;
            bsw = cands[li];
        }
        if (li < 4 && rs < best_rs) {
            best_rs = rs;
            brs = cands[li];
        }
        if ((li < 4 || tiles) && qg < best_qg) {
            best_qg = qg;
            bqg = tiles ? 0 : cands[li];
        }
    }
    std::swap(tmp.s, b->s);
    s.prm = keep;
    s.prm.sweep_lanes = bsw;
    s.prm.residual_lanes = brs;
    s.prm.qgrad_lanes = bqg;
    apply_lanes(s);
    if (s.graph) {
        (void)hipGraphExecDestroy(s.graph);
        s.graph = nullptr;
    }
    HIPCHK(hipMemcpyAsync(s.U, saved.data(), b->c.n * sizeof(lskum::D4), hipMemcpyHostToDevice,
                          s.stream));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(hipStreamSynchronize(s.stream));
    if (rc) return rc;
    if (sweep_lanes) *sweep_lanes = bsw;
    if (residual_lanes) *residual_lanes = brs;
    if (qgrad_lanes) *qgrad_lanes = bqg;
    return LSKUM_OK;
}

void lskum_batch_destroy(lskum_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->s.stream);
    free_state(b->s);
    free_cloud(b->c);
    delete b;
}

}  // extern "C"
