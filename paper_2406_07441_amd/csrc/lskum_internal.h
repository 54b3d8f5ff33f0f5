// Internal declarations shared by the device kernels and the host API of the
// MI355X LSKUM library.  Not part of the public C ABI (include/lskum.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lskum.h"

namespace lskum {

// Four-component point record (conserved vector, q-variables, ...).  One
// record per point keeps a neighbour gather to one or two wide loads.
template <class T>
struct alignas(4 * sizeof(T)) Vec4 {
    T x, y, z, w;
};
using D4 = Vec4<double>;
using F4 = Vec4<float>;

struct alignas(16) D2 {
    double x, y;
};
struct alignas(8) F2 {
    float x, y;
};
// sweep-list weights in the sweep arithmetic
template <class T>
using W2 = std::conditional_t<std::is_same_v<T, float>, F2, D2>;

// Geometry precomputed once per cloud (one record per point).
//   lsq:   inverse of the full-stencil LS normal matrix, (a11, a12, a22, rmin)
//          so that q_x = a11 bx + a12 by, q_y = a12 bx + a22 by, and rmin the
//          distance to the nearest neighbour (time-step rule).
//   split: for split k (interior x+, x-, y+, y-; wall t+, t-, n-), the
//          weight coefficients (cb, cab): w_i = cb * da_i + cab * db_i.
//   ls1:   LS_k(1), the weight sums of the four splits.
struct alignas(32) PointGeom {
    D4 lsq;
    D2 split[4];
    D4 ls1;
};

constexpr uint8_t kSwA = 1, kSwNegA = 2, kSwB = 4, kSwNegB = 8, kSwWall = 16;

// q-derivative tiles: points per tile (one per four lanes of a 256-thread
// block), the block shape for clouds stored row by row (kQTileJ points by
// kQTileK rows), and the longest neighbour list a tile may stage in LDS (the
// inner pass holds 112 bytes per listed point: at most 56 KiB)
constexpr int kQTile = 64;
constexpr int kQTileJ = 16;
constexpr int kQTileK = 4;
constexpr int kQTileMax = 512;
static_assert(kQTileJ * kQTileK <= kQTile, "a row block fits one tile");

struct Cloud {
    int device = 0;
    int64_t n = 0, nnz = 0;
    int32_t ncolour = 0;
    int64_t n_degenerate = 0;
    int64_t n_active = 0;      // non-outer points
    int64_t n_wall = 0;
    double wall_orient = 1.0;  // +1 if the wall polygon runs counter-clockwise
    bool outer_frames = true;  // every outer point has a unit tangent (kinetic far field)
    // device
    D2* xy = nullptr;          // coordinates
    D2* frame = nullptr;       // unit tangent (wall points); (1, 0) elsewhere
    int8_t* type = nullptr;
    int32_t* off = nullptr;
    int32_t* idx = nullptr;
    int32_t* colour = nullptr;
    int32_t* col_perm = nullptr;   // points sorted by colour, then index
    int32_t* wall_list = nullptr;  // wall points in storage order
    // Sweep lists: the neighbours of each point split by colour -- lower
    // colours (read by the forward sweep) and higher colours (backward) --
    // with CSR order kept, laid out in colour-sorted point order (list of the
    // point col_perm[q] at entries [lo_off[q], lo_off[q+1])), so that a colour
    // phase reads one contiguous block.  Per entry: the neighbour, the weights
    // (w_a, w_b) of the point's a-split (x+/x-, or t+/t- at a wall) and b-split
    // (y+/y-, or n- at a wall) the neighbour lies in, and kSw* split bits.
    int32_t* lo_off = nullptr;
    int32_t* lo_idx = nullptr;
    D2* lo_w = nullptr;
    F2* lo_wf = nullptr;  // the weights rounded to fp32 (mixed-precision sweeps)
    uint8_t* lo_code = nullptr;
    int32_t* up_off = nullptr;
    int32_t* up_idx = nullptr;
    D2* up_w = nullptr;
    F2* up_wf = nullptr;
    uint8_t* up_code = nullptr;
    // Components: a batch cloud is the disjoint union of one copy of a cloud
    // per flow condition.  Component k owns points [comp_off[k], comp_off[k+1])
    // and wall-list entries [wall_off[k], wall_off[k+1]).  A plain cloud has
    // one component and comp == nullptr.
    int32_t ncomp = 1;
    int32_t* comp = nullptr;        // component of each point (batch clouds only)
    int32_t* comp_off = nullptr;    // device, ncomp + 1
    int32_t* wall_off = nullptr;    // device, ncomp + 1
    std::vector<int64_t> h_comp_off, h_wall_off, h_comp_active;
    std::vector<double> h_comp_orient;
    std::vector<double> h_comp_inv_active;
    double* comp_inv_active = nullptr;  // device, 1 / non-outer points per component
    double* comp_orient = nullptr;      // device, wall polygon orientation per component
    // reduction chunks: chunk c covers points [chunk_start[c], chunk_start[c+1]) of
    // component chunk_comp[c]; component k owns chunks [comp_chunk_off[k], ...+1)
    int32_t nchunk = 0;
    int32_t* chunk_start = nullptr;     // device, nchunk + 1
    int32_t* chunk_comp = nullptr;      // device, nchunk
    int32_t* comp_chunk_off = nullptr;  // device, ncomp + 1
    // host copies kept for building batch clouds
    std::vector<double> h_x, h_y, h_tx, h_ty;
    std::vector<int8_t> h_type;
    std::vector<int32_t> h_off, h_idx;
    PointGeom* geom = nullptr;
    // LDS tiles of the q-derivative passes (lskum_tiles.h): tile b holds the
    // points tile_pts[b kQTile ...] (-1 past its end), either kQTile
    // consecutive points or a block of rows; tile_idx[tile_off[b] ..
    // tile_off[b+1]) lists the union of their neighbours (sorted) and lnbr[e]
    // gives CSR entry e's neighbour as a position in its point's tile list.
    // ntile = 0 when some tile's list is longer than kQTileMax (the passes
    // then gather directly).
    int32_t ntile = 0;
    int32_t tile_hmax = 0;              // longest tile list
    int32_t* tile_pts = nullptr;        // device, ntile * kQTile
    int32_t* tile_off = nullptr;        // device, ntile + 1
    int32_t* tile_idx = nullptr;        // device
    uint16_t* lnbr = nullptr;           // device, nnz
    // host
    std::vector<int32_t> h_colour;
    std::vector<int32_t> h_col_off;  // ncolour + 1
    std::vector<int32_t> h_grp_off;  // 3 ncolour + 1: (colour, point type) ranges
};

struct Params {
    double gamma, cfl;
    int inner_iters, jvp_mode, precision, check_every;
    double tol_rel;
    int max_iters;
    int sweep_lanes, residual_lanes;
    int limiter;
    double limiter_k;
    int variant;  // 0 Anandhanarayanan et al., 1 Manish et al.
    int scheme;   // 0 implicit (LU-SGS), 1 explicit
    int order;    // 0 colour order (Algorithm 6), 1 wall points first (Algorithm 5)
    int farfield; // 0 outer points at the free stream, 1 kinetic far field
    int qgrad_lanes;  // 0 LDS tiles (library choice), else direct gathers with these lanes
};

// Device work arrays of one flow state.
struct State {
    const Cloud* cloud = nullptr;
    Params prm{};
    double mach = 0, aoa_deg = 0;          // component 0 (plain states)
    std::vector<double> h_mach, h_aoa;     // per component
    std::vector<double> h_res_fs;          // per component free-stream residual
    // per-component device bookkeeping, written by the norm kernel:
    //   active: 1 while the component iterates; status: 0 running,
    //   1 converged (res <= tol_abs), -1 non-finite residual;
    //   iters: iterations taken; res_last: last residual norm.
    int32_t* active = nullptr;
    int32_t* status = nullptr;
    int32_t* iters = nullptr;
    double* res_last = nullptr;
    double* tol_abs = nullptr;             // 0 disables device-side retirement
    double* cfl = nullptr;                 // per component CFL number (params.cfl unless set)
    std::vector<double> h_cfl;             // host copy of cfl
    double* vinf = nullptr;                // 2 per component: free-stream velocity
    double* rr = nullptr;                  // per point R_rho^2 (0 at outer points)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int sweep_lanes = 4;         // lanes per point in the sweep kernels (1, 2, 4 or 8)
    int residual_lanes = 4;      // lanes per point in the residual kernel (1, 2, 4 or 8)
    int qgrad_lanes = 4;         // lanes per point in the q-derivative kernels
    bool qgrad_tiled = true;     // LDS-tiled q-derivative passes when the cloud has tiles
    double res_fs = 0.0;
    // fp64
    D4* U = nullptr;
    D4* q = nullptr;
    D4* qx[2] = {nullptr, nullptr};
    D4* qy[2] = {nullptr, nullptr};
    D4* qxl = nullptr;   // limited q-derivatives (limiter on)
    D4* qyl = nullptr;
    D4* R = nullptr;
    D4* Rs = nullptr;    // forward-sweep right-hand side R - S (Manish variant)
    D4* dU = nullptr;    // increment; kept between iterations (zero after a new U)
    D4* jv0 = nullptr;   // (rho, u1, u2, p) at the state the sweeps linearise about
    D4* jv2 = nullptr;   // (erf(Sx), exp(-Sx^2), erf(Sy), exp(-Sy^2))
    double* D = nullptr; // scalar diagonal
    // fp32 copies for the mixed-precision sweeps
    F4* jv0f = nullptr;
    F4* jv2f = nullptr;
    F4* dUf = nullptr;
    float* Df = nullptr;
    // reductions
    double* fsum = nullptr;      // 2 doubles per component: pressure force
    double* partial = nullptr;   // one partial sum of R_rho^2 per reduction chunk
    double* res_hist = nullptr;  // residual norms, [slot][component]
    int res_cap = 0;             // slots
    int32_t* flags = nullptr;    // [0] non-physical
    int qsel = 0;                // which qx/qy buffer holds the final pass
    bool have_dU = false;
    // graph of check_every iterations for lskum_solve
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    hipEvent_t ev[8] = {};
    bool have_events = false;
};

// Residual-driven CFL control of a batch (lskum_batch_set_cfl_control): a
// condition whose residual reaches no new minimum during a window of
// iterations has its CFL number reduced.
struct CflControl {
    int window = 0;                           // iterations per window; 0 = off
    double factor = 1.0, cfl_min = 0.0;
    int since = 0;                            // iterations into the current window
    std::vector<double> best_prev, best_cur;  // lowest residual of the previous / current window
    std::vector<int32_t> cuts;                // reductions applied, per condition
};

// Kernel launchers (lskum_device.hip).  All enqueue on s->stream.
hipError_t launch_precompute(Cloud& c, hipStream_t st);
// split weights and bits of the sweep lists (after launch_precompute)
hipError_t launch_sweep_weights(Cloud& c, hipStream_t st);
hipError_t launch_free_stream(State& s);
hipError_t launch_q_from_U(State& s);
// q-derivative passes, with the limiter when on.  With the limiter the last
// pass writes only the limited derivatives (all the residual reads) unless
// keep_unlimited asks for the unlimited ones too (in qx/qy[qsel]).
hipError_t launch_q_derivatives(State& s, bool keep_unlimited = false);
// residual + time step/diagonal + sweep intermediates (per-point R_rho^2)
// in_step: part of an implicit step (the kernel then also does the forward
// sweep's first colour phase); false for a residual evaluation alone
hipError_t launch_residual(State& s, int slot, bool in_step = false);
// per-component residual norms into res_hist[slot][k]; retires components
hipError_t launch_norm(State& s, int slot);
hipError_t launch_reset_components(State& s);
hipError_t launch_sweeps(State& s);
hipError_t launch_sweep_dir(State& s, bool forward);
hipError_t launch_update(State& s);
hipError_t launch_explicit_update(State& s);  // U -= dt R (explicit scheme)
hipError_t launch_forces(State& s);  // fsum[2k..2k+1] = force of component k
hipError_t launch_soa_to_aos(const double* soa, D4* aos, int64_t n, hipStream_t st);
hipError_t launch_aos_to_soa(const D4* aos, double* soa, int64_t n, hipStream_t st);
hipError_t launch_aosf_to_soa(const F4* aos, double* soa, int64_t n, hipStream_t st);
hipError_t launch_clear_flags(int32_t* flags, hipStream_t st);
// zero increment (both precisions) of points [p0, p0 + n): after a new U
hipError_t clear_increment(State& s, int64_t p0, int64_t n);
// every component's CFL number to params.cfl
hipError_t reset_cfl(State& s);

// fill n doubles with v, and copy one int32 (kernels, so that graph capture
// records no memset node)
hipError_t launch_fill(double* p, int n, double v, hipStream_t st);
hipError_t launch_copy_flag(const int32_t* src, int32_t* dst, hipStream_t st);
// out[0] = res[0], out[1] = 1 if flags[0] is set else 0
hipError_t launch_residual_out(const double* res, const int32_t* flags, double* out,
                               hipStream_t st);

// Error reporting shared by the C-ABI source files: records msg for
// lskum_last_error() and returns code.
int api_error(int code, const std::string& msg);
void api_clear_error();
// lskum_params validation and conversion (as lskum_state_create applies them)
int api_check_params(const lskum_params* p);
Params api_params(const lskum_params* p);

}  // namespace lskum

// Opaque handles of the C ABI.
struct lskum_cloud {
    lskum::Cloud c;
};
struct lskum_state {
    lskum::State s;
};
struct lskum_batch {
    lskum::Cloud c;  // union of the conditions' clouds
    lskum::State s;
    std::vector<int32_t> cond_cloud;
    lskum::CflControl ctl;
};
