// Internal declarations shared by the device kernels and the host API of the
// MI355X LSKUM library.  Not part of the public C ABI (include/lskum.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

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

struct Cloud {
    int device = 0;
    int64_t n = 0, nnz = 0;
    int32_t ncolour = 0;
    int64_t n_degenerate = 0;
    int64_t n_active = 0;      // non-outer points
    int64_t n_wall = 0;
    double wall_orient = 1.0;  // +1 if the wall polygon runs counter-clockwise
    // device
    D2* xy = nullptr;          // coordinates
    D2* frame = nullptr;       // unit tangent (wall points); (1, 0) elsewhere
    int8_t* type = nullptr;
    int32_t* off = nullptr;
    int32_t* idx = nullptr;
    int32_t* colour = nullptr;
    int32_t* col_perm = nullptr;   // points sorted by colour, then index
    int32_t* wall_list = nullptr;  // wall points in storage order
    // neighbours of each point split by colour, CSR order kept within each list:
    // lower colours (read by the forward sweep) and higher colours (backward)
    int32_t* lo_off = nullptr;
    int32_t* lo_idx = nullptr;
    int32_t* up_off = nullptr;
    int32_t* up_idx = nullptr;
    PointGeom* geom = nullptr;
    // host
    std::vector<int32_t> h_colour;
    std::vector<int32_t> h_col_off;  // ncolour + 1
};

struct Params {
    double gamma, cfl;
    int inner_iters, jvp_mode, precision, check_every;
    double tol_rel;
    int max_iters;
    int sweep_lanes, residual_lanes;
};

// Device work arrays of one flow state.
struct State {
    const Cloud* cloud = nullptr;
    Params prm{};
    double mach = 0, aoa_deg = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int sweep_lanes = 4;         // lanes per point in the sweep kernels (1, 2, 4 or 8)
    int residual_lanes = 4;      // lanes per point in the residual kernel (1, 2, 4 or 8)
    double res_fs = 0.0;
    // fp64
    D4* U = nullptr;
    D4* q = nullptr;
    D4* qx[2] = {nullptr, nullptr};
    D4* qy[2] = {nullptr, nullptr};
    D4* R = nullptr;
    D4* dU = nullptr;
    D4* jv0 = nullptr;   // (rho, u1, u2, p) at the state the sweeps linearise about
    D4* jv1 = nullptr;   // (sqrt(beta), beta, 1/rho, 1/p)
    D4* jv2 = nullptr;   // (erf(Sx), exp(-Sx^2), erf(Sy), exp(-Sy^2))
    double* D = nullptr; // scalar diagonal
    // fp32 copies for the mixed-precision sweeps
    F4* jv0f = nullptr;
    F4* jv1f = nullptr;
    F4* jv2f = nullptr;
    F4* dUf = nullptr;
    float* Df = nullptr;
    // reductions
    double* partial = nullptr;   // per-block partial sums of R_rho^2
    int nblk_partial = 0;        // blocks of the last residual launch
    int partial_cap = 0;
    double* res_hist = nullptr;  // residual norms written by the iteration
    int res_cap = 0;
    int32_t* flags = nullptr;    // [0] non-physical
    int qsel = 0;                // which qx/qy buffer holds the final pass
    bool have_dU = false;
    // graph of check_every iterations for lskum_solve
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    hipEvent_t ev[8] = {};
    bool have_events = false;
};

// Kernel launchers (lskum_device.hip).  All enqueue on s->stream.
hipError_t launch_precompute(Cloud& c, hipStream_t st);
hipError_t launch_free_stream(State& s);
hipError_t launch_q_from_U(State& s);
hipError_t launch_q_derivatives(State& s);
// residual + time step/diagonal + sweep intermediates (block partial norms)
hipError_t launch_residual(State& s, int slot);
// residual norm from the block partials into res_hist[slot]
hipError_t launch_norm(State& s, int slot);
hipError_t launch_sweeps(State& s);
hipError_t launch_sweep_dir(State& s, bool forward);
hipError_t launch_update(State& s);
hipError_t launch_forces(State& s, double* d_out2);
hipError_t launch_soa_to_aos(const double* soa, D4* aos, int64_t n, hipStream_t st);
hipError_t launch_aos_to_soa(const D4* aos, double* soa, int64_t n, hipStream_t st);
hipError_t launch_aosf_to_soa(const F4* aos, double* soa, int64_t n, hipStream_t st);
hipError_t launch_clear_flags(int32_t* flags, hipStream_t st);

}  // namespace lskum
