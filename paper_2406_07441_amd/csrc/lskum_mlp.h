// Internal declarations of the per-point warm-start MLP (lskum_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lskum_internal.h"

namespace lskum {
namespace mlp {

constexpr int kIn = 5, kWidth = 128, kOut = 4;
// flat parameter layout: W1[128][5] b1 W2[128][128] b2 W3[128][128] b3 W4[4][128] b4
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kWidth * kIn;
constexpr int kOffW2 = kOffB1 + kWidth;
constexpr int kOffB2 = kOffW2 + kWidth * kWidth;
constexpr int kOffW3 = kOffB2 + kWidth;
constexpr int kOffB3 = kOffW3 + kWidth * kWidth;
constexpr int kOffW4 = kOffB3 + kWidth;
constexpr int kOffB4 = kOffW4 + kOut * kWidth;
constexpr int kParams = kOffB4 + kOut;
static_assert(kParams == 34308, "parameter count");
constexpr int kChunk = 256;   // rows per partial sum of the gradients (multiple of 32)
constexpr int kRowAlign = 32; // workspace rows are padded to a multiple of this
constexpr int kMaxSumJobs = 8; // sums over rows in one backward pass
constexpr int kMaxColJobs = 6; // of which column sums computed without matrix cores

struct Net {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t capacity = 0;  // workspace rows (multiple of kRowAlign)
    int64_t step = 0;      // Adam steps taken
    float* theta = nullptr;  // fp32 master weights
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    __bf16 *W1b = nullptr, *W2b = nullptr, *W3b = nullptr, *W4b = nullptr;
    // workspace, capacity rows
    float* Xin = nullptr;   // [cap][5] staged features
    float* Tin = nullptr;   // [cap][4] staged targets
    float* Yout = nullptr;  // [cap][4] predictions
    __bf16* Xb = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr;
    __bf16 *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
    float* dY = nullptr;
    float* se = nullptr;
    __bf16 *dZ3 = nullptr, *dZ2 = nullptr;
    float* dZ1 = nullptr;
    float* part = nullptr;  // gradient partials of one backward pass, part_floats(capacity)
    double* d_loss = nullptr;
    int32_t* d_bad = nullptr;      // per component: 1 if the prediction is unusable
    double* d_res_fs = nullptr;    // per component free-stream residual (residual check)
    int64_t ncomp_cap = 0;
    hipEvent_t ev[2] = {};
};

// Forward over workspace rows [0, M) (M a multiple of kRowAlign, Mvalid <= M);
// X [Mvalid][5]; with T ([Mvalid][4]) also the loss terms for backward;
// with Y ([Mvalid][4]) the predictions.
hipError_t forward(Net& net, const float* X, int M, int Mvalid, const float* T, float* Y);
hipError_t backward(Net& net, int M);
// Floats of gradient partials a workspace of cap rows needs (Net::part).
int64_t part_floats(int64_t cap);
hipError_t loss(Net& net, int M, double* d_out);
hipError_t adam_step(Net& net, float lr);
hipError_t refresh_weights(Net& net);
// Rows r of a minibatch: row idx(r) = floor(h(seed, step, r) * n / 2^64) of X, T.
hipError_t gather(Net& net, int64_t n, const float* X, const float* T, int B, uint64_t seed,
                  int64_t step);
// Features of points [p0, p0 + m) of a state (into Xin) and, optionally,
// targets from its U (into Tout, [m][4]).
hipError_t features(const State& s, int64_t p0, int64_t m, float* Xout, float* Tout);
// U of points [p0, p0 + m) from the predictions Y; marks d_bad[comp] for
// non-finite or non-physical predictions.
hipError_t pred_to_U(Net& net, const State& s, int64_t p0, int64_t m, const float* Y);
// Residual check: components whose residual res[k] is not finite or not below the
// free-stream residual are flagged in d_bad and reset to the free stream.
hipError_t vet_and_fallback(Net& net, const State& s, const double* res);

}  // namespace mlp
}  // namespace lskum
