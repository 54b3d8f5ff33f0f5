// Host side of the learned warm start: the lskum_mlp_* and *_features
// entry points of include/lskum.h.
#include "../../include/lskum.h"
#include "lskum_mlp.h"

#include <chrono>
#include <cmath>
#include <new>
#include <vector>

struct lskum_mlp {
    lskum::mlp::Net n;
};

namespace {

using lskum::api_error;
namespace M = lskum::mlp;

int hip_err(hipError_t e, const char* what) {
    return api_error(e == hipErrorOutOfMemory ? LSKUM_ERR_OOM : LSKUM_ERR_HIP,
                     std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                     \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_err(e_, #expr); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

int64_t round_up(int64_t m, int64_t a) { return (m + a - 1) / a * a; }

void free_net(M::Net& n) {
    void* ptrs[] = {n.theta, n.grad, n.m,  n.v,  n.W1b, n.W2b, n.W3b, n.W4b, n.Xin,
                    n.Tin,   n.Yout, n.Xb, n.Z1, n.Z2,  n.Z3,  n.H1,  n.H2,  n.H3,
                    n.dY,    n.se,   n.dZ3, n.dZ2, n.dZ1, n.part, n.d_loss, n.d_bad,
                    n.d_res_fs};
    for (void* p : ptrs) (void)hipFree(p);
    for (hipEvent_t e : n.ev)
        if (e) (void)hipEventDestroy(e);
    if (n.own_stream && n.stream) (void)hipStreamDestroy(n.stream);
    n = M::Net{};
}

uint64_t splitmix64(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Glorot-uniform weights, zero biases.
std::vector<float> init_params(uint64_t seed) {
    std::vector<float> th(M::kParams, 0.0f);
    uint64_t st = seed;
    auto fill = [&](int off, int fan_out, int fan_in) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int k = 0; k < fan_out * fan_in; ++k) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            th[off + k] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(M::kOffW1, M::kWidth, M::kIn);
    fill(M::kOffW2, M::kWidth, M::kWidth);
    fill(M::kOffW3, M::kWidth, M::kWidth);
    fill(M::kOffW4, M::kOut, M::kWidth);
    return th;
}

int reset_moments(M::Net& n) {
    HIPCHK(hipMemsetAsync(n.m, 0, M::kParams * sizeof(float), n.stream));
    HIPCHK(hipMemsetAsync(n.v, 0, M::kParams * sizeof(float), n.stream));
    n.step = 0;
    return LSKUM_OK;
}

// Forward (and, with T, loss terms) of m rows staged in the workspace.
int run_forward(M::Net& n, const float* X, int64_t m, const float* T, float* Y) {
    const int64_t M_ = round_up(m, M::kRowAlign);
    HIPCHK(M::forward(n, X, (int)M_, (int)m, T, Y));
    return LSKUM_OK;
}

int read_loss(M::Net& n, int64_t m, double* loss) {
    HIPCHK(M::loss(n, (int)round_up(m, M::kRowAlign), n.d_loss));
    double s = 0.0;
    HIPCHK(hipMemcpyAsync(&s, n.d_loss, sizeof(double), hipMemcpyDeviceToHost, n.stream));
    HIPCHK(hipStreamSynchronize(n.stream));
    if (loss) *loss = s / (4.0 * (double)m);
    return LSKUM_OK;
}

// Orders the network's stream after the state's stream (and back).
int join(hipStream_t wait_on, hipStream_t other, hipEvent_t ev) {
    if (wait_on == other) return LSKUM_OK;
    HIPCHK(hipEventRecord(ev, other));
    HIPCHK(hipStreamWaitEvent(wait_on, ev, 0));
    return LSKUM_OK;
}

int state_features(lskum::State& s, float* X, float* T) {
    if (!X) return api_error(LSKUM_ERR_ARG, "X is NULL");
    HIPCHK(M::features(s, 0, s.cloud->n, X, T));
    HIPCHK(hipStreamSynchronize(s.stream));
    return LSKUM_OK;
}

// Predicts U chunk by chunk on the network's workspace, then checks every
// component's residual norm and sends rejected ones to the free stream.
int warm_start(M::Net& n, lskum::State& s, int32_t* fallback, double* res_warm) {
    const lskum::Cloud& c = *s.cloud;
    const int nc = c.ncomp;
    if (n.ncomp_cap < nc) {
        (void)hipFree(n.d_bad);
        (void)hipFree(n.d_res_fs);
        n.d_bad = nullptr;
        n.d_res_fs = nullptr;
        n.ncomp_cap = 0;
        HIPCHK(dalloc(&n.d_bad, nc));
        HIPCHK(dalloc(&n.d_res_fs, nc));
        n.ncomp_cap = nc;
    }
    // the network's own stream is used for its layers; the state's stream
    // for the state's kernels: order them with events both ways
    if (int r = join(n.stream, s.stream, n.ev[0])) return r;
    HIPCHK(hipMemsetAsync(n.d_bad, 0, nc * sizeof(int32_t), s.stream));
    HIPCHK(hipMemcpyAsync(n.d_res_fs, s.h_res_fs.data(), nc * sizeof(double),
                          hipMemcpyHostToDevice, s.stream));
    for (int64_t p0 = 0; p0 < c.n; p0 += n.capacity) {
        const int64_t m = std::min<int64_t>(n.capacity, c.n - p0);
        HIPCHK(M::features(s, p0, m, n.Xin, nullptr));
        if (int r = join(n.stream, s.stream, n.ev[0])) return r;
        if (int r = run_forward(n, n.Xin, m, nullptr, n.Yout)) return r;
        if (int r = join(s.stream, n.stream, n.ev[1])) return r;
        HIPCHK(M::pred_to_U(n, s, p0, m, n.Yout));
    }
    // residual of the predicted state (q from U first; a non-physical q
    // shows up as a non-finite residual of its component)
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(lskum::launch_q_derivatives(s));
    HIPCHK(lskum::launch_residual(s, 0));
    HIPCHK(lskum::launch_norm(s, 0));
    HIPCHK(M::vet_and_fallback(n, s, s.res_hist));
    HIPCHK(lskum::launch_reset_components(s));
    HIPCHK(lskum::launch_clear_flags(s.flags, s.stream));
    HIPCHK(lskum::launch_q_from_U(s));
    HIPCHK(lskum::clear_increment(s, 0, c.n));
    std::vector<int32_t> bad(nc);
    std::vector<double> res(nc);
    HIPCHK(hipMemcpyAsync(bad.data(), n.d_bad, nc * sizeof(int32_t), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipMemcpyAsync(res.data(), s.res_hist, nc * sizeof(double), hipMemcpyDeviceToHost,
                          s.stream));
    HIPCHK(hipStreamSynchronize(s.stream));
    s.have_dU = false;
    for (int k = 0; k < nc; ++k) {
        if (fallback) fallback[k] = bad[k];
        if (res_warm) res_warm[k] = res[k];
    }
    return LSKUM_OK;
}

}  // namespace

extern "C" {

int lskum_mlp_create(uint64_t seed, int64_t max_rows, void* hip_stream, lskum_mlp** out) {
    lskum::api_clear_error();
    if (!out) return api_error(LSKUM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_rows < 1 || max_rows > ((int64_t)1 << 24))
        return api_error(LSKUM_ERR_ARG, "max_rows must be in [1, 2^24]");
    lskum_mlp* h = new (std::nothrow) lskum_mlp();
    if (!h) return api_error(LSKUM_ERR_OOM, "host allocation");
    M::Net& n = h->n;
    (void)hipGetDevice(&n.device);
    n.stream = (hipStream_t)hip_stream;
    int rc = LSKUM_OK;
    auto bail = [&](int r) {
        free_net(n);
        delete h;
        return r;
    };
    if (!n.stream) {
        hipError_t e = hipStreamCreateWithFlags(&n.stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_err(e, "hipStreamCreateWithFlags"));
        n.own_stream = true;
    }
    const int64_t cap = round_up(max_rows, M::kChunk);
    n.capacity = cap;
    const int64_t W = M::kWidth;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    chk(dalloc(&n.theta, M::kParams));
    chk(dalloc(&n.grad, M::kParams));
    chk(dalloc(&n.m, M::kParams));
    chk(dalloc(&n.v, M::kParams));
    chk(dalloc(&n.W1b, W * M::kIn));
    chk(dalloc(&n.W2b, W * W));
    chk(dalloc(&n.W3b, W * W));
    chk(dalloc(&n.W4b, M::kOut * W));
    chk(dalloc(&n.Xin, cap * M::kIn));
    chk(dalloc(&n.Tin, cap * M::kOut));
    chk(dalloc(&n.Yout, cap * M::kOut));
    chk(dalloc(&n.Xb, cap * M::kIn));
    chk(dalloc(&n.Z1, cap * W));
    chk(dalloc(&n.Z2, cap * W));
    chk(dalloc(&n.Z3, cap * W));
    chk(dalloc(&n.H1, cap * W));
    chk(dalloc(&n.H2, cap * W));
    chk(dalloc(&n.H3, cap * W));
    chk(dalloc(&n.dY, cap * M::kOut));
    chk(dalloc(&n.se, cap * M::kOut));
    chk(dalloc(&n.dZ3, cap * W));
    chk(dalloc(&n.dZ2, cap * W));
    chk(dalloc(&n.dZ1, cap * W));
    chk(dalloc(&n.part, M::part_floats(cap)));
    chk(dalloc(&n.d_loss, 1));
    for (hipEvent_t& ev : n.ev) chk(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (e != hipSuccess) return bail(hip_err(e, "network allocation"));
    const std::vector<float> th = init_params(seed);
    e = hipMemcpyAsync(n.theta, th.data(), M::kParams * sizeof(float), hipMemcpyHostToDevice,
                       n.stream);
    if (e != hipSuccess) return bail(hip_err(e, "parameter upload"));
    if ((rc = reset_moments(n))) return bail(rc);
    if ((e = M::refresh_weights(n)) != hipSuccess) return bail(hip_err(e, "refresh_weights"));
    if ((e = hipStreamSynchronize(n.stream)) != hipSuccess) return bail(hip_err(e, "sync"));
    *out = h;
    return LSKUM_OK;
}

void lskum_mlp_destroy(lskum_mlp* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->n.stream);
    free_net(h->n);
    delete h;
}

int lskum_mlp_get_params(lskum_mlp* h, float* theta, int on_device) {
    if (!h || !theta) return api_error(LSKUM_ERR_ARG, "NULL argument");
    M::Net& n = h->n;
    HIPCHK(hipMemcpyAsync(theta, n.theta, M::kParams * sizeof(float),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, n.stream));
    HIPCHK(hipStreamSynchronize(n.stream));
    return LSKUM_OK;
}

int lskum_mlp_set_params(lskum_mlp* h, const float* theta, int on_device) {
    if (!h || !theta) return api_error(LSKUM_ERR_ARG, "NULL argument");
    M::Net& n = h->n;
    HIPCHK(hipMemcpyAsync(n.theta, theta, M::kParams * sizeof(float),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, n.stream));
    if (int r = reset_moments(n)) return r;
    HIPCHK(M::refresh_weights(n));
    HIPCHK(hipStreamSynchronize(n.stream));
    return LSKUM_OK;
}

int lskum_mlp_forward(lskum_mlp* h, int64_t m, const float* X, float* Y) {
    if (!h || m < 0 || (m > 0 && (!X || !Y))) return api_error(LSKUM_ERR_ARG, "invalid argument");
    M::Net& n = h->n;
    // inference reads X and writes Y directly (no workspace): one launch per
    // 2^30 rows
    const int64_t step = (int64_t)1 << 30;
    for (int64_t r0 = 0; r0 < m; r0 += step) {
        const int64_t k = std::min<int64_t>(step, m - r0);
        if (int r = run_forward(n, X + r0 * M::kIn, k, nullptr, Y + r0 * M::kOut)) return r;
    }
    HIPCHK(hipStreamSynchronize(n.stream));
    return LSKUM_OK;
}

int lskum_mlp_gradient(lskum_mlp* h, int64_t m, const float* X, const float* T, float* grad,
                       double* loss) {
    if (!h || !X || !T) return api_error(LSKUM_ERR_ARG, "NULL argument");
    M::Net& n = h->n;
    if (m < 1 || m > n.capacity) return api_error(LSKUM_ERR_ARG, "m must be in [1, max_rows]");
    if (int r = run_forward(n, X, m, T, nullptr)) return r;
    HIPCHK(M::backward(n, (int)round_up(m, M::kRowAlign)));
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, n.grad, M::kParams * sizeof(float), hipMemcpyDeviceToDevice,
                              n.stream));
    return read_loss(n, m, loss);
}

int lskum_mlp_train_step(lskum_mlp* h, int64_t m, const float* X, const float* T, float lr,
                         double* loss) {
    if (!h || !X || !T) return api_error(LSKUM_ERR_ARG, "NULL argument");
    M::Net& n = h->n;
    if (m < 1 || m > n.capacity) return api_error(LSKUM_ERR_ARG, "m must be in [1, max_rows]");
    if (!(lr > 0.0f)) return api_error(LSKUM_ERR_ARG, "lr must be > 0");
    if (int r = run_forward(n, X, m, T, nullptr)) return r;
    HIPCHK(M::backward(n, (int)round_up(m, M::kRowAlign)));
    HIPCHK(M::loss(n, (int)round_up(m, M::kRowAlign), n.d_loss));
    HIPCHK(M::adam_step(n, lr));
    double s = 0.0;
    HIPCHK(hipMemcpyAsync(&s, n.d_loss, sizeof(double), hipMemcpyDeviceToHost, n.stream));
    HIPCHK(hipStreamSynchronize(n.stream));
    if (loss) *loss = s / (4.0 * (double)m);
    return LSKUM_OK;
}

int lskum_mlp_train(lskum_mlp* h, int64_t nrows, const float* X, const float* T, int32_t steps,
                    int32_t batch, float lr, float lr_final, uint64_t seed, double* loss_hist,
                    double* seconds) {
    if (!h || !X || !T) return api_error(LSKUM_ERR_ARG, "NULL argument");
    M::Net& n = h->n;
    if (nrows < 1 || steps < 0 || batch < 1 || batch > n.capacity || !(lr > 0.0f) ||
        !(lr_final >= 0.0f))
        return api_error(LSKUM_ERR_ARG, "invalid training arguments");
    double* d_hist = nullptr;
    HIPCHK(dalloc(&d_hist, steps));
    const int Mp = (int)round_up(batch, M::kRowAlign);
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = hipSuccess;
    for (int32_t t = 0; t < steps && e == hipSuccess; ++t) {
        const double frac = steps > 1 ? (double)t / (double)(steps - 1) : 0.0;
        const float lr_t =
            (float)(lr_final + 0.5 * (lr - lr_final) * (1.0 + std::cos(3.14159265358979323846 * frac)));
        e = M::gather(n, nrows, X, T, batch, seed, t);
        if (e == hipSuccess) e = M::forward(n, n.Xin, Mp, batch, n.Tin, nullptr);
        if (e == hipSuccess) e = M::backward(n, Mp);
        if (e == hipSuccess) e = M::loss(n, Mp, d_hist + t);
        if (e == hipSuccess) e = M::adam_step(n, lr_t);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(n.stream);
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::vector<double> hist(steps > 0 ? steps : 1);
    if (e == hipSuccess && steps > 0)
        e = hipMemcpy(hist.data(), d_hist, steps * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d_hist);
    if (e != hipSuccess) return hip_err(e, "training");
    if (loss_hist)
        for (int32_t t = 0; t < steps; ++t) loss_hist[t] = hist[t] / (4.0 * (double)batch);
    if (seconds) *seconds = secs;
    return LSKUM_OK;
}

int lskum_state_features(lskum_state* so, float* X, float* T) {
    if (!so) return api_error(LSKUM_ERR_ARG, "state is NULL");
    return state_features(so->s, X, T);
}

int lskum_batch_features(lskum_batch* b, float* X, float* T) {
    if (!b) return api_error(LSKUM_ERR_ARG, "batch is NULL");
    return state_features(b->s, X, T);
}

int lskum_mlp_warm_start(lskum_mlp* h, lskum_state* so, int32_t* fallback, double* res_warm) {
    if (!h || !so) return api_error(LSKUM_ERR_ARG, "NULL argument");
    return warm_start(h->n, so->s, fallback, res_warm);
}

int lskum_mlp_warm_start_batch(lskum_mlp* h, lskum_batch* b, int32_t* fallback,
                               double* res_warm) {
    if (!h || !b) return api_error(LSKUM_ERR_ARG, "NULL argument");
    return warm_start(h->n, b->s, fallback, res_warm);
}

}  // extern "C"
