// Per-point warm-start MLP on gfx950: 5 -> 128 -> 128 -> 128 -> 4, GELU (erf
// form) on the hidden layers, bfloat16 weights/activations with fp32
// accumulation, Adam on fp32 master weights.
//
// The two 128 x 128 layers and their backward products are dense
// contractions and run on the matrix cores (v_mfma_f32_16x16x32_bf16): one
// wavefront computes one 16 x 16 output tile, K is walked 32 at a time.
// Operand registers: lane l holds row (A) or column (B) l % 16 and the eight
// consecutive K entries 8 (l / 16) .. 8 (l / 16) + 7; the accumulator lane l
// holds column l % 16 of rows 4 (l / 16) .. 4 (l / 16) + 3.  The thin 5 -> 128
// and 128 -> 4 layers run on the vector ALUs.
//
// Quantisation points (shared with the float64 reference of the tests):
// bf16 copies of W1..W4, of the input features and of each hidden activation;
// the backward pass rounds the pre-activation gradients of layers 3 and 2 to
// bf16 before their products; everything else is fp32.
#include "lskum_mlp.h"

#include <cmath>

namespace lskum {
namespace mlp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * kInvSqrt2)); }
__device__ __forceinline__ float gelu_prime(float z) {
    return 0.5f * (1.0f + erff(z * kInvSqrt2)) + z * expf(-0.5f * z * z) * kInvSqrt2Pi;
}

// One 16 x 16 tile of C = A B over K range [k0, k1) (k1 - k0 a multiple of 32).
// a(r, k) = A[r * a_rs + k * a_ks], b(k, c) = B[k * b_ks + c * b_cs].
__device__ __forceinline__ f32x4 tile_mma(const __bf16* __restrict__ A, int64_t a_rs,
                                          int64_t a_ks, const __bf16* __restrict__ B,
                                          int64_t b_ks, int64_t b_cs, int r0, int c0, int k0,
                                          int k1) {
    const int l = threadIdx.x & 63;
    const int rr = r0 + (l & 15), cc = c0 + (l & 15), kq = 8 * (l >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k = k0; k < k1; k += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            a[t] = A[rr * a_rs + (int64_t)(k + kq + t) * a_ks];
            b[t] = B[(int64_t)(k + kq + t) * b_ks + cc * b_cs];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Whole forward pass of 128 rows per workgroup (8 waves x 16 rows).  W2, then
// W3, is staged in one LDS buffer with rows padded to kLdsW bf16 (a 16-byte operand read
// by 16 lanes of different rows then hits distinct banks).  Layer 1 is
// evaluated directly in the matrix-core operand layout (each lane computes the
// 32 hidden units its A fragments hold); the 128 x 128 layers run on the
// matrix cores, their outputs going back through a per-wave LDS tile to the
// operand layout of the next layer; layer 4 sums each lane's 8 columns and
// then across the 16 lanes of a row group with shuffles (fixed order).
// TRAIN also writes what the backward pass reads (Xb, Z1-3, H1-3) and the
// loss terms dY, se; otherwise Y.
constexpr int kLdsW = kWidth + 8;
constexpr int kFwdWaves = 8;

template <bool TRAIN>
__global__ void __launch_bounds__(64 * kFwdWaves) k_mlp_forward(
    int M, int Mvalid, const float* __restrict__ X, const __bf16* __restrict__ W1,
    const float* __restrict__ b1, const __bf16* __restrict__ W2, const float* __restrict__ b2,
    const __bf16* __restrict__ W3, const float* __restrict__ b3, const __bf16* __restrict__ W4,
    const float* __restrict__ b4, const float* __restrict__ T, float* __restrict__ Y,
    __bf16* __restrict__ Xb, float* __restrict__ Z1, float* __restrict__ Z2,
    float* __restrict__ Z3, __bf16* __restrict__ H1, __bf16* __restrict__ H2,
    __bf16* __restrict__ H3, float* __restrict__ dY, float* __restrict__ se) {
    // one weight buffer: W2 for layer 2, then W3 for layer 3 (70 KB of LDS
    // per block instead of 104 KB, so that two blocks share a CU)
    __shared__ __attribute__((aligned(16))) __bf16 sW[kWidth * kLdsW];
    __shared__ __attribute__((aligned(16))) __bf16 sH[kFwdWaves][16 * kLdsW];
    auto stage = [&](const __bf16* __restrict__ Wg) {  // 16-byte chunks
        for (int ch = threadIdx.x; ch < kWidth * kWidth / 8; ch += blockDim.x) {
            const int row = ch / (kWidth / 8), c8 = (ch % (kWidth / 8)) * 8;
            *(bf16x8*)&sW[row * kLdsW + c8] = *(const bf16x8*)&Wg[row * kWidth + c8];
        }
    };
    stage(W2);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row0 = (blockIdx.x * kFwdWaves + w) * 16;
    // a wave past the last row does no work but takes part in the barriers
    const bool act = row0 < M;
    const int r = l & 15, g = l >> 4, kq = 8 * g;
    const int64_t m = row0 + r;
    __bf16* hs = sH[w];
    // ---- layer 1 (5 -> 128) in the A-operand layout
    float x[kIn];
#pragma unroll
    for (int f = 0; f < kIn; ++f) {
        const __bf16 xb = (__bf16)(act && m < Mvalid ? X[m * kIn + f] : 0.0f);
        x[f] = (float)xb;
        if (TRAIN && act && g == 0) Xb[m * kIn + f] = xb;
    }
    bf16x8 a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float zz[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int n = 32 * s + kq + j;
            float z = b1[n];
#pragma unroll
            for (int f = 0; f < kIn; ++f) z += x[f] * (float)W1[n * kIn + f];
            zz[j] = z;
            a[s][j] = (__bf16)gelu(z);
        }
        if (TRAIN && act) {
            float* z1 = Z1 + m * kWidth + 32 * s + kq;
#pragma unroll
            for (int j = 0; j < 8; ++j) z1[j] = zz[j];
            *(bf16x8*)(H1 + m * kWidth + 32 * s + kq) = a[s];
        }
    }
    // ---- layers 2 and 3 (128 -> 128) on the matrix cores
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        if (layer == 1) {
            // every wave has read W2: replace it by W3
            __syncthreads();
            stage(W3);
            __syncthreads();
        }
        if (!act) continue;
        const float* bias = layer == 0 ? b2 : b3;
        float* Zg = layer == 0 ? Z2 : Z3;
        __bf16* Hg = layer == 0 ? H2 : H3;
        f32x4 acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bf16x8 b = *(const bf16x8*)&sW[(16 * c + r) * kLdsW + 32 * s + kq];
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b, acc[c], 0, 0, 0);
            }
        }
        // bias + GELU in the accumulator layout: lane holds rows 4g..4g+3 of column 16c + r
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int col = 16 * c + r;
            const float bc = bias[col];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int rr = 4 * g + t;
                const float z = acc[c][t] + bc;
                const __bf16 h = (__bf16)gelu(z);
                acc[c][t] = (float)h;  // keep the rounded activation for layer 4
                hs[rr * kLdsW + col] = h;
                if (TRAIN) {
                    const int64_t mm = row0 + rr;
                    Zg[mm * kWidth + col] = z;
                    Hg[mm * kWidth + col] = h;
                }
            }
        }
        if (layer == 0) {
            // back to the A-operand layout for layer 3 (wave-local tile; LDS
            // operations of one wave complete in order)
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int s = 0; s < 4; ++s) a[s] = *(const bf16x8*)&hs[r * kLdsW + 32 * s + kq];
        } else {
            // ---- layer 4 (128 -> 4): lane partial sums over its 8 columns
            float ysum[4][kOut];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int o = 0; o < kOut; ++o) {
                    float sacc = 0.0f;
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        sacc += acc[c][t] * (float)W4[o * kWidth + 16 * c + r];
                    ysum[t][o] = sacc;
                }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1)
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int o = 0; o < kOut; ++o) ysum[t][o] += __shfl_xor(ysum[t][o], off, 64);
            if (r < kOut) {
                const int o = r;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int64_t mm = row0 + 4 * g + t;
                    float yv = 0.0f;
#pragma unroll
                    for (int oo = 0; oo < kOut; ++oo)
                        if (oo == o) yv = ysum[t][oo];
                    yv += b4[o];
                    if (TRAIN) {
                        const float res = mm < Mvalid ? yv - T[mm * kOut + o] : 0.0f;
                        dY[mm * kOut + o] = 2.0f * res / (4.0f * (float)Mvalid);
                        se[mm * kOut + o] = res * res;
                    } else if (mm < Mvalid) {
                        Y[mm * kOut + o] = yv;
                    }
                }
            }
        }
    }
}

// Backward through a dense layer: dH = dZn W (dZn [M][128] bf16, W [out][in]),
// then dZ = dH * GELU'(Zprev); stored as bf16 (ROUND) or fp32.
template <bool ROUND>
__global__ void __launch_bounds__(64) k_dense_bwd_data(int M, const __bf16* __restrict__ dZn,
                                                       const __bf16* __restrict__ W,
                                                       const float* __restrict__ Zprev,
                                                       __bf16* __restrict__ dZb,
                                                       float* __restrict__ dZf) {
    const int tile = blockIdx.x;
    const int r0 = 16 * (tile >> 3), c0 = 16 * (tile & 7);
    if (r0 >= M) return;
    // C[m][i] = sum_o dZn[m][o] W[o][i]: A row stride 128, B k stride 128
    const f32x4 acc = tile_mma(dZn, kWidth, 1, W, kWidth, 1, r0, c0, 0, kWidth);
    const int l = threadIdx.x;
    const int c = c0 + (l & 15);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t o = (int64_t)(r0 + 4 * (l >> 4) + t) * kWidth + c;
        const float v = acc[t] * gelu_prime(Zprev[o]);
        if (ROUND) dZb[o] = (__bf16)v;
        else dZf[o] = v;
    }
}

// Weight gradient partials: P[chunk][o][i] = sum_{m in chunk} dZ[m][o] H[m][i]
// (both [M][128] bf16).  Grid: (64 tiles, nchunks).
__global__ void __launch_bounds__(64) k_dense_wgrad(int M, int mchunk, const __bf16* __restrict__ dZ,
                                                    const __bf16* __restrict__ H,
                                                    float* __restrict__ P) {
    const int tile = blockIdx.x, ch = blockIdx.y;
    const int r0 = 16 * (tile >> 3), c0 = 16 * (tile & 7);
    const int k0 = ch * mchunk, k1 = min(M, k0 + mchunk);
    if (k0 >= k1) return;
    // C[o][i] = sum_m A[o][m] B[m][i]: A = dZ^T (row stride 1, k stride 128)
    const f32x4 acc = tile_mma(dZ, 1, kWidth, H, kWidth, 1, r0, c0, k0, k1);
    const int l = threadIdx.x;
    const int c = c0 + (l & 15);
    float* out = P + (int64_t)ch * kWidth * kWidth;
#pragma unroll
    for (int t = 0; t < 4; ++t) out[(r0 + 4 * (l >> 4) + t) * kWidth + c] = acc[t];
}

// Layer 4 backward: dZ3 = bf16((dY W4) * GELU'(Z3)).
__global__ void __launch_bounds__(256) k_layer_out_bwd(int M, const float* __restrict__ dY,
                                                       const __bf16* __restrict__ W4,
                                                       const float* __restrict__ Z3,
                                                       __bf16* __restrict__ dZ3) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)M * kWidth) return;
    const int m = (int)(g / kWidth), k = (int)(g % kWidth);
    float s = 0.0f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) s += dY[(int64_t)m * kOut + o] * (float)W4[o * kWidth + k];
    dZ3[g] = (__bf16)(s * gelu_prime(Z3[g]));
}

// Partial sums of small products over one chunk of rows, one thread per
// output, rows in fixed order: part[chunk][r][c] = sum_{m in chunk} P[m][r]
// Q[m][c] (no Q: P[m][r]).  All such sums of a backward pass in one launch:
// grid.y = chunk, grid.z = job.
struct ColJobs {
    int32_t R[kMaxColJobs], Cn[kMaxColJobs], ldp[kMaxColJobs], ldq[kMaxColJobs];
    int32_t p_bf16[kMaxColJobs];  // P stored as bf16, else fp32
    const void* P[kMaxColJobs];
    const __bf16* Q[kMaxColJobs];  // nullptr: plain column sums of P
    float* part[kMaxColJobs];
};

template <class TP>
__device__ __forceinline__ float colsum_rows(const TP* __restrict__ P, int ldp,
                                             const __bf16* __restrict__ Q, int ldq, int r, int c,
                                             int m0, int m1) {
    float s = 0.0f;
    if (Q) {
        for (int m = m0; m < m1; ++m)
            s += (float)P[(int64_t)m * ldp + r] * (float)Q[(int64_t)m * ldq + c];
    } else {
        for (int m = m0; m < m1; ++m) s += (float)P[(int64_t)m * ldp + r];
    }
    return s;
}

__global__ void __launch_bounds__(256) k_colsum_jobs(int M, int mchunk, ColJobs J) {
    const int y = blockIdx.z;
    const int R = J.R[y], Cn = J.Cn[y];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= R * Cn) return;
    const int r = g / Cn, c = g % Cn;
    const int m0 = blockIdx.y * mchunk, m1 = min(M, m0 + mchunk);
    const float s =
        J.p_bf16[y]
            ? colsum_rows((const __bf16*)J.P[y], J.ldp[y], J.Q[y], J.ldq[y], r, c, m0, m1)
            : colsum_rows((const float*)J.P[y], J.ldp[y], J.Q[y], J.ldq[y], r, c, m0, m1);
    J.part[y][(int64_t)blockIdx.y * R * Cn + g] = s;
}

// All second-stage sums of one backward pass in one launch: out_y[k] =
// sum_ch P_y[ch][k], where the partials of sum y start at P + off[y] (nch[y]
// chunks of n[y] values).  Block (x, y) covers outputs [64 x, 64 x + 64) of
// sum y with 4 thread groups, group g adding chunks g, g + 4, ... in order;
// the four group sums are then added in group order (a fixed order throughout).
struct SumJobs {
    int32_t n[kMaxSumJobs];
    int32_t nch[kMaxSumJobs];
    int64_t off[kMaxSumJobs];
    float* out[kMaxSumJobs];
};

__global__ void __launch_bounds__(256) k_sum_jobs(SumJobs J, const float* __restrict__ P) {
    __shared__ float part[4][64];
    const int y = blockIdx.y;
    const int n = J.n[y], nch = J.nch[y];
    if ((int)blockIdx.x * 64 >= n) return;  // uniform over the block
    const float* Py = P + J.off[y];
    const int j = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + j;
    float s = 0.0f;
    if (k < n)
        for (int c = g; c < nch; c += 4) s += Py[(int64_t)c * n + k];
    part[g][j] = s;
    __syncthreads();
    if (g == 0 && k < n) J.out[y][k] = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
}

// One block of 1024 threads; fixed-order partial sums then a fixed tree.
__global__ void __launch_bounds__(1024) k_sum_all(int n, const float* __restrict__ v,
                                                  double* __restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += v[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[w];
        out[0] = t;
    }
}

// bf16 copies of the weights (and the transposes are not needed: the MFMA
// operands address W through strides).
__global__ void __launch_bounds__(256) k_refresh(const float* __restrict__ theta,
                                                 __bf16* __restrict__ W1, __bf16* __restrict__ W2,
                                                 __bf16* __restrict__ W3, __bf16* __restrict__ W4) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kWidth * kIn) W1[k] = (__bf16)theta[kOffW1 + k];
    if (k < kWidth * kWidth) {
        W2[k] = (__bf16)theta[kOffW2 + k];
        W3[k] = (__bf16)theta[kOffW3 + k];
    }
    if (k < kOut * kWidth) W4[k] = (__bf16)theta[kOffW4 + k];
}

// Adam (fp32): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void __launch_bounds__(256) k_adam(int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              float* __restrict__ theta, __bf16* __restrict__ W1,
                                              __bf16* __restrict__ W2, __bf16* __restrict__ W3,
                                              __bf16* __restrict__ W4) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float t = theta[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    theta[k] = t;
    // the bf16 copy the forward and backward kernels read (as k_refresh makes it)
    if (k >= kOffW1 && k < kOffW1 + kWidth * kIn) W1[k - kOffW1] = (__bf16)t;
    else if (k >= kOffW2 && k < kOffW2 + kWidth * kWidth) W2[k - kOffW2] = (__bf16)t;
    else if (k >= kOffW3 && k < kOffW3 + kWidth * kWidth) W3[k - kOffW3] = (__bf16)t;
    else if (k >= kOffW4 && k < kOffW4 + kOut * kWidth) W4[k - kOffW4] = (__bf16)t;
}

// Minibatch gather: row r takes dataset row floor(h * n / 2^64), h the
// splitmix64 hash of seed + step * B + r.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_gather(int64_t n, int B, uint64_t seed, int64_t step,
                                                const float* __restrict__ X,
                                                const float* __restrict__ T,
                                                float* __restrict__ Xo, float* __restrict__ To) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    const uint64_t h = splitmix64(seed + (uint64_t)step * (uint64_t)B + (uint64_t)r);
    const int64_t i = (int64_t)__umul64hi(h, (uint64_t)n);
#pragma unroll
    for (int k = 0; k < kIn; ++k) Xo[(int64_t)r * kIn + k] = X[i * kIn + k];
#pragma unroll
    for (int k = 0; k < kOut; ++k) To[(int64_t)r * kOut + k] = T[i * kOut + k];
}

// Features of a point: position squashed into the unit disc about mid-chord,
// distance to the nearest wall point of its own cloud, Mach number and angle
// of attack recovered from the free-stream velocity.
__global__ void __launch_bounds__(256) k_features(int64_t p0, int64_t m, const D2* __restrict__ xy,
                                                  const int32_t* __restrict__ comp,
                                                  const int32_t* __restrict__ wall_list,
                                                  const int32_t* __restrict__ wall_off,
                                                  const double* __restrict__ vinf,
                                                  const D4* __restrict__ U, double gamma,
                                                  float* __restrict__ X, float* __restrict__ T) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int64_t p = p0 + r;
    const int k = comp ? comp[p] : 0;
    const D2 c = xy[p];
    double d2 = 1e300;
    for (int w = wall_off[k]; w < wall_off[k + 1]; ++w) {
        const D2 q = xy[wall_list[w]];
        const double dx = c.x - q.x, dy = c.y - q.y;
        d2 = fmin(d2, dx * dx + dy * dy);
    }
    const double d = wall_off[k + 1] > wall_off[k] ? sqrt(d2) : 1e3;
    const double ex = c.x - 0.5, rc = sqrt(ex * ex + c.y * c.y);
    const double u1 = vinf[2 * k], u2 = vinf[2 * k + 1];
    const double mach = sqrt(u1 * u1 + u2 * u2);
    const double aoa = atan2(u2, u1) * (180.0 / 3.14159265358979323846);
    float* x = X + r * kIn;
    x[0] = (float)(ex / (1.0 + rc));
    x[1] = (float)(c.y / (1.0 + rc));
    x[2] = (float)(2.0 * d / (d + 0.1) - 1.0);
    x[3] = (float)((mach - 0.6) / 0.25);
    x[4] = (float)((aoa - 2.0) / 6.0);
    if (T) {
        const D4 u = U[p];
        const double irho = 1.0 / u.x, v1 = u.y * irho, v2 = u.z * irho;
        const double pr = (gamma - 1.0) * (u.w - 0.5 * u.x * (v1 * v1 + v2 * v2));
        float* t = T + r * kOut;
        t[0] = (float)(u.x - 1.0);
        t[1] = (float)(v1 - u1);
        t[2] = (float)(v2 - u2);
        t[3] = (float)(gamma * pr - 1.0);
    }
}

// U of points [p0, p0 + m) from predicted deviations from the free stream
// (rho - 1, u - u_inf, v - v_inf, gamma p - 1).  Outer points stay at the free
// stream and wall points keep only the tangential velocity.  With FALLBACK,
// only points of components flagged in bad are written, at the free stream.
template <bool FALLBACK>
__global__ void __launch_bounds__(256) k_pred_to_U(int64_t p0, int64_t m, const float* __restrict__ Y,
                                                   const int8_t* __restrict__ type,
                                                   const D2* __restrict__ frame,
                                                   const int32_t* __restrict__ comp,
                                                   const double* __restrict__ vinf, double gamma,
                                                   int32_t* __restrict__ bad, D4* __restrict__ U) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int64_t p = p0 + r;
    const int k = comp ? comp[p] : 0;
    if (FALLBACK && !bad[k]) return;
    double rho = 1.0, u1 = vinf[2 * k], u2 = vinf[2 * k + 1], gp = 1.0;
    if (!FALLBACK && type[p] != 2) {
        const float* y = Y + r * kOut;
        rho += (double)y[0];
        u1 += (double)y[1];
        u2 += (double)y[2];
        gp += (double)y[3];
        // unusable prediction: the residual check sends the whole component back to the free stream
        if (!(rho > 0.05) || !(gp > 0.05) || !(fabs(u1) + fabs(u2) < 1e3)) {
            bad[k] = 1;
            rho = 1.0;
            u1 = vinf[2 * k];
            u2 = vinf[2 * k + 1];
            gp = 1.0;
        }
    }
    if (type[p] == 0) {
        const D2 t = frame[p];
        const double ut = u1 * t.x + u2 * t.y;
        u1 = ut * t.x;
        u2 = ut * t.y;
    }
    const double pr = gp / gamma;
    U[p] = {rho, rho * u1, rho * u2, pr / (gamma - 1.0) + 0.5 * rho * (u1 * u1 + u2 * u2)};
}

__global__ void k_vet(int ncomp, const double* __restrict__ res, const double* __restrict__ res_fs,
                      int32_t* __restrict__ bad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncomp) return;
    if (!(res[k] < res_fs[k])) bad[k] = 1;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t refresh_weights(Net& net) {
    hipLaunchKernelGGL(k_refresh, dim3(nblk(kWidth * kWidth, 256)), dim3(256), 0, net.stream,
                       net.theta, net.W1b, net.W2b, net.W3b, net.W4b);
    return hipGetLastError();
}

// Forward over rows [0, M) of the workspace (M a multiple of 16, Mvalid <= M).
hipError_t forward(Net& net, const float* X, int M, int Mvalid, const float* T, float* Y) {
    hipStream_t st = net.stream;
    const float* th = net.theta;
    const dim3 grid(nblk(M, 16 * kFwdWaves)), block(64 * kFwdWaves);
    if (T)
        hipLaunchKernelGGL(k_mlp_forward<true>, grid, block, 0, st, M, Mvalid, X, net.W1b,
                           th + kOffB1, net.W2b, th + kOffB2, net.W3b, th + kOffB3, net.W4b,
                           th + kOffB4, T, (float*)nullptr, net.Xb, net.Z1, net.Z2, net.Z3,
                           net.H1, net.H2, net.H3, net.dY, net.se);
    else
        hipLaunchKernelGGL(k_mlp_forward<false>, grid, block, 0, st, M, Mvalid, X, net.W1b,
                           th + kOffB1, net.W2b, th + kOffB2, net.W3b, th + kOffB3, net.W4b,
                           th + kOffB4, (const float*)nullptr, Y, net.Xb, net.Z1, net.Z2,
                           net.Z3, net.H1, net.H2, net.H3, net.dY, net.se);
    return hipGetLastError();
}

// Backward after a forward with targets: gradient (flat, fp32) into net.grad.
// Two-stage sum over rows: chunk partials, then a fixed-order sum of the chunks.
// The sums over rows of one backward pass: each first stage writes its chunk
// partials to its own region of net.part (sized by part_floats for the
// workspace), and one launch adds them all at the end.
struct SumPlan {
    SumJobs jobs{};
    int njobs = 0;
    int nmax = 0;
    int64_t off = 0;
    // registers a sum of nch chunk partials of n values; returns where its
    // partials start in net.part
    ColJobs cols{};
    int ncols = 0;
    int colmax = 0;
    int64_t add(int n, int nch, float* out) {
        jobs.n[njobs] = n;
        jobs.nch[njobs] = nch;
        jobs.off[njobs] = off;
        jobs.out[njobs] = out;
        nmax = std::max(nmax, n);
        const int64_t at = off;
        off += (int64_t)nch * n;
        ++njobs;
        return at;
    }
};

constexpr int kColRows = 64;  // rows per thread in a column-sum first stage

// Registers the column sums of P (times Q when given) over rows; their first
// stage runs with the others at the end of the backward pass.
static void colsum(Net& net, SumPlan& plan, int M, int R, int Cn, const void* P, bool p_bf16,
                   int ldp, const __bf16* Q, int ldq, float* out) {
    const int nch = (M + kColRows - 1) / kColRows;
    const int k = plan.ncols++;
    plan.cols.R[k] = R;
    plan.cols.Cn[k] = Cn;
    plan.cols.ldp[k] = ldp;
    plan.cols.ldq[k] = ldq;
    plan.cols.p_bf16[k] = p_bf16;
    plan.cols.P[k] = P;
    plan.cols.Q[k] = Q;
    plan.cols.part[k] = net.part + plan.add(R * Cn, nch, out);
    plan.colmax = std::max(plan.colmax, R * Cn);
}

static void wgrad(Net& net, SumPlan& plan, int M, const __bf16* dZ, const __bf16* H, float* out) {
    const int nch = (M + kChunk - 1) / kChunk;
    float* dst = net.part + plan.add(kWidth * kWidth, nch, out);
    hipLaunchKernelGGL(k_dense_wgrad, dim3(64, nch), dim3(64), 0, net.stream, M, kChunk, dZ, H,
                       dst);
}

int64_t part_floats(int64_t cap) {
    const int64_t nw = (cap + kChunk - 1) / kChunk, nc = (cap + kColRows - 1) / kColRows;
    return 2 * nw * kWidth * kWidth +
           nc * (kOut * kWidth + kOut + kWidth + kWidth + kWidth * kIn + kWidth);
}

hipError_t backward(Net& net, int M) {
    hipStream_t st = net.stream;
    float* g = net.grad;
    SumPlan plan;
    // layer 4
    colsum(net, plan, M, kOut, kWidth, net.dY, false, kOut, net.H3, kWidth, g + kOffW4);
    colsum(net, plan, M, kOut, 1, net.dY, false, kOut, nullptr, 0, g + kOffB4);
    hipLaunchKernelGGL(k_layer_out_bwd, dim3(nblk((int64_t)M * kWidth, 256)), dim3(256), 0, st, M,
                       net.dY, net.W4b, net.Z3, net.dZ3);
    // layer 3
    wgrad(net, plan, M, net.dZ3, net.H2, g + kOffW3);
    colsum(net, plan, M, kWidth, 1, net.dZ3, true, kWidth, nullptr, 0, g + kOffB3);
    hipLaunchKernelGGL(k_dense_bwd_data<true>, dim3((M / 16) * 8), dim3(64), 0, st, M, net.dZ3,
                       net.W3b, net.Z2, net.dZ2, (float*)nullptr);
    // layer 2
    wgrad(net, plan, M, net.dZ2, net.H1, g + kOffW2);
    colsum(net, plan, M, kWidth, 1, net.dZ2, true, kWidth, nullptr, 0, g + kOffB2);
    hipLaunchKernelGGL(k_dense_bwd_data<false>, dim3((M / 16) * 8), dim3(64), 0, st, M, net.dZ2,
                       net.W2b, net.Z1, (__bf16*)nullptr, net.dZ1);
    // layer 1
    colsum(net, plan, M, kWidth, kIn, net.dZ1, false, kWidth, net.Xb, kIn, g + kOffW1);
    colsum(net, plan, M, kWidth, 1, net.dZ1, false, kWidth, nullptr, 0, g + kOffB1);
    // the column sums' first stage, then every second stage
    hipLaunchKernelGGL(k_colsum_jobs, dim3(nblk(plan.colmax, 256), (M + kColRows - 1) / kColRows,
                                           plan.ncols),
                       dim3(256), 0, st, M, kColRows, plan.cols);
    hipLaunchKernelGGL(k_sum_jobs, dim3(nblk(plan.nmax, 64), plan.njobs), dim3(256), 0, st,
                       plan.jobs, net.part);
    return hipGetLastError();
}

hipError_t loss(Net& net, int M, double* d_out) {
    hipLaunchKernelGGL(k_sum_all, dim3(1), dim3(1024), 0, net.stream, M * kOut, net.se, d_out);
    return hipGetLastError();
}

hipError_t adam_step(Net& net, float lr) {
    net.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)net.step);
    const float c2 = 1.0f - std::pow(b2, (float)net.step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(kParams, 256)), dim3(256), 0, net.stream, kParams, lr, b1,
                       b2, 1e-8f, c1, c2, net.grad, net.m, net.v, net.theta, net.W1b, net.W2b,
                       net.W3b, net.W4b);
    return hipGetLastError();
}

hipError_t gather(Net& net, int64_t n, const float* X, const float* T, int B, uint64_t seed,
                  int64_t step) {
    hipLaunchKernelGGL(k_gather, dim3(nblk(B, 256)), dim3(256), 0, net.stream, n, B, seed, step, X,
                       T, net.Xin, net.Tin);
    return hipGetLastError();
}

hipError_t features(const State& s, int64_t p0, int64_t m, float* Xout, float* Tout) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_features, dim3(nblk(m, 256)), dim3(256), 0, s.stream, p0, m, c.xy, c.comp,
                       c.wall_list, c.wall_off, s.vinf, s.U, s.prm.gamma, Xout, Tout);
    return hipGetLastError();
}

hipError_t pred_to_U(Net& net, const State& s, int64_t p0, int64_t m, const float* Y) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_pred_to_U<false>, dim3(nblk(m, 256)), dim3(256), 0, s.stream, p0, m, Y,
                       c.type, c.frame, c.comp, s.vinf, s.prm.gamma, net.d_bad, s.U);
    return hipGetLastError();
}

hipError_t vet_and_fallback(Net& net, const State& s, const double* res) {
    const Cloud& c = *s.cloud;
    hipLaunchKernelGGL(k_vet, dim3(nblk(c.ncomp, 256)), dim3(256), 0, s.stream, c.ncomp, res,
                       net.d_res_fs, net.d_bad);
    hipLaunchKernelGGL(k_pred_to_U<true>, dim3(nblk(c.n, 256)), dim3(256), 0, s.stream, (int64_t)0,
                       c.n, (const float*)nullptr, c.type, c.frame, c.comp, s.vinf, s.prm.gamma,
                       net.d_bad, s.U);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace lskum
