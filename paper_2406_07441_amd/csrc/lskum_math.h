// Double-precision exp and erf for the solver kernels.
//
// exp: x = k ln2 + r with k = rint(x / ln2) and r formed with ln2 split into
// a high and a low part, e^r = 1 + r + r^2 Q(r) with Q of degree 10, scaled
// by 2^k.  erf: x P(x^2) with P of degree 11 for |x| < 1, the library erf
// beyond.  The coefficients (lskum_math_coef.h) are near-minimax Chebyshev
// fits written by gen_lskum_math.py; evaluated with fused multiply-adds both
// are within one unit in the last place of the correctly rounded values on
// the reduced ranges.
//
// The coefficients are read from __constant__ tables: the loads are uniform,
// hoisted out of the neighbour loops, and the values stay in scalar
// registers, so every Horner step is one v_fma_f64 with a scalar operand.
// Written with literal coefficients, each step costs two more instructions
// (the literal is rebuilt in a register pair before every step), which made
// the library's polynomials and literal-coefficient versions of these about
// 10% slower in the residual kernel.
#pragma once
// Defines __constant__ tables: include it from one translation unit only
// (the solver kernels' lskum_device.hip).

#include <hip/hip_runtime.h>

#include "lskum_math_coef.h"

namespace lskum {

__constant__ double cExpQ[11] = {kExpQ[0], kExpQ[1], kExpQ[2], kExpQ[3], kExpQ[4], kExpQ[5],
                                 kExpQ[6], kExpQ[7], kExpQ[8], kExpQ[9], kExpQ[10]};
__constant__ double cErfP[12] = {kErfP[0], kErfP[1], kErfP[2], kErfP[3], kErfP[4],  kErfP[5],
                                 kErfP[6], kErfP[7], kErfP[8], kErfP[9], kErfP[10], kErfP[11]};

// round-to-nearest-even double -> int32 with the hardware's defined result
// out of range (saturated; 0 for NaN), where a C++ conversion is undefined
__device__ __forceinline__ int cvt_i32_sat(double k) {
    int r;
    asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(k));
    return r;
}

__device__ __forceinline__ double exp_fast(double x) {
    const double k = rint(x * kLog2e);
    double r = fma(-k, kLn2Hi, x);
    r = fma(-k, kLn2Lo, r);
    // the first step with literals: two fewer scalar register pairs
    double q = fma(kExpQ[0], r, kExpQ[1]);
#pragma unroll
    for (int i = 2; i < 11; ++i) q = fma(q, r, cExpQ[i]);
    const double e = 1.0 + fma(r * r, q, r);
    return ldexp(e, cvt_i32_sat(k));
}

__device__ __forceinline__ double erf_fast(double x) {
    if (fabs(x) < 1.0) {
        const double t = x * x;
        double p = fma(kErfP[0], t, kErfP[1]);
#pragma unroll
        for (int i = 2; i < 12; ++i) p = fma(p, t, cErfP[i]);
        return x * p;
    }
    return erf(x);
}

// the same names for the precision-generic sweep code
__device__ __forceinline__ double exp_k(double x) { return exp_fast(x); }
__device__ __forceinline__ double erf_k(double x) { return erf_fast(x); }
__device__ __forceinline__ float exp_k(float x) { return expf(x); }
__device__ __forceinline__ float erf_k(float x) { return erff(x); }

}  // namespace lskum
