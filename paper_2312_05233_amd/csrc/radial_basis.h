// Radial basis of the descriptor (Sec. 2.1, NEP radial functions) and pair
// distances, shared by the neighbour search (which accumulates the radial
// descriptor sums) and the evaluation kernels.  The basis functions are also
// compiled for the host by the CPU self-check; the pair distances use the
// hardware square roots and are device-only.
#pragma once

#include <hip/hip_runtime.h>

namespace tnep {

// Cosine cutoff f_c(r) = (1 + cos(pi r / r_c)) / 2 = sin^2(w), w = (pi/2)(1 - r/r_c),
// which keeps relative accuracy as r -> r_c; f_c'(r) = -(pi / r_c) sin(w) cos(w).
// sin and cos of w in [0, pi/2] from their Taylor series to w^13 / w^14
// (truncation below 1e-9).  v = 1 - r / r_c.
__host__ __device__ __forceinline__ float sin_half_pi(float w) {
    const float w2 = w * w;
    float p = 1.f / 6227020800.f;
    p = p * w2 - 1.f / 39916800.f;
    p = p * w2 + 1.f / 362880.f;
    p = p * w2 - 1.f / 5040.f;
    p = p * w2 + 1.f / 120.f;
    p = p * w2 - 1.f / 6.f;
    p = p * w2 + 1.f;
    return w * p;
}
__host__ __device__ __forceinline__ float cos_half_pi(float w) {
    const float w2 = w * w;
    float p = -1.f / 87178291200.f;
    p = p * w2 + 1.f / 479001600.f;
    p = p * w2 - 1.f / 3628800.f;
    p = p * w2 + 1.f / 40320.f;
    p = p * w2 - 1.f / 720.f;
    p = p * w2 + 1.f / 24.f;
    p = p * w2 - 0.5f;
    p = p * w2 + 1.f;
    return p;
}
__host__ __device__ __forceinline__ float cutoff_fc(float v) {
    const float s = sin_half_pi(1.57079632679489662f * v);
    return s * s;
}
__host__ __device__ __forceinline__ void cutoff_fc_d(float v, float rc_inv, float& fc, float& dfc) {
    const float w = 1.57079632679489662f * v;
    const float s = sin_half_pi(w), c = cos_half_pi(w);
    fc = s * s;
    dfc = -3.14159265358979323846f * rc_inv * s * c;
}

// Pair distances from the hardware square root and reciprocal square root
// (about 1 ulp): squared pair distances lie far inside the normal range, so
// the scaling and correction steps that the library forms add (about 16 and 6
// instructions) buy nothing here.
__device__ __forceinline__ float pair_rsqrt(float r2) { return __builtin_amdgcn_rsqf(r2); }
__device__ __forceinline__ float pair_sqrt(float r2) { return __builtin_amdgcn_sqrtf(r2); }

// Chebyshev polynomials T_k(x), k = 0..K-1 (three-term recurrence).  The
// radial basis is f_k = (T_k(x) + 1)/2 f_c, so sums of f_k and of their
// contractions with coefficients are formed from sums of T_k (one fused
// multiply-add per term) instead of building every f_k.
template <int K>
__host__ __device__ __forceinline__ void cheb_T(float x, float* T) {
    T[0] = 1.f;
    if (K > 1) T[1] = x;
    const float x2 = x + x;
#pragma unroll
    for (int k = 2; k < K; ++k) T[k] = x2 * T[k - 1] - T[k - 2];
}

// T_k(x) and dT_k/dx.
template <int K>
__host__ __device__ __forceinline__ void cheb_T_d(float x, float* T, float* dT) {
    T[0] = 1.f;
    dT[0] = 0.f;
    if (K > 1) {
        T[1] = x;
        dT[1] = 1.f;
    }
    const float x2 = x + x;
#pragma unroll
    for (int k = 2; k < K; ++k) {
        T[k] = x2 * T[k - 1] - T[k - 2];
        dT[k] = 2.f * T[k - 1] + x2 * dT[k - 1] - dT[k - 2];
    }
}

}  // namespace tnep
