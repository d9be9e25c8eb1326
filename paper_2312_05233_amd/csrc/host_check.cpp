// Host build of the per-pair descriptor arithmetic of the evaluation kernels,
// for the CPU self-check tests (not part of libtnep).  Every function here
// calls the same inline functions the gfx950 kernels call (tnep_math.h,
// radial_basis.h) in the same way, in FP32, so that a mistake in them shows
// against the FP64 oracle without a GPU.
#include <cmath>

#include "radial_basis.h"
#include "tnep_math.h"

// Normalised harmonics Y_lm(u) and their gradients with respect to u, as the
// kernels form them: raw polynomials P_lm times kShNorm.
extern "C" void tnep_hc_sh(const float* u, float* P, float* dP) {
    tnep::sh_foreach_raw(u[0], u[1], u[2], [&](int idx, int, float p, float px, float py, float pz) {
        const float c = tnep::kShNorm[idx];
        P[idx] = c * p;
        dP[3 * idx] = c * px;
        dP[3 * idx + 1] = c * py;
        dP[3 * idx + 2] = c * pz;
    });
}

extern "C" float tnep_hc_four_body(const float* a, float* d) { return tnep::four_body_l2(a, d); }

// Radial basis f_k(r) = (T_k(x) + 1)/2 f_c(r), k = 0..8, and its radial
// derivative, from the kernels' cutoff (cutoff_fc_d of v = 1 - r/r_c) and
// Chebyshev recurrences (cheb_T_d), x = 2 (r/r_c - 1)^2 - 1, dx/dr = 4 (r/r_c - 1)/r_c.
extern "C" void tnep_hc_basis9(float r, float rc, float* f, float* df) {
    const float rc_inv = 1.f / rc;
    float fc, dfc, T[9], dT[9];
    tnep::cutoff_fc_d(1.f - r * rc_inv, rc_inv, fc, dfc);
    const float t = r * rc_inv - 1.f;
    tnep::cheb_T_d<9>(2.f * t * t - 1.f, T, dT);
    for (int k = 0; k < 9; ++k) {
        f[k] = 0.5f * (T[k] + 1.f) * fc;
        df[k] = 0.5f * dT[k] * (4.f * t * rc_inv) * fc + 0.5f * (T[k] + 1.f) * dfc;
    }
}

// q for one atom as the FP32 evaluation kernel forms it: n neighbours vec[n][3]
// (all inside rc_radial) of species tj[n]; coefficient blocks of the atom's own
// species row cR[T][NR][9], cA[T][NA][9]; NR = NA = 5, four-body on.  Radial
// sums of cutoff_fc * T_k (as the neighbour search forms them) contracted with
// c^R; angular functions g_n = fc/2 (sum_k c_nk T_k + sum_k c_nk); harmonics
// accumulated raw and scaled by kShNorm once.  q[30].
extern "C" void tnep_hc_descriptor(int n, const float* vec, const int* tj, const float* cR, const float* cA,
                                   float rcR, float rcA, float* q) {
    constexpr int NR = 5, NA = 5, K = 9;
    const float rcR_inv = 1.f / rcR, rcA_inv = 1.f / rcA;
    int T = 0;
    for (int j = 0; j < n; ++j) T = tj[j] + 1 > T ? tj[j] + 1 : T;
    float qR[NR] = {0}, A[NA][tnep::kLM] = {{0}};
    for (int t = 0; t < T; ++t) {
        float FT[K] = {0}, Fs = 0.f;
        const float* cRt = cR + t * NR * K;
        const float* cAt = cA + t * NA * K;
        float Cs[NA];
        for (int m = 0; m < NA; ++m) {
            float c = 0.f;
            for (int k = 0; k < K; ++k) c += cAt[m * K + k];
            Cs[m] = c;
        }
        for (int j = 0; j < n; ++j) {
            if (tj[j] != t) continue;
            const float* v = vec + 3 * j;
            const float r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            const float r = std::sqrt(r2), rinv = 1.f / r;
            float Tk[K];
            const float fc = tnep::cutoff_fc(1.f - r * rcR_inv);
            const float tt = r * rcR_inv - 1.f;
            tnep::cheb_T<K>(2.f * tt * tt - 1.f, Tk);
            Fs += fc;
            for (int k = 0; k < K; ++k) FT[k] += fc * Tk[k];
            if (r < rcA) {
                const float hfc = 0.5f * tnep::cutoff_fc(1.f - r * rcA_inv);
                const float ta = r * rcA_inv - 1.f;
                tnep::cheb_T<K>(2.f * ta * ta - 1.f, Tk);
                float gA[NA];
                for (int m = 0; m < NA; ++m) {
                    float g = Cs[m];
                    for (int k = 0; k < K; ++k) g += cAt[m * K + k] * Tk[k];
                    gA[m] = hfc * g;
                }
                tnep::sh_foreach_raw(v[0] * rinv, v[1] * rinv, v[2] * rinv,
                                     [&](int idx, int, float P, float, float, float) {
                                         for (int m = 0; m < NA; ++m) A[m][idx] += gA[m] * P;
                                     });
            }
        }
        float F[K];
        for (int k = 0; k < K; ++k) F[k] = 0.5f * (FT[k] + Fs);
        for (int m = 0; m < NR; ++m)
            for (int k = 0; k < K; ++k) qR[m] += cRt[m * K + k] * F[k];
    }
    for (int m = 0; m < NA; ++m)
        for (int c = 0; c < tnep::kLM; ++c) A[m][c] *= tnep::kShNorm[c];
    for (int m = 0; m < NR; ++m) q[m] = qR[m];
    const int lo[5] = {0, 0, 3, 8, 15}, hi[5] = {0, 3, 8, 15, 24};
    for (int l = 1; l <= 4; ++l)
        for (int m = 0; m < NA; ++m) {
            float s = 0.f;
            for (int c = lo[l]; c < hi[l]; ++c) s += A[m][c] * A[m][c];
            q[NR + (l - 1) * NA + m] = s;
        }
    float d[5];
    for (int m = 0; m < NA; ++m) q[NR + 4 * NA + m] = tnep::four_body_l2(&A[m][3], d);
}
