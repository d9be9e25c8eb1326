// Host build of the per-pair descriptor arithmetic in tnep_math.h, for the
// CPU self-check tests (not part of libtnep).  Computes one atom's
// descriptor q from neighbour vectors with the same functions the gfx950
// kernel uses, in FP32.
#include <cmath>

#include "tnep_math.h"

extern "C" void tnep_hc_sh(const float* u, float* P, float* dP) {
    tnep::sh_foreach(u[0], u[1], u[2], [&](int idx, int, float p, float px, float py, float pz) {
        P[idx] = p;
        dP[3 * idx] = px;
        dP[3 * idx + 1] = py;
        dP[3 * idx + 2] = pz;
    });
}

extern "C" float tnep_hc_four_body(const float* a, float* d) { return tnep::four_body_l2(a, d); }

extern "C" void tnep_hc_basis9(float r, float rc, float* f, float* df) {
    const float pi = 3.14159265358979323846f;
    const float fc = 0.5f * (1.f + std::cos(pi * r / rc));
    const float dfc = -0.5f * pi / rc * std::sin(pi * r / rc);
    tnep::cheb_basis_d<9>(r, 1.f / rc, fc, dfc, f, df);
}

// q for one atom: n neighbours vec[n][3] (all inside rc_radial) of species
// tj[n]; c tables of the atom's own species row: cR[T][NR][9], cA[T][NA][9];
// NR = NA = 5, four-body on.  q[30].
extern "C" void tnep_hc_descriptor(int n, const float* vec, const int* tj, const float* cR, const float* cA,
                                   float rcR, float rcA, float* q) {
    const int NR = 5, NA = 5, K = 9;
    float qR[5] = {0}, A[5][24] = {{0}};
    const float pi = 3.14159265358979323846f;
    for (int j = 0; j < n; ++j) {
        const float* v = vec + 3 * j;
        const float r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        float f[9];
        tnep::cheb_basis<9>(r, 1.f / rcR, 0.5f * (1.f + std::cos(pi * r / rcR)), f);
        for (int m = 0; m < NR; ++m) {
            float g = 0.f;
            for (int k = 0; k < K; ++k) g += cR[(tj[j] * NR + m) * K + k] * f[k];
            qR[m] += g;
        }
        if (r < rcA) {
            tnep::cheb_basis<9>(r, 1.f / rcA, 0.5f * (1.f + std::cos(pi * r / rcA)), f);
            float gA[5];
            for (int m = 0; m < NA; ++m) {
                float g = 0.f;
                for (int k = 0; k < K; ++k) g += cA[(tj[j] * NA + m) * K + k] * f[k];
                gA[m] = g;
            }
            tnep::sh_foreach(v[0] / r, v[1] / r, v[2] / r, [&](int idx, int, float p, float, float, float) {
                for (int m = 0; m < NA; ++m) A[m][idx] += gA[m] * p;
            });
        }
    }
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
