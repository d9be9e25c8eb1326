// Per-pair and per-atom arithmetic of the TNEP descriptor (NEP form, Sec. 2.1)
// shared by the gfx950 kernels.  Plain inline functions on float, callable
// from device code and from the host-side self-check.
#pragma once

#include <hip/hip_runtime.h>

namespace tnep {

// Real orthonormal spherical harmonics, l = 1..4, written as homogeneous
// polynomials P_lm(x, y, z) in the components of a unit vector u; the
// gradient of Y_lm(r/|r|) with respect to r is (grad_u P - l P u) / |r|.
// Channel index: idx = l*l - 1 + (l + m), i.e. l=1 -> 0..2, l=2 -> 3..7,
// l=3 -> 8..14, l=4 -> 15..23.  f(idx, l, P, dPx, dPy, dPz) is called for
// every channel (all inlined by the compiler).
constexpr int kLM = 24;

template <class F>
__host__ __device__ __forceinline__ void sh_foreach(float x, float y, float z, F&& f) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    // l = 1
    {
        const float c = 0.48860251190291992f;  // sqrt(3/(4 pi))
        f(0, 1, c * y, 0.f, c, 0.f);
        f(1, 1, c * z, 0.f, 0.f, c);
        f(2, 1, c * x, c, 0.f, 0.f);
    }
    // l = 2
    {
        const float a = 1.0925484305920792f;   // sqrt(15/pi)/2
        const float b = 0.31539156525252005f;  // sqrt(5/pi)/4
        const float c = 0.54627421529603959f;  // sqrt(15/pi)/4
        f(3, 2, a * xy, a * y, a * x, 0.f);
        f(4, 2, a * yz, 0.f, a * z, a * y);
        f(5, 2, b * (2.f * z2 - x2 - y2), -2.f * b * x, -2.f * b * y, 4.f * b * z);
        f(6, 2, a * xz, a * z, 0.f, a * x);
        f(7, 2, c * (x2 - y2), 2.f * c * x, -2.f * c * y, 0.f);
    }
    // l = 3
    {
        const float a = 0.59004358992664352f;  // sqrt(35/(2 pi))/4
        const float b = 2.8906114426405538f;   // sqrt(105/pi)/2
        const float c = 0.45704579946446572f;  // sqrt(21/(2 pi))/4
        const float d = 0.37317633259011540f;  // sqrt(7/pi)/4
        const float e = 1.4453057213202769f;   // sqrt(105/pi)/4
        f(8, 3, a * (3.f * x2 * y - y2 * y), 6.f * a * xy, 3.f * a * (x2 - y2), 0.f);
        f(9, 3, b * xy * z, b * yz, b * xz, b * xy);
        f(10, 3, c * y * (4.f * z2 - x2 - y2), -2.f * c * xy, c * (4.f * z2 - x2 - 3.f * y2), 8.f * c * yz);
        f(11, 3, d * z * (2.f * z2 - 3.f * x2 - 3.f * y2), -6.f * d * xz, -6.f * d * yz,
          3.f * d * (2.f * z2 - x2 - y2));
        f(12, 3, c * x * (4.f * z2 - x2 - y2), c * (4.f * z2 - 3.f * x2 - y2), -2.f * c * xy, 8.f * c * xz);
        f(13, 3, e * z * (x2 - y2), 2.f * e * xz, -2.f * e * yz, e * (x2 - y2));
        f(14, 3, a * (x2 * x - 3.f * x * y2), 3.f * a * (x2 - y2), -6.f * a * xy, 0.f);
    }
    // l = 4
    {
        const float a = 2.5033429417967046f;   // 3 sqrt(35/pi)/4
        const float b = 1.7701307697799304f;   // 3 sqrt(35/(2 pi))/4
        const float c = 0.94617469575756008f;  // 3 sqrt(5/pi)/4
        const float d = 0.66904654355728917f;  // 3 sqrt(5/(2 pi))/4
        const float e = 0.10578554691520431f;  // 3 / (16 sqrt(pi))
        const float g = 0.47308734787878004f;  // 3 sqrt(5/pi)/8
        const float h = 0.62583573544917614f;  // 3 sqrt(35/pi)/16
        const float xyz = xy * z;
        f(15, 4, a * xy * (x2 - y2), a * y * (3.f * x2 - y2), a * x * (x2 - 3.f * y2), 0.f);
        f(16, 4, b * yz * (3.f * x2 - y2), 6.f * b * xyz, 3.f * b * z * (x2 - y2), b * y * (3.f * x2 - y2));
        f(17, 4, c * xy * (6.f * z2 - x2 - y2), c * y * (6.f * z2 - 3.f * x2 - y2), c * x * (6.f * z2 - x2 - 3.f * y2),
          12.f * c * xyz);
        f(18, 4, d * yz * (4.f * z2 - 3.f * x2 - 3.f * y2), -6.f * d * xyz, d * z * (4.f * z2 - 3.f * x2 - 9.f * y2),
          3.f * d * y * (4.f * z2 - x2 - y2));
        f(19, 4, e * (8.f * z2 * z2 - 24.f * (x2 + y2) * z2 + 3.f * (x2 + y2) * (x2 + y2)),
          12.f * e * x * (x2 + y2 - 4.f * z2), 12.f * e * y * (x2 + y2 - 4.f * z2),
          16.f * e * z * (2.f * z2 - 3.f * (x2 + y2)));
        f(20, 4, d * xz * (4.f * z2 - 3.f * x2 - 3.f * y2), d * z * (4.f * z2 - 9.f * x2 - 3.f * y2), -6.f * d * xyz,
          3.f * d * x * (4.f * z2 - x2 - y2));
        f(21, 4, g * (6.f * (x2 - y2) * z2 - x2 * x2 + y2 * y2), 4.f * g * x * (3.f * z2 - x2),
          4.f * g * y * (y2 - 3.f * z2), 12.f * g * z * (x2 - y2));
        f(22, 4, b * xz * (x2 - 3.f * y2), 3.f * b * z * (x2 - y2), -6.f * b * xyz, b * x * (x2 - 3.f * y2));
        f(23, 4, h * (x2 * x2 - 6.f * x2 * y2 + y2 * y2), 4.f * h * x * (x2 - 3.f * y2), 4.f * h * y * (y2 - 3.f * x2),
          0.f);
    }
}

// Chebyshev radial basis with the cosine cutoff.  Given r, 1/r_c and the
// cutoff value fc = (1 + cos(pi r / r_c))/2, writes f_k = (T_k(x) + 1)/2 fc,
// x = 2 (r/r_c - 1)^2 - 1, for k = 0..K-1.
template <int K>
__host__ __device__ __forceinline__ void cheb_basis(float r, float rc_inv, float fc, float* f) {
    const float t = r * rc_inv - 1.f;
    const float x = 2.f * t * t - 1.f;
    float tm1 = 1.f, tk = x;
    f[0] = fc;
    if (K > 1) f[1] = 0.5f * (x + 1.f) * fc;
#pragma unroll
    for (int k = 2; k < K; ++k) {
        const float tn = 2.f * x * tk - tm1;
        f[k] = 0.5f * (tn + 1.f) * fc;
        tm1 = tk;
        tk = tn;
    }
}

// Same with radial derivatives: dfc = d fc / dr = -(pi / (2 r_c)) sin(pi r / r_c).
template <int K>
__host__ __device__ __forceinline__ void cheb_basis_d(float r, float rc_inv, float fc, float dfc, float* f,
                                                      float* df) {
    const float t = r * rc_inv - 1.f;
    const float x = 2.f * t * t - 1.f;
    const float dx = 4.f * t * rc_inv;
    float tm1 = 1.f, tk = x;     // T_{k-1}, T_k
    float dm1 = 0.f, dk = 1.f;   // T'_{k-1}, T'_k (d/dx)
    f[0] = fc;
    df[0] = dfc;
    if (K > 1) {
        f[1] = 0.5f * (x + 1.f) * fc;
        df[1] = 0.5f * dx * fc + 0.5f * (x + 1.f) * dfc;
    }
#pragma unroll
    for (int k = 2; k < K; ++k) {
        const float tn = 2.f * x * tk - tm1;
        const float dn = 2.f * tk + 2.f * x * dk - dm1;
        f[k] = 0.5f * (tn + 1.f) * fc;
        df[k] = 0.5f * dn * dx * fc + 0.5f * (tn + 1.f) * dfc;
        tm1 = tk;
        tk = tn;
        dm1 = dk;
        dk = dn;
    }
}

// l = 2 four-body invariant.  With the real l = 2 sums a[0..4] (channels
// m = -2..2 of sh_foreach), form the symmetric traceless tensor
// T = sum_m a_m E_m, where u^T E_m u = P_2m(u).  The only cubic rotation
// invariant of T is tr(T^3); it is scaled so that one neighbour along z gives
// (2 2 2; 0 0 0) (5/(4 pi))^(3/2) g^3, i.e. the Wigner-3j triple product of the
// complex-basis sums.  Returns q4 and writes dq4/da_m to d[0..4].
__host__ __device__ __forceinline__ float four_body_l2(const float* a, float* d) {
    const float ca = 1.0925484305920792f;   // sqrt(15/pi)/2
    const float cb = 0.31539156525252005f;  // sqrt(5/pi)/4
    const float cc = 0.54627421529603959f;  // sqrt(15/pi)/4
    // kappa = -(32/3) sqrt(2/35) (pi/5)^(3/2)
    const float kappa = -1.2699291782903164f;
    const float txx = -cb * a[2] + cc * a[4];
    const float tyy = -cb * a[2] - cc * a[4];
    const float tzz = 2.f * cb * a[2];
    const float txy = 0.5f * ca * a[0];
    const float tyz = 0.5f * ca * a[1];
    const float txz = 0.5f * ca * a[3];
    // S = T^2 (symmetric)
    const float sxx = txx * txx + txy * txy + txz * txz;
    const float syy = txy * txy + tyy * tyy + tyz * tyz;
    const float szz = txz * txz + tyz * tyz + tzz * tzz;
    const float sxy = txx * txy + txy * tyy + txz * tyz;
    const float syz = txy * txz + tyy * tyz + tyz * tzz;
    const float sxz = txx * txz + txy * tyz + txz * tzz;
    // tr(T^3) = sum_ab T_ab S_ab
    const float tr3 = txx * sxx + tyy * syy + tzz * szz + 2.f * (txy * sxy + tyz * syz + txz * sxz);
    // d tr(T^3)/d a_m = 3 tr(S E_m)
    const float k3 = 3.f * kappa;
    d[0] = k3 * ca * sxy;
    d[1] = k3 * ca * syz;
    d[2] = k3 * cb * (2.f * szz - sxx - syy);
    d[3] = k3 * ca * sxz;
    d[4] = k3 * cc * (sxx - syy);
    return kappa * tr3;
}

}  // namespace tnep
