// Angular arithmetic of the TNEP descriptor (NEP form, Sec. 2.1) used by the
// gfx950 kernels: the real spherical harmonics and the l = 2 four-body
// invariant.  Plain inline functions on float, callable from device code and
// from the host-side self-check.
#pragma once

#include <hip/hip_runtime.h>

namespace tnep {

// Real orthonormal spherical harmonics, l = 1..4, written as
// Y_lm(u) = kShNorm[idx] * P_lm(u) with P_lm a homogeneous polynomial of
// degree l with integer coefficients in the components of the unit vector u;
// the gradient of Y_lm(r/|r|) with respect to r is
// kShNorm[idx] (grad_u P_lm - l P_lm u) / |r|.  Channel index idx = l*l - 1 +
// (l + m): l = 1 -> 0..2, l = 2 -> 3..7, l = 3 -> 8..14, l = 4 -> 15..23.
// The per-pair loops use P_lm and fold the constants into the per-atom sums
// A_nlm and dU/dA_nlm once per atom.
constexpr int kLM = 24;

constexpr float kShNorm[kLM] = {
    0.48860251190291992f, 0.48860251190291992f, 0.48860251190291992f,                         // l = 1: sqrt(3/4pi)
    1.0925484305920792f,  1.0925484305920792f,  0.31539156525252005f, 1.0925484305920792f,   // l = 2
    0.54627421529603959f,
    0.59004358992664352f, 2.8906114426405538f,  0.45704579946446572f, 0.37317633259011540f,  // l = 3
    0.45704579946446572f, 1.4453057213202769f,  0.59004358992664352f,
    2.5033429417967046f,  1.7701307697799304f,  0.94617469575756008f, 0.66904654355728917f,  // l = 4
    0.10578554691520431f, 0.66904654355728917f, 0.47308734787878004f, 1.7701307697799304f,
    0.62583573544917614f};

// f(idx, l, P, dP/dx, dP/dy, dP/dz) for every channel (all inlined).
template <typename F>
__host__ __device__ __forceinline__ void sh_foreach_raw(float x, float y, float z, F&& f) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    f(0, 1, y, 0.f, 1.f, 0.f);
    f(1, 1, z, 0.f, 0.f, 1.f);
    f(2, 1, x, 1.f, 0.f, 0.f);
    f(3, 2, xy, y, x, 0.f);
    f(4, 2, yz, 0.f, z, y);
    f(5, 2, 2.f * z2 - x2 - y2, -2.f * x, -2.f * y, 4.f * z);
    f(6, 2, xz, z, 0.f, x);
    f(7, 2, x2 - y2, 2.f * x, -2.f * y, 0.f);
    f(8, 3, 3.f * x2 * y - y2 * y, 6.f * xy, 3.f * (x2 - y2), 0.f);
    f(9, 3, xy * z, yz, xz, xy);
    f(10, 3, y * (4.f * z2 - x2 - y2), -2.f * xy, 4.f * z2 - x2 - 3.f * y2, 8.f * yz);
    f(11, 3, z * (2.f * z2 - 3.f * x2 - 3.f * y2), -6.f * xz, -6.f * yz, 3.f * (2.f * z2 - x2 - y2));
    f(12, 3, x * (4.f * z2 - x2 - y2), 4.f * z2 - 3.f * x2 - y2, -2.f * xy, 8.f * xz);
    f(13, 3, z * (x2 - y2), 2.f * xz, -2.f * yz, x2 - y2);
    f(14, 3, x2 * x - 3.f * x * y2, 3.f * (x2 - y2), -6.f * xy, 0.f);
    const float xyz = xy * z;
    f(15, 4, xy * (x2 - y2), y * (3.f * x2 - y2), x * (x2 - 3.f * y2), 0.f);
    f(16, 4, yz * (3.f * x2 - y2), 6.f * xyz, 3.f * z * (x2 - y2), y * (3.f * x2 - y2));
    f(17, 4, xy * (6.f * z2 - x2 - y2), y * (6.f * z2 - 3.f * x2 - y2), x * (6.f * z2 - x2 - 3.f * y2), 12.f * xyz);
    f(18, 4, yz * (4.f * z2 - 3.f * x2 - 3.f * y2), -6.f * xyz, z * (4.f * z2 - 3.f * x2 - 9.f * y2),
      3.f * y * (4.f * z2 - x2 - y2));
    f(19, 4, 8.f * z2 * z2 - 24.f * (x2 + y2) * z2 + 3.f * (x2 + y2) * (x2 + y2), 12.f * x * (x2 + y2 - 4.f * z2),
      12.f * y * (x2 + y2 - 4.f * z2), 16.f * z * (2.f * z2 - 3.f * (x2 + y2)));
    f(20, 4, xz * (4.f * z2 - 3.f * x2 - 3.f * y2), z * (4.f * z2 - 9.f * x2 - 3.f * y2), -6.f * xyz,
      3.f * x * (4.f * z2 - x2 - y2));
    f(21, 4, 6.f * (x2 - y2) * z2 - x2 * x2 + y2 * y2, 4.f * x * (3.f * z2 - x2), 4.f * y * (y2 - 3.f * z2),
      12.f * z * (x2 - y2));
    f(22, 4, xz * (x2 - 3.f * y2), 3.f * z * (x2 - y2), -6.f * xyz, x * (x2 - 3.f * y2));
    f(23, 4, x2 * x2 - 6.f * x2 * y2 + y2 * y2, 4.f * x * (x2 - 3.f * y2), 4.f * y * (y2 - 3.f * x2), 0.f);
}

// l = 2 four-body invariant.  With the real l = 2 sums a[0..4] (channels
// m = -2..2, Y_2m = kShNorm[3 + m + 2] P_2m), form the symmetric traceless tensor
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
