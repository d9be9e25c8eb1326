// Fused TNEP evaluation on gfx950: one lane per atom.
//
// For atom i (Sec. 2.1, Eq. site-energy) the kernel
//   1. walks the neighbour list once, accumulating the radial descriptor
//      q^R_n = sum_j g^R_n(r_ij) and the angular sums
//      A_nlm = sum_j g^A_n(r_ij) Y_lm(r_ij / r_ij) in registers (5 x 24 floats);
//   2. forms the invariants q_nl = sum_m A_nlm^2 (l = 1..4) and the l = 2
//      four-body term, scales them and runs the tanh network forward and
//      backward to dU_i/dq (one or two heads);
//   3. walks the list again and forms the partial forces dU_i/dr_ij
//      (Sec. 2.1, text after Eq. virial), contracting them at once into the
//      atom's dipole term -r_ij^2 dU_i/dr_ij (Sec. 2.2, Eq. mu) or virial term
//      -r_ij (x) dU_i/dr_ij plus U^s_i delta (Sec. 2.3, Eq. polarizability-model).
// Per-pair work is FP32; the atom terms are written as FP64 and summed per
// frame by k_frame_reduce in a fixed order.
#include "internal.h"
#include "tnep_math.h"

namespace tnep {

namespace {

// Cosine cutoff f_c(r) = (1 + cos(pi r / r_c)) / 2 = sin^2(w), w = (pi/2)(1 - r/r_c),
// which keeps relative accuracy as r -> r_c; f_c'(r) = -(pi / r_c) sin(w) cos(w).
// sin and cos of w in [0, pi/2] from their Taylor series to w^13 / w^14
// (truncation below 1e-9).  v = 1 - r / r_c.
__device__ __forceinline__ float sin_half_pi(float w) {
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
__device__ __forceinline__ float cos_half_pi(float w) {
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
__device__ __forceinline__ float cutoff_fc(float v) {
    const float s = sin_half_pi(1.57079632679489662f * v);
    return s * s;
}
__device__ __forceinline__ void cutoff_fc_d(float v, float rc_inv, float& fc, float& dfc) {
    const float w = 1.57079632679489662f * v;
    const float s = sin_half_pi(w), c = cos_half_pi(w);
    fc = s * s;
    dfc = -3.14159265358979323846f * rc_inv * s * c;
}

// Tile species: wave-uniform (tiles are species-pure).
__device__ __forceinline__ int tile_species(const int32_t* tile_base, int T, int tile) {
    int ti = 0;
    for (int t = 1; t < T; ++t)
        if (tile >= tile_base[t]) ti = t;
    return __builtin_amdgcn_readfirstlane(ti);
}

// One lane per tile slot (atom); 4 wavefronts per work-group, no LDS.  The
// coefficient blocks c[t_i][t] are wave-uniform and read with scalar loads.
template <int NR, int NA, int KR, int KA, bool FOURB, int KIND>
__global__ void __launch_bounds__(256, 2) k_eval(DevModel m, NeighborLists nl, double* __restrict__ per_atom) {
    constexpr int D = NR + 4 * NA + (FOURB ? NA : 0);
    constexpr int NT = KIND == 1 ? 3 : 9;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int T = nl.T;
    const int tile = __builtin_amdgcn_readfirstlane((int)(p >> 6));
    const int lane = (int)(p & 63);
    if (tile >= nl.meta[kMetaTileBase + T]) return;
    const int a = nl.perm[p];
    if (a < 0) return;
    const int ti = tile_species(nl.meta + kMetaTileBase, T, tile);
    const float rcR_inv = 1.f / m.rc_radial, rcA_inv = 1.f / m.rc_angular;
    const float4* lane_base = nl.entries + ((int64_t)tile * (nl.slots >> 2) * 64 + lane) * 4;

    // ---- 1. descriptor sums ---------------------------------------------
    float qR[NR];
    float A[NA][kLM];
#pragma unroll
    for (int n = 0; n < NR; ++n) qR[n] = 0.f;
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int c = 0; c < kLM; ++c) A[n][c] = 0.f;

    for (int t = 0; t < T; ++t) {
        const float* __restrict__ cR = m.c_radial + (ti * T + t) * (NR * KR);
        const float* __restrict__ cA = m.c_angular + (ti * T + t) * (NA * KA);
        const int n_ang = nl.counts[(int64_t)(2 * t) * nl.n_pad + p];
        const int n_rad = nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p];
        const float4* ga = lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256;
        const float4* gr = lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256;
        float F[KR];  // sum over neighbours of species t of f_k(r_ij)
#pragma unroll
        for (int k = 0; k < KR; ++k) F[k] = 0.f;
        float4 nxt = n_ang > 0 ? ga[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = 0; s < n_ang; ++s) {
            const float4 e = nxt;
            if (s + 1 < n_ang) nxt = ga[((s + 1) >> 2) * 256 + ((s + 1) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = rsqrtf(r2);
            const float r = r2 * rinv;
            float f[KR > KA ? KR : KA];
            float v = 1.f - r * rcR_inv;
            cheb_basis<KR>(r, rcR_inv, cutoff_fc(v), f);
#pragma unroll
            for (int k = 0; k < KR; ++k) F[k] += f[k];
            v = 1.f - r * rcA_inv;
            cheb_basis<KA>(r, rcA_inv, cutoff_fc(v), f);
            float gA[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float g = 0.f;
#pragma unroll
                for (int k = 0; k < KA; ++k) g += cA[n * KA + k] * f[k];
                gA[n] = g;
            }
            sh_foreach(e.x * rinv, e.y * rinv, e.z * rinv, [&](int idx, int, float P, float, float, float) {
#pragma unroll
                for (int n = 0; n < NA; ++n) A[n][idx] += gA[n] * P;
            });
        }
        nxt = n_rad > 0 ? gr[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = 0; s < n_rad; ++s) {
            const float4 e = nxt;
            if (s + 1 < n_rad) nxt = gr[((s + 1) >> 2) * 256 + ((s + 1) & 3)];
            const float r = sqrtf(e.x * e.x + e.y * e.y + e.z * e.z);
            float f[KR];
            cheb_basis<KR>(r, rcR_inv, cutoff_fc(1.f - r * rcR_inv), f);
#pragma unroll
            for (int k = 0; k < KR; ++k) F[k] += f[k];
        }
#pragma unroll
        for (int n = 0; n < NR; ++n)
#pragma unroll
            for (int k = 0; k < KR; ++k) qR[n] += cR[n * KR + k] * F[k];
    }

    // ---- 2. invariants, network forward and backward ---------------------
    float qs[D];
#pragma unroll
    for (int n = 0; n < NR; ++n) qs[n] = qR[n];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) s1 += A[n][c] * A[n][c];
#pragma unroll
        for (int c = 3; c < 8; ++c) s2 += A[n][c] * A[n][c];
#pragma unroll
        for (int c = 8; c < 15; ++c) s3 += A[n][c] * A[n][c];
#pragma unroll
        for (int c = 15; c < 24; ++c) s4 += A[n][c] * A[n][c];
        qs[NR + 0 * NA + n] = s1;
        qs[NR + 1 * NA + n] = s2;
        qs[NR + 2 * NA + n] = s3;
        qs[NR + 3 * NA + n] = s4;
    }
    if constexpr (FOURB) {
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float d4[5];
            qs[NR + 4 * NA + n] = four_body_l2(&A[n][3], d4);
        }
    }
#pragma unroll
    for (int v = 0; v < D; ++v) qs[v] *= m.scaler[v];

    const int H = m.n_hidden;
    float Us = 0.f;
    if constexpr (KIND == 2) {
        const float* __restrict__ w0 = m.w0[1];
        const float* __restrict__ b0 = m.b0[1];
        const float* __restrict__ w1 = m.w1[1];
        Us = -m.b1[1];
        for (int mu = 0; mu < H; ++mu) {
            float x = -b0[mu];
#pragma unroll
            for (int v = 0; v < D; ++v) x += w0[mu * D + v] * qs[v];
            Us += w1[mu] * tanhf(x);
        }
    }
    float dq[D];
#pragma unroll
    for (int v = 0; v < D; ++v) dq[v] = 0.f;
    {
        const float* __restrict__ w0 = m.w0[0];
        const float* __restrict__ b0 = m.b0[0];
        const float* __restrict__ w1 = m.w1[0];
        for (int mu = 0; mu < H; ++mu) {
            float x = -b0[mu];
#pragma unroll
            for (int v = 0; v < D; ++v) x += w0[mu * D + v] * qs[v];
            const float h = tanhf(x);
            const float t = w1[mu] * (1.f - h * h);
#pragma unroll
            for (int v = 0; v < D; ++v) dq[v] += t * w0[mu * D + v];
        }
    }
#pragma unroll
    for (int v = 0; v < D; ++v) dq[v] *= m.scaler[v];

    // G_nlm = dU/dA_nlm, stored over A.
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float d4[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (FOURB) four_body_l2(&A[n][3], d4);
#pragma unroll
        for (int c = 0; c < kLM; ++c) {
            const int l = c < 3 ? 1 : (c < 8 ? 2 : (c < 15 ? 3 : 4));
            float g = 2.f * dq[NR + (l - 1) * NA + n] * A[n][c];
            if constexpr (FOURB) {
                if (l == 2) g += dq[NR + 4 * NA + n] * d4[c - 3];
            }
            A[n][c] = g;
        }
    }

    // ---- 3. partial forces and contraction --------------------------------
    float acc[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = 0.f;
    auto contract = [&](float dx, float dy, float dz, float r2, float Fx, float Fy, float Fz) {
        if constexpr (KIND == 1) {
            acc[0] -= r2 * Fx;
            acc[1] -= r2 * Fy;
            acc[2] -= r2 * Fz;
        } else {
            acc[0] -= dx * Fx;
            acc[1] -= dx * Fy;
            acc[2] -= dx * Fz;
            acc[3] -= dy * Fx;
            acc[4] -= dy * Fy;
            acc[5] -= dy * Fz;
            acc[6] -= dz * Fx;
            acc[7] -= dz * Fy;
            acc[8] -= dz * Fz;
        }
    };

    for (int t = 0; t < T; ++t) {
        const float* __restrict__ cR = m.c_radial + (ti * T + t) * (NR * KR);
        const float* __restrict__ cA = m.c_angular + (ti * T + t) * (NA * KA);
        const int n_ang = nl.counts[(int64_t)(2 * t) * nl.n_pad + p];
        const int n_rad = nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p];
        const float4* ga = lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256;
        const float4* gr = lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256;
        // d/dr of sum_n dU/dq^R_n g^R_n(r) = sum_k Dk[k] f_k'(r)
        float Dk[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            float d = 0.f;
#pragma unroll
            for (int n = 0; n < NR; ++n) d += dq[n] * cR[n * KR + k];
            Dk[k] = d;
        }
        auto radial_slope = [&](float r) {
            float fc, dfc, f[KR], df[KR];
            cutoff_fc_d(1.f - r * rcR_inv, rcR_inv, fc, dfc);
            cheb_basis_d<KR>(r, rcR_inv, fc, dfc, f, df);
            float sr = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) sr += Dk[k] * df[k];
            return sr;
        };
        float4 nxt = n_ang > 0 ? ga[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = 0; s < n_ang; ++s) {
            const float4 e = nxt;
            if (s + 1 < n_ang) nxt = ga[((s + 1) >> 2) * 256 + ((s + 1) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = rsqrtf(r2);
            const float r = r2 * rinv;
            const float ux = e.x * rinv, uy = e.y * rinv, uz = e.z * rinv;
            const float sr = radial_slope(r);
            float fc, dfc, f[KA], df[KA];
            cutoff_fc_d(1.f - r * rcA_inv, rcA_inv, fc, dfc);
            cheb_basis_d<KA>(r, rcA_inv, fc, dfc, f, df);
            float gA[NA], dgA[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float g = 0.f, dg = 0.f;
#pragma unroll
                for (int k = 0; k < KA; ++k) {
                    g += cA[n * KA + k] * f[k];
                    dg += cA[n * KA + k] * df[k];
                }
                gA[n] = g;
                dgA[n] = dg;
            }
            float Fx = 0.f, Fy = 0.f, Fz = 0.f, sc = 0.f;
            sh_foreach(ux, uy, uz, [&](int idx, int l, float P, float px, float py, float pz) {
                float av = 0.f, bv = 0.f;
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    av += A[n][idx] * gA[n];
                    bv += A[n][idx] * dgA[n];
                }
                Fx += av * px;
                Fy += av * py;
                Fz += av * pz;
                sc += (bv - (float)l * av * rinv) * P;
            });
            const float su = sc + sr;
            contract(e.x, e.y, e.z, r2, Fx * rinv + ux * su, Fy * rinv + uy * su, Fz * rinv + uz * su);
        }
        nxt = n_rad > 0 ? gr[0] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = 0; s < n_rad; ++s) {
            const float4 e = nxt;
            if (s + 1 < n_rad) nxt = gr[((s + 1) >> 2) * 256 + ((s + 1) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = rsqrtf(r2);
            const float su = radial_slope(r2 * rinv) * rinv;
            contract(e.x, e.y, e.z, r2, e.x * su, e.y * su, e.z * su);
        }
    }

    double* out = per_atom + (int64_t)a * NT;
    if constexpr (KIND == 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = (double)acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = (double)acc[k] + ((k % 4 == 0) ? (double)Us : 0.0);
    }
}

// One work-group of 256 lanes per frame: lane l sums atoms l, l + 256, ... in
// FP64, then a fixed pairwise tree in LDS; the order depends only on the
// frame's atom count, never on how frames were batched.
__global__ void __launch_bounds__(256) k_frame_reduce(const FrameInfo* __restrict__ frames,
                                                      const double* __restrict__ per_atom, int nt,
                                                      double* __restrict__ out) {
    __shared__ double part[9][256];
    const int f = blockIdx.x;
    const FrameInfo fi = frames[f];
    const int lane = threadIdx.x;
    double s[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = 0.0;
    for (int64_t a = lane; a < fi.n_atoms; a += 256) {
        const double* q = per_atom + (fi.atom_begin + a) * nt;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (k < nt) s[k] += q[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) part[k][lane] = s[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (lane < off)
#pragma unroll
            for (int k = 0; k < 9; ++k) part[k][lane] += part[k][lane + off];
        __syncthreads();
    }
    if (lane < nt) out[(int64_t)f * nt + lane] = part[lane][0];
}

template <int NR, int NA, int KR, int KA, bool FOURB, int KIND>
hipError_t launch_t(const DevModel& m, const NeighborLists& nl, double* per_atom, hipStream_t s) {
    const unsigned grid = (unsigned)((nl.n_pad + 255) / 256);
    k_eval<NR, NA, KR, KA, FOURB, KIND><<<grid, 256, 0, s>>>(m, nl, per_atom);
    return hipGetLastError();
}

}  // namespace

#define TNEP_SHAPES(X)   \
    X(5, 5, 9, 9, true)  \
    X(5, 5, 9, 9, false) \
    X(7, 5, 9, 9, false) \
    X(7, 5, 9, 9, true)

bool eval_shape_supported(const Shape& s) {
#define X(NR_, NA_, KR_, KA_, FB_) \
    if (s.nr == NR_ && s.na == NA_ && s.kr == KR_ && s.ka == KA_ && (bool)s.four_body == FB_) return true;
    TNEP_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_eval(const Shape& shape, const DevModel& m, const NeighborLists& nl, double* per_atom,
                       const EvalLaunch& cfg, hipStream_t s) {
    (void)cfg;
    if (nl.n_pad == 0) return hipSuccess;
#define X(NR_, NA_, KR_, KA_, FB_)                                                                         \
    if (shape.nr == NR_ && shape.na == NA_ && shape.kr == KR_ && shape.ka == KA_ &&                         \
        (bool)shape.four_body == FB_) {                                                                    \
        if (shape.kind == 1) return launch_t<NR_, NA_, KR_, KA_, FB_, 1>(m, nl, per_atom, s);               \
        return launch_t<NR_, NA_, KR_, KA_, FB_, 2>(m, nl, per_atom, s);                                    \
    }
    TNEP_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_frame_reduce(const FrameInfo* d_frames, int n_frames, const double* per_atom, int nt, double* out,
                               hipStream_t s) {
    if (n_frames == 0) return hipSuccess;
    k_frame_reduce<<<n_frames, 256, 0, s>>>(d_frames, per_atom, nt, out);
    return hipGetLastError();
}

}  // namespace tnep
