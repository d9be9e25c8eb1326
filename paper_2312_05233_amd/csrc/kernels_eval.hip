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

constexpr int round4(int x) { return (x + 3) & ~3; }

__device__ __forceinline__ void cutoff_fc(float r, float rc_inv, float& fc) {
    fc = 0.5f * (1.f + cospif(r * rc_inv));
}

__device__ __forceinline__ void cutoff_fc_d(float r, float rc_inv, float& fc, float& dfc) {
    float s, c;
    sincospif(r * rc_inv, &s, &c);
    fc = 0.5f * (1.f + c);
    dfc = -0.5f * 3.14159265358979323846f * rc_inv * s;
}

template <int NR, int NA, int KR, int KA, bool FOURB, int KIND>
__global__ void __launch_bounds__(256) k_eval(DevModel m, NeighborLists nl, const int32_t* __restrict__ species,
                                              double* __restrict__ per_atom) {
    constexpr int D = NR + 4 * NA + (FOURB ? NA : 0);
    constexpr int SR = round4(NR * KR);  // LDS stride of one (t_i, t_j) radial block
    constexpr int SA = round4(NA * KA);
    constexpr int NT = KIND == 1 ? 3 : 9;
    extern __shared__ float lds[];
    const int T = m.n_species;
    {
        const int nblk = T * T;
        for (int k = threadIdx.x; k < nblk * SR; k += blockDim.x) {
            const int b = k / SR, o = k % SR;
            lds[k] = o < NR * KR ? m.c_radial[b * NR * KR + o] : 0.f;
        }
        for (int k = threadIdx.x; k < nblk * SA; k += blockDim.x) {
            const int b = k / SA, o = k % SA;
            lds[nblk * SR + k] = o < NA * KA ? m.c_angular[b * NA * KA + o] : 0.f;
        }
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nl.n_atoms) return;
    const int64_t N = nl.n_atoms;
    const int ti = min(max(species[i], 0), T - 1);
    const float* cR = lds + ti * T * SR;
    const float* cA = lds + T * T * SR + ti * T * SA;
    const int n_ang = nl.n_ang[i], n_rad = nl.n_rad[i];
    const float rcR_inv = 1.f / m.rc_radial, rcA_inv = 1.f / m.rc_angular;

    // ---- 1. descriptor sums ---------------------------------------------
    float qR[NR];
    float A[NA][kLM];
#pragma unroll
    for (int n = 0; n < NR; ++n) qR[n] = 0.f;
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int c = 0; c < kLM; ++c) A[n][c] = 0.f;

    for (int s = 0; s < n_ang; ++s) {
        const float4 e = nl.entries[(int64_t)s * N + i];
        const int tj = min(max(__float_as_int(e.w), 0), T - 1);
        const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
        const float rinv = rsqrtf(r2);
        const float r = r2 * rinv;
        float fc;
        float f[KR > KA ? KR : KA];
        cutoff_fc(r, rcR_inv, fc);
        cheb_basis<KR>(r, rcR_inv, fc, f);
        const float* c = cR + tj * SR;
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            float g = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) g += c[n * KR + k] * f[k];
            qR[n] += g;
        }
        cutoff_fc(r, rcA_inv, fc);
        cheb_basis<KA>(r, rcA_inv, fc, f);
        const float* ca = cA + tj * SA;
        float gA[NA];
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float g = 0.f;
#pragma unroll
            for (int k = 0; k < KA; ++k) g += ca[n * KA + k] * f[k];
            gA[n] = g;
        }
        sh_foreach(e.x * rinv, e.y * rinv, e.z * rinv, [&](int idx, int, float P, float, float, float) {
#pragma unroll
            for (int n = 0; n < NA; ++n) A[n][idx] += gA[n] * P;
        });
    }
    for (int s = 0; s < n_rad; ++s) {
        const float4 e = nl.entries[(int64_t)(nl.cap_ang + s) * N + i];
        const int tj = min(max(__float_as_int(e.w), 0), T - 1);
        const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
        const float r = sqrtf(r2);
        float fc, f[KR];
        cutoff_fc(r, rcR_inv, fc);
        cheb_basis<KR>(r, rcR_inv, fc, f);
        const float* c = cR + tj * SR;
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            float g = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) g += c[n * KR + k] * f[k];
            qR[n] += g;
        }
    }

    // ---- 2. invariants, network forward and backward ---------------------
    float q[D];
#pragma unroll
    for (int n = 0; n < NR; ++n) q[n] = qR[n];
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
        q[NR + 0 * NA + n] = s1;
        q[NR + 1 * NA + n] = s2;
        q[NR + 2 * NA + n] = s3;
        q[NR + 3 * NA + n] = s4;
    }
    float d4[FOURB ? NA : 1][5];
    if constexpr (FOURB) {
#pragma unroll
        for (int n = 0; n < NA; ++n) q[NR + 4 * NA + n] = four_body_l2(&A[n][3], d4[n]);
    }
    float qs[D];
#pragma unroll
    for (int v = 0; v < D; ++v) qs[v] = q[v] * m.scaler[v];

    const int H = m.n_hidden;
    float dq[D];
#pragma unroll
    for (int v = 0; v < D; ++v) dq[v] = 0.f;
    float Ut = -m.b1[0];
    {
        const float* __restrict__ w0 = m.w0[0];
        const float* __restrict__ b0 = m.b0[0];
        const float* __restrict__ w1 = m.w1[0];
        for (int mu = 0; mu < H; ++mu) {
            float x = -b0[mu];
#pragma unroll
            for (int v = 0; v < D; ++v) x += w0[mu * D + v] * qs[v];
            const float h = tanhf(x);
            Ut += w1[mu] * h;
            const float t = w1[mu] * (1.f - h * h);
#pragma unroll
            for (int v = 0; v < D; ++v) dq[v] += t * w0[mu * D + v];
        }
    }
#pragma unroll
    for (int v = 0; v < D; ++v) dq[v] *= m.scaler[v];
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
    (void)Ut;

    // G_nlm = dU/dA_nlm, stored over A.
#pragma unroll
    for (int n = 0; n < NA; ++n) {
#pragma unroll
        for (int c = 0; c < kLM; ++c) {
            const int l = c < 3 ? 1 : (c < 8 ? 2 : (c < 15 ? 3 : 4));
            float g = 2.f * dq[NR + (l - 1) * NA + n] * A[n][c];
            if constexpr (FOURB) {
                if (l == 2) g += dq[NR + 4 * NA + n] * d4[n][c - 3];
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

    for (int s = 0; s < n_ang; ++s) {
        const float4 e = nl.entries[(int64_t)s * N + i];
        const int tj = min(max(__float_as_int(e.w), 0), T - 1);
        const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
        const float rinv = rsqrtf(r2);
        const float r = r2 * rinv;
        const float ux = e.x * rinv, uy = e.y * rinv, uz = e.z * rinv;
        float fc, dfc;
        float f[KR > KA ? KR : KA], df[KR > KA ? KR : KA];
        // radial term: d/dr of sum_n dU/dq^R_n g^R_n(r)
        cutoff_fc_d(r, rcR_inv, fc, dfc);
        cheb_basis_d<KR>(r, rcR_inv, fc, dfc, f, df);
        const float* c = cR + tj * SR;
        float sr = 0.f;
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            float dg = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) dg += c[n * KR + k] * df[k];
            sr += dq[n] * dg;
        }
        // angular term
        cutoff_fc_d(r, rcA_inv, fc, dfc);
        cheb_basis_d<KA>(r, rcA_inv, fc, dfc, f, df);
        const float* ca = cA + tj * SA;
        float gA[NA], dgA[NA];
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float g = 0.f, dg = 0.f;
#pragma unroll
            for (int k = 0; k < KA; ++k) {
                g += ca[n * KA + k] * f[k];
                dg += ca[n * KA + k] * df[k];
            }
            gA[n] = g;
            dgA[n] = dg;
        }
        float Fx = 0.f, Fy = 0.f, Fz = 0.f, sc = 0.f;
        sh_foreach(ux, uy, uz, [&](int idx, int l, float P, float px, float py, float pz) {
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                a += A[n][idx] * gA[n];
                b += A[n][idx] * dgA[n];
            }
            Fx += a * px;
            Fy += a * py;
            Fz += a * pz;
            sc += (b - (float)l * a * rinv) * P;
        });
        const float su = sc + sr;
        contract(e.x, e.y, e.z, r2, Fx * rinv + ux * su, Fy * rinv + uy * su, Fz * rinv + uz * su);
    }
    for (int s = 0; s < n_rad; ++s) {
        const float4 e = nl.entries[(int64_t)(nl.cap_ang + s) * N + i];
        const int tj = min(max(__float_as_int(e.w), 0), T - 1);
        const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
        const float rinv = rsqrtf(r2);
        const float r = r2 * rinv;
        float fc, dfc, f[KR], df[KR];
        cutoff_fc_d(r, rcR_inv, fc, dfc);
        cheb_basis_d<KR>(r, rcR_inv, fc, dfc, f, df);
        const float* c = cR + tj * SR;
        float sr = 0.f;
#pragma unroll
        for (int n = 0; n < NR; ++n) {
            float dg = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) dg += c[n * KR + k] * df[k];
            sr += dq[n] * dg;
        }
        const float su = sr * rinv;
        contract(e.x, e.y, e.z, r2, e.x * su, e.y * su, e.z * su);
    }

    double* out = per_atom + i * NT;
    if constexpr (KIND == 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = (double)acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = (double)acc[k] + ((k % 4 == 0) ? (double)Us : 0.0);
    }
}

// One wavefront per frame: every lane sums a fixed stride of atoms in FP64,
// then a butterfly over the 64 lanes; the order depends only on the frame.
__global__ void __launch_bounds__(64) k_frame_reduce(const FrameInfo* __restrict__ frames,
                                                     const double* __restrict__ per_atom, int nt,
                                                     double* __restrict__ out) {
    const int f = blockIdx.x;
    const FrameInfo fi = frames[f];
    const int lane = threadIdx.x;
    double s[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = 0.0;
    for (int64_t a = lane; a < fi.n_atoms; a += 64) {
        const double* p = per_atom + (fi.atom_begin + a) * nt;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (k < nt) s[k] += p[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (k >= nt) break;
        double v = s[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) out[(int64_t)f * nt + k] = v;
    }
}

template <int NR, int NA, int KR, int KA, bool FOURB, int KIND>
hipError_t launch_t(const DevModel& m, const NeighborLists& nl, const int32_t* species, double* per_atom,
                    const EvalLaunch& cfg, hipStream_t s) {
    const int T = m.n_species;
    const size_t lds = sizeof(float) * (size_t)T * T * (round4(NR * KR) + round4(NA * KA));
    const int bs = cfg.atoms_per_block;
    const unsigned grid = (unsigned)((nl.n_atoms + bs - 1) / bs);
    k_eval<NR, NA, KR, KA, FOURB, KIND><<<grid, bs, lds, s>>>(m, nl, species, per_atom);
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

hipError_t launch_eval(const Shape& shape, const DevModel& m, const NeighborLists& nl, const int32_t* species,
                       double* per_atom, const EvalLaunch& cfg, hipStream_t s) {
    if (nl.n_atoms == 0) return hipSuccess;
#define X(NR_, NA_, KR_, KA_, FB_)                                                                         \
    if (shape.nr == NR_ && shape.na == NA_ && shape.kr == KR_ && shape.ka == KA_ &&                         \
        (bool)shape.four_body == FB_) {                                                                    \
        if (shape.kind == 1) return launch_t<NR_, NA_, KR_, KA_, FB_, 1>(m, nl, species, per_atom, cfg, s); \
        return launch_t<NR_, NA_, KR_, KA_, FB_, 2>(m, nl, species, per_atom, cfg, s);                      \
    }
    TNEP_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_frame_reduce(const FrameInfo* d_frames, int n_frames, const double* per_atom, int nt, double* out,
                               hipStream_t s) {
    if (n_frames == 0) return hipSuccess;
    k_frame_reduce<<<n_frames, 64, 0, s>>>(d_frames, per_atom, nt, out);
    return hipGetLastError();
}

}  // namespace tnep
