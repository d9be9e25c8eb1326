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
//
// Two layouts of the same kernel: one lane per atom (G = 1, the throughput
// layout), or G = 16 lanes per atom for launch batches of few atoms (one atom
// per 16-lane DPP row): lane g takes the neighbour rows g, g + G, ... and the
// hidden neurons g, g + G, ..., and group_sum adds the lanes' shares of the
// descriptor sums, of dU/dq and of the atom's tensor term by a fixed tree, so
// an atom's result still depends only on its own list.
#include <type_traits>

#include "../../include/tnep.h"
#include "internal.h"
#include "tnep_math.h"
#include "radial_basis.h"

namespace tnep {

namespace {

// Tile species: wave-uniform (tiles are species-pure).
__device__ __forceinline__ int tile_species(const int32_t* tile_base, int T, int tile) {
    int ti = 0;
    for (int t = 1; t < T; ++t)
        if (tile >= tile_base[t]) ti = t;
    return __builtin_amdgcn_readfirstlane(ti);
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// Sum over the G lanes of an aligned group (G = 1, 8 or 16 within a DPP row),
// the result in every lane of the group: lanes exchanged with lane ^ 1, then
// lane ^ 2 (quad permutations), then lane i with 7 - i (half-row mirror), then
// i with 15 - i (row mirror).  Each step adds two equal-rank partial sums in
// both orders, which IEEE addition makes bitwise equal, so every lane of the
// group ends with the same value.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int G, class V>
__device__ __forceinline__ V group_sum(V v) {
    static_assert(G == 1 || G == 8 || G == 16, "groups of 1, 8 or 16 lanes");
    auto step = [](V x, auto ctrl) {
        constexpr int C = decltype(ctrl)::value;
        if constexpr (sizeof(V) == 8)
            return x + dpp_f64<C>(x);
        else
            return x + dpp_f32<C>(x);
    };
    if constexpr (G >= 8) {
        v = step(v, std::integral_constant<int, 0xB1>{});   // quad_perm(1, 0, 3, 2)
        v = step(v, std::integral_constant<int, 0x4E>{});   // quad_perm(2, 3, 0, 1)
        v = step(v, std::integral_constant<int, 0x141>{});  // row_half_mirror
    }
    if constexpr (G == 16) v = step(v, std::integral_constant<int, 0x140>{});  // row_mirror
    return v;
}

// Order the wavefront's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Hidden layer of the 64 atoms of one wavefront on the matrix cores
// (Sec. 2.1: one shared single-hidden-layer tanh network per head):
//   X = Qs W0^T (64 x H), h = tanh(X - b0),
//   scalar head: U^s = h w1 - b1;   tensor head: dU/dq = ((1 - h^2) * w1) W0 * s.
// Qs, dU/dq and the hidden activations pass through a per-wavefront LDS tile;
// W0 comes as per-lane operand fragments prepared at model creation.
// MODE: TNEP_MLP_FP32_MFMA (v_mfma_f32_16x16x4_f32), TNEP_MLP_BF16_MFMA
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation) or TNEP_MLP_BF16X3_MFMA
// (both operands split into bf16 hi + lo, three products hi*hi + hi*lo + lo*hi).
template <int D, int KIND, int MODE>
__device__ __forceinline__ void mlp_matrix(const DevModel& m, const float (&qs)[D], float (&dq)[D], float& Us,
                                           float* wl, int lane) {
    constexpr int Dp4 = (D + 3) / 4 * 4;
    constexpr int Dp16 = (D + 15) / 16 * 16;
    constexpr int Dp32 = (D + 31) / 32 * 32;
    constexpr int LDQ = Dp32 + 4;
    const int H = m.n_hidden;
    const int Hp = (H + 31) / 32 * 32;
    const int LDT = Hp + 4;
    float* Qs = wl;
    float* Tb = wl + 64 * LDQ;
    const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int k = 0; k < Dp32; ++k) Qs[lane * LDQ + k] = k < D ? qs[k] : 0.f;
    wave_lds_sync();

    auto split8 = [](const float* src, bf8v& hi, bf8v& lo) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float x = src[j];
            const __bf16 h = (__bf16)x;
            hi[j] = h;
            lo[j] = (__bf16)(x - (float)h);
        }
    };
    // acc[mt][i] = X[16 mt + 4 g4 + i][16 nt + r16]
    auto forward = [&](int hd, int nt, f4v (&acc)[4]) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = f4v{0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE == TNEP_MLP_FP32_MFMA) {
            const float* fr = m.f32_fwd[hd] + (size_t)nt * (Dp4 / 4) * 64 + lane;
#pragma unroll
            for (int ks = 0; ks < Dp4 / 4; ++ks) {
                const float b = fr[ks * 64];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const float a = Qs[(16 * mt + r16) * LDQ + 4 * ks + g4];
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[mt], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int kc = 0; kc < Dp32 / 32; ++kc) {
                const size_t fi = ((size_t)nt * (Dp32 / 32) + kc) * 64 + lane;
                const bf8v bh = __builtin_bit_cast(bf8v, m.bf_fwd_hi[hd][fi]);
                const bf8v bl = __builtin_bit_cast(bf8v, m.bf_fwd_lo[hd][fi]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    bf8v ah, al;
                    split8(Qs + (16 * mt + r16) * LDQ + 32 * kc + 8 * g4, ah, al);
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[mt], 0, 0, 0);
                    if constexpr (MODE == TNEP_MLP_BF16X3_MFMA) {
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[mt], 0, 0, 0);
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[mt], 0, 0, 0);
                    }
                }
            }
        }
    };

    if constexpr (KIND == 2) {
        for (int nt = 0; nt < Hp / 16; ++nt) {
            f4v acc[4];
            forward(1, nt, acc);
            const int n = 16 * nt + r16;
            const bool nv = n < H;
            const float b0n = nv ? m.b0[1][n] : 0.f, w1n = nv ? m.w1[1][n] : 0.f;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) Tb[(16 * mt + 4 * g4 + i) * LDT + n] = w1n * tanhf(acc[mt][i] - b0n);
        }
        wave_lds_sync();
        float u = -m.b1[1];
        for (int n = 0; n < H; ++n) u += Tb[lane * LDT + n];
        Us = u;
        wave_lds_sync();
    }
    for (int nt = 0; nt < Hp / 16; ++nt) {
        f4v acc[4];
        forward(0, nt, acc);
        const int n = 16 * nt + r16;
        const bool nv = n < H;
        const float b0n = nv ? m.b0[0][n] : 0.f, w1n = nv ? m.w1[0][n] : 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h = tanhf(acc[mt][i] - b0n);
                Tb[(16 * mt + 4 * g4 + i) * LDT + n] = w1n * (1.f - h * h);
            }
    }
    wave_lds_sync();
    // dU/dq~[atom][k] = sum_n Tb[atom][n] W0[n][k], written over Qs
#pragma unroll
    for (int kt = 0; kt < Dp16 / 16; ++kt) {
        f4v acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = f4v{0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE == TNEP_MLP_FP32_MFMA) {
            const float* fr = m.f32_bwd + (size_t)kt * (Hp / 4) * 64 + lane;
            for (int ns = 0; ns < Hp / 4; ++ns) {
                const float b = fr[ns * 64];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const float a = Tb[(16 * mt + r16) * LDT + 4 * ns + g4];
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[mt], 0, 0, 0);
                }
            }
        } else {
            for (int nc = 0; nc < Hp / 32; ++nc) {
                const size_t fi = ((size_t)kt * (Hp / 32) + nc) * 64 + lane;
                const bf8v bh = __builtin_bit_cast(bf8v, m.bf_bwd_hi[fi]);
                const bf8v bl = __builtin_bit_cast(bf8v, m.bf_bwd_lo[fi]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    bf8v ah, al;
                    split8(Tb + (16 * mt + r16) * LDT + 32 * nc + 8 * g4, ah, al);
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[mt], 0, 0, 0);
                    if constexpr (MODE == TNEP_MLP_BF16X3_MFMA) {
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[mt], 0, 0, 0);
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[mt], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) Qs[(16 * mt + 4 * g4 + i) * LDQ + 16 * kt + r16] = acc[mt][i];
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < D; ++k) dq[k] = Qs[lane * LDQ + k] * m.scaler[k];
}

// LDS floats per wavefront used by mlp_matrix.
__host__ __device__ constexpr int mlp_lds_floats(int D, int H) {
    return 64 * (((D + 31) / 32 * 32 + 4) + ((H + 31) / 32 * 32 + 4));
}

// Row counts of one species' two segments of a slot.
struct SegCounts {
    int n_ang, n_rad;
    __device__ __forceinline__ void fetch(const NeighborLists& nl, int64_t p, int t) {
        n_ang = nl.counts[(int64_t)(2 * t) * nl.n_pad + p];
        n_rad = nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p];
    }
};

// One lane per tile slot (atom).  The coefficient blocks c[t_i][t] are
// wave-uniform and read with scalar loads.  MODE selects the hidden layer:
// FP32 vector ALU (no LDS) or one of the matrix-core variants (LDS tile per
// wavefront).  Padding lanes run with empty neighbour lists and store nothing.
// LOAD: the radial descriptor sums come from rad_v (the neighbour search
// accumulated them); otherwise the kernel forms them.  G: lanes per atom (1, or
// 16 for the pair-parallel layout of the dipole and polarizability models with
// the FP32 vector hidden layer).  pes_rec, pes_pair and
// pes_slot (the potential-energy outputs of PesOut) are restrict parameters, so that
// their stores cannot clobber the model's parameters and these stay
// wave-uniform scalar loads.
template <int NR, int NA, int KR, int KA, int MB, int KIND, int MODE, bool LOAD = false, int G = 1>
__global__ void __launch_bounds__(256, 2) k_eval(DevModel m, NeighborLists nl, double* __restrict__ per_atom,
                                                 PesOut pes, const float* __restrict__ rad_v,
                                                 float* __restrict__ pes_rec, float4* __restrict__ pes_pair,
                                                 int32_t* __restrict__ pes_slot) {
    constexpr bool FOURB = (MB & 1) != 0, FIVEB = (MB & 2) != 0;
    constexpr int D = NR + 4 * NA + (FOURB ? NA : 0) + (FIVEB ? NA : 0);
    constexpr int NT = KIND == 1 ? 3 : 9;  // accumulated tensor: mu, or the virial-like W
    static_assert(G == 1 || (KIND != 3 && MODE == TNEP_MLP_FP32_VALU && !LOAD),
                  "the pair-parallel layout serves the tensor models with the vector hidden layer");
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = G == 1 ? tid : tid / G;  // tile slot
    const int g = G == 1 ? 0 : (int)(tid % G);  // lane within the atom's group
    const int T = nl.T;
    const int tile = __builtin_amdgcn_readfirstlane((int)(p >> 6));
    const int lane = (int)(p & 63);
    if (tile >= nl.meta[kMetaTileBase + T]) return;
    const int a = nl.perm[p];
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

    // a species' row counts are loaded while the species before it runs, so that
    // its pass does not begin with two dependent loads (counts, then entries)
    SegCounts ahead;
    ahead.fetch(nl, p, 0);
    for (int t = 0; t < T; ++t) {
        const float* __restrict__ cR = m.c_radial + (ti * T + t) * (NR * KR);
        const float* __restrict__ cA = m.c_angular + (ti * T + t) * (NA * KA);
        const SegCounts cur = ahead;
        if (t + 1 < T) ahead.fetch(nl, p, t + 1);
        const int n_ang = cur.n_ang, n_rad = cur.n_rad;
        const float4* ga = lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256;
        const float4* gr = lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256;
        // sum over neighbours of species t of f_k(r_ij) = (sum fc T_k + sum fc) / 2
        float FT[KR], Fs = 0.f;
#pragma unroll
        for (int k = 0; k < KR; ++k) FT[k] = 0.f;
        float Cs[NA];  // sum_k c_nk (wave-uniform)
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float c = 0.f;
#pragma unroll
            for (int k = 0; k < KA; ++k) c += cA[n * KA + k];
            Cs[n] = c;
        }
        float4 nxt = n_ang > g ? ga[(g >> 2) * 256 + (g & 3)] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = g; s < n_ang; s += G) {
            const float4 e = nxt;
            if (s + G < n_ang) nxt = ga[((s + G) >> 2) * 256 + ((s + G) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = pair_rsqrt(r2);
            const float r = r2 * rinv;
            float Tk[KR > KA ? KR : KA];
            if constexpr (!LOAD) {
                const float fc = cutoff_fc(1.f - r * rcR_inv);
                const float tt = r * rcR_inv - 1.f;
                cheb_T<KR>(2.f * tt * tt - 1.f, Tk);
                Fs += fc;
#pragma unroll
                for (int k = 0; k < KR; ++k) FT[k] += fc * Tk[k];
            }
            const float hfc = 0.5f * cutoff_fc(1.f - r * rcA_inv);
            const float ta = r * rcA_inv - 1.f;
            cheb_T<KA>(2.f * ta * ta - 1.f, Tk);
            // g_n = sum_k c_nk f_k = fc/2 (sum_k c_nk T_k + sum_k c_nk)
            float gA[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float g = Cs[n];
#pragma unroll
                for (int k = 0; k < KA; ++k) g += cA[n * KA + k] * Tk[k];
                gA[n] = hfc * g;
            }
            sh_foreach_raw(e.x * rinv, e.y * rinv, e.z * rinv, [&](int idx, int, float P, float, float, float) {
#pragma unroll
                for (int n = 0; n < NA; ++n) A[n][idx] += gA[n] * P;
            });
        }
        float F[KR];
        if constexpr (LOAD) {
#pragma unroll
            for (int k = 0; k < KR; ++k) F[k] = rad_v[(int64_t)(t * KR + k) * nl.n_pad + p];
        } else {
            nxt = n_rad > g ? gr[(g >> 2) * 256 + (g & 3)] : make_float4(0.f, 0.f, 0.f, 0.f);
            for (int s = g; s < n_rad; s += G) {
                const float4 e = nxt;
                if (s + G < n_rad) nxt = gr[((s + G) >> 2) * 256 + ((s + G) & 3)];
                const float r = pair_sqrt(e.x * e.x + e.y * e.y + e.z * e.z);
                const float fc = cutoff_fc(1.f - r * rcR_inv);
                const float tt = r * rcR_inv - 1.f;
                float Tk[KR];
                cheb_T<KR>(2.f * tt * tt - 1.f, Tk);
                Fs += fc;
#pragma unroll
                for (int k = 0; k < KR; ++k) FT[k] += fc * Tk[k];
            }
#pragma unroll
            for (int k = 0; k < KR; ++k) F[k] = 0.5f * (FT[k] + Fs);
        }
#pragma unroll
        for (int n = 0; n < NR; ++n)
#pragma unroll
            for (int k = 0; k < KR; ++k) qR[n] += cR[n * KR + k] * F[k];
    }
    if constexpr (G > 1) {  // the lanes' shares of the sums (linear in the pair terms)
#pragma unroll
        for (int n = 0; n < NR; ++n) qR[n] = group_sum<G>(qR[n]);
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int c = 0; c < kLM; ++c) A[n][c] = group_sum<G>(A[n][c]);
    }

    // ---- 2. invariants, network forward and backward ---------------------
    // the pair loops summed the unnormalised harmonics: A_nlm = kShNorm[lm] * sum
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int c = 0; c < kLM; ++c) A[n][c] *= kShNorm[c];
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
    // five-body: the squared l = 1 invariant, q5_n = (sum_m A_n1m^2)^2
    constexpr int kOff5 = NR + 4 * NA + (FOURB ? NA : 0);
    if constexpr (FIVEB) {
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            const float s1 = A[n][0] * A[n][0] + A[n][1] * A[n][1] + A[n][2] * A[n][2];
            qs[kOff5 + n] = s1 * s1;
        }
    }
#pragma unroll
    for (int v = 0; v < D; ++v) qs[v] *= m.scaler[v];

    float Us = 0.f;  // scalar head (polarizability) or site energy (potential)
    float dq[D];
    if constexpr (MODE == TNEP_MLP_FP32_VALU) {
        const int H = m.n_hidden;
        if constexpr (KIND == 2) {
            const float* __restrict__ w0 = m.w0[1] + ti * m.sp_w0;
            const float* __restrict__ b0 = m.b0[1] + ti * m.sp_h;
            const float* __restrict__ w1 = m.w1[1] + ti * m.sp_h;
            const float b1 = m.b1s[1] ? m.b1s[1][ti] : m.b1[1];
            Us = G == 1 ? -b1 : 0.f;
            for (int mu = g; mu < H; mu += G) {
                float x = -b0[mu];
#pragma unroll
                for (int v = 0; v < D; ++v) x += w0[mu * D + v] * qs[v];
                Us += w1[mu] * tanhf(x);
            }
            if constexpr (G > 1) Us = group_sum<G>(Us) - b1;
        }
#pragma unroll
        for (int v = 0; v < D; ++v) dq[v] = 0.f;
        {
            const float* __restrict__ w0 = m.w0[0] + ti * m.sp_w0;
            const float* __restrict__ b0 = m.b0[0] + ti * m.sp_h;
            const float* __restrict__ w1 = m.w1[0] + ti * m.sp_h;
            if constexpr (KIND == 3) Us = -(m.b1s[0] ? m.b1s[0][ti] : m.b1[0]);
            for (int mu = g; mu < H; mu += G) {
                float x = -b0[mu];
#pragma unroll
                for (int v = 0; v < D; ++v) x += w0[mu * D + v] * qs[v];
                const float h = tanhf(x);
                if constexpr (KIND == 3) Us += w1[mu] * h;
                const float t = w1[mu] * (1.f - h * h);
#pragma unroll
                for (int v = 0; v < D; ++v) dq[v] += t * w0[mu * D + v];
            }
        }
        if constexpr (G > 1) {
#pragma unroll
            for (int v = 0; v < D; ++v) dq[v] = group_sum<G>(dq[v]);
        }
#pragma unroll
        for (int v = 0; v < D; ++v) dq[v] *= m.scaler[v];
    } else {
        extern __shared__ float lds[];
        float* wl = lds + (threadIdx.x >> 6) * mlp_lds_floats(D, m.n_hidden);
        mlp_matrix<D, KIND, MODE>(m, qs, dq, Us, wl, (int)(threadIdx.x & 63));
    }

    // G_nlm = dU/dA_nlm, stored over A.
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        float d4[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (FOURB) four_body_l2(&A[n][3], d4);
        // d q5_n / d A_n1m = 4 (sum_m' A_n1m'^2) A_n1m, folded into the l = 1 factor
        float w5 = 0.f;
        if constexpr (FIVEB) w5 = 4.f * dq[kOff5 + n] * (A[n][0] * A[n][0] + A[n][1] * A[n][1] + A[n][2] * A[n][2]);
#pragma unroll
        for (int c = 0; c < kLM; ++c) {
            const int l = c < 3 ? 1 : (c < 8 ? 2 : (c < 15 ? 3 : 4));
            float g = 2.f * dq[NR + (l - 1) * NA + n] * A[n][c];
            if constexpr (FOURB) {
                if (l == 2) g += dq[NR + 4 * NA + n] * d4[c - 3];
            }
            if constexpr (FIVEB) {
                if (l == 1) g += w5 * A[n][c];
            }
            A[n][c] = g;
        }
    }

    // potential: the record that the force kernel reads for this atom as a neighbour
    constexpr int KRP = (KR + 3) / 4 * 4;
    float* rec = nullptr;
    if constexpr (KIND == 3) {
        if (a >= 0) {
            rec = pes_rec + p * pes.rec_stride;
            for (int t = 0; t < T; ++t) {
                const float* __restrict__ cR = m.c_radial + (ti * T + t) * (NR * KR);
#pragma unroll
                for (int k = 0; k < KRP; ++k) {
                    float v = 0.f;
                    if (k < KR)
#pragma unroll
                        for (int n = 0; n < NR; ++n) v += dq[n] * cR[n * KR + (k < KR ? k : 0)];
                    rec[t * KRP + k] = v;
                }
            }
        }
    }

    // ---- 3. partial forces and contraction --------------------------------
    // the pair loop below uses the unnormalised harmonics: fold kShNorm into dU/dA
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int c = 0; c < kLM; ++c) A[n][c] *= kShNorm[c];
    // the dipole's atom term sums FP32 pair terms r^2 dU_i/dr_ij that can cancel
    // (a molecule's dipole can be a small remainder of its atom terms): FP64 sum
    float acc[NT];
    double accd[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NT; ++k) acc[k] = 0.f;
    float own[3] = {0.f, 0.f, 0.f};  // potential: sum_j dU_i/dr_ij, the atom's own force term
    int sq0 = -1, sq1 = -1, sq2 = -1, sq3 = -1;  // potential: slots of the current group of angular rows
    // (Fx, Fy, Fz) = dU_i/dr_ij for the pair vector (dx, dy, dz)
    auto contract = [&](float dx, float dy, float dz, float r2, float Fx, float Fy, float Fz) {
        if constexpr (KIND == 3) {
            own[0] += Fx;
            own[1] += Fy;
            own[2] += Fz;
        }
        if constexpr (KIND == 1) {
            const double r2d = (double)r2;
            accd[0] -= r2d * (double)Fx;
            accd[1] -= r2d * (double)Fy;
            accd[2] -= r2d * (double)Fz;
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

    ahead.fetch(nl, p, 0);
    for (int t = 0; t < T; ++t) {
        const float* __restrict__ cR = m.c_radial + (ti * T + t) * (NR * KR);
        const float* __restrict__ cA = m.c_angular + (ti * T + t) * (NA * KA);
        const float* __restrict__ cAd = m.c_angular_d + (ti * T + t) * (NA * KA);
        const SegCounts cur = ahead;
        if (t + 1 < T) ahead.fetch(nl, p, t + 1);
        const int n_ang = cur.n_ang, n_rad = cur.n_rad;
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
        // sum_k Dk f_k'(r) = (fc x' sum_k Dk T_k' + fc' (sum_k Dk T_k + sum_k Dk)) / 2, with
        // sum_k Dk T_k'(x) = sum_k Ek T_k(x): Ek the Chebyshev coefficients of the
        // derivative series (E_k = E_{k+2} + 2 (k+1) D_{k+1}, E_0 halved), so a pair
        // needs the T_k only, not their derivatives
        float Dsum = 0.f;
#pragma unroll
        for (int k = 0; k < KR; ++k) Dsum += Dk[k];
        float Ek[KR > 1 ? KR - 1 : 1];
#pragma unroll
        for (int k = KR - 2; k >= 0; --k) Ek[k] = (k + 2 <= KR - 2 ? Ek[k + 2] : 0.f) + (float)(2 * (k + 1)) * Dk[k + 1];
        Ek[0] *= 0.5f;
        float CsA[NA];  // sum_k c_nk of the angular coefficients (wave-uniform)
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            float c = 0.f;
#pragma unroll
            for (int k = 0; k < KA; ++k) c += cA[n * KA + k];
            CsA[n] = c;
        }
        auto radial_slope = [&](float r) {
            float fc, dfc, Tk[KR];
            cutoff_fc_d(1.f - r * rcR_inv, rcR_inv, fc, dfc);
            const float tt = r * rcR_inv - 1.f;
            cheb_T<KR>(2.f * tt * tt - 1.f, Tk);
            float s0 = Dsum, s1 = 0.f;
#pragma unroll
            for (int k = 0; k < KR; ++k) s0 += Dk[k] * Tk[k];
#pragma unroll
            for (int k = 0; k + 1 < KR; ++k) s1 += Ek[k] * Tk[k];
            return 0.5f * (fc * (4.f * tt * rcR_inv) * s1 + dfc * s0);
        };
        float4 nxt = n_ang > g ? ga[(g >> 2) * 256 + (g & 3)] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = g; s < n_ang; s += G) {
            const float4 e = nxt;
            if (s + G < n_ang) nxt = ga[((s + G) >> 2) * 256 + ((s + G) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = pair_rsqrt(r2);
            const float r = r2 * rinv;
            const float ux = e.x * rinv, uy = e.y * rinv, uz = e.z * rinv;
            const float sr = radial_slope(r);
            float fc, dfc, Tk[KA];
            cutoff_fc_d(1.f - r * rcA_inv, rcA_inv, fc, dfc);
            const float ta = r * rcA_inv - 1.f;
            cheb_T<KA>(2.f * ta * ta - 1.f, Tk);
            // g_n = fc/2 (P_n + C_n), g_n' = (fc x' Q_n + fc' (P_n + C_n)) / 2 with
            // P_n = sum_k c_nk T_k, Q_n = sum_k c_nk T_k' = sum_k c'_nk T_k (the model's
            // derivative-series coefficients), C_n = sum_k c_nk
            const float hfc = 0.5f * fc, hdfc = 0.5f * dfc, hfx = hfc * (4.f * ta * rcA_inv);
            float gA[NA], dgA[NA];
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                float pn = CsA[n], qn = 0.f;
#pragma unroll
                for (int k = 0; k < KA; ++k) pn += cA[n * KA + k] * Tk[k];
#pragma unroll
                for (int k = 0; k + 1 < KA; ++k) qn += cAd[n * KA + k] * Tk[k];
                gA[n] = hfc * pn;
                dgA[n] = hfx * qn + hdfc * pn;
            }
            // radial part: sum_lm (bv - l av / r) P, with sum_lm av P kept per l
            float Fx = 0.f, Fy = 0.f, Fz = 0.f, sb = 0.f, sa[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            sh_foreach_raw(ux, uy, uz, [&](int idx, int l, float P, float px, float py, float pz) {
                float av = 0.f, bv = 0.f;
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    av += A[n][idx] * gA[n];
                    bv += A[n][idx] * dgA[n];
                }
                Fx += av * px;
                Fy += av * py;
                Fz += av * pz;
                sb += bv * P;
                sa[l] += av * P;
            });
            const float su = sb - rinv * (sa[1] + 2.f * sa[2] + 3.f * sa[3] + 4.f * sa[4]) + sr;
            const float fx = Fx * rinv + ux * su, fy = Fy * rinv + uy * su, fz = Fz * rinv + uz * su;
            contract(e.x, e.y, e.z, r2, fx, fy, fz);
            if constexpr (KIND == 3) {
                if (a >= 0) {
                    const int u = s & 3;
                    const int64_t at = (ga - nl.entries) + ((s >> 2) * 256 + u);
                    pes_pair[at] = make_float4(fx, fy, fz, 0.f);
                    // the slots of a group of four rows leave as one 16-byte store
                    const int v = __float_as_int(e.w);
                    sq0 = u == 0 ? v : sq0;
                    sq1 = u == 1 ? v : sq1;
                    sq2 = u == 2 ? v : sq2;
                    sq3 = u == 3 ? v : sq3;
                    if (u == 3 || s + 1 == n_ang)
                        *reinterpret_cast<int4*>(pes_slot + (at - u)) = make_int4(sq0, sq1, sq2, sq3);
                }
            }
        }
        nxt = n_rad > g ? gr[(g >> 2) * 256 + (g & 3)] : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int s = g; s < n_rad; s += G) {
            const float4 e = nxt;
            if (s + G < n_rad) nxt = gr[((s + G) >> 2) * 256 + ((s + G) & 3)];
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            const float rinv = pair_rsqrt(r2);
            const float su = radial_slope(r2 * rinv) * rinv;
            contract(e.x, e.y, e.z, r2, e.x * su, e.y * su, e.z * su);
        }
    }

    if constexpr (G > 1) {
#pragma unroll
        for (int k = 0; k < NT; ++k) acc[k] = group_sum<G>(acc[k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) accd[k] = group_sum<G>(accd[k]);
    }
    if (a < 0 || g != 0) return;
    if constexpr (KIND == 3) {
        double* out = per_atom + (int64_t)a * 10;
        out[0] = (double)Us;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[1 + k] = (double)acc[k];
        *reinterpret_cast<float4*>(rec + T * KRP) = make_float4(own[0], own[1], own[2], 0.f);
        return;
    }
    double* out = per_atom + (int64_t)a * NT;
    if constexpr (KIND == 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] = accd[k];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = (double)acc[k] + ((k % 4 == 0) ? (double)Us : 0.0);
    }
}

// Frame sums in two steps.  k_frame_reduce: work-group (f, c) sums chunk c of
// frame f (atoms [c L, (c + 1) L), L = ceil(n / kReduceChunks)): lane l takes
// atoms l, l + 256, ... of the chunk in FP64, then a fixed tree, within each
// wavefront by shuffles and over the 4 wavefronts in LDS.  Frames of at most
// kSmallFrame atoms are left to k_frame_reduce_small: one wavefront per frame,
// lane l takes atoms l, l + 64, ..., then the shuffle tree; it stores the sum
// as chunk 0 and zeros as chunks 1..3.  k_frame_finish adds the chunk sums in
// chunk order.  A batch of small frames only skips k_frame_finish: the small
// kernel stores 0 + sum itself, which is what the chunk order gives bit for bit
// (the zero chunks add nothing; 0 + (-0) = +0 as there).  The order depends only on the frame's atom count, never on
// how frames were batched; the chunks spread a launch batch of large frames
// over all compute units, and a batch of small frames takes one wavefront,
// not sixteen, per frame.
constexpr int kReduceBlock = 256;
__global__ void __launch_bounds__(kReduceBlock) k_frame_reduce_small(const FrameInfo* __restrict__ frames,
                                                                     const int32_t* __restrict__ meta,
                                                                     const double* __restrict__ per_atom, int nt,
                                                                     double* __restrict__ part_out, int na,
                                                                     double* __restrict__ out_a,
                                                                     double* __restrict__ out_b, bool direct) {
    const int f = blockIdx.x * (kReduceBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= meta[kMetaNFrames]) return;
    const FrameInfo fi = frames[f];
    if (fi.n_atoms > kSmallFrame) return;
    double s[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) s[k] = 0.0;
    for (int64_t a = lane; a < fi.n_atoms; a += 64) {
        const double* q = per_atom + (fi.atom_begin + a) * nt;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (k < nt) s[k] += q[k];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        if (k < nt) {
            double v = s[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            s[k] = v;
        }
    }
    if (direct) {
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                if (k >= nt) continue;
                const double v = 0.0 + s[k];
                if (k < na)
                    out_a[(int64_t)f * na + k] = v;
                else if (out_b)
                    out_b[(int64_t)f * (nt - na) + k - na] = v;
            }
        return;
    }
    if (lane < kReduceChunks) {
        double* o = part_out + ((int64_t)f * kReduceChunks + lane) * 10;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (k < nt) o[k] = lane == 0 ? s[k] : 0.0;
    }
}

__global__ void __launch_bounds__(kReduceBlock) k_frame_reduce(const FrameInfo* __restrict__ frames,
                                                               const int32_t* __restrict__ meta,
                                                               const double* __restrict__ per_atom, int nt,
                                                               double* __restrict__ part_out) {
    constexpr int kWaves = kReduceBlock / 64;
    __shared__ double part[10][kWaves];
    const int f = blockIdx.x, c = blockIdx.y;
    if (f >= meta[kMetaNFrames]) return;
    const FrameInfo fi = frames[f];
    if (fi.n_atoms <= kSmallFrame) return;
    const int64_t len = (fi.n_atoms + kReduceChunks - 1) / kReduceChunks;
    const int64_t a0 = c * len, a1 = min((int64_t)fi.n_atoms, a0 + len);
    const int lane = threadIdx.x;
    double s[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) s[k] = 0.0;
    for (int64_t a = a0 + lane; a < a1; a += kReduceBlock) {
        const double* q = per_atom + (fi.atom_begin + a) * nt;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            if (k < nt) s[k] += q[k];
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        if (k < nt) {
            double v = s[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if ((lane & 63) == 0) part[k][lane >> 6] = v;
        }
    }
    __syncthreads();
    if (lane < nt) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += part[lane][w];
        part_out[((int64_t)f * kReduceChunks + c) * 10 + lane] = v;
    }
}

__global__ void k_frame_finish(const int32_t* __restrict__ meta, const double* __restrict__ part, int nt, int na,
                               double* __restrict__ out_a, double* __restrict__ out_b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f = (int)(i / nt), k = (int)(i % nt);
    if (f >= meta[kMetaNFrames]) return;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < kReduceChunks; ++c) v += part[((int64_t)f * kReduceChunks + c) * 10 + k];
    if (k < na)
        out_a[(int64_t)f * na + k] = v;
    else if (out_b)
        out_b[(int64_t)f * (nt - na) + k - na] = v;
}

// Charged molecules (the dipole of a charged system depends on the reference
// point; the model gives it relative to the centre of mass):
//   mu[f] += Q_f * unit * sum_i m_i r_i / sum_i m_i,
// one work-group per frame, FP64 sums in a fixed order.
__global__ void __launch_bounds__(256) k_com_shift(const int64_t* __restrict__ offsets,
                                                   const double* __restrict__ pos,
                                                   const int32_t* __restrict__ species,
                                                   const double* __restrict__ masses,
                                                   const double* __restrict__ charges, double unit,
                                                   double* __restrict__ mu) {
    __shared__ double part[4][256];
    const int f = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t a0 = offsets[f], a1 = offsets[f + 1];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t a = a0 + lane; a < a1; a += 256) {
        const double w = masses[species[a]];
        s[0] += w * pos[3 * a];
        s[1] += w * pos[3 * a + 1];
        s[2] += w * pos[3 * a + 2];
        s[3] += w;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) part[k][lane] = s[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (lane < off)
#pragma unroll
            for (int k = 0; k < 4; ++k) part[k][lane] += part[k][lane + off];
        __syncthreads();
    }
    if (lane < 3 && part[3][0] > 0.0) mu[3 * (int64_t)f + lane] += charges[f] * unit * part[lane][0] / part[3][0];
}

// angular pairs whose lookups k_pes_forces overlaps
constexpr int kLookups = 8;

// Forces of a potential-energy model (Sec. 2.1): with r_ij = r_j - r_i,
//   F_k = -dU/dr_k = sum_j dU_k/dr_kj - sum_j dU_j/dr_jk.
// The first sum is in the atom's record (evaluation kernel).  For the second,
// the lane of atom k takes, for every neighbour j:
//   r_kj < r_c^A: the pair force dU_j/dr_jk that j's evaluation stored at k's
//     entry in j's angular segment of k's species; the lane finds that entry by
//     its slot (the segment holds ~10-20 entries; j's evaluation also stored the
//     entries' slots compactly, four rows per 16-byte load);
//   otherwise: the radial part sum_k' Dk_j[k'] f'_k'(r) from j's record with
//     j's coefficients c_{t_j t_k} (48 bytes and ~60 instructions per pair).
// A pair that j's search classified on the other side of r_c^A (rounding at
// the boundary) is not in that segment and takes the radial form, the angular
// terms vanishing there with f_c(r_c^A).  Every term is summed in the lane's
// fixed list order: no atomics.
template <int NR, int NA, int KR, int KA, int MB>
__global__ void __launch_bounds__(256) k_pes_forces(DevModel m, NeighborLists nl, PesOut pes,
                                                    const double* __restrict__ per_atom,
                                                    double* __restrict__ forces, double* __restrict__ energies) {
    constexpr int KRP = (KR + 3) / 4 * 4;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int T = nl.T;
    const int tile = __builtin_amdgcn_readfirstlane((int)(p >> 6));
    const int lane = (int)(p & 63);
    if (tile >= nl.meta[kMetaTileBase + T]) return;
    const int a = nl.perm[p];
    const int tk = tile_species(nl.meta + kMetaTileBase, T, tile);
    const float rcR_inv = 1.f / m.rc_radial;
    const float4* lane_base = nl.entries + ((int64_t)tile * (nl.slots >> 2) * 64 + lane) * 4;
    const int64_t seg_a_k = (int64_t)(nl.meta[kMetaSegA + tk] >> 2) * 256;  // angular segment of k's species
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;  // - sum_j dU_j/dr_jk
    // sum_k D_k f_k'(r) from Chebyshev sums (as in k_eval), D from j's record
    auto radial_slope = [&](const float* rj, float r) {
        float fc, dfc, Tk[KRP], dT[KRP];
        cutoff_fc_d(1.f - r * rcR_inv, rcR_inv, fc, dfc);
        const float tt = r * rcR_inv - 1.f;
        cheb_T_d<KR>(2.f * tt * tt - 1.f, Tk, dT);
        const float4* d4 = reinterpret_cast<const float4*>(rj + tk * KRP);
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int k = 0; k < KRP; k += 4) {
            const float4 d = d4[k / 4];
            const float dd[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k + u < KR) {
                    s0 += dd[u] * (Tk[k + u] + 1.f);
                    s1 += dd[u] * dT[k + u];
                }
        }
        return 0.5f * (fc * (4.f * tt * rcR_inv) * s1 + dfc * s0);
    };
    // - dU_j/dr_jk, radial part, for the entry vector e = r_kj
    auto radial_term = [&](const float4& e) {
        const float* rj = pes.rec + (int64_t)__float_as_int(e.w) * pes.rec_stride;
        const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
        const float rinv = pair_rsqrt(r2);
        const float su = radial_slope(rj, r2 * rinv) * rinv;
        Fx += e.x * su;
        Fy += e.y * su;
        Fz += e.z * su;
    };
    for (int t = 0; t < T; ++t) {
        const int n_ang = nl.counts[(int64_t)(2 * t) * nl.n_pad + p];
        const int n_rad = nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p];
        const float4* ga = lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256;
        const float4* gr = lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256;
        // kLookups pairs at a time: the loads of their lookups (the neighbour's count
        // and the slots of the first four rows of its segment, one 16-byte word, in
        // bounds since segment capacities are multiples of four) are issued before any
        // is used
        for (int s = 0; s < n_ang; s += kLookups) {
            float4 e[kLookups];
            int g[kLookups][4];
            int64_t ja[kLookups];
            int nj[kLookups], row[kLookups];
#pragma unroll
            for (int w = 0; w < kLookups; ++w) {
                const int sw = min(s + w, n_ang - 1);  // past the end: repeat the last pair, unused
                e[w] = ga[(sw >> 2) * 256 + (sw & 3)];
                const int j = __float_as_int(e[w].w);
                // j's angular segment of species t_k, searched for this lane's slot
                ja[w] = ((int64_t)(j >> 6) * (nl.slots >> 2) * 64 + (j & 63)) * 4 + seg_a_k;
                nj[w] = s + w < n_ang ? nl.counts[(int64_t)(2 * tk) * nl.n_pad + j] : 0;
                const int4 q = *reinterpret_cast<const int4*>(pes.slot + ja[w]);
                g[w][0] = q.x;
                g[w][1] = q.y;
                g[w][2] = q.z;
                g[w][3] = q.w;
            }
#pragma unroll
            for (int w = 0; w < kLookups; ++w) {
                row[w] = -1;
#pragma unroll
                for (int u = 3; u >= 0; --u)
                    if (u < nj[w] && g[w][u] == (int)p) row[w] = u;
                for (int r0 = 4; r0 < nj[w] && row[w] < 0; r0 += 4) {
                    const int4 q = *reinterpret_cast<const int4*>(pes.slot + ja[w] + (int64_t)(r0 >> 2) * 256);
                    const int gq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (r0 + u < nj[w] && gq[u] == (int)p) row[w] = r0 + u;
                }
            }
            float4 f[kLookups];
#pragma unroll
            for (int w = 0; w < kLookups; ++w)
                f[w] = row[w] >= 0 ? pes.pair[ja[w] + (int64_t)(row[w] >> 2) * 256 + (row[w] & 3)]
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int w = 0; w < kLookups; ++w) {
                if (s + w >= n_ang) break;
                if (row[w] >= 0) {
                    Fx -= f[w].x;
                    Fy -= f[w].y;
                    Fz -= f[w].z;
                } else {
                    radial_term(e[w]);
                }
            }
        }
#pragma unroll 2
        for (int s = 0; s < n_rad; ++s) radial_term(gr[(s >> 2) * 256 + (s & 3)]);
    }
    if (a < 0) return;
    const float4 own = *reinterpret_cast<const float4*>(pes.rec + p * pes.rec_stride + T * KRP);
    if (forces) {
        forces[3 * (int64_t)a] = (double)own.x + (double)Fx;
        forces[3 * (int64_t)a + 1] = (double)own.y + (double)Fy;
        forces[3 * (int64_t)a + 2] = (double)own.z + (double)Fz;
    }
    if (energies) energies[a] = per_atom[10 * (int64_t)a];
}

template <int NR, int NA, int KR, int KA, int MB, int KIND, int MODE>
hipError_t launch_t(const DevModel& m, const NeighborLists& nl, double* per_atom, const PesOut& pes,
                    const RadSums& rs, int block, bool pair_parallel, hipStream_t s) {
    constexpr int D = NR + 4 * NA + ((MB & 1) ? NA : 0) + ((MB & 2) ? NA : 0);
    if constexpr (MODE == TNEP_MLP_FP32_VALU && KIND != 3) {
        if (pair_parallel) {  // kPairLanes lanes per tile slot; n_pad is a multiple of 64
            const unsigned grid = (unsigned)(nl.n_pad * kPairLanes / 256);
            k_eval<NR, NA, KR, KA, MB, KIND, MODE, false, kPairLanes><<<grid, 256, 0, s>>>(
                m, nl, per_atom, pes, nullptr, pes.rec, pes.pair, pes.slot);
            return hipGetLastError();
        }
    }
    if constexpr (MODE == TNEP_MLP_FP32_VALU) {
        const int bs = (block == 64 || block == 128) ? block : 256;
        const unsigned grid = (unsigned)((nl.n_pad + bs - 1) / bs);
        if (rs.mode == 2 && KR == kRadialTerms)
            k_eval<NR, NA, KR, KA, MB, KIND, MODE, KR == kRadialTerms><<<grid, bs, 0, s>>>(m, nl, per_atom, pes, rs.v,
                                                                                        pes.rec, pes.pair, pes.slot);
        else
            k_eval<NR, NA, KR, KA, MB, KIND, MODE><<<grid, bs, 0, s>>>(m, nl, per_atom, pes, nullptr, pes.rec, pes.pair, pes.slot);
    } else {
        // two wavefronts per work-group keep the LDS tiles at <= 2 x 27 KB
        const unsigned grid = (unsigned)((nl.n_pad + 127) / 128);
        const size_t lds = sizeof(float) * 2 * (size_t)mlp_lds_floats(D, m.n_hidden);
        k_eval<NR, NA, KR, KA, MB, KIND, MODE><<<grid, 128, lds, s>>>(m, nl, per_atom, pes, nullptr, pes.rec, pes.pair, pes.slot);
    }
    return hipGetLastError();
}

template <int NR, int NA, int KR, int KA, int MB, int KIND>
hipError_t launch_mode(int mode, bool matrix, const DevModel& m, const NeighborLists& nl, double* per_atom,
                       const PesOut& pes, const RadSums& rs, int block, bool pp, hipStream_t s) {
    if (matrix) {
        if (mode == TNEP_MLP_FP32_MFMA)
            return launch_t<NR, NA, KR, KA, MB, KIND, TNEP_MLP_FP32_MFMA>(m, nl, per_atom, pes, rs, block, pp, s);
        if (mode == TNEP_MLP_BF16_MFMA)
            return launch_t<NR, NA, KR, KA, MB, KIND, TNEP_MLP_BF16_MFMA>(m, nl, per_atom, pes, rs, block, pp, s);
        if (mode == TNEP_MLP_BF16X3_MFMA)
            return launch_t<NR, NA, KR, KA, MB, KIND, TNEP_MLP_BF16X3_MFMA>(m, nl, per_atom, pes, rs, block, pp, s);
    }
    return launch_t<NR, NA, KR, KA, MB, KIND, TNEP_MLP_FP32_VALU>(m, nl, per_atom, pes, rs, block, pp, s);
}

// Potential-energy models always use the FP32 vector hidden layer.
// pp: the pair-parallel layout (tensor models, FP32 vector hidden layer).
template <int NR, int NA, int KR, int KA, int MB, bool MX>
hipError_t dispatch(const Shape& shape, int mode, bool matrix, const DevModel& m, const NeighborLists& nl,
                    double* per_atom, const PesOut& pes, const RadSums& rs, int block, bool pp, hipStream_t s) {
    if (shape.kind == 3)
        return launch_t<NR, NA, KR, KA, MB, 3, TNEP_MLP_FP32_VALU>(m, nl, per_atom, pes, rs, block, false, s);
    if constexpr (MX) {
        if (shape.kind == 1)
            return launch_mode<NR, NA, KR, KA, MB, 1>(mode, matrix, m, nl, per_atom, pes, rs, block, pp, s);
        return launch_mode<NR, NA, KR, KA, MB, 2>(mode, matrix, m, nl, per_atom, pes, rs, block, pp, s);
    } else {
        if (shape.kind == 1)
            return launch_t<NR, NA, KR, KA, MB, 1, TNEP_MLP_FP32_VALU>(m, nl, per_atom, pes, rs, block, pp, s);
        return launch_t<NR, NA, KR, KA, MB, 2, TNEP_MLP_FP32_VALU>(m, nl, per_atom, pes, rs, block, pp, s);
    }
}

}  // namespace

// Compiled descriptor shapes (radial functions, angular functions, radial and
// angular Chebyshev terms, many-body terms: 1 four-body, 2 five-body) and
// whether the matrix-core hidden layers are compiled for them.
#define TNEP_SHAPES(X)      \
    X(5, 5, 9, 9, 1, true)  \
    X(5, 5, 9, 9, 0, false) \
    X(7, 5, 9, 9, 0, true)  \
    X(7, 5, 9, 9, 1, false) \
    X(5, 5, 9, 9, 3, false)

static int shape_bodies(const Shape& s) { return (s.four_body ? 1 : 0) | (s.five_body ? 2 : 0); }

bool eval_shape_supported(const Shape& s) {
#define X(NR_, NA_, KR_, KA_, FB_, MX_) \
    if (s.nr == NR_ && s.na == NA_ && s.kr == KR_ && s.ka == KA_ && shape_bodies(s) == FB_) return true;
    TNEP_SHAPES(X)
#undef X
    return false;
}

bool eval_matrix_supported(const Shape& s, int n_hidden) {
    if (n_hidden > 64) return false;
#define X(NR_, NA_, KR_, KA_, FB_, MX_) \
    if (s.nr == NR_ && s.na == NA_ && s.kr == KR_ && s.ka == KA_ && shape_bodies(s) == FB_) return MX_;
    TNEP_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_eval(const Shape& shape, const DevModel& m, const NeighborLists& nl, double* per_atom,
                       const PesOut& pes, const RadSums& rs, const EvalLaunch& cfg, hipStream_t s) {
    if (nl.n_pad == 0) return hipSuccess;
    // the matrix-core hidden layer holds one shared network; the pair-parallel
    // layout takes the vector hidden layer
    const bool pp = cfg.pair_parallel != 0;
    const bool matrix = !pp && cfg.mlp_mode != TNEP_MLP_FP32_VALU && eval_matrix_supported(shape, m.n_hidden) &&
                        m.sp_w0 == 0;
#define X(NR_, NA_, KR_, KA_, FB_, MX_)                                                             \
    if (shape.nr == NR_ && shape.na == NA_ && shape.kr == KR_ && shape.ka == KA_ &&                \
        shape_bodies(shape) == FB_)                                                             \
        return dispatch<NR_, NA_, KR_, KA_, FB_, MX_>(shape, cfg.mlp_mode, matrix, m, nl, per_atom, pes, rs,  \
                                                      cfg.atoms_per_block, pp, s);
    TNEP_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_frame_reduce(const FrameInfo* d_frames, int cap_frames, const int32_t* meta, const double* per_atom,
                               int nt, int na, double* part, double* out_a, double* out_b, bool small, bool large,
                               hipStream_t s) {
    if (cap_frames == 0) return hipSuccess;
    const bool direct = small && !large;
    if (small)
        k_frame_reduce_small<<<(unsigned)((cap_frames + kReduceBlock / 64 - 1) / (kReduceBlock / 64)), kReduceBlock, 0,
                               s>>>(d_frames, meta, per_atom, nt, part, na, out_a, out_b, direct);
    if (direct) return hipGetLastError();
    if (large)
        k_frame_reduce<<<dim3(cap_frames, kReduceChunks), kReduceBlock, 0, s>>>(d_frames, meta, per_atom, nt, part);
    const int64_t n = (int64_t)cap_frames * nt;
    k_frame_finish<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(meta, part, nt, na, out_a, out_b);
    return hipGetLastError();
}

hipError_t launch_com_shift(const int64_t* offsets, int n_frames, const double* pos, const int32_t* species,
                            const double* masses, const double* charges, double unit, double* mu, hipStream_t s) {
    if (n_frames == 0) return hipSuccess;
    k_com_shift<<<n_frames, 256, 0, s>>>(offsets, pos, species, masses, charges, unit, mu);
    return hipGetLastError();
}

hipError_t launch_pes_forces(const Shape& shape, const DevModel& m, const NeighborLists& nl, const PesOut& pes,
                             const double* per_atom, double* forces, double* energies, int block, hipStream_t s) {
    if (nl.n_pad == 0 || (!forces && !energies)) return hipSuccess;
    const int bs = (block == 64 || block == 128) ? block : 256;
    const unsigned grid = (unsigned)((nl.n_pad + bs - 1) / bs);
#define X(NR_, NA_, KR_, KA_, FB_, MX_)                                                                 \
    if (shape.nr == NR_ && shape.na == NA_ && shape.kr == KR_ && shape.ka == KA_ &&                    \
        shape_bodies(shape) == FB_) {                                                               \
        k_pes_forces<NR_, NA_, KR_, KA_, FB_><<<grid, bs, 0, s>>>(m, nl, pes, per_atom, forces, energies); \
        return hipGetLastError();                                                                     \
    }
    TNEP_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace tnep
