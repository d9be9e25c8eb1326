// Spectra from tensor time series on gfx950, all FP64 (Sec. 2.6 The IR
// intensity, Sec. 2.7 The Raman intensity).
//
// Correlation functions are averages over time origins (Sec. 2.6):
//   C_xy(tau) = 1/(N - tau) sum_{t=0}^{N-1-tau} x(t) y(t + tau).
// They are computed through zero-padded FFTs of length P >= 2N (no circular
// wrap-around): IFFT(conj(X) Y)[tau] / P = sum_t x(t) y(t + tau).
// Channels:
//   IR     (1/3) sum_a C_{mu_a mu_a}                         (isotropic sample)
//   iso    C_{gamma gamma},  gamma = Tr(alpha)/3             (Eq. raman-lineshape-isotropic-anisotropic)
//   aniso  sum_ab C_{beta_ab beta_ba}, beta = alpha - gamma I  (<Tr beta(0) beta(t)>)
//   proj   C_{s s}, s = n^T alpha e                          (Eq. raman-cross-section)
//   map    C_{PQ}, P, Q over the nine components of alpha, symmetrised, for the
//          orientation-resolved lineshape sum n_g n_m L_gdmn e_d e_n
//          (Eqs. raman-cross-section, raman-lineshape): one pass, any number
//          of polarisation pairs by contraction of the 45 channel spectra
// The one-sided cosine transform with the lag window,
//   S(w_k) = dt/(2 pi) [w(0) C(0) + 2 sum_{tau=1}^{M-1} w(tau) C(tau) cos(pi k tau / M)],
// is summed directly with an exact integer phase index into a cosine table;
// IR spectra carry the classical w^2 prefactor (Eq. ir-intensity); Raman
// spectra optionally the ((w_in - w) / c)^4 factor of Eq. raman-cross-section.
// Long series can also be fed in chunks (streaming accumulators below).
#include <algorithm>

#include "internal.h"

namespace tnep {

namespace {

constexpr int kB = 256;
constexpr int kFftBlock = 64;      // FFT launches: small batches still spread over every compute unit
constexpr int kStateBlock = 1024;  // k_stream_state: one work-group per signal
constexpr int kBlkThreads = 256;   // blocked streaming transforms: 16 points per lane per pass

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

int signals_per_series(int kind) {
    switch (kind) {
        case 0: return 3;   // mu_x, mu_y, mu_z
        case 1: return 1;   // gamma
        case 2: return 9;   // beta_ab
        case 4: return 9;   // alpha_ab (orientation map)
        default: return 1;  // n^T alpha e
    }
}

// Mean of every component of every series: one work-group per (series, component).
__global__ void k_means(const double* __restrict__ series, int64_t n_steps, int comps, double* __restrict__ means) {
    const int s = blockIdx.x / comps, c = blockIdx.x % comps;
    __shared__ double part[kB];
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < n_steps; t += kB) acc += series[((int64_t)s * n_steps + t) * comps + c];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) means[blockIdx.x] = part[0] / (double)n_steps;
}

// Derived scalar signals, zero-padded to P, as complex numbers.
// grid: (ceil(P / kB), n_series)
__global__ void k_signals(const double* __restrict__ series, const double* __restrict__ means, int64_t n_steps,
                          int64_t P, int kind, int comps, int nsig, double nx, double ny, double nz, double ex,
                          double ey, double ez, cplx* __restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
    const int s = blockIdx.y;
    if (t >= P) return;
    cplx* out = X + (int64_t)s * nsig * P;
    if (t >= n_steps) {
        for (int g = 0; g < nsig; ++g) out[(int64_t)g * P + t] = {0.0, 0.0};
        return;
    }
    double v[9];
    const double* row = series + ((int64_t)s * n_steps + t) * comps;
    for (int c = 0; c < comps; ++c) v[c] = row[c] - (means ? means[s * comps + c] : 0.0);
    if (kind == 0) {
        for (int a = 0; a < 3; ++a) out[(int64_t)a * P + t] = {v[a], 0.0};
    } else if (kind == 4) {
        for (int c = 0; c < 9; ++c) out[(int64_t)c * P + t] = {v[c], 0.0};
    } else {
        const double gamma = (v[0] + v[4] + v[8]) / 3.0;
        if (kind == 1) {
            out[t] = {gamma, 0.0};
        } else if (kind == 2) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) out[(int64_t)(3 * a + b) * P + t] = {v[3 * a + b] - (a == b ? gamma : 0.0), 0.0};
        } else {
            const double n[3] = {nx, ny, nz}, e[3] = {ex, ey, ez};
            double p = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) p += n[a] * v[3 * a + b] * e[b];
            out[t] = {p, 0.0};
        }
    }
}

// One radix-2 Stockham pass over `batch` sequences of length P (ping-pong).
// Pass with half-size span m = 2^p: out[j*2m + k] and out[j*2m + k + m] from
// in[j*m + k] and in[j*m + k + P/2], twiddle exp(-+ 2 pi i k / (2m)).
__global__ void k_fft_pass(const cplx* __restrict__ in, cplx* __restrict__ out, int64_t P, int64_t m, double sign) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t half = P >> 1;
    if (tid >= half) return;
    const int64_t b = blockIdx.y;
    const cplx* src = in + b * P;
    cplx* dst = out + b * P;
    const int64_t k = tid % m;
    const int64_t j = tid / m;
    const cplx a = src[tid];
    const cplx c = src[tid + half];
    double sn, cs;
    sincospi(sign * (double)k / (double)m, &sn, &cs);
    const cplx w = cmul({cs, sn}, c);
    dst[j * 2 * m + k] = {a.re + w.re, a.im + w.im};
    dst[j * 2 * m + k + m] = {a.re - w.re, a.im - w.im};
}

// R = 2^r consecutive radix-2 passes (half spans m, 2m, ..., (R/2) m) in one
// launch, each butterfly with the twiddle and arithmetic of k_fft_pass, so the
// result is that of the r passes.  Thread tid < P/R (k = tid % m, j = tid / m)
// reads in[tid + a P/R], a < R.  Before pass s (half span M = 2^s m) it holds
// the elements j 2^s m + k + c m + a 2^s P/R (c < 2^s, a < R/2^s) at x[c + 2^s a];
// the pass pairs a with a + R/2^(s+1) (index t and t + P/2) under the twiddle
// of K = k + c m, and the thread ends with out[j R m + k + c m], c < R.
template <int R>
__global__ void k_fft_radix(const cplx* __restrict__ in, cplx* __restrict__ out, int64_t P, int64_t m, double sign) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = P / R;
    if (tid >= q) return;
    const int64_t b = blockIdx.y;
    const cplx* src = in + b * P;
    cplx* dst = out + b * P;
    const int64_t k = tid % m;
    const int64_t j = tid / m;
    cplx x[R], y[R];
#pragma unroll
    for (int a = 0; a < R; ++a) x[a] = src[tid + a * q];
#pragma unroll
    for (int S = 1; S < R; S <<= 1) {  // S = 2^s
        const int64_t M = S * m;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            double sn, cs;
            sincospi(sign * (double)(k + c * m) / (double)M, &sn, &cs);
#pragma unroll
            for (int a = 0; a < R / (2 * S); ++a) {
                const cplx lo = x[c + S * a], hi = x[c + S * (a + R / (2 * S))];
                const cplx w = cmul({cs, sn}, hi);
                y[c + 2 * S * a] = {lo.re + w.re, lo.im + w.im};
                y[c + S + 2 * S * a] = {lo.re - w.re, lo.im - w.im};
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = y[i];
    }
    cplx* o = dst + j * R * m + k;
#pragma unroll
    for (int c = 0; c < R; ++c) o[c * m] = x[c];
}

// Per series: combine the signal spectra into the channel's cross power.
__global__ void k_power(const cplx* __restrict__ X, int64_t P, int kind, int nsig, cplx* __restrict__ Z) {
    const int64_t f = (int64_t)blockIdx.x * kB + threadIdx.x;
    const int s = blockIdx.y;
    if (f >= P) return;
    const cplx* x = X + (int64_t)s * nsig * P;
    double p = 0.0;
    if (kind == 2) {
        // sum_ab conj(B_ab) B_ba
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const cplx u = x[(int64_t)(3 * a + b) * P + f];
                const cplx v = x[(int64_t)(3 * b + a) * P + f];
                p += u.re * v.re + u.im * v.im;
            }
    } else {
        for (int g = 0; g < nsig; ++g) {
            const cplx u = x[(int64_t)g * P + f];
            p += u.re * u.re + u.im * u.im;
        }
        if (kind == 0) p /= 3.0;
    }
    Z[(int64_t)s * P + f] = {p, 0.0};
}

// C(tau) averaged over series, unbiased normalisation; Re(IFFT)/P.
__global__ void k_acf(const cplx* __restrict__ Z, int64_t P, int n_series, int64_t n_steps, int64_t M,
                      double* __restrict__ acf) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    double s = 0.0;
    for (int k = 0; k < n_series; ++k) s += Z[(int64_t)k * P + tau].re;
    acf[tau] = s / (double)P / (double)(n_steps - tau) / (double)n_series;
}

__global__ void k_cos_table(int64_t M, double* __restrict__ tab) {
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j < 2 * M) tab[j] = cospi((double)j / (double)M);
}

// S_k for k = 0..M of channel blockIdx.y; one thread per k.  Phase index
// (k tau) mod 2M kept exact.  laser_cm1 > 0 multiplies by (2 pi (laser - nu_k))^4.
__global__ void k_transform(const double* __restrict__ acf, int64_t acf_stride, const double* __restrict__ tab,
                            int64_t M, int window, int omega2, double laser_cm1, double dt_fs,
                            double* __restrict__ freq, double* __restrict__ intensity, int64_t out_stride) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k > M) return;
    const double* a = acf + (int64_t)blockIdx.y * acf_stride;
    const int64_t twoM = 2 * M;
    const int64_t step = k % twoM;
    int64_t idx = step;  // (k * tau) mod 2M for tau = 1
    double s = a[0];     // w(0) = 1
    for (int64_t tau = 1; tau < M; ++tau) {
        const double w = window == 0 ? 0.5 * (1.0 + tab[tau]) : 1.0;  // tab[tau] = cos(pi tau / M)
        s += 2.0 * w * a[tau] * tab[idx];
        idx += step;
        if (idx >= twoM) idx -= twoM;
    }
    const double pi = 3.14159265358979323846;
    s *= dt_fs / (2.0 * pi);
    const double omega = pi * (double)k / ((double)M * dt_fs);
    if (omega2) s *= omega * omega;
    const double nu = (double)k / (2.0 * (double)M * dt_fs * 2.99792458e-5);
    if (laser_cm1 > 0.0) {
        const double d = 2.0 * pi * (laser_cm1 - nu);
        s *= (d * d) * (d * d);
    }
    intensity[(int64_t)blockIdx.y * out_stride + k] = s;
    if (blockIdx.y == 0 && freq) freq[k] = nu;
}

// ---- orientation map: 45 symmetrised channels (P <= Q over the nine components)

__device__ __forceinline__ void pair_of(int q, int& P, int& Q) {
    P = 0;
    int left = q;
    while (left >= 9 - P) {
        left -= 9 - P;
        ++P;
    }
    Q = P + left;
}

// Z[q][f] = sum_s Re(conj(X_sP) X_sQ): the spectrum of (C_PQ + C_QP) / 2, summed over series.
__global__ void k_power_sym(const cplx* __restrict__ X, int64_t P_len, int n_series, cplx* __restrict__ Z) {
    const int64_t f = (int64_t)blockIdx.x * kB + threadIdx.x;
    const int q = blockIdx.y;
    if (f >= P_len) return;
    int P, Q;
    pair_of(q, P, Q);
    double acc = 0.0;
    for (int sr = 0; sr < n_series; ++sr) {
        const cplx u = X[((int64_t)sr * 9 + P) * P_len + f];
        const cplx v = X[((int64_t)sr * 9 + Q) * P_len + f];
        acc += u.re * v.re + u.im * v.im;
    }
    Z[(int64_t)q * P_len + f] = {acc, 0.0};
}

// acf[q][tau] = Re(Z[q][tau]) / P / (N - tau) / n_series
__global__ void k_acf_channels(const cplx* __restrict__ Z, int64_t P_len, int n_series, int64_t n_steps, int64_t M,
                               double* __restrict__ acf) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    const int q = blockIdx.y;
    acf[(int64_t)q * M + tau] = Z[(int64_t)q * P_len + tau].re / (double)P_len / (double)(n_steps - tau) /
                                (double)n_series;
}

// out[o][k] = sum_q W[o][q] L[q][k]
__global__ void k_contract(const double* __restrict__ L, int64_t M, const double* __restrict__ W, int nq,
                           double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k > M) return;
    const int o = blockIdx.y;
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += W[o * nq + q] * L[(int64_t)q * (M + 1) + k];
    out[(int64_t)o * (M + 1) + k] = s;
}

// ---- streaming accumulators ------------------------------------------------
// A run is fed in chunks.  For every channel (x, y) the run keeps
// S(tau) = sum_{t + tau < N} x(t) y(t + tau); a chunk adds the pairs whose
// later sample is new: with u = [carry | chunk] (carry = last M - 1 samples)
// and v = [0 | chunk], IFFT(conj(U) V)[tau] / P.

__device__ __forceinline__ void derive_signals(int kind, const double* v, double nx, double ny, double nz, double ex,
                                               double ey, double ez, double* out) {
    if (kind == 0) {
        for (int a = 0; a < 3; ++a) out[a] = v[a];
    } else if (kind == 4) {
        for (int c = 0; c < 9; ++c) out[c] = v[c];
    } else {
        const double gamma = (v[0] + v[4] + v[8]) / 3.0;
        if (kind == 1) {
            out[0] = gamma;
        } else if (kind == 2) {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) out[3 * a + b] = v[3 * a + b] - (a == b ? gamma : 0.0);
        } else {
            const double n[3] = {nx, ny, nz}, e[3] = {ex, ey, ez};
            double p = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) p += n[a] * v[3 * a + b] * e[b];
            out[0] = p;
        }
    }
}

// U[g][t] = (carry | signals of the chunk | 0), V[g][t] = (0 | signals | 0).
__global__ void k_stream_build(const double* __restrict__ chunk, int64_t n, int comps, int kind, int nsig,
                               double nx, double ny, double nz, double ex, double ey, double ez,
                               const double* __restrict__ carry, int64_t carry_cap, int64_t c, int64_t P_len,
                               cplx* __restrict__ U, cplx* __restrict__ V) {
    const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (t >= P_len) return;
    if (t < c) {
        for (int g = 0; g < nsig; ++g) {
            U[(int64_t)g * P_len + t] = {carry[(int64_t)g * carry_cap + t], 0.0};
            V[(int64_t)g * P_len + t] = {0.0, 0.0};
        }
    } else if (t < c + n) {
        double v[9], sg[9];
        const double* row = chunk + (t - c) * comps;
        for (int k = 0; k < comps; ++k) v[k] = row[k];
        derive_signals(kind, v, nx, ny, nz, ex, ey, ez, sg);
        for (int g = 0; g < nsig; ++g) {
            U[(int64_t)g * P_len + t] = {sg[g], 0.0};
            V[(int64_t)g * P_len + t] = {sg[g], 0.0};
        }
    } else {
        for (int g = 0; g < nsig; ++g) {
            U[(int64_t)g * P_len + t] = {0.0, 0.0};
            V[(int64_t)g * P_len + t] = {0.0, 0.0};
        }
    }
}

// Run state from U before its transform: new carry (last min(M-1, c+n)
// samples), the first M samples of the run (head) and per-signal totals.
// One work-group per signal.
__global__ void __launch_bounds__(kStateBlock) k_stream_state(const cplx* __restrict__ U, int64_t P_len, int64_t c, int64_t n,
                               int64_t carry_cap, double* __restrict__ carry_new, int64_t run_len,
                               double* __restrict__ head, int64_t M, double* __restrict__ totals) {
    const int g = blockIdx.x;
    const cplx* u = U + (int64_t)g * P_len;
    const int64_t L = c + n;
    const int64_t keep = L < carry_cap ? L : carry_cap;
    for (int64_t i = threadIdx.x; i < keep; i += kStateBlock) carry_new[(int64_t)g * carry_cap + i] = u[L - keep + i].re;
    for (int64_t i = threadIdx.x; i < n; i += kStateBlock) {
        const int64_t r = run_len + i;  // position in the run
        if (r < M) head[(int64_t)g * M + r] = u[c + i].re;
    }
    __shared__ double part[kStateBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kStateBlock) acc += u[c + i].re;
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kStateBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[g] += part[0];
}

// Z[ch][f] = conj(U_x) V_y, or (conj(U_x) V_y + conj(U_y) V_x) / 2 for symmetric channels.
__global__ void k_stream_power(const cplx* __restrict__ U, const cplx* __restrict__ V, int64_t P_len,
                               const int32_t* __restrict__ chx, const int32_t* __restrict__ chy,
                               const int32_t* __restrict__ chsym, cplx* __restrict__ Z) {
    const int64_t f = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (f >= P_len) return;
    const int ch = blockIdx.y;
    const int x = chx[ch], y = chy[ch];
    const cplx ux = U[(int64_t)x * P_len + f], vy = V[(int64_t)y * P_len + f];
    cplx z = {ux.re * vy.re + ux.im * vy.im, ux.re * vy.im - ux.im * vy.re};
    if (chsym[ch]) {
        const cplx uy = U[(int64_t)y * P_len + f], vx = V[(int64_t)x * P_len + f];
        z.re = 0.5 * (z.re + uy.re * vx.re + uy.im * vx.im);
        z.im = 0.5 * (z.im + uy.re * vx.im - uy.im * vx.re);
    }
    Z[(int64_t)ch * P_len + f] = z;
}

// S[ch][tau] += Re(Z[ch][tau]) / P
__global__ void k_stream_accum(const cplx* __restrict__ Z, int64_t P_len, int64_t M, double* __restrict__ S) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    const int ch = blockIdx.y;
    S[(int64_t)ch * M + tau] += Z[(int64_t)ch * P_len + tau].re / (double)P_len;
}

// End of a run of N samples: C(tau) = S'(tau) / (N - tau) added to run_sum,
// where S' subtracts the run means when asked:
//   S' = S - xm sum_{t>=tau} y(t) - ym sum_{t<N-tau} x(t) + (N - tau) xm ym,
// sum_{t>=tau} y = Y - (first tau samples of y), sum_{t<N-tau} x = X - (last tau of x).
__global__ void k_stream_end(const double* __restrict__ S, int64_t M, int64_t N, int subtract,
                             const double* __restrict__ totals, const double* __restrict__ head,
                             const double* __restrict__ tail, int64_t tail_cap, int64_t tail_len,
                             const int32_t* __restrict__ chx, const int32_t* __restrict__ chy,
                             const int32_t* __restrict__ chsym, double* __restrict__ run_sum) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    const int ch = blockIdx.y;
    double v = S[(int64_t)ch * M + tau];
    if (subtract) {
        auto corr = [&](int x, int y) {
            const double xm = totals[x] / (double)N, ym = totals[y] / (double)N;
            double hy = 0.0, tx = 0.0;
            for (int64_t i = 0; i < tau; ++i) {
                hy += head[(int64_t)y * M + i];
                tx += tail[(int64_t)x * tail_cap + tail_len - 1 - i];
            }
            return -xm * (totals[y] - hy) - ym * (totals[x] - tx) + (double)(N - tau) * xm * ym;
        };
        const int x = chx[ch], y = chy[ch];
        v += chsym[ch] ? 0.5 * (corr(x, y) + corr(y, x)) : corr(x, y);
    }
    run_sum[(int64_t)ch * M + tau] += v / (double)(N - tau);
}

// acf[tau] = sum_ch w[ch] run_sum[ch][tau] / n_runs
__global__ void k_stream_combine(const double* __restrict__ run_sum, int nch, int64_t M,
                                 const double* __restrict__ w, double inv_runs, double* __restrict__ acf) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += w[ch] * run_sum[(int64_t)ch * M + tau];
    acf[tau] = s * inv_runs;
}

// ---- streaming, blocked: 4096-point transforms inside one work-group ------
// For max lags M <= kBlkMaxLag a chunk's new samples are split into blocks of
// B = kBlkN - (M - 1).  Block [s0, s1) adds the pairs whose later sample lies
// in it: with u = samples s0 - (M - 1) .. s1 - 1 (zero before the run's first
// sample) and v = (M - 1 zeros | samples s0 .. s1 - 1), both kBlkN long,
// IFFT(conj(U) V)[tau] / kBlkN = sum_s u(s) v(s + tau) for tau < M: a
// circular wrap-around would need s + tau >= kBlkN + M - 1, beyond the last
// sample of u plus the largest lag, so those lags are the linear ones.
// u and v of a signal share one complex transform (z = u + i v, then
// U(f) = (Z(f) + conj Z(-f)) / 2, V(f) = (Z(f) - conj Z(-f)) / 2i), and two
// channels share one inverse transform (both correlations are real:
// IFFT(P1 + i P2) = c1 + i c2).  Transforms run in LDS, so a block costs one
// global read of its samples and one write of its spectrum or lags.

// Element i of a transform lives at LDS index i + i / 16: the strided stores
// of the first two radix-16 passes (stride 16 and 256 elements) then fall on
// distinct banks.
__device__ __forceinline__ int blk_pad(int i) { return i + (i >> 4); }

// Unnormalised 4096-point transform of buf (padded layout) by the 256 threads
// of the work-group, in place: three radix-16 Stockham passes (half spans m =
// 1, 16, 256), each four radix-2 sub-stages with the butterflies and index
// scheme of k_fft_radix<16> (thread t holds elements t + 256 a; every thread
// reads its sixteen before any thread writes).  Twiddles exp(sign i pi K / M)
// from tw[j] = exp(2 pi i j / kBlkN), j < kBlkN / 2, at j = K kBlkN / (2 M).
__device__ __forceinline__ void blk_fft(cplx* buf, const cplx* __restrict__ tw, double sign) {
    const int t = threadIdx.x;
#pragma unroll
    for (int lm = 0; lm < 12; lm += 4) {
        const int m = 1 << lm;
        const int k = t & (m - 1), j = t >> lm;
        cplx x[16], y[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) x[a] = buf[blk_pad(t + a * (kBlkN / 16))];
        __syncthreads();
#pragma unroll
        for (int S = 1; S < 16; S <<= 1) {
            const int Ms = S * m;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                cplx w = tw[(k + c * m) * (kBlkN / (2 * Ms))];
                w.im *= sign;
#pragma unroll
                for (int a = 0; a < 16 / (2 * S); ++a) {
                    const cplx lo = x[c + S * a], hi = x[c + S * (a + 16 / (2 * S))];
                    const cplx wh = cmul(w, hi);
                    y[c + 2 * S * a] = {lo.re + wh.re, lo.im + wh.im};
                    y[c + S + 2 * S * a] = {lo.re - wh.re, lo.im - wh.im};
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i] = y[i];
        }
        const int o = j * 16 * m + k;
#pragma unroll
        for (int c = 0; c < 16; ++c) buf[blk_pad(o + c * m)] = x[c];
        __syncthreads();
    }
}

__global__ void k_blk_twiddles(cplx* __restrict__ tw) {
    const int j = blockIdx.x * kB + threadIdx.x;
    if (j >= kBlkN / 2) return;
    double sn, cs;
    sincospi((double)j / (double)(kBlkN / 2), &sn, &cs);
    tw[j] = {cs, sn};
}

// Signal g of one sample (a row of 3 or 9 components), as derive_signals.
__device__ __forceinline__ double signal_value(int kind, int g, const double* row, double nx, double ny, double nz,
                                               double ex, double ey, double ez) {
    if (kind == 0 || kind == 4) return row[g];
    const double gamma = (row[0] + row[4] + row[8]) / 3.0;
    if (kind == 1) return gamma;
    if (kind == 2) return row[g] - (g % 4 == 0 ? gamma : 0.0);
    const double n[3] = {nx, ny, nz}, e[3] = {ex, ey, ez};
    double p = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) p += n[a] * row[3 * a + b] * e[b];
    return p;
}

struct BlkChunk {
    const double* chunk;  // [n][comps]
    int64_t n;
    int comps, kind;
    double nx, ny, nz, ex, ey, ez;
    const double* carry;  // [nsig][carry_cap]: the last c samples before the chunk
    int64_t carry_cap, c;
    // sample p of the sequence (carry | chunk), 0 <= p < c + n
    __device__ __forceinline__ double at(int g, int64_t p) const {
        return p < c ? carry[(int64_t)g * carry_cap + p]
                     : signal_value(kind, g, chunk + (p - c) * comps, nx, ny, nz, ex, ey, ez);
    }
};

// grid (blocks of this launch [+ 1 state work-group], nsig), kBlkThreads lanes:
// the spectrum Z of z = u + i v of block blk0 + blockIdx.x and signal
// blockIdx.y into Zf[blockIdx.x][g]; with `state`, work-group x = nb also writes
// the run state of signal g: the new carry (last min(M - 1, c + n) samples),
// the run's first M samples and the run total.
__global__ void __launch_bounds__(kBlkThreads) __attribute__((amdgpu_waves_per_eu(2))) k_blk_forward(BlkChunk ch, int64_t M, int64_t blk0, int64_t B, int nb,
                                                             const cplx* __restrict__ tw, cplx* __restrict__ Zf,
                                                             int state, double* __restrict__ carry_new,
                                                             int64_t run_len, double* __restrict__ head,
                                                             double* __restrict__ totals) {
    __shared__ cplx buf[kBlkN + kBlkN / 16];
    const int g = blockIdx.y, nsig = gridDim.y;
    if ((int)blockIdx.x == nb) {
        if (!state) return;
        const int64_t L = ch.c + ch.n;
        const int64_t keep = L < ch.carry_cap ? L : ch.carry_cap;
        for (int64_t i = threadIdx.x; i < keep; i += kBlkThreads)
            carry_new[(int64_t)g * ch.carry_cap + i] = ch.at(g, L - keep + i);
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < ch.n; i += kBlkThreads) {
            const double v = ch.at(g, ch.c + i);
            if (run_len + i < M) head[(int64_t)g * M + run_len + i] = v;
            acc += v;
        }
        double* part = reinterpret_cast<double*>(buf);
        part[threadIdx.x] = acc;
        __syncthreads();
        for (int off = kBlkThreads / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) totals[g] += part[0];
        return;
    }
    const int64_t s0 = ch.c + (blk0 + blockIdx.x) * B;
    const int64_t s1 = s0 + B < ch.c + ch.n ? s0 + B : ch.c + ch.n;
    const int64_t base = s0 - (M - 1);
    for (int i = threadIdx.x; i < kBlkN; i += kBlkThreads) {
        const int64_t p = base + i;
        const double val = (p >= 0 && p < s1) ? ch.at(g, p) : 0.0;
        buf[blk_pad(i)] = {val, i >= M - 1 ? val : 0.0};
    }
    __syncthreads();
    blk_fft(buf, tw, -1.0);
    cplx* out = Zf + ((int64_t)blockIdx.x * nsig + g) * kBlkN;
    for (int f = threadIdx.x; f < kBlkN; f += kBlkThreads) out[f] = buf[blk_pad(f)];
}

// grid (blocks, ceil(nch / 2)): channels 2q and 2q + 1 of a block, from the
// signal spectra: P = conj(U_x) V_y (symmetric channels (conj(U_x) V_y +
// conj(U_y) V_x) / 2), one inverse transform of P1 + i P2, lags tau < M of
// both divided by kBlkN into part[block][ch].
__global__ void __launch_bounds__(kBlkThreads) __attribute__((amdgpu_waves_per_eu(2))) k_blk_inverse(const cplx* __restrict__ Zf, int nsig,
                                                             const int32_t* __restrict__ chx,
                                                             const int32_t* __restrict__ chy,
                                                             const int32_t* __restrict__ chsym, int nch, int64_t M,
                                                             const cplx* __restrict__ tw, double* __restrict__ part) {
    __shared__ cplx buf[kBlkN + kBlkN / 16];
    const int ch1 = 2 * blockIdx.y, ch2 = ch1 + 1;
    const cplx* Z = Zf + (int64_t)blockIdx.x * nsig * kBlkN;
    auto U = [&](int x, int f, int fm) {
        const cplx a = Z[(int64_t)x * kBlkN + f], b = Z[(int64_t)x * kBlkN + fm];
        return cplx{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
    };
    auto V = [&](int x, int f, int fm) {
        const cplx a = Z[(int64_t)x * kBlkN + f], b = Z[(int64_t)x * kBlkN + fm];
        return cplx{0.5 * (a.im + b.im), -0.5 * (a.re - b.re)};
    };
    auto power = [&](int q, int f, int fm) {
        const int x = chx[q], y = chy[q];
        const cplx ux = U(x, f, fm), vy = V(y, f, fm);
        cplx z = {ux.re * vy.re + ux.im * vy.im, ux.re * vy.im - ux.im * vy.re};
        if (chsym[q]) {
            const cplx uy = U(y, f, fm), vx = V(x, f, fm);
            z.re = 0.5 * (z.re + uy.re * vx.re + uy.im * vx.im);
            z.im = 0.5 * (z.im + uy.re * vx.im - uy.im * vx.re);
        }
        return z;
    };
    for (int f = threadIdx.x; f < kBlkN; f += kBlkThreads) {
        const int fm = (kBlkN - f) & (kBlkN - 1);
        const cplx p1 = power(ch1, f, fm);
        const cplx p2 = ch2 < nch ? power(ch2, f, fm) : cplx{0.0, 0.0};
        buf[blk_pad(f)] = {p1.re - p2.im, p1.im + p2.re};
    }
    __syncthreads();
    blk_fft(buf, tw, 1.0);
    const double scale = 1.0 / (double)kBlkN;
    double* o1 = part + ((int64_t)blockIdx.x * nch + ch1) * M;
    for (int64_t tau = threadIdx.x; tau < M; tau += kBlkThreads) {
        const cplx v = buf[blk_pad((int)tau)];
        o1[tau] = v.re * scale;
        if (ch2 < nch) o1[M + tau] = v.im * scale;
    }
}

// S[ch][tau] += sum over the launch's blocks, in block order, of part[block][ch][tau]
__global__ void k_blk_accum(const double* __restrict__ part, int nb, int nch, int64_t M, double* __restrict__ S) {
    const int64_t tau = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (tau >= M) return;
    const int ch = blockIdx.y;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[((int64_t)b * nch + ch) * M + tau];
    S[(int64_t)ch * M + tau] += acc;
}

__global__ void k_scale(const double* __restrict__ a, int64_t n, double f, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) out[i] = a[i] * f;
}

__global__ void k_zero(double* __restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }
inline unsigned nfft(int64_t n) { return (unsigned)((n + kFftBlock - 1) / kFftBlock); }

// Unnormalised FFTs (sign -1 forward, +1 inverse) of `batch` sequences of
// length P (a power of two) in a, ping-ponging with b: radix-16 launches while
// four passes remain, then one radix-8, radix-4 or radix-2 launch.  On return a
// holds the result.
void fft_batch(cplx*& a, cplx*& b, int64_t P, unsigned batch, double sign, hipStream_t s) {
    for (int64_t m = 1; m < P;) {
        if (16 * m <= P) {
            k_fft_radix<16><<<dim3(nfft(P / 16), batch), kFftBlock, 0, s>>>(a, b, P, m, sign);
            m *= 16;
        } else if (8 * m <= P) {
            k_fft_radix<8><<<dim3(nfft(P / 8), batch), kFftBlock, 0, s>>>(a, b, P, m, sign);
            m *= 8;
        } else if (4 * m <= P) {
            k_fft_radix<4><<<dim3(nfft(P / 4), batch), kFftBlock, 0, s>>>(a, b, P, m, sign);
            m *= 4;
        } else {
            k_fft_pass<<<dim3(nfft(P / 2), batch), kFftBlock, 0, s>>>(a, b, P, m, sign);
            m *= 2;
        }
        cplx* t = a;
        a = b;
        b = t;
    }
}

}  // namespace

size_t spectrum_workspace_bytes(const SpectrumPlan& p) {
    const int nsig = signals_per_series(p.kind);
    const size_t P = (size_t)p.fft_len;
    size_t b = 0;
    b += sizeof(double) * (size_t)p.n_series * 9;          // means
    b += 2 * sizeof(cplx) * P * p.n_series * nsig;         // X and ping-pong
    b += sizeof(double) * (size_t)(2 * p.max_lag + 2);     // cos table
    b += sizeof(double) * (size_t)p.max_lag;               // acf scratch
    return b + 1024;
}

hipError_t launch_spectrum(const SpectrumPlan& p, const double* d_series, double* d_freq, double* d_intensity,
                           double* d_acf, void* d_work, hipStream_t s) {
    const int nsig = signals_per_series(p.kind);
    const int comps = p.kind == 0 ? 3 : 9;
    const int64_t P = p.fft_len;
    char* w = (char*)d_work;
    auto take = [&](size_t bytes) {
        char* r = w;
        w += (bytes + 255) & ~(size_t)255;
        return r;
    };
    double* means = (double*)take(sizeof(double) * p.n_series * 9);
    cplx* X = (cplx*)take(sizeof(cplx) * (size_t)P * p.n_series * nsig);
    cplx* Y = (cplx*)take(sizeof(cplx) * (size_t)P * p.n_series * nsig);
    double* tab = (double*)take(sizeof(double) * (size_t)(2 * p.max_lag + 2));
    double* acf = d_acf ? d_acf : (double*)take(sizeof(double) * (size_t)p.max_lag);

    const bool sub = (p.flags & 1) != 0;
    if (sub) k_means<<<p.n_series * comps, kB, 0, s>>>(d_series, p.n_steps, comps, means);
    k_signals<<<dim3(nblk(P), p.n_series), kB, 0, s>>>(d_series, sub ? means : nullptr, p.n_steps, P, p.kind, comps,
                                                        nsig, p.n_hat[0], p.n_hat[1], p.n_hat[2], p.e_hat[0],
                                                        p.e_hat[1], p.e_hat[2], X);
    // forward FFTs of every signal
    const unsigned batch = (unsigned)(p.n_series * nsig);
    cplx* a = X;
    cplx* b = Y;
    fft_batch(a, b, P, batch, -1.0, s);
    // channel power into b (first n_series sequences), inverse FFT
    k_power<<<dim3(nblk(P), p.n_series), kB, 0, s>>>(a, P, p.kind, nsig, b);
    cplx* c = b;
    cplx* d = a;
    fft_batch(c, d, P, p.n_series, 1.0, s);
    k_acf<<<nblk(p.max_lag), kB, 0, s>>>(c, P, p.n_series, p.n_steps, p.max_lag, acf);
    k_cos_table<<<nblk(2 * p.max_lag), kB, 0, s>>>(p.max_lag, tab);
    const int omega2 = (p.kind == 0 && !(p.flags & 2)) ? 1 : 0;
    k_transform<<<dim3(nblk(p.max_lag + 1), 1), kB, 0, s>>>(acf, p.max_lag, tab, p.max_lag, p.window, omega2,
                                                            p.kind == 0 ? 0.0 : p.laser_cm1, p.dt_fs, d_freq,
                                                            d_intensity, p.max_lag + 1);
    return hipGetLastError();
}

// ---- orientation map ------------------------------------------------------

size_t raman_map_workspace_bytes(const SpectrumPlan& p, int n_orient) {
    const size_t P = (size_t)p.fft_len, M = (size_t)p.max_lag;
    size_t b = 0;
    b += sizeof(double) * (size_t)p.n_series * 9 + 256;
    b += 2 * (sizeof(cplx) * P * p.n_series * 9 + 256);  // X and ping-pong
    b += 2 * (sizeof(cplx) * P * 45 + 256);              // channel spectra and ping-pong
    b += sizeof(double) * (2 * M + 2) + 256;             // cos table
    b += sizeof(double) * 45 * M + 256;                  // channel acfs
    b += sizeof(double) * 45 * (M + 1) + 256;            // channel lineshapes
    b += sizeof(double) * (size_t)n_orient * 45 + 256;   // weights
    return b + 1024;
}

hipError_t launch_raman_map(const SpectrumPlan& p, const double* d_series, const double* h_weights, int n_orient,
                            double* d_freq, double* d_intensity, void* d_work, hipStream_t s) {
    const int64_t P = p.fft_len, M = p.max_lag;
    char* w = (char*)d_work;
    auto take = [&](size_t bytes) {
        char* r = w;
        w += (bytes + 255) & ~(size_t)255;
        return r;
    };
    double* means = (double*)take(sizeof(double) * p.n_series * 9);
    cplx* X = (cplx*)take(sizeof(cplx) * (size_t)P * p.n_series * 9);
    cplx* Y = (cplx*)take(sizeof(cplx) * (size_t)P * p.n_series * 9);
    cplx* Z1 = (cplx*)take(sizeof(cplx) * (size_t)P * 45);
    cplx* Z2 = (cplx*)take(sizeof(cplx) * (size_t)P * 45);
    double* tab = (double*)take(sizeof(double) * (size_t)(2 * M + 2));
    double* acf = (double*)take(sizeof(double) * (size_t)(45 * M));
    double* L = (double*)take(sizeof(double) * (size_t)(45 * (M + 1)));
    double* W = (double*)take(sizeof(double) * (size_t)n_orient * 45);
    hipError_t e = hipMemcpyAsync(W, h_weights, sizeof(double) * (size_t)n_orient * 45, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const bool sub = (p.flags & 1) != 0;
    if (sub) k_means<<<p.n_series * 9, kB, 0, s>>>(d_series, p.n_steps, 9, means);
    k_signals<<<dim3(nblk(P), p.n_series), kB, 0, s>>>(d_series, sub ? means : nullptr, p.n_steps, P, 4, 9, 9, 0, 0,
                                                        0, 0, 0, 0, X);
    cplx* a = X;
    cplx* b = Y;
    fft_batch(a, b, P, (unsigned)(p.n_series * 9), -1.0, s);
    k_power_sym<<<dim3(nblk(P), 45), kB, 0, s>>>(a, P, p.n_series, Z1);
    cplx* c = Z1;
    cplx* d = Z2;
    fft_batch(c, d, P, 45, 1.0, s);
    k_acf_channels<<<dim3(nblk(M), 45), kB, 0, s>>>(c, P, p.n_series, p.n_steps, M, acf);
    k_cos_table<<<nblk(2 * M), kB, 0, s>>>(M, tab);
    k_transform<<<dim3(nblk(M + 1), 45), kB, 0, s>>>(acf, M, tab, M, p.window, 0, p.laser_cm1, p.dt_fs, d_freq, L,
                                                     M + 1);
    k_contract<<<dim3(nblk(M + 1), (unsigned)n_orient), kB, 0, s>>>(L, M, W, 45, d_intensity);
    return hipGetLastError();
}

// ---- streaming ------------------------------------------------------------

size_t stream_push_workspace_bytes(int nsig, int nch, int64_t P) {
    return 2 * (sizeof(cplx) * (size_t)P * 2 * nsig + 256) + 2 * (sizeof(cplx) * (size_t)P * nch + 256) + 1024;
}

hipError_t launch_stream_push(const StreamState& st, const double* d_chunk, int64_t n, int64_t P, void* d_work,
                              hipStream_t s) {
    char* w = (char*)d_work;
    auto take = [&](size_t bytes) {
        char* r = w;
        w += (bytes + 255) & ~(size_t)255;
        return r;
    };
    cplx* UV = (cplx*)take(sizeof(cplx) * (size_t)P * 2 * st.nsig);
    cplx* UV2 = (cplx*)take(sizeof(cplx) * (size_t)P * 2 * st.nsig);
    cplx* Z1 = (cplx*)take(sizeof(cplx) * (size_t)P * st.nch);
    cplx* Z2 = (cplx*)take(sizeof(cplx) * (size_t)P * st.nch);
    cplx* U = UV;
    cplx* V = UV + (size_t)P * st.nsig;
    const int comps = st.kind == 0 ? 3 : 9;
    k_stream_build<<<nblk(P), kB, 0, s>>>(d_chunk, n, comps, st.kind, st.nsig, st.n_hat[0], st.n_hat[1],
                                          st.n_hat[2], st.e_hat[0], st.e_hat[1], st.e_hat[2], st.carry,
                                          st.carry_cap, st.carry_len, P, U, V);
    k_stream_state<<<st.nsig, kStateBlock, 0, s>>>(U, P, st.carry_len, n, st.carry_cap, st.carry_next, st.run_len, st.head,
                                          st.M, st.totals);
    cplx* a = UV;
    cplx* b = UV2;
    fft_batch(a, b, P, (unsigned)(2 * st.nsig), -1.0, s);
    k_stream_power<<<dim3(nblk(P), (unsigned)st.nch), kB, 0, s>>>(a, a + (size_t)P * st.nsig, P, st.chx, st.chy,
                                                                  st.chsym, Z1);
    cplx* c = Z1;
    cplx* d = Z2;
    fft_batch(c, d, P, (unsigned)st.nch, 1.0, s);
    k_stream_accum<<<dim3(nblk(st.M), (unsigned)st.nch), kB, 0, s>>>(c, P, st.M, st.S);
    return hipGetLastError();
}

size_t stream_blk_twiddle_bytes() { return sizeof(cplx) * (kBlkN / 2); }

hipError_t launch_stream_twiddles(void* tw, hipStream_t s) {
    k_blk_twiddles<<<nblk(kBlkN / 2), kB, 0, s>>>((cplx*)tw);
    return hipGetLastError();
}

size_t stream_blk_workspace_bytes(int nsig, int nch, int64_t M, int64_t n) {
    const int64_t B = kBlkN - (M - 1);
    const size_t nbr = (size_t)std::min<int64_t>((n + B - 1) / B, kBlkRound);
    return sizeof(cplx) * nbr * nsig * kBlkN + 256 + sizeof(double) * nbr * nch * (size_t)M + 256;
}

hipError_t launch_stream_push_blocked(const StreamState& st, const double* d_chunk, int64_t n, void* d_work,
                                      hipStream_t s) {
    const int64_t M = st.M, B = kBlkN - (M - 1);
    const int64_t nb_all = (n + B - 1) / B;
    const size_t nbr = (size_t)std::min<int64_t>(nb_all, kBlkRound);
    cplx* Zf = (cplx*)d_work;
    double* part = (double*)((char*)d_work + ((sizeof(cplx) * nbr * st.nsig * kBlkN + 255) & ~(size_t)255));
    const BlkChunk ch{d_chunk, n, st.kind == 0 ? 3 : 9, st.kind, st.n_hat[0], st.n_hat[1], st.n_hat[2],
                      st.e_hat[0], st.e_hat[1], st.e_hat[2], st.carry, st.carry_cap, st.carry_len};
    const cplx* tw = (const cplx*)st.blk_tw;
    const unsigned npair = (unsigned)((st.nch + 1) / 2);
    for (int64_t b0 = 0; b0 < nb_all; b0 += kBlkRound) {
        const int nb = (int)std::min<int64_t>(nb_all - b0, kBlkRound);
        const int state = b0 == 0 ? 1 : 0;
        k_blk_forward<<<dim3(nb + state, st.nsig), kBlkThreads, 0, s>>>(ch, M, b0, B, nb, tw, Zf, state,
                                                                         st.carry_next, st.run_len, st.head,
                                                                         st.totals);
        k_blk_inverse<<<dim3(nb, npair), kBlkThreads, 0, s>>>(Zf, st.nsig, st.chx, st.chy, st.chsym, st.nch, M, tw,
                                                               part);
        k_blk_accum<<<dim3(nblk(M), st.nch), kB, 0, s>>>(part, nb, st.nch, M, st.S);
    }
    return hipGetLastError();
}

hipError_t launch_stream_end_run(const StreamState& st, int subtract, hipStream_t s) {
    k_stream_end<<<dim3(nblk(st.M), (unsigned)st.nch), kB, 0, s>>>(st.S, st.M, st.run_len, subtract, st.totals,
                                                                   st.head, st.carry, st.carry_cap, st.carry_len,
                                                                   st.chx, st.chy, st.chsym, st.run_sum);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_zero<<<nblk(n), kB, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_stream_spectrum(const StreamState& st, double dt_fs, int window, int omega2, double laser_cm1,
                                  double* d_tab, double* d_acf, double* d_freq, double* d_intensity, hipStream_t s) {
    const int64_t M = st.M;
    k_stream_combine<<<nblk(M), kB, 0, s>>>(st.run_sum, st.nch, M, st.chw, 1.0 / (double)st.n_runs, d_acf);
    k_cos_table<<<nblk(2 * M), kB, 0, s>>>(M, d_tab);
    k_transform<<<dim3(nblk(M + 1), 1), kB, 0, s>>>(d_acf, M, d_tab, M, window, omega2, laser_cm1, dt_fs, d_freq,
                                                    d_intensity, M + 1);
    return hipGetLastError();
}

hipError_t launch_stream_map(const StreamState& st, double dt_fs, int window, double laser_cm1, const double* d_w,
                             int n_orient, double* d_tab, double* d_acf, double* d_L, double* d_freq,
                             double* d_intensity, hipStream_t s) {
    const int64_t M = st.M;
    k_scale<<<nblk((int64_t)st.nch * M), kB, 0, s>>>(st.run_sum, (int64_t)st.nch * M, 1.0 / (double)st.n_runs,
                                                     d_acf);
    k_cos_table<<<nblk(2 * M), kB, 0, s>>>(M, d_tab);
    k_transform<<<dim3(nblk(M + 1), (unsigned)st.nch), kB, 0, s>>>(d_acf, M, d_tab, M, window, 0, laser_cm1, dt_fs,
                                                                   d_freq, d_L, M + 1);
    k_contract<<<dim3(nblk(M + 1), (unsigned)n_orient), kB, 0, s>>>(d_L, M, d_w, st.nch, d_intensity);
    return hipGetLastError();
}

}  // namespace tnep
