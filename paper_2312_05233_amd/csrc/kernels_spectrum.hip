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
// The one-sided cosine transform with the lag window,
//   S(w_k) = dt/(2 pi) [w(0) C(0) + 2 sum_{tau=1}^{M-1} w(tau) C(tau) cos(pi k tau / M)],
// is summed directly with an exact integer phase index into a cosine table;
// IR spectra carry the classical w^2 prefactor (Eq. ir-intensity).
#include "internal.h"

namespace tnep {

namespace {

constexpr int kB = 256;

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

int signals_per_series(int kind) {
    switch (kind) {
        case 0: return 3;   // mu_x, mu_y, mu_z
        case 1: return 1;   // gamma
        case 2: return 9;   // beta_ab
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
    const int64_t tid = (int64_t)blockIdx.x * kB + threadIdx.x;
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

// S_k for k = 0..M; one thread per k.  Phase index (k tau) mod 2M kept exact.
__global__ void k_transform(const double* __restrict__ acf, const double* __restrict__ tab, int64_t M, int window,
                            int omega2, double dt_fs, double* __restrict__ freq, double* __restrict__ intensity) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k > M) return;
    const int64_t twoM = 2 * M;
    const int64_t step = k % twoM;
    int64_t idx = step;  // (k * tau) mod 2M for tau = 1
    double s = acf[0];   // w(0) = 1
    for (int64_t tau = 1; tau < M; ++tau) {
        const double w = window == 0 ? 0.5 * (1.0 + tab[tau]) : 1.0;  // tab[tau] = cos(pi tau / M)
        s += 2.0 * w * acf[tau] * tab[idx];
        idx += step;
        if (idx >= twoM) idx -= twoM;
    }
    const double pi = 3.14159265358979323846;
    s *= dt_fs / (2.0 * pi);
    const double omega = pi * (double)k / ((double)M * dt_fs);
    if (omega2) s *= omega * omega;
    intensity[k] = s;
    freq[k] = (double)k / (2.0 * (double)M * dt_fs * 2.99792458e-5);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

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
    for (int64_t m = 1; m < P; m <<= 1) {
        k_fft_pass<<<dim3(nblk(P / 2), batch), kB, 0, s>>>(a, b, P, m, -1.0);
        cplx* t = a;
        a = b;
        b = t;
    }
    // channel power into b (first n_series sequences), inverse FFT
    k_power<<<dim3(nblk(P), p.n_series), kB, 0, s>>>(a, P, p.kind, nsig, b);
    cplx* c = b;
    cplx* d = a;
    for (int64_t m = 1; m < P; m <<= 1) {
        k_fft_pass<<<dim3(nblk(P / 2), p.n_series), kB, 0, s>>>(c, d, P, m, 1.0);
        cplx* t = c;
        c = d;
        d = t;
    }
    k_acf<<<nblk(p.max_lag), kB, 0, s>>>(c, P, p.n_series, p.n_steps, p.max_lag, acf);
    k_cos_table<<<nblk(2 * p.max_lag), kB, 0, s>>>(p.max_lag, tab);
    const int omega2 = (p.kind == 0 && !(p.flags & 2)) ? 1 : 0;
    k_transform<<<nblk(p.max_lag + 1), kB, 0, s>>>(acf, tab, p.max_lag, p.window, omega2, p.dt_fs, d_freq,
                                                   d_intensity);
    return hipGetLastError();
}

}  // namespace tnep
