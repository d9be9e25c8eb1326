// C ABI of the orientation-resolved Raman map and of the streaming
// correlation accumulators (Sec. 2.6 The IR intensity, Sec. 2.7 The Raman
// intensity; kernels in kernels_spectrum.hip).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace tnep;

namespace {

// Weights of the 45 symmetric channels for one polarisation pair:
// s = n^T alpha e = sum_P v_P alpha_P with v = n (x) e, and
// <s s> = sum_{P<=Q} (2 - [P==Q]) v_P v_Q (C_PQ + C_QP) / 2.
void map_weights(const double* n, const double* e, double* w) {
    double v[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) v[3 * a + b] = n[a] * e[b];
    int q = 0;
    for (int P = 0; P < 9; ++P)
        for (int Q = P; Q < 9; ++Q) w[q++] = (P == Q ? 1.0 : 2.0) * v[P] * v[Q];
}

int64_t fft_len_for(int64_t n) {
    int64_t P = 1;
    while (P < n) P <<= 1;
    return P;
}

}  // namespace

extern "C" int tnep_raman_map(tnep_ctx* ctx, const tnep_spectrum_args* a, int32_t n_orient, const double* n_hat,
                              const double* e_hat, double* freq_cm1, double* intensity) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!a || !freq_cm1 || !intensity || !n_hat || !e_hat) return c->fail(TNEP_E_INVALID, "NULL argument");
    if (n_orient < 1 || n_orient > 65535) return c->fail(TNEP_E_INVALID, "need 1 <= n_orient <= 65535");
    if (a->n_series < 1 || a->n_steps < 2 || !a->series) return c->fail(TNEP_E_INVALID, "empty series");
    if (a->max_lag < 1 || a->max_lag > a->n_steps) return c->fail(TNEP_E_INVALID, "need 1 <= max_lag <= n_steps");
    if (!(a->dt_fs > 0) || !std::isfinite(a->dt_fs)) return c->fail(TNEP_E_INVALID, "dt_fs must be positive");
    if (a->window != TNEP_WIN_HANN && a->window != TNEP_WIN_NONE) return c->fail(TNEP_E_INVALID, "bad window");
    if (a->location != TNEP_HOST && a->location != TNEP_DEVICE) return c->fail(TNEP_E_INVALID, "bad location");
    if (a->n_steps > ((int64_t)1 << 26)) return c->fail(TNEP_E_INVALID, "n_steps above 2^26");
    if (!(a->laser_cm1 >= 0) || !std::isfinite(a->laser_cm1)) return c->fail(TNEP_E_INVALID, "bad laser_cm1");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    std::vector<double> w((size_t)n_orient * 45);
    for (int o = 0; o < n_orient; ++o) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(n_hat[3 * o + k]) || !std::isfinite(e_hat[3 * o + k]))
                return c->fail(TNEP_E_INVALID, "non-finite polarisation vector %d", o);
        map_weights(n_hat + 3 * o, e_hat + 3 * o, w.data() + (size_t)o * 45);
    }
    SpectrumPlan p{};
    p.kind = 4;
    p.window = a->window;
    p.flags = a->flags;
    p.n_series = a->n_series;
    p.n_steps = a->n_steps;
    p.max_lag = a->max_lag;
    p.dt_fs = a->dt_fs;
    p.laser_cm1 = a->laser_cm1;
    p.fft_len = fft_len_for(2 * a->n_steps);
    const size_t M = (size_t)a->max_lag;
    const size_t series_bytes = sizeof(double) * (size_t)a->n_series * a->n_steps * 9;
    int e;
    if ((e = c->reserve(c->spec_work, raman_map_workspace_bytes(p, n_orient)))) return e;
    const double* d_series = a->series;
    double *d_freq = freq_cm1, *d_int = intensity;
    if (a->location == TNEP_HOST) {
        if ((e = c->reserve(c->spec_series, series_bytes))) return e;
        if ((e = c->reserve(c->spec_out, sizeof(double) * ((M + 1) * (1 + (size_t)n_orient))))) return e;
        HIP_CHECK_RET(c, hipMemcpyAsync(c->spec_series.p, a->series, series_bytes, hipMemcpyHostToDevice, c->stream));
        d_series = (const double*)c->spec_series.p;
        d_freq = (double*)c->spec_out.p;
        d_int = d_freq + (M + 1);
    }
    const int tr = c->timer_begin(TNEP_KERNEL_SPECTRUM);
    HIP_CHECK_RET(c, launch_raman_map(p, d_series, w.data(), n_orient, d_freq, d_int, c->spec_work.p, c->stream));
    c->timer_end(tr);
    if (a->location == TNEP_HOST) {
        HIP_CHECK_RET(c, hipMemcpyAsync(freq_cm1, d_freq, sizeof(double) * (M + 1), hipMemcpyDeviceToHost, c->stream));
        HIP_CHECK_RET(c, hipMemcpyAsync(intensity, d_int, sizeof(double) * (M + 1) * n_orient, hipMemcpyDeviceToHost,
                                        c->stream));
    }
    // the weights are read from pageable host memory by the copy above: wait here
    HIP_CHECK_RET(c, hipStreamSynchronize(c->stream));
    c->timer_flush();
    return TNEP_OK;
}

// ---------------------------------------------------------------------------
// streaming accumulators

struct tnep_acf_stream {
    Ctx* ctx = nullptr;
    int flags = 0;
    StreamState st{};
    DevBuf tables, carry_a, carry_b, head, totals, S, run_sum, work, chunk, out;
    std::vector<int32_t> hx, hy, hsym;
    std::vector<double> hw;
};

namespace {

int stream_fail(tnep_acf_stream* s, int code, const char* msg) { return s->ctx->fail(code, "%s", msg); }

}  // namespace

extern "C" int tnep_acf_stream_create(tnep_ctx* ctx, int32_t kind, int64_t max_lag, int32_t flags,
                                      const double* n_hat, const double* e_hat, tnep_acf_stream** out) {
    if (!ctx || !out) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    *out = nullptr;
    if (kind < TNEP_IR || kind > TNEP_RAMAN_MAP) return c->fail(TNEP_E_INVALID, "unknown stream kind");
    if (max_lag < 1 || max_lag > ((int64_t)1 << 24)) return c->fail(TNEP_E_INVALID, "need 1 <= max_lag <= 2^24");
    if (kind == TNEP_RAMAN_PROJ && (!n_hat || !e_hat)) return c->fail(TNEP_E_INVALID, "projection needs n_hat, e_hat");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    tnep_acf_stream* s = new tnep_acf_stream();
    s->ctx = c;
    s->flags = flags;
    StreamState& st = s->st;
    st.kind = kind;
    st.M = max_lag;
    for (int k = 0; k < 3; ++k) {
        st.n_hat[k] = n_hat ? n_hat[k] : 0.0;
        st.e_hat[k] = e_hat ? e_hat[k] : 0.0;
    }
    switch (kind) {
        case TNEP_IR:
            st.nsig = 3;
            for (int a = 0; a < 3; ++a) {
                s->hx.push_back(a);
                s->hy.push_back(a);
                s->hsym.push_back(0);
                s->hw.push_back(1.0 / 3.0);
            }
            break;
        case TNEP_RAMAN_ANISO:
            st.nsig = 9;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    s->hx.push_back(3 * a + b);
                    s->hy.push_back(3 * b + a);
                    s->hsym.push_back(0);
                    s->hw.push_back(1.0);
                }
            break;
        case TNEP_RAMAN_MAP:
            st.nsig = 9;
            for (int P = 0; P < 9; ++P)
                for (int Q = P; Q < 9; ++Q) {
                    s->hx.push_back(P);
                    s->hy.push_back(Q);
                    s->hsym.push_back(1);
                    s->hw.push_back(0.0);
                }
            break;
        default:  // iso, projection: one signal
            st.nsig = 1;
            s->hx.push_back(0);
            s->hy.push_back(0);
            s->hsym.push_back(0);
            s->hw.push_back(1.0);
    }
    st.nch = (int)s->hx.size();
    st.carry_cap = std::max<int64_t>(1, max_lag - 1);
    const size_t nch = (size_t)st.nch, nsig = (size_t)st.nsig, M = (size_t)max_lag;
    int e = 0;
    auto fail_free = [&](int code) {
        tnep_acf_stream_free(s);
        return code;
    };
    const bool blocked = max_lag <= kBlkMaxLag;
    const size_t tab_bytes = (nch * (3 * sizeof(int32_t) + sizeof(double)) + 255) & ~(size_t)255;
    if ((e = c->reserve(s->tables, tab_bytes + (blocked ? stream_blk_twiddle_bytes() : 0) + 64)))
        return fail_free(e);
    if ((e = c->reserve(s->carry_a, sizeof(double) * nsig * st.carry_cap))) return fail_free(e);
    if ((e = c->reserve(s->carry_b, sizeof(double) * nsig * st.carry_cap))) return fail_free(e);
    if ((e = c->reserve(s->head, sizeof(double) * nsig * M))) return fail_free(e);
    if ((e = c->reserve(s->totals, sizeof(double) * nsig))) return fail_free(e);
    if ((e = c->reserve(s->S, sizeof(double) * nch * M))) return fail_free(e);
    if ((e = c->reserve(s->run_sum, sizeof(double) * nch * M))) return fail_free(e);
    std::vector<char> tab(nch * (3 * sizeof(int32_t) + sizeof(double)));
    char* q = tab.data();
    std::memcpy(q, s->hw.data(), nch * sizeof(double));
    std::memcpy(q + nch * 8, s->hx.data(), nch * 4);
    std::memcpy(q + nch * 12, s->hy.data(), nch * 4);
    std::memcpy(q + nch * 16, s->hsym.data(), nch * 4);
    if (hipMemcpy(s->tables.p, tab.data(), tab.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail_free(c->fail(TNEP_E_HIP, "stream table upload failed"));
    char* d = (char*)s->tables.p;
    st.chw = (const double*)d;
    st.chx = (const int32_t*)(d + nch * 8);
    st.chy = (const int32_t*)(d + nch * 12);
    st.chsym = (const int32_t*)(d + nch * 16);
    st.blk_tw = blocked ? (const void*)(d + tab_bytes) : nullptr;
    st.carry = (double*)s->carry_a.p;
    st.carry_next = (double*)s->carry_b.p;
    st.head = (double*)s->head.p;
    st.totals = (double*)s->totals.p;
    st.S = (double*)s->S.p;
    st.run_sum = (double*)s->run_sum.p;
    st.carry_len = 0;
    st.run_len = 0;
    st.n_runs = 0;
    hipError_t he = blocked ? launch_stream_twiddles(d + tab_bytes, c->stream) : hipSuccess;
    if (he == hipSuccess) he = launch_fill_zero(st.S, (int64_t)(nch * M), c->stream);
    if (he == hipSuccess) he = launch_fill_zero(st.run_sum, (int64_t)(nch * M), c->stream);
    if (he == hipSuccess) he = launch_fill_zero(st.totals, (int64_t)nsig, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return fail_free(c->fail(TNEP_E_HIP, "stream initialisation failed"));
    *out = s;
    return TNEP_OK;
}

extern "C" int tnep_acf_stream_push(tnep_acf_stream* s, const double* samples, int64_t n_samples, int32_t location) {
    if (!s) return TNEP_E_INVALID;
    Ctx* c = s->ctx;
    if (n_samples < 0 || (n_samples > 0 && !samples)) return stream_fail(s, TNEP_E_INVALID, "bad samples");
    if (location != TNEP_HOST && location != TNEP_DEVICE) return stream_fail(s, TNEP_E_INVALID, "bad location");
    if (n_samples == 0) return TNEP_OK;
    if (n_samples > ((int64_t)1 << 26)) return stream_fail(s, TNEP_E_INVALID, "chunk above 2^26 samples");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    StreamState& st = s->st;
    const int comps = st.kind == TNEP_IR ? 3 : 9;
    // max lags up to kBlkMaxLag: blocks of kBlkN-point transforms in LDS;
    // longer lags: one zero-padded transform of the whole chunk
    const bool blocked = st.blk_tw != nullptr;
    const int64_t P = blocked ? 0 : fft_len_for(st.carry_len + n_samples + st.M);
    int e;
    if ((e = c->reserve(s->work, blocked ? stream_blk_workspace_bytes(st.nsig, st.nch, st.M, n_samples)
                                         : stream_push_workspace_bytes(st.nsig, st.nch, P))))
        return e;
    const double* d_chunk = samples;
    if (location == TNEP_HOST) {
        const size_t bytes = sizeof(double) * (size_t)n_samples * comps;
        if ((e = c->reserve(s->chunk, bytes))) return e;
        HIP_CHECK_RET(c, hipMemcpyAsync(s->chunk.p, samples, bytes, hipMemcpyHostToDevice, c->stream));
        d_chunk = (const double*)s->chunk.p;
    }
    const int tr = c->timer_begin(TNEP_KERNEL_SPECTRUM);
    HIP_CHECK_RET(c, blocked ? launch_stream_push_blocked(st, d_chunk, n_samples, s->work.p, c->stream)
                             : launch_stream_push(st, d_chunk, n_samples, P, s->work.p, c->stream));
    c->timer_end(tr);
    // device chunks: no wait, so that consecutive pushes queue back to back
    // (the run state is device-resident and the kernels run in stream order)
    if (location == TNEP_HOST || c->timing) {
        HIP_CHECK_RET(c, hipStreamSynchronize(c->stream));
        c->timer_flush();
    }
    std::swap(st.carry, st.carry_next);
    st.carry_len = std::min(st.carry_cap, st.carry_len + n_samples);
    st.run_len += n_samples;
    return TNEP_OK;
}

extern "C" int tnep_acf_stream_end_run(tnep_acf_stream* s) {
    if (!s) return TNEP_E_INVALID;
    Ctx* c = s->ctx;
    StreamState& st = s->st;
    if (st.run_len < st.M || st.run_len < 2)
        return stream_fail(s, TNEP_E_INVALID, "a run needs at least max_lag (and 2) samples");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    HIP_CHECK_RET(c, launch_stream_end_run(st, (s->flags & TNEP_SUBTRACT_MEAN) ? 1 : 0, c->stream));
    HIP_CHECK_RET(c, launch_fill_zero(st.S, (int64_t)st.nch * st.M, c->stream));
    HIP_CHECK_RET(c, launch_fill_zero(st.totals, st.nsig, c->stream));
    HIP_CHECK_RET(c, hipStreamSynchronize(c->stream));
    st.n_runs += 1;
    st.run_len = 0;
    st.carry_len = 0;
    return TNEP_OK;
}

static int stream_output(tnep_acf_stream* s, double dt_fs, int32_t window, double laser_cm1, int n_orient,
                         const double* n_hat, const double* e_hat, double* freq_cm1, double* intensity, double* acf) {
    Ctx* c = s->ctx;
    StreamState& st = s->st;
    if (!freq_cm1 || !intensity) return stream_fail(s, TNEP_E_INVALID, "NULL output");
    if (st.n_runs < 1) return stream_fail(s, TNEP_E_INVALID, "no finished run (call tnep_acf_stream_end_run)");
    if (!(dt_fs > 0) || !std::isfinite(dt_fs)) return stream_fail(s, TNEP_E_INVALID, "dt_fs must be positive");
    if (window != TNEP_WIN_HANN && window != TNEP_WIN_NONE) return stream_fail(s, TNEP_E_INVALID, "bad window");
    if (!(laser_cm1 >= 0) || !std::isfinite(laser_cm1)) return stream_fail(s, TNEP_E_INVALID, "bad laser_cm1");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    const size_t M = (size_t)st.M;
    const size_t no = (size_t)std::max(n_orient, 1);
    std::vector<double> w;
    if (n_orient > 0) {
        w.resize(no * 45);
        for (int o = 0; o < n_orient; ++o) map_weights(n_hat + 3 * o, e_hat + 3 * o, w.data() + (size_t)o * 45);
    }
    // device scratch: table, acf [nch][M], L [nch][M+1], weights, freq, intensity
    const size_t doubles = (2 * M + 2) + (size_t)st.nch * M + (size_t)st.nch * (M + 1) + w.size() + (M + 1) +
                           no * (M + 1) + 64;
    int e;
    if ((e = c->reserve(s->out, sizeof(double) * doubles))) return e;
    double* tab = (double*)s->out.p;
    double* d_acf = tab + (2 * M + 2);
    double* d_L = d_acf + (size_t)st.nch * M;
    double* d_w = d_L + (size_t)st.nch * (M + 1);
    double* d_freq = d_w + w.size();
    double* d_int = d_freq + (M + 1);
    if (!w.empty())
        HIP_CHECK_RET(c, hipMemcpyAsync(d_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, c->stream));
    if (n_orient > 0) {
        HIP_CHECK_RET(c, launch_stream_map(st, dt_fs, window, laser_cm1, d_w, n_orient, tab, d_acf, d_L, d_freq, d_int,
                                           c->stream));
    } else {
        const int omega2 = (st.kind == TNEP_IR && !(s->flags & TNEP_NO_OMEGA2)) ? 1 : 0;
        HIP_CHECK_RET(c, launch_stream_spectrum(st, dt_fs, window, omega2, st.kind == TNEP_IR ? 0.0 : laser_cm1,
                                                tab, d_acf, d_freq, d_int, c->stream));
    }
    HIP_CHECK_RET(c, hipMemcpyAsync(freq_cm1, d_freq, sizeof(double) * (M + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK_RET(c, hipMemcpyAsync(intensity, d_int, sizeof(double) * (M + 1) * no, hipMemcpyDeviceToHost,
                                    c->stream));
    if (acf && n_orient == 0)
        HIP_CHECK_RET(c, hipMemcpyAsync(acf, d_acf, sizeof(double) * M, hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK_RET(c, hipStreamSynchronize(c->stream));
    return TNEP_OK;
}

extern "C" int tnep_acf_stream_spectrum(tnep_acf_stream* s, double dt_fs, int32_t window, double laser_cm1,
                                        double* freq_cm1, double* intensity, double* acf) {
    if (!s) return TNEP_E_INVALID;
    if (s->st.kind == TNEP_RAMAN_MAP) return stream_fail(s, TNEP_E_INVALID, "map streams: tnep_acf_stream_raman_map");
    return stream_output(s, dt_fs, window, laser_cm1, 0, nullptr, nullptr, freq_cm1, intensity, acf);
}

extern "C" int tnep_acf_stream_raman_map(tnep_acf_stream* s, double dt_fs, int32_t window, double laser_cm1,
                                         int32_t n_orient, const double* n_hat, const double* e_hat,
                                         double* freq_cm1, double* intensity) {
    if (!s) return TNEP_E_INVALID;
    if (s->st.kind != TNEP_RAMAN_MAP) return stream_fail(s, TNEP_E_INVALID, "not a map stream");
    if (n_orient < 1 || n_orient > 65535 || !n_hat || !e_hat)
        return stream_fail(s, TNEP_E_INVALID, "need 1 <= n_orient <= 65535 and polarisation vectors");
    for (int k = 0; k < 3 * n_orient; ++k)
        if (!std::isfinite(n_hat[k]) || !std::isfinite(e_hat[k]))
            return stream_fail(s, TNEP_E_INVALID, "non-finite polarisation vector");
    return stream_output(s, dt_fs, window, laser_cm1, n_orient, n_hat, e_hat, freq_cm1, intensity, nullptr);
}

extern "C" void tnep_acf_stream_free(tnep_acf_stream* s) {
    if (!s) return;
    Ctx* c = s->ctx;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : {&s->tables, &s->carry_a, &s->carry_b, &s->head, &s->totals, &s->S, &s->run_sum, &s->work,
                      &s->chunk, &s->out})
        c->release(*b);
    delete s;
}
