// C ABI of libtnep (declared in include/tnep.h): contexts, resident models,
// batched evaluation of the TNEP dipole (Sec. 2.2, Eq. mu) and
// polarizability / susceptibility (Sec. 2.3, Eq. polarizability-model), and
// spectra (Sec. 2.6 The IR intensity, Sec. 2.7 The Raman intensity).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tnep.h"
#include "internal.h"
#include "runtime.h"

using namespace tnep;

// ---------------------------------------------------------------------------
// error plumbing

static thread_local std::string g_create_error;

void tnep::set_create_error(const std::string& msg) { g_create_error = msg; }

int tnep::Ctx::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

#define HIP_TRY HIP_CHECK_RET

// ---------------------------------------------------------------------------
// device buffers

int tnep::Ctx::reserve(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes) return TNEP_OK;
    const size_t want = std::max(bytes, b.bytes + b.bytes / 4);
    if (in_use - b.bytes + want > budget)
        return fail(TNEP_E_BUDGET, "device budget exceeded: need %zu more bytes (budget %llu, in use %llu)",
                    want - b.bytes, (unsigned long long)budget, (unsigned long long)in_use);
    if (b.p) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(b.p);
        in_use -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    ++epoch;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) return fail(TNEP_E_HIP, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    b.bytes = want;
    in_use += want;
    peak = std::max(peak, in_use);
    return TNEP_OK;
}

void tnep::Ctx::release(DevBuf& b) {
    if (b.p) {
        (void)hipFree(b.p);
        in_use -= b.bytes;
        ++epoch;
    }
    b.p = nullptr;
    b.bytes = 0;
}

int tnep::Ctx::timer_begin(int which) {
    if (!timing) return -1;
    hipEvent_t ev[2];
    for (int k = 0; k < 2; ++k) {
        if (event_pool.empty()) {
            if (hipEventCreate(&ev[k]) != hipSuccess) return -1;
        } else {
            ev[k] = event_pool.back();
            event_pool.pop_back();
        }
    }
    (void)hipEventRecord(ev[0], stream);
    pending.push_back({ev[0], ev[1], which});
    return (int)pending.size() - 1;
}

void tnep::Ctx::timer_end(int idx) {
    if (idx < 0) return;
    (void)hipEventRecord(pending[idx].b, stream);
}

void tnep::Ctx::timer_flush() {
    for (Range& r : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            kernel_ms[r.which] += ms;
            kernel_launches[r.which] += 1;
        }
        event_pool.push_back(r.a);
        event_pool.push_back(r.b);
    }
    pending.clear();
    if (timing && counters.p) {
        unsigned long long h[3];
        if (hipMemcpy(h, counters.p, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess)
            for (int k = 0; k < 3; ++k) pair_counts[k] = h[k];
    }
}

void tnep::Ctx::drop_graphs() {
    if (graphs.empty()) return;
    (void)hipStreamSynchronize(stream);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
}

tnep::Ctx::~Ctx() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    for (hipEvent_t ev : event_pool) (void)hipEventDestroy(ev);
    for (DevBuf* b : all_buffers()) release(*b);
    if (h_flags) (void)hipHostFree(h_flags);
    if (meta_host) (void)hipHostFree(meta_host);
    if (rb_host) (void)hipHostFree(rb_host);
    if (in_host) (void)hipHostFree(in_host);
    if (pop_host) (void)hipHostFree(pop_host);
    if (side) (void)hipStreamSynchronize(side);
    if (copy_stream) (void)hipStreamSynchronize(copy_stream);
    for (int h = 0; h < 2; ++h) {
        if (in_copied[h]) (void)hipEventDestroy(in_copied[h]);
        if (in_used[h]) (void)hipEventDestroy(in_used[h]);
    }
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (side) (void)hipStreamDestroy(side);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ---------------------------------------------------------------------------
// context

extern "C" int tnep_ctx_create(int device, void* hip_stream, uint64_t mem_budget_bytes, tnep_ctx** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return TNEP_E_INVALID;
    }
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        g_create_error = "no such HIP device";
        return TNEP_E_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return TNEP_E_HIP;
    }
    Ctx* c = new Ctx();
    c->device = device;
    c->budget = mem_budget_bytes ? mem_budget_bytes : (uint64_t)32 << 30;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            g_create_error = "hipStreamCreate failed";
            return TNEP_E_HIP;
        }
        c->own_stream = true;
    }
    if (hipHostMalloc((void**)&c->h_flags, sizeof(int32_t) * 32, hipHostMallocDefault) != hipSuccess) {
        delete c;
        g_create_error = "hipHostMalloc failed";
        return TNEP_E_HIP;
    }
    // device address of this device's fixed workspace (tnep_spectrum_noalloc)
    std::string err;
    if (noalloc_scratch_setup(device, err) != TNEP_OK) {
        delete c;
        g_create_error = err;
        return TNEP_E_HIP;
    }
    *out = reinterpret_cast<tnep_ctx*>(c);
    return TNEP_OK;
}

extern "C" void tnep_ctx_destroy(tnep_ctx* ctx) {
    if (!ctx) return;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    server_shutdown(c);
    (void)hipSetDevice(c->device);
    delete c;
}

extern "C" const char* tnep_last_error(const tnep_ctx* ctx) {
    if (!ctx) return g_create_error.c_str();
    return reinterpret_cast<const Ctx*>(ctx)->err.c_str();
}

extern "C" const char* tnep_autotune_report(const tnep_ctx* ctx) {
    return ctx ? reinterpret_cast<const Ctx*>(ctx)->tune_log.c_str() : "";
}

extern "C" uint64_t tnep_ctx_memory_in_use(const tnep_ctx* ctx) {
    return ctx ? reinterpret_cast<const Ctx*>(ctx)->in_use : 0;
}

extern "C" int tnep_ctx_kernel_time(const tnep_ctx* ctx, int32_t which, double* total_ms, uint64_t* launches) {
    if (!ctx || which < 0 || which > TNEP_KERNEL_PES_FORCES) return TNEP_E_INVALID;
    const Ctx* c = reinterpret_cast<const Ctx*>(ctx);
    if (total_ms) *total_ms = c->kernel_ms[which];
    if (launches) *launches = c->kernel_launches[which];
    return TNEP_OK;
}

extern "C" int tnep_ctx_pair_counts(const tnep_ctx* ctx, uint64_t* atoms, uint64_t* radial_pairs,
                                    uint64_t* angular_pairs) {
    if (!ctx) return TNEP_E_INVALID;
    const Ctx* c = reinterpret_cast<const Ctx*>(ctx);
    if (atoms) *atoms = c->pair_counts[0];
    if (radial_pairs) *radial_pairs = c->pair_counts[1];
    if (angular_pairs) *angular_pairs = c->pair_counts[2];
    return TNEP_OK;
}

extern "C" int tnep_ctx_reuse_fallbacks(const tnep_ctx* ctx, uint64_t* count) {
    if (!ctx || !count) return TNEP_E_INVALID;
    *count = reinterpret_cast<const Ctx*>(ctx)->reuse_fallbacks;
    return TNEP_OK;
}

extern "C" int tnep_ctx_graph_counts(const tnep_ctx* ctx, uint64_t* captures, uint64_t* launches) {
    if (!ctx) return TNEP_E_INVALID;
    const Ctx* c = reinterpret_cast<const Ctx*>(ctx);
    uint64_t nc = c->graph_captures, nl = c->graph_launches;
    if (c->server) server_graph_counts(c, nc, nl);
    if (captures) *captures = nc;
    if (launches) *launches = nl;
    return TNEP_OK;
}

extern "C" int tnep_ctx_reset_timing(tnep_ctx* ctx) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    (void)hipStreamSynchronize(c->stream);
    c->timer_flush();
    for (int k = 0; k < 8; ++k) {
        c->kernel_ms[k] = 0;
        c->kernel_launches[k] = 0;
    }
    for (int k = 0; k < 3; ++k) c->pair_counts[k] = 0;
    if (c->counters.p) {
        if (hipMemset(c->counters.p, 0, 64) != hipSuccess) return c->fail(TNEP_E_HIP, "counter reset failed");
    }
    return TNEP_OK;
}

extern "C" int tnep_set_option(tnep_ctx* ctx, int32_t key, int64_t value) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    switch (key) {
        case TNEP_OPT_MLP:
            if (value < TNEP_MLP_FP32_VALU || value > TNEP_MLP_BF16X3_MFMA)
                return c->fail(TNEP_E_INVALID, "unknown MLP mode %lld", (long long)value);
            c->launch.mlp_mode = (int)value;
            return TNEP_OK;
        case TNEP_OPT_ATOMS_PER_BLOCK:
            if (value != 64 && value != 128 && value != 256)
                return c->fail(TNEP_E_INVALID, "atoms per block must be 64, 128 or 256");
            c->launch.atoms_per_block = (int)value;
            return TNEP_OK;
        case TNEP_OPT_NEIGH_BLOCK:
            if (value != 64 && value != 128 && value != 256)
                return c->fail(TNEP_E_INVALID, "neighbour work-group size must be 64, 128 or 256");
            c->launch.neigh_block = (int)value;
            return TNEP_OK;
        case TNEP_OPT_AUTOTUNE:
            c->autotune = value != 0;
            return TNEP_OK;
        case TNEP_OPT_DETERMINISTIC:
            if (value == 0) return c->fail(TNEP_E_INVALID, "only the deterministic reduction is implemented");
            return TNEP_OK;
        case TNEP_OPT_TIMING:
            c->timing = value != 0;
            return TNEP_OK;
        case TNEP_OPT_GRAPHS:
            if (value != 0 && !c->stream) return c->fail(TNEP_E_INVALID, "graphs need a non-null stream");
            c->use_graphs = value != 0;
            if (!c->use_graphs) c->drop_graphs();
            return TNEP_OK;
        case TNEP_OPT_TRAJECTORY_WINDOW:
            if (value < 0 || value > 4096) return c->fail(TNEP_E_INVALID, "trajectory window must be 0..4096");
            c->traj_window = (int)value;
            return TNEP_OK;
        case TNEP_OPT_SKIN_MA:
            if (value < 1 || value > 5000) return c->fail(TNEP_E_INVALID, "skin must be 1..5000 mA");
            c->skin = (double)value * 1e-3;
            return TNEP_OK;
        case TNEP_OPT_PAIR_PARALLEL:
            if (value != 0 && value != 1) return c->fail(TNEP_E_INVALID, "pair-parallel layout must be 0 or 1");
            c->launch.pair_parallel = (int)value;
            return TNEP_OK;
        case TNEP_OPT_MAX_BATCH_ATOMS:
            if (value < 1) return c->fail(TNEP_E_INVALID, "max batch atoms must be positive");
            c->max_batch_atoms = value;
            return TNEP_OK;
        default:
            return c->fail(TNEP_E_INVALID, "unknown option %d", key);
    }
}

// ---------------------------------------------------------------------------
// models

// Model validation error: the message goes to the context when there is one
// (staging on worker threads passes none).
#define model_error(c, ...) ((c) ? (c)->fail(TNEP_E_MODEL, __VA_ARGS__) : TNEP_E_MODEL)

int tnep::stage_model(Ctx* c, const tnep_model_desc* d, std::vector<float>& h, Model& m, ModelLayout& lay) {
    if (d->kind != TNEP_KIND_DIPOLE && d->kind != TNEP_KIND_POLARIZABILITY && d->kind != TNEP_KIND_PES)
        return model_error(c, "unknown model kind %d", d->kind);
    if (d->n_species < 1 || d->n_species > 8) return model_error(c, "n_species must be 1..8");
    if (!(d->rc_radial > 0) || !(d->rc_angular > 0) || d->rc_angular > d->rc_radial)
        return model_error(c, "need 0 < rc_angular <= rc_radial");
    if (d->l_max != 4) return model_error(c, "only l_max = 4 is compiled");
    if (d->n_hidden < 1 || d->n_hidden > 128) return model_error(c, "n_hidden must be 1..128");
    Shape sh{d->n_max_radial + 1, d->n_max_angular + 1, d->basis_radial + 1, d->basis_angular + 1,
             d->four_body ? 1 : 0, d->kind, d->five_body ? 1 : 0};
    if (!eval_shape_supported(sh))
        return model_error(c, "descriptor shape (nR=%d, nA=%d, KR=%d, KA=%d, 4b=%d, 5b=%d) is not compiled",
                           d->n_max_radial, d->n_max_angular, d->basis_radial, d->basis_angular, d->four_body,
                           d->five_body);
    if (!d->c_radial || !d->c_angular || !d->q_scaler || !d->w0[0] || !d->b0[0] || !d->w1[0])
        return model_error(c, "missing parameter arrays");
    const int heads = d->kind == TNEP_KIND_POLARIZABILITY ? 2 : 1;
    if (heads == 2 && (!d->w0[1] || !d->b0[1] || !d->w1[1]))
        return model_error(c, "polarizability model needs the scalar head");
    const bool per_species = d->per_species != 0;
    for (int hd = 0; hd < heads && per_species; ++hd)
        if (!d->b1_species[hd]) return model_error(c, "per-species model needs b1_species");
    const int T = d->n_species, H = d->n_hidden;
    const size_t NS = per_species ? (size_t)T : 1;  // networks per head
    const int D = sh.nr + 4 * sh.na + (sh.four_body ? sh.na : 0) + (sh.five_body ? sh.na : 0);
    const size_t ncr = (size_t)T * T * sh.nr * sh.kr, nca = (size_t)T * T * sh.na * sh.ka;

    // host staging in FP32, fixed layout, appended to h at a 256-byte boundary
    while (h.size() % 64) h.push_back(0.f);
    auto put = [&](const double* src, size_t n) {
        size_t off = h.size();
        for (size_t k = 0; k < n; ++k) h.push_back((float)src[k]);
        while (h.size() % 64) h.push_back(0.f);  // 256-byte alignment
        return off;
    };
    for (size_t k = 0; k < ncr; ++k)
        if (!std::isfinite(d->c_radial[k])) return model_error(c, "non-finite c_radial");
    size_t o_cr = put(d->c_radial, ncr);
    size_t o_ca = put(d->c_angular, nca);
    // derivative series of every angular radial function: b_k = b_{k+2} + 2 (k+1) c_{k+1}, b_0 halved
    std::vector<double> cad(nca, 0.0);
    for (size_t row = 0; row < nca / sh.ka; ++row) {
        const double* cr = d->c_angular + row * sh.ka;
        double* b = cad.data() + row * sh.ka;
        for (int k = sh.ka - 2; k >= 0; --k) b[k] = (k + 2 <= sh.ka - 2 ? b[k + 2] : 0.0) + 2.0 * (k + 1) * cr[k + 1];
        b[0] *= 0.5;
    }
    size_t o_cad = put(cad.data(), nca);
    size_t o_s = put(d->q_scaler, D);
    size_t o_w0[2] = {0, 0}, o_b0[2] = {0, 0}, o_w1[2] = {0, 0}, o_w0t[2] = {0, 0}, o_b1s[2] = {0, 0};
    for (int hd = 0; hd < heads; ++hd) {
        o_w0[hd] = put(d->w0[hd], NS * H * D);
        o_b0[hd] = put(d->b0[hd], NS * H);
        o_w1[hd] = put(d->w1[hd], NS * H);
        if (per_species) o_b1s[hd] = put(d->b1_species[hd], T);
        std::vector<double> t((size_t)D * H);
        for (int mu = 0; mu < H; ++mu)
            for (int nu = 0; nu < D; ++nu) t[(size_t)nu * H + mu] = d->w0[hd][(size_t)mu * D + nu];
        o_w0t[hd] = put(t.data(), t.size());
    }
    for (float v : h)
        if (!std::isfinite(v)) return model_error(c, "non-finite model parameter");

    // matrix-core fragments (see DevModel)
    auto rup = [](int x, int m) { return (x + m - 1) / m * m; };
    const int Hp = rup(H, 32), Dp4 = rup(D, 4), Dp16 = rup(D, 16), Dp32 = rup(D, 32);
    auto W = [&](int hd, int mu, int nu) -> double {
        return (mu < H && nu < D) ? d->w0[hd][(size_t)mu * D + nu] : 0.0;
    };
    auto bf16_bits = [](float x) -> uint16_t {  // round to nearest even
        uint32_t u;
        std::memcpy(&u, &x, 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    };
    auto bf16_value = [](uint16_t b) -> float {
        uint32_t u = (uint32_t)b << 16;
        float x;
        std::memcpy(&x, &u, 4);
        return x;
    };
    auto put_u16 = [&](const std::vector<uint16_t>& v) {
        size_t off = h.size();
        const size_t nf = (v.size() * 2 + 3) / 4;
        h.resize(off + nf, 0.f);
        std::memcpy(h.data() + off, v.data(), v.size() * 2);
        while (h.size() % 64) h.push_back(0.f);
        return off;
    };
    size_t o_f32_fwd[2] = {0, 0}, o_bf_fwd_hi[2] = {0, 0}, o_bf_fwd_lo[2] = {0, 0};
    for (int hd = 0; hd < heads; ++hd) {
        std::vector<double> f((size_t)(Hp / 16) * (Dp4 / 4) * 64);
        for (int nt = 0; nt < Hp / 16; ++nt)
            for (int ks = 0; ks < Dp4 / 4; ++ks)
                for (int l = 0; l < 64; ++l)
                    f[((size_t)nt * (Dp4 / 4) + ks) * 64 + l] = W(hd, 16 * nt + l % 16, 4 * ks + l / 16);
        o_f32_fwd[hd] = put(f.data(), f.size());
        std::vector<uint16_t> bh((size_t)(Hp / 16) * (Dp32 / 32) * 64 * 8), bl(bh.size());
        for (int nt = 0; nt < Hp / 16; ++nt)
            for (int kc = 0; kc < Dp32 / 32; ++kc)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        const float x = (float)W(hd, 16 * nt + l % 16, 32 * kc + 8 * (l / 16) + j);
                        const uint16_t hi = bf16_bits(x);
                        const size_t idx = (((size_t)nt * (Dp32 / 32) + kc) * 64 + l) * 8 + j;
                        bh[idx] = hi;
                        bl[idx] = bf16_bits(x - bf16_value(hi));
                    }
        o_bf_fwd_hi[hd] = put_u16(bh);
        o_bf_fwd_lo[hd] = put_u16(bl);
    }
    size_t o_f32_bwd, o_bf_bwd_hi, o_bf_bwd_lo;
    {
        std::vector<double> f((size_t)(Dp16 / 16) * (Hp / 4) * 64);
        for (int kt = 0; kt < Dp16 / 16; ++kt)
            for (int ns = 0; ns < Hp / 4; ++ns)
                for (int l = 0; l < 64; ++l)
                    f[((size_t)kt * (Hp / 4) + ns) * 64 + l] = W(0, 4 * ns + l / 16, 16 * kt + l % 16);
        o_f32_bwd = put(f.data(), f.size());
        std::vector<uint16_t> bh((size_t)(Dp16 / 16) * (Hp / 32) * 64 * 8), bl(bh.size());
        for (int kt = 0; kt < Dp16 / 16; ++kt)
            for (int nc = 0; nc < Hp / 32; ++nc)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        const float x = (float)W(0, 32 * nc + 8 * (l / 16) + j, 16 * kt + l % 16);
                        const uint16_t hi = bf16_bits(x);
                        const size_t idx = (((size_t)kt * (Hp / 32) + nc) * 64 + l) * 8 + j;
                        bh[idx] = hi;
                        bl[idx] = bf16_bits(x - bf16_value(hi));
                    }
        o_bf_bwd_hi = put_u16(bh);
        o_bf_bwd_lo = put_u16(bl);
    }

    static std::atomic<uint64_t> next_serial{1};
    m.serial = next_serial++;
    m.ctx = c;
    m.device = c ? c->device : 0;
    m.shape = sh;
    m.kind = d->kind;
    m.T = T;
    m.D = D;
    m.H = H;
    m.rc_radial = d->rc_radial;
    m.rc_angular = d->rc_angular;
    lay.cr = o_cr;
    lay.ca = o_ca;
    lay.cad = o_cad;
    lay.s = o_s;
    for (int hd = 0; hd < 2; ++hd) {
        const int src = hd < heads ? hd : 0;
        lay.w0[hd] = o_w0[src];
        lay.b0[hd] = o_b0[src];
        lay.w1[hd] = o_w1[src];
        lay.w0t[hd] = o_w0t[src];
        lay.b1[hd] = (float)d->b1[src];
        lay.b1s[hd] = per_species ? (int64_t)o_b1s[src] : -1;
        lay.f32_fwd[hd] = o_f32_fwd[src];
        lay.bf_fwd_hi[hd] = o_bf_fwd_hi[src];
        lay.bf_fwd_lo[hd] = o_bf_fwd_lo[src];
    }
    lay.f32_bwd = o_f32_bwd;
    lay.bf_bwd_hi = o_bf_bwd_hi;
    lay.bf_bwd_lo = o_bf_bwd_lo;
    lay.per_species = per_species;
    return TNEP_OK;
}

void tnep::bind_model(Model& m, const float* base, const ModelLayout& lay) {
    DevModel& dm = m.dm;
    dm.c_radial = base + lay.cr;
    dm.c_angular = base + lay.ca;
    dm.c_angular_d = base + lay.cad;
    dm.scaler = base + lay.s;
    for (int hd = 0; hd < 2; ++hd) {
        dm.w0[hd] = base + lay.w0[hd];
        dm.b0[hd] = base + lay.b0[hd];
        dm.w1[hd] = base + lay.w1[hd];
        dm.w0t[hd] = base + lay.w0t[hd];
        dm.b1[hd] = lay.b1[hd];
        dm.b1s[hd] = lay.b1s[hd] >= 0 ? base + lay.b1s[hd] : nullptr;
        dm.f32_fwd[hd] = base + lay.f32_fwd[hd];
        dm.bf_fwd_hi[hd] = reinterpret_cast<const uint4*>(base + lay.bf_fwd_hi[hd]);
        dm.bf_fwd_lo[hd] = reinterpret_cast<const uint4*>(base + lay.bf_fwd_lo[hd]);
    }
    dm.f32_bwd = base + lay.f32_bwd;
    dm.bf_bwd_hi = reinterpret_cast<const uint4*>(base + lay.bf_bwd_hi);
    dm.bf_bwd_lo = reinterpret_cast<const uint4*>(base + lay.bf_bwd_lo);
    dm.sp_w0 = lay.per_species ? m.H * m.D : 0;
    dm.sp_h = lay.per_species ? m.H : 0;
    dm.rc_radial = (float)m.rc_radial;
    dm.rc_angular = (float)m.rc_angular;
    dm.n_species = m.T;
    dm.n_hidden = m.H;
}

extern "C" int tnep_model_create(tnep_ctx* ctx, const tnep_model_desc* d, tnep_model** out) {
    if (!ctx || !d || !out) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    *out = nullptr;
    std::vector<float> h;
    ModelLayout lay;
    Model* m = new Model();
    int e = stage_model(c, d, h, *m, lay);
    if (e) {
        delete m;
        return e;
    }
    (void)hipSetDevice(c->device);
    if (hipMalloc(&m->dbuf, h.size() * sizeof(float)) != hipSuccess) {
        delete m;
        return c->fail(TNEP_E_HIP, "hipMalloc for model failed");
    }
    m->bytes = h.size() * sizeof(float);
    if (hipMemcpy(m->dbuf, h.data(), m->bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->dbuf);
        delete m;
        return c->fail(TNEP_E_HIP, "model upload failed");
    }
    bind_model(*m, (const float*)m->dbuf, lay);
    *out = reinterpret_cast<tnep_model*>(m);
    return TNEP_OK;
}

extern "C" int tnep_model_info(const tnep_model* model, int32_t* kind, int32_t* n_species,
                               int32_t* descriptor_length) {
    if (!model) return TNEP_E_INVALID;
    const Model* m = reinterpret_cast<const Model*>(model);
    if (kind) *kind = m->kind;
    if (n_species) *n_species = m->T;
    if (descriptor_length) *descriptor_length = m->D;
    return TNEP_OK;
}

extern "C" void tnep_model_free(tnep_model* model) {
    if (!model) return;
    Model* m = reinterpret_cast<Model*>(model);
    if (m->dbuf) {
        (void)hipSetDevice(m->device);  // the context may already be destroyed
        (void)hipDeviceSynchronize();
        (void)hipFree(m->dbuf);
    }
    delete m;
}

// ---------------------------------------------------------------------------
// evaluation

static int check_frames(Ctx* c, const tnep_frames* f) {
    if (!f) return c->fail(TNEP_E_INVALID, "frames is NULL");
    if (f->n_frames < 0) return c->fail(TNEP_E_INVALID, "negative n_frames");
    if (f->location != TNEP_HOST && f->location != TNEP_DEVICE && f->location != TNEP_DEVICE_META_HOST)
        return c->fail(TNEP_E_INVALID, "bad location %d", f->location);
    if (f->n_frames > 0 && (!f->atom_offsets || !f->positions || !f->species))
        return c->fail(TNEP_E_INVALID, "NULL frame arrays");
    return TNEP_OK;
}

extern "C" int tnep_eval_dipole(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames, double* mu_out,
                                double* per_atom) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    const Model* m = reinterpret_cast<const Model*>(model);
    if (!m || m->kind != TNEP_KIND_DIPOLE) return c->fail(TNEP_E_INVALID, "a dipole model is required");
    int e = check_frames(c, frames);
    if (e) return e;
    if (frames->n_frames > 0 && !mu_out) return c->fail(TNEP_E_INVALID, "mu_out is NULL");
    EvalJob job;
    job.models[0] = m;
    job.out[0] = mu_out;
    job.per_atom[0] = per_atom;
    job.n_models = 1;
    return run_eval(c, *frames, job);
}

extern "C" int tnep_eval_polarizability(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames,
                                        double* alpha_out, double* per_atom) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    const Model* m = reinterpret_cast<const Model*>(model);
    if (!m || m->kind != TNEP_KIND_POLARIZABILITY)
        return c->fail(TNEP_E_INVALID, "a polarizability model is required");
    int e = check_frames(c, frames);
    if (e) return e;
    if (frames->n_frames > 0 && !alpha_out) return c->fail(TNEP_E_INVALID, "alpha_out is NULL");
    EvalJob job;
    job.models[0] = m;
    job.out[0] = alpha_out;
    job.per_atom[0] = per_atom;
    job.n_models = 1;
    return run_eval(c, *frames, job);
}

extern "C" int tnep_eval_dipole_polarizability(tnep_ctx* ctx, const tnep_model* dipole_model,
                                               const tnep_model* polarizability_model, const tnep_frames* frames,
                                               double* mu_out, double* alpha_out) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    const Model* md = reinterpret_cast<const Model*>(dipole_model);
    const Model* mp = reinterpret_cast<const Model*>(polarizability_model);
    if (!md || md->kind != TNEP_KIND_DIPOLE || !mp || mp->kind != TNEP_KIND_POLARIZABILITY)
        return c->fail(TNEP_E_INVALID, "need a dipole model and a polarizability model");
    int e = check_frames(c, frames);
    if (e) return e;
    if (frames->n_frames > 0 && (!mu_out || !alpha_out)) return c->fail(TNEP_E_INVALID, "NULL output");
    EvalJob job;
    job.models[0] = md;
    job.models[1] = mp;
    job.out[0] = mu_out;
    job.out[1] = alpha_out;
    job.n_models = 2;
    return run_eval(c, *frames, job);
}

extern "C" int tnep_eval_dipole_charged(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames,
                                        const double* charges, const double* species_masses, double length_unit,
                                        double* mu_out, double* per_atom) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    const Model* m = reinterpret_cast<const Model*>(model);
    if (!m || m->kind != TNEP_KIND_DIPOLE) return c->fail(TNEP_E_INVALID, "a dipole model is required");
    int e = check_frames(c, frames);
    if (e) return e;
    if (frames->location == TNEP_DEVICE_META_HOST)
        return c->fail(TNEP_E_INVALID, "charged frames take TNEP_HOST or TNEP_DEVICE");
    const int F = frames->n_frames;
    if (F > 0 && (!charges || !species_masses || !mu_out)) return c->fail(TNEP_E_INVALID, "NULL argument");
    if (!(length_unit > 0) || !std::isfinite(length_unit)) return c->fail(TNEP_E_INVALID, "length_unit must be > 0");
    for (int t = 0; t < m->T && F > 0; ++t)
        if (!(species_masses[t] > 0) || !std::isfinite(species_masses[t]))
            return c->fail(TNEP_E_INVALID, "species mass %d must be positive", t);
    if (F == 0) return TNEP_OK;
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();
    // host copies of the charges, periodic flags and offsets
    std::vector<double> q(F);
    std::vector<uint8_t> pbc(frames->pbc ? 3 * (size_t)F : 0);
    std::vector<int64_t> offs(F + 1);
    const hipMemcpyKind to_host = frames->location == TNEP_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    HIP_TRY(c, hipMemcpy(q.data(), charges, sizeof(double) * F, to_host));
    HIP_TRY(c, hipMemcpy(offs.data(), frames->atom_offsets, sizeof(int64_t) * (F + 1), to_host));
    if (frames->pbc) HIP_TRY(c, hipMemcpy(pbc.data(), frames->pbc, 3 * (size_t)F, to_host));
    for (int f = 0; f < F; ++f) {
        if (!std::isfinite(q[f])) return c->fail(TNEP_E_INVALID, "frame %d: non-finite charge", f);
        const bool periodic = !pbc.empty() && (pbc[3 * f] || pbc[3 * f + 1] || pbc[3 * f + 2]);
        if (q[f] != 0.0 && periodic)
            return c->fail(TNEP_E_BOX, "frame %d: charged frame with periodic axes (no centre of mass)", f);
    }
    if ((e = tnep_eval_dipole(ctx, model, frames, mu_out, per_atom))) return e;
    const int64_t A = offs[F];
    const int T = m->T;
    // device layout: masses [T], then for host frames: charges [F], mu [F][3], offsets, positions, species
    size_t bytes = sizeof(double) * T + 256;
    if (frames->location == TNEP_HOST)
        bytes += sizeof(double) * 4 * (size_t)F + sizeof(int64_t) * (F + 1) + sizeof(double) * 3 * A +
                 sizeof(int32_t) * A + 1024;
    if ((e = c->reserve(c->com, bytes))) return e;
    char* base = (char*)c->com.p;
    double* d_masses = (double*)base;
    HIP_TRY(c, hipMemcpyAsync(d_masses, species_masses, sizeof(double) * T, hipMemcpyHostToDevice, c->stream));
    if (frames->location == TNEP_DEVICE) {
        HIP_TRY(c, launch_com_shift(frames->atom_offsets, F, frames->positions, frames->species, d_masses, charges,
                                    length_unit, mu_out, c->stream));
    } else {
        const size_t o = (sizeof(double) * T + 255) & ~(size_t)255;
        double* d_q = (double*)(base + o);
        double* d_mu = d_q + F;
        int64_t* d_offs = (int64_t*)(d_mu + 3 * (size_t)F);
        double* d_pos = (double*)(d_offs + F + 1);
        int32_t* d_spc = (int32_t*)(d_pos + 3 * (size_t)A);
        HIP_TRY(c, hipMemcpyAsync(d_q, q.data(), sizeof(double) * F, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d_mu, mu_out, sizeof(double) * 3 * F, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d_offs, offs.data(), sizeof(int64_t) * (F + 1), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d_pos, frames->positions, sizeof(double) * 3 * A, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(d_spc, frames->species, sizeof(int32_t) * A, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, launch_com_shift(d_offs, F, d_pos, d_spc, d_masses, d_q, length_unit, d_mu, c->stream));
        HIP_TRY(c, hipMemcpyAsync(mu_out, d_mu, sizeof(double) * 3 * F, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TNEP_OK;
}

extern "C" int tnep_eval_pes(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames, double* energy,
                             double* virial, double* forces, double* per_atom_energy) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    const Model* m = reinterpret_cast<const Model*>(model);
    if (!m || m->kind != TNEP_KIND_PES) return c->fail(TNEP_E_INVALID, "a potential-energy model is required");
    int e = check_frames(c, frames);
    if (e) return e;
    if (frames->n_frames > 0 && !energy) return c->fail(TNEP_E_INVALID, "energy is NULL");
    EvalJob job;
    job.models[0] = m;
    job.out[0] = energy;
    job.aux[0] = virial;
    job.per_atom[0] = per_atom_energy;
    job.forces = forces;
    job.n_models = 1;
    return run_eval(c, *frames, job);
}

// ---------------------------------------------------------------------------
// spectra

extern "C" int tnep_spectrum(tnep_ctx* ctx, const tnep_spectrum_args* a, double* freq_cm1, double* intensity,
                             double* acf) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!a || !freq_cm1 || !intensity) return c->fail(TNEP_E_INVALID, "NULL argument");
    if (a->kind < TNEP_IR || a->kind > TNEP_RAMAN_PROJ) return c->fail(TNEP_E_INVALID, "unknown spectrum kind");
    if (a->n_series < 1 || a->n_steps < 2 || !a->series) return c->fail(TNEP_E_INVALID, "empty series");
    if (a->max_lag < 1 || a->max_lag > a->n_steps) return c->fail(TNEP_E_INVALID, "need 1 <= max_lag <= n_steps");
    if (!(a->dt_fs > 0) || !std::isfinite(a->dt_fs)) return c->fail(TNEP_E_INVALID, "dt_fs must be positive");
    if (a->window != TNEP_WIN_HANN && a->window != TNEP_WIN_NONE) return c->fail(TNEP_E_INVALID, "bad window");
    if (a->location != TNEP_HOST && a->location != TNEP_DEVICE) return c->fail(TNEP_E_INVALID, "bad location");
    if (a->n_steps > ((int64_t)1 << 26)) return c->fail(TNEP_E_INVALID, "n_steps above 2^26");
    if (!(a->laser_cm1 >= 0) || !std::isfinite(a->laser_cm1)) return c->fail(TNEP_E_INVALID, "bad laser_cm1");
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();  // launch checks below must only see this call's launches
    SpectrumPlan p{};
    p.laser_cm1 = a->laser_cm1;
    p.kind = a->kind;
    p.window = a->window;
    p.flags = a->flags;
    p.n_series = a->n_series;
    p.n_steps = a->n_steps;
    p.max_lag = a->max_lag;
    p.dt_fs = a->dt_fs;
    for (int k = 0; k < 3; ++k) {
        p.n_hat[k] = a->n_hat[k];
        p.e_hat[k] = a->e_hat[k];
    }
    int64_t P = 1;
    while (P < 2 * a->n_steps) P <<= 1;
    p.fft_len = P;
    const int comps = a->kind == TNEP_IR ? 3 : 9;
    const size_t series_bytes = sizeof(double) * (size_t)a->n_series * a->n_steps * comps;
    const size_t M = (size_t)a->max_lag;
    int e;
    if ((e = c->reserve(c->spec_work, spectrum_workspace_bytes(p)))) return e;
    const double* d_series = a->series;
    double *d_freq = freq_cm1, *d_int = intensity, *d_acf = acf;
    if (a->location == TNEP_HOST) {
        if ((e = c->reserve(c->spec_series, series_bytes))) return e;
        if ((e = c->reserve(c->spec_out, sizeof(double) * (3 * M + 2)))) return e;
        HIP_TRY(c, hipMemcpyAsync(c->spec_series.p, a->series, series_bytes, hipMemcpyHostToDevice, c->stream));
        d_series = (const double*)c->spec_series.p;
        d_freq = (double*)c->spec_out.p;
        d_int = d_freq + (M + 1);
        d_acf = acf ? d_int + (M + 1) : nullptr;
    }
    const int tr = c->timer_begin(TNEP_KERNEL_SPECTRUM);
    HIP_TRY(c, launch_spectrum(p, d_series, d_freq, d_int, d_acf, c->spec_work.p, c->stream));
    c->timer_end(tr);
    if (a->location == TNEP_HOST) {
        HIP_TRY(c, hipMemcpyAsync(freq_cm1, d_freq, sizeof(double) * (M + 1), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(intensity, d_int, sizeof(double) * (M + 1), hipMemcpyDeviceToHost, c->stream));
        if (acf) HIP_TRY(c, hipMemcpyAsync(acf, d_acf, sizeof(double) * M, hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->timer_flush();
    return TNEP_OK;
}
