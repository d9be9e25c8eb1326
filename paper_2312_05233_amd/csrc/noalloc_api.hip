// Spectrum entry point that allocates nothing, for callers that cannot call
// hipMalloc (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).  It is tnep_spectrum (Secs. 2.6-2.7) for device-resident
// series and outputs, with the workspace of the FFT correlation (signals,
// their transforms and the cosine table) in one fixed device array of this
// file instead of the context's allocated buffers.
//
// The array, `scratch`, is a file-scope __device__ array: every GPU the
// library runs on holds its own copy (kNoallocScratchBytes) until the process
// ends, and every call on that GPU shares it, so calls that overlap on one
// GPU (other streams, other contexts, other threads) race.  In host code its
// name is a host-side stand-in, not a device address: the device address of
// each GPU's copy is resolved once per device with hipGetSymbolAddress when a
// context is created on that device, and only that address is handed to the
// kernels.  Every byte of the workspace is written by the kernels before it is
// read, so nothing needs clearing between calls.
#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/tnep.h"
#include "internal.h"
#include "runtime.h"

namespace tnep {

namespace {

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_scratch_setup(int device, std::string& err) {
    if (device < 0 || device >= kMaxDevices) {
        err = "device index out of range for the no-allocation workspace";
        return TNEP_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return TNEP_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
        return TNEP_E_HIP;
    }
    g_scratch_ptr[device] = p;
    return TNEP_OK;
}

static void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace tnep

using namespace tnep;

extern "C" int tnep_spectrum_noalloc(tnep_ctx* ctx, const tnep_spectrum_args* a, double* freq_cm1, double* intensity,
                                     double* acf) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!a || !freq_cm1 || !intensity) return c->fail(TNEP_E_INVALID, "NULL argument");
    if (a->location != TNEP_DEVICE)
        return c->fail(TNEP_E_INVALID, "tnep_spectrum_noalloc takes device-resident series and outputs only");
    if (a->kind < TNEP_IR || a->kind > TNEP_RAMAN_PROJ) return c->fail(TNEP_E_INVALID, "unknown spectrum kind");
    if (a->n_series < 1 || a->n_steps < 2 || !a->series) return c->fail(TNEP_E_INVALID, "empty series");
    if (a->max_lag < 1 || a->max_lag > a->n_steps) return c->fail(TNEP_E_INVALID, "need 1 <= max_lag <= n_steps");
    if (!(a->dt_fs > 0) || !std::isfinite(a->dt_fs)) return c->fail(TNEP_E_INVALID, "dt_fs must be positive");
    if (a->window != TNEP_WIN_HANN && a->window != TNEP_WIN_NONE) return c->fail(TNEP_E_INVALID, "bad window");
    if (a->n_steps > ((int64_t)1 << 26)) return c->fail(TNEP_E_INVALID, "n_steps above 2^26");
    if (!(a->laser_cm1 >= 0) || !std::isfinite(a->laser_cm1)) return c->fail(TNEP_E_INVALID, "bad laser_cm1");
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
    const size_t need = spectrum_workspace_bytes(p);
    if (need > kNoallocScratchBytes)
        return c->fail(TNEP_E_BUDGET,
                       "workspace of %zu bytes exceeds the fixed no-allocation workspace of %zu bytes (n_series x "
                       "signals x FFT length too large; use tnep_spectrum)",
                       need, kNoallocScratchBytes);
    void* work = noalloc_scratch(c->device);
    if (!work) return c->fail(TNEP_E_HIP, "no-allocation workspace not set up on device %d", c->device);
    HIP_CHECK_RET(c, hipSetDevice(c->device));
    (void)hipGetLastError();  // the launch check below must only see this call's launches
    HIP_CHECK_RET(c, launch_spectrum(p, a->series, freq_cm1, intensity, acf, work, c->stream));
    return TNEP_OK;
}
