// Continuous-batching server of libtnep (filled in below).
#include "runtime.h"

namespace tnep {
void server_shutdown(Ctx*) {}
}  // namespace tnep

using namespace tnep;

extern "C" int tnep_server_start(tnep_ctx* ctx, const tnep_server_opts*) {
    return ctx ? reinterpret_cast<Ctx*>(ctx)->fail(TNEP_E_INVALID, "server not available") : TNEP_E_INVALID;
}
extern "C" int tnep_submit(tnep_ctx* ctx, const tnep_model*, int32_t, const tnep_frames*, double*, uint64_t*) {
    return ctx ? reinterpret_cast<Ctx*>(ctx)->fail(TNEP_E_INVALID, "server not available") : TNEP_E_INVALID;
}
extern "C" int tnep_wait(tnep_ctx* ctx, uint64_t, int32_t*, double*) {
    return ctx ? reinterpret_cast<Ctx*>(ctx)->fail(TNEP_E_INVALID, "server not available") : TNEP_E_INVALID;
}
extern "C" int tnep_server_stop(tnep_ctx* ctx) { return ctx ? TNEP_OK : TNEP_E_INVALID; }
extern "C" int tnep_server_stats(tnep_ctx* ctx, uint64_t*, uint64_t*, uint64_t*, uint64_t*) {
    return ctx ? reinterpret_cast<Ctx*>(ctx)->fail(TNEP_E_INVALID, "server not available") : TNEP_E_INVALID;
}
