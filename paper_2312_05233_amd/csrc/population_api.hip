// Population loss of a set of parameter vectors (Sec. 2.4 Loss functions):
// every individual is a model with the base model's hyperparameters and its
// own trainable parameters; all individuals are evaluated over the same frames
// (jobs of up to EvalJob::kMax models share each neighbour build), and
//   L(z) = RMSE(T(z), T_ref) + lambda1 sum|z| / N + lambda2 sqrt(sum z^2 / N).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace tnep;

namespace {

// out[p] = sum_i (pred[p][i] - ref[i])^2, one work-group per individual, fixed order.
__global__ void __launch_bounds__(256) k_pop_sse(const double* __restrict__ pred, const double* __restrict__ ref,
                                                 int64_t n, double* __restrict__ out) {
    __shared__ double part[256];
    const int p = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = pred[(int64_t)p * n + i] - ref[i];
        s += d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = part[0];
}

// l1[p] = sum |z|, l2[p] = sum z^2 over the individual's parameters.
__global__ void __launch_bounds__(256) k_pop_reg(const double* __restrict__ z, int64_t n, double* __restrict__ l1,
                                                 double* __restrict__ l2) {
    __shared__ double a[256], b[256];
    const int p = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = z[(int64_t)p * n + i];
        s1 += fabs(v);
        s2 += v * v;
    }
    a[threadIdx.x] = s1;
    b[threadIdx.x] = s2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            a[threadIdx.x] += a[threadIdx.x + off];
            b[threadIdx.x] += b[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        l1[p] = a[0];
        l2[p] = b[0];
    }
}

__global__ void k_pop_finish(const double* __restrict__ sse, const double* __restrict__ l1,
                             const double* __restrict__ l2, int P, int64_t n_values, int64_t n_params, double lambda1,
                             double lambda2, double* __restrict__ loss, double* __restrict__ rmse) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double e = sqrt(sse[p] / (double)n_values);
    rmse[p] = e;
    loss[p] = e + lambda1 * l1[p] / (double)n_params + lambda2 * sqrt(l2[p] / (double)n_params);
}

// Number of trainable parameters and their layout: c_radial, c_angular, then
// per head w0 [H][D], b0 [H], w1 [H], b1.
struct ParamLayout {
    size_t ncr, nca, nw0, nh, per_head, total;
    int heads;
};

ParamLayout layout_of(const tnep_model_desc* d) {
    ParamLayout L{};
    const int T = d->n_species;
    const int nr = d->n_max_radial + 1, na = d->n_max_angular + 1, kr = d->basis_radial + 1,
              ka = d->basis_angular + 1;
    const int D = nr + d->l_max * na + (d->four_body ? na : 0) + (d->five_body ? na : 0);
    L.ncr = (size_t)T * T * nr * kr;
    L.nca = (size_t)T * T * na * ka;
    L.nw0 = (size_t)d->n_hidden * D;
    L.nh = (size_t)d->n_hidden;
    L.per_head = L.nw0 + 2 * L.nh + 1;
    L.heads = d->kind == TNEP_KIND_POLARIZABILITY ? 2 : 1;
    L.total = L.ncr + L.nca + L.heads * L.per_head;
    return L;
}

}  // namespace

extern "C" int tnep_population_loss(tnep_ctx* ctx, const tnep_model_desc* base, int32_t n_individuals,
                                    const double* params, const tnep_frames* frames, const double* reference,
                                    double lambda1, double lambda2, double* loss_out, double* rmse_out) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!base || !params || !frames || !reference || !loss_out) return c->fail(TNEP_E_INVALID, "NULL argument");
    if (base->kind != TNEP_KIND_DIPOLE && base->kind != TNEP_KIND_POLARIZABILITY)
        return c->fail(TNEP_E_INVALID, "population loss is for dipole and polarizability models");
    if (base->per_species) return c->fail(TNEP_E_INVALID, "population loss takes shared-network models");
    if (n_individuals < 1 || n_individuals > 65535) return c->fail(TNEP_E_INVALID, "need 1..65535 individuals");
    if (!std::isfinite(lambda1) || !std::isfinite(lambda2) || lambda1 < 0 || lambda2 < 0)
        return c->fail(TNEP_E_INVALID, "regularization weights must be finite and >= 0");
    if (frames->n_frames < 1 || !frames->atom_offsets || !frames->positions || !frames->species)
        return c->fail(TNEP_E_INVALID, "need at least one frame");
    if (frames->location != TNEP_HOST && frames->location != TNEP_DEVICE)
        return c->fail(TNEP_E_INVALID, "bad location");
    const ParamLayout L = layout_of(base);
    const int P = n_individuals, F = frames->n_frames;
    const int nt = base->kind == TNEP_KIND_DIPOLE ? 3 : 9;
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();

    // frames on the device (host frames are staged once for all individuals)
    std::vector<int64_t> offs(F + 1);
    const hipMemcpyKind to_host = frames->location == TNEP_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    HIP_CHECK_RET(c, hipMemcpy(offs.data(), frames->atom_offsets, sizeof(int64_t) * (F + 1), to_host));
    const int64_t A = offs[F];
    DevBuf& stage = c->pop_stage;
    DevBuf& work = c->pop_work;
    DevBuf& mimg = c->pop_img;
    tnep_frames dfr = *frames;
    const size_t n_values = (size_t)F * nt;
    int e;
    if (frames->location == TNEP_HOST) {
        const size_t bytes = sizeof(int64_t) * (F + 1) + sizeof(double) * 3 * A + sizeof(int32_t) * A +
                             (frames->cells ? sizeof(double) * 9 * F : 0) + (frames->pbc ? 3 * (size_t)F : 0) +
                             sizeof(double) * n_values + 1024;
        if ((e = c->reserve(stage, bytes))) return e;
        char* q = (char*)stage.p;
        auto put = [&](const void* src, size_t nb) {
            char* dst = q;
            q += (nb + 255) & ~(size_t)255;
            return std::make_pair(dst, hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, c->stream));
        };
        auto r1 = put(offs.data(), sizeof(int64_t) * (F + 1));
        auto r2 = put(frames->positions, sizeof(double) * 3 * A);
        auto r3 = put(frames->species, sizeof(int32_t) * A);
        dfr.atom_offsets = (const int64_t*)r1.first;
        dfr.positions = (const double*)r2.first;
        dfr.species = (const int32_t*)r3.first;
        hipError_t he = r1.second != hipSuccess ? r1.second : (r2.second != hipSuccess ? r2.second : r3.second);
        if (frames->cells) {
            auto r = put(frames->cells, sizeof(double) * 9 * F);
            dfr.cells = (const double*)r.first;
            if (r.second != hipSuccess) he = r.second;
        }
        if (frames->pbc) {
            auto r = put(frames->pbc, 3 * (size_t)F);
            dfr.pbc = (const uint8_t*)r.first;
            if (r.second != hipSuccess) he = r.second;
        }
        auto rr = put(reference, sizeof(double) * n_values);
        reference = (const double*)rr.first;
        if (rr.second != hipSuccess) he = rr.second;
        if (he != hipSuccess) return c->fail(TNEP_E_HIP, "staging frames failed: %s", hipGetErrorString(he));
        dfr.location = TNEP_DEVICE;
    }
    // predictions [P][F][nt], parameters [P][N], per-individual sums
    const size_t wbytes = sizeof(double) * ((size_t)P * n_values + (size_t)P * L.total + 5 * (size_t)P) + 4096;
    if ((e = c->reserve(work, wbytes))) return e;
    double* pred = (double*)work.p;
    double* zdev = pred + (size_t)P * n_values;
    double* sse = zdev + (size_t)P * L.total;
    double *l1 = sse + P, *l2 = l1 + P, *dloss = l2 + P, *drmse = dloss + P;
    auto cleanup = [&](int code) {
        (void)hipStreamSynchronize(c->stream);  // the uploads read host memory owned by this call
        return code;
    };
    if (hipMemcpyAsync(zdev, params, sizeof(double) * (size_t)P * L.total, hipMemcpyHostToDevice, c->stream) !=
        hipSuccess)
        return cleanup(c->fail(TNEP_E_HIP, "parameter upload failed"));

    // all individuals' model images (built on host threads) in one upload
    std::vector<Model> models(P);
    std::vector<ModelLayout> lays(P);
    std::vector<std::vector<float>> imgs(P);
    std::vector<int> errs(P, TNEP_OK);
    auto desc_of = [&](int p) {
        const double* z = params + (size_t)p * L.total;
        tnep_model_desc d = *base;
        d.c_radial = z;
        d.c_angular = z + L.ncr;
        for (int h = 0; h < L.heads; ++h) {
            const double* hz = z + L.ncr + L.nca + h * L.per_head;
            d.w0[h] = hz;
            d.b0[h] = hz + L.nw0;
            d.w1[h] = hz + L.nw0 + L.nh;
            d.b1[h] = hz[L.nw0 + 2 * L.nh];
        }
        return d;
    };
    // the first individual on this thread (structural errors get their message), the rest in parallel
    {
        const tnep_model_desc d = desc_of(0);
        if ((e = stage_model(c, &d, imgs[0], models[0], lays[0]))) return cleanup(e);
    }
    auto stage_range = [&](int pa, int pb) {
        for (int p = pa; p < pb; ++p) {
            const tnep_model_desc d = desc_of(p);
            errs[p] = stage_model(nullptr, &d, imgs[p], models[p], lays[p]);
        }
    };
    const int rest = P - 1;
    const int n_threads = std::max(1, std::min({rest, 16, (int)std::thread::hardware_concurrency()}));
    if (rest > 0) {
        std::vector<std::thread> pool;
        const int per = (rest + n_threads - 1) / n_threads;
        for (int t = 1; t < n_threads; ++t)
            if (1 + t * per < P) pool.emplace_back(stage_range, 1 + t * per, std::min(P, 1 + (t + 1) * per));
        stage_range(1, std::min(P, 1 + per));
        for (auto& th : pool) th.join();
    }
    // every individual has the same image layout; pack them into pinned memory for one DMA
    const size_t isz = imgs[0].size();
    for (int p = 0; p < P; ++p) {
        if (errs[p]) return cleanup(c->fail(errs[p], "individual %d: non-finite parameters", p));
        if (imgs[p].size() != isz) return cleanup(c->fail(TNEP_E_INVALID, "individual %d: image size differs", p));
    }
    const size_t img_bytes = (size_t)P * isz * sizeof(float);
    if (c->pop_host_bytes < img_bytes) {
        if (c->pop_host) (void)hipHostFree(c->pop_host);
        c->pop_host = nullptr;
        c->pop_host_bytes = 0;
        if (hipHostMalloc((void**)&c->pop_host, img_bytes, hipHostMallocDefault) != hipSuccess) {
            c->pop_host = nullptr;
            return cleanup(c->fail(TNEP_E_HIP, "pinned staging of %zu bytes failed", img_bytes));
        }
        c->pop_host_bytes = img_bytes;
    }
    for (int p = 0; p < P; ++p) std::memcpy(c->pop_host + (size_t)p * isz, imgs[p].data(), isz * sizeof(float));
    if ((e = c->reserve(mimg, img_bytes))) return cleanup(e);
    if (hipMemcpyAsync(mimg.p, c->pop_host, img_bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return cleanup(c->fail(TNEP_E_HIP, "model upload failed"));
    for (int p = 0; p < P; ++p) {
        models[p].ctx = c;
        models[p].device = c->device;
        bind_model(models[p], (const float*)mimg.p + (size_t)p * isz, lays[p]);
    }

    // individuals in jobs of up to EvalJob::kMax models sharing a neighbour build
    for (int p0 = 0; p0 < P; p0 += EvalJob::kMax) {
        EvalJob job;
        job.n_models = std::min(EvalJob::kMax, P - p0);
        for (int k = 0; k < job.n_models; ++k) {
            job.models[k] = &models[p0 + k];
            job.out[k] = pred + (size_t)(p0 + k) * n_values;
        }
        if ((e = run_eval(c, dfr, job))) return cleanup(e);
    }
    k_pop_sse<<<P, 256, 0, c->stream>>>(pred, reference, (int64_t)n_values, sse);
    k_pop_reg<<<P, 256, 0, c->stream>>>(zdev, (int64_t)L.total, l1, l2);
    k_pop_finish<<<(P + 255) / 256, 256, 0, c->stream>>>(sse, l1, l2, P, (int64_t)n_values, (int64_t)L.total, lambda1,
                                                         lambda2, dloss, drmse);
    hipError_t he = hipGetLastError();
    if (he == hipSuccess) he = hipMemcpyAsync(loss_out, dloss, sizeof(double) * P, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess && rmse_out)
        he = hipMemcpyAsync(rmse_out, drmse, sizeof(double) * P, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return cleanup(c->fail(TNEP_E_HIP, "population loss: %s", hipGetErrorString(he)));
    return cleanup(TNEP_OK);
}
