// Batched evaluation of TNEP tensors: host-side planning around the kernels.
//
// A call's frames are cut into launch batches of whole frames that fit the
// context's neighbour-list capacity.  Per batch: upload frame geometry,
// build neighbour lists once, then for every model run the fused evaluation
// kernel and the fixed-order FP64 frame reduction.  Neighbour capacities are
// learned: a batch whose atoms exceed them is detected after the call and
// the whole call is repeated with larger lists.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <string>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "runtime.h"

namespace tnep {

namespace {

__global__ void k_init_flags(int32_t* f) {
    if (threadIdx.x < 32) f[threadIdx.x] = threadIdx.x == kFlagBadAtom ? INT_MAX : 0;
}

// Device-resident frame metadata (atom offsets, cells, periodic flags) gathered
// into pinned host memory by one launch: dst = [offsets | cells | pbc].
__global__ void k_gather_meta(const int64_t* __restrict__ offs, int64_t n_offs, const double* __restrict__ cells,
                              int64_t n_cells, const uint8_t* __restrict__ pbc, int64_t n_pbc, char* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_offs) reinterpret_cast<int64_t*>(dst)[i] = offs[i];
    if (i < n_cells) reinterpret_cast<double*>(dst + 8 * n_offs)[i] = cells[i];
    if (i < n_pbc) reinterpret_cast<uint8_t*>(dst + 8 * (n_offs + n_cells))[i] = pbc[i];
}

}  // namespace

hipError_t launch_init_flags(int32_t* d_flags, hipStream_t s) {
    k_init_flags<<<1, 64, 0, s>>>(d_flags);
    return hipGetLastError();
}

namespace {

// Inverse of the row-vector cell H (rows = lattice vectors) and its
// face-to-face widths; false if singular.
bool cell_inverse(const double* H, double* Hinv, double* w) {
    double cof[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof[3 * i + j] = H[3 * i1 + j1] * H[3 * i2 + j2] - H[3 * i1 + j2] * H[3 * i2 + j1];
        }
    const double det = H[0] * cof[0] + H[1] * cof[1] + H[2] * cof[2];
    if (!(std::fabs(det) > 0.0)) return false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hinv[3 * i + j] = cof[3 * j + i] / det;
    for (int k = 0; k < 3; ++k)
        w[k] = std::fabs(det) /
               std::sqrt(cof[3 * k] * cof[3 * k] + cof[3 * k + 1] * cof[3 * k + 1] + cof[3 * k + 2] * cof[3 * k + 2]);
    return true;
}

// The same lattice in a reduced basis: each row is shortened by integer
// multiples of the others (a_i -= round(a_i.a_j / a_j.a_j) a_j) until no row
// changes.  Integer row operations of determinant 1 keep the lattice, so the
// periodic system, its images and every pair vector are unchanged; the rows
// get shorter and more orthogonal, the face widths larger.
void reduce_lattice(const double* H, double* R) {
    for (int i = 0; i < 9; ++i) R[i] = H[i];
    for (int it = 0; it < 64; ++it) {
        bool changed = false;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                if (i == j) continue;
                const double* aj = R + 3 * j;
                double* ai = R + 3 * i;
                const double jj = aj[0] * aj[0] + aj[1] * aj[1] + aj[2] * aj[2];
                const double mu = std::nearbyint((ai[0] * aj[0] + ai[1] * aj[1] + ai[2] * aj[2]) / jj);
                if (mu == 0.0) continue;
                for (int k = 0; k < 3; ++k) ai[k] -= mu * aj[k];
                changed = true;
            }
        if (!changed) break;
    }
}

// Rows along distinct coordinate axes (a signed permutation of a diagonal):
// the lattice is orthorhombic, L[axis] = |row component|.
bool axis_aligned(const double* R, double* L) {
    bool used[3] = {false, false, false};
    for (int i = 0; i < 3; ++i) {
        int nz = -1, count = 0;
        for (int k = 0; k < 3; ++k)
            if (R[3 * i + k] != 0.0) {
                nz = k;
                ++count;
            }
        if (count != 1 || used[nz]) return false;
        used[nz] = true;
        L[nz] = std::fabs(R[3 * i + nz]);
    }
    return true;
}

}  // namespace

int frame_geometry(Ctx* c, int f, const double* cell, const uint8_t* pbc, double rc, int64_t n_atoms, FrameGeom& g) {
    g = FrameGeom();
    bool any = false;
    for (int d = 0; d < 3; ++d) {
        g.per[d] = pbc ? (pbc[d] != 0) : 0;
        any = any || g.per[d];
    }
    if (!any) return TNEP_OK;
    if (!cell) return c->fail(TNEP_E_BOX, "frame %d: periodic axes but no cell", f);
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(cell[k])) return c->fail(TNEP_E_NONFINITE, "frame %d: non-finite cell", f);
    bool skew = false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) skew = skew || (a != b && cell[3 * a + b] != 0.0);
    double ortho[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (skew) {
        // triclinic: all axes periodic, every face-to-face width of the cell as given >= 2 r_c
        if (!(g.per[0] && g.per[1] && g.per[2]))
            return c->fail(TNEP_E_BOX, "frame %d: a skewed cell needs all three axes periodic", f);
        double Hinv[9], w[3];
        if (!cell_inverse(cell, Hinv, w)) return c->fail(TNEP_E_BOX, "frame %d: singular cell", f);
        for (int k = 0; k < 3; ++k)
            if (!(w[k] >= 2.0 * rc))
                return c->fail(TNEP_E_BOX, "frame %d: cell width %g shorter than 2 r_c = %g", f, w[k], 2.0 * rc);
        // the search runs on a reduced basis of the same lattice
        double R[9], Rinv[9], wr[3], L[3];
        reduce_lattice(cell, R);
        const bool reduced = cell_inverse(R, Rinv, wr) && wr[0] >= 2.0 * rc && wr[1] >= 2.0 * rc && wr[2] >= 2.0 * rc;
        if (reduced && axis_aligned(R, L)) {
            // a skewed description of an orthorhombic lattice: the orthorhombic path below
            for (int d = 0; d < 3; ++d) ortho[4 * d] = L[d];
            cell = ortho;
        } else {
            const double* H = reduced ? R : cell;
            g.tric = 1;
            bool ok = true;
            for (int i = 0; i < 9; ++i) {
                g.H[i] = H[i];
                g.Hinv[i] = reduced ? Rinv[i] : Hinv[i];
            }
            // fractional bins of perpendicular width >= rc / reach, as for the
            // orthorhombic grid below
            const int reach[3] = {kCellReachXY, kCellReachXY, kCellReachZ};
            for (int k = 0; k < 3; ++k) {
                g.w[k] = reduced ? wr[k] : w[k];
                g.nc[k] = (int)std::min(1024.0, std::floor(reach[k] * g.w[k] / rc));
                ok = ok && g.nc[k] >= 2 * reach[k] + 1;
            }
            if (ok) {
                const double lim = std::max(2.0 * (double)n_atoms,
                                            (2.0 * reach[0] + 1) * (2.0 * reach[1] + 1) * (2.0 * reach[2] + 1));
                const double prod = (double)g.nc[0] * g.nc[1] * g.nc[2];
                if (prod > lim) {
                    const double s = std::cbrt(prod / lim);
                    for (int k = 0; k < 3; ++k) g.nc[k] = std::max(2 * reach[k] + 1, (int)std::floor(g.nc[k] / s));
                }
                g.mode = 1;
            } else {
                for (int k = 0; k < 3; ++k) g.nc[k] = 1;
            }
            return TNEP_OK;
        }
    }
    bool all = true;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = cell[4 * d];
        if (g.per[d] && !(g.L[d] >= 2.0 * rc))
            return c->fail(TNEP_E_BOX, "frame %d: box edge %g shorter than 2 r_c = %g", f, g.L[d], 2.0 * rc);
        all = all && g.per[d];
    }
    if (all) {
        // cells of edge >= rc / reach along each axis (the search reaches that
        // many cells each way), at least 2 reach + 1 cells per axis so that the
        // reach holds distinct cells; a sparse frame gets larger cells (about
        // two cells per atom at most)
        const int reach[3] = {kCellReachXY, kCellReachXY, kCellReachZ};
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            g.nc[d] = (int)std::min(1024.0, std::floor(reach[d] * g.L[d] / rc));
            ok = ok && g.nc[d] >= 2 * reach[d] + 1;
        }
        if (ok) {
            const double lim = std::max(2.0 * (double)n_atoms,
                                        (2.0 * reach[0] + 1) * (2.0 * reach[1] + 1) * (2.0 * reach[2] + 1));
            const double prod = (double)g.nc[0] * g.nc[1] * g.nc[2];
            if (prod > lim) {
                const double s = std::cbrt(prod / lim);
                for (int d = 0; d < 3; ++d) g.nc[d] = std::max(2 * reach[d] + 1, (int)std::floor(g.nc[d] / s));
            }
            g.mode = 1;
        }
    }
    return TNEP_OK;
}

namespace {

// Host frames of one launch batch up to this many atoms (1.8 MB of inputs) are
// copied to the device through the context's pinned staging.
constexpr int64_t kPinnedInputAtoms = 65536;

struct HostMeta {
    std::vector<int64_t> offs;
    std::vector<double> cells;
    std::vector<uint8_t> pbc;
};

int fetch_meta(Ctx* c, const tnep_frames& fr, HostMeta& m) {
    const int F = fr.n_frames;
    m.offs.resize(F + 1);
    if (fr.cells) m.cells.resize((size_t)9 * F);
    if (fr.pbc) m.pbc.resize((size_t)3 * F);
    if (fr.location != TNEP_DEVICE) {  // TNEP_HOST, TNEP_DEVICE_META_HOST: the layout is in host memory
        std::memcpy(m.offs.data(), fr.atom_offsets, sizeof(int64_t) * (F + 1));
        if (fr.cells) std::memcpy(m.cells.data(), fr.cells, sizeof(double) * 9 * F);
        if (fr.pbc) std::memcpy(m.pbc.data(), fr.pbc, 3 * (size_t)F);
    } else {
        // through pinned memory (a pageable destination costs a staged copy), on the
        // legacy default stream like a synchronous hipMemcpy, so that work the caller
        // queued there first has completed
        const size_t ob = sizeof(int64_t) * (F + 1), cb = fr.cells ? sizeof(double) * 9 * F : 0,
                     pb = fr.pbc ? 3 * (size_t)F : 0;
        const size_t need = ob + cb + pb;
        hipError_t e = hipSuccess;
        if (c->rb_host_bytes < need) {
            if (c->rb_host) (void)hipHostFree(c->rb_host);
            c->rb_host = nullptr;
            c->rb_host_bytes = 0;
            e = hipHostMalloc((void**)&c->rb_host, need, hipHostMallocDefault);
            if (e == hipSuccess) c->rb_host_bytes = need;
        }
        if (e == hipSuccess && !fr.cells && !fr.pbc) {
            e = hipMemcpyAsync(c->rb_host, fr.atom_offsets, ob, hipMemcpyDeviceToHost, nullptr);
        } else if (e == hipSuccess) {
            // one gather launch instead of a copy per array
            const int64_t n_max = std::max<int64_t>({(int64_t)F + 1, (int64_t)(cb / 8), (int64_t)pb});
            k_gather_meta<<<(unsigned)((n_max + 255) / 256), 256, 0, nullptr>>>(
                fr.atom_offsets, F + 1, fr.cells, (int64_t)(cb / 8), fr.pbc, (int64_t)pb, c->rb_host);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return c->fail(TNEP_E_HIP, "reading frame metadata: %s", hipGetErrorString(e));
        std::memcpy(m.offs.data(), c->rb_host, ob);
        if (fr.cells) std::memcpy(m.cells.data(), c->rb_host + ob, cb);
        if (fr.pbc) std::memcpy(m.pbc.data(), c->rb_host + ob + cb, pb);
    }
    if (m.offs[0] != 0) return c->fail(TNEP_E_INVALID, "atom_offsets[0] must be 0");
    for (int f = 0; f < F; ++f)
        if (m.offs[f + 1] < m.offs[f]) return c->fail(TNEP_E_INVALID, "atom_offsets decrease at frame %d", f);
    if (m.offs[F] >= ((int64_t)1 << 31)) return c->fail(TNEP_E_INVALID, "more than 2^31 atoms in one call");
    return TNEP_OK;
}

}  // namespace

int64_t BatchBytes::per_atom() const {
    // tile slots: entries, counts, perm, FP64 positions + cell records, radial sums
    const int64_t per_slot = (int64_t)slots * 16 + 8 * T + 4 + 48 + 4 * T * kRadialTerms +
                             (pes_rec_stride > 0 ? 4 * (int64_t)pes_rec_stride + (int64_t)slots * 20 : 0);
    // per atom: frame_of, slot_of, key_of, bucket_atoms; per-atom records; staged inputs
    const int64_t per_atom = 16 + 80 * (int64_t)n_models + (host ? 56 : 0) + (pes_rec_stride > 0 && host ? 32 : 0);
    return per_slot + per_atom;
}

uint64_t BatchBytes::bound(int64_t atoms, int64_t frames) const {
    const int64_t n_pad = (atoms + 63) / 64 * 64 + 64 * (int64_t)T;
    // cells: a periodic frame gets at most max(2 atoms, 125) of them, a vacuum frame one
    const int64_t cells = 2 * atoms + 125 * frames;
    const int64_t buckets = cells * T + T + 1;
    const int64_t fixed = 16 * buckets + 72 * (cells / 1024 + 1) + (int64_t)frames * (sizeof(FrameInfo) + 80 * n_models +
                                                                                        80 * kReduceChunks * n_models) +
                          4 * kMetaInts + 32 * 4 + 64;
    const int64_t bytes = per_atom() * atoms + (per_atom() - 16 - 80 * (int64_t)n_models) * (n_pad - atoms) + fixed;
    // reserve() grows a buffer to at least 1.25 times its previous size
    return (uint64_t)bytes / 4 * 5 + 4096;
}

static int run_eval_core(Ctx* c, const tnep_frames& fr, const EvalJob& job);

// Autotuning of launch parameters that do not change results: the work-group
// sizes of the evaluation and neighbour kernels and the launch-batch size.
// The call's leading frames (up to 2^20 atoms) are evaluated once per
// candidate; every candidate writes the same values, which the real run then
// overwrites.  Coordinate search: work-group sizes at the default batch size,
// then the batch size with the best work-group sizes.
static int autotune(Ctx* c, const tnep_frames& fr, const EvalJob& job, const std::string& key,
                    const std::vector<int64_t>& offs) {
    int K = 0;
    while (K < fr.n_frames && offs[K + 1] <= ((int64_t)1 << 20)) ++K;
    if (K == 0) K = 1;
    tnep_frames sub = fr;
    sub.n_frames = K;
    const int64_t atoms = offs[K];
    const EvalLaunch saved = c->launch;
    const int64_t saved_batch = c->max_batch_atoms;
    const bool saved_timing = c->timing;
    c->timing = false;
    auto measure = [&](double& ms) -> int {
        int e = run_eval_core(c, sub, job);  // warm-up (also grows neighbour capacities)
        if (e) return e;
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return c->fail(TNEP_E_HIP, "hipEventCreate failed");
        (void)hipEventRecord(a, c->stream);
        e = run_eval_core(c, sub, job);
        (void)hipEventRecord(b, c->stream);
        (void)hipEventSynchronize(b);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        ms = t;
        return e;
    };
    Ctx::Tuned best{saved.atoms_per_block, saved.neigh_block, saved_batch};
    double best_ms = 1e30;
    char buf[160];
    std::string log = "autotune " + key + ":";
    const int sizes[3] = {64, 128, 256};
    for (int eb : sizes)
        for (int nb : sizes) {
            c->launch.atoms_per_block = eb;
            c->launch.neigh_block = nb;
            double ms;
            int e = measure(ms);
            if (e) {
                c->launch = saved;
                c->timing = saved_timing;
                return e;
            }
            snprintf(buf, sizeof(buf), " eval%d/neigh%d=%.3fms", eb, nb, ms);
            log += buf;
            if (ms < best_ms) {
                best_ms = ms;
                best.atoms_per_block = eb;
                best.neigh_block = nb;
            }
        }
    c->launch.atoms_per_block = best.atoms_per_block;
    c->launch.neigh_block = best.neigh_block;
    double best_rate = atoms / best_ms;
    for (int64_t bsz : {(int64_t)1 << 18, (int64_t)1 << 19}) {
        if (bsz >= atoms) continue;
        c->max_batch_atoms = bsz;
        double ms;
        int e = measure(ms);
        if (e) {
            c->launch = saved;
            c->max_batch_atoms = saved_batch;
            c->timing = saved_timing;
            return e;
        }
        snprintf(buf, sizeof(buf), " batch%lld=%.3fms", (long long)bsz, ms);
        log += buf;
        if (atoms / ms > best_rate * 1.02) {
            best_rate = atoms / ms;
            best.max_batch_atoms = bsz;
        }
    }
    c->launch = saved;
    c->max_batch_atoms = saved_batch;
    c->timing = saved_timing;
    c->tuned[key] = best;
    snprintf(buf, sizeof(buf), " -> eval%d neigh%d batch%lld", best.atoms_per_block, best.neigh_block,
             (long long)best.max_batch_atoms);
    c->tune_log = log + buf;
    return TNEP_OK;
}

int run_eval(Ctx* c, const tnep_frames& fr, const EvalJob& job) {
    if (!c->autotune || fr.n_frames == 0) return run_eval_core(c, fr, job);
    HostMeta meta;
    int e = fetch_meta(c, fr, meta);
    if (e) return e;
    int64_t largest = 1;
    for (int f = 0; f < fr.n_frames; ++f) largest = std::max(largest, meta.offs[f + 1] - meta.offs[f]);
    int size_class = 0;
    while (((int64_t)1 << (size_class + 1)) <= largest) ++size_class;
    char key[160];
    const Shape& sh = job.models[0]->shape;
    snprintf(key, sizeof(key), "%d.%d.%d.%d.%d.%d/T%d/H%d/n%d/m%d/loc%d/mlp%d", sh.nr, sh.na, sh.kr, sh.ka,
             sh.four_body + 2 * sh.five_body, sh.kind, job.models[0]->T, job.models[0]->H, size_class, job.n_models, fr.location,
             c->launch.mlp_mode);
    auto it = c->tuned.find(key);
    if (it == c->tuned.end()) {
        e = autotune(c, fr, job, key, meta.offs);
        if (e) return e;
        it = c->tuned.find(key);
    }
    const EvalLaunch saved = c->launch;
    const int64_t saved_batch = c->max_batch_atoms;
    c->launch.atoms_per_block = it->second.atoms_per_block;
    c->launch.neigh_block = it->second.neigh_block;
    c->max_batch_atoms = it->second.max_batch_atoms;
    e = run_eval_core(c, fr, job);
    c->launch = saved;
    c->max_batch_atoms = saved_batch;
    return e;
}

static int64_t pow2_at_least(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Everything that a captured batch bakes into its kernel arguments and grids,
// apart from work-buffer addresses (covered by the context's epoch).
static std::string graph_key(const Ctx* c, const EvalJob& job, int first, int last, int T, int64_t cap_atoms,
                             int cap_frames, int64_t cap_cells, int64_t B_res) {
    std::string k;
    char buf[96];
    for (int m = first; m < last; ++m) {
        snprintf(buf, sizeof(buf), "m%llu.", (unsigned long long)job.models[m]->serial);
        k += buf;
    }
    for (int t = 0; t < T; ++t) {
        snprintf(buf, sizeof(buf), "c%d.%d.", c->cap_ang[t], c->cap_rad[t]);
        k += buf;
    }
    snprintf(buf, sizeof(buf), "l%d.%d.%d.%d/a%lld/f%d/c%lld/b%lld", c->launch.mlp_mode, c->launch.atoms_per_block,
             c->launch.neigh_block, c->launch.pair_parallel, (long long)cap_atoms, cap_frames, (long long)cap_cells,
             (long long)B_res);
    return k + buf;
}

// Launch the graph stored under `key`, capturing `launch` into it first if it
// is missing or older than the last work-buffer reallocation.
template <class Launch>
static int replay_graph(Ctx* c, const std::string& key, Launch&& launch) {
    // all stored graphs share one epoch: a reallocation drops them together
    if (!c->graphs.empty() && c->graphs.begin()->second.epoch != c->epoch) c->drop_graphs();
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= 64) c->drop_graphs();
        HIP_CHECK_RET(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = launch();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(c->stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return c->fail(TNEP_E_HIP, "graph capture failed: %s",
                           hipGetErrorString(le != hipSuccess ? le : ce));
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return c->fail(TNEP_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
        it = c->graphs.emplace(key, Ctx::Graph{ex, c->epoch}).first;
        ++c->graph_captures;
    }
    HIP_CHECK_RET(c, hipGraphLaunch(it->second.exec, c->stream));
    ++c->graph_launches;
    return TNEP_OK;
}

static int run_eval_core(Ctx* c, const tnep_frames& fr, const EvalJob& job) {
    const int F = fr.n_frames;
    if (F == 0) return TNEP_OK;
    (void)hipSetDevice(c->device);
    (void)hipGetLastError();  // launch checks below must only see this call's launches
    HostMeta meta;
    int e = fetch_meta(c, fr, meta);
    if (e) return e;
    const int64_t A = meta.offs[F];

    // models with the same cutoffs and species count share one neighbour build
    const Model* m0 = job.models[0];
    bool shared = true;
    for (int k = 1; k < job.n_models; ++k)
        shared = shared && job.models[k]->rc_radial == m0->rc_radial &&
                 job.models[k]->rc_angular == m0->rc_angular && job.models[k]->T == m0->T;

    for (int group = 0; group < (shared ? 1 : job.n_models); ++group) {
        const Model* gm = job.models[group];
        const int first = shared ? 0 : group, last = shared ? job.n_models : group + 1;
        const int T = gm->T;
        std::vector<FrameGeom> geom(F);
        for (int f = 0; f < F; ++f) {
            e = frame_geometry(c, f, fr.cells ? meta.cells.data() + 9 * (size_t)f : nullptr,
                               fr.pbc ? meta.pbc.data() + 3 * (size_t)f : nullptr, gm->rc_radial,
                               meta.offs[f + 1] - meta.offs[f], geom[f]);
            if (e) return e;
        }
        // trajectory reuse: frames with a cell grid for r_c + skin (all axes
        // periodic, every edge >= 2 (r_c + skin), >= 5 cells per axis)
        const double rc_search = gm->rc_radial + c->skin;
        bool reuse = c->traj_window > 1;
        std::vector<FrameGeom> geom_rs(reuse ? F : 0);
        std::vector<char> eligible(reuse ? F : 0, 0);
        for (int f = 0; reuse && f < F; ++f) {
            const FrameGeom& g = geom[f];
            // (packed candidates hold a rank below 2^23)
            bool ok = g.per[0] && g.per[1] && g.per[2] && meta.offs[f + 1] - meta.offs[f] < ((int64_t)1 << 23);
            for (int d = 0; d < 3 && ok; ++d) ok = g.L[d] >= 2.0 * rc_search;
            if (ok) {
                e = frame_geometry(c, f, meta.cells.data() + 9 * (size_t)f, meta.pbc.data() + 3 * (size_t)f,
                                   rc_search, meta.offs[f + 1] - meta.offs[f], geom_rs[f]);
                if (e) return e;
                ok = geom_rs[f].mode == 1;
            }
            eligible[f] = ok;
        }
        bool done = false;
        for (int attempt = 0; attempt < 6 && !done; ++attempt) {
            // rows per tile slot: per-species angular and radial-only segments
            int segA[8] = {0}, segR[8] = {0}, slots = 0;
            for (int t = 0; t < T; ++t) {
                segA[t] = slots;
                slots += c->cap_ang[t];
                segR[t] = slots;
                slots += c->cap_rad[t];
            }
            // batch size in atoms
            int64_t largest = 0;
            for (int f = 0; f < F; ++f) largest = std::max(largest, meta.offs[f + 1] - meta.offs[f]);
            int rec_stride = 0;  // potential-energy model: floats per atom record
            for (int k = first; k < last; ++k)
                if (job.models[k]->kind == TNEP_KIND_PES) rec_stride = pes_rec_stride(job.models[k]->shape, T);
            const bool pes = rec_stride > 0;
            // the pair-parallel evaluation layout (tensor models) searches frames without
            // a cell grid with 16 lanes per atom and forms no radial sums
            const bool pp_eval = c->launch.pair_parallel != 0 && !pes;
            const BatchBytes bb{T, slots, last - first, fr.location == TNEP_HOST, rec_stride};
            const int64_t per_atom_bytes = bb.per_atom();
            int64_t B = std::min<int64_t>(A, c->max_batch_atoms);
            B = std::max(B, largest);
            const int64_t room = (int64_t)c->budget - (int64_t)(c->in_use - c->nbr.bytes - c->per_atom.bytes);
            if (room > 0 && B * per_atom_bytes > room) B = std::max(largest, room / per_atom_bytes);
            // Graph replay: grids are sized for power-of-two capacities of the
            // batch's atoms, frames and cells; kernels read the actual sizes
            // from meta.  Host-resident frames: every address a kernel sees is a
            // work buffer of this context; device-resident frames: the caller's
            // input and output addresses are part of the graph key.
            const int64_t B_graph = pow2_at_least(std::max<int64_t>(B, 64));
            const bool graphs = c->use_graphs && !c->timing && c->stream &&
                                (room <= 0 || B_graph * per_atom_bytes <= room);
            const int64_t B_res = graphs ? B_graph : B;
            const int64_t n_pad_max = (B_res + 63) / 64 * 64 + 64 * T;
            if ((e = c->reserve(c->nbr, (size_t)n_pad_max * slots * sizeof(float4)))) return e;
            if ((e = c->reserve(c->counts, (size_t)n_pad_max * 2 * T * 4))) return e;
            if ((e = c->reserve(c->perm, (size_t)n_pad_max * 4))) return e;
            if ((e = c->reserve(c->frame_of, (size_t)B_res * 4))) return e;
            if ((e = c->reserve(c->slot_of, (size_t)B_res * 4))) return e;
            if ((e = c->reserve(c->key_of, (size_t)B_res * 4))) return e;
            if ((e = c->reserve(c->bucket_atoms, (size_t)B_res * 4))) return e;
            // by tile slot: FP64 positions, then the 16-byte cell records
            if ((e = c->reserve(c->bucket_pos, (size_t)n_pad_max * 48))) return e;
            if ((e = c->reserve(c->per_atom, (size_t)B_res * 10 * sizeof(double) * (last - first)))) return e;
            if (pes) {
                if ((e = c->reserve(c->pes_rec, (size_t)n_pad_max * rec_stride * sizeof(float)))) return e;
                if ((e = c->reserve(c->pes_pair, (size_t)n_pad_max * slots * sizeof(float4)))) return e;
                if ((e = c->reserve(c->pes_slot, (size_t)n_pad_max * slots * sizeof(int32_t)))) return e;
                if (fr.location == TNEP_HOST && (e = c->reserve(c->pes_stage, (size_t)B_res * 4 * sizeof(double))))
                    return e;
            }
            // the radial descriptor sums depend only on the lists, r_c^R and KR: the
            // neighbour search accumulates them, and the FP32 vector kernels of models
            // with KR = kRadialTerms load them
            if ((e = c->reserve(c->rad_sums, (size_t)n_pad_max * T * kRadialTerms * sizeof(float)))) return e;
            if ((e = c->reserve(c->flags, 32 * 4))) return e;
            // host frames in several launch batches: two input halves, the next batch's
            // inputs copied on a stream of their own while this one is evaluated (a call
            // of one batch copies on the context's stream: no stream more per context)
            const bool overlap_inputs = fr.location == TNEP_HOST && A > B;
            if (fr.location == TNEP_HOST) {
                if ((e = c->reserve(c->pos, (size_t)B_res * (overlap_inputs ? 48 : 24)))) return e;
                if ((e = c->reserve(c->species, (size_t)B_res * (overlap_inputs ? 8 : 4)))) return e;
                // every frame's outputs, copied back to the caller once at the end
                if ((e = c->reserve(c->out_call, sizeof(double) * 10 * (size_t)F * (last - first)))) return e;
            }
            // host frames are staged through pinned memory, so their copies are plain
            // DMA that the host does not wait for: two halves when the inputs of the
            // next batch are copied during this one; one for a call of one batch of at
            // most kPinnedInputAtoms atoms (larger ones keep the runtime's pageable
            // copy, which overlaps its own staging with the transfer)
            const bool stage_inputs = fr.location == TNEP_HOST && !overlap_inputs && A <= kPinnedInputAtoms;
            const size_t in_need = overlap_inputs ? (size_t)B_res * 56 : (stage_inputs ? (size_t)B_res * 28 : 0);
            if (in_need > 0 && c->in_host_bytes < in_need) {
                if (c->in_host) (void)hipHostFree(c->in_host);
                c->in_host = nullptr;
                c->in_host_bytes = 0;
                HIP_CHECK_RET(c, hipHostMalloc((void**)&c->in_host, in_need, hipHostMallocDefault));
                c->in_host_bytes = in_need;
            }
            if (overlap_inputs) {
                if (!c->copy_stream) {
                    HIP_CHECK_RET(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
                    for (int h = 0; h < 2; ++h) {
                        HIP_CHECK_RET(c, hipEventCreateWithFlags(&c->in_copied[h], hipEventDisableTiming));
                        HIP_CHECK_RET(c, hipEventCreateWithFlags(&c->in_used[h], hipEventDisableTiming));
                    }
                }
            }
            if (c->timing && !c->counters.p) {
                if ((e = c->reserve(c->counters, 64))) return e;
                HIP_CHECK_RET(c, hipMemsetAsync(c->counters.p, 0, 64, c->stream));
            }
            HIP_CHECK_RET(c, launch_init_flags((int32_t*)c->flags.p, c->stream));

            // Header of every launch batch, staged in pinned host memory (alive
            // until the sync below) so that its copy is plain DMA: the meta ints
            // the host writes (segment table, capacities, sizes) followed by the
            // FrameInfo records, one copy per batch into the device header
            // (tile_base: the meta ints, then the records at kHeaderFrames).
            // Copies from pageable memory went through host-side staging and
            // left the device idle before every batch.
            constexpr size_t kHostMeta = sizeof(int32_t) * (kMetaInts - kMetaSegA);
            static_assert(kHostMeta % 32 == 0 && kHeaderFrames == sizeof(int32_t) * kMetaInts, "header layout");
            const size_t fi_bytes = (sizeof(FrameInfo) + kHostMeta) * (size_t)F, sizes_bytes = 256;
            const size_t meta_need = fi_bytes + sizes_bytes + sizeof(FrameTric) * (size_t)F;
            if (c->meta_host_bytes < meta_need) {
                if (c->meta_host) (void)hipHostFree(c->meta_host);
                c->meta_host = nullptr;
                c->meta_host_bytes = 0;
                HIP_CHECK_RET(c, hipHostMalloc((void**)&c->meta_host, meta_need, hipHostMallocDefault));
                c->meta_host_bytes = meta_need;
            }
            char* hdr_next = c->meta_host;
            FrameTric* tri_next = reinterpret_cast<FrameTric*>(c->meta_host + fi_bytes + sizes_bytes);
            int f0 = 0;
            int batch = 0;  // launch batches of this pass (host frames alternate input halves)
            while (f0 < F) {
                int f1 = f0;
                while (f1 < F && meta.offs[f1 + 1] - meta.offs[f0] <= B) ++f1;
                if (f1 == f0) f1 = f0 + 1;
                const int nf = f1 - f0;
                const int64_t a0 = meta.offs[f0], na = meta.offs[f1] - a0;
                // host meta ints kMetaSegA.. (int index k at hmeta[k - kMetaSegA]), then the records
                int32_t* hmeta = reinterpret_cast<int32_t*>(hdr_next);
                FrameInfo* fi = reinterpret_cast<FrameInfo*>(hdr_next + kHostMeta);
                FrameTric* tri = tri_next;
                hdr_next += kHostMeta + sizeof(FrameInfo) * nf;
                tri_next += nf;
                int n_cells = 0;
                int64_t n_ref_lists = 0;  // candidate lists of the batch's reference frames (CandLists)
                bool followers = false, triclinic = false;
                bool small_frames = false, large_frames = false;  // frame-sum kernels the batch needs
                bool plain_grid = false;  // plain frames on an orthorhombic cell grid
                int ref_k = -1;  // reference frame of the open window
                for (int k = 0; k < nf; ++k) {
                    const int f = f0 + k;
                    FrameInfo& x = fi[k];
                    std::memset(&x, 0, sizeof(x));
                    x.atom_begin = meta.offs[f] - a0;
                    x.n_atoms = (int32_t)(meta.offs[f + 1] - meta.offs[f]);
                    (x.n_atoms <= kSmallFrame ? small_frames : large_frames) = true;
                    x.role = kRolePlain;
                    if (reuse && eligible[f]) {
                        const FrameInfo* r = ref_k >= 0 ? &fi[ref_k] : nullptr;
                        bool follow = r && k - ref_k < c->traj_window && r->n_atoms == x.n_atoms;
                        for (int d = 0; d < 3 && follow; ++d) follow = geom_rs[f].L[d] == r->L[d];
                        if (follow) {
                            x.role = kRoleFollower;
                            x.ref_begin = r->atom_begin;
                            x.cl_base = r->cl_base;
                            followers = true;
                        } else {
                            x.role = kRoleReference;
                            x.cl_base = n_ref_lists;
                            n_ref_lists += (int64_t)T * ((x.n_atoms + 63) / 64 * 64);
                            ref_k = k;
                        }
                    } else {
                        ref_k = -1;
                    }
                    const FrameGeom& g = x.role == kRolePlain ? geom[f] : geom_rs[f];
                    x.mode = g.mode;
                    for (int d = 0; d < 3; ++d) {
                        x.nc[d] = g.nc[d];
                        x.per[d] = g.per[d];
                        x.L[d] = g.L[d];
                        x.Linv[d] = (g.per[d] && !g.tric) ? 1.0 / g.L[d] : 0.0;
                    }
                    x.tric = g.tric;
                    if (g.mode == 1 && !g.tric && x.role == kRolePlain) plain_grid = true;
                    if (g.mode == 1) {
                        // fixed-point unit of the cell records: offsets within a cell (in A,
                        // or in fractional units for triclinic bins) stay below 2^30 units
                        double hmax = 0;
                        for (int d = 0; d < 3; ++d) hmax = std::max(hmax, g.tric ? 1.0 / g.nc[d] : g.L[d] / g.nc[d]);
                        const int kq = std::min(60, std::max(0, (int)std::floor(std::log2(std::ldexp(1.0, 30) / hmax))));
                        x.q_unit = std::ldexp(1.0, -kq);
                    }
                    if (g.tric) {
                        triclinic = true;
                        for (int i = 0; i < 9; ++i) {
                            tri[k].H[i] = g.H[i];
                            tri[k].Hinv[i] = g.Hinv[i];
                        }
                        for (int d = 0; d < 3; ++d) tri[k].w[d] = g.w[d];
                    }
                    x.cell_base = n_cells;
                    n_cells += g.mode == 1 ? g.n_cells() : 1;
                }
                // launch capacities: exact sizes, or power-of-two buckets for graphs
                const int64_t cap_atoms = graphs ? pow2_at_least(std::max<int64_t>(na, 64)) : na;
                const int cap_frames = graphs ? (int)pow2_at_least(nf) : nf;
                const int64_t cap_cells = graphs ? pow2_at_least(n_cells) : n_cells;
                const int64_t n_buckets = cap_cells * T;
                if (n_buckets >= ((int64_t)1 << 30)) return c->fail(TNEP_E_INVALID, "too many cells in one batch");
                if ((e = c->reserve(c->tile_base, kHeaderFrames + sizeof(FrameInfo) * cap_frames))) return e;
                if (triclinic && (e = c->reserve(c->frames_tric, sizeof(FrameTric) * cap_frames))) return e;
                if (n_ref_lists > 0) {
                    if ((e = c->reserve(c->cand, (size_t)n_ref_lists * T * c->cap_cand * 4))) return e;
                    if ((e = c->reserve(c->cand_count, (size_t)n_ref_lists * T * 4))) return e;
                }
                if ((e = c->reserve(c->bucket_count, (size_t)4 * (n_buckets + 1)))) return e;
                if ((e = c->reserve(c->bucket_start, (size_t)4 * (n_buckets + 1)))) return e;
                if ((e = c->reserve(c->bucket_fill, (size_t)4 * (n_buckets + 1)))) return e;
                if ((e = c->reserve(c->perm_start, (size_t)4 * (n_buckets + T + 1)))) return e;
                if ((e = c->reserve(c->scan_chunks, (size_t)4 * 18 * (cap_cells / 1024 + 1)))) return e;
                const int nt_max = 10;
                if ((e = c->reserve(c->out, sizeof(double) * nt_max * cap_frames * (last - first)))) return e;
                if ((e = c->reserve(c->red_part, sizeof(double) * 10 * kReduceChunks * cap_frames * (last - first))))
                    return e;
                // models after the first alternate with it on a second stream (not while
                // timing: the timing events are recorded on the context's stream)
                const bool two_streams = last - first >= 2 && !c->timing && c->stream != nullptr;
                if (two_streams && !c->side) {
                    HIP_CHECK_RET(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
                    HIP_CHECK_RET(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
                    HIP_CHECK_RET(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
                }
                std::memset(hmeta, 0, kHostMeta);
                for (int t = 0; t < T; ++t) {
                    hmeta[kMetaSegA - kMetaSegA + t] = segA[t];
                    hmeta[kMetaSegR - kMetaSegA + t] = segR[t];
                    hmeta[kMetaCapA - kMetaSegA + t] = c->cap_ang[t];
                    hmeta[kMetaCapR - kMetaSegA + t] = c->cap_rad[t];
                }
                hmeta[kMetaNAtoms - kMetaSegA] = (int32_t)na;
                hmeta[kMetaNFrames - kMetaSegA] = nf;
                hmeta[kMetaNCells - kMetaSegA] = n_cells;
                hmeta[kMetaAtomBase - kMetaSegA] = (int32_t)std::min<int64_t>(a0, INT32_MAX);
                // not the tile bases (ints below kMetaSegA): the scan kernel writes them
                HIP_CHECK_RET(c, hipMemcpyAsync((int32_t*)c->tile_base.p + kMetaSegA, hmeta,
                                                kHostMeta + sizeof(FrameInfo) * nf, hipMemcpyHostToDevice, c->stream));
                if (triclinic)
                    HIP_CHECK_RET(c, hipMemcpyAsync(c->frames_tric.p, tri, sizeof(FrameTric) * nf, hipMemcpyHostToDevice,
                                                    c->stream));
                const double* pos;
                const int32_t* spc;
                const int half = overlap_inputs ? (batch & 1) : 0;
                if (fr.location == TNEP_HOST && !overlap_inputs) {
                    if (stage_inputs) {
                        // the call's one batch (the staging is free: the previous call
                        // ended with a sync of the stream)
                        std::memcpy(c->in_host, fr.positions + 3 * a0, (size_t)na * 24);
                        std::memcpy(c->in_host + (size_t)B_res * 24, fr.species + a0, (size_t)na * 4);
                        HIP_CHECK_RET(c, hipMemcpyAsync(c->pos.p, c->in_host, (size_t)na * 24, hipMemcpyHostToDevice,
                                                        c->stream));
                        HIP_CHECK_RET(c, hipMemcpyAsync(c->species.p, c->in_host + (size_t)B_res * 24, (size_t)na * 4,
                                                        hipMemcpyHostToDevice, c->stream));
                    } else {
                        HIP_CHECK_RET(c, hipMemcpyAsync(c->pos.p, fr.positions + 3 * a0, (size_t)na * 24,
                                                        hipMemcpyHostToDevice, c->stream));
                        HIP_CHECK_RET(c, hipMemcpyAsync(c->species.p, fr.species + a0, (size_t)na * 4,
                                                        hipMemcpyHostToDevice, c->stream));
                    }
                    pos = (const double*)c->pos.p;
                    spc = (const int32_t*)c->species.p;
                } else if (fr.location == TNEP_HOST) {
                    // staging half: free once the copy out of it two batches ago is done;
                    // device half: free once the batch that read it two batches ago is done
                    char* stage = c->in_host + (size_t)half * B_res * 28;
                    double* dpos = (double*)c->pos.p + (size_t)half * B_res * 3;
                    int32_t* dspc = (int32_t*)c->species.p + (size_t)half * B_res;
                    if (batch >= 2) HIP_CHECK_RET(c, hipEventSynchronize(c->in_copied[half]));
                    std::memcpy(stage, fr.positions + 3 * a0, (size_t)na * 24);
                    std::memcpy(stage + (size_t)B_res * 24, fr.species + a0, (size_t)na * 4);
                    if (batch >= 2) HIP_CHECK_RET(c, hipStreamWaitEvent(c->copy_stream, c->in_used[half], 0));
                    HIP_CHECK_RET(c, hipMemcpyAsync(dpos, stage, (size_t)na * 24, hipMemcpyHostToDevice,
                                                    c->copy_stream));
                    HIP_CHECK_RET(c, hipMemcpyAsync(dspc, stage + (size_t)B_res * 24, (size_t)na * 4,
                                                    hipMemcpyHostToDevice, c->copy_stream));
                    HIP_CHECK_RET(c, hipEventRecord(c->in_copied[half], c->copy_stream));
                    HIP_CHECK_RET(c, hipStreamWaitEvent(c->stream, c->in_copied[half], 0));
                    pos = dpos;
                    spc = dspc;
                } else {
                    pos = fr.positions + 3 * a0;
                    spc = fr.species + a0;
                }
                NeighborWork w{(int32_t*)c->frame_of.p,     (int32_t*)c->key_of.p,       (int32_t*)c->bucket_count.p,
                               (int32_t*)c->bucket_start.p, (int32_t*)c->bucket_fill.p,  (int32_t*)c->bucket_atoms.p,
                               (double4*)c->bucket_pos.p,
                               (int4*)((char*)c->bucket_pos.p + (size_t)n_pad_max * 32),
                               (int32_t*)c->perm_start.p,   (int32_t*)c->perm.p,
                               (int32_t*)c->tile_base.p,    (int32_t*)c->scan_chunks.p,  (int32_t*)c->slot_of.p};
                const CandLists cl{(int32_t*)c->cand.p, (int32_t*)c->cand_count.p, c->cap_cand,
                                   (float)rc_search, (float)(0.25 * c->skin * c->skin)};
                NeighborLists nl{};
                nl.entries = (float4*)c->nbr.p;
                nl.counts = (int32_t*)c->counts.p;
                nl.perm = (const int32_t*)c->perm.p;
                nl.meta = (const int32_t*)c->tile_base.p;
                nl.n_pad = (cap_atoms + 63) / 64 * 64 + 64 * T;
                nl.T = T;
                nl.slots = slots;
                // per model: per-atom records, per-frame outputs (a: tensor or
                // energy, b: virial of a potential-energy model)
                double* pa_of[EvalJob::kMax];
                double* out_of[EvalJob::kMax];
                double* aux_of[EvalJob::kMax] = {};
                int nt_of[EvalJob::kMax], na_of[EvalJob::kMax];
                double *forces_dst = nullptr, *energies_dst = nullptr;
                for (int k = first; k < last; ++k) {
                    const int kind = job.models[k]->kind;
                    const int q = k - first;
                    nt_of[q] = kind == TNEP_KIND_DIPOLE ? 3 : (kind == TNEP_KIND_POLARIZABILITY ? 9 : 10);
                    na_of[q] = kind == TNEP_KIND_PES ? 1 : nt_of[q];
                    pa_of[q] = (double*)c->per_atom.p + (size_t)B_res * 10 * q;
                    if (kind != TNEP_KIND_PES && job.per_atom[k] && fr.location != TNEP_HOST)
                        pa_of[q] = job.per_atom[k] + a0 * nt_of[q];
                    double* staged = (double*)c->out.p + (size_t)nt_max * cap_frames * q;
                    out_of[q] = fr.location != TNEP_HOST ? job.out[k] + (size_t)f0 * na_of[q] : staged;
                    if (kind == TNEP_KIND_PES) {
                        if (fr.location != TNEP_HOST) {
                            aux_of[q] = job.aux[k] ? job.aux[k] + (size_t)f0 * 9 : nullptr;
                            forces_dst = job.forces ? job.forces + a0 * 3 : nullptr;
                            energies_dst = job.per_atom[k] ? job.per_atom[k] + a0 : nullptr;
                        } else {
                            aux_of[q] = staged + cap_frames;
                            forces_dst = job.forces ? (double*)c->pes_stage.p : nullptr;
                            energies_dst = job.per_atom[k] ? (double*)c->pes_stage.p + 3 * B_res : nullptr;
                        }
                    }
                }
                const PesOut pes_out{(float*)c->pes_rec.p, rec_stride, (float4*)c->pes_pair.p, (int32_t*)c->pes_slot.p};
                // Frames without a cell grid: in the pair-parallel layout always the 16-lane
                // search; otherwise in batches of few atoms (whose time the one-lane search
                // sets by one atom's walk over its frame) the 16-lane search with the radial
                // sums, which gives the one-lane search's rows and sums bit for bit.
                const bool pair_search = pp_eval || na <= kPairSearchAtoms;
                const bool pair_radial = !pp_eval;
                // the batch's kernels; with graphs on, captured once and replayed
                auto launch_batch = [&]() -> hipError_t {
                    hipError_t he;
                    int tr = c->timer_begin(TNEP_KERNEL_NEIGHBORS);
                    he = launch_neighbors((const FrameInfo*)((char*)c->tile_base.p + kHeaderFrames),
                                          triclinic ? (const FrameTric*)c->frames_tric.p : nullptr, cap_frames, pos,
                                          spc, cap_atoms,
                                          (int)cap_cells, (float)gm->rc_radial, (float)gm->rc_angular, w, nl, cl,
                                          n_ref_lists > 0, followers, triclinic, pair_search, pair_radial, plain_grid,
                                          (int32_t*)c->flags.p,
                                          c->launch.neigh_block, (float*)c->rad_sums.p, c->stream);
                    c->timer_end(tr);
                    if (he != hipSuccess) return he;
                    if (c->timing) {
                        he = launch_count_pairs(nl, (unsigned long long*)c->counters.p, c->stream);
                        if (he != hipSuccess) return he;
                    }
                    // the side stream waits for the search (the fork event), enqueued after
                    // the first model's kernels so that they reach the device sooner
                    if (two_streams && (he = hipEventRecord(c->fork_ev, c->stream)) != hipSuccess) return he;
                    for (int k = first; k < last; ++k) {
                        const Model* m = job.models[k];
                        const int q = k - first;
                        hipStream_t sq = (two_streams && (q & 1)) ? c->side : c->stream;
                        if (two_streams && q == 1 && (he = hipStreamWaitEvent(c->side, c->fork_ev, 0)) != hipSuccess)
                            return he;
                        tr = c->timer_begin(m->kind == TNEP_KIND_DIPOLE           ? TNEP_KERNEL_EVAL_DIPOLE
                                            : m->kind == TNEP_KIND_POLARIZABILITY ? TNEP_KERNEL_EVAL_POLARIZABILITY
                                                                                  : TNEP_KERNEL_EVAL_PES);
                        const RadSums rs{(float*)c->rad_sums.p, 2};
                        he = launch_eval(m->shape, m->dm, nl, pa_of[q], pes_out, rs, c->launch, sq);
                        c->timer_end(tr);
                        if (he != hipSuccess) return he;
                        tr = c->timer_begin(TNEP_KERNEL_FRAME_REDUCE);
                        he = launch_frame_reduce((const FrameInfo*)((char*)c->tile_base.p + kHeaderFrames), cap_frames,
                                                 nl.meta, pa_of[q], nt_of[q], na_of[q],
                                                 (double*)c->red_part.p + (size_t)10 * kReduceChunks * cap_frames * q,
                                                 out_of[q], aux_of[q], small_frames, large_frames, sq);
                        c->timer_end(tr);
                        if (he != hipSuccess) return he;
                        if (m->kind == TNEP_KIND_PES) {
                            tr = c->timer_begin(TNEP_KERNEL_PES_FORCES);
                            he = launch_pes_forces(m->shape, m->dm, nl, pes_out, pa_of[q], forces_dst, energies_dst,
                                                   c->launch.atoms_per_block, sq);
                            c->timer_end(tr);
                            if (he != hipSuccess) return he;
                        }
                    }
                    if (two_streams) {
                        if ((he = hipEventRecord(c->join_ev, c->side)) != hipSuccess) return he;
                        if ((he = hipStreamWaitEvent(c->stream, c->join_ev, 0)) != hipSuccess) return he;
                    }
                    return hipSuccess;
                };
                if (graphs) {
                    std::string key = graph_key(c, job, first, last, T, cap_atoms, cap_frames, cap_cells, B_res);
                    if (n_ref_lists > 0) {
                        char rb[64];
                        // the candidate radius and displacement guard are kernel arguments
                        snprintf(rb, sizeof(rb), "/r%d.%d.%a.%a", c->cap_cand, followers ? 1 : 0, (double)cl.rc_search,
                                 (double)cl.half_skin2);
                        key += rb;
                    }
                    // potential-energy outputs: k_pes_forces runs only when forces or site
                    // energies are asked for, and writes them to fixed staging places
                    if (pes) {
                        char pb[16];
                        snprintf(pb, sizeof(pb), "/p%d%d", forces_dst ? 1 : 0, energies_dst ? 1 : 0);
                        key += pb;
                    }
                    if (triclinic) key += "/tric";
                    // host frames: the input half the kernels read
                    if (fr.location == TNEP_HOST) key += half ? "/h1" : "/h0";
                    // which frame-sum kernels run (frames of at most / above kSmallFrame atoms)
                    key += small_frames ? (large_frames ? "/s11" : "/s10") : "/s01";
                    // whether the plain cell-grid search runs beside the pair-parallel one
                    if (pair_search) key += pair_radial ? (plain_grid ? "/rg1" : "/rg0") : (plain_grid ? "/g1" : "/g0");
                    // device-resident frames: the caller's buffers the kernels read and write
                    if (fr.location != TNEP_HOST) {
                        char db[64];
                        snprintf(db, sizeof(db), "/d%p.%p", (const void*)pos, (const void*)spc);
                        key += db;
                        for (int q = 0; q < last - first; ++q) {
                            snprintf(db, sizeof(db), "/o%p.%p.%p", (void*)out_of[q], (void*)pa_of[q], (void*)aux_of[q]);
                            key += db;
                        }
                        if (pes) {
                            snprintf(db, sizeof(db), "/f%p.%p", (void*)forces_dst, (void*)energies_dst);
                            key += db;
                        }
                    }
                    if ((e = replay_graph(c, key, launch_batch)))
                        return e;
                } else {
                    HIP_CHECK_RET(c, launch_batch());
                }
                if (fr.location == TNEP_HOST) {
                    if (overlap_inputs) HIP_CHECK_RET(c, hipEventRecord(c->in_used[half], c->stream));
                    for (int k = first; k < last; ++k) {
                        const int q = k - first;
                        const int na_ = na_of[q];
                        // tensors (and virials) into the call's output buffer: device copies,
                        // so the host goes on staging the next batch
                        double* oc = (double*)c->out_call.p + (size_t)10 * F * q;
                        HIP_CHECK_RET(c, hipMemcpyAsync(oc + (size_t)f0 * na_, out_of[q], sizeof(double) * na_ * nf,
                                                        hipMemcpyDeviceToDevice, c->stream));
                        if (job.models[k]->kind == TNEP_KIND_PES) {
                            if (job.aux[k])
                                HIP_CHECK_RET(c, hipMemcpyAsync(oc + (size_t)F * na_ + (size_t)f0 * 9, aux_of[q],
                                                                sizeof(double) * 9 * nf, hipMemcpyDeviceToDevice,
                                                                c->stream));
                            if (job.forces)
                                HIP_CHECK_RET(c, hipMemcpyAsync(job.forces + a0 * 3, forces_dst,
                                                                sizeof(double) * 3 * na, hipMemcpyDeviceToHost,
                                                                c->stream));
                            if (job.per_atom[k])
                                HIP_CHECK_RET(c, hipMemcpyAsync(job.per_atom[k] + a0, energies_dst,
                                                                sizeof(double) * na, hipMemcpyDeviceToHost,
                                                                c->stream));
                        } else if (job.per_atom[k]) {
                            HIP_CHECK_RET(c, hipMemcpyAsync(job.per_atom[k] + a0 * nt_of[q], pa_of[q],
                                                            sizeof(double) * nt_of[q] * na, hipMemcpyDeviceToHost,
                                                            c->stream));
                        }
                    }
                }
                f0 = f1;
                ++batch;
            }
            // host frames: every model's outputs back into pinned memory in one copy
            // (the models' regions of out_call are adjacent), handed to the caller
            // after the sync below
            const size_t out_bytes = sizeof(double) * 10 * (size_t)F * (last - first);
            if (fr.location == TNEP_HOST) {
                if (c->rb_host_bytes < out_bytes) {
                    if (c->rb_host) (void)hipHostFree(c->rb_host);
                    c->rb_host = nullptr;
                    c->rb_host_bytes = 0;
                    HIP_CHECK_RET(c, hipHostMalloc((void**)&c->rb_host, out_bytes, hipHostMallocDefault));
                    c->rb_host_bytes = out_bytes;
                }
                HIP_CHECK_RET(c, hipMemcpyAsync(c->rb_host, c->out_call.p, out_bytes, hipMemcpyDeviceToHost, c->stream));
            }
            HIP_CHECK_RET(c, hipMemcpyAsync(c->h_flags, c->flags.p, sizeof(int32_t) * 32, hipMemcpyDeviceToHost,
                                            c->stream));
            HIP_CHECK_RET(c, hipStreamSynchronize(c->stream));
            if (fr.location == TNEP_HOST) {
                for (int k = first; k < last; ++k) {
                    const int q = k - first;
                    const int kind = job.models[k]->kind;
                    const int na_ = kind == TNEP_KIND_DIPOLE ? 3 : (kind == TNEP_KIND_POLARIZABILITY ? 9 : 1);
                    const double* oc = reinterpret_cast<const double*>(c->rb_host) + (size_t)10 * F * q;
                    std::memcpy(job.out[k], oc, sizeof(double) * na_ * F);
                    if (kind == TNEP_KIND_PES && job.aux[k])
                        std::memcpy(job.aux[k], oc + (size_t)F * na_, sizeof(double) * 9 * F);
                }
            }
            c->timer_flush();
            const int32_t* fl = c->h_flags;
            if (reuse && fl[kFlagReuse]) {
                // an atom moved more than skin / 2 (or changed species): plain searches
                reuse = false;
                ++c->reuse_fallbacks;
                continue;
            }
            if (fl[kFlagError]) {
                const int code = (fl[kFlagError] & kErrNonFinite) ? TNEP_E_NONFINITE
                                 : (fl[kFlagError] & kErrSpecies) ? TNEP_E_SPECIES
                                                                  : TNEP_E_OVERLAP;
                // the first offending atom (index in the call) and its frame
                const int64_t bad = fl[kFlagBadAtom];
                int bad_frame = 0;
                while (bad_frame + 1 < F && meta.offs[bad_frame + 1] <= bad) ++bad_frame;
                return c->fail(code, "invalid input (%s) at atom %lld of frame %d",
                               code == TNEP_E_NONFINITE ? "non-finite position"
                               : code == TNEP_E_SPECIES ? "species out of range"
                                                        : "atoms closer than 1e-4 A",
                               (long long)(bad - meta.offs[bad_frame]), bad_frame);
            }
            bool grow = false;
            for (int t = 0; t < T; ++t) {
                if (fl[kFlagCapAng + t] > c->cap_ang[t]) {
                    c->cap_ang[t] = (fl[kFlagCapAng + t] * 5 / 4 + 3) / 4 * 4;
                    grow = true;
                }
                if (fl[kFlagCapRad + t] > c->cap_rad[t]) {
                    c->cap_rad[t] = (fl[kFlagCapRad + t] * 5 / 4 + 3) / 4 * 4;
                    grow = true;
                }
            }
            if (reuse && fl[kFlagCapCand] > c->cap_cand) {
                c->cap_cand = (fl[kFlagCapCand] * 5 / 4 + 3) / 4 * 4;
                grow = true;
            }
            if (!grow) done = true;
        }
        if (!done) return c->fail(TNEP_E_NEIGH_OVERFLOW, "neighbour lists still overflow after growing them");
    }
    return TNEP_OK;
}

}  // namespace tnep
