// Host-side runtime objects behind the opaque C handles of libtnep.
#pragma once

#include <stdarg.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tnep.h"
#include "internal.h"

#define HIP_CHECK_RET(ctx, expr)                                                             \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return (ctx)->fail(TNEP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

namespace tnep {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Server;  // continuous-batching server (server.hip)

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream for the models of a call after the first (every second model
    // runs on it, forked from and joined back into stream by the two events), so
    // that one model's last wavefronts overlap the next model's first
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    uint64_t peak = 0;
    std::string err;
    EvalLaunch launch{0, 256, 256, 0};
    bool autotune = false;
    // autotuned launch parameters per (shape, species count, frame-size class, location)
    struct Tuned {
        int atoms_per_block, neigh_block;
        int64_t max_batch_atoms;
    };
    std::map<std::string, Tuned> tuned;
    std::string tune_log;  // last autotuning decision (for tnep_last_error-style inspection)
    int64_t max_batch_atoms = 1 << 20;
    int cap_ang[8] = {16, 16, 16, 16, 16, 16, 16, 16};  // learned per-species neighbour capacities
    int cap_rad[8] = {32, 32, 32, 32, 32, 32, 32, 32};  // (grow-only, multiples of 4)
    int cap_cand = 64;                                   // trajectory candidates per atom and species
    int traj_window = 0;                                 // TNEP_OPT_TRAJECTORY_WINDOW (0 = off)
    double skin = 1.0;                                   // TNEP_OPT_SKIN_MA / 1000, Angstrom
    uint64_t reuse_fallbacks = 0;                        // calls redone with plain searches
    int32_t* h_flags = nullptr;       // pinned
    char* meta_host = nullptr;        // pinned staging of the launch batches' frame records and sizes
    size_t meta_host_bytes = 0;
    char* rb_host = nullptr;          // pinned staging of device-resident frame metadata read back
    size_t rb_host_bytes = 0;
    // Host frames: positions and species of two launch batches in pinned memory
    // and in two device halves (pos, species), copied on copy_stream while the
    // other half's batch is evaluated; in_copied[h] marks the copy into half h,
    // in_used[h] the end of the batch that read it.
    char* in_host = nullptr;
    size_t in_host_bytes = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t in_copied[2] = {nullptr, nullptr}, in_used[2] = {nullptr, nullptr};

    // work buffers
    DevBuf frames_tric, flags, frame_of, key_of, bucket_count, bucket_start, bucket_fill, bucket_atoms, bucket_pos, perm_start;
    // tile_base: the launch batch's device header (meta ints, then its FrameInfo records)
    DevBuf perm, tile_base, scan_chunks, nbr, counts, per_atom, out, pos, species;
    DevBuf spec_work, spec_series, spec_out;
    DevBuf pes_rec, pes_stage, pes_pair, pes_slot;  // potential-energy models: per-atom records, host-bound staging,
                                                    // pair forces, slots of the angular entries
    DevBuf slot_of, cand, cand_count;  // tile slot per atom; trajectory candidate lists
    DevBuf com;                        // charged-dipole shift: staging of frames, masses, charges, mu
    DevBuf out_call;                   // host frames: every frame's outputs of a call, copied back once
    DevBuf red_part;                   // frame sums: per-chunk partial sums
    DevBuf rad_sums;                   // radial descriptor sums shared by the models of a call
    DevBuf pop_stage, pop_work, pop_img;  // population loss: staged frames, predictions, model images
    float* pop_host = nullptr;            // pinned host staging of the population's model images
    size_t pop_host_bytes = 0;

    std::vector<DevBuf*> all_buffers() {
        return {&frames_tric, &flags, &frame_of, &key_of, &bucket_count, &bucket_start, &bucket_fill,
                &bucket_atoms, &bucket_pos, &perm_start, &perm, &tile_base, &scan_chunks, &nbr, &counts, &per_atom, &out, &pos, &species,
                &spec_work, &spec_series, &spec_out, &counters, &pes_rec, &pes_stage, &pes_pair, &pes_slot, &slot_of, &cand, &cand_count, &com,
                &pop_stage, &pop_work, &pop_img, &red_part, &rad_sums, &out_call};
    }

    Server* server = nullptr;

    // HIP graphs (TNEP_OPT_GRAPHS): one executable graph per launch-batch
    // signature, replayed for every batch with that signature.  Kernel
    // arguments hold work-buffer addresses, so every reallocation bumps
    // `epoch` and drops all graphs.
    bool use_graphs = false;
    uint64_t epoch = 0;
    struct Graph {
        hipGraphExec_t exec;
        uint64_t epoch;
    };
    std::map<std::string, Graph> graphs;
    std::atomic<uint64_t> graph_captures{0}, graph_launches{0};
    void drop_graphs();

    // launch timing (TNEP_OPT_TIMING)
    bool timing = false;
    struct Range {
        hipEvent_t a, b;
        int which;
    };
    std::vector<hipEvent_t> event_pool;
    std::vector<Range> pending;
    double kernel_ms[8] = {0};
    uint64_t kernel_launches[8] = {0};
    uint64_t pair_counts[3] = {0, 0, 0};  // atoms, radial pairs, angular pairs
    DevBuf counters;                       // device uint64[3]
    int timer_begin(int which);            // returns a range index or -1
    void timer_end(int idx);
    void timer_flush();                    // after a stream sync

    int fail(int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
    int reserve(DevBuf& b, size_t bytes);
    void release(DevBuf& b);
    ~Ctx();
};

struct Model {
    Ctx* ctx = nullptr;
    int device = 0;
    uint64_t serial = 0;  // unique per process: identifies the model in graph keys
    Shape shape{};
    DevModel dm{};
    void* dbuf = nullptr;
    size_t bytes = 0;
    int kind = 0, T = 0, D = 0, H = 0;
    double rc_radial = 0, rc_angular = 0;
};

// Offsets (in floats) of a model's arrays inside its FP32 device image.
struct ModelLayout {
    size_t cr = 0, ca = 0, cad = 0, s = 0;
    size_t w0[2] = {}, b0[2] = {}, w1[2] = {}, w0t[2] = {}, f32_fwd[2] = {}, bf_fwd_hi[2] = {}, bf_fwd_lo[2] = {};
    int64_t b1s[2] = {-1, -1};
    float b1[2] = {};
    size_t f32_bwd = 0, bf_bwd_hi = 0, bf_bwd_lo = 0;
    bool per_species = false;
};

// Validate d and append its device image to h (256-byte aligned); fills the
// model's host fields and the image layout, not its device pointers.
int stage_model(Ctx* c, const tnep_model_desc* d, std::vector<float>& h, Model& m, ModelLayout& lay);
// Point the model's DevModel at an uploaded image (base = device address of h[0]).
void bind_model(Model& m, const float* base, const ModelLayout& lay);

// One evaluation request: up to kMax models over the same frames.
// Potential-energy model (one model per job): out = energies [F], aux =
// virials [F][9] (or NULL), per_atom = site energies [A] (or NULL), forces
// [A][3] (or NULL).
struct EvalJob {
    static constexpr int kMax = 64;  // models per job (one neighbour build serves all)
    const Model* models[kMax] = {};
    double* out[kMax] = {};
    double* aux[kMax] = {};
    double* per_atom[kMax] = {};
    double* forces = nullptr;
    int n_models = 0;
};

// Frame geometry decided on the host.
struct FrameGeom {
    int mode = 0;
    int nc[3] = {1, 1, 1};
    int per[3] = {0, 0, 0};
    double L[3] = {0, 0, 0};
    int tric = 0;  // triclinic cell (then L = 0; H, Hinv, w below)
    double H[9] = {0}, Hinv[9] = {0}, w[3] = {0, 0, 0};
    int n_cells() const { return mode == 1 ? nc[0] * nc[1] * nc[2] : 0; }
};

// Device bytes of the work buffers that an evaluation reserves: per atom of a
// launch batch (used to size launch batches to the budget), and an upper
// bound for a whole launch batch of `atoms` atoms in `frames` frames (cells
// as many as the grid rules allow, every buffer grown by reserve's factor
// 1.25), used by the server's admission.  slots: neighbour rows per tile slot
// (sum of the per-species capacities); pes_rec_stride: floats per atom record
// of a potential-energy model, 0 otherwise.
struct BatchBytes {
    int T, slots, n_models;
    bool host;
    int pes_rec_stride;
    int64_t per_atom() const;
    uint64_t bound(int64_t atoms, int64_t frames) const;
};

int frame_geometry(Ctx* c, int f, const double* cell, const uint8_t* pbc, double rc_radial, int64_t n_atoms,
                   FrameGeom& g);
// Message for tnep_last_error(NULL) (calls without a context, on this thread).
void set_create_error(const std::string& msg);
int run_eval(Ctx* c, const tnep_frames& frames, const EvalJob& job);
void server_shutdown(Ctx* c);
void server_graph_counts(const Ctx* c, uint64_t& captures, uint64_t& launches);  // adds the slots' counts

hipError_t launch_init_flags(int32_t* d_flags, hipStream_t s);

// Fixed device workspace of tnep_spectrum_noalloc (noalloc_api.hip): its
// size, and the per-device resolution of its address, done once per device
// by tnep_ctx_create with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
int noalloc_scratch_setup(int device, std::string& err);

}  // namespace tnep
