// Continuous-batching server of libtnep.
//
// Requests (frames + model + output buffer) are queued by any host thread.
// Each of max_inflight slot threads owns a private work context (own HIP
// stream and device buffers) and repeatedly
//   1. takes, under the queue lock, frames from the oldest pending requests
//      that use the same model, in arrival order, up to max_batch_atoms atoms
//      (a request may be split over several launches, at frame granularity);
//   2. stages them and evaluates the batch on its stream;
//   3. copies every frame's tensor into its request's output and completes
//      requests whose frames are all done.
// While one slot's batch runs on the GPU, the next slot packs whatever has
// arrived in the meantime, so work from different requests overlaps on the
// device.  Every frame is evaluated independently (its neighbour order and
// FP64 reduction order depend only on the frame itself), so a request gives
// bit-identical results alone or in any mix.
//
// Admission against the memory budget: the slots draw their work buffers from
// one pool (the server budget).  Before a batch, a slot makes sure that its
// grant covers the batch (the bytes that evaluating it in one launch batch
// reserves, at least those of its largest frame); if the pool cannot give
// that, the slot returns its own buffers and waits until other slots return
// theirs (a slot returns its buffers after every batch while another slot is
// waiting), so a request that fits the pool but not what is free now is
// queued until memory frees up.  Only a request whose largest frame alone
// exceeds the pool is rejected at submission (TNEP_E_BUDGET).  Model weights
// stay resident on the device; each slot keeps its neighbour-list and work
// buffers allocated between launches while nobody waits for memory.
// Neighbour lists are rebuilt for every launch: the trajectory reuse of
// candidates (TNEP_OPT_TRAJECTORY_WINDOW, inherited by the slots) is slower
// than a fresh search on the water workload.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.h"

namespace tnep {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const Model* model = nullptr;
    int kind = 0;
    int n_frames = 0;
    const int64_t* offsets = nullptr;
    const double* pos = nullptr;
    const int32_t* species = nullptr;
    const double* cells = nullptr;
    const uint8_t* pbc = nullptr;
    double* out = nullptr;
    int next_frame = 0;
    int frames_done = 0;
    int status = TNEP_OK;
    bool done = false;
    bool waited = false;  // a tnep_wait call owns the request
    Clock::time_point t_submit;
    double latency = 0.0;
};

struct Piece {
    Request* req;
    int f0, f1;  // frames [f0, f1) of the request
};

struct Server {
    Ctx* ctx = nullptr;
    tnep_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::map<uint64_t, Request*> live;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<std::thread> threads;
    std::vector<Ctx*> slots;
    // memory pool shared by the slots (under mu): pool = the server budget,
    // granted = sum of the slots' grants (each slot context's budget)
    uint64_t pool = 0, granted = 0;
    int mem_waiters = 0;  // slots waiting for pool memory
    std::condition_variable cv_mem;
    // neighbour capacities learned by the slots (maximum over slots, under mu)
    int cap_ang[8] = {0}, cap_rad[8] = {0};
    int waiters = 0;  // tnep_wait calls in progress
    // stats
    uint64_t n_requests = 0, n_launches = 0, n_atom_frames = 0, n_mem_waits = 0, peak_granted = 0;
};

namespace {

Ctx* slot_ctx_new(Ctx* parent) {
    Ctx* c = new Ctx();
    c->device = parent->device;
    c->budget = 0;  // granted from the server's pool batch by batch
    c->launch = parent->launch;
    c->max_batch_atoms = parent->max_batch_atoms;
    c->use_graphs = parent->use_graphs;
    c->traj_window = parent->traj_window;
    c->skin = parent->skin;
    for (int t = 0; t < 8; ++t) {
        c->cap_ang[t] = parent->cap_ang[t];
        c->cap_rad[t] = parent->cap_rad[t];
    }
    (void)hipSetDevice(c->device);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&c->h_flags, sizeof(int32_t) * 32, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return nullptr;
    }
    c->own_stream = true;
    return c;
}

// Bytes that evaluating frames of the given sizes reserves on a slot
// context: one launch batch of min(atoms, launch-batch size) atoms (the
// preferred grant) and of the largest frame alone (the least that lets the
// evaluation proceed, in launch batches of one frame).  Capacities: the
// largest that any slot has published, and those of `own` (the calling
// slot's context, or null).  Caller holds s->mu.
void batch_need(const Server* s, const Ctx* own, const Model* m, int64_t atoms, int frames, int64_t largest,
                uint64_t& want, uint64_t& least) {
    int slots = 0;
    for (int t = 0; t < m->T; ++t)
        slots += std::max(s->cap_ang[t], own ? own->cap_ang[t] : 0) + std::max(s->cap_rad[t], own ? own->cap_rad[t] : 0);
    const BatchBytes bb{m->T, slots, 1, true, 0};
    const int64_t batch = own ? own->max_batch_atoms : s->ctx->max_batch_atoms;
    const int64_t b = std::min<int64_t>(atoms, std::max<int64_t>(largest, batch));
    want = bb.bound(b, frames);
    least = bb.bound(largest, 1);
}

// Return all of the slot's work buffers and its grant to the pool (slot
// thread; caller holds s->mu).
void slot_release_locked(Server* s, Ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    c->drop_graphs();
    for (DevBuf* b : c->all_buffers()) c->release(*b);
    s->granted -= c->budget;
    c->budget = 0;
    s->cv_mem.notify_all();
}

// Make the slot's grant cover a batch: at least `least` bytes, up to `want`.
// Waits (holding nothing) while the pool cannot give `least`.  Returns false
// if the server stops meanwhile.
bool slot_acquire(Server* s, Ctx* c, uint64_t want, uint64_t least) {
    std::unique_lock<std::mutex> lk(s->mu);
    if (c->budget >= want) return true;
    const uint64_t avail = s->pool - s->granted + c->budget;
    if (avail < least) {
        // give back what this slot holds, then wait for others to do the same
        slot_release_locked(s, c);
        ++s->mem_waiters;
        ++s->n_mem_waits;
        s->cv_work.notify_all();  // idle slots return their buffers
        s->cv_mem.wait(lk, [&] { return s->stopping || s->pool - s->granted >= least; });
        --s->mem_waiters;
        if (s->pool - s->granted < least) return false;
    }
    const uint64_t grant = std::min(std::max(want, c->budget), s->pool - s->granted + c->budget);
    s->granted += grant - c->budget;
    s->peak_granted = std::max(s->peak_granted, s->granted);
    c->budget = grant;
    return true;
}

// Take the next batch from the queue (caller holds the lock).
std::vector<Piece> take_batch(Server* s, int64_t max_atoms) {
    std::vector<Piece> pieces;
    if (s->pending.empty()) return pieces;
    const Model* model = s->pending.front()->model;
    int64_t atoms = 0;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request* r = *it;
        if (r->model != model) {
            ++it;
            continue;
        }
        int f = r->next_frame;
        const int f_start = f;
        while (f < r->n_frames) {
            const int64_t na = r->offsets[f + 1] - r->offsets[f];
            if (atoms > 0 && atoms + na > max_atoms) break;
            atoms += na;
            ++f;
        }
        if (f > f_start) pieces.push_back({r, f_start, f});
        r->next_frame = f;
        if (f == r->n_frames)
            it = s->pending.erase(it);
        else
            break;  // batch full
        if (atoms >= max_atoms) break;
    }
    return pieces;
}

void finish_pieces(Server* s, const std::vector<Piece>& pieces, int status) {
    std::lock_guard<std::mutex> lk(s->mu);
    const auto now = Clock::now();
    for (const Piece& p : pieces) {
        Request* r = p.req;
        if (status != TNEP_OK && r->status == TNEP_OK) r->status = status;
        r->frames_done += p.f1 - p.f0;
        if (r->frames_done == r->n_frames) {
            r->done = true;
            r->latency = std::chrono::duration<double>(now - r->t_submit).count();
            s->n_requests += 1;
        }
    }
    s->cv_done.notify_all();
}

// Evaluate pieces as one batch on the slot context; returns a TNEP status.
int run_pieces(Server* s, Ctx* c, const std::vector<Piece>& pieces, std::vector<int64_t>& offs,
               std::vector<double>& pos, std::vector<int32_t>& spc, std::vector<double>& cells,
               std::vector<uint8_t>& pbc, std::vector<double>& out) {
    const Model* model = pieces.front().req->model;
    const int nt = model->kind == TNEP_KIND_DIPOLE ? 3 : 9;
    offs.assign(1, 0);
    pos.clear();
    spc.clear();
    cells.clear();
    pbc.clear();
    bool periodic = false;
    for (const Piece& p : pieces)
        if (p.req->pbc) periodic = true;
    for (const Piece& p : pieces) {
        const Request* r = p.req;
        const int64_t a0 = r->offsets[p.f0], a1 = r->offsets[p.f1];
        for (int f = p.f0; f < p.f1; ++f) offs.push_back(offs.back() + (r->offsets[f + 1] - r->offsets[f]));
        pos.insert(pos.end(), r->pos + 3 * a0, r->pos + 3 * a1);
        spc.insert(spc.end(), r->species + a0, r->species + a1);
        if (periodic) {
            for (int f = p.f0; f < p.f1; ++f) {
                if (r->cells)
                    cells.insert(cells.end(), r->cells + 9 * f, r->cells + 9 * f + 9);
                else
                    cells.insert(cells.end(), 9, 0.0);
                if (r->pbc)
                    pbc.insert(pbc.end(), r->pbc + 3 * f, r->pbc + 3 * f + 3);
                else
                    pbc.insert(pbc.end(), 3, (uint8_t)0);
            }
        }
    }
    const int F = (int)offs.size() - 1;
    out.assign((size_t)F * nt, 0.0);
    tnep_frames fr{F, offs.data(), pos.data(), spc.data(), periodic ? cells.data() : nullptr,
                   periodic ? pbc.data() : nullptr, TNEP_HOST};
    EvalJob job;
    job.models[0] = model;
    job.out[0] = out.data();
    job.n_models = 1;
    const int e = run_eval(c, fr, job);
    if (e == TNEP_OK) {
        int f = 0;
        for (const Piece& p : pieces) {
            std::memcpy(p.req->out + (size_t)p.f0 * nt, out.data() + (size_t)f * nt,
                        sizeof(double) * nt * (p.f1 - p.f0));
            f += p.f1 - p.f0;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->n_launches += 1;
        s->n_atom_frames += (uint64_t)offs.back();
    }
    return e;
}

// Evaluate pieces with a grant that covers them: acquire pool memory first,
// and once more if the evaluation grew its neighbour capacities beyond the
// grant.  Afterwards the slot's learned capacities join the server's.
int run_granted(Server* s, Ctx* c, const std::vector<Piece>& pieces, std::vector<int64_t>& offs,
                std::vector<double>& pos, std::vector<int32_t>& spc, std::vector<double>& cells,
                std::vector<uint8_t>& pbc, std::vector<double>& out) {
    const Model* m = pieces.front().req->model;
    int64_t atoms = 0, largest = 0;
    int frames = 0;
    for (const Piece& p : pieces)
        for (int f = p.f0; f < p.f1; ++f) {
            const int64_t na = p.req->offsets[f + 1] - p.req->offsets[f];
            atoms += na;
            largest = std::max(largest, na);
            ++frames;
        }
    int e = TNEP_E_BUDGET;
    for (int attempt = 0; attempt < 3 && e == TNEP_E_BUDGET; ++attempt) {
        uint64_t want, least;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            batch_need(s, c, m, atoms, frames, largest, want, least);
        }
        if (least > s->pool) {
            e = c->fail(TNEP_E_BUDGET, "a frame of %lld atoms needs %llu bytes, more than the server budget",
                        (long long)largest, (unsigned long long)least);
            break;
        }
        if (!slot_acquire(s, c, want, least)) return TNEP_E_CANCELLED;
        e = run_pieces(s, c, pieces, offs, pos, spc, cells, pbc, out);
        std::lock_guard<std::mutex> lk(s->mu);
        for (int t = 0; t < 8; ++t) {
            s->cap_ang[t] = std::max(s->cap_ang[t], c->cap_ang[t]);
            s->cap_rad[t] = std::max(s->cap_rad[t], c->cap_rad[t]);
        }
    }
    return e;
}

void slot_main(Server* s, Ctx* c) {
    (void)hipSetDevice(c->device);
    std::vector<int64_t> offs;
    std::vector<double> pos, cells, out;
    std::vector<int32_t> spc;
    std::vector<uint8_t> pbc;
    const int64_t max_atoms = s->opts.max_batch_atoms > 0 ? s->opts.max_batch_atoms : 262144;
    for (;;) {
        std::vector<Piece> pieces;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // an idle slot also wakes to return its buffers to a slot waiting for memory
            s->cv_work.wait(lk, [&] {
                return s->stopping || !s->pending.empty() || (s->mem_waiters > 0 && c->budget > 0);
            });
            if (s->mem_waiters > 0 && c->budget > 0) slot_release_locked(s, c);
            if (s->pending.empty() && s->stopping) return;
            pieces = take_batch(s, max_atoms);
        }
        if (pieces.empty()) continue;
        int e = run_granted(s, c, pieces, offs, pos, spc, cells, pbc, out);
        if (e != TNEP_OK && e != TNEP_E_CANCELLED && pieces.size() > 1) {
            // attribute the failure: evaluate each request's piece on its own
            for (const Piece& p : pieces) {
                std::vector<Piece> one{p};
                const int e1 = run_granted(s, c, one, offs, pos, spc, cells, pbc, out);
                finish_pieces(s, one, e1);
            }
        } else {
            finish_pieces(s, pieces, e);
        }
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->mem_waiters > 0 && c->budget > 0) slot_release_locked(s, c);
    }
}

}  // namespace

void server_shutdown(Ctx* c) {
    Server* s = c->server;
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    s->cv_mem.notify_all();
    for (std::thread& t : s->threads) t.join();
    for (Ctx* sc : s->slots) {
        c->peak = std::max(c->peak, sc->peak);
        delete sc;
    }
    {
        // requests nobody has waited for are cancelled; wait calls in progress
        // are woken and finish before the server's memory goes away
        std::unique_lock<std::mutex> lk(s->mu);
        for (auto& kv : s->live) {
            if (!kv.second->done) kv.second->status = TNEP_E_CANCELLED;
            kv.second->done = true;
        }
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    for (auto& kv : s->live) delete kv.second;
    delete s;
    c->server = nullptr;
}

void server_graph_counts(const Ctx* c, uint64_t& captures, uint64_t& launches) {
    Server* s = c->server;
    if (!s) return;
    std::lock_guard<std::mutex> lk(s->mu);
    for (const Ctx* sc : s->slots) {
        captures += sc->graph_captures;
        launches += sc->graph_launches;
    }
}

}  // namespace tnep

using namespace tnep;

extern "C" int tnep_server_start(tnep_ctx* ctx, const tnep_server_opts* opts) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (c->server) return c->fail(TNEP_E_INVALID, "server already running");
    Server* s = new Server();
    s->ctx = c;
    if (opts) s->opts = *opts;
    const int n = s->opts.max_inflight > 0 ? std::min(s->opts.max_inflight, 8) : 2;
    s->pool = s->opts.mem_budget_bytes ? s->opts.mem_budget_bytes : c->budget;
    for (int t = 0; t < 8; ++t) {
        s->cap_ang[t] = c->cap_ang[t];
        s->cap_rad[t] = c->cap_rad[t];
    }
    for (int k = 0; k < n; ++k) {
        Ctx* sc = slot_ctx_new(c);
        if (!sc) {
            for (Ctx* x : s->slots) delete x;
            delete s;
            return c->fail(TNEP_E_HIP, "could not create a server slot");
        }
        s->slots.push_back(sc);
    }
    c->server = s;
    for (Ctx* sc : s->slots) s->threads.emplace_back(slot_main, s, sc);
    return TNEP_OK;
}

extern "C" int tnep_submit(tnep_ctx* ctx, const tnep_model* model, int32_t kind, const tnep_frames* frames,
                           double* out, uint64_t* ticket) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    Server* s = c->server;
    if (!s) return TNEP_E_INVALID;
    const Model* m = reinterpret_cast<const Model*>(model);
    // the server takes dipole and polarizability requests (one output array each)
    if (!m || !frames || !out || !ticket || m->kind != kind || kind == TNEP_KIND_PES || frames->location != TNEP_HOST ||
        frames->n_frames < 1 || !frames->atom_offsets || !frames->positions || !frames->species)
        return TNEP_E_INVALID;
    // admission: the largest frame alone must fit the pool; anything more waits
    // for pool memory in the slot that takes it
    int64_t largest = 0;
    for (int f = 0; f < frames->n_frames; ++f) {
        const int64_t na = frames->atom_offsets[f + 1] - frames->atom_offsets[f];
        if (na < 0) return TNEP_E_INVALID;
        largest = std::max(largest, na);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        uint64_t want, least;
        batch_need(s, nullptr, m, largest, 1, largest, want, least);
        if (least > s->pool) return TNEP_E_BUDGET;
    }
    Request* r = new Request();
    r->model = m;
    r->kind = kind;
    r->n_frames = frames->n_frames;
    r->offsets = frames->atom_offsets;
    r->pos = frames->positions;
    r->species = frames->species;
    r->cells = frames->cells;
    r->pbc = frames->pbc;
    r->out = out;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete r;
            return TNEP_E_CANCELLED;
        }
        r->ticket = s->next_ticket++;
        s->live[r->ticket] = r;
        s->pending.push_back(r);
    }
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return TNEP_OK;
}

extern "C" int tnep_wait(tnep_ctx* ctx, uint64_t ticket, int32_t* status, double* latency_s) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    Server* s = c->server;
    if (!s) return TNEP_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    // unknown, already waited for, or waited for by another call right now
    if (it == s->live.end() || it->second->waited) return TNEP_E_INVALID;
    Request* r = it->second;
    r->waited = true;
    ++s->waiters;
    s->cv_done.wait(lk, [&] { return r->done; });
    --s->waiters;
    if (status) *status = r->status;
    if (latency_s) *latency_s = r->latency;
    if (s->stopping) {
        // shutdown frees the request; let it know this call is finished with it
        s->cv_done.notify_all();
        return TNEP_OK;
    }
    s->live.erase(it);
    delete r;
    return TNEP_OK;
}

extern "C" int tnep_server_stop(tnep_ctx* ctx) {
    if (!ctx) return TNEP_E_INVALID;
    server_shutdown(reinterpret_cast<Ctx*>(ctx));
    return TNEP_OK;
}

extern "C" int tnep_server_stats(tnep_ctx* ctx, uint64_t* requests, uint64_t* launches, uint64_t* atom_frames,
                                 uint64_t* peak_bytes) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    Server* s = c->server;
    if (!s) return TNEP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (requests) *requests = s->n_requests;
    if (launches) *launches = s->n_launches;
    if (atom_frames) *atom_frames = s->n_atom_frames;
    if (peak_bytes) *peak_bytes = s->peak_granted;
    return TNEP_OK;
}

extern "C" int tnep_server_memory(tnep_ctx* ctx, uint64_t* pool_bytes, uint64_t* granted_bytes, uint64_t* memory_waits) {
    if (!ctx) return TNEP_E_INVALID;
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    Server* s = c->server;
    if (!s) return TNEP_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pool_bytes) *pool_bytes = s->pool;
    if (granted_bytes) *granted_bytes = s->granted;
    if (memory_waits) *memory_waits = s->n_mem_waits;
    return TNEP_OK;
}
