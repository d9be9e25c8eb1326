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
// Admission: the server budget is split evenly over the slots; a request
// with a frame too large for one slot is rejected at submission
// (TNEP_E_BUDGET).  Model weights stay resident on the device; each slot keeps
// its neighbour-list and work buffers allocated between launches.
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
    uint64_t slot_budget = 0;
    int64_t per_atom_bytes_est = 0;
    // stats
    uint64_t n_requests = 0, n_launches = 0, n_atom_frames = 0;
};

namespace {

Ctx* slot_ctx_new(Ctx* parent, uint64_t budget) {
    Ctx* c = new Ctx();
    c->device = parent->device;
    c->budget = budget;
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
            s->cv_work.wait(lk, [&] { return s->stopping || !s->pending.empty(); });
            if (s->pending.empty() && s->stopping) return;
            pieces = take_batch(s, max_atoms);
        }
        if (pieces.empty()) continue;
        int e = run_pieces(s, c, pieces, offs, pos, spc, cells, pbc, out);
        if (e != TNEP_OK && pieces.size() > 1) {
            // attribute the failure: evaluate each request's piece on its own
            for (const Piece& p : pieces) {
                std::vector<Piece> one{p};
                const int e1 = run_pieces(s, c, one, offs, pos, spc, cells, pbc, out);
                finish_pieces(s, one, e1);
            }
            continue;
        }
        finish_pieces(s, pieces, e);
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
    for (std::thread& t : s->threads) t.join();
    for (Ctx* sc : s->slots) {
        c->peak = std::max(c->peak, sc->peak);
        delete sc;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& kv : s->live) {
            kv.second->status = TNEP_E_CANCELLED;
            kv.second->done = true;
        }
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
    const uint64_t budget = s->opts.mem_budget_bytes ? s->opts.mem_budget_bytes : c->budget;
    s->slot_budget = budget / n;
    for (int k = 0; k < n; ++k) {
        Ctx* sc = slot_ctx_new(c, s->slot_budget);
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
    // admission: the largest frame must fit one slot's budget
    int64_t largest = 0;
    for (int f = 0; f < frames->n_frames; ++f) {
        const int64_t na = frames->atom_offsets[f + 1] - frames->atom_offsets[f];
        if (na < 0) return TNEP_E_INVALID;
        largest = std::max(largest, na);
    }
    int slots_per_atom = 0;
    for (int t = 0; t < m->T; ++t) slots_per_atom += c->cap_ang[t] + c->cap_rad[t];
    const int64_t need = (largest + 64 * m->T + 64) * ((int64_t)slots_per_atom * 16 + 8 * m->T + 24 + 72 + 28 + 32);
    if ((uint64_t)need > s->slot_budget) return TNEP_E_BUDGET;
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
    if (it == s->live.end()) return TNEP_E_INVALID;
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    if (status) *status = r->status;
    if (latency_s) *latency_s = r->latency;
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
    if (peak_bytes) {
        uint64_t p = 0;
        for (Ctx* sc : s->slots) p += sc->peak;
        *peak_bytes = p;
    }
    return TNEP_OK;
}
