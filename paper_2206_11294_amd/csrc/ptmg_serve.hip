// Continuous-batching serving engine of libptmg (C ABI in pt_serve.h).
//
// One device arena (first-fit, coalescing free list) holds the handles of
// admitted requests; one stream and one pinned status block per slot.
// pt_server_progress runs the loop: admit queued requests in arrival order
// while a slot is free and the head request fits, poll every active
// request's last event, and enqueue its next step (right-hand side, each
// IR iteration, final copy) as soon as the previous one has finished.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "ptmg_internal.h"
#include "pt_serve.h"

using namespace ptmg;

namespace {

thread_local std::string g_serve_err = "no error";
constexpr size_t kAlign = 256;

struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    size_t used = 0;

    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t o2 = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum Stage { QUEUED, SETUP, SOLVING, DONE };

struct Request {
    long long id;
    pt_problem prob;
    int prec;
    const double *b_p, *b_T, *div;
    double *p, *T;
    pt_solve_opts opts;
    Stage stage = QUEUED;
    int slot = -1;
    pt_mg_t h = nullptr;
    size_t off = 0, bytes = 0, handle_bytes = 0;
    double *own_b = nullptr;      // engine-formed right-hand side (in the arena block)
    pt_request_info info;
};

struct Slot {
    hipStream_t stream = nullptr;
    void *pinned = nullptr;
    long long req = -1;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct pt_server_s {
    pt_server_config cfg;
    Arena arena;
    char *pinned = nullptr;
    std::vector<Slot> slots;
    std::map<long long, Request> reqs;
    std::deque<long long> queue;
    long long next_id = 1;
    long long finished = 0;
    int active = 0;
    std::string err = "no error";
};

namespace {

int sfail(pt_server_t s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    else g_serve_err = msg;
    return code;
}

void finish(pt_server_t s, Request &r, int status)
{
    if (r.h) {
        pt_mg_destroy(r.h);   // its stream has finished the request's work
        r.h = nullptr;
    }
    if (r.bytes) s->arena.release(r.off, r.bytes);
    if (r.slot >= 0) {
        s->slots[r.slot].req = -1;
        s->active--;
    }
    r.slot = -1;
    r.bytes = 0;
    r.stage = DONE;
    r.info.status = status;
    r.info.t_done = now_s();
    s->finished++;
}

// Admit the head of the queue if a slot is free and its block fits.
bool admit_one(pt_server_t s)
{
    if (s->queue.empty()) return false;
    int slot = -1;
    for (int q = 0; q < (int)s->slots.size(); q++)
        if (s->slots[q].req < 0) {
            slot = q;
            break;
        }
    if (slot < 0) return false;
    Request &r = s->reqs[s->queue.front()];
    if (r.bytes > s->arena.size) {   // can never fit
        s->queue.pop_front();
        r.bytes = 0;
        finish(s, r, PT_ERR_OOM);
        return true;
    }
    size_t off;
    if (!s->arena.alloc(r.bytes, &off)) return false;   // wait for memory
    s->queue.pop_front();
    r.off = off;
    r.slot = slot;
    s->slots[slot].req = r.id;
    s->active++;
    r.stage = SETUP;
    r.info.status = PT_SERVE_ACTIVE;
    r.info.t_admit = now_s();
    char *mem = s->arena.base + off;
    std::string err;
    int rc = handle_create(&r.prob, r.prec, s->slots[slot].stream, mem, r.handle_bytes,
                           s->slots[slot].pinned, &r.h, &err);
    if (rc != PT_OK) {
        r.h = nullptr;
        finish(s, r, rc);
        return true;
    }
    pt_mg_set_option(r.h, PT_OPT_GRAPHS, s->cfg.use_graphs);
    if (s->cfg.omega_milli) pt_mg_set_option(r.h, PT_OPT_OMEGA, s->cfg.omega_milli);
    if (s->cfg.coarse_sweeps) pt_mg_set_option(r.h, PT_OPT_COARSE_SWEEPS, s->cfg.coarse_sweeps);
    if (!r.b_p) r.own_b = (double *)(mem + r.handle_bytes);
    return true;
}

// Poll one active request; enqueue its next step when the last finished.
bool poll_one(pt_server_t s, Request &r)
{
    hipError_t e = hipEventQuery(handle_event(r.h));
    if (e == hipErrorNotReady) {
        if (hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
        return false;
    }
    if (e != hipSuccess) {
        finish(s, r, PT_ERR_HIP);
        return true;
    }
    if (r.stage == SETUP) {
        int rc = handle_setup_check(r.h);
        const double *b_p = r.b_p, *b_T = r.b_T;
        const long long N = (long long)r.prob.n[0] * r.prob.n[1] * r.prob.n[2];
        if (rc == PT_OK && !b_p) {
            b_p = r.own_b;
            b_T = r.own_b + N;
            rc = handle_paper_rhs_async(r.h, r.prob.p_adv, r.prob.T_adv, r.div, r.own_b,
                                        r.own_b + N);
        }
        if (rc == PT_OK) rc = solve_begin(r.h, b_p, b_T, r.p, r.T, &r.opts);
        if (rc != PT_OK) {
            finish(s, r, rc);
            return true;
        }
        r.stage = SOLVING;
        return true;
    }
    pt_solve_info inf;
    int rc = solve_advance(r.h, &inf);
    if (rc == PT_RUNNING) return true;
    r.info.cycles = inf.cycles;
    r.info.relres[0] = inf.relres[0];
    r.info.relres[1] = inf.relres[1];
    finish(s, r, rc);
    return true;
}

}  // namespace

double pt_server_now(void) { return now_s(); }

int pt_server_create(const pt_server_config *cfg, pt_server_t *out)
{
    if (!out) return sfail(nullptr, PT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->max_active < 1 || cfg->max_active > 64 || cfg->hbm_budget < kAlign ||
        cfg->omega_milli < 0 || cfg->omega_milli > 1999 || cfg->coarse_sweeps < 0 ||
        cfg->coarse_sweeps > 255 || (cfg->coarse_sweeps && ((cfg->coarse_sweeps >> 4) > 8 ||
                                                            (cfg->coarse_sweeps & 15) > 8)))
        return sfail(nullptr, PT_ERR_ARG, "bad server config");
    pt_server_t s = new pt_server_s();
    s->cfg = *cfg;
    s->arena.size = cfg->hbm_budget & ~(kAlign - 1);
    if (hipMalloc(&s->arena.base, s->arena.size) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return sfail(nullptr, PT_ERR_OOM, "arena allocation failed");
    }
    s->arena.free_[0] = s->arena.size;
    const size_t per = 16 * sizeof(double) + 16 * sizeof(int);
    if (hipHostMalloc((void **)&s->pinned, per * cfg->max_active, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->pinned = nullptr;
        pt_server_destroy(s);
        return sfail(nullptr, PT_ERR_OOM, "pinned allocation failed");
    }
    s->slots.resize(cfg->max_active);
    for (int q = 0; q < cfg->max_active; q++) {
        s->slots[q].pinned = s->pinned + per * q;
        if (hipStreamCreateWithFlags(&s->slots[q].stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            s->slots[q].stream = nullptr;
            pt_server_destroy(s);
            return sfail(nullptr, PT_ERR_HIP, "stream creation failed");
        }
    }
    *out = s;
    return PT_OK;
}

int pt_server_submit(pt_server_t s, const pt_problem *prob, int precision, const double *b_p,
                     const double *b_T, const double *div_ustar, double *p, double *T,
                     const pt_solve_opts *opts, double t_arrival, long long *id)
{
    if (!s || !prob || !p || !T) return sfail(s, PT_ERR_ARG, "NULL argument");
    const size_t hb = handle_plan_bytes(prob, precision);
    if (hb == 0) return sfail(s, PT_ERR_ARG, "invalid problem");
    if ((b_p == nullptr) != (b_T == nullptr)) return sfail(s, PT_ERR_ARG, "give both b_p and b_T or neither");
    if (!b_p && prob->mode == PT_COEF_EXPLICIT)
        return sfail(s, PT_ERR_ARG, "explicit mode needs its right-hand side");
    Request r;
    r.id = s->next_id++;
    r.prob = *prob;
    r.prec = precision;
    r.b_p = b_p;
    r.b_T = b_T;
    r.div = div_ustar;
    r.p = p;
    r.T = T;
    r.opts = opts ? *opts : pt_solve_opts{1e-9, 50, 2, 2, 1, PT_SOLVE_DEFECT};
    const long long N = (long long)prob->n[0] * prob->n[1] * prob->n[2];
    r.handle_bytes = (hb + kAlign - 1) & ~(kAlign - 1);
    r.bytes = r.handle_bytes + (b_p ? 0 : (size_t)16 * N);
    std::memset(&r.info, 0, sizeof r.info);
    r.info.status = PT_SERVE_QUEUED;
    r.info.t_arrival = t_arrival;
    r.info.bytes = r.bytes;
    s->reqs[r.id] = r;
    s->queue.push_back(r.id);
    if (id) *id = r.id;
    return PT_OK;
}

int pt_server_progress(pt_server_t s, double until, int *n_done)
{
    if (!s) return sfail(nullptr, PT_ERR_ARG, "server is NULL");
    const long long f0 = s->finished;
    for (;;) {
        while (admit_one(s)) {
        }
        for (auto &sl : s->slots) {
            if (sl.req < 0) continue;
            (void)poll_one(s, s->reqs[sl.req]);
        }
        const double t = now_s();
        if (t >= until) break;
        if (s->queue.empty() && s->active == 0) {
            // idle: wait for the deadline (the caller submits at that time)
            if (!std::isfinite(until)) break;
            const double dt = until - t;
            if (dt > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 1e-4));
        }
    }
    if (n_done) *n_done = (int)(s->finished - f0);
    return PT_OK;
}

int pt_server_request(pt_server_t s, long long id, pt_request_info *info)
{
    if (!s || !info) return sfail(s, PT_ERR_ARG, "NULL argument");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return sfail(s, PT_ERR_ARG, "unknown request");
    *info = it->second.info;
    return PT_OK;
}

int pt_server_stats(pt_server_t s, int *queued, int *active, long long *finished,
                    size_t *bytes_in_use)
{
    if (!s) return sfail(nullptr, PT_ERR_ARG, "server is NULL");
    if (queued) *queued = (int)s->queue.size();
    if (active) *active = s->active;
    if (finished) *finished = s->finished;
    if (bytes_in_use) *bytes_in_use = s->arena.used;
    return PT_OK;
}

void pt_server_destroy(pt_server_t s)
{
    if (!s) return;
    for (auto &kv : s->reqs)
        if (kv.second.h) {
            pt_mg_destroy(kv.second.h);
            kv.second.h = nullptr;
        }
    for (auto &sl : s->slots)
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (s->arena.base) (void)hipFree(s->arena.base);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
}

const char *pt_server_last_error(pt_server_t s) { return s ? s->err.c_str() : g_serve_err.c_str(); }
