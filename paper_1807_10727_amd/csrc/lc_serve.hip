// Serving: continuous batching of connected-components requests on one GPU (cc_server_*).
//
// A scheduler thread owns the device.  Requests are admitted while a slot and HBM budget
// are free, and their work overlaps on the device:
//   - small requests (int32 records within the LDS limits of the configured variant) that
//     are waiting are fused into one launch of the persistent LDS solver, which solves
//     each of them in one workgroup;
//   - every other request gets a slot stream, the slot's host mirror of the round state
//     (allocated once: freeing pinned memory would synchronise the whole device each time a
//     request completes) and a workspace carved from the caller's arena, and advances one
//     round per step: the scheduler enqueues a round and an
//     asynchronous readback of its state, and picks the request up again when the event
//     behind that readback has completed, so rounds of different requests run
//     concurrently on their streams.
// Requests that arrive while others run are admitted as soon as a slot and memory are
// free (a request waiting for memory is deferred, never failed).  Each request runs the
// same arithmetic as a solo solve with its seed, so its labels do not depend on the mix.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cc.h"
#include "lc_engine.hpp"
#include "lc_small.hpp"

namespace lc {

__global__ void k_zero_u32(uint32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// first-fit allocator over [0, size) with coalescing of freed ranges
struct ArenaAlloc {
    std::map<size_t, size_t> free_;   // offset -> size
    size_t size = 0, used = 0;
    void init(size_t n) {
        free_.clear();
        size = n;
        used = 0;
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) / 256 * 256;
        used -= n;
        auto it = free_.emplace(off, n).first;
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

struct Request {
    uint64_t id = 0;
    cc_graph_desc g{};
    uint64_t seed = 0;
    void *labels = nullptr;
    size_t footprint = 0;
    bool small = false;
    bool cancelled = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    cc_status status = CC_OK;
    int32_t rounds = 0;
    // large path
    cc_ctx *ctx = nullptr;
    size_t off = 0;
    int slot = -1;
    int phase = 0;   // 1: a round in flight, 2: labels in flight
    int32_t cohort = 0;       // requests of the cohort it was solved in
};

// Large requests solved together as one disjoint union on one slot (cohort_*).
struct Cohort {
    std::vector<Request *> reqs;
    cc_batch *b = nullptr;
    size_t off = 0, footprint = 0;
};

struct SmallLaunch {
    std::vector<Request *> reqs;
    size_t off = 0, bytes = 0;
    SmallDesc *h = nullptr;      // pinned staging: descriptors then rounds
    int32_t *h_rounds = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
};

}  // namespace lc

using namespace lc;

struct cc_server {
    char *arena = nullptr;
    size_t budget = 0;
    cc_server_config cfg{};
    ArenaAlloc alloc;
    std::vector<hipStream_t> streams;       // one per slot
    std::vector<hipEvent_t> events;         // one per slot
    std::vector<Request *> slot_req;
    std::vector<Cohort *> slot_cohort;      // a slot holds a request or a cohort
    RoundState *mirrors = nullptr;          // pinned host mirrors of the round state, one per slot
    bool mirrors_pageable = false;
    int32_t *rounds_pinned = nullptr;       // per slot: the round counts of a cohort's requests
    int64_t n_cohorts = 0;
    hipStream_t small_stream = nullptr;
    std::vector<SmallLaunch> small;         // small launches (in flight or free)
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> done;
    std::unordered_map<uint64_t, Request *> live;
    uint64_t next_id = 1;
    bool stop = false;
    bool paused = false;                    // admit nothing new (cc_server_pause)
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    std::string err;
    size_t peak_used = 0;
    int64_t n_small_launches = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

bool small_ok(const cc_server *s, const cc_graph_desc &g) {
    if (s->cfg.small_variant <= 0 || g.layout != CC_EDGES_SOA_I32) return false;
    const SmallVariant v = kSmallVariants[s->cfg.small_variant];
    return g.n_vertices <= v.nmax && g.n_edges <= v.mmax;
}

// completes a request (caller holds the lock)
void finish_locked(cc_server *s, Request *r, cc_status st) {
    r->status = st;
    r->t_done = s->now();
    s->done.push_back(r);
    s->cv_done.notify_all();
}

void release_large(cc_server *s, Request *r) {
    if (r->ctx) {
        cc_destroy(r->ctx);
        r->ctx = nullptr;
    }
    if (r->footprint) s->alloc.release(r->off, r->footprint);
    if (r->slot >= 0) s->slot_req[r->slot] = nullptr;
    r->slot = -1;
}

// admit a large request on slot k (lock held); returns false when memory is short
bool admit_large(cc_server *s, Request *r, int k) {
    size_t off = 0;
    if (!s->alloc.alloc(r->footprint, &off)) return false;
    s->peak_used = std::max(s->peak_used, s->alloc.used);
    r->off = off;
    r->slot = k;
    s->slot_req[k] = r;
    r->t_admit = s->now();
    cc_options o{};
    o.seed = r->seed;
    o.stream = s->streams[k];
    cc_status st = ctx_create(&r->g, &o, s->mirrors + k, &r->ctx);
    if (st == CC_OK) st = cc_set_workspace(r->ctx, s->arena + off, r->footprint);
    int launched = 0;
    if (st == CC_OK) st = ctx_round_enqueue(r->ctx, &launched);
    if (st == CC_OK && launched) {
        r->phase = 1;
        if (hipEventRecord(s->events[k], s->streams[k]) != hipSuccess) st = CC_E_HIP;
    } else if (st == CC_DONE) {   // no records: labels are the ids
        r->ctx->labels_ready = true;
        st = ctx_labels_enqueue(r->ctx, r->labels);
        r->phase = 2;
        if (st == CC_OK && hipEventRecord(s->events[k], s->streams[k]) != hipSuccess) st = CC_E_HIP;
    }
    if (st < 0) {
        release_large(s, r);
        s->live.erase(r->id);
        finish_locked(s, r, st);
    }
    return true;
}

// a slot's event has completed: next round, labels, or done (lock held)
void advance_large(cc_server *s, int k) {
    Request *r = s->slot_req[k];
    cc_status st = CC_OK;
    if (r->phase == 1) {
        st = ctx_round_complete(r->ctx, nullptr);
        if (st >= 0 && r->cancelled) st = CC_E_STATE;
        if (st == CC_OK && !r->ctx->done) {
            int launched = 0;
            st = ctx_round_enqueue(r->ctx, &launched);
            if (st == CC_OK && launched) {
                if (hipEventRecord(s->events[k], s->streams[k]) != hipSuccess) st = CC_E_HIP;
                if (st == CC_OK) return;
            }
        }
        if (st == CC_OK || st == CC_DONE) {
            r->ctx->labels_ready = true;
            r->rounds = r->ctx->rounds;
            st = ctx_labels_enqueue(r->ctx, r->labels);
            if (st == CC_OK && hipEventRecord(s->events[k], s->streams[k]) != hipSuccess) st = CC_E_HIP;
            if (st == CC_OK) {
                r->phase = 2;
                return;
            }
        }
    } else {
        r->rounds = r->ctx->rounds;
        st = r->cancelled ? CC_E_STATE : CC_OK;
    }
    release_large(s, r);
    s->live.erase(r->id);
    finish_locked(s, r, st);
}

constexpr int kCohortMax = 64;

bool cohort_ok(const cc_server *s, const Request *r) {
    const int64_t nmax = s->cfg.cohort_max_vertices > 0 ? s->cfg.cohort_max_vertices : (int64_t)1 << 20;
    return s->cfg.cohort_max > 1 && !r->small && !r->cancelled && r->g.layout == CC_EDGES_SOA_I32 &&
           r->g.n_vertices > 0 && r->g.n_vertices <= nmax;
}

void release_cohort(cc_server *s, int k) {
    Cohort *c = s->slot_cohort[k];
    if (c->b) cc_batch_destroy(c->b);   // the slot's mirror is borrowed: nothing to free on the host
    if (c->footprint) s->alloc.release(c->off, c->footprint);
    s->slot_cohort[k] = nullptr;
    delete c;
}

// start the requests `reqs` as one cohort on slot k (lock held); false when it cannot start
// (memory short, or a HIP failure, after which the requests stay pending)
bool admit_cohort(cc_server *s, const std::vector<Request *> &reqs, int k) {
    const int32_t G = (int32_t)reqs.size();
    std::vector<int64_t> voff(G + 1, 0), eoff(G + 1, 0);
    std::vector<uint64_t> seeds(G);
    std::vector<const int32_t *> src(G), dst(G);
    std::vector<int32_t *> lab(G);
    for (int32_t i = 0; i < G; ++i) {
        const Request *r = reqs[i];
        voff[i + 1] = voff[i] + r->g.n_vertices;
        eoff[i + 1] = eoff[i] + r->g.n_edges;
        seeds[i] = r->seed;
        src[i] = (const int32_t *)r->g.src;
        dst[i] = (const int32_t *)r->g.dst;
        lab[i] = (int32_t *)r->labels;
    }
    if (voff[G] > 0x7FFFFFFFLL || eoff[G] > 0xFFFFFFFELL) return false;
    Cohort *c = new (std::nothrow) Cohort();
    if (!c) return false;
    if (cohort_create(G, voff.data(), eoff.data(), seeds.data(), src.data(), dst.data(), lab.data(), s->streams[k],
                      s->mirrors + k, &c->b) != CC_OK) {
        delete c;
        return false;
    }
    size_t need = 0;
    (void)cc_batch_workspace_size(c->b, &need);
    if (!s->alloc.alloc(need, &c->off)) {
        cc_batch_destroy(c->b);
        delete c;
        return false;
    }
    c->footprint = need;
    s->peak_used = std::max(s->peak_used, s->alloc.used);
    s->slot_cohort[k] = c;
    int32_t *h_rounds = s->rounds_pinned + (size_t)k * kCohortMax;
    if (cc_batch_set_workspace(c->b, s->arena + c->off, need) != CC_OK || cohort_begin(c->b, h_rounds) != CC_OK ||
        hipEventRecord(s->events[k], s->streams[k]) != hipSuccess) {
        (void)hipStreamSynchronize(s->streams[k]);
        release_cohort(s, k);
        return false;
    }
    const double t = s->now();
    for (Request *r : reqs) {
        r->t_admit = t;
        r->cohort = G;
    }
    c->reqs = reqs;
    s->n_cohorts += 1;
    return true;
}

// a cohort slot's event has completed: its next round, its labels, or its end (lock held)
void advance_cohort(cc_server *s, int k) {
    Cohort *c = s->slot_cohort[k];
    int32_t *h_rounds = s->rounds_pinned + (size_t)k * kCohortMax;
    bool finished = false;
    const cc_status st = cohort_advance(c->b, h_rounds, &finished);
    if (st == CC_OK && !finished) {
        if (hipEventRecord(s->events[k], s->streams[k]) == hipSuccess) return;
    }
    (void)hipStreamSynchronize(s->streams[k]);
    std::vector<Request *> reqs = c->reqs;
    release_cohort(s, k);
    for (size_t i = 0; i < reqs.size(); ++i) {
        Request *r = reqs[i];
        cc_status rs = st;
        if (rs == CC_OK) rs = h_rounds[i] < 0 ? CC_E_INPUT : (r->cancelled ? CC_E_STATE : CC_OK);   // -1: bad input
        r->rounds = rs == CC_OK ? h_rounds[i] : 0;
        s->live.erase(r->id);
        finish_locked(s, r, rs);
    }
}

// fuse waiting small requests into one LDS-solver launch (lock held)
void launch_small_batch(cc_server *s, std::vector<Request *> &batch) {
    SmallLaunch *L = nullptr;
    for (auto &x : s->small)
        if (!x.busy) {
            L = &x;
            break;
        }
    if (!L || batch.empty()) return;
    const size_t cnt = batch.size();
    const size_t bytes = sizeof(SmallDesc) * cnt + 4 * cnt + 256;
    size_t off = 0;
    if (!s->alloc.alloc(bytes, &off)) return;   // wait for memory; they stay pending
    s->peak_used = std::max(s->peak_used, s->alloc.used);
    char *base = s->arena + off;
    SmallDesc *d_desc = (SmallDesc *)base;
    int32_t *d_rounds = (int32_t *)(base + sizeof(SmallDesc) * cnt);
    uint32_t *d_ctl = (uint32_t *)(base + (sizeof(SmallDesc) * cnt + 4 * cnt + 127) / 128 * 128);   // queue, err
    const double t = s->now();
    for (size_t i = 0; i < cnt; ++i) {
        Request *r = batch[i];
        SmallDesc &d = L->h[i];
        d.src = (const int32_t *)r->g.src;
        d.dst = (const int32_t *)r->g.dst;
        d.m = r->g.n_edges;
        d.n = (int32_t)r->g.n_vertices;
        d.status = 0;
        d.seed = r->seed;
        d.labels = (int32_t *)r->labels;
        d.rounds = d_rounds + i;
        r->t_admit = t;
    }
    hipStream_t st = s->small_stream;
    SmallArgs a;
    a.desc = d_desc;
    a.count = (int32_t)cnt;
    a.queue = d_ctl;
    a.err = d_ctl + 1;
    bool ok = hipMemcpyAsync(d_desc, L->h, sizeof(SmallDesc) * cnt, hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, d_ctl, 2);
        ok = hipGetLastError() == hipSuccess;
    }
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(cnt, 256 * (size_t)std::max(1, s->cfg.small_blocks_per_cu)));
    if (ok) ok = launch_small(s->cfg.small_variant, s->cfg.small_threads, a, grid, st) == hipSuccess;
    if (ok) ok = hipMemcpyAsync(L->h, d_desc, sizeof(SmallDesc) * cnt, hipMemcpyDeviceToHost, st) == hipSuccess;
    if (ok) ok = hipMemcpyAsync(L->h_rounds, d_rounds, 4 * cnt, hipMemcpyDeviceToHost, st) == hipSuccess;
    if (ok) ok = hipEventRecord(L->ev, st) == hipSuccess;
    if (!ok) {
        s->alloc.release(off, bytes);
        for (Request *r : batch) {
            s->live.erase(r->id);
            finish_locked(s, r, CC_E_HIP);
        }
        batch.clear();
        return;
    }
    L->reqs = batch;
    L->off = off;
    L->bytes = bytes;
    L->busy = true;
    s->n_small_launches += 1;
    batch.clear();
}

void complete_small(cc_server *s, SmallLaunch &L) {
    for (size_t i = 0; i < L.reqs.size(); ++i) {
        Request *r = L.reqs[i];
        r->rounds = L.h_rounds[i];
        s->live.erase(r->id);
        finish_locked(s, r, L.h[i].status ? CC_E_INPUT : (r->cancelled ? CC_E_STATE : CC_OK));
    }
    s->alloc.release(L.off, L.bytes);
    L.reqs.clear();
    L.busy = false;
}

// the server's streams, events and host buffers (its scheduler has stopped)
void free_server(cc_server *s) {
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto ev : s->events) (void)hipEventDestroy(ev);
    if (s->small_stream) (void)hipStreamDestroy(s->small_stream);
    for (auto &L : s->small) {
        if (L.h) (void)hipHostFree(L.h);
        if (L.ev) (void)hipEventDestroy(L.ev);
    }
    if (s->mirrors) {
        if (s->mirrors_pageable)
            free(s->mirrors);
        else
            (void)hipHostFree(s->mirrors);
    }
    delete s;
}

void worker_loop(cc_server *s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<Request *> small_batch;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        // completions
        for (size_t k = 0; k < s->slot_req.size(); ++k) {
            if (!s->slot_req[k] && !s->slot_cohort[k]) continue;
            if (hipEventQuery(s->events[k]) == hipSuccess) {
                if (s->slot_req[k])
                    advance_large(s, (int)k);
                else
                    advance_cohort(s, (int)k);
                progress = true;
            }
        }
        for (auto &L : s->small) {
            if (L.busy && hipEventQuery(L.ev) == hipSuccess) {
                complete_small(s, L);
                progress = true;
            }
        }
        // admission, in arrival order; a large request waiting for memory keeps later large
        // requests waiting too (no starvation), small ones may pass it
        bool large_blocked = false;
        const bool admitting = !s->paused || s->stop;
        for (auto it = s->pending.begin(); admitting && it != s->pending.end();) {
            Request *r = *it;
            if (r->cancelled) {
                s->live.erase(r->id);
                finish_locked(s, r, CC_E_STATE);
                it = s->pending.erase(it);
                progress = true;
                continue;
            }
            if (r->small) {
                if ((int)small_batch.size() < s->cfg.max_small_per_launch) {
                    small_batch.push_back(r);
                    it = s->pending.erase(it);
                    continue;
                }
                ++it;
                continue;
            }
            if (large_blocked) {
                ++it;
                continue;
            }
            int free_slot = -1;
            for (size_t k = 0; k < s->slot_req.size(); ++k)
                if (!s->slot_req[k] && !s->slot_cohort[k]) {
                    free_slot = (int)k;
                    break;
                }
            if (free_slot >= 0 && cohort_ok(s, r)) {
                // this request and the waiting ones after it that can join, up to cohort_max
                std::vector<Request *> co{r};
                const int cmax = std::min(s->cfg.cohort_max, kCohortMax);
                for (auto jt = std::next(it); jt != s->pending.end() && (int)co.size() < cmax; ++jt)
                    if (cohort_ok(s, *jt)) co.push_back(*jt);
                if (co.size() > 1 && admit_cohort(s, co, free_slot)) {
                    for (Request *q : co) s->pending.erase(std::find(s->pending.begin(), s->pending.end(), q));
                    progress = true;
                    break;   // the pending list changed: scan it again on the next pass
                }
            }
            if (free_slot < 0 || !admit_large(s, r, free_slot)) {
                large_blocked = true;
                ++it;
                continue;
            }
            it = s->pending.erase(it);
            progress = true;
        }
        if (!small_batch.empty()) {
            const size_t before = small_batch.size();
            launch_small_batch(s, small_batch);
            if (small_batch.empty()) {
                progress = true;
            } else {
                // no free launch or memory: put them back at the front, in order
                for (auto rit = small_batch.rbegin(); rit != small_batch.rend(); ++rit) s->pending.push_front(*rit);
                small_batch.clear();
                (void)before;
            }
        }
        bool active = !s->pending.empty() && admitting;
        for (auto *r : s->slot_req) active |= r != nullptr;
        for (auto *c : s->slot_cohort) active |= c != nullptr;
        for (auto &L : s->small) active |= L.busy;
        if (s->stop && !active && s->pending.empty()) break;
        if (!progress) {
            // device work in flight: poll again shortly; otherwise sleep until a submit
            if (active)
                s->cv.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv.wait(lk);
        }
    }
}

}  // namespace

extern "C" {

cc_status cc_server_create(void *d_arena, size_t budget_bytes, const cc_server_config *cfg, cc_server **out) {
    if (!out) return CC_E_ARG;
    *out = nullptr;
    if (!d_arena || (uintptr_t)d_arena % 256 != 0 || budget_bytes < 4096 || !cfg) return CC_E_ARG;
    if (cfg->n_slots < 1 || cfg->n_slots > 64 || cfg->small_variant < 0 || cfg->small_variant >= kNumSmallVariants ||
        (cfg->small_threads != 256 && cfg->small_threads != 512) || cfg->small_blocks_per_cu < 1 ||
        cfg->max_small_per_launch < 1 || cfg->max_small_per_launch > 65536 || cfg->small_launches < 1 ||
        cfg->small_launches > 8 || cfg->cohort_max < 0 || cfg->cohort_max > kCohortMax || cfg->cohort_max_vertices < 0)
        return CC_E_ARG;
    cc_server *s = new (std::nothrow) cc_server();
    if (!s) return CC_E_NOMEM;
    s->arena = (char *)d_arena;
    s->budget = budget_bytes;
    s->cfg = *cfg;
    s->alloc.init(budget_bytes);
    s->t0 = std::chrono::steady_clock::now();
    bool ok = true;
    if (cfg->small_variant > 0) {
        int dev = 0, lds = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (small_bytes(cfg->small_variant, cfg->small_threads) > (size_t)lds) ok = false;
        if (ok) ok = prepare_small(cfg->small_variant, cfg->small_threads) == hipSuccess;
    }
    for (int k = 0; ok && k < cfg->n_slots; ++k) {
        hipStream_t st;
        hipEvent_t ev;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (!ok) break;
        s->streams.push_back(st);
        ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (!ok) break;
        s->events.push_back(ev);
    }
    s->slot_req.assign(s->streams.size(), nullptr);
    s->slot_cohort.assign(s->streams.size(), nullptr);
    // pinned host memory for every slot, allocated once: a mirror of the round state and a
    // cohort's round counts (freeing pinned memory later would synchronise the whole device)
    const size_t host_bytes = (sizeof(RoundState) + 4 * (size_t)kCohortMax) * (size_t)cfg->n_slots;
    if (ok && hipHostMalloc((void **)&s->mirrors, host_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();   // pageable host memory still works, only slower to copy
        s->mirrors = (RoundState *)calloc(1, host_bytes);
        s->mirrors_pageable = true;
        ok = s->mirrors != nullptr;
    }
    if (ok) s->rounds_pinned = (int32_t *)(s->mirrors + cfg->n_slots);
    if (ok) ok = hipStreamCreateWithFlags(&s->small_stream, hipStreamNonBlocking) == hipSuccess;
    s->small.resize(cfg->small_launches);
    for (auto &L : s->small) {
        if (!ok) break;
        const size_t bytes = sizeof(SmallDesc) * cfg->max_small_per_launch + 4 * (size_t)cfg->max_small_per_launch;
        ok = hipHostMalloc((void **)&L.h, bytes, hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            L.h = nullptr;
            break;
        }
        L.h_rounds = (int32_t *)(L.h + cfg->max_small_per_launch);
        ok = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_server(s);
        return CC_E_HIP;
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return CC_OK;
}

cc_status cc_server_submit(cc_server *s, const cc_graph_desc *g, uint64_t seed, void *d_labels, uint64_t *req_id) {
    if (!s || !g || !req_id) return CC_E_ARG;
    if (g->n_vertices > 0 && !d_labels) return CC_E_ARG;
    if (g->n_vertices < 0 || g->n_vertices > 0x7FFFFFFFLL || g->n_edges < 0 || g->n_edges > 0xFFFFFFFELL ||
        g->layout < CC_EDGES_SOA_I32 || g->layout > CC_EDGES_PACKED_U64 || g->reserved != 0)
        return CC_E_ARG;
    if (g->n_edges > 0 && (!g->src || (g->layout != CC_EDGES_PACKED_U64 && !g->dst))) return CC_E_ARG;
    Request *r = new (std::nothrow) Request();
    if (!r) return CC_E_NOMEM;
    r->g = *g;
    r->seed = seed;
    r->labels = d_labels;
    r->small = small_ok(s, *g);
    r->footprint = r->small ? 0
                            : plan_workspace(g->n_vertices, g->n_edges, false,
                                             choose_tiled(g->n_vertices, g->n_edges, 0), nullptr, nullptr);
    if (r->footprint > s->budget) {
        delete r;
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = "request needs more device memory than the whole serving budget";
        return CC_E_BUDGET;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->pending.push_back(r);
        s->live[r->id] = r;
        *req_id = r->id;
    }
    s->cv.notify_all();
    return CC_OK;
}

static int32_t take_done(cc_server *s, cc_request_result *out, int32_t cap) {
    int32_t n = 0;
    while (n < cap && !s->done.empty()) {
        Request *r = s->done.front();
        s->done.erase(s->done.begin());
        cc_request_result &o = out[n++];
        o.id = r->id;
        o.status = r->status;
        o.rounds = r->rounds;
        o.small_path = r->small ? 1 : 0;
        o.cohort = r->cohort;
        o.t_submit = r->t_submit;
        o.t_admit = r->t_admit;
        o.t_done = r->t_done;
        delete r;
    }
    return n;
}

cc_status cc_server_poll(cc_server *s, cc_request_result *out, int32_t cap, int32_t *n) {
    if (!s || !n || (cap > 0 && !out)) return CC_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *n = take_done(s, out, cap);
    return CC_OK;
}

cc_status cc_server_wait(cc_server *s, cc_request_result *out, int32_t cap, int32_t *n, double timeout_s) {
    if (!s || !n || cap < 1 || !out) return CC_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !s->done.empty(); });
    *n = take_done(s, out, cap);
    return CC_OK;
}

cc_status cc_server_cancel(cc_server *s, uint64_t req_id) {
    if (!s) return CC_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->live.find(req_id);
        if (it == s->live.end()) return CC_E_ARG;
        it->second->cancelled = true;
    }
    s->cv.notify_all();
    return CC_OK;
}

cc_status cc_server_pause(cc_server *s, int32_t paused) {
    if (!s) return CC_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = paused != 0;
    }
    s->cv.notify_all();
    return CC_OK;
}

cc_status cc_server_info(cc_server *s, cc_server_info_t *info) {
    if (!s || !info) return CC_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    info->now = s->now();
    info->pending = (int64_t)s->pending.size();
    int64_t active = 0;
    for (auto *r : s->slot_req) active += r != nullptr;
    for (auto *c : s->slot_cohort) active += c ? (int64_t)c->reqs.size() : 0;
    for (auto &L : s->small) active += L.busy ? (int64_t)L.reqs.size() : 0;
    info->active = active;
    info->bytes_in_use = (int64_t)s->alloc.used;
    info->peak_bytes = (int64_t)s->peak_used;
    info->small_launches = s->n_small_launches;
    return CC_OK;
}

cc_status cc_server_destroy(cc_server *s) {
    if (!s) return CC_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto *r : s->pending) r->cancelled = true;
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto *r : s->done) delete r;
    free_server(s);
    return CC_OK;
}

const char *cc_server_last_error(const cc_server *s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
