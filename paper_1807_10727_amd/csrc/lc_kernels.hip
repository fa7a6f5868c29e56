// Round kernels of LocalContraction on gfx950.
//
// One round (one phase of the method, Section 3 "LocalContraction"):
//   round_begin  reset counters, m1 = lv = +inf (or rho), flags = 0 over the N_r nodes
//   min1         m1[x] = min over the closed neighbourhood N(x) of rho   (Section 2: x in N(x))
//   min2         lv[x] = min over N(x) of m1 = min over N(N(x)) of rho
//   parent       parent of x = the node whose priority is lv[x] (inverse of the bijection)
//   relabel      every record (a, b) -> (p(a), p(b)); loops dropped; survivors compacted
//   sort/unique  duplicates dropped (lc_sort.hip)
//   nodes/map    next node set, names, per-round map of the label composition; then the
//                unique write emits the next graph's edges in its compact index space
//   round_end    advance the device state
// Merged nodes are named by the original id of their parent vertex, and the per-round
// maps are composed at the end into the label of every original vertex.
//
// In round 0 (and in batches) both min passes fold the node's own priority into each update
// (min(rho(a), rho(b)) is sent to both endpoints), so the +inf fill replaces an
// initialisation pass; ids without a loop-free record keep +inf and are their own parent.
// From round 1 on every node has a record, and round_begin seeds the node words with the
// own priority instead, so that the one-hop pass needs no name lookups.  Each update first reads the
// current value and only issues the atomic when it can lower it: values only decrease, so
// a stale read can only cause a redundant atomic, never a missed one.

#include "lc_steps.hpp"

namespace lc {

// ---------------------------------------------------------------------------------------
// priorities of nodes
// ---------------------------------------------------------------------------------------

template <bool kFirst, bool kBatch>
__device__ inline uint32_t node_prio(const PrioCtx &pc, const Work &w, const uint32_t *names, const uint32_t *gids,
                                     uint32_t i) {
    const uint32_t name = kFirst ? i : names[i];
    if (!kBatch) return rho_of(pc, name);
    const uint32_t g = kFirst ? w.gid0[i] : gids[i];
    return prio(pc.keys[g], name - pc.voff[g]);
}

// ---------------------------------------------------------------------------------------

template <bool kSeeded>
__global__ __launch_bounds__(kThreads) void k_round_begin(Work w, const uint32_t *names, const uint32_t *tab) {
    step_round_begin<kSeeded>(w, names, tab);
}

__global__ __launch_bounds__(kThreads) void k_min1_seeded(ReadInternal rd, Work w) {
    step_min1_seeded(rd, w);
}

template <class R, bool kFirst, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_min1(R rd, Work w, PrioCtx pc, const uint32_t *names,
                                                   const uint32_t *gids) {
    constexpr int V = R::kV;
    rd.init(w.st);
    if (!kBatch) pc.key = w.st->key;
    const int64_t nch = rd.chunks();
    uint32_t *m1 = w.ml;   // one-hop minimum of node x at m1[2x]
    bool bad = false;
    // grid-stride with a loop bound that is uniform per wave, so the wave shuffles of the
    // sorted variant always see every lane
    for (int64_t cb = (int64_t)blockIdx.x * kThreads; cb < nch; cb += (int64_t)gridDim.x * kThreads) {
        const int64_t c = cb + threadIdx.x;
        uint32_t a[V], b[V], v[V], ca[V], cb_[V];
        bool ok[V];
        if (c < nch) {
            rd.read(c, a, b, bad);
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) a[j] = b[j] = 0u;
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            ok[j] = a[j] != b[j];
            v[j] = kInf;
            if (ok[j]) {
                uint32_t pa = node_prio<kFirst, kBatch>(pc, w, names, gids, a[j]);
                uint32_t pb = node_prio<kFirst, kBatch>(pc, w, names, gids, b[j]);
                v[j] = min(pa, pb);
            }
        }
        bool la[V];
        uint32_t va[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (R::kSorted) {
                va[j] = run_min(ok[j] ? a[j] : 0xFFFFFFFFu, v[j], la[j]);
            } else {
                va[j] = v[j];
                la[j] = true;
            }
            if (ok[j]) {
                if (la[j]) ca[j] = m1[2 * (size_t)a[j]];
                cb_[j] = m1[2 * (size_t)b[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (ok[j]) {
                if (la[j] && ca[j] > va[j]) atomicMin(&m1[2 * (size_t)a[j]], va[j]);
                if (cb_[j] > v[j]) atomicMin(&m1[2 * (size_t)b[j]], v[j]);
            }
        }
    }
    if (bad) atomicOr(&w.st->err, 1u);
}

template <class R>
__global__ __launch_bounds__(kThreads) void k_min2(R rd, Work w) {
    step_min2<R>(rd, w);
}

template <bool kFirst, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_parent(Work w, PrioCtx pc, const uint32_t *gids, int word) {
    step_parent<kFirst, kBatch>(w, pc, gids, word);
}

template <class R>
__global__ __launch_bounds__(kThreads) void k_relabel(R rd, Work w) {
    step_relabel<R>(rd, w);
}

// The label ranks, and (one thread) the key width of the round's sort, which needs only the
// label count that the label map's scan has already written.
__global__ __launch_bounds__(kThreads) void k_rank_parents(Work w) {
    step_rank_parents(w);
    if (blockIdx.x == 0 && threadIdx.x == 0) step_plan_blocks(w);
}

template <bool kFirst, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_nodes(Work w, const uint32_t *names_cur, uint32_t *names_next,
                                                    const uint32_t *gids_cur, uint32_t *gids_next) {
    step_nodes<kFirst, kBatch>(w, names_cur, names_next, gids_cur, gids_next);
}

template <bool kFirst>
__global__ __launch_bounds__(kThreads) void k_map(Work w, const uint32_t *names_cur) {
    step_map<kFirst>(w, names_cur);
}

template <bool kFirst>
__global__ void k_round_end(Work w, int dedup) {
    step_round_end<kFirst>(w, dedup);
}

// label of every original vertex: chase its map0 entry through the kept levels
template <bool kOut64, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_compose(Work w, int identity, const uint32_t *names_cur,
                                                      void *labels, const uint32_t *voff) {
    const RoundState *st = w.st;
    const int levels = st->levels;
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < w.n0; v += (int64_t)gridDim.x * kThreads) {
        uint32_t name;
        if (identity) {
            name = (uint32_t)v;
        } else {
            uint32_t x = w.map0[v];
            for (int l = 0; l < levels && !(x & kFinal); ++l) x = w.maps[st->level_off[l] + x];
            name = (x & kFinal) ? (x & ~kFinal) : (names_cur ? names_cur[x] : x);
        }
        const uint32_t lab = kBatch ? name - voff[w.gid0[v]] : name;
        if (kOut64)
            ((int64_t *)labels)[v] = (int64_t)lab;
        else
            ((int32_t *)labels)[v] = (int32_t)lab;
    }
}

// Folding the per-round maps, last level first: level l - 1 (the map of one round's nodes
// into the next round's) is composed with level l, so that after every fold level 0 maps
// straight to the last level's targets.  The levels shrink round by round, so the folds
// cost far less than chasing every vertex through every level.
__global__ __launch_bounds__(kThreads) void k_fold_level(Work w, int l) {
    const RoundState *st = w.st;
    if (l <= 0 || l >= st->levels) return;
    const int64_t a = (int64_t)st->level_off[l - 1], b = (int64_t)st->level_off[l];
    for (int64_t i = a + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < b; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t x = w.maps[i];
        if (!(x & kFinal)) w.maps[i] = w.maps[b + x];
    }
}

// map0 through the folded level 0: every vertex then maps to a final name or to a node of
// the current graph, and the arena is empty again.  `folded`: the levels the host folded
// (a device with more would hold unfolded levels: flagged as an inconsistency).
__global__ __launch_bounds__(kThreads) void k_flatten(Work w, int folded) {
    RoundState *st = w.st;
    const int levels = st->levels;
    if (levels > (folded > 1 ? folded : 1)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->err, 4u);
        return;
    }
    const int64_t off0 = (int64_t)st->level_off[0];
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < w.n0; v += (int64_t)gridDim.x * kThreads) {
        const uint32_t x = w.map0[v];
        if (levels > 0 && !(x & kFinal)) w.map0[v] = w.maps[off0 + x];
    }
}

__global__ void k_flatten_reset(Work w) {
    w.st->levels = 0;
    w.st->map_off = 0;
}

template <bool kOut64, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_canon_min(Work w, const void *labels, const uint32_t *voff) {
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < w.n0; v += (int64_t)gridDim.x * kThreads) {
        uint32_t lab = kOut64 ? (uint32_t)((const int64_t *)labels)[v] : (uint32_t)((const int32_t *)labels)[v];
        const uint32_t base = kBatch ? voff[w.gid0[v]] : 0u;
        atomicMin(&w.newidx[lab + base], (uint32_t)v);
    }
}

template <bool kOut64, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_canon_apply(Work w, void *labels, const uint32_t *voff) {
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < w.n0; v += (int64_t)gridDim.x * kThreads) {
        uint32_t lab = kOut64 ? (uint32_t)((const int64_t *)labels)[v] : (uint32_t)((const int32_t *)labels)[v];
        const uint32_t base = kBatch ? voff[w.gid0[v]] : 0u;
        const uint32_t c = w.newidx[lab + base] - base;
        if (kOut64)
            ((int64_t *)labels)[v] = (int64_t)c;
        else
            ((int32_t *)labels)[v] = (int32_t)c;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = v;
}

// parents of the round that just ended, by name (inspection aid; par holds label ranks).
// In round 0 an id without a loop-free record has no parent and is nobody's (it is in no
// neighbourhood): it is reported as not being a node.
__global__ __launch_bounds__(kThreads) void k_dump_parents(Work w, int first, const uint32_t *names_prev,
                                                           int32_t *out) {
    const int64_t n = (int64_t)w.st->n_prev;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        if (w.par[i] == kNoParent) continue;
        const uint32_t p = w.lab_at[w.par[i]];
        const uint32_t x = first ? (uint32_t)i : names_prev[i];
        out[x] = (int32_t)(first ? p : names_prev[p]);
    }
}

// The edges of the next graph by name (cc_round_edges): each record (a, b) of node indices
// becomes (smaller name << 32) | larger name.
__global__ __launch_bounds__(kThreads) void k_dump_edges(Work w, const uint32_t *names, uint64_t *out) {
    const RoundState *st = w.st;
    const int64_t m = (int64_t)st->m_cur;
    const uint64_t *rec = w.keys[st->e_sel];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m; i += (int64_t)gridDim.x * kThreads) {
        const uint64_t r = rec[i];
        const uint32_t a = names[(uint32_t)(r >> 32)], b = names[(uint32_t)r];
        out[i] = ((uint64_t)min(a, b) << 32) | max(a, b);
    }
}

// per-graph round keys of the current round (the round index is read on the device, so
// the launch can be replayed from a captured graph)
__global__ void k_batch_keys(Work w, RoundKey *keys, const uint64_t *seeds, int32_t g) {
    const int32_t round = w.st->round;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g; i += gridDim.x * blockDim.x)
        keys[i] = round_key(seeds[i], round);
}

__global__ __launch_bounds__(kThreads) void k_fill_gid(uint32_t *gid0, const uint32_t *voff, int32_t g) {
    for (int32_t j = blockIdx.x; j < g; j += gridDim.x)
        for (uint32_t v = voff[j] + threadIdx.x; v < voff[j + 1]; v += kThreads) gid0[v] = (uint32_t)j;
}

// ---------------------------------------------------------------------------------------
// explicit priorities, round records and inspection (off the measured path)
// ---------------------------------------------------------------------------------------

// inv[tab[x]] = x; a value outside [0, n0) sets err bit 3
__global__ __launch_bounds__(kThreads) void k_prio_inverse(Work w, const uint32_t *tab) {
    bool bad = false;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < w.n0; x += (int64_t)gridDim.x * kThreads) {
        const uint32_t t = tab[x];
        if ((int64_t)t < w.n0)
            w.pinv[t] = (uint32_t)x;
        else
            bad = true;
    }
    if (bad) atomicOr(&w.st->err, 8u);
}

// A table whose values all lie in [0, n0) is a permutation iff no two names share a value,
// i.e. iff every name reads itself back through the inverse.
__global__ __launch_bounds__(kThreads) void k_prio_inverse_check(Work w, const uint32_t *tab) {
    bool bad = false;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < w.n0; x += (int64_t)gridDim.x * kThreads) {
        const uint32_t t = tab[x];
        if ((int64_t)t < w.n0 && w.pinv[t] != (uint32_t)x) bad = true;
    }
    if (bad) atomicOr(&w.st->err, 8u);
}

// Parent of node i of the round that just ended, as a name (kNoParent: not a node).
__device__ inline uint32_t parent_name(const Work &w, int first, const uint32_t *names_prev, int64_t i) {
    const uint32_t q = w.par[i];
    if (q == kNoParent) return kNoParent;
    const uint32_t p = w.lab_at[q];
    return first ? p : names_prev[p];
}

__global__ __launch_bounds__(kThreads) void k_record_parents(Work w, int first, const uint32_t *names_prev,
                                                             uint32_t *rec) {
    const int64_t n = (int64_t)w.st->n_prev;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t p = parent_name(w, first, names_prev, i);
        if (first) {
            rec[i] = p;
        } else {
            rec[2 * i] = names_prev[i];
            rec[2 * i + 1] = p;
        }
    }
}

// out (filled with -1 before) receives the recorded parents by name
__global__ __launch_bounds__(kThreads) void k_expand_record(Work w, int first, const uint32_t *rec, int64_t count,
                                                            int32_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count; i += (int64_t)gridDim.x * kThreads) {
        if (first) {
            out[i] = (int32_t)rec[i];
        } else {
            const uint32_t x = rec[2 * i];
            if ((int64_t)x < w.n0) out[x] = (int32_t)rec[2 * i + 1];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_dump_minima(Work w, int first, int dense, PrioCtx pc,
                                                          const uint32_t *names_prev, uint32_t *m1o, uint32_t *l2o) {
    const RoundState *st = w.st;
    if (!pc.tab) pc.key = st->key;   // the key of the round that just ended
    const int64_t n = (int64_t)st->n_prev;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t p = parent_name(w, first, names_prev, i);
        if (p == kNoParent) continue;
        const uint32_t x = first ? (uint32_t)i : names_prev[i];
        if (dense) {
            m1o[x] = w.ml[i];
            l2o[x] = rho_of(pc, p);
        } else {
            m1o[x] = w.ml[2 * i];
            l2o[x] = w.ml[2 * i + 1];
        }
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

#define LC_LAUNCH(kern, grid, ...)                                            \
    do {                                                                      \
        hipLaunchKernelGGL((kern), dim3(grid), dim3(kThreads), 0, s, __VA_ARGS__); \
        return hipGetLastError();                                             \
    } while (0)

hipError_t launch_round_begin(const Work &w, bool seeded, int round, int grid, hipStream_t s, const uint32_t *tab) {
    const uint32_t *names = w.names[round & 1];
    if (seeded) LC_LAUNCH(k_round_begin<true>, grid, w, names, tab);
    LC_LAUNCH(k_round_begin<false>, grid, w, names, tab);
}

template <bool kBatch>
static hipError_t min1_in(const Work &w, const EdgeIn &e, const PrioCtx &p, int grid, hipStream_t s) {
    const uint32_t *nul = nullptr;
    switch (e.layout) {
        case kSoa32:
            if (e.vec) LC_LAUNCH((k_min1<ReadSoa32<4>, true, kBatch>), grid, ReadSoa32<4>(e), w, p, nul, nul);
            LC_LAUNCH((k_min1<ReadSoa32<1>, true, kBatch>), grid, ReadSoa32<1>(e), w, p, nul, nul);
        case kSoa64:
            if (e.vec) LC_LAUNCH((k_min1<ReadSoa64<2>, true, kBatch>), grid, ReadSoa64<2>(e), w, p, nul, nul);
            LC_LAUNCH((k_min1<ReadSoa64<1>, true, kBatch>), grid, ReadSoa64<1>(e), w, p, nul, nul);
        default:
            if (e.vec) LC_LAUNCH((k_min1<ReadPacked<2>, true, kBatch>), grid, ReadPacked<2>(e), w, p, nul, nul);
            LC_LAUNCH((k_min1<ReadPacked<1>, true, kBatch>), grid, ReadPacked<1>(e), w, p, nul, nul);
    }
}

hipError_t launch_min1(const Work &w, const EdgeIn *in, const PrioCtx &p, bool batch, int round, int grid,
                       hipStream_t s) {
    if (in) return batch ? min1_in<true>(w, *in, p, grid, s) : min1_in<false>(w, *in, p, grid, s);
    const uint32_t *names = w.names[round & 1];
    const uint32_t *gids = w.gids[round & 1];
    if (batch) LC_LAUNCH((k_min1<ReadInternal, false, true>), grid, ReadInternal(w), w, p, names, gids);
    LC_LAUNCH(k_min1_seeded, grid, ReadInternal(w), w);
}

hipError_t launch_min2(const Work &w, const EdgeIn *in, int grid, hipStream_t s) {
    if (!in) LC_LAUNCH(k_min2<ReadInternal>, grid, ReadInternal(w), w);
    const EdgeIn &e = *in;
    switch (e.layout) {
        case kSoa32:
            if (e.vec) LC_LAUNCH(k_min2<ReadSoa32<4>>, grid, ReadSoa32<4>(e), w);
            LC_LAUNCH(k_min2<ReadSoa32<1>>, grid, ReadSoa32<1>(e), w);
        case kSoa64:
            if (e.vec) LC_LAUNCH(k_min2<ReadSoa64<2>>, grid, ReadSoa64<2>(e), w);
            LC_LAUNCH(k_min2<ReadSoa64<1>>, grid, ReadSoa64<1>(e), w);
        default:
            if (e.vec) LC_LAUNCH(k_min2<ReadPacked<2>>, grid, ReadPacked<2>(e), w);
            LC_LAUNCH(k_min2<ReadPacked<1>>, grid, ReadPacked<1>(e), w);
    }
}

hipError_t launch_parent(const Work &w, const PrioCtx &p, bool batch, int round, int grid, hipStream_t s,
                         bool one_hop) {
    const uint32_t *gids = w.gids[round & 1];
    const int word = one_hop ? 0 : 1;
    if (round == 0) {
        if (batch) LC_LAUNCH((k_parent<true, true>), grid, w, p, gids, word);
        LC_LAUNCH((k_parent<true, false>), grid, w, p, gids, word);
    }
    if (batch) LC_LAUNCH((k_parent<false, true>), grid, w, p, gids, word);
    LC_LAUNCH((k_parent<false, false>), grid, w, p, gids, word);
}

hipError_t launch_relabel(const Work &w, const EdgeIn *in, int grid, hipStream_t s) {
    if (!in) LC_LAUNCH(k_relabel<ReadInternal>, grid, ReadInternal(w), w);
    const EdgeIn &e = *in;
    switch (e.layout) {
        case kSoa32:
            if (e.vec) LC_LAUNCH(k_relabel<ReadSoa32<4>>, grid, ReadSoa32<4>(e), w);
            LC_LAUNCH(k_relabel<ReadSoa32<1>>, grid, ReadSoa32<1>(e), w);
        case kSoa64:
            if (e.vec) LC_LAUNCH(k_relabel<ReadSoa64<2>>, grid, ReadSoa64<2>(e), w);
            LC_LAUNCH(k_relabel<ReadSoa64<1>>, grid, ReadSoa64<1>(e), w);
        default:
            if (e.vec) LC_LAUNCH(k_relabel<ReadPacked<2>>, grid, ReadPacked<2>(e), w);
            LC_LAUNCH(k_relabel<ReadPacked<1>>, grid, ReadPacked<1>(e), w);
    }
}

hipError_t launch_rank_parents(const Work &w, int grid, int grid_scan, hipStream_t s) {
    hipError_t e = hipSuccess;
    if (grid_scan == 0) {   // one workgroup
        e = launch_map_scan(w, true, 1, s, 3);
    } else {
        for (int stage = 0; stage < 3 && e == hipSuccess; ++stage)
            e = launch_map_scan(w, true, stage == 1 ? 1 : grid_scan, s, stage);
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_parents, dim3(grid), dim3(kThreads), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_nodes(const Work &w, bool batch, int round, int grid, hipStream_t s) {
    const uint32_t *nc = w.names[round & 1];
    uint32_t *nn = w.names[(round + 1) & 1];
    const uint32_t *gc = w.gids[round & 1];
    uint32_t *gn = w.gids[(round + 1) & 1];
    if (round == 0) {
        if (batch) LC_LAUNCH((k_nodes<true, true>), grid, w, nc, nn, gc, gn);
        LC_LAUNCH((k_nodes<true, false>), grid, w, nc, nn, gc, gn);
    }
    if (batch) LC_LAUNCH((k_nodes<false, true>), grid, w, nc, nn, gc, gn);
    LC_LAUNCH((k_nodes<false, false>), grid, w, nc, nn, gc, gn);
}

hipError_t launch_map(const Work &w, int round, int grid, hipStream_t s) {
    if (round == 0) LC_LAUNCH(k_map<true>, grid, w, (const uint32_t *)nullptr);
    LC_LAUNCH(k_map<false>, grid, w, (const uint32_t *)w.names[round & 1]);
}

hipError_t launch_round_end(const Work &w, int round, int dedup, hipStream_t s) {
    if (round == 0) {
        hipLaunchKernelGGL(k_round_end<true>, dim3(1), dim3(1), 0, s, w, dedup);
    } else {
        hipLaunchKernelGGL(k_round_end<false>, dim3(1), dim3(1), 0, s, w, dedup);
    }
    return hipGetLastError();
}

hipError_t launch_compose(const Work &w, bool identity, int cur_round, void *labels, bool out64, bool batch,
                          const uint32_t *voff, int grid, hipStream_t s) {
    const uint32_t *names_cur = cur_round == 0 ? nullptr : w.names[cur_round & 1];
    const int id = identity ? 1 : 0;
    if (out64) {
        if (batch) LC_LAUNCH((k_compose<true, true>), grid, w, id, names_cur, labels, voff);
        LC_LAUNCH((k_compose<true, false>), grid, w, id, names_cur, labels, voff);
    }
    if (batch) LC_LAUNCH((k_compose<false, true>), grid, w, id, names_cur, labels, voff);
    LC_LAUNCH((k_compose<false, false>), grid, w, id, names_cur, labels, voff);
}

hipError_t launch_flatten(const Work &w, int levels, int grid, hipStream_t s) {
    for (int l = levels - 1; l >= 1; --l) {
        hipLaunchKernelGGL(k_fold_level, dim3(grid), dim3(kThreads), 0, s, w, l);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_flatten, dim3(grid), dim3(kThreads), 0, s, w, levels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_flatten_reset, dim3(1), dim3(1), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_canonical(const Work &w, void *labels, bool out64, bool batch, const uint32_t *voff, int grid,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kThreads), 0, s, w.newidx, kInf, w.n0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (out64) {
        if (batch) {
            hipLaunchKernelGGL((k_canon_min<true, true>), dim3(grid), dim3(kThreads), 0, s, w, labels, voff);
            LC_LAUNCH((k_canon_apply<true, true>), grid, w, labels, voff);
        }
        hipLaunchKernelGGL((k_canon_min<true, false>), dim3(grid), dim3(kThreads), 0, s, w, labels, voff);
        LC_LAUNCH((k_canon_apply<true, false>), grid, w, labels, voff);
    }
    if (batch) {
        hipLaunchKernelGGL((k_canon_min<false, true>), dim3(grid), dim3(kThreads), 0, s, w, labels, voff);
        LC_LAUNCH((k_canon_apply<false, true>), grid, w, labels, voff);
    }
    hipLaunchKernelGGL((k_canon_min<false, false>), dim3(grid), dim3(kThreads), 0, s, w, labels, voff);
    LC_LAUNCH((k_canon_apply<false, false>), grid, w, labels, voff);
}

hipError_t launch_dump_parents(const Work &w, int32_t *out, int last_round, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kThreads), 0, s, (uint32_t *)out, 0xFFFFFFFFu, w.n0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LC_LAUNCH(k_dump_parents, grid, w, last_round == 0 ? 1 : 0, (const uint32_t *)w.names[last_round & 1], out);
}

hipError_t launch_prio_inverse(const Work &w, const uint32_t *tab, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_prio_inverse, dim3(grid), dim3(kThreads), 0, s, w, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LC_LAUNCH(k_prio_inverse_check, grid, w, tab);
}

hipError_t launch_record_parents(const Work &w, int round, uint32_t *rec, int grid, hipStream_t s) {
    LC_LAUNCH(k_record_parents, grid, w, round == 0 ? 1 : 0, (const uint32_t *)w.names[round & 1], rec);
}

hipError_t launch_expand_record(const Work &w, int round, const uint32_t *rec, int64_t count, int32_t *out,
                                int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kThreads), 0, s, (uint32_t *)out, 0xFFFFFFFFu, w.n0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LC_LAUNCH(k_expand_record, grid, w, round == 0 ? 1 : 0, rec, count, out);
}

hipError_t launch_dump_minima(const Work &w, int last_round, bool dense_m1, const PrioCtx &p, uint32_t *m1,
                              uint32_t *l2, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kThreads), 0, s, m1, kInf, w.n0);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kThreads), 0, s, l2, kInf, w.n0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LC_LAUNCH(k_dump_minima, grid, w, last_round == 0 ? 1 : 0, dense_m1 ? 1 : 0, p,
              (const uint32_t *)w.names[last_round & 1], m1, l2);
}

hipError_t launch_dump_edges(const Work &w, uint64_t *out, int next_round, int grid, hipStream_t s) {
    LC_LAUNCH(k_dump_edges, grid, w, (const uint32_t *)w.names[next_round & 1], out);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, int grid, hipStream_t s) {
    LC_LAUNCH(k_fill_u32, grid, p, v, n);
}

hipError_t launch_batch_keys(const Work &w, RoundKey *keys, const uint64_t *seeds, int32_t n_graphs, hipStream_t s) {
    int grid = (int)ceil_div(n_graphs, kThreads);
    if (grid < 1) grid = 1;
    LC_LAUNCH(k_batch_keys, grid, w, keys, seeds, n_graphs);
}

hipError_t launch_fill_gid(uint32_t *gid0, const uint32_t *voff, int32_t n_graphs, int grid, hipStream_t s) {
    LC_LAUNCH(k_fill_gid, grid, gid0, voff, n_graphs);
}

}  // namespace lc
