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

#include "lc_internal.hpp"
#include "lc_readers.hpp"

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

__device__ inline int ceil_log2(uint64_t n) { return n <= 1 ? 0 : 64 - __clzll((long long)(n - 1)); }


// ---------------------------------------------------------------------------------------

// kSeeded (plain solve, rounds >= 1, where every node has a loop-free record): both halves of
// the node word start at the node's own priority rather than +inf.  The one-hop minimum over
// the closed neighbourhood then only needs the far endpoint's priority, which the same 8-byte
// load that fetches the current minimum brings along; the two-hop accumulator may start at
// rho(x) because it ends at most at m1[x] <= rho(x).
template <bool kSeeded>
__global__ __launch_bounds__(kThreads) void k_round_begin(Work w, const uint32_t *names, const uint32_t *tab) {
    RoundState *st = w.st;
    const int64_t n = (int64_t)st->n_cur;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_active = 0;
        st->s_count = 0;
        st->s_keys = 0;
        st->n_slabs = 0;
        st->m_next = 0;
        st->n_next = 0;
        st->n_final = 0;
        st->n_labels = 0;
        st->kb = ceil_log2(n < 2 ? 2 : (uint64_t)n);
        st->hb_shift = st->kb;
        st->nbits = 2 * st->kb;
        st->key = round_key(st->seed, st->round);
    }
    RoundKey key{};
    if (kSeeded) key = round_key(st->seed, st->round);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        uint64_t v = ~0ull;
        if (kSeeded) {
            const uint64_t p = tab ? tab[names[i]] : prio(key, names[i]);
            v = (p << 32) | p;
        }
        ((uint64_t *)w.ml)[i] = v;
        w.is_label[i] = 0;
        w.has_edge[i] = 0;
    }
}

// One-hop minimum, plain solve, rounds >= 1 (node words seeded with the own priority): each
// record sends rho(b) to a and rho(a) to b, read from the high halves of the two words.
__global__ __launch_bounds__(kThreads) void k_min1_seeded(ReadInternal rd, Work w) {
    constexpr int V = ReadInternal::kV;
    rd.init(w.st);
    const int64_t nch = rd.chunks();
    const uint64_t *word = (const uint64_t *)w.ml;
    uint32_t *m1 = w.ml;
    bool bad = false;
    for (int64_t cb = (int64_t)blockIdx.x * kThreads; cb < nch; cb += (int64_t)gridDim.x * kThreads) {
        const int64_t c = cb + threadIdx.x;
        uint32_t a[V], b[V];
        uint64_t wa[V], wb[V];
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
            wa[j] = wb[j] = ~0ull;
            if (ok[j]) {
                wa[j] = word[a[j]];
                wb[j] = word[b[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t pa = (uint32_t)(wa[j] >> 32), pb = (uint32_t)(wb[j] >> 32);
            bool la;
            const uint32_t va = run_min(ok[j] ? a[j] : 0xFFFFFFFFu, pb, la);
            if (ok[j]) {
                if (la && (uint32_t)wa[j] > va) atomicMin(&m1[2 * (size_t)a[j]], va);
                if ((uint32_t)wb[j] > pa) atomicMin(&m1[2 * (size_t)b[j]], pa);
            }
        }
    }
    if (bad) atomicOr(&w.st->err, 1u);
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
    constexpr int V = R::kV;
    rd.init(w.st);
    const int64_t nch = rd.chunks();
    const uint64_t *word = (const uint64_t *)w.ml;   // low half: one-hop min, high half: two-hop min
    uint32_t *ml = w.ml;
    bool bad = false;
    for (int64_t cb = (int64_t)blockIdx.x * kThreads; cb < nch; cb += (int64_t)gridDim.x * kThreads) {
        const int64_t c = cb + threadIdx.x;
        uint32_t a[V], b[V];
        uint64_t wa[V], wb[V];
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
            if (ok[j]) {
                wa[j] = word[a[j]];
                wb[j] = word[b[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t v = ok[j] ? min((uint32_t)wa[j], (uint32_t)wb[j]) : kInf;
            bool la = true;
            const uint32_t va = R::kSorted ? run_min(ok[j] ? a[j] : 0xFFFFFFFFu, v, la) : v;
            if (ok[j]) {
                if (la && (uint32_t)(wa[j] >> 32) > va) atomicMin(&ml[2 * (size_t)a[j] + 1], va);
                if ((uint32_t)(wb[j] >> 32) > v) atomicMin(&ml[2 * (size_t)b[j] + 1], v);
            }
        }
    }
}

// word 1: the two-hop minimum (LocalContraction); word 0: the one-hop minimum (one-hop label)
template <bool kFirst, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_parent(Work w, PrioCtx pc, const uint32_t *gids, int word) {
    RoundState *st = w.st;
    if (!kBatch) pc.key = st->key;
    const int64_t n = (int64_t)st->n_cur;
    uint32_t active = 0;
    bool broken = false;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t l = w.ml[2 * i + word];
        if (l == kInf) {  // no loop-free record touches this id (round 0 only)
            w.par[i] = (uint32_t)i;
            continue;
        }
        uint32_t name;
        if (!kBatch) {
            name = rho_name(pc, l, w.n0);
        } else {
            const uint32_t g = kFirst ? w.gid0[i] : gids[i];
            name = prio_inv(pc.keys[g], l) + pc.voff[g];
        }
        uint32_t p;
        if (kFirst) {
            p = name;
        } else {
            p = (int64_t)name < w.n0 ? w.idx_of[name] : 0xFFFFFFFFu;
        }
        if ((int64_t)p >= n) {  // cannot happen for a consistent state; never index out of range
            broken = true;
            p = (uint32_t)i;
        }
        w.par[i] = p;
        w.is_label[p] = 1;
        if (kBatch) w.g_rounds[kFirst ? w.gid0[i] : gids[i]] = st->round + 1;
        ++active;
    }
    __shared__ uint32_t red[kThreads / kWave];
    active = block_sum<kThreads>(active, red);   // one atomic per workgroup
    if (threadIdx.x == 0 && active) atomicAdd(&st->n_active, (u64c)active);
    if (broken) atomicOr(&st->err, 4u);
}

// Workgroup-local set of sort keys already written (sorted records, i.e. rounds >= 1).
constexpr int kDedupLog2 = LC_DEDUP_LOG2;   // slots: 1 << kDedupLog2
constexpr int kDedupProbes = 8;
constexpr unsigned long long kNoKey = ~0ull;   // no sort key has all 64 bits set (lo < hi)

// False when `key` is in the set already; true when it was added now, or when its probes
// all met other keys (the key is then written again: later passes drop any repeat).
template <int kLog2 = kDedupLog2>
__device__ inline bool set_insert(unsigned long long *set, uint64_t key) {
    if (key == kNoKey) return true;
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - kLog2));
    for (int p = 0; p < kDedupProbes; ++p) {
        const unsigned long long old = atomicCAS(&set[h], kNoKey, (unsigned long long)key);
        if (old == kNoKey) return true;
        if (old == key) return false;
        h = (h + 1) & ((1 << kLog2) - 1);
    }
    return true;
}

// Round 0 read directly from the caller's records: the same per-workgroup set, smaller (the
// unsorted records repeat only on power-law inputs), switched off by a workgroup once
// kInputSetTrial of its keys found fewer than 1/16 repeats (uniform random inputs, where the
// probes would cost more than they save).
constexpr int kInputSetLog2 = 11;
constexpr uint32_t kInputSetTrial = 4096;

// Relabel every record through the parents and keep the loop-free ones as sort keys
// (edge_key of (min, max) of the two parents).  Each workgroup owns a slab of kSlab
// consecutive records and writes its survivors, in order, to the start of the same slab of
// the output: no global counter is involved (one shared cursor, taken per chunk, measured
// slower: the first chunks of every workgroup all write and contend on it).  slab_cnt holds
// the keys per slab; the first radix pass reads the slabs.
//
// A workgroup also drops every key it has written before: a dense region that contracts
// onto a few parents maps many records onto the same parent pairs (rounds >= 1, and round 0
// of power-law inputs), and a hash set in LDS (kept for the whole launch) removes most of
// those repeats before they reach the sort.  s_count still counts every survivor; s_keys
// counts the keys.
template <class R>
__global__ __launch_bounds__(kThreads) void k_relabel(R rd, Work w) {
    constexpr int V = R::kV;
    constexpr bool kDedup = true;
    constexpr bool kAdaptive = !R::kSorted;
    constexpr int kSetLog2 = R::kSorted ? kDedupLog2 : kInputSetLog2;
    constexpr int64_t kChunksPerSlab = kSlab / V;
    RoundState *st = w.st;
    __shared__ uint32_t lds[kThreads / kWave + 1];
    __shared__ unsigned long long set[1 << kSetLog2];
    __shared__ uint32_t set_tries, set_drops, set_on;
    for (int i = threadIdx.x; i < (1 << kSetLog2); i += kThreads) set[i] = kNoKey;
    if (threadIdx.x == 0) {
        set_tries = 0;
        set_drops = 0;
        set_on = 1;
    }
    __syncthreads();
    rd.init(st);
    const int64_t nch = rd.chunks();
    const int64_t nslabs = ceil_div(rd.records(), kSlab);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->n_slabs = (u64c)nslabs;
        st->keys_dense = 0;
    }
    uint64_t *out = w.keys[sort_src(st->round, st->e_sel)];
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    bool bad = false;
    uint32_t survived = 0;   // this thread's loop-free records
    uint64_t written = 0;    // this workgroup's keys (thread 0)
    for (int64_t slab = blockIdx.x; slab < nslabs; slab += gridDim.x) {
        const int64_t c_end = min(nch, (slab + 1) * kChunksPerSlab);
        uint64_t *dst = out + slab * kSlab;
        uint32_t cursor = 0;
        for (int64_t cb = slab * kChunksPerSlab; cb < c_end; cb += kThreads) {
            const int64_t c = cb + threadIdx.x;
            uint64_t key[V];
            bool keep[V];
            uint32_t cnt = 0, tries = 0, drops = 0;
            // read without a barrier: either value is valid
            const bool use_set = !kAdaptive || (set_on != 0 && !w.round0_sets_off);
            if (c < c_end) {
                uint32_t a[V], b[V], pa[V], pb[V];
                rd.read(c, a, b, bad);
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    pa[j] = a[j] != b[j] ? w.par[a[j]] : 0u;
                    pb[j] = a[j] != b[j] ? w.par[b[j]] : 0u;
                }
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    keep[j] = pa[j] != pb[j];
                    survived += keep[j];
                    const uint32_t lo = min(pa[j], pb[j]), hi = max(pa[j], pb[j]);
                    key[j] = edge_key(lo, hi, kb, hbs);
                    if (kDedup && use_set && keep[j]) {
                        ++tries;
                        keep[j] = set_insert<kSetLog2>(set, key[j]);
                        drops += !keep[j];
                    }
                    cnt += keep[j];
                }
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) keep[j] = false;
            }
            if (kAdaptive && tries) {
                atomicAdd(&set_tries, tries);
                if (drops) atomicAdd(&set_drops, drops);
            }
            uint32_t total;
            uint32_t off = cursor + block_excl_scan<kThreads>(cnt, lds, &total);   // (its barriers also order
                                                                                // the counts above)
            if (kAdaptive && threadIdx.x == 0 && set_on && set_tries >= kInputSetTrial && 16 * set_drops < set_tries)
                set_on = 0;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                if (keep[j]) dst[off++] = key[j];
            }
            cursor += total;
        }
        if (threadIdx.x == 0) w.slab_cnt[slab] = cursor;
        written += cursor;
    }
    survived = block_sum<kThreads>(survived, lds);
    if (threadIdx.x == 0) {
        if (survived) atomicAdd(&st->s_count, (u64c)survived);
        if (written) atomicAdd(&st->s_keys, (u64c)written);
    }
}

// Parents become ranks among the labels (the distinct parents, marked in lmap, whose scan
// has just run): the relabelled edges then name their endpoints with ceil(log2 L) bits
// instead of ceil(log2 N), and everything after the relabel works over the L labels.
// lab_at inverts the ranking.
__global__ __launch_bounds__(kThreads) void k_rank_parents(Work w) {
    const int64_t n = (int64_t)w.st->n_cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t p = w.par[i];
        w.par[i] = nmap_has(w.lmap, p) ? nmap_rank(w.lmap, p) : kNoParent;
        if (nmap_has(w.lmap, i)) w.lab_at[nmap_rank(w.lmap, i)] = (uint32_t)i;
    }
}

// Key width of the round's sort (2 ceil(log2 L) bits) and the block width of the next
// round's edge order: kBlockNodes labels, which become about as many next-round nodes.
__global__ void k_plan_blocks(Work w) {
    RoundState *st = w.st;
    const uint64_t L = st->n_labels;
    const int kb = ceil_log2(L < 2 ? 2 : L);
    st->kb = kb;
    st->hb_shift = kb < LC_BLOCK_NODES_LOG2 ? kb : LC_BLOCK_NODES_LOG2;
    st->nbits = 2 * kb;
}

// The next graph's nodes: the labels that keep an edge, named and indexed; the others are
// final (counted).
template <bool kFirst, bool kBatch>
__global__ __launch_bounds__(kThreads) void k_nodes(Work w, const uint32_t *names_cur, uint32_t *names_next,
                                                    const uint32_t *gids_cur, uint32_t *gids_next) {
    RoundState *st = w.st;
    const int64_t L = (int64_t)st->n_labels;
    uint32_t fin = 0;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < L; j += (int64_t)gridDim.x * kThreads) {
        if (nmap_has(w.nmap, j)) {
            const uint32_t k = nmap_rank(w.nmap, j);
            const uint32_t x = w.lab_at[j];
            const uint32_t nm = kFirst ? x : names_cur[x];
            names_next[k] = nm;
            w.idx_of[nm] = k;
            if (kBatch) gids_next[k] = kFirst ? w.gid0[x] : gids_cur[x];
        } else {
            ++fin;
        }
    }
    __shared__ uint32_t red[kThreads / kWave];
    fin = block_sum<kThreads>(fin, red);
    if (threadIdx.x == 0 && fin) atomicAdd(&st->n_final, (u64c)fin);
}

template <bool kFirst>
__global__ __launch_bounds__(kThreads) void k_map(Work w, const uint32_t *names_cur) {
    RoundState *st = w.st;
    const int64_t n = (int64_t)st->n_cur;
    uint32_t *out;
    if (kFirst) {
        out = w.map0;
    } else {
        if (n == 0) return;
        if (st->map_off + (u64c)n > st->map_cap || st->levels >= kMaxLevels) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->err, 2u);
            return;
        }
        out = w.maps + st->map_off;
    }
    // the parent's bit and its index in the next graph come from one 8-byte word of the map;
    // a final parent is named through the label of its rank.  When every label keeps an edge,
    // a parent's index in the next graph is its rank.
    const bool same = st->n_next == st->n_labels;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t q = w.par[i];
        if (q == kNoParent) {   // round 0: an id without a loop-free record is final on its own
            out[i] = kFinal | (uint32_t)i;
            continue;
        }
        if (same) {
            out[i] = q;
            continue;
        }
        const uint2 e = *(const uint2 *)(w.nmap + 2 * (q >> 5));
        if ((e.x >> (q & 31)) & 1u) {
            out[i] = e.y + (uint32_t)__popc(e.x & ((1u << (q & 31)) - 1u));
        } else {
            const uint32_t x = w.lab_at[q];
            out[i] = kFinal | (kFirst ? x : names_cur[x]);
        }
    }
}

template <bool kFirst>
__global__ void k_round_end(Work w, int dedup) {
    RoundState *st = w.st;
    if (st->m_cur > 0) {
        const int r = st->round;
        if (r < kStatRounds) {
            u64c *s = st->rstats[r];
            s[0] = (u64c)r;
            s[1] = st->n_active;
            s[2] = st->m_cur;
            s[3] = st->s_count;
            s[4] = st->m_next;
            s[5] = st->n_final;
            s[6] = st->s_keys;
        }
        st->rounds_active = r + 1;
    }
    st->n_prev = st->n_cur;
    if (!kFirst && st->n_cur > 0 && !(st->err & 2u)) {
        st->level_off[st->levels] = st->map_off;
        st->levels += 1;
        st->map_off += st->n_cur;
    }
    // the unique write's output (the hashed drop writes into the relabel's buffer)
    const bool hashed = dedup == kDedupHash || (dedup == kDedupDevice && st->hash_slots != 0);
    st->e_sel = hashed ? sort_src(st->round, st->e_sel) : 1 - sorted_sel(st->round, st->e_sel, st->nbits);
    st->n_cur = st->n_next;
    st->m_cur = st->m_next;
    st->round += 1;
    st->done = st->m_next == 0 ? 1 : 0;
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
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_blocks, dim3(1), dim3(1), 0, s, w);
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
