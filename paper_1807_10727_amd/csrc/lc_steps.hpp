// Device bodies of the steps of a round (rounds >= 1 and their scans and hashed duplicate
// drop), shared by the kernels that run each step in a launch of its own (lc_kernels.hip,
// lc_sort.hip) and by the persistent launch that runs whole small rounds with a grid-wide
// barrier between steps (lc_fused.hip).  Every step strides over blockIdx.x / gridDim.x, or
// runs in one workgroup, so it is correct for any grid: its own launch's, or the persistent
// one's between two barriers.
#pragma once

#include "lc_internal.hpp"
#include "lc_readers.hpp"

namespace lc {

__device__ inline int ceil_log2(uint64_t n) { return n <= 1 ? 0 : 64 - __clzll((long long)(n - 1)); }

// kSeeded (plain solve, rounds >= 1, where every node has a loop-free record): both halves of
// the node word start at the node's own priority rather than +inf.  The one-hop minimum over
// the closed neighbourhood then only needs the far endpoint's priority, which the same 8-byte
// load that fetches the current minimum brings along; the two-hop accumulator may start at
// rho(x) because it ends at most at m1[x] <= rho(x).
template <bool kSeeded>
__device__ inline void step_round_begin(Work w, const uint32_t *names, const uint32_t *tab) {
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
__device__ inline void step_min1_seeded(ReadInternal rd, Work w) {
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

template <class R>
__device__ inline void step_min2(R rd, Work w) {
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
__device__ inline void step_parent(Work w, PrioCtx pc, const uint32_t *gids, int word) {
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
// of power-law inputs), and a hash set in LDS (kept for the whole pass over the records)
// removes most of those repeats before they reach the sort.  s_count still counts every
// survivor; s_keys counts the keys.
template <class R>
__device__ inline void step_relabel(R rd, Work w) {
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
__device__ inline void step_rank_parents(Work w) {
    const int64_t n = (int64_t)w.st->n_cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t p = w.par[i];
        w.par[i] = nmap_has(w.lmap, p) ? nmap_rank(w.lmap, p) : kNoParent;
        if (nmap_has(w.lmap, i)) w.lab_at[nmap_rank(w.lmap, i)] = (uint32_t)i;
    }
}

// Key width of the round's sort (2 ceil(log2 L) bits) and the block width of the next
// round's edge order: kBlockNodes labels, which become about as many next-round nodes.
__device__ inline void step_plan_blocks(Work w) {
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
__device__ inline void step_nodes(Work w, const uint32_t *names_cur, uint32_t *names_next,
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
__device__ inline void step_map(Work w, const uint32_t *names_cur) {
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
__device__ inline void step_round_end(Work w, int dedup) {
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

template <typename T>
__device__ inline void load16(const T *in, int64_t base, int64_t n, uint32_t (&v)[16]) {
    if (base + 16 <= n) {
        if (sizeof(T) == 1) {
            uint4 x = *(const uint4 *)(in + base);
            uint32_t wds[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = (wds[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint4 x = *(const uint4 *)(in + base + 4 * q);
                v[4 * q + 0] = x.x;
                v[4 * q + 1] = x.y;
                v[4 * q + 2] = x.z;
                v[4 * q + 3] = x.w;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = base + j < n ? (uint32_t)in[base + j] : 0u;
    }
}

// One workgroup scans `cnt` values in place (cnt = *n_ptr, or ceil(*n_ptr / per_entry)).
__device__ inline void step_scan_single(uint32_t *data, const u64c *n_ptr, int per_entry,
                                        u64c *total_out) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t cnt = per_entry ? ceil_div(n, per_entry) : n;
    uint32_t carry = 0;
    for (int64_t base = 0; base < cnt; base += kScanTile) {
        uint32_t v[16];
        const int64_t my = base + threadIdx.x * 16;
        load16(data, my, cnt, v);
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) sum += v[j];
        uint32_t total;
        uint32_t run = carry + block_excl_scan<kThreads>(sum, lds, &total);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (my + j < cnt) data[my + j] = run;
            run += v[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// Bit map from byte flags (label map, node map): thread t of a block turns the 32 flags of
// word blk * kThreads + t into bits; the blocks' counts are scanned like any other.
__device__ inline uint32_t label_bits(const uint8_t *f, int64_t w, int64_t n) {
    const int64_t base = w * 32;
    uint32_t bits = 0;
    if (base + 32 <= n) {
        const uint4 a = *(const uint4 *)(f + base), b = *(const uint4 *)(f + base + 16);
        const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) bits |= (((v[q] >> (8 * k)) & 0xFFu) != 0u ? 1u : 0u) << (4 * q + k);
    } else {
        for (int k = 0; k < 32; ++k)
            if (base + k < n && f[base + k]) bits |= 1u << k;
    }
    return bits;
}

__device__ inline void step_flags_reduce(const uint8_t *f, const u64c *n_ptr, uint32_t *partials) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t nw = ceil_div(n, 32);
    const int64_t nblk = ceil_div(nw, kThreads);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t wd = blk * kThreads + threadIdx.x;
        const uint32_t c = wd < nw ? (uint32_t)__popc(label_bits(f, wd, n)) : 0u;
        uint32_t total;
        block_excl_scan<kThreads>(c, lds, &total);
        if (threadIdx.x == 0) partials[blk] = total;
    }
}

__device__ inline void step_flags_down(const uint8_t *f, const u64c *n_ptr,
                                       const uint32_t *partials, uint32_t *lmap) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t nw = ceil_div(n, 32);
    const int64_t nblk = ceil_div(nw, kThreads);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t wd = blk * kThreads + threadIdx.x;
        const uint32_t bits = wd < nw ? label_bits(f, wd, n) : 0u;
        uint32_t total;
        const uint32_t before = partials[blk] + block_excl_scan<kThreads>((uint32_t)__popc(bits), lds, &total);
        if (wd < nw) *(uint2 *)(lmap + 2 * wd) = make_uint2(bits, before);
    }
}

// The same in one workgroup, for small rounds: every stage in a single launch (four words a
// thread per step, a running carry across steps).
__device__ inline void step_flags_single(const uint8_t *f, const u64c *n_ptr, uint32_t *map,
                                         u64c *total_out) {
    constexpr int kW = 4;
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t nw = ceil_div(n, 32);
    uint32_t carry = 0;
    for (int64_t base = 0; base < nw; base += (int64_t)kThreads * kW) {
        uint32_t bits[kW], c[kW], sum = 0;
#pragma unroll
        for (int q = 0; q < kW; ++q) {
            const int64_t wd = base + (int64_t)threadIdx.x * kW + q;
            bits[q] = wd < nw ? label_bits(f, wd, n) : 0u;
            c[q] = (uint32_t)__popc(bits[q]);
            sum += c[q];
        }
        uint32_t total;
        uint32_t run = carry + block_excl_scan<kThreads>(sum, lds, &total);
#pragma unroll
        for (int q = 0; q < kW; ++q) {
            const int64_t wd = base + (int64_t)threadIdx.x * kW + q;
            if (wd < nw) *(uint2 *)(map + 2 * wd) = make_uint2(bits[q], run);
            run += c[q];
        }
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

// Keys hold 2 ceil(log2 L) <= 62 bits, so no key has every bit set.
constexpr uint64_t kEmptySlot = ~0ull;

// The key set lives in the round's own edge buffer (E_r, consumed by the relabel) and the kept
// keys go back into the relabel's buffer, so the round ends with the edges in the other buffer
// than a sorted round of an even pass count would leave them (the host tells the round end).
__device__ inline uint64_t *hash_table(const Work &w) { return w.keys[w.st->e_sel]; }

// A key's home slot: a multiplicative hash, its high word scaled to [0, slots).
__device__ inline uint64_t home_slot(uint64_t key, uint64_t slots) {
    return __umul64hi(key * 0x9E3779B97F4A7C15ull, slots);
}

// The table: 2 K + 1 slots (at most half full), cleared to empty.  Every workgroup derives
// the size from K; workgroup 0 records it for the kernels that follow.  decide: the host could
// not bound K (a round of many records), and a round whose keys do not fit sorts instead
// (hash_slots 0: every hashing kernel returns at once, the gated sort runs).  Otherwise a
// round with more keys than the host's bound allowed, or than its buffer holds, is flagged
// and keeps a table that fits the buffer: the inserts then run out of probes and flag it
// again, and no access leaves the buffer.
__device__ inline void step_hash_clear(Work w, int decide) {
    RoundState *st = w.st;
    const uint64_t K = st->s_keys;
    uint64_t slots = 2 * K + 1;
    const bool over = K > (uint64_t)kHashMaxRecords || slots > (uint64_t)w.kcap;
    if (over) slots = decide ? 0 : (uint64_t)min((int64_t)2 * kHashMaxRecords + 1, w.kcap);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->hash_slots = (int32_t)slots;
        if (over && !decide) atomicOr(&st->err, 4u);
    }
    uint64_t *tab = hash_table(w);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < (int64_t)slots; i += (int64_t)gridDim.x * kThreads)
        tab[i] = kEmptySlot;
}

// Every key the relabel wrote (in its slabs) joins the set: linear probing from its home slot,
// an empty slot claimed with a compare-and-swap, a repeat stopping at its own key.
__device__ inline void step_hash_insert(Work w) {
    RoundState *st = w.st;
    const uint64_t slots = (uint64_t)st->hash_slots;
    if (slots == 0) return;   // the round sorts
    const Tiles tl = tiles_of(w, 0);
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel)];
    u64c *tab = (u64c *)hash_table(w);
    bool lost = false;
    for (int64_t tile = blockIdx.x; tile < tl.ntiles; tile += gridDim.x) {
        const int tv = tl.valid(tile);
        for (int i = threadIdx.x; i < tv; i += kSortThreads) {
            const uint64_t key = in[tile * kSortTile + i];
            uint64_t h = home_slot(key, slots);
            bool placed = false;
            for (uint64_t probe = 0; probe < slots; ++probe) {
                // the swap returns the slot's key whether or not it claims the slot
                const uint64_t cur = atomicCAS(&tab[h], (u64c)kEmptySlot, (u64c)key);
                if (cur == kEmptySlot || cur == key) {
                    placed = true;
                    break;
                }
                h = h + 1 == slots ? 0 : h + 1;
            }
            lost |= !placed;
        }
    }
    if (lost) atomicOr(&st->err, 4u);
}

// Kept keys per table tile (kSortTile slots, the last one ragged), and the next graph's nodes:
// both endpoints of every kept edge.
__device__ inline void step_hash_count(Work w) {
    RoundState *st = w.st;
    __shared__ uint32_t lds[kSortThreads / kWave + 1];
    const int64_t slots = st->hash_slots;
    if (slots == 0) return;   // the round sorts
    const int64_t ntiles = ceil_div(slots, kSortTile);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->aux_n = (u64c)ntiles;   // entries of the count scan
    const uint64_t *tab = hash_table(w);
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    const uint64_t n_lab = st->n_labels;
    bool broken = false;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint64_t kk[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int64_t idx = tile * kSortTile + j * kSortThreads + threadIdx.x;
            kk[j] = idx < slots ? tab[idx] : kEmptySlot;
        }
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (kk[j] == kEmptySlot) continue;
            ++cnt;
            uint64_t lo, hi;
            edge_key_split(kk[j], kb, hbs, lo, hi);
            if (lo < n_lab && hi < n_lab) {
                w.has_edge[lo] = 1;
                w.has_edge[hi] = 1;
            } else {
                broken = true;
            }
        }
        uint32_t total;
        block_excl_scan<kSortThreads>(cnt, lds, &total);
        if (threadIdx.x == 0) w.tile_cnt[tile] = total;
    }
    if (broken) atomicOr(&st->err, 4u);
}

// The next graph's edge list: the kept keys, tile by tile at the scanned tile offsets, renamed
// into the next round's indices (as the unique write renames the sorted heads).
__device__ inline void step_hash_write(Work w) {
    constexpr int kWaves = kSortThreads / kWave;
    RoundState *st = w.st;
    __shared__ uint32_t rowcnt[kSortItems * kWaves];
    const int64_t slots = st->hash_slots;   // 0: the round sorts
    const int64_t ntiles = ceil_div(slots, kSortTile);
    const uint64_t *tab = hash_table(w);
    uint64_t *out = w.keys[sort_src(st->round, st->e_sel)];
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    const uint64_t n_lab = st->n_labels;
    const bool same = st->n_next == n_lab;   // every label keeps an edge: index = rank
    const int wave = threadIdx.x / kWave;
    const uint64_t lt = lanemask_lt();
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint64_t k[kSortItems];
        uint64_t bal[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int64_t idx = tile * kSortTile + j * kSortThreads + threadIdx.x;
            k[j] = idx < slots ? tab[idx] : kEmptySlot;
            bal[j] = ballot(k[j] != kEmptySlot);
            if (lane_id() == 0) rowcnt[j * kWaves + wave] = (uint32_t)__popcll(bal[j]);
        }
        __syncthreads();
        static_assert(kSortItems * kWaves == kWave, "one (row, wave) count per lane of wave 0");
        if (threadIdx.x < kWave) {   // exclusive prefix over (row, wave)
            const uint32_t c = rowcnt[threadIdx.x];
            rowcnt[threadIdx.x] = (uint32_t)w.tile_cnt[tile] + wave_incl_scan(c) - c;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (k[j] != kEmptySlot) {
                const uint32_t off = rowcnt[j * kWaves + wave] + (uint32_t)__popcll(bal[j] & lt);
                uint64_t lo, hi;
                edge_key_split(k[j], kb, hbs, lo, hi);
                const uint32_t a = lo < n_lab ? (same ? (uint32_t)lo : nmap_rank(w.nmap, lo)) : 0u;
                const uint32_t b = hi < n_lab ? (same ? (uint32_t)hi : nmap_rank(w.nmap, hi)) : 0u;
                out[off] = ((uint64_t)a << 32) | b;
            }
        }
        __syncthreads();
    }
}

// ---- TreeContraction (Section 4) ----

template <bool kFirst>
__device__ inline uint32_t tree_prio(const PrioCtx &pc, const uint32_t *names, uint32_t i) {
    return rho_of(pc, kFirst ? i : names[i]);
}

// Open one-hop minimum: each loop-free record sends rho(b) to a and rho(a) to b (no self
// term), into the low half of the node word, which round_begin filled with +inf.
template <class R, bool kFirst>
__device__ inline void step_min1_open(R rd, Work w, PrioCtx pc, const uint32_t *names) {
    constexpr int V = R::kV;
    rd.init(w.st);
    pc.key = w.st->key;
    const int64_t nch = rd.chunks();
    uint32_t *m1 = w.ml;
    bool bad = false;
    for (int64_t cb = (int64_t)blockIdx.x * kThreads; cb < nch; cb += (int64_t)gridDim.x * kThreads) {
        const int64_t c = cb + threadIdx.x;
        uint32_t a[V], b[V];
        if (c < nch) {
            rd.read(c, a, b, bad);
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) a[j] = b[j] = 0u;
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const bool ok = a[j] != b[j];
            const uint32_t pa = ok ? tree_prio<kFirst>(pc, names, a[j]) : kInf;
            const uint32_t pb = ok ? tree_prio<kFirst>(pc, names, b[j]) : kInf;
            bool la = true;
            const uint32_t va = R::kSorted ? run_min(ok ? a[j] : 0xFFFFFFFFu, pb, la) : pb;
            if (ok) {
                if (la && m1[2 * (size_t)a[j]] > va) atomicMin(&m1[2 * (size_t)a[j]], va);
                if (m1[2 * (size_t)b[j]] > pa) atomicMin(&m1[2 * (size_t)b[j]], pa);
            }
        }
    }
    if (bad) atomicOr(&w.st->err, 1u);
}

// Where the open one-hop minimum and f live: the node word (low half m1, high half f), or
// after the tiled round 0's row pass, a dense m1 array with f kept in lab_at (free until the
// labels are ranked).
template <bool kDense>
__device__ inline uint32_t tree_m1(const Work &w, int64_t i) { return kDense ? w.ml[i] : w.ml[2 * i]; }
template <bool kDense>
__device__ inline uint32_t *tree_f_ptr(const Work &w, int64_t i) { return kDense ? w.lab_at + i : w.ml + 2 * i + 1; }

// f(v) (see tree_f_ptr) and the starting jump pointer (par); a node without a loop-free
// record (round 0 only) points to itself.  Resets the jump flags.
template <bool kFirst, bool kDense>
__device__ inline void step_tree_f(Work w, PrioCtx pc) {
    RoundState *st = w.st;
    pc.key = st->key;
    const int64_t n = (int64_t)st->n_cur;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->jflag[0] = 0u;
        st->jdone = 0u;
    }
    uint32_t active = 0;
    bool broken = false;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const uint32_t m = tree_m1<kDense>(w, i);
        uint32_t p = (uint32_t)i;
        if (m != kInf) {
            const uint32_t name = rho_name(pc, m, w.n0);
            p = kFirst ? name : ((int64_t)name < w.n0 ? w.idx_of[name] : 0xFFFFFFFFu);
            if ((int64_t)p >= n) {   // cannot happen for a consistent state
                broken = true;
                p = (uint32_t)i;
            }
            ++active;
        }
        *tree_f_ptr<kDense>(w, i) = p;
        w.par[i] = p;
    }
    __shared__ uint32_t red[kThreads / kWave];
    active = block_sum<kThreads>(active, red);
    if (threadIdx.x == 0 && active) atomicAdd(&st->n_active, (u64c)active);
    if (broken) atomicOr(&st->err, 4u);
}

// A pointer found on its 2-cycle is final: the top bit of par marks it (node indices are
// below 2^31), so later passes stream over it without gathering.
constexpr uint32_t kOnCycle = 0x80000000u;

// One pointer-jumping pass: a pointer not yet on a 2-cycle takes its target's pointer; one
// found on its cycle is marked final.  Pass `it` reads whether pass it-1 moved a pointer
// (flag slot (it + 2) % 3), records its own moves in slot it % 3 and clears slot
// (it + 1) % 3 for the next pass; once a pass moves nothing, every pointer is on its cycle,
// the next pass sets jdone and every later pass returns at once.  Passes never read a slot
// that the same pass writes, so every workgroup decides alike.  Pointers read while another
// thread updates them are valid either way (the old or the new position on the same path).
template <bool kDense>
__device__ inline void step_tree_jump(Work w, int it) {
    RoundState *st = w.st;
    if (st->jdone) return;
    if (it > 0 && st->jflag[(it + 2) % 3] == 0u) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->jdone = 1u;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->jflag[(it + 1) % 3] = 0u;
    const int64_t n = (int64_t)st->n_cur;
    bool changed = false;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const uint32_t pj = w.par[x];
        if (pj & kOnCycle) continue;
        const uint32_t fj = *tree_f_ptr<kDense>(w, pj);
        if (*tree_f_ptr<kDense>(w, fj) != pj) {
            w.par[x] = w.par[pj] & ~kOnCycle;
            changed = true;
        } else {
            w.par[x] = pj | kOnCycle;
        }
    }
    if (__any(changed) && lane_id() == 0) st->jflag[it % 3] = 1u;
}

// The label of each node: the member of smaller priority of the 2-cycle its pointer reached.
template <bool kFirst, bool kDense>
__device__ inline void step_tree_label(Work w, PrioCtx pc, const uint32_t *names) {
    RoundState *st = w.st;
    pc.key = st->key;
    const int64_t n = (int64_t)st->n_cur;
    bool broken = false;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        if (*tree_f_ptr<kDense>(w, x) == (uint32_t)x) {   // no neighbour: its own parent, nobody's label
            w.par[x] = (uint32_t)x;
            continue;
        }
        const uint32_t pj = w.par[x];
        const uint32_t j = pj & ~kOnCycle;
        const uint32_t fj = *tree_f_ptr<kDense>(w, j);
        // a pointer without the mark was never found on its cycle: check it (the passes
        // should have converged)
        if (!(pj & kOnCycle) && *tree_f_ptr<kDense>(w, fj) != j) broken = true;
        const uint32_t lab = tree_prio<kFirst>(pc, names, j) < tree_prio<kFirst>(pc, names, fj) ? j : fj;
        w.par[x] = lab;
        w.is_label[lab] = 1;
    }
    if (broken) atomicOr(&st->err, 4u);
}

// ---- MergeToLarge (Section 5) ----

// index in the next graph of the class of node i of this round, or -1 (final or not a node)
__device__ inline int64_t mtl_next_class(const Work &w, int64_t i) {
    const uint32_t q = w.par[i];
    if (q == kNoParent || !nmap_has(w.nmap, q)) return -1;
    return (int64_t)nmap_rank(w.nmap, q);
}

__device__ inline void step_mtl_clear(Work w) {
    const int64_t n = (int64_t)w.st->n_next;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
        w.mtl_size[k] = 0;
        w.mtl_v[k] = 0;
        w.mtl_cnt[k] = 0;
    }
}

__device__ inline void step_mtl_size(Work w) {
    const int64_t n = (int64_t)w.st->n_cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const int64_t k = mtl_next_class(w, i);
        if (k >= 0) atomicAdd(&w.mtl_size[k], 1u);
    }
}

// The alpha-th largest member priority v of a large class, one bit at a time from the top:
// with the bits above b settled, bit b is set when at least alpha members have a priority of
// at least v | 2^b.  Count pass, then keep pass, for b = 31 .. 0.
template <bool kFirst>
__device__ inline void step_mtl_count(Work w, PrioCtx pc, const uint32_t *names, int bit,
                                      uint64_t alpha) {
    const RoundState *st = w.st;
    if (!pc.tab) pc.key = st->key;
    const int64_t n = (int64_t)st->n_cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const int64_t k = mtl_next_class(w, i);
        if (k < 0 || w.mtl_size[k] < alpha) continue;
        const uint32_t cand = w.mtl_v[k] | (1u << bit);
        if (rho_of(pc, kFirst ? (uint32_t)i : names[i]) >= cand) atomicAdd(&w.mtl_cnt[k], 1u);
    }
}

__device__ inline void step_mtl_keep(Work w, int bit, uint64_t alpha) {
    const int64_t n = (int64_t)w.st->n_next;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n; k += (int64_t)gridDim.x * kThreads) {
        if (w.mtl_size[k] >= alpha && w.mtl_cnt[k] >= alpha) w.mtl_v[k] |= 1u << bit;
        w.mtl_cnt[k] = 0;
    }
}

// Candidate of node u in the step: (priority, u) of a large node, 0 otherwise (bit 31 of the
// low word marks a candidate, so that a priority of 0 still beats "none").
__device__ inline uint64_t mtl_cand(const Work &w, uint32_t u, uint64_t alpha) {
    return w.mtl_size[u] >= alpha ? ((uint64_t)w.mtl_v[u] << 32) | 0x80000000ull | u : 0ull;
}

__device__ inline void step_mtl_seed(Work w, uint64_t alpha, int pass) {
    const int64_t n = (int64_t)w.st->n_cur;
    for (int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x; u < n; u += (int64_t)gridDim.x * kThreads)
        w.mtl_acc[pass][u] = pass == 0 ? mtl_cand(w, (uint32_t)u, alpha) : w.mtl_acc[0][u];
}

// pass 0: best candidate over the closed one-hop neighbourhood; pass 1: over two hops
template <class R>
__device__ inline void step_mtl_max(R rd, Work w, uint64_t alpha, int pass) {
    constexpr int V = R::kV;
    rd.init(w.st);
    const int64_t nch = rd.chunks();
    u64c *acc = (u64c *)w.mtl_acc[pass];
    const uint64_t *prev = w.mtl_acc[0];
    bool bad = false;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < nch; c += (int64_t)gridDim.x * kThreads) {
        uint32_t a[V], b[V];
        rd.read(c, a, b, bad);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (a[j] == b[j]) continue;
            const uint64_t va = pass == 0 ? mtl_cand(w, a[j], alpha) : prev[a[j]];
            const uint64_t vb = pass == 0 ? mtl_cand(w, b[j], alpha) : prev[b[j]];
            if (vb > acc[a[j]]) atomicMax(&acc[a[j]], (u64c)vb);
            if (va > acc[b[j]]) atomicMax(&acc[b[j]], (u64c)va);
        }
    }
}

__device__ inline void step_mtl_parent(Work w) {
    RoundState *st = w.st;
    const int64_t n = (int64_t)st->n_cur;
    uint32_t active = 0;
    bool broken = false;
    for (int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x; u < n; u += (int64_t)gridDim.x * kThreads) {
        const uint64_t x = w.mtl_acc[1][u];
        uint32_t p = x ? (uint32_t)(x & 0x7FFFFFFFull) : (uint32_t)u;
        if ((int64_t)p >= n) {   // cannot happen for a consistent state
            broken = true;
            p = (uint32_t)u;
        }
        w.par[u] = p;
        w.is_label[p] = 1;
        ++active;
    }
    __shared__ uint32_t red[kThreads / kWave];
    active = block_sum<kThreads>(active, red);
    if (threadIdx.x == 0 && active) atomicAdd(&st->n_active, (u64c)active);
    if (broken) atomicOr(&st->err, 4u);
}

}  // namespace lc
