// Round 0 of LocalContraction over a tiled layout of the input records.
//
// The first round reads the raw input, whose endpoints are uniformly scattered over the
// whole id space: every per-record access to a node value misses L2 and costs a full
// cache line.  This file first partitions the input, once, into directed records
// (x << 32 | y), two per loop-free input record, grouped by the row block x >> xs and,
// inside a row, by the column block y >> ys (two counting passes: pass A by column into
// one key buffer, pass B by row into the other; the order inside a tile is free), or by
// row only in one counting pass (no column order).  Then:
//
//   min1     one workgroup per row: LDS minimum of rho(y) over the row's records, folded
//            with rho(x); no global atomics (Section 2: x is in its own neighbourhood)
//   min2     the same with the gathered one-hop minimum m1[y], folded with m1[x], and the
//            parent written directly (the node whose priority is the two-hop minimum)
//   relabel  one direction of every record becomes (p(x), p(y)); loops are dropped;
//            survivors go to fixed output slabs, as the first radix pass expects
//
// Rows that run at the same time sweep the column blocks in the same order, so the values
// gathered at y come from one or two column blocks per XCD, resident in its L2.

#include "lc_internal.hpp"
#include "lc_readers.hpp"

namespace lc {

// ---------------------------------------------------------------------------------------
// partition pass A: input records -> directed records ordered by column block
// ---------------------------------------------------------------------------------------

template <class R>
__global__ __launch_bounds__(kThreads) void k_part_a_hist(R rd, Work w, TPlan tp) {
    constexpr int V = R::kV;
    constexpr int kIter = kTaIn / (V * kThreads);
    static_assert(kIter * V * kThreads == kTaIn, "pass-A tile must be whole reader chunks");
    static_assert(kThreads == 256, "one column digit per thread");
    RoundState *st = w.st;
    __shared__ uint32_t hist[256];
    rd.init(st);
    const int64_t nt = tp.tiles_a;
    const int64_t nch = rd.chunks();
    const int ys = tp.ys;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->aux_n = (u64c)256 * (u64c)nt;
    bool bad = false;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        hist[threadIdx.x] = 0;
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kIter; ++it) {
            const int64_t c = tile * (kTaIn / V) + (int64_t)it * kThreads + threadIdx.x;
            if (c < nch) {
                uint32_t a[V], b[V];
                rd.read(c, a, b, bad);
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    if (a[j] != b[j]) {
                        atomicAdd(&hist[b[j] >> ys], 1u);
                        atomicAdd(&hist[a[j] >> ys], 1u);
                    }
                }
            }
        }
        __syncthreads();
        w.counts[(int64_t)threadIdx.x * nt + tile] = hist[threadIdx.x];
        __syncthreads();
    }
    if (bad) atomicOr(&st->err, 1u);
}

template <class R>
__global__ __launch_bounds__(kThreads) void k_part_a_scatter(R rd, Work w, TPlan tp) {
    constexpr int V = R::kV;
    constexpr int kIter = kTaIn / (V * kThreads);
    constexpr int kItems = 2 * V * kIter;   // directed records per thread
    RoundState *st = w.st;
    __shared__ uint32_t cnt[256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint64_t skeys[2 * kTaIn];
    __shared__ uint32_t lds[kThreads / kWave + 1];
    rd.init(st);
    const int64_t nt = tp.tiles_a;
    const int64_t nch = rd.chunks();
    const int ys = tp.ys;
    uint64_t *out = w.keys[0];
    bool bad = false;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        cnt[threadIdx.x] = 0;
        __syncthreads();
        uint64_t k[kItems];
        uint32_t rk[kItems];
#pragma unroll
        for (int it = 0; it < kIter; ++it) {
            const int64_t c = tile * (kTaIn / V) + (int64_t)it * kThreads + threadIdx.x;
            uint32_t a[V], b[V];
            if (c < nch) {
                rd.read(c, a, b, bad);
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) a[j] = b[j] = 0u;
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int q = 2 * (it * V + j);
                const bool valid = a[j] != b[j];
                k[q] = ((uint64_t)a[j] << 32) | b[j];
                k[q + 1] = ((uint64_t)b[j] << 32) | a[j];
                rk[q] = valid ? atomicAdd(&cnt[b[j] >> ys], 1u) : ~0u;
                rk[q + 1] = valid ? atomicAdd(&cnt[a[j] >> ys], 1u) : ~0u;
            }
        }
        __syncthreads();
        uint32_t total;
        {
            const uint32_t c0 = cnt[threadIdx.x];
            dstart[threadIdx.x] = block_excl_scan<kThreads>(c0, lds, &total);
            gofs[threadIdx.x] = w.counts[(int64_t)threadIdx.x * nt + tile];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kItems; ++q) {
            if (rk[q] != ~0u) skeys[dstart[(uint32_t)k[q] >> ys] + rk[q]] = k[q];
        }
        __syncthreads();
        for (uint32_t pos = threadIdx.x; pos < total; pos += kThreads) {
            const uint64_t kk = skeys[pos];
            const uint32_t d = (uint32_t)kk >> ys;
            out[gofs[d] + pos - dstart[d]] = kk;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// partition pass B: directed records -> ordered by row block, column order kept per tile
// ---------------------------------------------------------------------------------------

// columns of the row partition's count table (pass B's tiles, or the one-pass form's), set by
// the partition's count pass
__device__ inline int64_t tiles_b_of(const RoundState *st) { return (int64_t)st->t_tiles; }

// Load the two records at even position p of a key array that holds an even number of
// records (so p + 1 is in range whenever p is).
// Directed records stream through each row kernel once: non-temporal loads keep them from
// evicting the gathered column values from L2 (measured: the two-hop row pass ~7 % faster).
#ifndef LC_ROW_GENERATIONS
#define LC_ROW_GENERATIONS 1
#endif
#ifndef LC_NT_RECORDS
#define LC_NT_RECORDS 1
#endif
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));

__device__ inline void load_pair(const uint64_t *k, int64_t p, int64_t T, uint64_t &r0, uint64_t &r1, bool &v0,
                                 bool &v1) {
    v0 = p < T;
    v1 = p + 1 < T;
    if (v1) {
        u64x2_t x;
        if (LC_NT_RECORDS)
            x = __builtin_nontemporal_load((const u64x2_t *)(k + p));
        else
            x = *(const u64x2_t *)(k + p);
        r0 = x.x;
        r1 = x.y;
    } else {
        r0 = v0 ? k[p] : 0ull;
        r1 = 0ull;
    }
}

__global__ __launch_bounds__(kTbThreads) void k_part_b_hist(Work w, TPlan tp) {
    RoundState *st = w.st;
    __shared__ uint32_t hist[kTRowsMax];
    const int64_t T = (int64_t)st->t_count;
    const int64_t nt = ceil_div(T, kTbTile);
    const int64_t nslabs = ceil_div(T, kSlab);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->aux_n = (u64c)tp.rows * (u64c)nt;
        st->n_slabs = (u64c)nslabs;
        st->t_tiles = (u64c)nt;
    }
    const uint64_t *in = w.keys[0];
    const int xs = tp.xs;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        for (int i = threadIdx.x; i < tp.rows; i += kTbThreads) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kTbTile / (2 * kTbThreads); ++j) {
            const int64_t p = tile * kTbTile + 2 * ((int64_t)j * kTbThreads + threadIdx.x);
            uint64_t r0, r1;
            bool v0, v1;
            load_pair(in, p, T, r0, r1, v0, v1);
            if (v0) atomicAdd(&hist[(uint32_t)(r0 >> 32) >> xs], 1u);
            if (v1) atomicAdd(&hist[(uint32_t)(r1 >> 32) >> xs], 1u);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tp.rows; i += kTbThreads) w.counts[(int64_t)i * nt + tile] = hist[i];
        __syncthreads();
    }
}

// LDS: digit counts (scanned in place into tile starts), global offsets and the staged tile:
// 80 KiB, so that two workgroups share a CU.  The scan's scratch words borrow the staging
// area, which is idle while the counts are scanned.
__global__ __launch_bounds__(kTbThreads) void k_part_b_scatter(Work w, TPlan tp) {
    constexpr int kPairs = kTbTile / (2 * kTbThreads);
    constexpr int kPerThread = kTRowsMax / kTbThreads;   // row digits scanned by each thread
    static_assert(kPerThread * kTbThreads == kTRowsMax, "row digits per thread");
    RoundState *st = w.st;
    __shared__ uint32_t dstart[kTRowsMax];
    __shared__ uint32_t gofs[kTRowsMax];
    __shared__ uint64_t skeys[kTbTile];
    uint32_t *lds = (uint32_t *)skeys;
    const int64_t T = (int64_t)st->t_count;
    const int64_t nt = tiles_b_of(st);
    const uint64_t *in = w.keys[0];
    uint64_t *out = w.keys[1];
    const int xs = tp.xs;
    const int rows = tp.rows;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        for (int i = threadIdx.x; i < rows; i += kTbThreads) dstart[i] = 0;
        __syncthreads();
        uint64_t k[2 * kPairs];
        uint32_t rk[2 * kPairs];
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
            const int64_t p = tile * kTbTile + 2 * ((int64_t)j * kTbThreads + threadIdx.x);
            bool v0, v1;
            load_pair(in, p, T, k[2 * j], k[2 * j + 1], v0, v1);
            rk[2 * j] = v0 ? atomicAdd(&dstart[(uint32_t)(k[2 * j] >> 32) >> xs], 1u) : ~0u;
            rk[2 * j + 1] = v1 ? atomicAdd(&dstart[(uint32_t)(k[2 * j + 1] >> 32) >> xs], 1u) : ~0u;
        }
        __syncthreads();
        uint32_t total;
        {
            uint32_t c[kPerThread];
            uint32_t sum = 0;
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int i = kPerThread * threadIdx.x + q;
                c[q] = i < rows ? dstart[i] : 0u;
                sum += c[q];
            }
            uint32_t run = block_excl_scan<kTbThreads>(sum, lds, &total);
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int i = kPerThread * threadIdx.x + q;
                if (i < rows) {
                    dstart[i] = run;
                    gofs[i] = w.counts[(int64_t)i * nt + tile];
                }
                run += c[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2 * kPairs; ++q) {
            if (rk[q] != ~0u) skeys[dstart[(uint32_t)(k[q] >> 32) >> xs] + rk[q]] = k[q];
        }
        __syncthreads();
        for (uint32_t pos = threadIdx.x; pos < total; pos += kTbThreads) {
            const uint64_t kk = skeys[pos];
            const uint32_t d = (uint32_t)(kk >> 32) >> xs;
            out[gofs[d] + pos - dstart[d]] = kk;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// the one-pass row partition: input records -> directed records ordered by row block only
// ---------------------------------------------------------------------------------------
//
// Both directed records of every loop-free input record go straight to their rows, in one
// counting pass over the input (pass A and its column order skipped): the row kernels only
// need a row's records together, and the column order inside a row serves the L2 locality
// of their gathers, which this form gives up for two passes fewer over the records.

template <class R>
__global__ __launch_bounds__(kTbThreads) void k_part_r_hist(R rd, Work w, TPlan tp) {
    constexpr int V = R::kV;
    constexpr int kChunks = kTrIn / V;   // reader chunks per tile
    static_assert(kChunks * V == kTrIn, "tile of whole reader chunks");
    RoundState *st = w.st;
    __shared__ uint32_t hist[kTRowsMax];
    rd.init(st);
    const int64_t M = rd.records();
    const int64_t nch = rd.chunks();
    const int64_t nt = ceil_div(M, kTrIn);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->aux_n = (u64c)tp.rows * (u64c)nt;
        st->n_slabs = (u64c)ceil_div(2 * M, kSlab);
        st->t_tiles = (u64c)nt;
    }
    const int xs = tp.xs;
    bool bad = false;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        for (int i = threadIdx.x; i < tp.rows; i += kTbThreads) hist[i] = 0;
        __syncthreads();
        for (int it = threadIdx.x; it < kChunks; it += kTbThreads) {
            const int64_t c = tile * kChunks + it;
            if (c < nch) {
                uint32_t a[V], b[V];
                rd.read(c, a, b, bad);
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    if (a[j] != b[j]) {
                        atomicAdd(&hist[a[j] >> xs], 1u);
                        atomicAdd(&hist[b[j] >> xs], 1u);
                    }
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < tp.rows; i += kTbThreads) w.counts[(int64_t)i * nt + tile] = hist[i];
        __syncthreads();
    }
    if (bad) atomicOr(&st->err, 1u);
}

// LDS as pass B's scatter (80 KiB): the tile's row counts, scanned in place into tile starts,
// the global offsets, and the staged directed records.
template <class R>
__global__ __launch_bounds__(kTbThreads) void k_part_r_scatter(R rd, Work w, TPlan tp) {
    constexpr int V = R::kV;
    constexpr int kChunks = kTrIn / V;
    constexpr int kPer = kChunks / kTbThreads;   // reader chunks per thread and tile
    static_assert(kPer * kTbThreads == kChunks, "whole reader chunks per thread");
    constexpr int kItems = 2 * V * kPer;        // directed records per thread and tile
    constexpr int kPerThread = kTRowsMax / kTbThreads;
    static_assert(kPerThread * kTbThreads == kTRowsMax, "row digits per thread");
    RoundState *st = w.st;
    __shared__ uint32_t dstart[kTRowsMax];
    __shared__ uint32_t gofs[kTRowsMax];
    __shared__ uint64_t skeys[kTbTile];
    uint32_t *lds = (uint32_t *)skeys;
    rd.init(st);
    const int64_t nch = rd.chunks();
    const int64_t nt = tiles_b_of(st);
    uint64_t *out = w.keys[1];
    const int xs = tp.xs;
    const int rows = tp.rows;
    bool bad = false;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < nt; tile += gridDim.x) {
        for (int i = threadIdx.x; i < rows; i += kTbThreads) dstart[i] = 0;
        __syncthreads();
        uint64_t k[kItems];
        uint32_t rk[kItems];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t c = tile * kChunks + (int64_t)u * kTbThreads + threadIdx.x;
            uint32_t a[V], b[V];
            if (c < nch) {
                rd.read(c, a, b, bad);
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) a[j] = b[j] = 0u;
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int q = 2 * (u * V + j);
                const bool valid = a[j] != b[j];
                k[q] = ((uint64_t)a[j] << 32) | b[j];
                k[q + 1] = ((uint64_t)b[j] << 32) | a[j];
                rk[q] = valid ? atomicAdd(&dstart[a[j] >> xs], 1u) : ~0u;
                rk[q + 1] = valid ? atomicAdd(&dstart[b[j] >> xs], 1u) : ~0u;
            }
        }
        __syncthreads();
        uint32_t total;
        {
            uint32_t c[kPerThread];
            uint32_t sum = 0;
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int i = kPerThread * threadIdx.x + q;
                c[q] = i < rows ? dstart[i] : 0u;
                sum += c[q];
            }
            uint32_t run = block_excl_scan<kTbThreads>(sum, lds, &total);
#pragma unroll
            for (int q = 0; q < kPerThread; ++q) {
                const int i = kPerThread * threadIdx.x + q;
                if (i < rows) {
                    dstart[i] = run;
                    gofs[i] = w.counts[(int64_t)i * nt + tile];
                }
                run += c[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kItems; ++q) {
            if (rk[q] != ~0u) skeys[dstart[(uint32_t)(k[q] >> 32) >> xs] + rk[q]] = k[q];
        }
        __syncthreads();
        for (uint32_t pos = threadIdx.x; pos < total; pos += kTbThreads) {
            const uint64_t kk = skeys[pos];
            const uint32_t d = (uint32_t)(kk >> 32) >> xs;
            out[gofs[d] + pos - dstart[d]] = kk;
        }
        __syncthreads();
    }
    if (bad) atomicOr(&st->err, 1u);
}

// ---------------------------------------------------------------------------------------
// per-row kernels
// ---------------------------------------------------------------------------------------

// Records [start, end) of row X in the tiled array; the scanned pass-B count table holds
// the first position of each row in the column of tile 0.
__device__ inline void row_range(const Work &w, const TPlan &tp, int X, int64_t nt, int64_t T, int64_t &start,
                                 int64_t &end) {
    if (nt == 0) {
        start = end = 0;
        return;
    }
    start = w.counts[(int64_t)X * nt];
    end = X + 1 < tp.rows ? (int64_t)w.counts[(int64_t)(X + 1) * nt] : T;
}

// kStep 1: m1[x] = min(rho(x), min over the row's records (x, y) of rho(y)), or +inf for an
// id without a loop-free record; kOpen leaves rho(x) out (TreeContraction's open
// neighbourhood).  kStep 2: two-hop minimum min(m1[x], min m1[y]) and the parent it names
// (the inverse of the priority bijection); an id without records is its own parent.
template <int kStep, bool kOpen = false, int kPairs2 = LC_TMIN2_PAIRS>
__global__ __launch_bounds__(kTRowThreads) void k_tiled_min(Work w, PrioCtx pc, TPlan tp, int row0) {
    constexpr int kUnroll = kStep == 1 ? 4 : kPairs2;   // record pairs in flight per thread
    __shared__ uint32_t acc[1 << kTxShiftMax];
    RoundState *st = w.st;
    pc.key = st->key;
    const int64_t T = (int64_t)st->t_count;
    const int64_t nt = tiles_b_of(st);
    const int64_t n = (int64_t)st->n_cur;
    const uint64_t *rec = w.keys[1];
    uint32_t *m1 = w.ml;
    uint32_t active = 0;
    bool broken = false;
    // one workgroup per row of [row0, row0 + gridDim.x)
    const int row_end = min(tp.rows, row0 + (int)gridDim.x);
    for (int X = row0 + blockIdx.x; X < row_end; X += gridDim.x) {
        const int64_t base = (int64_t)X << tp.xs;
        const int cnt = (int)min((int64_t)1 << tp.xs, n - base);
        for (int i = threadIdx.x; i < cnt; i += kTRowThreads) acc[i] = kInf;
        __syncthreads();
        int64_t start, end;
        row_range(w, tp, X, nt, T, start, end);
        const int64_t p0 = start & ~(int64_t)1;
        for (int64_t pb = p0 + 2 * (int64_t)threadIdx.x; pb < end; pb += 2 * kUnroll * kTRowThreads) {
            uint64_t r[2 * kUnroll];
            bool v[2 * kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t p = pb + 2 * (int64_t)u * kTRowThreads;
                load_pair(rec, p, end, r[2 * u], r[2 * u + 1], v[2 * u], v[2 * u + 1]);
                v[2 * u] = v[2 * u] && p >= start;
            }
            uint32_t val[2 * kUnroll];
#pragma unroll
            for (int q = 0; q < 2 * kUnroll; ++q) {
                const uint32_t y = (uint32_t)r[q];
                if (kStep == 1)
                    val[q] = prio(pc.key, y);
                else
                    val[q] = v[q] ? m1[y] : kInf;
            }
#pragma unroll
            for (int q = 0; q < 2 * kUnroll; ++q) {
                const int64_t xi = (int64_t)(uint32_t)(r[q] >> 32) - base;
                if (v[q]) {
                    if (xi >= 0 && xi < cnt)
                        atomicMin(&acc[xi], val[q]);
                    else
                        broken = true;
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kTRowThreads) {
            const uint32_t a = acc[i];
            const uint32_t x = (uint32_t)(base + i);
            if (kStep == 1) {
                m1[x] = (a == kInf || kOpen) ? a : min(a, prio(pc.key, x));
            } else if (a == kInf) {
                w.par[x] = x;   // no loop-free record: not a label, ranked as kNoParent
            } else {
                uint32_t p = prio_inv(pc.key, min(a, m1[x]));
                if ((int64_t)p >= n) {   // cannot happen for a consistent state
                    broken = true;
                    p = x;
                }
                w.par[x] = p;
                w.is_label[p] = 1;
                ++active;
            }
        }
        __syncthreads();
    }
    if (kStep == 2) {
        __shared__ uint32_t red[kTRowThreads / kWave];
        active = block_sum<kTRowThreads>(active, red);
        if (threadIdx.x == 0 && active) atomicAdd(&st->n_active, (u64c)active);
    }
    if (broken) atomicOr(&st->err, 4u);
}

// Repeats in the relabel's output.  A workgroup keeps the keys it has written in an LDS set
// (open addressing, kRowSetProbes linear probes, kept for the whole launch) and drops a key it
// finds there: on power-law inputs most survivors of round 0 repeat a few parent pairs (hubs
// and their neighbourhoods contract onto the same parents), and they need not reach the sort.
// A key whose probes all meet other keys is written anyway; the sort drops every repeat left.
// Where keys hardly repeat (uniform random graphs) the probes cost more than they save, so a
// workgroup stops using the set once kRowSetTrial keys found fewer than 1/16 repeats.
#ifndef LC_ROW_SET_LOG2
#define LC_ROW_SET_LOG2 11
#endif
constexpr int kRowSetLog2 = LC_ROW_SET_LOG2;
constexpr int kRowSetSlots = 1 << kRowSetLog2;
constexpr int kRowSetProbes = 8;
constexpr uint32_t kRowSetTrial = 8192;

// false when `key` is in the set already
__device__ inline bool row_set_insert(unsigned long long *set, uint64_t key) {
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - kRowSetLog2));
    for (int p = 0; p < kRowSetProbes; ++p) {
        const unsigned long long old = atomicCAS(&set[h], ~0ull, (unsigned long long)key);
        if (old == ~0ull) return true;
        if (old == key) return false;
        h = (h + 1) & (kRowSetSlots - 1);
    }
    return true;
}

// Relabel one direction of each record through the parents: (x, y) is taken when
// (x < y) differs from the parity of x + y, which takes exactly one of (x, y) and (y, x) and
// about half of every row's records, so all rows advance through the columns at the same
// pace.  The row's parents are staged in LDS; the parents at y are gathered from the column
// block that the concurrent rows share in L2.  The row is walked in chunks of kChunk
// records; each chunk reserves its survivors' space at the end of the packed key array with
// one atomic, so the first radix pass reads full tiles (only about half of the directed
// records are taken, which would leave slabs aligned to the records half empty).
template <int kPairs>   // record pairs per thread and chunk (LC_TRELABEL_PAIRS by default)
__global__ __launch_bounds__(kTRowThreads) void k_tiled_relabel(Work w, TPlan tp, int row0) {
    constexpr int kChunk = 2 * kPairs * kTRowThreads;
    RoundState *st = w.st;
    __shared__ uint32_t lpar[1 << kTxShiftMax];
    __shared__ uint32_t lds[kTRowThreads / kWave + 1];
    __shared__ u64c sbase;
    __shared__ unsigned long long rset[kRowSetSlots];
    __shared__ uint32_t set_tries, set_drops, set_on;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->keys_dense = 1;
    for (int i = threadIdx.x; i < kRowSetSlots; i += kTRowThreads) rset[i] = ~0ull;   // no key has all bits set
    if (threadIdx.x == 0) {
        set_tries = 0;
        set_drops = 0;
        set_on = 1;
    }
    __syncthreads();
    const int64_t T = (int64_t)st->t_count;
    const int64_t nt = tiles_b_of(st);
    const int64_t n = (int64_t)st->n_cur;
    const uint64_t *rec = w.keys[1];
    uint64_t *out = w.keys[0];
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    uint32_t survived = 0;   // this thread's survivors (repeats counted)
    bool broken = false;
    // one workgroup per row of [row0, row0 + gridDim.x)
    const int row_end = min(tp.rows, row0 + (int)gridDim.x);
    for (int X = row0 + blockIdx.x; X < row_end; X += gridDim.x) {
        const int64_t base = (int64_t)X << tp.xs;
        const int cnt = (int)min((int64_t)1 << tp.xs, n - base);
        for (int i = threadIdx.x; i < cnt; i += kTRowThreads) lpar[i] = w.par[base + i];
        __syncthreads();
        int64_t start, end;
        row_range(w, tp, X, nt, T, start, end);
        for (int64_t cb = start & ~(int64_t)(kChunk - 1); cb < end; cb += kChunk) {
            uint64_t r[2 * kPairs];
            bool v[2 * kPairs];
#pragma unroll
            for (int u = 0; u < kPairs; ++u) {
                const int64_t p = cb + 2 * ((int64_t)u * kTRowThreads + threadIdx.x);
                load_pair(rec, p, end, r[2 * u], r[2 * u + 1], v[2 * u], v[2 * u + 1]);
                v[2 * u] = v[2 * u] && p >= start;
                v[2 * u + 1] = v[2 * u + 1] && p + 1 >= start;
            }
            uint32_t pb[2 * kPairs];
#pragma unroll
            for (int q = 0; q < 2 * kPairs; ++q) {
                const uint32_t x = (uint32_t)(r[q] >> 32), y = (uint32_t)r[q];
                v[q] = v[q] && ((x < y) != (((x ^ y) & 1u) != 0u));
                pb[q] = v[q] ? w.par[y] : 0u;
            }
            uint64_t key[2 * kPairs];
            uint32_t c = 0, tries = 0, drops = 0;
            const bool use_set = set_on != 0 && !w.round0_sets_off;   // read without a barrier: either
                                                                        // value is valid
#pragma unroll
            for (int q = 0; q < 2 * kPairs; ++q) {
                const int64_t xi = (int64_t)(uint32_t)(r[q] >> 32) - base;
                uint32_t pa = 0;
                if (v[q]) {
                    if (xi >= 0 && xi < cnt) {
                        pa = lpar[xi];
                    } else {
                        broken = true;
                        v[q] = false;
                    }
                }
                v[q] = v[q] && pa != pb[q];
                survived += v[q];
                const uint32_t lo = min(pa, pb[q]), hi = max(pa, pb[q]);
                key[q] = edge_key(lo, hi, kb, hbs);
                if (use_set && v[q]) {
                    ++tries;
                    if (!row_set_insert(rset, key[q])) {
                        v[q] = false;
                        ++drops;
                    }
                }
                c += v[q];
            }
            if (tries) {
                atomicAdd(&set_tries, tries);
                if (drops) atomicAdd(&set_drops, drops);
            }
            uint32_t total;
            const uint32_t off = block_excl_scan<kTRowThreads>(c, lds, &total);   // (its barriers also
                                                                                  // order the counts above)
            if (threadIdx.x == 0 && set_on && set_tries >= kRowSetTrial && 16 * set_drops < set_tries) set_on = 0;
            if (total == 0) continue;
            if (threadIdx.x == 0) sbase = atomicAdd(&st->s_keys, (u64c)total);
            __syncthreads();
            uint64_t *dst = out + sbase + off;
#pragma unroll
            for (int q = 0; q < 2 * kPairs; ++q) {
                if (v[q]) *dst++ = key[q];
            }
        }
        __syncthreads();   // lpar is rewritten for the next row
    }
    survived = block_sum<kTRowThreads>(survived, lds);
    if (threadIdx.x == 0 && survived) atomicAdd(&st->s_count, (u64c)survived);
    if (broken) atomicOr(&st->err, 4u);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

template <class R>
static hipError_t part_a(const R &rd, const Work &w, const TPlan &tp, int grid, hipStream_t s, bool scatter) {
    if (scatter)
        hipLaunchKernelGGL(k_part_a_scatter<R>, dim3(grid), dim3(kThreads), 0, s, rd, w, tp);
    else
        hipLaunchKernelGGL(k_part_a_hist<R>, dim3(grid), dim3(kThreads), 0, s, rd, w, tp);
    return hipGetLastError();
}

template <class R>
static hipError_t part_r(const R &rd, const Work &w, const TPlan &tp, int grid, hipStream_t s, bool scatter) {
    if (scatter)
        hipLaunchKernelGGL(k_part_r_scatter<R>, dim3(grid), dim3(kTbThreads), 0, s, rd, w, tp);
    else
        hipLaunchKernelGGL(k_part_r_hist<R>, dim3(grid), dim3(kTbThreads), 0, s, rd, w, tp);
    return hipGetLastError();
}

static hipError_t part_r_layout(const EdgeIn &e, const Work &w, const TPlan &tp, int grid, hipStream_t s,
                                bool scatter) {
    switch (e.layout) {
        case kSoa32:
            if (e.vec) return part_r(ReadSoa32<4>(e), w, tp, grid, s, scatter);
            return part_r(ReadSoa32<1>(e), w, tp, grid, s, scatter);
        case kSoa64:
            if (e.vec) return part_r(ReadSoa64<2>(e), w, tp, grid, s, scatter);
            return part_r(ReadSoa64<1>(e), w, tp, grid, s, scatter);
        default:
            if (e.vec) return part_r(ReadPacked<2>(e), w, tp, grid, s, scatter);
            return part_r(ReadPacked<1>(e), w, tp, grid, s, scatter);
    }
}

static hipError_t part_a_layout(const EdgeIn &e, const Work &w, const TPlan &tp, int grid, hipStream_t s,
                                bool scatter) {
    switch (e.layout) {
        case kSoa32:
            if (e.vec) return part_a(ReadSoa32<4>(e), w, tp, grid, s, scatter);
            return part_a(ReadSoa32<1>(e), w, tp, grid, s, scatter);
        case kSoa64:
            if (e.vec) return part_a(ReadSoa64<2>(e), w, tp, grid, s, scatter);
            return part_a(ReadSoa64<1>(e), w, tp, grid, s, scatter);
        default:
            if (e.vec) return part_a(ReadPacked<2>(e), w, tp, grid, s, scatter);
            return part_a(ReadPacked<1>(e), w, tp, grid, s, scatter);
    }
}

hipError_t launch_tiled_partition(const Work &w, const EdgeIn &in, const TPlan &tp, int grid, hipStream_t s,
                                  int stage) {
    switch (stage) {
        case 0:
            return part_a_layout(in, w, tp, grid, s, false);
        case 1:
        case 2:
        case 3:
            return launch_scan_u32(w.counts, w.partials, &w.st->aux_n, &w.st->t_count, grid, s, stage - 1);
        case 4:
            return part_a_layout(in, w, tp, grid, s, true);
        case 5:
            hipLaunchKernelGGL(k_part_b_hist, dim3(grid), dim3(kTbThreads), 0, s, w, tp);
            return hipGetLastError();
        case 6:
        case 7:
        case 8:
            return launch_scan_u32(w.counts, w.partials, &w.st->aux_n, nullptr, grid, s, stage - 6);
        case 9:
            hipLaunchKernelGGL(k_part_b_scatter, dim3(grid), dim3(kTbThreads), 0, s, w, tp);
            return hipGetLastError();
        case 10:
            return part_r_layout(in, w, tp, grid, s, false);
        case 11:
        case 12:
        case 13:
            return launch_scan_u32(w.counts, w.partials, &w.st->aux_n, &w.st->t_count, grid, s, stage - 11);
        case 14:
            return part_r_layout(in, w, tp, grid, s, true);
        default:
            return hipErrorInvalidValue;
    }
}

// Row kernels run in generations of `gen` rows (one workgroup per CU, all of a generation
// starting together), so that the rows in flight sweep the column blocks in step and share
// the gathered column values in L2; a single launch of every row would start late rows at
// column 0 while early ones are near the end.  gen <= 0: one launch.
template <class Launch>
static hipError_t by_generations(const TPlan &tp, int gen, Launch launch) {
    if (gen <= 0 || !LC_ROW_GENERATIONS) return launch(0, tp.rows);
    for (int r0 = 0; r0 < tp.rows; r0 += gen) {
        const hipError_t e = launch(r0, std::min(gen, tp.rows - r0));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tiled_min1(const Work &w, const PrioCtx &p, const TPlan &tp, hipStream_t s, bool open) {
    if (open)
        hipLaunchKernelGGL((k_tiled_min<1, true>), dim3(tp.rows), dim3(kTRowThreads), 0, s, w, p, tp, 0);
    else
        hipLaunchKernelGGL((k_tiled_min<1, false>), dim3(tp.rows), dim3(kTRowThreads), 0, s, w, p, tp, 0);
    return hipGetLastError();
}

// The one-hop label over the tiled round 0: the parent named by the closed one-hop minimum
// (one value per id, as the row pass left it).
__global__ __launch_bounds__(kThreads) void k_tiled_parent1(Work w, PrioCtx pc) {
    RoundState *st = w.st;
    pc.key = st->key;
    const int64_t n = (int64_t)st->n_cur;
    uint32_t active = 0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const uint32_t a = w.ml[x];
        if (a == kInf) {
            w.par[x] = (uint32_t)x;
            continue;
        }
        const uint32_t p = prio_inv(pc.key, a);
        w.par[x] = p;
        w.is_label[p] = 1;
        ++active;
    }
    __shared__ uint32_t red[kThreads / kWave];
    active = block_sum<kThreads>(active, red);
    if (threadIdx.x == 0 && active) atomicAdd(&st->n_active, (u64c)active);
}

hipError_t launch_tiled_parent1(const Work &w, const PrioCtx &p, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_tiled_parent1, dim3(grid), dim3(kThreads), 0, s, w, p);
    return hipGetLastError();
}

hipError_t launch_tiled_min2(const Work &w, const PrioCtx &p, const TPlan &tp, hipStream_t s, int gen, int pairs) {
    return by_generations(tp, gen, [&](int r0, int g) {
        if (pairs == 2)
            hipLaunchKernelGGL((k_tiled_min<2, false, 2>), dim3(g), dim3(kTRowThreads), 0, s, w, p, tp, r0);
        else if (pairs == 8)
            hipLaunchKernelGGL((k_tiled_min<2, false, 8>), dim3(g), dim3(kTRowThreads), 0, s, w, p, tp, r0);
        else
            hipLaunchKernelGGL((k_tiled_min<2, false, 4>), dim3(g), dim3(kTRowThreads), 0, s, w, p, tp, r0);
        return hipGetLastError();
    });
}

hipError_t launch_tiled_relabel(const Work &w, const TPlan &tp, hipStream_t s, int gen, int pairs) {
    return by_generations(tp, gen, [&](int r0, int g) {
        if (pairs == 1)
            hipLaunchKernelGGL(k_tiled_relabel<1>, dim3(g), dim3(kTRowThreads), 0, s, w, tp, r0);
        else if (pairs == 4)
            hipLaunchKernelGGL(k_tiled_relabel<4>, dim3(g), dim3(kTRowThreads), 0, s, w, tp, r0);
        else
            hipLaunchKernelGGL(k_tiled_relabel<2>, dim3(g), dim3(kTRowThreads), 0, s, w, tp, r0);
        return hipGetLastError();
    });
}

}  // namespace lc
