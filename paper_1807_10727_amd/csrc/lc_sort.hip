// Scans, LSD radix sort and unique for the duplicate-dropping step of a round (the
// contraction step keeps one copy of each edge between two different parents; proof of
// the contraction-step lemma, Section 3).
//
// Sort: least-significant-digit radix sort of the round's survivor keys
// (lo << b | hi, b = ceil(log2 N_r)), 8-bit digits, only as many passes as the key has
// bits.  Each pass: per-tile digit counts (wave-aggregated LDS atomics), an exclusive scan
// of the digit-major count table, then a scatter in which each 4096-key tile is ranked
// stably in LDS (wave ballots find lanes with equal digits; per-wave digit counters give
// the order across iterations and waves), staged in LDS in sorted order and written out
// as contiguous runs per digit.
// Unique: a head flag per sorted key, per-tile counts (which also mark both endpoints of
// every kept edge as nodes of the next graph), one-workgroup scan; after the next graph's
// index is known, an ordered write of the heads renamed into it.

#include "lc_steps.hpp"

namespace lc {

// ---------------------------------------------------------------------------------------
// generic exclusive scan of uint8 or uint32 values into uint32 (count on the device)
// ---------------------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const T *in, const u64c *n_ptr, uint32_t *partials) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t nblk = ceil_div(n, kScanTile);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        uint32_t v[16];
        load16(in, blk * kScanTile + threadIdx.x * 16, n, v);
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) sum += v[j];
        uint32_t total;
        block_excl_scan<kThreads>(sum, lds, &total);
        if (threadIdx.x == 0) partials[blk] = total;
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_single(uint32_t *data, const u64c *n_ptr, int per_entry,
                                                          u64c *total_out) {
    step_scan_single(data, n_ptr, per_entry, total_out);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_down(const T *in, uint32_t *out, const u64c *n_ptr,
                                                        const uint32_t *partials) {
    __shared__ uint32_t lds[kThreads / kWave + 1];
    const int64_t n = (int64_t)*n_ptr;
    const int64_t nblk = ceil_div(n, kScanTile);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        uint32_t v[16];
        const int64_t my = blk * kScanTile + threadIdx.x * 16;
        load16(in, my, n, v);
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) sum += v[j];
        uint32_t total;
        uint32_t run = partials[blk] + block_excl_scan<kThreads>(sum, lds, &total);
        uint32_t o[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            o[j] = run;
            run += v[j];
        }
        if (my + 16 <= n) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *(uint4 *)(out + my + 4 * q) = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (my + j < n) out[my + j] = o[j];
        }
    }
}

// ---------------------------------------------------------------------------------------
// radix sort passes
// ---------------------------------------------------------------------------------------

// Keys stream through each radix pass once: non-temporal loads leave L2 to the per-tile
// tables and the output runs (measured: count pass ~11 % faster, scatter ~2 %).
#ifndef LC_NT_KEYS
#define LC_NT_KEYS 1
#endif
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));

__device__ inline bool is_leader(uint64_t peers) { return (int)(__ffsll((long long)peers) - 1) == lane_id(); }

// gated: the round chose its duplicate drop on the device, and a hashed choice (hash_slots
// nonzero) skips the sort (an empty count table, so the scans that follow do nothing)
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(Work w, int pass, int gated) {
    RoundState *st = w.st;
    const int passes = npasses(st->nbits);
    if (pass >= passes || (gated && st->hash_slots != 0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->aux_n = 0;
        return;
    }
    int shift, width;
    pass_digit(st->nbits, pass, shift, width);
    const int nbins = 1 << width;
    const uint32_t dmask = (uint32_t)nbins - 1u;
    const Tiles tl = tiles_of(w, pass);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->aux_n = (u64c)nbins * (u64c)tl.ntiles;
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel) ^ (pass & 1)];
    __shared__ uint32_t hist[kRadixMax];
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < tl.ntiles; tile += gridDim.x) {
        const int tv = tl.valid(tile);
        for (int i = threadIdx.x; i < nbins; i += kSortThreads) hist[i] = 0;
        // every load of the tile in flight at once: pairs of keys, 16-byte aligned
        uint32_t d[kSortItems];
        bool valid[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems / 2; ++j) {
            const int it = 2 * (j * kSortThreads + threadIdx.x);
            uint64_t k0 = 0, k1 = 0;
            if (it + 1 < tv) {
                const u64x2_t x = LC_NT_KEYS ? __builtin_nontemporal_load((const u64x2_t *)(in + tile * kSortTile + it))
                                             : *(const u64x2_t *)(in + tile * kSortTile + it);
                k0 = x.x;
                k1 = x.y;
            } else if (it < tv) {
                k0 = in[tile * kSortTile + it];
            }
            valid[2 * j] = it < tv;
            valid[2 * j + 1] = it + 1 < tv;
            d[2 * j] = (uint32_t)(k0 >> shift) & dmask;
            d[2 * j + 1] = (uint32_t)(k1 >> shift) & dmask;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const uint64_t act = ballot(valid[j]);
            if (!act) continue;
            const int first = __ffsll((long long)act) - 1;
            const uint32_t d0 = __shfl(d[j], first, kWave);
            if (ballot(valid[j] && d[j] == d0) == act) {
                if (lane_id() == first) atomicAdd(&hist[d0], (uint32_t)__popcll(act));
            } else if (valid[j]) {
                atomicAdd(&hist[d[j]], 1u);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nbins; i += kSortThreads) w.counts[(int64_t)i * tl.ntiles + tile] = hist[i];
        __syncthreads();
    }
}

// Waves per SIMD the scatter is compiled for: 3 (the default, LC_SCATTER_WAVES) trades a few
// spilled words for a third more waves in flight than the unconstrained register count
// allows (measured faster on the bench graph).  Builds for 2 and 4 waves exist for the tuner.
//
// kSweep: the one-sweep form (cc_tuning.radix_form = 2).  No count pass or scan precedes the
// scatter: every digit's start in the output is known from k_sweep_count, and a tile finds
// how many keys of each digit the tiles before it hold by decoupled look-back.  Tiles are
// numbered in the order workgroups take them (a counter per pass), so a tile only ever waits
// for tiles that running workgroups already hold, whatever the grid.  Each tile publishes, per
// digit, first its own count (an aggregate) and then, once its look-back is done, the count
// of that digit in itself and every tile before it (an inclusive prefix, kSweepPrefix set).
// The look-back of digit d walks back over the previous tiles' words, adding aggregates,
// until it meets a prefix; a word still empty is polled again.  The words of a pass live in
// one of two tables, and every tile of pass p empties its own words in the other table for
// pass p + 1 (the count pass empties the first one).
template <int kWavesPerSimd, bool kSweep>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd)))
void k_sort_scatter(Work w, int pass, int gated) {
    RoundState *st = w.st;
    const int passes = npasses(st->nbits);
    if (pass >= passes || (gated && st->hash_slots != 0)) return;
    if (kSweep && st->s_keys >= (u64c)kSweepMaxKeys) return;   // flagged by k_sweep_count
    int shift, width;
    pass_digit(st->nbits, pass, shift, width);
    const int nbins = 1 << width;
    const uint32_t dmask = (uint32_t)nbins - 1u;
    const Tiles tl = tiles_of(w, pass);
    const int64_t ntiles = tl.ntiles;
    const int src = sort_src(st->round, st->e_sel) ^ (pass & 1);
    const uint64_t *in = w.keys[src];
    uint64_t *out = w.keys[src ^ 1];
    uint32_t *desc = (pass & 1) ? w.sweep_desc : w.counts;        // this pass's look-back words
    uint32_t *desc_next = (pass & 1) ? w.counts : w.sweep_desc;   // the next pass's

    constexpr int kWaves = kSortThreads / kWave;
    constexpr int kPer = (kRadixMax + kSortThreads - 1) / kSortThreads;   // digits per thread at most
    __shared__ uint32_t wcnt[kWaves][kRadixMax];
    __shared__ uint64_t skeys[kSortTile];
    __shared__ uint32_t dstart[kRadixMax];
    __shared__ uint32_t gofs[kRadixMax];
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint32_t base[kSweep ? kRadixMax : 1];   // one sweep: each digit's start in the output
    __shared__ int64_t s_tile;

    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    // thread t owns digits [t * per, (t + 1) * per) of this pass
    const int per = nbins > kSortThreads ? nbins / kSortThreads : 1;

    if (kSweep) {   // digit starts: exclusive prefix of the pass's digit totals
        uint32_t c[kPer];
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int d = threadIdx.x * per + q;
            c[q] = (q < per && d < nbins) ? w.sweep[pass * kRadixMax + d] : 0u;
            sum += c[q];
        }
        uint32_t total;
        uint32_t run = block_excl_scan<kSortThreads>(sum, lds, &total);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int d = threadIdx.x * per + q;
            if (q < per && d < nbins) base[d] = run;
            run += c[q];
        }
    }

    int64_t tile = xcd_rank(blockIdx.x, gridDim.x);
    for (;;) {
        if (kSweep) {   // the next tile in the order workgroups ask for one
            if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(&w.sweep[kMaxPasses * kRadixMax + pass], 1u);
            __syncthreads();
            tile = s_tile;
        }
        if (tile >= ntiles) break;
        const int tv = tl.valid(tile);
        // this tile's global digit offsets: loaded now, used after the ranking
        uint32_t my_gofs[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int d = threadIdx.x * per + q;
            my_gofs[q] = (!kSweep && q < per && d < nbins) ? w.counts[(int64_t)d * ntiles + tile] : 0u;
        }
        if (kSweep)
            for (int i = threadIdx.x; i < kRadixMax; i += kSortThreads) desc_next[tile * kRadixMax + i] = kSweepEmpty;
        for (int i = threadIdx.x; i < kWaves * kRadixMax; i += kSortThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();

        // Slab tiles of the first pass are often partly or wholly empty: positions past tv
        // are neither ranked nor staged, and rows of the tile with no valid key are skipped.
        uint64_t k[kSortItems];
        uint32_t rk[kSortItems];
        const int wbase = wave * (kSortItems * kWave);
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int it = wbase + j * kWave + lane;
            k[j] = it < tv ? (LC_NT_KEYS ? __builtin_nontemporal_load(in + tile * kSortTile + it) : in[tile * kSortTile + it])
                           : ~0ull;
        }
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (wbase + j * kWave >= tv) break;   // uniform over the wave
            const bool valid = wbase + j * kWave + lane < tv;
            const uint32_t d = (uint32_t)(k[j] >> shift) & dmask;
            const uint64_t peers = match_bits<kRadixMaxBits>(d, ballot(valid));
            uint32_t cur = 0;
            if (valid) cur = wcnt[wave][d];
            rk[j] = cur + (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && is_leader(peers)) wcnt[wave][d] = cur + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();

        {   // per digit: prefix over waves, start within the tile, global offset
            uint32_t tot[kPer];
            uint32_t sum = 0;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int d = threadIdx.x * per + q;
                uint32_t run = 0;
                if (q < per && d < nbins) {
#pragma unroll
                    for (int v = 0; v < kWaves; ++v) {
                        const uint32_t c = wcnt[v][d];
                        wcnt[v][d] = run;
                        run += c;
                    }
                }
                tot[q] = run;
                sum += run;
            }
            if (kSweep) {
                // publish this tile's own counts, then look back for the keys before it
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int d = threadIdx.x * per + q;
                    if (q < per && d < nbins)
                        store_agent(&desc[tile * kRadixMax + d], tile == 0 ? (kSweepPrefix | tot[q]) : tot[q]);
                }
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int d = threadIdx.x * per + q;
                    if (q < per && d < nbins && tile > 0) {
                        uint32_t before = 0, polls = 0;
                        for (int64_t j = tile - 1; j >= 0;) {
                            const uint32_t v = load_agent(&desc[j * kRadixMax + d]);
                            if (v == kSweepEmpty) {   // not published yet: poll again
                                if (++polls > kSweepMaxPolls) {   // never published: flagged, not waited for
                                    atomicOr(&st->err, 4u);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                                continue;
                            }
                            before += v & ~kSweepPrefix;
                            if (v & kSweepPrefix) break;
                            --j;
                        }
                        store_agent(&desc[tile * kRadixMax + d], kSweepPrefix | (before + tot[q]));
                        my_gofs[q] = base[d] + before;
                    } else if (q < per && d < nbins) {
                        my_gofs[q] = base[d];
                    }
                }
            }
            uint32_t total;
            uint32_t ds = block_excl_scan<kSortThreads>(sum, lds, &total);
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int d = threadIdx.x * per + q;
                if (q < per && d < nbins) {
                    dstart[d] = ds;
                    gofs[d] = my_gofs[q];
                }
                ds += tot[q];
            }
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (wbase + j * kWave + lane < tv) {
                const uint32_t d = (uint32_t)(k[j] >> shift) & dmask;
                skeys[dstart[d] + wcnt[wave][d] + rk[j]] = k[j];
            }
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int pos = j * kSortThreads + threadIdx.x;
            if (pos < tv) {
                const uint64_t kk = skeys[pos];
                const uint32_t d = (uint32_t)(kk >> shift) & dmask;
                out[gofs[d] + (uint32_t)pos - dstart[d]] = kk;
            }
        }
        __syncthreads();
        if (!kSweep) tile += gridDim.x;
    }
}

// One sweep, before the scatters: the digit totals of every pass from one read of the keys
// (wave-aggregated LDS counts, one global add per digit and workgroup), and the first pass's
// look-back words emptied.  k_sweep_reset zeroes the totals and the tile counters before it.
__global__ __launch_bounds__(kSortThreads) void k_sweep_count(Work w, int gated) {
    RoundState *st = w.st;
    if (gated && st->hash_slots != 0) return;   // the round hashed
    if (st->s_keys >= (u64c)kSweepMaxKeys) {      // a prefix word could not hold the counts
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->err, 4u);
        return;
    }
    const int nbits = st->nbits;
    const int passes = npasses(nbits);
    const Tiles tl = tiles_of(w, 0);
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel)];
    __shared__ uint32_t hist[kMaxPasses * kRadixMax];
    for (int i = threadIdx.x; i < kMaxPasses * kRadixMax; i += kSortThreads) hist[i] = 0;
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < tl.ntiles * kRadixMax;
         i += (int64_t)gridDim.x * kSortThreads)
        w.counts[i] = kSweepEmpty;
    // every pass's digit position, worked out once
    int shifts[kMaxPasses];
    uint32_t masks[kMaxPasses];
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) {
        int width = 0;
        shifts[p] = 0;
        if (p < passes) pass_digit(nbits, p, shifts[p], width);
        masks[p] = (1u << width) - 1u;
    }
    __syncthreads();
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < tl.ntiles; tile += gridDim.x) {
        const int tv = tl.valid(tile);
        if (tv == 0) continue;   // uniform over the workgroup
#pragma unroll 4
        for (int j = 0; j < kSortItems; ++j) {
            const int it = j * kSortThreads + threadIdx.x;
            const bool valid = it < tv;
            const uint64_t k = valid ? in[tile * kSortTile + it] : 0ull;
            const uint64_t act = ballot(valid);
            if (!act) continue;   // uniform over the wave
            const int first = __ffsll((long long)act) - 1;
#pragma unroll
            for (int p = 0; p < kMaxPasses; ++p) {
                if (p >= passes) break;   // uniform
                const uint32_t d = (uint32_t)(k >> shifts[p]) & masks[p];
                const uint32_t d0 = __shfl(d, first, kWave);
                if (ballot(valid && d == d0) == act) {   // the whole wave in one digit: one add
                    if (lane_id() == first) atomicAdd(&hist[p * kRadixMax + d0], (uint32_t)__popcll(act));
                } else if (valid) {
                    atomicAdd(&hist[p * kRadixMax + d], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * kRadixMax; i += kSortThreads)
        if (hist[i]) atomicAdd(&w.sweep[i], hist[i]);
}

__global__ __launch_bounds__(kSortThreads) void k_sweep_reset(Work w, int gated) {
    if (gated && w.st->hash_slots != 0) return;
    for (int i = threadIdx.x; i < kSweepWords; i += kSortThreads) w.sweep[i] = 0;
}

// ---------------------------------------------------------------------------------------
// next-graph node map: prefix counts over the bit words
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_flags_reduce(const uint8_t *f, const u64c *n_ptr, uint32_t *partials) {
    step_flags_reduce(f, n_ptr, partials);
}

__global__ __launch_bounds__(kThreads) void k_flags_down(const uint8_t *f, const u64c *n_ptr,
                                                         const uint32_t *partials, uint32_t *lmap) {
    step_flags_down(f, n_ptr, partials, lmap);
}

__global__ __launch_bounds__(kThreads) void k_flags_single(const uint8_t *f, const u64c *n_ptr, uint32_t *map,
                                                           u64c *total_out) {
    step_flags_single(f, n_ptr, map, total_out);
}

// ---------------------------------------------------------------------------------------
// unique
// ---------------------------------------------------------------------------------------

// Heads (first key of every run of equal sorted keys) per tile, and the next graph's node
// marks: both endpoints of every kept edge (the endpoints of all survivors, the same set).
// Keys with equal lo are adjacent, so lo is marked by the first key of its run only.
__global__ __launch_bounds__(kSortThreads) void k_unique_count(Work w, int gated) {
    RoundState *st = w.st;
    if (gated && st->hash_slots != 0) return;   // the round hashed
    __shared__ uint32_t lds[kSortThreads / kWave + 1];
    const int64_t S = (int64_t)st->s_keys;
    const int64_t ntiles = ceil_div(S, kSortTile);
    if (blockIdx.x == 0 && threadIdx.x == 0) st->aux_n = (u64c)ntiles;
    const uint64_t *in = w.keys[sorted_sel(st->round, st->e_sel, st->nbits)];
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    const uint64_t n_lab = st->n_labels;   // key endpoints are label ranks
    bool broken = false;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        uint32_t cnt = 0;
        // every load of the tile in flight before any key is looked at
        uint64_t kk[kSortItems], pk[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {   // consecutive lanes take consecutive keys
            const int64_t idx = tile * kSortTile + j * kSortThreads + threadIdx.x;
            kk[j] = idx < S ? in[idx] : 0ull;
            pk[j] = (idx > 0 && idx < S) ? in[idx - 1] : ~0ull;
        }
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int64_t idx = tile * kSortTile + j * kSortThreads + threadIdx.x;
            const uint64_t k = kk[j], prev = pk[j];
            if (idx < S && (idx == 0 || k != prev)) {
                ++cnt;
                uint64_t lo, hi, plo = ~0ull, phi;
                edge_key_split(k, kb, hbs, lo, hi);
                if (idx > 0) edge_key_split(prev, kb, hbs, plo, phi);
                if (lo < n_lab && hi < n_lab) {
                    if (plo != lo) w.has_edge[lo] = 1;
                    w.has_edge[hi] = 1;
                } else {
                    broken = true;
                }
            }
        }
        uint32_t total;
        block_excl_scan<kSortThreads>(cnt, lds, &total);
        if (threadIdx.x == 0) w.tile_cnt[tile] = total;
    }
    if (broken) atomicOr(&st->err, 4u);
}

// The next graph's edge list: the heads, in sorted order, renamed into the next round's
// compact index space (nmap_rank), written to the other key buffer.  Row j of a tile is the
// kSortThreads consecutive keys [j * kSortThreads, (j + 1) * kSortThreads): a wave ballot
// per row and a prefix over (row, wave) give each head its place, so consecutive lanes read,
// gather and write consecutive keys.
__global__ __launch_bounds__(kSortThreads) void k_unique_write(Work w, int gated) {
    constexpr int kWaves = kSortThreads / kWave;
    RoundState *st = w.st;
    if (gated && st->hash_slots != 0) return;   // the round hashed
    __shared__ uint32_t rowcnt[kSortItems * kWaves];
    const int64_t S = (int64_t)st->s_keys;
    const int64_t ntiles = ceil_div(S, kSortTile);
    const int t = sorted_sel(st->round, st->e_sel, st->nbits);
    const uint64_t *in = w.keys[t];
    uint64_t *out = w.keys[1 - t];
    const int kb = st->kb;
    const int hbs = st->hb_shift;
    const uint64_t n_lab = st->n_labels;   // key endpoints are label ranks
    // every label keeps an edge (none is final this round): the next round's index of label
    // q is q itself, and the renaming lookups are skipped
    const bool same = st->n_next == n_lab;
    const int wave = threadIdx.x / kWave;
    const uint64_t lt = lanemask_lt();
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        uint64_t k[kSortItems];
        bool h[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int64_t idx = tile * kSortTile + j * kSortThreads + threadIdx.x;
            k[j] = idx < S ? in[idx] : 0ull;
            const uint64_t prev = (idx > 0 && idx < S) ? in[idx - 1] : ~0ull;
            h[j] = idx < S && (idx == 0 || k[j] != prev);
        }
        uint64_t bal[kSortItems];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            bal[j] = ballot(h[j]);
            if (lane_id() == 0) rowcnt[j * kWaves + wave] = (uint32_t)__popcll(bal[j]);
        }
        __syncthreads();
        static_assert(kSortItems * kWaves == kWave, "one (row, wave) count per lane of wave 0");
        if (threadIdx.x < kWave) {   // exclusive prefix over (row, wave) in key order
            const uint32_t c = rowcnt[threadIdx.x];
            rowcnt[threadIdx.x] = (uint32_t)w.tile_cnt[tile] + wave_incl_scan(c) - c;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (h[j]) {
                const uint32_t off = rowcnt[j * kWaves + wave] + (uint32_t)__popcll(bal[j] & lt);
                uint64_t lo, hi;
                edge_key_split(k[j], kb, hbs, lo, hi);
                // ids were checked by the count pass (a failed check flags the round)
                const uint32_t a = lo < n_lab ? (same ? (uint32_t)lo : nmap_rank(w.nmap, lo)) : 0u;
                const uint32_t b = hi < n_lab ? (same ? (uint32_t)hi : nmap_rank(w.nmap, hi)) : 0u;
                out[off] = ((uint64_t)a << 32) | b;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// duplicate drop by hashing (small rounds)
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_hash_clear(Work w, int decide) {
    step_hash_clear(w, decide);
}

__global__ __launch_bounds__(kSortThreads) void k_hash_insert(Work w) {
    step_hash_insert(w);
}

__global__ __launch_bounds__(kSortThreads) void k_hash_count(Work w) {
    step_hash_count(w);
}

__global__ __launch_bounds__(kSortThreads) void k_hash_write(Work w) {
    step_hash_write(w);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------

hipError_t launch_scan_u32(uint32_t *data, uint32_t *partials, const u64c *n, u64c *total, int grid, hipStream_t s,
                           int stage) {
    if (stage == 0)
        hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3(grid), dim3(kThreads), 0, s, (const uint32_t *)data, n,
                           partials);
    else if (stage == 1)
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kThreads), 0, s, partials, n, kScanTile, total);
    else
        hipLaunchKernelGGL(k_scan_down<uint32_t>, dim3(grid), dim3(kThreads), 0, s, (const uint32_t *)data, data, n,
                           (const uint32_t *)partials);
    return hipGetLastError();
}

template <bool kSweep>
static hipError_t launch_scatter(const Work &w, int pass, int grid, hipStream_t s, bool gated, int scatter_waves) {
    const dim3 g(grid), b(kSortThreads);
    if (scatter_waves == 2)
        hipLaunchKernelGGL((k_sort_scatter<2, kSweep>), g, b, 0, s, w, pass, (int)gated);
    else if (scatter_waves == 4)
        hipLaunchKernelGGL((k_sort_scatter<4, kSweep>), g, b, 0, s, w, pass, (int)gated);
    else
        hipLaunchKernelGGL((k_sort_scatter<3, kSweep>), g, b, 0, s, w, pass, (int)gated);
    return hipGetLastError();
}

hipError_t launch_sort_pass(const Work &w, int pass, int grid, hipStream_t s, int stage, bool gated,
                            int scatter_waves) {
    switch (stage) {
        case 5:   // the count table scanned by one workgroup (small rounds)
            hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kThreads), 0, s, w.counts, &w.st->aux_n, 0,
                               (u64c *)nullptr);
            return hipGetLastError();
        case 0:
            hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kSortThreads), 0, s, w, pass, (int)gated);
            return hipGetLastError();
        case 1:
        case 2:
        case 3:
            return launch_scan_u32(w.counts, w.partials, &w.st->aux_n, nullptr, grid, s, stage - 1);
        case 6:   // one sweep: totals and tile counters zeroed
            hipLaunchKernelGGL(k_sweep_reset, dim3(1), dim3(kSortThreads), 0, s, w, (int)gated);
            return hipGetLastError();
        case 7:   // one sweep: the digit totals of every pass
            hipLaunchKernelGGL(k_sweep_count, dim3(grid), dim3(kSortThreads), 0, s, w, (int)gated);
            return hipGetLastError();
        case 8:   // one sweep: the scatter of pass `pass`, its offsets by look-back
            return launch_scatter<true>(w, pass, grid, s, gated, scatter_waves);
        default:
            return launch_scatter<false>(w, pass, grid, s, gated, scatter_waves);
    }
}

hipError_t launch_map_scan(const Work &w, bool labels, int grid, hipStream_t s, int stage) {
    // label map: flags of this round's nodes; node map: flags of the labels
    const uint8_t *f = labels ? w.is_label : w.has_edge;
    uint32_t *map = labels ? w.lmap : w.nmap;
    const u64c *n = labels ? &w.st->n_cur : &w.st->n_labels;
    u64c *total = labels ? &w.st->n_labels : &w.st->n_next;
    if (stage == 0)
        hipLaunchKernelGGL(k_flags_reduce, dim3(grid), dim3(kThreads), 0, s, f, n, w.partials);
    else if (stage == 1)   // one partial per kThreads words of 32 flags
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kThreads), 0, s, w.partials, n, 32 * kThreads, total);
    else if (stage == 2)
        hipLaunchKernelGGL(k_flags_down, dim3(grid), dim3(kThreads), 0, s, f, n, (const uint32_t *)w.partials, map);
    else   // all of it in one workgroup (small rounds)
        hipLaunchKernelGGL(k_flags_single, dim3(1), dim3(kThreads), 0, s, f, n, map, total);
    return hipGetLastError();
}

hipError_t launch_hash_dedup(const Work &w, int grid, hipStream_t s, int stage, bool decide) {
    switch (stage) {
        case 1:
            hipLaunchKernelGGL(k_hash_clear, dim3(grid), dim3(kThreads), 0, s, w, (int)decide);
            break;
        case 2:
            hipLaunchKernelGGL(k_hash_insert, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        case 3:
            hipLaunchKernelGGL(k_hash_count, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        default:
            hipLaunchKernelGGL(k_hash_write, dim3(grid), dim3(kSortThreads), 0, s, w);
    }
    return hipGetLastError();
}

hipError_t launch_unique(const Work &w, int grid, hipStream_t s, int stage, bool gated) {
    if (stage == 0)
        hipLaunchKernelGGL(k_unique_count, dim3(grid), dim3(kSortThreads), 0, s, w, (int)gated);
    else if (stage == 1)
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kThreads), 0, s, w.tile_cnt, &w.st->aux_n, 0,
                           &w.st->m_next);
    else
        hipLaunchKernelGGL(k_unique_write, dim3(grid), dim3(kSortThreads), 0, s, w, (int)gated);
    return hipGetLastError();
}

}  // namespace lc
