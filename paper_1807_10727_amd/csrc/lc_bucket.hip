// Sampled-bucket duplicate drop of round 0: a tuning alternative to the LSD radix passes.
//
// The contraction step keeps one copy of each edge between two different parents (proof of
// the contraction-step lemma, Section 3); the unique passes that follow need only the round's
// keys in ascending order.  The radix passes read and write every key once per 8-bit digit
// (five or six times on round 0's 38-46-bit keys).  Here the keys move twice instead, into
// buckets of ascending key ranges, and each final bucket is sorted inside LDS:
//
//   level 1   splitters from a sorted sample of the keys (one workgroup), then a count and a
//             scatter pass that put every key into one of up to 256 buckets;
//   level 2   the same inside every first-level bucket (its own sample and splitters), the
//             tiles of a pass never crossing a first-level bucket;
//   final     one workgroup per final bucket (up to 65,536 of them, ~K / 65,536 keys each)
//             sorts the bucket in LDS and writes it where the radix passes would have left
//             the keys.  A bucket larger than LDS holds is sorted in place by the same
//             network, its chunk-local stages in LDS and only the others in global memory
//             (rare: buckets average half the capacity at 2^28 keys, and a heavy key gets a
//             bucket of its own, which needs no sort).
//
// Splitters only decide where the buckets are cut, never what the result is: every key lands
// in the one bucket whose range holds it, buckets follow in key order, and every bucket ends
// up sorted.  Sampling therefore needs no randomness.

#include "lc_internal.hpp"

namespace lc {

constexpr int kBkSampleThreads = 1024;
constexpr int kBkSample1 = 8192;   // keys sampled for the first level (one workgroup, 64 KB)
#ifndef LC_BUCKET_SAMPLE2
#define LC_BUCKET_SAMPLE2 4096     // keys sampled in each first-level bucket
#endif
constexpr int kBkSample2 = LC_BUCKET_SAMPLE2;
#ifndef LC_BUCKET_CAP
#define LC_BUCKET_CAP 8192         // keys of a final bucket sorted in LDS (64 KB)
#endif
constexpr int kBkCap = LC_BUCKET_CAP;
constexpr int kBkSegs = 256;       // first-level buckets
static_assert(kSortThreads == 256, "the bucket passes give each thread one of the 256 buckets");

// Ascending sort of a[0, n) by the bitonic network of the next power of two in its
// all-ascending form (the first comparator of each merge mirrors the block), whose
// comparators always put the smaller key at the lower index.  Positions from n up are
// treated as +infinity: every comparator that reaches one keeps its keys where they are, so
// they are never read or written.  One stage: merge size k, comparator distance j, over
// `half` comparator slots (half the network's size); the caller orders stages with barriers.
template <typename Idx>
__device__ inline void network_stage(uint64_t *a, Idx n, Idx half, Idx k, Idx j) {
    const bool mirror = j == (k >> 1);
    const int sh = __builtin_ctzll((unsigned long long)j);
    for (Idx t = threadIdx.x; t < half; t += blockDim.x) {
        const Idx i = ((t >> sh) << (sh + 1)) | (t & (j - 1));   // bit sh of i is 0
        const Idx l = mirror ? (i ^ (k - 1)) : (i | j);        // l > i
        if (l < n) {
            const uint64_t x = a[i], y = a[l];
            if (y < x) {
                a[i] = y;
                a[l] = x;
            }
        }
    }
}

template <typename Idx>
__device__ void sort_network(uint64_t *a, Idx n) {
    Idx N = 1;
    while (N < n) N <<= 1;
    for (Idx k = 2; k <= N; k <<= 1) {
        for (Idx j = k >> 1; j > 0; j >>= 1) {
            network_stage<Idx>(a, n, N >> 1, k, j);
            __syncthreads();
        }
    }
}

// The same network for a bucket larger than LDS holds, g[0, n) in global memory, with the
// stages that stay inside one LDS-sized chunk run in LDS (`lds`: kBkCap keys): first every
// chunk is sorted there (the stages of merge size up to kBkCap), then, for each larger merge
// size, the stages whose comparators cross chunks run in global memory and the rest chunk by
// chunk in LDS.  Only log2(n / kBkCap) (log2(n / kBkCap) + 1) / 2 stages touch global memory.
__device__ void sort_large(uint64_t *g, int64_t n, uint64_t *lds) {
    int64_t N = 1;
    while (N < n) N <<= 1;
    auto chunk_pass = [&](bool full) {
        for (int64_t c0 = 0; c0 < n; c0 += kBkCap) {
            const int len = (int)(n - c0 < kBkCap ? n - c0 : kBkCap);
            for (int i = threadIdx.x; i < len; i += blockDim.x) lds[i] = g[c0 + i];
            __syncthreads();
            if (full) {
                sort_network<int>(lds, len);
            } else {   // half-cleaners only (a merge size above kBkCap never mirrors here)
                for (int j = kBkCap >> 1; j > 0; j >>= 1) {
                    network_stage<int>(lds, len, kBkCap >> 1, 2 * kBkCap, j);
                    __syncthreads();
                }
            }
            for (int i = threadIdx.x; i < len; i += blockDim.x) g[c0 + i] = lds[i];
            __syncthreads();
        }
    };
    chunk_pass(true);
    for (int64_t k = 2 * (int64_t)kBkCap; k <= N; k <<= 1) {
        for (int64_t j = k >> 1; j >= kBkCap; j >>= 1) {
            network_stage<int64_t>(g, n, N >> 1, k, j);
            __syncthreads();
        }
        chunk_pass(false);
    }
}

// Splitters from a sorted sample s[0, S) (thread 0): the sample values at ranks j S / 256,
// j = 1 .. 255; a value met at several of those ranks is heavy and gets its own bucket.
__device__ void build_tab(BucketTab *T, const uint64_t *s, int S) {
    int m = 0;
    if (S > 0) {
        int j = 1;
        while (j < 256) {
            const uint64_t v = s[((int64_t)j * S) >> 8];
            int mult = 0;
            while (j < 256 && s[((int64_t)j * S) >> 8] == v) {
                ++mult;
                ++j;
            }
            T->u[m] = v;
            T->heavy[m] = mult >= 2 ? 1 : 0;
            ++m;
        }
    }
    for (int b = 0; b < 256; ++b) T->eqb[b] = 0;
    int next = 0;
    for (int i = 0; i < m; ++i) {
        T->open_id[i] = (uint8_t)next++;
        if (T->heavy[i]) {
            T->eq_id[i] = (uint8_t)next;
            T->eqb[next] = 1;
            ++next;
        }
    }
    T->open_id[m] = (uint8_t)next++;   // light splitters use one rank each, heavy ones two: next <= 256
    T->m = m;
    T->nb = next;
}

__device__ inline uint32_t bucket_of(const BucketTab &T, uint64_t k) {
    int lo = 0, hi = T.m;   // the first splitter >= k
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (T.u[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < T.m && T.heavy[lo] && T.u[lo] == k) return T.eq_id[lo];
    return T.open_id[lo];
}

__device__ inline void load_tab(BucketTab &dst, const BucketTab *src) {
    const uint4 *s = (const uint4 *)src;
    uint4 *d = (uint4 *)&dst;
    for (int i = threadIdx.x; i < (int)(sizeof(BucketTab) / 16); i += blockDim.x) d[i] = s[i];
}

__device__ inline uint64_t mix_index(uint64_t i) {   // a fixed scramble of sample offsets
    i = (i ^ (i >> 31)) * 0x7FB5D329728EA185ull;
    return i ^ (i >> 27);
}

// ---- tile geometry of the two levels ------------------------------------------------------

// Level 1 reads the relabel's output (packed, or in slabs) through the radix passes' first
// tiles; level 2 reads the first level's output in tiles that stay inside one first-level
// bucket.  tile(): the tile's keys [off, off + valid), its bucket table, and where its
// count of digit d sits in the count table (base + d * stride).
template <int kLevel>
struct BkTiles {
    Tiles tl;                   // level 1
    const uint64_t *seg;        // level 2 (LDS copies)
    const uint32_t *tb;
    int64_t ntiles;
    __device__ void tile(int64_t t, int64_t &off, int &valid, int &tab, int64_t &base, int64_t &stride) const {
        if (kLevel == 1) {
            off = t * kSortTile;
            valid = tl.valid(t);
            tab = 0;
            base = t;
            stride = ntiles;
        } else {
            int lo = 0, hi = kBkSegs - 1;   // the bucket b with tb[b] <= t < tb[b + 1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((int64_t)tb[mid] <= t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int64_t first = tb[lo];
            off = (int64_t)seg[lo] + (t - first) * kSortTile;
            const int64_t rest = (int64_t)seg[lo + 1] - off;
            valid = (int)(rest < kSortTile ? rest : kSortTile);
            tab = 1 + lo;
            base = (int64_t)kBkSegs * first + (t - first);
            stride = (int64_t)tb[lo + 1] - first;
        }
    }
};

// ---- stage 0 and 4: splitters --------------------------------------------------------------

__global__ __launch_bounds__(kBkSampleThreads) void k_bk_tab1(Work w) {
    __shared__ uint64_t s[kBkSample1];
    __shared__ int nvalid;
    const RoundState *st = w.st;
    const Tiles tl = tiles_of(w, 0);
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel)];
    if (threadIdx.x == 0) nvalid = 0;
    __syncthreads();
    int mine = 0;
    for (int i = threadIdx.x; i < kBkSample1; i += kBkSampleThreads) {
        uint64_t k = ~0ull;   // above every key (keys have at most 62 bits)
        if (tl.ntiles > 0) {
            const int64_t t = ((int64_t)i * tl.ntiles) / kBkSample1;
            const int v = tl.valid(t);
            if (v > 0) {
                k = in[t * kSortTile + (int64_t)(mix_index((uint64_t)i) % (uint64_t)v)];
                ++mine;
            }
        }
        s[i] = k;
    }
    if (mine) atomicAdd(&nvalid, mine);
    __syncthreads();
    sort_network<int>(s, kBkSample1);
    if (threadIdx.x == 0) build_tab(&w.btab[0], s, nvalid);
}

// first-level bucket starts (from the scanned first-level counts) and the second level's
// tiles per bucket
__global__ __launch_bounds__(kSortThreads) void k_bk_segments(Work w) {
    __shared__ uint32_t lds[kSortThreads / kWave + 1];
    RoundState *st = w.st;
    const int64_t nt1 = (int64_t)st->b_tiles1;
    const int64_t K = (int64_t)st->s_keys;
    const int b = threadIdx.x;
    const int64_t start = nt1 > 0 ? (int64_t)w.counts[(int64_t)b * nt1] : 0;
    w.bseg[b] = (uint64_t)start;
    if (b == 0) w.bseg[kBkSegs] = (uint64_t)K;
    __syncthreads();
    const int64_t end = b + 1 < kBkSegs ? (nt1 > 0 ? (int64_t)w.counts[(int64_t)(b + 1) * nt1] : 0) : K;
    const uint32_t tiles = (uint32_t)ceil_div(end - start, kSortTile);
    uint32_t total;
    const uint32_t first = block_excl_scan<kSortThreads>(tiles, lds, &total);
    w.btile[b] = first;
    if (b == 0) {
        w.btile[kBkSegs] = total;
        st->b_tiles2 = (u64c)total;
    }
}

__global__ __launch_bounds__(kBkSampleThreads) void k_bk_tab2(Work w) {
    __shared__ uint64_t s[kBkSample2];
    __shared__ int nvalid;
    const RoundState *st = w.st;
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel) ^ 1];
    for (int b = blockIdx.x; b < kBkSegs; b += gridDim.x) {
        const int64_t lo = (int64_t)w.bseg[b], cnt = (int64_t)w.bseg[b + 1] - lo;
        if (cnt <= 0 || w.btab[0].eqb[b]) {   // empty, or every key equal: one bucket
            if (threadIdx.x == 0) build_tab(&w.btab[1 + b], s, 0);
            continue;
        }
        const int S = cnt < kBkSample2 ? (int)cnt : kBkSample2;
        for (int i = threadIdx.x; i < kBkSample2; i += kBkSampleThreads)
            s[i] = i < S ? in[lo + (cnt <= kBkSample2 ? (int64_t)i : ((int64_t)i * cnt) / kBkSample2)] : ~0ull;
        if (threadIdx.x == 0) nvalid = S;
        __syncthreads();
        sort_network<int>(s, S);
        if (threadIdx.x == 0) build_tab(&w.btab[1 + b], s, nvalid);
        __syncthreads();
    }
}

// ---- stages 1, 2, 5, 6: counts and scatter -------------------------------------------------

template <int kLevel>
__device__ inline BkTiles<kLevel> bk_tiles(const Work &w, uint64_t *seg_lds, uint32_t *tb_lds) {
    BkTiles<kLevel> g;
    g.seg = seg_lds;
    g.tb = tb_lds;
    if (kLevel == 1) {
        g.tl = tiles_of(w, 0);
        g.ntiles = g.tl.ntiles;
    } else {
        for (int i = threadIdx.x; i <= kBkSegs; i += blockDim.x) {
            seg_lds[i] = w.bseg[i];
            tb_lds[i] = w.btile[i];
        }
        __syncthreads();
        g.ntiles = tb_lds[kBkSegs];
    }
    return g;
}

template <int kLevel>
__global__ __launch_bounds__(kSortThreads) void k_bk_hist(Work w) {
    __shared__ BucketTab tab;
    __shared__ uint32_t hist[256];
    __shared__ uint64_t seg_lds[kBkSegs + 1];
    __shared__ uint32_t tb_lds[kBkSegs + 1];
    RoundState *st = w.st;
    const BkTiles<kLevel> g = bk_tiles<kLevel>(w, seg_lds, tb_lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->aux_n = (u64c)256 * (u64c)g.ntiles;
        if (kLevel == 1) st->b_tiles1 = (u64c)g.ntiles;
    }
    const uint64_t *in = w.keys[sort_src(st->round, st->e_sel) ^ (kLevel == 1 ? 0 : 1)];
    int loaded = -1;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < g.ntiles; tile += gridDim.x) {
        int64_t off, base, stride;
        int tv, ti;
        g.tile(tile, off, tv, ti, base, stride);
        if (ti != loaded) {   // uniform over the workgroup
            __syncthreads();
            load_tab(tab, &w.btab[ti]);
            loaded = ti;
        }
        hist[threadIdx.x] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < tv; i += kSortThreads) {
            const uint32_t d = bucket_of(tab, in[off + i]);
            // a wave whose keys all fall in one bucket (a run of a repeated key) adds once
            const uint64_t act = ballot(true);
            const int lead = __ffsll((long long)act) - 1;
            if (ballot(d == __shfl(d, lead, kWave)) == act) {
                if (lane_id() == lead) atomicAdd(&hist[d], (uint32_t)__popcll(act));
            } else {
                atomicAdd(&hist[d], 1u);
            }
        }
        __syncthreads();
        w.counts[base + (int64_t)threadIdx.x * stride] = hist[threadIdx.x];
        __syncthreads();
    }
}

// Each tile is ranked stably in LDS by bucket (wave ballots find the lanes of equal buckets,
// per-wave counters order the waves), staged in bucket order and written as one run per
// bucket at the offsets the scan of the counts gave.  Built for the radix scatter's default
// waves per SIMD, like it.
template <int kLevel>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(LC_SCATTER_WAVES)))
void k_bk_scatter(Work w) {
    constexpr int kWaves = kSortThreads / kWave;
    __shared__ BucketTab tab;
    __shared__ uint64_t seg_lds[kBkSegs + 1];
    __shared__ uint32_t tb_lds[kBkSegs + 1];
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint64_t skeys[kSortTile];
    __shared__ uint8_t sdig[kSortTile];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t lds[kWaves + 1];
    RoundState *st = w.st;
    const BkTiles<kLevel> g = bk_tiles<kLevel>(w, seg_lds, tb_lds);
    const int src = sort_src(st->round, st->e_sel) ^ (kLevel == 1 ? 0 : 1);
    const uint64_t *in = w.keys[src];
    uint64_t *out = w.keys[src ^ 1];
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    int loaded = -1;
    for (int64_t tile = xcd_rank(blockIdx.x, gridDim.x); tile < g.ntiles; tile += gridDim.x) {
        int64_t off, base, stride;
        int tv, ti;
        g.tile(tile, off, tv, ti, base, stride);
        if (ti != loaded) {
            __syncthreads();
            load_tab(tab, &w.btab[ti]);
            loaded = ti;
        }
        const uint32_t my_gofs = w.counts[base + (int64_t)threadIdx.x * stride];
        for (int i = threadIdx.x; i < kWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        uint64_t k[kSortItems];
        uint32_t d[kSortItems], rk[kSortItems];
        const int wbase = wave * (kSortItems * kWave);
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int it = wbase + j * kWave + lane;
            k[j] = it < tv ? in[off + it] : ~0ull;
            d[j] = it < tv ? bucket_of(tab, k[j]) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (wbase + j * kWave >= tv) break;   // uniform over the wave
            const bool valid = wbase + j * kWave + lane < tv;
            const uint64_t peers = match_bits<8>(d[j], ballot(valid));
            uint32_t cur = 0;
            if (valid) cur = wcnt[wave][d[j]];
            rk[j] = cur + (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && (int)(__ffsll((long long)peers) - 1) == lane) wcnt[wave][d[j]] = cur + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        {   // bucket threadIdx.x: prefix over the waves, start in the tile, global offset
            const int b = threadIdx.x;
            uint32_t run = 0;
#pragma unroll
            for (int v = 0; v < kWaves; ++v) {
                const uint32_t c = wcnt[v][b];
                wcnt[v][b] = run;
                run += c;
            }
            uint32_t total;
            dstart[b] = block_excl_scan<kSortThreads>(run, lds, &total);
            gofs[b] = my_gofs;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            if (wbase + j * kWave + lane < tv) {
                const uint32_t pos = dstart[d[j]] + wcnt[wave][d[j]] + rk[j];
                skeys[pos] = k[j];
                sdig[pos] = (uint8_t)d[j];
            }
        }
        __syncthreads();
        for (int pos = threadIdx.x; pos < tv; pos += kSortThreads) {
            const uint32_t b = sdig[pos];
            out[(int64_t)gofs[b] + (uint32_t)pos - dstart[b]] = skeys[pos];
        }
        __syncthreads();
    }
}

// ---- stage 7: every final bucket sorted ------------------------------------------------------

__global__ __launch_bounds__(kSortThreads) void k_bk_final(Work w) {
    __shared__ uint64_t a[kBkCap];
    __shared__ uint8_t eq2[256];
    RoundState *st = w.st;
    const int src = sort_src(st->round, st->e_sel);   // where the second level left the keys
    const int dst = sorted_sel(st->round, st->e_sel, st->nbits);
    uint64_t *in = w.keys[src];
    uint64_t *out = w.keys[dst];
    int loaded = -1;
    for (int64_t f = blockIdx.x; f < (int64_t)kBkSegs * 256; f += gridDim.x) {
        const int b = (int)(f >> 8), d = (int)(f & 255);
        const int64_t first = w.btile[b], nt = (int64_t)w.btile[b + 1] - first;
        if (nt == 0) continue;   // empty first-level bucket (uniform over the workgroup)
        const int64_t cb = (int64_t)kBkSegs * first;
        const int64_t start = w.counts[cb + d * nt];
        const int64_t end = d < 255 ? (int64_t)w.counts[cb + (d + 1) * nt] : (int64_t)w.bseg[b + 1];
        const int64_t n = end - start;
        if (n <= 0) continue;
        if (b != loaded) {
            __syncthreads();
            for (int i = threadIdx.x; i < 256; i += kSortThreads) eq2[i] = w.btab[1 + b].eqb[i];
            __syncthreads();
            loaded = b;
        }
        const bool one_value = w.btab[0].eqb[b] || eq2[d];
        if (one_value || n == 1) {   // nothing to order
            if (dst != src)
                for (int64_t i = threadIdx.x; i < n; i += kSortThreads) out[start + i] = in[start + i];
        } else if (n <= kBkCap) {
            for (int i = threadIdx.x; i < (int)n; i += kSortThreads) a[i] = in[start + i];
            __syncthreads();
            sort_network<int>(a, (int)n);
            for (int i = threadIdx.x; i < (int)n; i += kSortThreads) out[start + i] = a[i];
        } else {   // larger than LDS: the same network, in place, its chunk-local stages in LDS
            sort_large(in + start, n, a);
            if (dst != src)
                for (int64_t i = threadIdx.x; i < n; i += kSortThreads) out[start + i] = in[start + i];
        }
        __syncthreads();
    }
}

hipError_t launch_bucket(const Work &w, int stage, int grid, hipStream_t s) {
    switch (stage) {
        case 0:
            hipLaunchKernelGGL(k_bk_tab1, dim3(1), dim3(kBkSampleThreads), 0, s, w);
            break;
        case 1:
            hipLaunchKernelGGL(k_bk_hist<1>, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        case 2:
            hipLaunchKernelGGL(k_bk_scatter<1>, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        case 3:
            hipLaunchKernelGGL(k_bk_segments, dim3(1), dim3(kSortThreads), 0, s, w);
            break;
        case 4:
            hipLaunchKernelGGL(k_bk_tab2, dim3(grid), dim3(kBkSampleThreads), 0, s, w);
            break;
        case 5:
            hipLaunchKernelGGL(k_bk_hist<2>, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        case 6:
            hipLaunchKernelGGL(k_bk_scatter<2>, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        case 7:
            hipLaunchKernelGGL(k_bk_final, dim3(grid), dim3(kSortThreads), 0, s, w);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lc
