// LDS-resident LocalContraction of one small graph per workgroup (batched mode).
//
// A persistent kernel: every workgroup pulls graph ids from an atomic queue and runs all
// rounds of that graph inside its LDS, reading the graph's records from HBM once and
// writing its labels once.  The arithmetic is the specification of the union path
// (priority of node name x in round r from the graph's own seed, nodes named by their
// parent's original id, labels composed round by round), so each graph's labels are
// identical to its solo solve.
//
// LDS layout for kNMax nodes and kMMax records (kMMax a power of two):
//   E[kMMax]       records (a << 16 | b) in the round's compact node space; ~0u = none
//   ml[kNMax]      node word: low half one-hop minimum, high half two-hop minimum;
//                  reused as byte flags during duplicate marking
//   names[2][kNMax], par, newidx, idx_of, L (per original vertex), has, lab
// Duplicates are not compacted: after the bitonic sort, repeats of a key become ~0u and
// the sort of the next round moves them behind the live records.
#pragma once

#include "lc_internal.hpp"

namespace lc {

// One graph for the LDS solver: records src[i], dst[i] (int32 local ids, i < m), n vertices.
struct SmallDesc {
    const int32_t *src;
    const int32_t *dst;
    int64_t m;
    int32_t n;
    int32_t status;          // written: 0 ok, 1 an id out of range
    uint64_t seed;
    int32_t *labels;         // [n] local labels (written)
    int32_t *rounds;         // rounds of the graph (written; may be null)
};

struct SmallArgs {
    SmallDesc *desc;         // [count]
    int32_t count;
    uint32_t *queue;         // next descriptor (zeroed before the launch)
    uint32_t *err;           // bit 0 set when any graph had an id out of range
};

constexpr uint16_t kSmallFinal = 0x8000u;

// Variants of the solver (index 1..3): at most nmax vertices and mmax records per graph.
struct SmallVariant {
    int nmax, mmax;
};
constexpr SmallVariant kSmallVariants[] = {{0, 0}, {512, 4096}, {1024, 8192}, {2048, 16384}};
constexpr int kNumSmallVariants = 4;

size_t small_bytes(int variant, int threads);                 // LDS bytes of a variant
hipError_t prepare_small(int variant, int threads);           // allow its LDS size (outside captures)
hipError_t launch_small(int variant, int threads, const SmallArgs &a, int grid, hipStream_t s);

template <int kNT, int kNMax, int kMMax>
struct SmallLds {
    static constexpr size_t kE = sizeof(uint32_t) * kMMax;
    static constexpr size_t kMl = sizeof(uint64_t) * kNMax;
    static constexpr size_t kHalf = sizeof(uint16_t) * kNMax;
    static constexpr size_t kBytes = kE + kMl + 6 * kHalf + 2 * kNMax + 64;
    static_assert(kMMax <= 8 * kNMax, "duplicate flags reuse the node words");
    static_assert(kNMax <= 0x7FFF, "16-bit node indices with a final flag");
};

template <int kNT>
__device__ inline uint32_t small_block_scan(uint32_t x, uint32_t *lds, uint32_t *total) {
    return block_excl_scan<kNT>(x, lds, total);
}

template <int kNT, int kNMax, int kMMax>
__global__ __launch_bounds__(kNT) void k_small(SmallArgs a) {
    using L = SmallLds<kNT, kNMax, kMMax>;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *E = (uint32_t *)smem;
    uint64_t *ml = (uint64_t *)(smem + L::kE);
    uint16_t *names0 = (uint16_t *)(smem + L::kE + L::kMl);
    uint16_t *names1 = names0 + kNMax;
    uint16_t *par = names1 + kNMax;
    uint16_t *newidx = par + kNMax;
    uint16_t *idx_of = newidx + kNMax;
    uint16_t *lab = idx_of + kNMax;             // per original vertex: node index or kSmallFinal | name
    uint8_t *has = (uint8_t *)(lab + kNMax);
    uint8_t *islab = has + kNMax;
    __shared__ uint32_t scan_lds[kNT / kWave + 1];
    __shared__ uint32_t sh_slot, sh_cnt, sh_bad;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) sh_slot = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t slot = sh_slot;
        __syncthreads();
        if (slot >= (uint32_t)a.count) break;
        SmallDesc *dsc = a.desc + slot;
        const int n = dsc->n;
        const int m = (int)dsc->m;
        const uint64_t seed = dsc->seed;
        const int32_t *gsrc = dsc->src;
        const int32_t *gdst = dsc->dst;

        // load: loop-free records as (min << 16 | max); everything else ~0u
        if (tid == 0) sh_bad = 0;
        for (int i = tid; i < kMMax; i += kNT) {
            uint32_t v = ~0u;
            if (i < m) {
                const int32_t x = gsrc[i], y = gdst[i];
                if ((uint32_t)x < (uint32_t)n && (uint32_t)y < (uint32_t)n) {
                    if (x != y) v = ((uint32_t)min(x, y) << 16) | (uint32_t)max(x, y);
                } else {
                    sh_bad = 1;
                }
            }
            E[i] = v;
        }
        for (int v = tid; v < n; v += kNT) {
            names0[v] = (uint16_t)v;
            lab[v] = (uint16_t)v;
        }
        __syncthreads();
        if (tid == 0) {
            dsc->status = sh_bad ? 1 : 0;
            if (sh_bad) atomicOr(a.err, 1u);
        }

        int N = n;          // nodes of this round (round 0: every id)
        int M = m;          // record slots of this round
        int r = 0;
        uint16_t *names = names0, *names_next = names1;
        for (;;) {
            // live records?
            if (tid == 0) sh_cnt = 0;
            __syncthreads();
            uint32_t live = 0;
            for (int i = tid; i < M; i += kNT) live += E[i] != ~0u;
            live = wave_sum(live);
            if (lane_id() == 0 && live) atomicAdd(&sh_cnt, live);
            __syncthreads();
            if (sh_cnt == 0) break;

            const RoundKey key = round_key(seed, r);
            for (int i = tid; i < N; i += kNT) {
                ml[i] = ~0ull;
                has[i] = 0;
                islab[i] = 0;
            }
            __syncthreads();
            uint32_t *w32 = (uint32_t *)ml;
            for (int i = tid; i < M; i += kNT) {
                const uint32_t e = E[i];
                if (e == ~0u) continue;
                const uint32_t x = e >> 16, y = e & 0xFFFFu;
                const uint32_t v = min(prio(key, names[x]), prio(key, names[y]));
                atomicMin(&w32[2 * x], v);
                atomicMin(&w32[2 * y], v);
            }
            __syncthreads();
            for (int i = tid; i < M; i += kNT) {
                const uint32_t e = E[i];
                if (e == ~0u) continue;
                const uint32_t x = e >> 16, y = e & 0xFFFFu;
                const uint32_t v = min(w32[2 * x], w32[2 * y]);
                atomicMin(&w32[2 * x + 1], v);
                atomicMin(&w32[2 * y + 1], v);
            }
            __syncthreads();
            for (int i = tid; i < N; i += kNT) {
                const uint32_t l = w32[2 * i + 1];
                uint16_t p = (uint16_t)i;
                if (l != kInf) {
                    const uint32_t nm = prio_inv(key, l);
                    p = r == 0 ? (uint16_t)nm : idx_of[nm < (uint32_t)n ? nm : 0];
                    if (p >= N) p = (uint16_t)i;   // cannot happen for a consistent state
                    islab[p] = 1;
                }
                par[i] = p;
            }
            __syncthreads();
            // relabel in place; loops become ~0u
            for (int i = tid; i < M; i += kNT) {
                const uint32_t e = E[i];
                if (e == ~0u) continue;
                const uint32_t px = par[e >> 16], py = par[e & 0xFFFFu];
                E[i] = px == py ? ~0u : ((min(px, py) << 16) | max(px, py));
            }
            // bitonic sort of the next power of two >= M (padding ~0u sorts last)
            int P2 = 1;
            while (P2 < M) P2 <<= 1;
            for (int i = M + tid; i < P2; i += kNT) E[i] = ~0u;
            __syncthreads();
            for (int k = 2; k <= P2; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = tid; i < P2; i += kNT) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const uint32_t u = E[i], v = E[ixj];
                            if (((i & k) == 0) ? (u > v) : (u < v)) {
                                E[i] = v;
                                E[ixj] = u;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            // live records now lead; mark repeats (flags in the free node words)
            uint8_t *dup = (uint8_t *)ml;
            int S = 0;
            {
                uint32_t c = 0;
                for (int i = tid; i < M; i += kNT) c += E[i] != ~0u;
                c = wave_sum(c);
                if (tid == 0) sh_cnt = 0;
                __syncthreads();
                if (lane_id() == 0 && c) atomicAdd(&sh_cnt, c);
                __syncthreads();
                S = (int)sh_cnt;
            }
            for (int i = tid; i < S; i += kNT) dup[i] = (i > 0 && E[i] == E[i - 1]) ? 1 : 0;
            __syncthreads();
            for (int i = tid; i < S; i += kNT) {
                if (dup[i]) {
                    E[i] = ~0u;
                } else {
                    has[E[i] >> 16] = 1;
                    has[E[i] & 0xFFFFu] = 1;
                }
            }
            __syncthreads();
            // next node indices: exclusive scan of has over the N nodes (contiguous chunks)
            {
                constexpr int kPer = (kNMax + kNT - 1) / kNT;
                const int lo = tid * kPer;
                uint32_t c = 0;
                for (int q = 0; q < kPer; ++q)
                    if (lo + q < N) c += has[lo + q];
                uint32_t total;
                uint32_t run = small_block_scan<kNT>(c, scan_lds, &total);
                for (int q = 0; q < kPer; ++q) {
                    const int j = lo + q;
                    if (j < N) {
                        newidx[j] = (uint16_t)run;
                        run += has[j];
                    }
                }
                __syncthreads();
            }
            for (int j = tid; j < N; j += kNT) {
                if (has[j]) {
                    const uint16_t k = newidx[j];
                    names_next[k] = names[j];
                    idx_of[names[j]] = k;
                }
            }
            // compose the labels of the original vertices through this round
            for (int v = tid; v < n; v += kNT) {
                const uint16_t x = lab[v];
                if (!(x & kSmallFinal)) {
                    const uint16_t p = par[x];
                    lab[v] = has[p] ? newidx[p] : (uint16_t)(kSmallFinal | names[p]);
                }
            }
            __syncthreads();
            // records into the next node space (order preserved: newidx is monotone)
            for (int i = tid; i < S; i += kNT) {
                const uint32_t e = E[i];
                if (e != ~0u) E[i] = ((uint32_t)newidx[e >> 16] << 16) | newidx[e & 0xFFFFu];
            }
            uint32_t nn = 0;
            for (int j = tid; j < N; j += kNT) nn += has[j];
            nn = wave_sum(nn);
            if (tid == 0) sh_cnt = 0;
            __syncthreads();
            if (lane_id() == 0 && nn) atomicAdd(&sh_cnt, nn);
            __syncthreads();
            N = (int)sh_cnt;
            M = S;
            uint16_t *t = names;
            names = names_next;
            names_next = t;
            ++r;
            __syncthreads();
        }
        int32_t *out = dsc->labels;
        for (int v = tid; v < n; v += kNT) {
            const uint16_t x = lab[v];
            out[v] = (x & kSmallFinal) ? (int32_t)(x & 0x7FFF) : (int32_t)names[x];
        }
        if (tid == 0 && dsc->rounds) *dsc->rounds = r;
        __syncthreads();
    }
}

}  // namespace lc
