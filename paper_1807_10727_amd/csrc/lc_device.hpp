// Device-side building blocks for gfx950 (CDNA4, 64-lane wavefronts):
// the keyed priority bijection and its inverse, wave ballot/shuffle helpers and a
// 256-thread block scan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

constexpr int kWave = 64;
constexpr uint32_t kInf = 0xFFFFFFFFu;      // "no priority seen yet"
constexpr uint32_t kFinal = 0x80000000u;    // map entry flag: final node, low 31 bits = its name

// ---------------------------------------------------------------------------------------
// Priority: a keyed bijection on 32-bit node names.  rho_r(x) = F(F(x ^ k0) ^ k1) with
// F = MurmurHash3's 32-bit finaliser and (k1:k0) = sm64(seed ^ sm64(r)), sm64 being
// SplitMix64's output function.  The inverse undoes every step, so the parent's name is
// recovered from the winning priority without storing (priority, name) pairs.
// ---------------------------------------------------------------------------------------

__host__ __device__ constexpr uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// multiplicative inverse of an odd constant modulo 2^32 (Newton iteration)
constexpr uint32_t inv_odd(uint32_t a) {
    uint32_t x = a;
    for (int i = 0; i < 5; ++i) x = x * (2u - a * x);
    return x;
}

constexpr uint32_t kMulA = 0x85EBCA6Bu;
constexpr uint32_t kMulB = 0xC2B2AE35u;
constexpr uint32_t kInvA = inv_odd(kMulA);
constexpr uint32_t kInvB = inv_odd(kMulB);
static_assert(kMulA * kInvA == 1u && kMulB * kInvB == 1u, "odd-constant inverses");

struct RoundKey {
    uint32_t k0, k1;
};

__host__ __device__ inline RoundKey round_key(uint64_t seed, int32_t r) {
    uint64_t k = sm64(seed ^ sm64((uint64_t)(uint32_t)r));
    return RoundKey{(uint32_t)k, (uint32_t)(k >> 32)};
}

__host__ __device__ inline uint32_t fmix(uint32_t h) {
    h ^= h >> 16;
    h *= kMulA;
    h ^= h >> 13;
    h *= kMulB;
    h ^= h >> 16;
    return h;
}

__host__ __device__ inline uint32_t fmix_inv(uint32_t h) {
    h ^= h >> 16;                 // a shift by >= 16 is its own inverse
    h *= kInvB;
    h ^= (h >> 13) ^ (h >> 26);   // inverse of h ^= h >> 13
    h *= kInvA;
    h ^= h >> 16;
    return h;
}

__host__ __device__ inline uint32_t prio(RoundKey k, uint32_t name) { return fmix(fmix(name ^ k.k0) ^ k.k1); }

__host__ __device__ inline uint32_t prio_inv(RoundKey k, uint32_t p) { return fmix_inv(fmix_inv(p) ^ k.k1) ^ k.k0; }

// ---------------------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------------------

__device__ inline int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// lanes of the wave whose `bits`-bit value equals this lane's (8 ballots for a digit)
template <int kBits>
__device__ inline uint64_t match_bits(uint32_t v, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
        uint64_t m = __ballot((v >> b) & 1u);
        peers &= ((v >> b) & 1u) ? m : ~m;
    }
    return peers;
}

template <typename T>
__device__ inline T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ inline T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Sum over a block of kThreads (multiple of 64), valid in thread 0.  `lds` holds
// kThreads/64 entries.  Every thread of the block must call it.
template <int kThreads, typename T>
__device__ inline T block_sum(T x, T *lds) {
    constexpr int kWaves = kThreads / kWave;
    x = wave_sum(x);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = x;
    __syncthreads();
    T r = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kWaves; ++i) r += lds[i];
    }
    __syncthreads();
    return r;
}

// Exclusive scan over a block of kThreads (multiple of 64).  Returns this thread's
// exclusive prefix; *total receives the block sum.  `lds` holds kThreads/64 + 1 entries.
template <int kThreads, typename T>
__device__ inline T block_excl_scan(T x, T *lds, T *total) {
    constexpr int kWaves = kThreads / kWave;
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    T inc = wave_incl_scan(x);
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < kWaves; ++i) {
            T t = lds[i];
            lds[i] = run;
            run += t;
        }
        lds[kWaves] = run;
    }
    __syncthreads();
    T res = lds[w] + inc - x;
    *total = lds[kWaves];
    __syncthreads();
    return res;
}

// Workgroup b of a launch runs on XCD b % 8 (MI355X: 8 XCDs, each with its own L2).  Tile
// loops number their workgroups so that consecutive logical ids share an XCD: neighbouring
// tiles then read and write the same lines of per-tile tables (digit counts, offsets) from
// one L2 instead of eight.
constexpr int kXcds = 8;

// Words that workgroups running at the same time hand to each other (the one-sweep radix
// passes' look-back): atomic at device scope, so that a store on one XCD is seen by a load
// on another without waiting for the kernel to end.
__device__ inline uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int64_t xcd_rank(int64_t b, int64_t g) {
    return g % kXcds ? b : (b % kXcds) * (g / kXcds) + b / kXcds;
}

// Lanes of a wave reading sorted records hold runs of equal first endpoints.  Combine the
// values of lanes with equal keys (a min over same-key lanes is a valid update for that key)
// so that only the last lane of each run touches memory.
__device__ inline uint32_t run_min(uint32_t key, uint32_t val, bool &last) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t ov = __shfl_up(val, d, kWave);
        const uint32_t ok = __shfl_up(key, d, kWave);
        if (lane >= d && ok == key) val = min(val, ov);
    }
    const uint32_t nk = __shfl_down(key, 1, kWave);
    last = lane == kWave - 1 || nk != key;
    return val;
}

}  // namespace lc
