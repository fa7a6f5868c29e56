// Edge-record readers shared by the round kernels: each yields the records of a chunk as
// endpoint pairs, turning out-of-range and padding records into loops that every kernel
// skips.
#pragma once

#include "lc_internal.hpp"

#ifndef LC_NT_INTERNAL
#define LC_NT_INTERNAL 1
#endif

namespace lc {

// ---------------------------------------------------------------------------------------
// edge readers: each thread handles a chunk of kV consecutive records.  Records that are
// out of range or past the end come back as a loop (a == b), which every kernel skips.
// ---------------------------------------------------------------------------------------

template <int V>
struct ReadSoa32 {
    static constexpr int kV = V;
    static constexpr bool kSorted = false;
    const int32_t *s, *d;
    int64_t m;
    uint32_t n;
    __host__ explicit ReadSoa32(const EdgeIn &e)
        : s((const int32_t *)e.s), d((const int32_t *)e.d), m(e.m), n(e.n) {}
    __device__ void init(const RoundState *) {}
    __device__ int64_t records() const { return m; }
    __device__ int64_t chunks() const { return (m + V - 1) / V; }
    __device__ void read(int64_t c, uint32_t *a, uint32_t *b, bool &bad) const {
        const int64_t base = c * V;
        int32_t sa[V], sb[V];
        if (V == 4 && base + 4 <= m) {
            int4 x = *(const int4 *)(s + base);
            int4 y = *(const int4 *)(d + base);
            sa[0] = x.x; sa[1 % V] = x.y; sa[2 % V] = x.z; sa[3 % V] = x.w;
            sb[0] = y.x; sb[1 % V] = y.y; sb[2 % V] = y.z; sb[3 % V] = y.w;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                sa[j] = base + j < m ? s[base + j] : 0;
                sb[j] = base + j < m ? d[base + j] : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            bool ok = (uint32_t)sa[j] < n && (uint32_t)sb[j] < n;
            bad |= (base + j < m) && !ok;
            a[j] = ok ? (uint32_t)sa[j] : 0u;
            b[j] = ok ? (uint32_t)sb[j] : 0u;
        }
    }
};

template <int V>
struct ReadSoa64 {
    static constexpr int kV = V;
    static constexpr bool kSorted = false;
    const int64_t *s, *d;
    int64_t m;
    uint32_t n;
    __host__ explicit ReadSoa64(const EdgeIn &e)
        : s((const int64_t *)e.s), d((const int64_t *)e.d), m(e.m), n(e.n) {}
    __device__ void init(const RoundState *) {}
    __device__ int64_t records() const { return m; }
    __device__ int64_t chunks() const { return (m + V - 1) / V; }
    __device__ void read(int64_t c, uint32_t *a, uint32_t *b, bool &bad) const {
        const int64_t base = c * V;
        int64_t sa[V], sb[V];
        if (V == 2 && base + 2 <= m) {
            longlong2 x = *(const longlong2 *)(s + base);
            longlong2 y = *(const longlong2 *)(d + base);
            sa[0] = x.x; sa[1 % V] = x.y;
            sb[0] = y.x; sb[1 % V] = y.y;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                sa[j] = base + j < m ? s[base + j] : 0;
                sb[j] = base + j < m ? d[base + j] : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            bool ok = (uint64_t)sa[j] < (uint64_t)n && (uint64_t)sb[j] < (uint64_t)n;
            bad |= (base + j < m) && !ok;
            a[j] = ok ? (uint32_t)sa[j] : 0u;
            b[j] = ok ? (uint32_t)sb[j] : 0u;
        }
    }
};

template <int V>
struct ReadPacked {
    static constexpr int kV = V;
    static constexpr bool kSorted = false;
    const uint64_t *k;
    int64_t m;
    uint32_t n;
    __host__ explicit ReadPacked(const EdgeIn &e) : k((const uint64_t *)e.s), m(e.m), n(e.n) {}
    __device__ void init(const RoundState *) {}
    __device__ int64_t records() const { return m; }
    __device__ int64_t chunks() const { return (m + V - 1) / V; }
    __device__ void read(int64_t c, uint32_t *a, uint32_t *b, bool &bad) const {
        const int64_t base = c * V;
        uint64_t r[V];
        if (V == 2 && base + 2 <= m) {
            ulonglong2 x = *(const ulonglong2 *)(k + base);
            r[0] = x.x; r[1 % V] = x.y;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) r[j] = base + j < m ? k[base + j] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            uint32_t x = (uint32_t)(r[j] >> 32), y = (uint32_t)r[j];
            bool ok = x < n && y < n;
            bad |= (base + j < m) && !ok;
            a[j] = ok ? x : 0u;
            b[j] = ok ? y : 0u;
        }
    }
};

// Edges of rounds >= 1: (a << 32 | b) in the round's compact index space, in the key
// buffer named by the device state; the count comes from the device state too.
#ifndef LC_INTERNAL_V
#define LC_INTERNAL_V 2
#endif
struct ReadInternal {
    static constexpr int kV = LC_INTERNAL_V;   // records per chunk (2 or 4)
    static constexpr bool kSorted = true;   // records ordered by (block of b, a, b): lanes share a
    uint64_t *k0, *k1;
    const uint64_t *k;
    int64_t m;
    __host__ explicit ReadInternal(const Work &w) : k0(w.keys[0]), k1(w.keys[1]), k(nullptr), m(0) {}
    __device__ void init(const RoundState *st) {
        k = st->e_sel ? k1 : k0;
        m = (int64_t)st->m_cur;
    }
    __device__ int64_t records() const { return m; }
    __device__ int64_t chunks() const { return (m + kV - 1) / kV; }
    __device__ void read(int64_t c, uint32_t *a, uint32_t *b, bool &) const {
        typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
        const int64_t base = c * kV;
        uint64_t r[kV];
        if (base + kV <= m) {
            // records stream through once: load them non-temporally, so that the node state
            // the same pass gathers keeps its place in L2
#pragma unroll
            for (int h = 0; h < kV; h += 2) {
                const u64x2 x = LC_NT_INTERNAL ? __builtin_nontemporal_load((const u64x2 *)(k + base + h))
                                               : *(const u64x2 *)(k + base + h);
                r[h] = x.x;
                r[h + 1] = x.y;
            }
        } else {
#pragma unroll
            for (int h = 0; h < kV; ++h) r[h] = base + h < m ? k[base + h] : 0ull;
        }
#pragma unroll
        for (int h = 0; h < kV; ++h) {
            a[h] = (uint32_t)(r[h] >> 32);
            b[h] = (uint32_t)r[h];
        }
    }
};

}  // namespace lc
