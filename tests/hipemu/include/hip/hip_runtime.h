// Host emulation of the subset of HIP that the library's sources use -- TEST INFRASTRUCTURE.
//
// The kernels of paper_1807_10727_amd/csrc are compiled unchanged as host C++ against this
// header, so their logic (indexing, bounds, barriers, wave ballots and shuffles, LDS, atomics,
// the host engine around them) can be checked against the oracle without a GPU.  It models
// the CDNA execution model, not its timing: every work-item is a fiber; a workgroup's fibers
// run on the calling thread until each one reaches a barrier, a wave operation or its end;
// a wave operation completes for the lanes of a wave that reach the same call site together
// once no lane of that wave can run (the lanes elsewhere are inactive for it, as under an
// execution mask); __syncthreads releases a workgroup once every live work-item waits at it.
// Workgroups of a launch run one after another; streams execute each call at once, in order;
// a captured graph records calls and replays them.  Device memory is host memory.
//
// Nothing in the product loads this: it is built only by tests/hipemu (see hipemu/__init__.py).
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <functional>
#include <tuple>
#include <type_traits>
#include <utility>

// ---- qualifiers ---------------------------------------------------------------------------
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ thread_local
#define __align__(n) __attribute__((aligned(n)))
#define __launch_bounds__(...)
#define __restrict__ __restrict
// a scheduling hint of the GPU compiler; on the host it becomes an attribute that is allowed
#define amdgpu_waves_per_eu(...) unused

struct dim3 {
    uint32_t x, y, z;
    constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

struct uint2 {
    uint32_t x, y;
} __attribute__((aligned(8)));
struct uint4 {
    uint32_t x, y, z, w;
} __attribute__((aligned(16)));
struct ulonglong2 {
    unsigned long long x, y;
} __attribute__((aligned(16)));
struct int4 {
    int32_t x, y, z, w;
} __attribute__((aligned(16)));
struct longlong2 {
    long long x, y;
} __attribute__((aligned(16)));
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return uint4{x, y, z, w}; }

// ---- execution model ----------------------------------------------------------------------
namespace hipemu {

constexpr int kWave = 64;

enum OpKind { kBallot, kShfl, kShflUp, kShflDown, kShflXor, kWaveBarrier };

struct Item {
    dim3 tid;
    int state;            // 0 runnable, 1 at a wave op, 2 at __syncthreads, 3 done
    const char *site;     // call site of the pending wave op (file, line: pointer identity)
    int line;
    int op;
    uint64_t val;         // operand of the pending wave op
    int arg, width;
    uint64_t result;
};

Item *current();
extern thread_local dim3 t_block_idx, t_block_dim, t_grid_dim;
uint64_t wave_op(int op, uint64_t val, int arg, int width, const char *file, int line);
void sync_threads();
void run_grid(const std::function<void()> &item, dim3 grid, dim3 block);
// A cooperative launch: every workgroup runs at once, each on a host thread of its own, so
// that grid-wide barriers (cooperative_groups, hip_cooperative_groups.h) can complete.
void run_grid_cooperative(const std::function<void()> &item, dim3 grid, dim3 block);
void grid_sync();
void count_launch();   // kernels executed so far (hipemu_launches), graph replays included

}  // namespace hipemu

#define threadIdx (::hipemu::current()->tid)
#define blockIdx (::hipemu::t_block_idx)
#define blockDim (::hipemu::t_block_dim)
#define gridDim (::hipemu::t_grid_dim)

inline void __syncthreads() { hipemu::sync_threads(); }

inline uint32_t hipemu_lane() { return threadIdx.x % hipemu::kWave; }

inline uint32_t hipemu_mbcnt_lo(uint32_t mask, uint32_t x) {
    const uint32_t lane = hipemu_lane();
    const uint32_t below = lane >= 32 ? 0xFFFFFFFFu : ((1u << lane) - 1u);
    return x + (uint32_t)__builtin_popcount(mask & below);
}
inline uint32_t hipemu_mbcnt_hi(uint32_t mask, uint32_t x) {
    const uint32_t lane = hipemu_lane();
    const uint32_t below = lane < 32 ? 0u : ((1u << (lane - 32)) - 1u);
    return x + (uint32_t)__builtin_popcount(mask & below);
}
#define __builtin_amdgcn_mbcnt_lo(m, x) hipemu_mbcnt_lo((m), (x))
#define __builtin_amdgcn_mbcnt_hi(m, x) hipemu_mbcnt_hi((m), (x))
#define __builtin_amdgcn_wave_barrier() \
    ((void)::hipemu::wave_op(::hipemu::kWaveBarrier, 0, 0, 64, __builtin_FILE(), __builtin_LINE()))

inline unsigned long long __ballot(int pred, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu::wave_op(hipemu::kBallot, pred != 0, 0, 64, f, l);
}
inline int __any(int pred, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu::wave_op(hipemu::kBallot, pred != 0, 0, 64, f, l) != 0;
}
inline int __all(int pred, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    // a lane that is not in the group reads as true
    return hipemu::wave_op(hipemu::kBallot, pred == 0, 0, 64, f, l) == 0;
}

template <typename T>
inline uint64_t hipemu_bits(T v) {
    static_assert(sizeof(T) <= 8, "shuffles of at most 8 bytes");
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    return u;
}
template <typename T>
inline T hipemu_from(uint64_t u) {
    T v;
    memcpy(&v, &u, sizeof(T));
    return v;
}
template <typename T>
inline T __shfl(T v, int src, int width = 64, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu_from<T>(hipemu::wave_op(hipemu::kShfl, hipemu_bits(v), src, width, f, l));
}
template <typename T>
inline T __shfl_up(T v, unsigned d, int width = 64, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu_from<T>(hipemu::wave_op(hipemu::kShflUp, hipemu_bits(v), (int)d, width, f, l));
}
template <typename T>
inline T __shfl_down(T v, unsigned d, int width = 64, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu_from<T>(hipemu::wave_op(hipemu::kShflDown, hipemu_bits(v), (int)d, width, f, l));
}
template <typename T>
inline T __shfl_xor(T v, int m, int width = 64, const char *f = __builtin_FILE(), int l = __builtin_LINE()) {
    return hipemu_from<T>(hipemu::wave_op(hipemu::kShflXor, hipemu_bits(v), m, width, f, l));
}

// the device min / max of two integers, in their common type
template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) {
    typedef typename std::common_type<A, B>::type T;
    return (T)a < (T)b ? (T)a : (T)b;
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) {
    typedef typename std::common_type<A, B>::type T;
    return (T)a < (T)b ? (T)b : (T)a;
}
inline unsigned long long __umul64hi(unsigned long long a, unsigned long long b) {
    return (unsigned long long)(((unsigned __int128)a * b) >> 64);
}

inline int __popc(uint32_t x) { return __builtin_popcount(x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __clzll(long long x) { return x == 0 ? 64 : __builtin_clzll((unsigned long long)x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }

// atomics: plain host atomics on the address (global memory and LDS alike)
template <typename T>
inline T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
template <typename T>
inline T atomicOr(T *p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
template <typename T>
inline T atomicMin(T *p, T v) {
    T old = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
    return old;
}
template <typename T>
inline T atomicMax(T *p, T v) {
    T old = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v > old && !__atomic_compare_exchange_n(p, &old, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
    return old;
}
template <typename T>
inline T atomicCAS(T *p, T cmp, T v) {
    __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
    return cmp;
}
template <typename T>
inline T atomicExch(T *p, T v) { return __atomic_exchange_n(p, v, __ATOMIC_RELAXED); }

// scoped atomics of HIP's clang: host atomics (every scope is the process here)
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), (order))
namespace hipemu {
void pause();   // a polling work-item lets the host thread breathe
}  // namespace hipemu
#define __builtin_amdgcn_s_sleep(n) ::hipemu::pause()

// ---- runtime ------------------------------------------------------------------------------
typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
    hipErrorCooperativeLaunchTooLarge = 720,
    hipErrorUnknown = 999
} hipError_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

typedef enum hipDeviceAttribute_t {
    hipDeviceAttributeMultiprocessorCount = 1,
    hipDeviceAttributeMaxSharedMemoryPerBlock = 2
} hipDeviceAttribute_t;

typedef enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 } hipFuncAttribute;

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph_t;
struct ihipGraphExec_t;
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
typedef ihipGraph_t *hipGraph_t;
typedef ihipGraphExec_t *hipGraphExec_t;
typedef void *hipGraphNode_t;

#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u

namespace hipemu {
// Runs `call` now, or appends it to the graph being captured on `s`.
void submit(hipStream_t s, std::function<void()> call);
void set_error(hipError_t e);
}  // namespace hipemu

hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *d);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipFuncSetAttribute(const void *f, hipFuncAttribute a, int v);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k);
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s = nullptr);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamCreate(hipStream_t *s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *err_node, char *log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags = 0);
hipError_t hipHostFree(void *p);
hipError_t hipMalloc(void **p, size_t n);
hipError_t hipFree(void *p);

// hipLaunchKernelGGL(kernel, grid, block, dynamic LDS bytes, stream, args...): the kernel
// and copies of its arguments are bound when the call is made (as a launch copies them).
template <typename F, typename... A>
inline void hipemu_launch(F kern, dim3 grid, dim3 block, size_t shmem, hipStream_t s, A... args) {
    (void)shmem;
    if (grid.x == 0 || block.x == 0 || block.x > 1024) {
        hipemu::set_error(hipErrorInvalidValue);
        return;
    }
    hipemu::submit(s, [=]() {
        hipemu::count_launch();
        hipemu::run_grid([=]() { kern(args...); }, grid, block);
    });
}
#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
    hipemu_launch((kern), dim3(grid), dim3(block), (size_t)(shmem), (stream), ##__VA_ARGS__)

// Workgroups of a kernel resident on one compute unit at once: the emulated device (4 compute
// units) takes resident_per_cu() of any kernel, 4 unless HIPEMU_RESIDENT_PER_CU says otherwise
// (0 models a kernel too large to keep even one workgroup resident), so a cooperative grid
// larger than 4 times that fails as on the GPU.
namespace hipemu {
constexpr int kCus = 4;
int resident_per_cu();
}  // namespace hipemu
template <typename F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, F, int block, size_t shmem) {
    if (block <= 0 || block > 1024 || shmem > 160 * 1024) return hipErrorInvalidValue;
    *n = hipemu::resident_per_cu();
    return hipSuccess;
}
template <typename... A, size_t... I>
inline std::tuple<typename std::decay<A>::type...> hipemu_unpack(void **args, std::index_sequence<I...>) {
    return std::tuple<typename std::decay<A>::type...>(*(typename std::decay<A>::type *)args[I]...);
}
// hipLaunchCooperativeKernel(kernel, grid, block, argument pointers, dynamic LDS, stream): the
// arguments are copied when the call is made, as a launch copies them.
template <typename... A>
inline hipError_t hipLaunchCooperativeKernel(void (*kern)(A...), dim3 grid, dim3 block, void **args, unsigned shmem,
                                             hipStream_t s) {
    (void)shmem;
    if (grid.x == 0 || block.x == 0 || block.x > 1024) return hipErrorInvalidValue;
    if ((size_t)grid.x * grid.y * grid.z > (size_t)hipemu::kCus * hipemu::resident_per_cu())
        return hipErrorCooperativeLaunchTooLarge;
    auto vals = hipemu_unpack<A...>(args, std::index_sequence_for<A...>{});
    hipemu::submit(s, [=]() {
        hipemu::count_launch();
        hipemu::run_grid_cooperative([=]() { std::apply(kern, vals); }, grid, block);
    });
    return hipSuccess;
}
