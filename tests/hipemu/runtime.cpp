// Host emulation of HIP (see include/hip/hip_runtime.h) -- TEST INFRASTRUCTURE.
//
// Work-items are fibers on the calling thread (x86-64 context switch below).  The scheduler
// runs every runnable fiber until it blocks; when none can run it completes one pending wave
// operation per wave (for the lanes of that wave waiting at the same call site), or, when
// every live work-item waits at __syncthreads, releases the barrier.  Anything else is a
// deadlock and aborts the process with a message that names the kernel's state.
#include <atomic>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

extern "C" void hipemu_switch(void **save_sp, void *new_sp);

// save the callee-saved registers and the stack pointer in *save_sp, switch to new_sp
asm(R"(
    .text
    .globl hipemu_switch
    .type hipemu_switch, @function
hipemu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size hipemu_switch, .-hipemu_switch
)");

namespace lc {
// dynamic LDS of the kernels that declare `extern __shared__ ... smem[]` (in namespace lc)
thread_local __attribute__((aligned(16))) unsigned char smem[160 * 1024];
}

namespace hipemu {

thread_local dim3 t_block_idx, t_block_dim, t_grid_dim;

namespace {

constexpr size_t kStack = 256 * 1024;

struct Fiber {
    Item item;
    void *sp = nullptr;
    char *stack = nullptr;
};

struct Group {   // one workgroup in flight on this thread
    std::vector<Fiber> fibers;
    const std::function<void()> *body = nullptr;
    void *sched_sp = nullptr;
    int cur = -1;
};

thread_local Group *g_group = nullptr;
thread_local std::vector<char *> g_stacks;   // reused across workgroups
thread_local hipError_t g_last_error = hipSuccess;

[[noreturn]] void die(const char *msg) {
    fprintf(stderr, "hipemu: %s\n", msg);
    fflush(stderr);
    abort();
}

void trampoline() {
    Group *g = g_group;
    Fiber &f = g->fibers[(size_t)g->cur];
    (*g->body)();
    f.item.state = 3;
    hipemu_switch(&f.sp, g->sched_sp);
    die("a finished work-item was resumed");
}

void init_fiber(Fiber &f, char *stack) {
    f.stack = stack;
    uintptr_t top = ((uintptr_t)(stack + kStack)) & ~(uintptr_t)15;
    void **sp = (void **)top;
    *--sp = nullptr;                       // keeps the entry's stack aligned like a call
    *--sp = (void *)&trampoline;           // returned to by the first switch
    for (int i = 0; i < 6; ++i) *--sp = nullptr;   // rbp rbx r12 r13 r14 r15
    f.sp = (void *)sp;
}

// back to the scheduler; returns when this work-item is resumed
void yield() {
    Group *g = g_group;
    Fiber &f = g->fibers[(size_t)g->cur];
    hipemu_switch(&f.sp, g->sched_sp);
}

uint64_t source_lane_value(const std::vector<Fiber> &fs, int wave_base, uint64_t in_group, const Item &me, int lane) {
    const int width = me.width <= 0 || me.width > kWave ? kWave : me.width;
    int src = lane;
    switch (me.op) {
        case kShfl:
            src = (lane & ~(width - 1)) + (me.arg & (width - 1));
            break;
        case kShflUp:
            src = (lane & (width - 1)) >= me.arg ? lane - me.arg : lane;
            break;
        case kShflDown:
            src = (lane & (width - 1)) + me.arg < width ? lane + me.arg : lane;
            break;
        case kShflXor: {
            const int idx = lane ^ me.arg;
            src = idx >= ((lane + width) & ~(width - 1)) ? lane : idx;
            break;
        }
        default:
            break;
    }
    if (src < 0 || src >= kWave || !((in_group >> src) & 1ull)) return me.val;   // inactive source
    return fs[(size_t)(wave_base + src)].item.val;
}

// Completes one wave operation of wave w, if some of its lanes wait at one.
bool resolve_wave(Group &g, int w) {
    const int base = w * kWave;
    const int end = std::min<int>((int)g.fibers.size(), base + kWave);
    int first = -1;
    for (int i = base; i < end; ++i)
        if (g.fibers[(size_t)i].item.state == 1) {
            first = i;
            break;
        }
    if (first < 0) return false;
    const Item &lead = g.fibers[(size_t)first].item;
    uint64_t group = 0;
    for (int i = base; i < end; ++i) {
        const Item &it = g.fibers[(size_t)i].item;
        if (it.state == 1 && it.site == lead.site && it.line == lead.line) group |= 1ull << (i - base);
    }
    for (int i = base; i < end; ++i) {
        const Item &it = g.fibers[(size_t)i].item;
        if (((group >> (i - base)) & 1ull) && it.op != lead.op) die("lanes of a wave meet different operations at one site");
    }
    uint64_t ballot = 0;
    for (int i = base; i < end; ++i)
        if (((group >> (i - base)) & 1ull) && g.fibers[(size_t)i].item.val) ballot |= 1ull << (i - base);
    for (int i = base; i < end; ++i) {
        if (!((group >> (i - base)) & 1ull)) continue;
        Item &it = g.fibers[(size_t)i].item;
        if (it.op == kBallot)
            it.result = ballot;
        else if (it.op == kWaveBarrier)
            it.result = 0;
        else
            it.result = source_lane_value(g.fibers, base, group, it, i - base);
    }
    for (int i = base; i < end; ++i)
        if ((group >> (i - base)) & 1ull) g.fibers[(size_t)i].item.state = 0;
    return true;
}

// HIPEMU_ITEM_ORDER=reverse runs the work-items of a workgroup last to first between their
// synchronisation points: a kernel that lets waves touch the same LDS or global words without
// a barrier between them then sees the other order.
bool items_reversed() {
    static const bool rev = [] {
        const char *m = getenv("HIPEMU_ITEM_ORDER");
        return m && strcmp(m, "reverse") == 0;
    }();
    return rev;
}

void run_group(Group &g) {
    const int n = (int)g.fibers.size();
    const int waves = (n + kWave - 1) / kWave;
    const bool rev = items_reversed();
    int done = 0;
    for (;;) {
        bool ran = false;
        for (int ii = 0; ii < n; ++ii) {
            const int i = rev ? n - 1 - ii : ii;
            Fiber &f = g.fibers[(size_t)i];
            if (f.item.state != 0) continue;
            g.cur = i;
            hipemu_switch(&g.sched_sp, f.sp);
            g.cur = -1;
            ran = true;
            if (f.item.state == 3) ++done;
        }
        if (done == n) return;
        if (ran) continue;
        bool progress = false;
        for (int w = 0; w < waves; ++w) progress |= resolve_wave(g, w);
        if (progress) continue;
        int at_bar = 0;
        for (int i = 0; i < n; ++i) at_bar += g.fibers[(size_t)i].item.state == 2;
        if (at_bar + done == n && at_bar > 0) {
            for (int i = 0; i < n; ++i)
                if (g.fibers[(size_t)i].item.state == 2) g.fibers[(size_t)i].item.state = 0;
            continue;
        }
        die("deadlock: no work-item can run and no wave operation or barrier can complete");
    }
}

}  // namespace

Item *current() {
    Group *g = g_group;
    if (!g || g->cur < 0) die("threadIdx used outside a kernel");
    return &g->fibers[(size_t)g->cur].item;
}

uint64_t wave_op(int op, uint64_t val, int arg, int width, const char *file, int line) {
    Item *it = current();
    it->state = 1;
    it->op = op;
    it->val = val;
    it->arg = arg;
    it->width = width;
    it->site = file;
    it->line = line;
    yield();
    return it->result;
}

void sync_threads() {
    Item *it = current();
    it->state = 2;
    yield();
}

namespace {

// Workgroups run in an order set by HIPEMU_BLOCK_ORDER: "forward" (default), "reverse", or a
// number seeding a shuffle.  Results that depend on the order in which workgroups run (which
// the GPU does not fix) show up as differences between orders.
std::vector<size_t> block_order(size_t nb) {
    std::vector<size_t> order(nb);
    for (size_t b = 0; b < nb; ++b) order[b] = b;
    const char *mode = getenv("HIPEMU_BLOCK_ORDER");
    if (mode && strcmp(mode, "reverse") == 0) {
        std::reverse(order.begin(), order.end());
    } else if (mode && strcmp(mode, "forward") != 0 && *mode) {
        uint64_t x = strtoull(mode, nullptr, 0) * 0x9E3779B97F4A7C15ull + 1;
        for (size_t b = nb; b > 1; --b) {   // Fisher-Yates with an xorshift stream
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            std::swap(order[b - 1], order[(size_t)(x % b)]);
        }
    }
    return order;
}

// Workgroup b of a launch, all its work-items on this thread (g holds the fibers).
void run_block(Group &g, size_t b, dim3 grid, dim3 block) {
    const size_t nt = (size_t)block.x * block.y * block.z;
    while (g_stacks.size() < nt) {
        char *st = (char *)malloc(kStack);
        if (!st) die("out of memory for work-item stacks");
        g_stacks.push_back(st);
    }
    t_block_idx = dim3((uint32_t)(b % grid.x), (uint32_t)((b / grid.x) % grid.y),
                       (uint32_t)(b / ((size_t)grid.x * grid.y)));
    for (size_t i = 0; i < nt; ++i) {
        Fiber &f = g.fibers[i];
        f.item = Item{};
        f.item.tid = dim3((uint32_t)(i % block.x), (uint32_t)((i / block.x) % block.y),
                          (uint32_t)(i / ((size_t)block.x * block.y)));
        init_fiber(f, g_stacks[i]);
    }
    run_group(g);
}

// One launch's workgroups, taken in `order` by whichever thread is free.
struct Job {
    const std::function<void()> *body;
    dim3 grid, block;
    const std::vector<size_t> *order;
    std::atomic<size_t> next{0};
};

void work_on(Job &job) {
    const size_t nt = (size_t)job.block.x * job.block.y * job.block.z;
    Group g;
    g.body = job.body;
    g.fibers.resize(nt);
    t_block_dim = job.block;
    t_grid_dim = job.grid;
    g_group = &g;
    for (size_t i; (i = job.next.fetch_add(1)) < job.order->size();) run_block(g, (*job.order)[i], job.grid, job.block);
    g_group = nullptr;
}

// HIPEMU_THREADS=n (n > 1) runs the workgroups of every launch on n host threads at once (the
// caller and n - 1 workers), so that workgroups that race on global memory without the
// atomics or the ordering the code relies on can give other results than one after another.
// Each thread has its own LDS and work-item stacks.
class Pool {
  public:
    explicit Pool(int n) {
        for (int i = 0; i + 1 < n; ++i) std::thread([this] { loop(); }).detach();
        workers_ = n - 1;
    }
    void run(Job &job) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &job;
            active_ = workers_;
            ++gen_;
        }
        cv_.notify_all();
        work_on(job);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return active_ == 0; });
        job_ = nullptr;
    }

  private:
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            Job *job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                job = job_;
            }
            work_on(*job);
            std::lock_guard<std::mutex> lk(mu_);
            if (--active_ == 0) done_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_, done_;
    Job *job_ = nullptr;
    int workers_ = 0, active_ = 0;
    uint64_t gen_ = 0;
};

int pool_threads() {
    static const int n = [] {
        const char *v = getenv("HIPEMU_THREADS");
        return v && *v ? std::max(1, atoi(v)) : 1;
    }();
    return n;
}

std::mutex g_pool_mu;   // launches from several host threads (the server's) take turns

}  // namespace

void run_grid(const std::function<void()> &body, dim3 grid, dim3 block) {
    if (g_group) die("a kernel launched from inside a kernel");
    const size_t nb = (size_t)grid.x * grid.y * grid.z;
    const std::vector<size_t> order = block_order(nb);
    Job job;
    job.body = &body;
    job.grid = grid;
    job.block = block;
    job.order = &order;
    const int nthreads = pool_threads();
    if (nthreads <= 1 || nb <= 1) {
        work_on(job);
        return;
    }
    static Pool *pool = new Pool(nthreads);   // kept for the process
    std::lock_guard<std::mutex> lk(g_pool_mu);
    pool->run(job);
}

namespace {

// The barrier of one cooperative launch, shared by its workgroups' threads.
struct GridBarrier {
    std::mutex mu;
    std::condition_variable cv;
    size_t n = 0, arrived = 0;
    uint64_t gen = 0;
};
thread_local GridBarrier *t_grid_barrier = nullptr;

}  // namespace

void run_grid_cooperative(const std::function<void()> &body, dim3 grid, dim3 block) {
    if (g_group) die("a kernel launched from inside a kernel");
    const size_t nb = (size_t)grid.x * grid.y * grid.z;
    const size_t nt = (size_t)block.x * block.y * block.z;
    GridBarrier bar;
    bar.n = nb;
    std::vector<std::thread> threads;
    threads.reserve(nb);
    for (size_t b = 0; b < nb; ++b) {
        threads.emplace_back([&, b]() {
            std::vector<char *> stacks(nt);
            for (auto &p : stacks)
                if (!(p = (char *)malloc(kStack))) die("out of memory for work-item stacks");
            Group g;
            g.body = &body;
            g.fibers.resize(nt);
            t_block_dim = block;
            t_grid_dim = grid;
            t_block_idx = dim3((uint32_t)(b % grid.x), (uint32_t)((b / grid.x) % grid.y),
                               (uint32_t)(b / ((size_t)grid.x * grid.y)));
            t_grid_barrier = &bar;
            for (size_t i = 0; i < nt; ++i) {
                Fiber &f = g.fibers[i];
                f.item = Item{};
                f.item.tid = dim3((uint32_t)(i % block.x), (uint32_t)((i / block.x) % block.y),
                                  (uint32_t)(i / ((size_t)block.x * block.y)));
                init_fiber(f, stacks[i]);
            }
            g_group = &g;
            run_group(g);
            g_group = nullptr;
            t_grid_barrier = nullptr;
            for (char *p : stacks) free(p);
        });
    }
    for (auto &t : threads) t.join();
}

// Every work-item of the workgroup meets at a workgroup barrier; its first work-item then
// waits for the other workgroups' first work-items, and a second workgroup barrier lets the
// rest go on.  A workgroup that never arrives (it left the kernel, or waits at another
// barrier) is reported instead of hanging the test.
void grid_sync() {
    GridBarrier *b = t_grid_barrier;
    if (!b) die("a grid barrier outside a cooperative launch");
    sync_threads();
    const Item *it = current();
    if (it->tid.x == 0 && it->tid.y == 0 && it->tid.z == 0) {
        std::unique_lock<std::mutex> lk(b->mu);
        const uint64_t gen = b->gen;
        if (++b->arrived == b->n) {
            b->arrived = 0;
            ++b->gen;
            b->cv.notify_all();
        } else if (!b->cv.wait_for(lk, std::chrono::seconds(120), [&] { return b->gen != gen; })) {
            die("grid barrier: not every workgroup arrived within 120 s");
        }
    }
    sync_threads();
}

std::atomic<long long> g_pauses{0};
std::atomic<long long> g_launches{0};
void count_launch() { ++g_launches; }
void pause() {
    ++g_pauses;
    std::this_thread::yield();
}

int resident_per_cu() {
    static const int n = [] {
        const char *v = getenv("HIPEMU_RESIDENT_PER_CU");
        return v && *v ? atoi(v) : 4;
    }();
    return n;
}

void set_error(hipError_t e) { g_last_error = e; }

}  // namespace hipemu

// ---- streams, graphs, events ----------------------------------------------------------------

struct ihipStream_t {
    bool capturing = false;
    std::vector<std::function<void()>> *capture = nullptr;
};
struct ihipGraph_t {
    std::vector<std::function<void()>> calls;
};
struct ihipGraphExec_t {
    std::vector<std::function<void()>> calls;
};
struct ihipEvent_t {
    std::chrono::steady_clock::time_point t;
};

namespace hipemu {
void submit(hipStream_t s, std::function<void()> call) {
    if (s && s->capturing) {
        s->capture->push_back(std::move(call));
        return;
    }
    call();
}
}  // namespace hipemu

hipError_t hipGetLastError() {
    const hipError_t e = hipemu::g_last_error;
    hipemu::g_last_error = hipSuccess;
    return e;
}
hipError_t hipPeekAtLastError() { return hipemu::g_last_error; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated HIP error"; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int) {
    // a small device keeps the emulated grids small: 4 compute units
    *v = a == hipDeviceAttributeMultiprocessorCount ? hipemu::kCus : 160 * 1024;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int v) {
    return v <= 160 * 1024 ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s) {
    hipemu::submit(s, [=]() { memmove(dst, src, n); });
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(dst, src, n, k, nullptr); }
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s) {
    hipemu::submit(s, [=]() { memset(dst, v, n); });
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
static std::atomic<long long> g_device_syncs{0};
hipError_t hipDeviceSynchronize() {
    ++g_device_syncs;
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new ihipStream_t();
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (!s || s->capturing) return hipErrorInvalidValue;
    s->capturing = true;
    s->capture = new std::vector<std::function<void()>>();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    if (!s || !s->capturing) return hipErrorInvalidValue;
    *g = new ihipGraph_t();
    (*g)->calls = std::move(*s->capture);
    delete s->capture;
    s->capture = nullptr;
    s->capturing = false;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    *e = new ihipGraphExec_t();
    (*e)->calls = g->calls;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
    for (auto &c : e->calls) hipemu::submit(s, c);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    hipemu::submit(s, [=]() { e->t = std::chrono::steady_clock::now(); });
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
// Calls that on the GPU wait for all work on the device (HIP frees synchronise the device
// before they release memory): counted, so that tests can check that a path makes none.
extern "C" long long hipemu_device_syncs(void) { return g_device_syncs.load(); }
// Polls of work-items waiting for another workgroup's word (__builtin_amdgcn_s_sleep).
extern "C" long long hipemu_pauses(void) { return hipemu::g_pauses.load(); }
// Kernels executed (a replayed graph counts each kernel it holds).
extern "C" long long hipemu_launches(void) { return hipemu::g_launches.load(); }

hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    *p = calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void *p) {
    ++g_device_syncs;
    free(p);
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n) { return hipHostMalloc(p, n, 0); }
hipError_t hipFree(void *p) { return hipHostFree(p); }
