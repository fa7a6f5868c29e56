// Batched LocalContraction: many independent graphs in one solve (C ABI cc_batch_*).
//
// Graph g (vertices voff[g] .. voff[g+1]-1 of the label array, records
// eoff[g] .. eoff[g+1]-1 with local ids) hashes its local node names with its own seed, and
// components never interact, so a graph's labels equal its solo solve (the method only
// compares priorities inside a component).  Two paths share that arithmetic:
//   - graphs that fit the LDS limits of the chosen small-graph variant are solved one per
//     workgroup by a persistent kernel (lc_small.hpp), all rounds in LDS;
//   - all others form one disjoint-union graph (union id = label slot), whose rounds run
//     the single-graph kernels with per-graph round keys.
// The whole sequence -- state reset, union input, union rounds, label composition and the
// small-graph kernel -- is captured once into a hipGraph and replayed by every later run;
// kernels read their element counts from the device round state, so the captured rounds
// serve any batch of the same shape.  The round loop continues eagerly only if a run needs
// more rounds than were captured.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cc.h"
#include "lc_engine.hpp"
#include "lc_small.hpp"

namespace lc {

// ---- device helpers of the union path --------------------------------------------------

// Union records of the large graphs as packed global ids; graph big[j] owns union records
// [ubase[j], ubase[j+1]).  Out-of-range local ids become loops and set the error bit.
// srcp/dstp non-null (cohorts of the serving scheduler): graph g's records are srcp[g][i],
// dstp[g][i] instead of src/dst at eoff[g] + i.
// bad_g[g] (all graphs) is set for a graph with a record out of range.
__global__ __launch_bounds__(kThreads) void k_globalize(const int32_t *src, const int32_t *dst,
                                                        const int32_t *const *srcp, const int32_t *const *dstp,
                                                        const int64_t *voff, const int64_t *eoff, const int32_t *big,
                                                        const int64_t *ubase, int32_t nbig, uint64_t *out,
                                                        uint32_t *err, int32_t *bad_g) {
    constexpr int64_t kChunk = 16384;
    const int64_t total = nbig ? ubase[nbig] : 0;
    const int64_t nchunks = ceil_div(total, kChunk);
    __shared__ int32_t j0;
    bool bad = false;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t lo = ch * kChunk;
        if (threadIdx.x == 0) {   // graph holding union record lo (binary search)
            int32_t a = 0, b = nbig - 1;
            while (a < b) {
                const int32_t mid = (a + b + 1) / 2;
                if (ubase[mid] <= lo) a = mid; else b = mid - 1;
            }
            j0 = a;
        }
        __syncthreads();
        int32_t j = j0;
        const int64_t hi = min(total, lo + kChunk);
        for (int64_t u = lo + threadIdx.x; u < hi; u += kThreads) {
            while (u >= ubase[j + 1]) ++j;
            const int32_t g = big[j];
            const int64_t base = voff[g];
            const int64_t n = voff[g + 1] - base;
            const int64_t li = u - ubase[j];
            const int32_t x = srcp ? srcp[g][li] : src[eoff[g] + li];
            const int32_t y = srcp ? dstp[g][li] : dst[eoff[g] + li];
            uint64_t rec;
            if ((uint32_t)x < (uint64_t)n && (uint32_t)y < (uint64_t)n) {
                rec = ((uint64_t)(base + x) << 32) | (uint64_t)(base + y);
            } else {
                bad = true;
                bad_g[g] = 1;
                rec = 0ull;   // a loop: skipped by every kernel
            }
            out[u] = rec;
        }
        __syncthreads();
    }
    if (bad) atomicOr(err, 1u);
}

// The whole state is cleared first (the workspace arrives with arbitrary bytes, and every
// field must start where the plain solve's zero-filled upload starts it), then the counts of
// the union graph are set.  A kernel rather than a memset: it is captured into the batch's
// graph, which records no memset nodes.
__global__ __launch_bounds__(kThreads) void k_state_init(RoundState *st, int64_t n0, int64_t m0, int64_t map_cap) {
    static_assert(sizeof(RoundState) % 8 == 0, "state cleared in 8-byte words");
    uint64_t *words = (uint64_t *)st;
    for (size_t i = threadIdx.x; i < sizeof(RoundState) / 8; i += kThreads) words[i] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->n_cur = (u64c)n0;
        st->m_cur = (u64c)m0;
        st->map_cap = (u64c)map_cap;
        st->done = m0 == 0 ? 1 : 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = v;
}

// a graph with a record out of range reports -1 rounds (cohorts: its request alone fails)
__global__ __launch_bounds__(kThreads) void k_mark_bad(int32_t *rounds, const int32_t *bad_g, int32_t G) {
    for (int32_t g = blockIdx.x * kThreads + threadIdx.x; g < G; g += gridDim.x * kThreads)
        if (bad_g[g]) rounds[g] = -1;
}

// labels of the union part (graphs not flagged `skip`), as local ids: at labels[v], or at
// labp[g][v - voff[g]] when labp is non-null (cohorts of the serving scheduler)
__global__ __launch_bounds__(kThreads) void k_compose_batch(Work w, const uint32_t *names_cur, int32_t *labels,
                                                            int32_t *const *labp, const uint32_t *voff,
                                                            const uint8_t *skip) {
    const RoundState *st = w.st;
    const int levels = st->levels;
    for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < w.n0; v += (int64_t)gridDim.x * kThreads) {
        const uint32_t g = w.gid0[v];
        if (skip[g]) continue;
        uint32_t x = w.map0[v];
        for (int l = 0; l < levels && !(x & kFinal); ++l) x = w.maps[st->level_off[l] + x];
        const uint32_t name = (x & kFinal) ? (x & ~kFinal) : (names_cur ? names_cur[x] : x);
        if (labp)
            labp[g][v - voff[g]] = (int32_t)(name - voff[g]);
        else
            labels[v] = (int32_t)(name - voff[g]);
    }
}

// ---- small-graph variants ----------------------------------------------------------------

template <int kNT, int kNMax, int kMMax>
static hipError_t prepare_small_t() {
    return hipFuncSetAttribute((const void *)k_small<kNT, kNMax, kMMax>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)SmallLds<kNT, kNMax, kMMax>::kBytes);
}

template <int kNT, int kNMax, int kMMax>
static hipError_t launch_small_t(const SmallArgs &a, int grid, hipStream_t s) {
    const size_t bytes = SmallLds<kNT, kNMax, kMMax>::kBytes;
    hipLaunchKernelGGL((k_small<kNT, kNMax, kMMax>), dim3(grid), dim3(kNT), bytes, s, a);
    return hipGetLastError();
}

size_t small_bytes(int variant, int threads) {
    switch (variant) {
        case 1: return threads == 512 ? SmallLds<512, 512, 4096>::kBytes : SmallLds<256, 512, 4096>::kBytes;
        case 2: return threads == 512 ? SmallLds<512, 1024, 8192>::kBytes : SmallLds<256, 1024, 8192>::kBytes;
        case 3: return threads == 512 ? SmallLds<512, 2048, 16384>::kBytes : SmallLds<256, 2048, 16384>::kBytes;
        default: return 0;
    }
}

// allow the variant's dynamic LDS size (done outside any capture)
hipError_t prepare_small(int variant, int threads) {
    switch (variant) {
        case 1: return threads == 512 ? prepare_small_t<512, 512, 4096>() : prepare_small_t<256, 512, 4096>();
        case 2: return threads == 512 ? prepare_small_t<512, 1024, 8192>() : prepare_small_t<256, 1024, 8192>();
        case 3: return threads == 512 ? prepare_small_t<512, 2048, 16384>() : prepare_small_t<256, 2048, 16384>();
        default: return hipSuccess;
    }
}

hipError_t launch_small(int variant, int threads, const SmallArgs &a, int grid, hipStream_t s) {
    switch (variant) {
        case 1: return threads == 512 ? launch_small_t<512, 512, 4096>(a, grid, s) : launch_small_t<256, 512, 4096>(a, grid, s);
        case 2: return threads == 512 ? launch_small_t<512, 1024, 8192>(a, grid, s) : launch_small_t<256, 1024, 8192>(a, grid, s);
        case 3: return threads == 512 ? launch_small_t<512, 2048, 16384>(a, grid, s) : launch_small_t<256, 2048, 16384>(a, grid, s);
        default: return hipSuccess;
    }
}

}  // namespace lc

using namespace lc;

struct cc_batch : public lc::Engine {
    int32_t G = 0;
    std::vector<int64_t> h_voff, h_eoff;
    std::vector<uint64_t> h_seeds;
    const int32_t *d_src = nullptr, *d_dst = nullptr;
    cc_options o{};
    cc_batch_config cfg{};
    size_t max_lds = 65536;
    // device arrays carved after the union workspace
    int64_t *d_voff64 = nullptr, *d_eoff64 = nullptr, *d_ubase = nullptr;
    uint32_t *d_voff32 = nullptr, *d_queue = nullptr;
    uint64_t *d_seeds_w = nullptr;
    int32_t *d_big = nullptr, *d_rounds = nullptr, *d_bad = nullptr;
    SmallDesc *d_desc = nullptr;
    std::vector<SmallDesc> h_desc;
    int32_t *desc_labels = nullptr;   // labels pointer the uploaded descriptors point into
    uint8_t *d_skip = nullptr;
    // host plan of the current configuration
    std::vector<int32_t> small_list, big_list;
    std::vector<int64_t> ubase;
    int64_t union_m = 0;
    bool planned = false;
    // captured graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *graph_labels = nullptr;
    int captured_rounds = 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    std::vector<int32_t> last_rounds;
    // a cohort of the serving scheduler: every graph's records and labels at pointers of its
    // own (int32 local ids), rounds driven one at a time by the scheduler (cohort_begin /
    // cohort_advance)
    bool ptr_mode = false;
    std::vector<const int32_t *> h_srcp, h_dstp;
    std::vector<int32_t *> h_labp;
    const int32_t **d_srcp = nullptr, **d_dstp = nullptr;
    int32_t **d_labp = nullptr;
    int async_round = 0, async_phase = 0;
};

namespace {

size_t batch_extra_bytes(int32_t G) {
    const size_t g = (size_t)G + 1;
    return (256 + LC_WS_GUARD) * 16 + 8 * g * 3 + 4 * g + 8 * g + sizeof(RoundKey) * g + 4 * g * 2 +
           sizeof(SmallDesc) * g + g + 64 + 3 * 8 * g + 4 * g;
}

char *carve(char *&p, size_t bytes) {
    char *r = p;
    const size_t step = (bytes + 255) / 256 * 256 + LC_WS_GUARD;
    ws_mark(r, bytes, step - bytes);
    p += step;
    return r;
}

cc_status bfail(cc_batch *b, cc_status s, const char *msg) {
    b->err = msg;
    return s;
}

bool batch_hip(cc_batch *b, hipError_t e, const char *what) { return b->hip_ok(e, what); }

void drop_graph(cc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_labels = nullptr;
}

// split the graphs between the LDS solver and the union path; upload the lists
cc_status plan(cc_batch *b) {
    const SmallVariant sv = kSmallVariants[b->cfg.small_variant];
    b->small_list.clear();
    b->big_list.clear();
    b->ubase.assign(1, 0);
    std::vector<uint8_t> skip(b->G, 0);
    for (int32_t g = 0; g < b->G; ++g) {
        const int64_t n = b->h_voff[g + 1] - b->h_voff[g];
        const int64_t m = b->h_eoff[g + 1] - b->h_eoff[g];
        if (b->cfg.small_variant > 0 && n <= sv.nmax && m <= sv.mmax) {
            b->small_list.push_back(g);
            skip[g] = 1;
        } else {
            b->big_list.push_back(g);
            b->ubase.push_back(b->ubase.back() + m);
        }
    }
    b->union_m = b->ubase.back();
    b->in.s = b->w.keys[1];   // the union input is written there before round 0 reads it
    b->in.d = nullptr;
    b->in.m = b->union_m;
    b->in.n = (uint32_t)b->w.n0;
    b->in.layout = kPacked;
    b->in.vec = 1;
    if (b->cfg.small_variant > 0 &&
        !batch_hip(b, prepare_small(b->cfg.small_variant, b->cfg.small_threads), "small-graph LDS size"))
        return CC_E_HIP;
    hipStream_t s = b->stream;
    b->desc_labels = nullptr;   // descriptors are written against the labels of the next run
    if (!b->big_list.empty() &&
        !batch_hip(b, hipMemcpyAsync(b->d_big, b->big_list.data(), 4 * b->big_list.size(), hipMemcpyHostToDevice, s),
                   "upload union list"))
        return CC_E_HIP;
    if (!batch_hip(b, hipMemcpyAsync(b->d_ubase, b->ubase.data(), 8 * b->ubase.size(), hipMemcpyHostToDevice, s),
                   "upload union offsets"))
        return CC_E_HIP;
    if (b->G && !batch_hip(b, hipMemcpyAsync(b->d_skip, skip.data(), b->G, hipMemcpyHostToDevice, s), "upload flags"))
        return CC_E_HIP;
    if (!batch_hip(b, hipStreamSynchronize(s), "stream synchronize")) return CC_E_HIP;
    b->planned = true;
    drop_graph(b);
    return CC_OK;
}

// Everything before the union rounds: state reset, union input, per-graph round marks.
bool enqueue_prologue(cc_batch *b) {
    hipStream_t s = b->stream;
    const int64_t n0 = b->w.n0;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(kThreads), 0, s, b->w.st, n0, b->union_m, std::max<int64_t>(n0, 1));
    if (!batch_hip(b, hipGetLastError(), "state init")) return false;
    hipLaunchKernelGGL(k_fill_i32, dim3(b->grid_for(b->G)), dim3(kThreads), 0, s, b->d_rounds, 0, (int64_t)b->G);
    if (!batch_hip(b, hipGetLastError(), "round counters")) return false;
    hipLaunchKernelGGL(k_fill_i32, dim3(b->grid_for(b->G)), dim3(kThreads), 0, s, b->d_bad, 0, (int64_t)b->G);
    if (!batch_hip(b, hipGetLastError(), "input flags")) return false;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kThreads), 0, s, (int32_t *)b->d_queue, 0, (int64_t)1);
    if (!batch_hip(b, hipGetLastError(), "queue reset")) return false;
    const int gch = (int)std::min<int64_t>(ceil_div(std::max<int64_t>(b->union_m, 1), 16384), b->grid_cap);
    const int32_t *const *srcp = b->ptr_mode ? b->d_srcp : nullptr;
    const int32_t *const *dstp = b->ptr_mode ? b->d_dstp : nullptr;
    hipLaunchKernelGGL(k_globalize, dim3(gch), dim3(kThreads), 0, s, b->d_src, b->d_dst, srcp, dstp, b->d_voff64,
                       b->d_eoff64, b->d_big, b->d_ubase, (int32_t)b->big_list.size(), b->w.keys[1], &b->w.st->err,
                       b->d_bad);
    return batch_hip(b, hipGetLastError(), "union input");
}

bool enqueue_epilogue(cc_batch *b, int32_t *labels, int cur_round) {
    hipStream_t s = b->stream;
    if (b->w.n0 > 0) {
        const uint32_t *names_cur = cur_round == 0 ? nullptr : b->w.names[cur_round & 1];
        int32_t *const *labp = b->ptr_mode ? b->d_labp : nullptr;
        hipLaunchKernelGGL(k_compose_batch, dim3(b->grid_for(b->w.n0)), dim3(kThreads), 0, s, b->w, names_cur, labels,
                           labp, (const uint32_t *)b->d_voff32, (const uint8_t *)b->d_skip);
        if (!batch_hip(b, hipGetLastError(), "compose")) return false;
    }
    return true;
}

// descriptors of the LDS-path graphs, pointing into `labels` (uploaded when it changes)
bool upload_desc(cc_batch *b, int32_t *labels) {
    if (b->small_list.empty() || b->desc_labels == labels) return true;
    b->h_desc.resize(b->small_list.size());
    for (size_t k = 0; k < b->small_list.size(); ++k) {
        const int32_t g = b->small_list[k];
        SmallDesc &d = b->h_desc[k];
        d.src = b->d_src + b->h_eoff[g];
        d.dst = b->d_dst + b->h_eoff[g];
        d.m = b->h_eoff[g + 1] - b->h_eoff[g];
        d.n = (int32_t)(b->h_voff[g + 1] - b->h_voff[g]);
        d.status = 0;
        d.seed = b->h_seeds[g];
        d.labels = labels + b->h_voff[g];
        d.rounds = b->d_rounds + g;
    }
    if (!batch_hip(b, hipMemcpyAsync(b->d_desc, b->h_desc.data(), sizeof(SmallDesc) * b->h_desc.size(),
                                     hipMemcpyHostToDevice, b->stream), "upload descriptors") ||
        !batch_hip(b, hipStreamSynchronize(b->stream), "stream synchronize"))
        return false;
    b->desc_labels = labels;
    return true;
}

bool enqueue_small(cc_batch *b, int32_t *labels) {
    (void)labels;
    if (b->small_list.empty()) return true;
    SmallArgs a;
    a.desc = b->d_desc;
    a.count = (int32_t)b->small_list.size();
    a.queue = b->d_queue;
    a.err = &b->w.st->err;
    const int grid = (int)std::min<int64_t>((int64_t)b->cus * std::max(1, b->cfg.small_blocks_per_cu), a.count);
    return batch_hip(b, launch_small(b->cfg.small_variant, b->cfg.small_threads, a, std::max(grid, 1), b->stream),
                     "small-graph solver");
}

bool enqueue_union_round(cc_batch *b, int r) {
    PrioCtx pc{};
    pc.keys = b->d_keys;
    pc.voff = b->d_voff32;
    const int kb = ceil_log2_host(std::max<int64_t>(b->w.n0, 2));
    const int passes = npasses(2 * kb);
    return b->enqueue_round(r, b->w.n0, std::max<int64_t>(b->union_m, 1), pc, passes);
}

cc_status capture(cc_batch *b, int32_t *labels) {
    drop_graph(b);
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    bool ok = batch_hip(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    const int rounds = std::max(1, b->cfg.rounds_per_graph);
    if (ok) ok = enqueue_prologue(b);
    if (ok && b->union_m > 0) {
        for (int r = 0; ok && r < rounds; ++r) ok = enqueue_union_round(b, r);
    }
    if (ok) ok = enqueue_epilogue(b, labels, rounds);
    if (ok) ok = enqueue_small(b, labels);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    b->stream = user;
    if (!ok) {
        if (g) (void)hipGraphDestroy(g);
        return CC_E_HIP;
    }
    if (!batch_hip(b, e, "end capture")) return CC_E_HIP;
    b->graph = g;
    if (!batch_hip(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate")) {
        drop_graph(b);
        return CC_E_HIP;
    }
    b->graph_labels = labels;
    b->captured_rounds = b->union_m > 0 ? rounds : 0;
    return CC_OK;
}

cc_status finish_checks(cc_batch *b) {
    const RoundState &st = *b->h_st;
    if (st.err & 1u) return bfail(b, CC_E_INPUT, "a record names a vertex outside its graph");
    if (st.err & ~1u) return bfail(b, CC_E_STATE, "internal consistency check failed on the device");
    return CC_OK;
}

// A batch over graphs packed in d_src/d_dst (cc_batch_create), or over graphs whose records
// and labels sit at per-graph pointers (psrc non-null: a cohort of the serving scheduler, which
// also lends its host mirror of the round state).
cc_status create_batch(int32_t n_graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off, const uint64_t *h_seeds,
                       const void *d_src, const void *d_dst, const cc_options *opts, RoundState *mirror,
                       const int32_t *const *psrc, const int32_t *const *pdst, int32_t *const *plab, cc_batch **out) {
    if (!out) return CC_E_ARG;
    *out = nullptr;
    if (n_graphs < 0 || !opts || (n_graphs > 0 && (!h_vtx_off || !h_edge_off || !h_seeds))) return CC_E_ARG;
    if (n_graphs > 0 && (h_vtx_off[0] != 0 || h_edge_off[0] != 0)) return CC_E_ARG;
    for (int32_t g = 0; g < n_graphs; ++g)
        if (h_vtx_off[g + 1] < h_vtx_off[g] || h_edge_off[g + 1] < h_edge_off[g]) return CC_E_ARG;
    const int64_t n0 = n_graphs ? h_vtx_off[n_graphs] : 0;
    const int64_t m0 = n_graphs ? h_edge_off[n_graphs] : 0;
    if (n0 > 0x7FFFFFFFLL || m0 > 0xFFFFFFFELL) return CC_E_ARG;
    if (m0 > 0 && !psrc && (!d_src || !d_dst)) return CC_E_ARG;
    cc_batch *b = new (std::nothrow) cc_batch();
    if (!b) return CC_E_NOMEM;
    b->G = n_graphs;
    b->h_voff.assign(h_vtx_off, h_vtx_off + n_graphs + 1);
    b->h_eoff.assign(h_edge_off, h_edge_off + n_graphs + 1);
    if (n_graphs == 0) {
        b->h_voff.assign(1, 0);
        b->h_eoff.assign(1, 0);
    }
    b->h_seeds.assign(h_seeds, h_seeds + n_graphs);
    b->d_src = (const int32_t *)d_src;
    b->d_dst = (const int32_t *)d_dst;
    b->o = *opts;
    b->stream = (hipStream_t)opts->stream;
    b->profile = (opts->flags & CC_PROFILE) != 0;
    b->batch = true;
    b->n_graphs = n_graphs;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            b->max_lds = (size_t)lds;
    }
    (void)hipGetLastError();
    b->cus = std::max(b->cus, 1);
    b->grid_cap = b->cus * 8;
    b->cfg.blocks_per_cu = 8;
    b->cfg.small_variant = 2;
    b->cfg.small_threads = 256;
    b->cfg.small_blocks_per_cu = 2;
    b->cfg.rounds_per_graph = 24;
    b->cfg.use_graph = 1;
    b->cfg.radix_form = 1;
    if (small_bytes(b->cfg.small_variant, b->cfg.small_threads) > b->max_lds) b->cfg.small_variant = 1;
    if (psrc) {   // a cohort: the records and labels of graph g at per-graph pointers
        b->ptr_mode = true;
        b->h_srcp.assign(psrc, psrc + n_graphs);
        b->h_dstp.assign(pdst, pdst + n_graphs);
        b->h_labp.assign(plab, plab + n_graphs);
        b->cfg.small_variant = 0;   // every graph takes the union path
        b->cfg.use_graph = 0;       // its rounds are driven one at a time
    }
    if (mirror) {
        b->h_st = mirror;
        b->h_st_borrowed = true;
    } else if (hipHostMalloc((void **)&b->h_st, sizeof(RoundState), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        b->h_st = (RoundState *)calloc(1, sizeof(RoundState));
        b->h_st_pageable = true;
        if (!b->h_st) {
            delete b;
            return CC_E_NOMEM;
        }
    }
    b->ws_need = plan_workspace(n0, m0, true, false, nullptr, nullptr) + batch_extra_bytes(n_graphs);
    *out = b;
    return CC_OK;
}

}  // namespace

extern "C" {

cc_status cc_batch_create(int32_t n_graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const uint64_t *h_seeds, const void *d_src, const void *d_dst, const cc_options *opts,
                          cc_batch **out) {
    return create_batch(n_graphs, h_vtx_off, h_edge_off, h_seeds, d_src, d_dst, opts, nullptr, nullptr, nullptr,
                        nullptr, out);
}

cc_status cc_batch_workspace_size(const cc_batch *b, size_t *bytes) {
    if (!b || !bytes) return CC_E_ARG;
    *bytes = b->ws_need;
    return CC_OK;
}

cc_status cc_batch_set_workspace(cc_batch *b, void *d_ws, size_t bytes) {
    if (!b || !d_ws) return CC_E_ARG;
    if (bytes < b->ws_need) return bfail(b, CC_E_NOMEM, "workspace smaller than cc_batch_workspace_size()");
    if ((uintptr_t)d_ws % 256 != 0) return bfail(b, CC_E_ARG, "workspace must be 256-byte aligned");
    const int64_t n0 = b->h_voff[b->G];
    const int64_t m0 = b->h_eoff[b->G];
    size_t off = plan_workspace(n0, m0, true, false, (char *)d_ws, &b->w);
    char *p = (char *)d_ws + off;
    const size_t g = (size_t)b->G + 1;
    b->d_voff64 = (int64_t *)carve(p, 8 * g);
    b->d_eoff64 = (int64_t *)carve(p, 8 * g);
    b->d_ubase = (int64_t *)carve(p, 8 * g);
    b->d_voff32 = (uint32_t *)carve(p, 4 * g);
    b->d_seeds_w = (uint64_t *)carve(p, 8 * g);
    b->d_keys = (RoundKey *)carve(p, sizeof(RoundKey) * g);
    b->d_desc = (SmallDesc *)carve(p, sizeof(SmallDesc) * g);
    b->d_big = (int32_t *)carve(p, 4 * g);
    b->d_rounds = (int32_t *)carve(p, 4 * g);
    b->d_skip = (uint8_t *)carve(p, g);
    b->d_queue = (uint32_t *)carve(p, 64);
    b->d_srcp = (const int32_t **)carve(p, 8 * g);
    b->d_dstp = (const int32_t **)carve(p, 8 * g);
    b->d_labp = (int32_t **)carve(p, 8 * g);
    b->d_bad = (int32_t *)carve(p, 4 * g);
    b->w.g_rounds = b->d_rounds;
    b->d_seeds = b->d_seeds_w;
    b->d_voff = b->d_voff32;
    b->ws = d_ws;
    b->ws_bytes = bytes;
    std::vector<uint32_t> v32(g);
    for (size_t i = 0; i < g; ++i) v32[i] = (uint32_t)b->h_voff[i];
    hipStream_t s = b->stream;
    bool ok = batch_hip(b, hipMemcpyAsync(b->d_voff64, b->h_voff.data(), 8 * g, hipMemcpyHostToDevice, s), "upload") &&
              batch_hip(b, hipMemcpyAsync(b->d_eoff64, b->h_eoff.data(), 8 * g, hipMemcpyHostToDevice, s), "upload") &&
              batch_hip(b, hipMemcpyAsync(b->d_voff32, v32.data(), 4 * g, hipMemcpyHostToDevice, s), "upload") &&
              (b->G == 0 || batch_hip(b, hipMemcpyAsync(b->d_seeds_w, b->h_seeds.data(), 8 * (size_t)b->G,
                                                        hipMemcpyHostToDevice, s), "upload"));
    if (ok && b->ptr_mode && b->G > 0)
        ok = batch_hip(b, hipMemcpyAsync(b->d_srcp, b->h_srcp.data(), 8 * (size_t)b->G, hipMemcpyHostToDevice, s),
                       "upload") &&
             batch_hip(b, hipMemcpyAsync(b->d_dstp, b->h_dstp.data(), 8 * (size_t)b->G, hipMemcpyHostToDevice, s),
                       "upload") &&
             batch_hip(b, hipMemcpyAsync(b->d_labp, b->h_labp.data(), 8 * (size_t)b->G, hipMemcpyHostToDevice, s),
                       "upload");
    if (!ok) return CC_E_HIP;
    if (n0 > 0) {
        const int ggrid = std::max(1, std::min(b->G, b->grid_cap));
        if (!batch_hip(b, launch_fill_gid(b->w.gid0, (const uint32_t *)b->d_voff32, b->G, ggrid, s), "graph ids"))
            return CC_E_HIP;
    }
    if (!batch_hip(b, hipStreamSynchronize(s), "stream synchronize")) return CC_E_HIP;
    b->planned = false;
    return plan(b);
}

cc_status cc_batch_set_config(cc_batch *b, const cc_batch_config *c) {
    if (!b || !c) return CC_E_ARG;
    if (c->blocks_per_cu < 1 || c->blocks_per_cu > 64 || c->small_variant < 0 ||
        c->small_variant >= kNumSmallVariants || (c->small_threads != 256 && c->small_threads != 512) ||
        c->small_blocks_per_cu < 1 || c->small_blocks_per_cu > 16 || c->rounds_per_graph < 1 ||
        c->rounds_per_graph > 64 || c->radix_form < 0 || c->radix_form > 2)
        return bfail(b, CC_E_ARG, "configuration out of range");
    if (c->small_variant > 0 && small_bytes(c->small_variant, c->small_threads) > b->max_lds)
        return bfail(b, CC_E_ARG, "small-graph variant needs more LDS than the device allows");
    b->cfg = *c;
    if (b->cfg.radix_form == 0) b->cfg.radix_form = 1;
    b->radix_form = b->cfg.radix_form;
    b->grid_cap = b->cus * c->blocks_per_cu;
    if (b->ws) return plan(b);
    return CC_OK;
}

cc_status cc_batch_get_config(const cc_batch *b, cc_batch_config *c) {
    if (!b || !c) return CC_E_ARG;
    *c = b->cfg;
    return CC_OK;
}

cc_status cc_batch_run(cc_batch *b, int32_t *d_labels, int32_t *h_rounds) {
    if (!b || (!d_labels && b->h_voff[b->G] > 0)) return CC_E_ARG;
    if (!b->ws) return bfail(b, CC_E_NOMEM, "no workspace: call cc_batch_set_workspace first");
    if (!b->planned) {
        cc_status st = plan(b);
        if (st != CC_OK) return st;
    }
    b->failed_status = 0;
    for (int i = 0; i < kFamilies; ++i) {
        b->fam_ms[i] = 0.0;
        b->fam_launches[i] = 0;
    }
    if (!upload_desc(b, d_labels)) return CC_E_HIP;
    int cur_round = 0;
    if (b->cfg.use_graph) {
        if (!b->exec || b->graph_labels != d_labels) {
            if (!b->cap_stream &&
                !batch_hip(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "capture stream"))
                return CC_E_HIP;
            const bool prof = b->profile;
            b->profile = false;   // no events inside a captured graph
            cc_status st = capture(b, d_labels);
            b->profile = prof;
            if (st != CC_OK) return st;
        }
        if (!batch_hip(b, hipGraphLaunch(b->exec, b->stream), "graph launch")) return CC_E_HIP;
        if (!b->read_state()) return CC_E_HIP;
        cur_round = b->captured_rounds;
        if (!b->h_st->done && b->union_m > 0) {
            // more rounds than were captured: continue eagerly, then compose again
            int r = cur_round;
            while (!b->h_st->done) {
                if (b->h_st->levels >= kMaxLevels) return bfail(b, CC_E_STATE, "too many rounds for the map arena");
                if (!enqueue_union_round(b, r)) return CC_E_HIP;
                if (!b->read_state()) return CC_E_HIP;
                ++r;
            }
            cur_round = r;
            if (!enqueue_epilogue(b, d_labels, cur_round)) return CC_E_HIP;
            if (!b->read_state()) return CC_E_HIP;
        }
    } else {
        if (!enqueue_prologue(b)) return CC_E_HIP;
        if (!b->read_state()) return CC_E_HIP;
        int r = 0;
        while (b->union_m > 0 && !b->h_st->done) {
            if (b->h_st->err) break;
            if (b->h_st->levels >= kMaxLevels) return bfail(b, CC_E_STATE, "too many rounds for the map arena");
            if (!enqueue_union_round(b, r)) return CC_E_HIP;
            if (!b->read_state()) return CC_E_HIP;
            ++r;
        }
        cur_round = r;
        if (!enqueue_epilogue(b, d_labels, cur_round)) return CC_E_HIP;
        if (!enqueue_small(b, d_labels)) return CC_E_HIP;
        if (!b->read_state()) return CC_E_HIP;
    }
    cc_status st = finish_checks(b);
    if (st != CC_OK) return st;
    if (h_rounds && b->G > 0) {
        if (!batch_hip(b, hipMemcpyAsync(h_rounds, b->d_rounds, 4 * (size_t)b->G, hipMemcpyDeviceToHost, b->stream),
                       "rounds readback") ||
            !batch_hip(b, hipStreamSynchronize(b->stream), "stream synchronize"))
            return CC_E_HIP;
    }
    return CC_OK;
}

cc_status cc_batch_split(const cc_batch *b, int32_t *n_small, int64_t *union_records) {
    if (!b) return CC_E_ARG;
    if (n_small) *n_small = (int32_t)b->small_list.size();
    if (union_records) *union_records = b->union_m;
    return CC_OK;
}

cc_status cc_batch_destroy(cc_batch *b) {
    if (!b) return CC_E_ARG;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (auto e : b->events) (void)hipEventDestroy(e);
    if (b->h_st && !b->h_st_borrowed) {
        if (b->h_st_pageable)
            free(b->h_st);
        else
            (void)hipHostFree(b->h_st);
    }
    delete b;
    return CC_OK;
}

const char *cc_batch_last_error(const cc_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"


// ---- cohorts of the serving scheduler --------------------------------------------------------
//
// A cohort is a batch in pointer mode whose rounds the scheduler drives one at a time on its
// slot stream: cohort_begin enqueues the union input and round 0, cohort_advance (once the
// state readback it enqueued has completed) the next round or the labels.  Each call ends with
// a state readback into the borrowed mirror; the caller records its event after it.

namespace lc {

cc_status cohort_create(int32_t G, const int64_t *h_voff, const int64_t *h_eoff, const uint64_t *h_seeds,
                        const int32_t *const *h_src, const int32_t *const *h_dst, int32_t *const *h_labels,
                        hipStream_t stream, RoundState *mirror, cc_batch **out) {
    if (!h_src || !h_dst || !h_labels || !mirror || G < 1) return CC_E_ARG;
    cc_options o{};
    o.stream = stream;
    return create_batch(G, h_voff, h_eoff, h_seeds, nullptr, nullptr, &o, mirror, h_src, h_dst, h_labels, out);
}

static bool cohort_readback(cc_batch *b) {
    return batch_hip(b, hipMemcpyAsync(b->h_st, b->w.st, sizeof(RoundState), hipMemcpyDeviceToHost, b->stream),
                     "state readback");
}

// the labels of every graph, then its round count into h_rounds (pinned, G entries; -1 for a
// graph with a record out of range)
static cc_status cohort_finish(cc_batch *b, int32_t *h_rounds) {
    if (!enqueue_epilogue(b, nullptr, b->async_round)) return CC_E_HIP;
    hipLaunchKernelGGL(k_mark_bad, dim3(b->grid_for(b->G)), dim3(kThreads), 0, b->stream, b->d_rounds,
                       (const int32_t *)b->d_bad, b->G);
    if (!batch_hip(b, hipGetLastError(), "input flags")) return CC_E_HIP;
    if (!batch_hip(b, hipMemcpyAsync(h_rounds, b->d_rounds, 4 * (size_t)b->G, hipMemcpyDeviceToHost, b->stream),
                   "rounds readback") ||
        !cohort_readback(b))
        return CC_E_HIP;
    b->async_phase = 2;
    return CC_OK;
}

cc_status cohort_begin(cc_batch *b, int32_t *h_rounds) {
    if (!b || !b->ptr_mode || !b->ws) return CC_E_ARG;
    if (!b->planned) {
        const cc_status st = plan(b);
        if (st != CC_OK) return st;
    }
    b->failed_status = 0;
    if (!enqueue_prologue(b)) return CC_E_HIP;
    b->async_round = 0;
    if (b->union_m == 0) return cohort_finish(b, h_rounds);
    if (!enqueue_union_round(b, 0) || !cohort_readback(b)) return CC_E_HIP;
    b->async_round = 1;
    b->async_phase = 1;
    return CC_OK;
}

cc_status cohort_advance(cc_batch *b, int32_t *h_rounds, bool *finished) {
    *finished = false;
    const RoundState &st = *b->h_st;
    // a record out of range (error bit 0) became a loop: its graph alone is reported (by its
    // round count), the others are solved as usual; any other error ends the cohort
    if (st.err & ~1u) {
        *finished = true;
        return bfail(b, CC_E_STATE, "internal consistency check failed on the device");
    }
    if (b->async_phase == 2) {
        *finished = true;
        return CC_OK;
    }
    if (st.done) return cohort_finish(b, h_rounds);
    if (st.levels >= kMaxLevels) {
        *finished = true;
        return bfail(b, CC_E_STATE, "too many rounds for the map arena");
    }
    if (!enqueue_union_round(b, b->async_round) || !cohort_readback(b)) return CC_E_HIP;
    ++b->async_round;
    return CC_OK;
}

}  // namespace lc
