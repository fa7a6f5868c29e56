// Other ways to choose a phase's labels, and the union-find finish.
//
// TreeContraction (Section 3, paragraph "TreeContraction"): every node v points to f(v), the
// node of smallest priority among its neighbours other than v; the nodes of one weakly
// connected component of the graph of f are merged.  Following f from any node ends in a
// 2-cycle {y, f(y)} (Lemma "cycle"), two nodes share a component exactly when they end in
// the same cycle (Lemma "wccs"), and the component's node of smallest priority lies on
// that cycle, so the merged node is named by the cycle's member of smaller priority.  The
// cycle is reached by pointer jumping (proof of the TreeContraction round theorem): every
// node keeps a pointer that starts at f(v) and is replaced by its target's pointer until it
// lands on a cycle, which at least doubles the distance covered per pass.
//
// The one-hop label (the rule Section 6 gives for its Cracker comparison, without the edge
// rewiring) reuses the LocalContraction kernels: the parent is read from the one-hop minimum.
//
// Union-find finish (Section 6): once a round leaves a small graph, its components are found
// by a lock-free union-find over its edges (roots are linked larger index under smaller, so a
// component's root is its smallest index, which is also its smallest name) and every node
// becomes final under its root's name, as one more per-round map.

#include "lc_steps.hpp"

namespace lc {

// ---------------------------------------------------------------------------------------
// TreeContraction
// ---------------------------------------------------------------------------------------

template <class R, bool kFirst>
__global__ __launch_bounds__(kThreads) void k_min1_open(R rd, Work w, PrioCtx pc, const uint32_t *names) {
    step_min1_open<R, kFirst>(rd, w, pc, names);
}

template <bool kFirst, bool kDense>
__global__ __launch_bounds__(kThreads) void k_tree_f(Work w, PrioCtx pc) {
    step_tree_f<kFirst, kDense>(w, pc);
}

template <bool kDense>
__global__ __launch_bounds__(kThreads) void k_tree_jump(Work w, int it) {
    step_tree_jump<kDense>(w, it);
}

template <bool kFirst, bool kDense>
__global__ __launch_bounds__(kThreads) void k_tree_label(Work w, PrioCtx pc, const uint32_t *names) {
    step_tree_label<kFirst, kDense>(w, pc, names);
}

hipError_t launch_min1_open(const Work &w, const EdgeIn *in, const PrioCtx &p, int round, int grid, hipStream_t s) {
    const uint32_t *names = w.names[round & 1];
    if (!in) {
        hipLaunchKernelGGL((k_min1_open<ReadInternal, false>), dim3(grid), dim3(kThreads), 0, s, ReadInternal(w), w,
                           p, names);
        return hipGetLastError();
    }
    const EdgeIn &e = *in;
    switch (e.layout) {
        case kSoa32:
            hipLaunchKernelGGL((k_min1_open<ReadSoa32<1>, true>), dim3(grid), dim3(kThreads), 0, s, ReadSoa32<1>(e),
                               w, p, names);
            break;
        case kSoa64:
            hipLaunchKernelGGL((k_min1_open<ReadSoa64<1>, true>), dim3(grid), dim3(kThreads), 0, s, ReadSoa64<1>(e),
                               w, p, names);
            break;
        default:
            hipLaunchKernelGGL((k_min1_open<ReadPacked<1>, true>), dim3(grid), dim3(kThreads), 0, s,
                               ReadPacked<1>(e), w, p, names);
    }
    return hipGetLastError();
}

template <bool kDense>
static hipError_t tree_labels(const Work &w, const PrioCtx &p, int round, int64_t n_bound, int grid, hipStream_t s) {
    const uint32_t *names = w.names[round & 1];
    if (round == 0)
        hipLaunchKernelGGL((k_tree_f<true, kDense>), dim3(grid), dim3(kThreads), 0, s, w, p);
    else
        hipLaunchKernelGGL((k_tree_f<false, kDense>), dim3(grid), dim3(kThreads), 0, s, w, p);
    hipError_t e = hipGetLastError();
    // a pass at least doubles how far every unfinished pointer has moved along f, so
    // ceil(log2 N) + 1 passes reach every cycle; one more observes that nothing changed
    const int passes = ceil_log2_i64(n_bound < 2 ? 2 : n_bound) + 2;
    for (int it = 0; it < passes && e == hipSuccess; ++it) {
        hipLaunchKernelGGL(k_tree_jump<kDense>, dim3(grid), dim3(kThreads), 0, s, w, it);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (round == 0)
        hipLaunchKernelGGL((k_tree_label<true, kDense>), dim3(grid), dim3(kThreads), 0, s, w, p, names);
    else
        hipLaunchKernelGGL((k_tree_label<false, kDense>), dim3(grid), dim3(kThreads), 0, s, w, p, names);
    return hipGetLastError();
}

hipError_t launch_tree_labels(const Work &w, const PrioCtx &p, int round, int64_t n_bound, int grid, hipStream_t s,
                              bool dense) {
    return dense ? tree_labels<true>(w, p, round, n_bound, grid, s) : tree_labels<false>(w, p, round, n_bound, grid, s);
}

// ---------------------------------------------------------------------------------------
// union-find finish
// ---------------------------------------------------------------------------------------

// Every pointer goes to a smaller index (links put the larger root under the smaller, and
// halving only shortens paths), so a find always ends.
__device__ inline uint32_t uf_find(uint32_t *up, uint32_t x) {
    for (;;) {
        const uint32_t p = up[x];
        if (p == x) return x;
        const uint32_t g = up[p];
        if (g != p) up[x] = g;   // path halving: any ancestor is a valid pointer
        x = g;
    }
}

__global__ __launch_bounds__(kThreads) void k_uf_init(Work w) {
    const int64_t n = (int64_t)w.st->n_cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        w.par[i] = (uint32_t)i;
}

// One union per edge.  A failed link means the other root was linked meanwhile: retry from
// the roots of both ends (the number of links is bounded by the number of nodes).
__global__ __launch_bounds__(kThreads) void k_uf_hook(ReadInternal rd, Work w) {
    constexpr int V = ReadInternal::kV;
    rd.init(w.st);
    const int64_t nch = rd.chunks();
    bool bad = false;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < nch; c += (int64_t)gridDim.x * kThreads) {
        uint32_t a[V], b[V];
        rd.read(c, a, b, bad);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            uint32_t x = a[j], y = b[j];
            while (x != y) {
                x = uf_find(w.par, x);
                y = uf_find(w.par, y);
                if (x == y) break;
                if (x > y) {
                    const uint32_t t = x;
                    x = y;
                    y = t;
                }
                const uint32_t old = atomicCAS(&w.par[y], y, x);
                if (old == y) break;
                y = old;
            }
        }
    }
}

// The finishing map: every node of the remaining graph is final under the name of its
// component's root; appended to the per-round maps like a round's map.
__global__ __launch_bounds__(kThreads) void k_uf_map(Work w, const uint32_t *names_cur) {
    RoundState *st = w.st;
    const int64_t n = (int64_t)st->n_cur;
    if (n == 0) return;
    if (st->map_off + (u64c)n > st->map_cap || st->levels >= kMaxLevels) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&st->err, 2u);
        return;
    }
    uint32_t *out = w.maps + st->map_off;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        out[i] = kFinal | names_cur[uf_find(w.par, (uint32_t)i)];
}

__global__ void k_uf_end(Work w) {
    RoundState *st = w.st;
    if (st->n_cur > 0 && !(st->err & 2u)) {
        st->level_off[st->levels] = st->map_off;
        st->levels += 1;
        st->map_off += st->n_cur;
    }
    st->n_prev = st->n_cur;
    st->n_cur = 0;
    st->m_cur = 0;
    st->done = 1;
}

hipError_t launch_uf_finish(const Work &w, int round, int grid_nodes, int grid_edges, hipStream_t s) {
    hipLaunchKernelGGL(k_uf_init, dim3(grid_nodes), dim3(kThreads), 0, s, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_uf_hook, dim3(grid_edges), dim3(kThreads), 0, s, ReadInternal(w), w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_uf_map, dim3(grid_nodes), dim3(kThreads), 0, s, w, (const uint32_t *)w.names[round & 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_uf_end, dim3(1), dim3(1), 0, s, w);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// MergeToLarge (Section 5, paragraph "MergeToLarge step")
//
// After a LocalContraction step (an even round), every node k of the graph the step left has
// a class: the step's nodes whose parent it is.  The class is large when it holds at least
// alpha nodes, and then its priority is the alpha-th largest priority (this step's) among
// them.  The next (odd) round is the MergeToLarge step on that graph: each node takes as its
// parent the large node of largest priority within distance 2, itself included, or keeps
// itself; the round's relabel, duplicate drop and maps then contract as in any round.
// Priorities of different large nodes are priorities of different vertices, so they never tie.
// ---------------------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_mtl_clear(Work w) {
    step_mtl_clear(w);
}

__global__ __launch_bounds__(kThreads) void k_mtl_size(Work w) {
    step_mtl_size(w);
}

template <bool kFirst>
__global__ __launch_bounds__(kThreads) void k_mtl_count(Work w, PrioCtx pc, const uint32_t *names, int bit,
                                                        uint64_t alpha) {
    step_mtl_count<kFirst>(w, pc, names, bit, alpha);
}

__global__ __launch_bounds__(kThreads) void k_mtl_keep(Work w, int bit, uint64_t alpha) {
    step_mtl_keep(w, bit, alpha);
}

__global__ __launch_bounds__(kThreads) void k_mtl_seed(Work w, uint64_t alpha, int pass) {
    step_mtl_seed(w, alpha, pass);
}

template <class R>
__global__ __launch_bounds__(kThreads) void k_mtl_max(R rd, Work w, uint64_t alpha, int pass) {
    step_mtl_max<R>(rd, w, alpha, pass);
}

__global__ __launch_bounds__(kThreads) void k_mtl_parent(Work w) {
    step_mtl_parent(w);
}

hipError_t launch_mtl_prep(const Work &w, const PrioCtx &p, int round, uint64_t alpha, int grid_cur, int grid_next,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mtl_clear, dim3(grid_next), dim3(kThreads), 0, s, w);
    hipLaunchKernelGGL(k_mtl_size, dim3(grid_cur), dim3(kThreads), 0, s, w);
    const uint32_t *names = w.names[round & 1];
    for (int bit = 31; bit >= 0; --bit) {
        if (round == 0)
            hipLaunchKernelGGL(k_mtl_count<true>, dim3(grid_cur), dim3(kThreads), 0, s, w, p, names, bit, alpha);
        else
            hipLaunchKernelGGL(k_mtl_count<false>, dim3(grid_cur), dim3(kThreads), 0, s, w, p, names, bit, alpha);
        hipLaunchKernelGGL(k_mtl_keep, dim3(grid_next), dim3(kThreads), 0, s, w, bit, alpha);
    }
    return hipGetLastError();
}

hipError_t launch_mtl_labels(const Work &w, uint64_t alpha, int grid_nodes, int grid_edges, hipStream_t s) {
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_mtl_seed, dim3(grid_nodes), dim3(kThreads), 0, s, w, alpha, pass);
        hipLaunchKernelGGL(k_mtl_max<ReadInternal>, dim3(grid_edges), dim3(kThreads), 0, s, ReadInternal(w), w, alpha,
                           pass);
    }
    hipLaunchKernelGGL(k_mtl_parent, dim3(grid_nodes), dim3(kThreads), 0, s, w);
    return hipGetLastError();
}

}  // namespace lc
