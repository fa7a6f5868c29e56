// Whole small rounds in one persistent launch.
//
// Once the remaining graph is small (rounds >= 1 with at most kHashMaxRecords records), a
// round costs far more in launches than in work: it is about sixteen dependent kernels of a
// few microseconds each (Section 3's phase: one-hop minimum, two-hop minimum, parents, label
// map, relabel, duplicate drop, next node set and map), and each waits for the one before.
// Here a single cooperative launch (every workgroup resident at once) runs round after round.
// Each step is the same device body that its own kernel runs (lc_steps.hpp); where a kernel
// boundary used to order two steps, a grid-wide barrier does: a step that reads what other
// workgroups wrote in the step before (m1 before the two-hop pass, the parents before the
// label map, and so on) starts only after every workgroup has finished that step.  Steps that
// touch disjoint data share a phase (the label ranks and the key width; the next node set,
// the per-round map and the write of the kept edges).  TreeContraction's rounds (Section 4)
// run their open one-hop minimum, f and pointer-jumping passes the same way, and MergeToLarge's
// (Section 5) the class sizes and priorities after a LocalContraction step and the two
// candidate passes of its own step.
//
// Every workgroup reads the round state at the top of the loop, after the barrier that ended
// the previous round, so all of them take the same decision.  The launch ends when no edge is
// left, or when the next round does not fit it (more records than the hashed drop takes, no
// room for another per-round map, the statistics table full, the caller's round limit reached,
// few enough records left for the union-find finish, an error flagged); the host then reads
// the state once and goes on with separate launches (or the finish) if edges remain.  The
// loop runs at most kStatRounds rounds in all, so every workgroup leaves it.

#include <hip/hip_cooperative_groups.h>

#include "lc_steps.hpp"

namespace lc {

namespace {

// Whether the next round runs inside this launch (the host's conditions for a hashed round,
// evaluated on the device state).  Rounds from a.round_limit on, and a graph of at most
// a.finish_edges records (which the union-find finish takes over), are left to the host.
// With MergeToLarge (kMerge), a LocalContraction step (an even round) also needs room for the
// map of the MergeToLarge step that follows it: no fold may come between the two.
template <bool kMerge>
__device__ inline bool next_round_fits(const Work &w, const RoundState *st, const FusedLimits &a) {
    const uint64_t m = st->m_cur, n = st->n_cur;
    const int levels = kMerge && !(st->round & 1) ? 2 : 1;
    return st->err == 0 && st->round >= 1 && st->round < a.round_limit && m > (uint64_t)a.finish_edges &&
           m > 0 && m <= (uint64_t)kHashMaxRecords && 2 * m + 1 <= (uint64_t)w.kcap &&
           st->levels + levels <= kMaxLevels && st->map_off + levels * n <= st->map_cap;
}

// Bit map with prefix counts of byte flags (label map or node map), as launch_map_scan builds
// it: one workgroup for small counts, else count, scan and write phases.  `extra` runs on
// workgroup 0 in the first phase (work of the same phase that touches other data).
template <class Extra>
__device__ inline void flag_map(cooperative_groups::grid_group &grid, bool single, const uint8_t *f, const u64c *n,
                                uint32_t *map, u64c *total, uint32_t *partials, Extra extra) {
    if (single) {
        // the one-workgroup scan on the last workgroup, so that `extra` runs beside it
        if (blockIdx.x == 0) extra();
        if (blockIdx.x == gridDim.x - 1) step_flags_single(f, n, map, total);
        return;
    }
    step_flags_reduce(f, n, partials);
    if (blockIdx.x == 0) extra();
    grid.sync();
    if (blockIdx.x == 0) step_scan_single(partials, n, 32 * kThreads, total);
    grid.sync();
    step_flags_down(f, n, partials, map);
}

// kRule: the label rule of the round (FusedRule): LocalContraction's two-hop minimum, the
// one-hop label, TreeContraction's pointer jumping to the 2-cycle of f (Section 4), or
// LocalContraction steps alternating with MergeToLarge steps (Section 5).
template <int kRule>
__global__ __launch_bounds__(kThreads) void k_fused_rounds(ReadInternal rd, Work w, PrioCtx pc, FusedLimits lim) {
    constexpr bool kMerge = kRule == kFusedMerge;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    RoundState *st = w.st;
    auto none = [] {};
    while (next_round_fits<kMerge>(w, st, lim)) {
        const int r = st->round;
        const bool single = st->n_cur <= (u64c)kSmallFlagNodes;
        const uint32_t *names = w.names[r & 1];
        // MergeToLarge: odd rounds are its steps; phase r / 2 takes alpha (the last repeating)
        const bool merge_step = kMerge && (r & 1);
        const uint64_t alpha = kMerge ? lim.alphas[min(r / 2, lim.n_alphas - 1)] : 0;
        if (merge_step) {
            step_round_begin<false>(w, names, nullptr);
            grid.sync();
            for (int pass = 0; pass < 2; ++pass) {
                step_mtl_seed(w, alpha, pass);
                grid.sync();
                step_mtl_max(rd, w, alpha, pass);
                grid.sync();
            }
            step_mtl_parent(w);
            grid.sync();
        } else if (kRule == kFusedTree) {
            step_round_begin<false>(w, names, nullptr);
            grid.sync();
            step_min1_open<ReadInternal, false>(rd, w, pc, names);
            grid.sync();
            step_tree_f<false, false>(w, pc);
            grid.sync();
            // as many jumping passes as a launch sequence enqueues for this round's nodes; the
            // passes after convergence return at once
            const int64_t n = (int64_t)st->n_cur;
            const int passes = ceil_log2_i64(n < 2 ? 2 : n) + 2;
            for (int it = 0; it < passes; ++it) {
                step_tree_jump<false>(w, it);
                grid.sync();
            }
            step_tree_label<false, false>(w, pc, names);
            grid.sync();
        } else {
            step_round_begin<true>(w, names, nullptr);
            grid.sync();
            step_min1_seeded(rd, w);
            grid.sync();
            if (kRule != kFusedOneHop) {   // the two-hop minimum (LocalContraction, its steps under MergeToLarge)
                step_min2(rd, w);
                grid.sync();
            }
            step_parent<false, false>(w, pc, nullptr, kRule == kFusedOneHop ? 0 : 1);
            grid.sync();
        }
        flag_map(grid, single, w.is_label, &st->n_cur, w.lmap, &st->n_labels, w.partials, none);
        grid.sync();
        step_rank_parents(w);
        if (blockIdx.x == 0 && threadIdx.x == 0) step_plan_blocks(w);
        grid.sync();
        step_relabel(rd, w);
        grid.sync();
        step_hash_clear(w, 0);
        grid.sync();
        step_hash_insert(w);
        grid.sync();
        step_hash_count(w);
        grid.sync();
        // the kept keys' tile offsets (and the next round's record count) beside the node map
        flag_map(grid, single, w.has_edge, &st->n_labels, w.nmap, &st->n_next, w.partials,
                 [&] { step_scan_single(w.tile_cnt, &st->aux_n, 0, &st->m_next); });
        grid.sync();
        step_nodes<false, false>(w, names, w.names[(r + 1) & 1], nullptr, nullptr);
        step_map<false>(w, names);
        step_hash_write(w);
        grid.sync();
        if (kMerge && !merge_step) {   // the classes' sizes and alpha-th priorities for the next step
            step_mtl_clear(w);
            grid.sync();
            step_mtl_size(w);
            grid.sync();
            for (int bit = 31; bit >= 0; --bit) {
                step_mtl_count<false>(w, pc, names, bit, alpha);
                grid.sync();
                step_mtl_keep(w, bit, alpha);
                grid.sync();
            }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) step_round_end<false>(w, kDedupHash);
        grid.sync();
    }
}

typedef void (*FusedKernel)(ReadInternal, Work, PrioCtx, FusedLimits);

FusedKernel fused_kernel(int rule) {
    switch (rule) {
        case kFusedTree: return k_fused_rounds<kFusedTree>;
        case kFusedOneHop: return k_fused_rounds<kFusedOneHop>;
        case kFusedMerge: return k_fused_rounds<kFusedMerge>;
        default: return k_fused_rounds<kFusedLocal>;
    }
}

}  // namespace

int fused_rounds_grid(int rule, int per_cu, int cus) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fused_kernel(rule), kThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return occ < 1 ? 0 : cus * (per_cu < occ ? per_cu : occ);
}

hipError_t launch_fused_rounds(const Work &w, int rule, int grid, FusedLimits lim, hipStream_t s) {
    ReadInternal rd(w);
    Work wk = w;
    PrioCtx pc{};
    if (lim.round_limit > kStatRounds) lim.round_limit = kStatRounds;
    void *args[] = {&rd, &wk, &pc, &lim};
    return hipLaunchCooperativeKernel(fused_kernel(rule), dim3(grid), dim3(kThreads), args, 0, s);
}

}  // namespace lc
