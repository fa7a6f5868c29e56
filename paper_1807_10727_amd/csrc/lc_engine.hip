// Round engine and C ABI (include/cc.h) of the plain single-graph solve.
//
// Host side of one LocalContraction round: enqueue the round's kernels on the caller's
// stream, read the device round state back once, keep the per-round statistics.  The
// library never allocates device memory; all arrays live in the caller's workspace.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cc.h"
#include "lc_engine.hpp"

#if defined(__has_feature)
#if __has_feature(address_sanitizer) && LC_WS_GUARD > 0
#define LC_WS_POISON 1
#include <sanitizer/asan_interface.h>
#endif
#endif

namespace lc {

// Kernel families timed with CC_PROFILE.  The round-0 passes over the input records
// ("_round0") are separate families, so each of them is exactly one kernel symbol.
const char *const kFamilyNames[kFamilies] = {
    "round_begin", "min1_round0", "min1",      "min2_round0", "min2",      "parent",    "label_ranks",
    "relabel_round0", "relabel",  "sort_hist", "sort_scan",   "sort_scatter", "unique", "node_scan",
    "nodes",       "map",         "round_end",   "compose",   "flatten",
    "part_a_hist", "part_a_scatter", "part_b_hist", "part_b_scatter", "part_scan", "min1_tiled", "min2_tiled",
    "relabel_tiled", "tail_graph", "uf_finish", "hash_dedup", "merge_large", "part_rows_hist", "part_rows_scatter", "bucket_sort",
    "fused_rounds"};

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

#ifdef LC_WS_POISON
void ws_mark(char *p, size_t bytes, size_t gap) {
    ASAN_UNPOISON_MEMORY_REGION(p, bytes);
    ASAN_POISON_MEMORY_REGION(p + bytes, gap);
}
#else
void ws_mark(char *, size_t, size_t) {}
#endif

bool choose_tiled(int64_t n0, int64_t m0, uint32_t flags) {
    if (flags & CC_ROUND0_DIRECT) return false;
    if (!tiled_fits(n0)) return false;
    if (flags & CC_ROUND0_TILED) return true;
    return n0 >= kTiledMinVertices && m0 >= kTiledMinVertices;
}

size_t plan_workspace(int64_t n0, int64_t m0, bool batch, bool tiled, char *base, Work *w, uint32_t extras) {
    const size_t n = (size_t)std::max<int64_t>(n0, 1);
    const size_t m = (size_t)std::max<int64_t>(m0, 2);
    // records a key buffer holds: the tiled round 0 keeps two directed records per input
    const size_t mk = tiled ? 2 * m : m;
    const size_t tiles = (size_t)ceil_div((int64_t)mk, kSortTile) + 2;
    const size_t slabs = (size_t)ceil_div((int64_t)mk, kSlab) + 1;
    size_t count_entries = (size_t)kRadixMax * tiles;
    if (tiled) {
        const TPlan tp = tiled_plan(n0, m0);
        count_entries = std::max(count_entries, (size_t)256 * (size_t)tp.tiles_a);
        count_entries = std::max(count_entries, (size_t)tp.rows * (size_t)tp.tiles_b);
    }
    // the sampled buckets' second level: tiles never cross a first-level bucket
    if (!batch) count_entries = std::max(count_entries, (size_t)256 * (tiles + kBucketLevel2Tiles));
    const size_t parts = std::max<size_t>((size_t)ceil_div((int64_t)n, kScanTile),
                                          (size_t)ceil_div((int64_t)count_entries, kScanTile)) + 16;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        const size_t next = align_up(off + bytes, 256) + LC_WS_GUARD;
        if (p) ws_mark(p, bytes, next - off - bytes);
        off = next;
        return p;
    };
    Work t{};
    t.st = (RoundState *)take(sizeof(RoundState));
    t.ml = (uint32_t *)take(8 * n);
    t.par = (uint32_t *)take(4 * n);
    t.has_edge = (uint8_t *)take(n + 64);
    t.nmap = (uint32_t *)take(8 * (size_t)ceil_div((int64_t)n, 32) + 64);
    t.is_label = (uint8_t *)take(n + 64);
    t.lmap = (uint32_t *)take(8 * (size_t)ceil_div((int64_t)n, 32) + 64);
    t.lab_at = (uint32_t *)take(4 * n);
    t.newidx = (uint32_t *)take(4 * n);
    t.names[0] = (uint32_t *)take(4 * n);
    t.names[1] = (uint32_t *)take(4 * n);
    t.idx_of = (uint32_t *)take(4 * n);
    t.map0 = (uint32_t *)take(4 * n);
    t.maps = (uint32_t *)take(4 * n);
    if (batch) {
        t.gids[0] = (uint32_t *)take(4 * n);
        t.gids[1] = (uint32_t *)take(4 * n);
        t.gid0 = (uint32_t *)take(4 * n);
    }
    t.keys[0] = (uint64_t *)take(8 * mk);
    t.keys[1] = (uint64_t *)take(8 * mk);
    t.counts = (uint32_t *)take(4 * count_entries);
    t.kcap = (int64_t)mk;
    t.tile_cnt = (uint32_t *)take(4 * tiles + 64);
    t.slab_cnt = (uint32_t *)take(4 * slabs + 64);
    t.partials = (uint32_t *)take(4 * parts);
    if (extras & kWsExplicit) t.pinv = (uint32_t *)take(4 * n);
    if (extras & kWsRecord) {
        t.rec_cap = kRecordPerVertex * (int64_t)n;
        t.rec = (uint32_t *)take(4 * (size_t)t.rec_cap);
    }
    t.sweep = (uint32_t *)take(4 * (size_t)kSweepWords);
    t.sweep_desc = (uint32_t *)take(4 * (size_t)kRadixMax * tiles);
    if (!batch) {
        t.btab = (BucketTab *)take(sizeof(BucketTab) * 257);
        t.bseg = (uint64_t *)take(8 * 257);
        t.btile = (uint32_t *)take(4 * 257);
    }
    if (extras & kWsMerge) {
        t.mtl_size = (uint32_t *)take(4 * n);
        t.mtl_v = (uint32_t *)take(4 * n);
        t.mtl_cnt = (uint32_t *)take(4 * n);
        t.mtl_acc[0] = (uint64_t *)take(8 * n);
        t.mtl_acc[1] = (uint64_t *)take(8 * n);
    }
    t.n0 = n0;
    t.m0 = m0;
    if (w) *w = t;
    return off;
}

int Engine::grid_for(int64_t units) const {
    int64_t g = ceil_div(std::max<int64_t>(units, 1), kThreads);
    return (int)std::min<int64_t>(g, grid_cap);
}

int Engine::grid_tiles(int64_t keys) const {
    int64_t g = ceil_div(std::max<int64_t>(keys, 1), kSortTile);
    return (int)std::min<int64_t>(g, grid_cap);
}

bool Engine::hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    err = buf;
    failed_status = CC_E_HIP;
    return false;
}

bool Engine::ev_begin(int family) {
    if (!profile || !((prof_mask >> family) & 1ull)) return false;
    if (ev_used + 2 > (int)events.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            events.push_back(e);
        }
    }
    (void)hipEventRecord(events[ev_used], stream);
    pending.push_back({family, ev_used});
    ev_used += 2;
    return true;
}

void Engine::ev_end(bool open) {
    if (!open || pending.empty()) return;
    (void)hipEventRecord(events[pending.back().second + 1], stream);
}

void Engine::ev_collect() {
    if (!profile) return;
    for (auto &p : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, events[p.second], events[p.second + 1]) == hipSuccess) {
            fam_ms[p.first] += ms;
            fam_launches[p.first] += 1;
        }
    }
    pending.clear();
    ev_used = 0;
}

#define RUN(fam, expr)                                  \
    do {                                                \
        const bool ev_ = ev_begin(fam);                 \
        hipError_t e_ = (expr);                         \
        ev_end(ev_);                                    \
        if (!hip_ok(e_, kFamilyNames[fam])) return false; \
    } while (0)

bool Engine::enqueue_round(int r, int64_t N, int64_t M, const PrioCtx &pc, int passes_bound) {
    const bool first = r == 0;
    const EdgeIn *src = first ? &in : nullptr;
    const int gn = grid_for(N);
    const int gm = grid_for(ceil_div(M, first ? 4 : 2));
    const int gt = grid_tiles(M);
    // the scatter keeps scatter_waves waves per SIMD resident (four-wave workgroups): a grid
    // of exactly that many workgroups runs in one go instead of a resident share and a tail
    const int gt_scatter = LC_SCATTER_GRID ? std::min(gt, std::max(1, cus * scatter_waves)) : gt;
    // rows of the gathering row passes launched together (0: all of them)
    const int row_gen = row_generation < 0 ? 0 : cus * row_generation;
    const int gscan_l = (int)std::min<int64_t>(ceil_div(std::max<int64_t>(N, 1), 32 * kThreads), grid_cap);
    const int kb = ceil_log2_host(std::max<int64_t>(N, 2));
    const int nbits = 2 * kb;   // edge_key
    const int passes = passes_bound >= 0 ? passes_bound : npasses(nbits);
    // the tiled round 0 hands the first radix pass up to twice as many slab tiles
    const int64_t scan_entries =
        (int64_t)kRadixMax * (ceil_div(std::max<int64_t>(first && tiled ? 2 * M : M, 1), kSortTile) + 2);
    const int gslab = (int)std::min<int64_t>(ceil_div(std::max<int64_t>(M, 1), kSlab), grid_cap);
    const int gscan_c = (int)std::min<int64_t>(ceil_div(scan_entries, kScanTile), grid_cap);
    // small rounds scan in one workgroup: one launch instead of three (launch-bound sizes)
    const bool small_sort = scan_entries <= kSmallScanEntries;
    const bool small_flags = N <= kSmallFlagNodes;

    RUN(kRoundBegin,
        launch_round_begin(w, !first && !batch && variant != kVarTree && mtl_mode != 2, r, gn, stream, pc.tab));
    if (batch) RUN(kRoundBegin, launch_batch_keys(w, d_keys, d_seeds, n_graphs, stream));
    if (first && tiled) {
        const int ga = (int)std::min<int64_t>(tp.tiles_a, grid_cap);
        const int gb = (int)std::min<int64_t>(tp.tiles_b, grid_cap);
        const int gsa = (int)std::min<int64_t>(ceil_div(256 * tp.tiles_a, kScanTile), grid_cap);
        const int gsb = (int)std::min<int64_t>(ceil_div((int64_t)tp.rows * tp.tiles_b, kScanTile), grid_cap);
        if (tiled_rows) {
            const int gr = (int)std::min<int64_t>(tp.tiles_r, grid_cap);
            const int gsr = (int)std::min<int64_t>(ceil_div((int64_t)tp.rows * tp.tiles_r, kScanTile), grid_cap);
            RUN(kPartRowsHist, launch_tiled_partition(w, in, tp, gr, stream, 10));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsr, stream, 11));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, 1, stream, 12));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsr, stream, 13));
            RUN(kPartRowsScatter, launch_tiled_partition(w, in, tp, gr, stream, 14));
        } else {
            RUN(kPartAHist, launch_tiled_partition(w, in, tp, ga, stream, 0));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsa, stream, 1));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, 1, stream, 2));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsa, stream, 3));
            RUN(kPartAScatter, launch_tiled_partition(w, in, tp, ga, stream, 4));
            RUN(kPartBHist, launch_tiled_partition(w, in, tp, gb, stream, 5));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsb, stream, 6));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, 1, stream, 7));
            RUN(kPartScan, launch_tiled_partition(w, in, tp, gsb, stream, 8));
            RUN(kPartBScatter, launch_tiled_partition(w, in, tp, gb, stream, 9));
        }
        RUN(kMin1Tiled, launch_tiled_min1(w, pc, tp, stream, variant == kVarTree));
        if (variant == kVarTree)
            RUN(kParent, launch_tree_labels(w, pc, r, N, gn, stream, true));
        else if (variant == kVarOneHop)
            RUN(kParent, launch_tiled_parent1(w, pc, gn, stream));
        else
            RUN(kMin2Tiled, launch_tiled_min2(w, pc, tp, stream, row_gen, row_pairs));
        RUN(kLabelRanks, launch_rank_parents(w, gn, small_flags ? 0 : gscan_l, stream));
        RUN(kRelabelTiled, launch_tiled_relabel(w, tp, stream, row_gen, relabel_pairs));
    } else if (mtl_mode == 2) {   // MergeToLarge step (rounds >= 1 only)
        RUN(kMergeLarge, launch_mtl_labels(w, mtl_alpha, gn, gm, stream));
        RUN(kLabelRanks, launch_rank_parents(w, gn, small_flags ? 0 : gscan_l, stream));
        RUN(kRelabel, launch_relabel(w, src, gslab, stream));
    } else if (variant == kVarTree) {
        RUN(first ? kMin1In : kMin1, launch_min1_open(w, src, pc, r, gm, stream));
        RUN(kParent, launch_tree_labels(w, pc, r, N, gn, stream));
        RUN(kLabelRanks, launch_rank_parents(w, gn, small_flags ? 0 : gscan_l, stream));
        RUN(first ? kRelabelIn : kRelabel, launch_relabel(w, src, gslab, stream));
    } else {
        RUN(first ? kMin1In : kMin1, launch_min1(w, src, pc, batch, r, gm, stream));
        if (variant != kVarOneHop) RUN(first ? kMin2In : kMin2, launch_min2(w, src, gm, stream));
        RUN(kParent, launch_parent(w, pc, batch, r, gn, stream, variant == kVarOneHop));
        RUN(kLabelRanks, launch_rank_parents(w, gn, small_flags ? 0 : gscan_l, stream));
        RUN(first ? kRelabelIn : kRelabel, launch_relabel(w, src, gslab, stream));
    }
    // rounds >= 1 small enough for the key set drop repeats by hashing; larger ones choose on
    // the device once their key count is known (both ways enqueued, the unused one returns at
    // once); round 0 sorts
    const int dedup = !LC_HASH_DEDUP || first                         ? kDedupSort
                      : (M <= kHashMaxRecords && 2 * M + 1 <= w.kcap) ? kDedupHash
                                                                      : kDedupDevice;
    const bool gated = dedup == kDedupDevice;
    const int64_t hmax = dedup == kDedupHash ? 2 * M + 1 : std::min<int64_t>(2 * kHashMaxRecords + 1, w.kcap);
    const int ghash = grid_tiles(hmax);
    // the table sized and cleared first: when gated, that kernel also records the choice
    if (dedup != kDedupSort) RUN(kHashDedup, launch_hash_dedup(w, grid_for(hmax), stream, 1, gated));
    const bool buckets = first && !batch && round0_sort == 2;
    if (buckets) {   // round 0's keys into sampled buckets, each sorted in LDS (lc_bucket.hip)
        const int64_t entries =
            (int64_t)256 * (ceil_div(std::max<int64_t>(tiled ? 2 * M : M, 1), kSortTile) + 2 + kBucketLevel2Tiles);
        const int gsb = (int)std::min<int64_t>(ceil_div(entries, kScanTile), grid_cap);
        RUN(kBucketSort, launch_bucket(w, 0, 1, stream));
        for (int level = 0; level < 2; ++level) {
            if (level == 1) {
                RUN(kBucketSort, launch_bucket(w, 3, 1, stream));
                RUN(kBucketSort, launch_bucket(w, 4, 256, stream));
            }
            RUN(kBucketSort, launch_bucket(w, level ? 5 : 1, gt, stream));
            RUN(kSortScan, launch_sort_pass(w, 0, gsb, stream, 1));
            RUN(kSortScan, launch_sort_pass(w, 0, 1, stream, 2));
            RUN(kSortScan, launch_sort_pass(w, 0, gsb, stream, 3));
            RUN(kBucketSort, launch_bucket(w, level ? 6 : 2, gt, stream));
        }
        RUN(kBucketSort, launch_bucket(w, 7, grid_cap, stream));
    }
    const bool sweep = radix_form == 2 && w.sweep && dedup != kDedupHash && !buckets && passes > 0 &&
                       (uint64_t)M < kSweepMaxKeys;   // a round's keys never outnumber its records
    if (sweep) {   // one count pass for every digit, then one scatter a digit (offsets by look-back)
        RUN(kSortHist, launch_sort_pass(w, 0, 1, stream, 6, gated));
        RUN(kSortHist, launch_sort_pass(w, 0, gt, stream, 7, gated));
        for (int p = 0; p < passes; ++p)
            RUN(kSortScatter, launch_sort_pass(w, p, gt_scatter, stream, 8, gated, scatter_waves));
    }
    for (int p = 0; p < (dedup == kDedupHash || buckets || sweep ? 0 : passes); ++p) {
        RUN(kSortHist, launch_sort_pass(w, p, gt, stream, 0, gated));
        if (small_sort) {
            RUN(kSortScan, launch_sort_pass(w, p, 1, stream, 5));
        } else {
            RUN(kSortScan, launch_sort_pass(w, p, gscan_c, stream, 1));
            RUN(kSortScan, launch_sort_pass(w, p, 1, stream, 2));
            RUN(kSortScan, launch_sort_pass(w, p, gscan_c, stream, 3));
        }
        RUN(kSortScatter, launch_sort_pass(w, p, gt_scatter, stream, 4, gated, scatter_waves));
    }
    if (dedup != kDedupSort) {   // after the gated sort, whose skipped count pass empties aux_n
        RUN(kHashDedup, launch_hash_dedup(w, gt, stream, 2));
        RUN(kHashDedup, launch_hash_dedup(w, ghash, stream, 3));
    }
    if (dedup != kDedupHash) RUN(kUnique, launch_unique(w, gt, stream, 0, gated));
    RUN(dedup == kDedupHash ? kHashDedup : kUnique, launch_unique(w, 1, stream, 1));   // tile counts scanned
    if (small_flags) {
        RUN(kNodeScan, launch_map_scan(w, false, 1, stream, 3));
    } else {
        RUN(kNodeScan, launch_map_scan(w, false, gscan_l, stream, 0));
        RUN(kNodeScan, launch_map_scan(w, false, 1, stream, 1));
        RUN(kNodeScan, launch_map_scan(w, false, gscan_l, stream, 2));
    }
    RUN(kNodes, launch_nodes(w, batch, r, gn, stream));
    RUN(kMap, launch_map(w, r, gn, stream));
    if (mtl_mode == 1) RUN(kMergeLarge, launch_mtl_prep(w, pc, r, mtl_alpha, gn, gn, stream));
    if (dedup != kDedupSort) RUN(kHashDedup, launch_hash_dedup(w, ghash, stream, 4));
    if (dedup != kDedupHash) RUN(kUnique, launch_unique(w, gt, stream, 2, gated));
    RUN(kRoundEnd, launch_round_end(w, r, dedup, stream));
    return true;
}

bool Engine::flatten() {
    RUN(kFlatten, launch_flatten(w, host_levels, grid_for(w.n0), stream));
    host_levels = 0;
    host_map_used = 0;
    return true;
}

bool Engine::read_state() {
    if (!hip_ok(hipMemcpyAsync(h_st, w.st, sizeof(RoundState), hipMemcpyDeviceToHost, stream), "state readback"))
        return false;
    if (!hip_ok(hipStreamSynchronize(stream), "stream synchronize")) return false;
    ev_collect();
    return true;
}

bool Engine::write_initial_state(int64_t n_cur, int64_t m_cur, uint64_t seed) {
    memset(h_st, 0, sizeof(RoundState));
    h_st->n_cur = (u64c)n_cur;
    h_st->m_cur = (u64c)m_cur;
    h_st->seed = seed;
    h_st->map_cap = (u64c)std::max<int64_t>(w.n0, 1);
    // ordered before every later kernel on the stream; the host buffer is next written by
    // the state readback of round 0, which the stream also orders after this copy
    return hip_ok(hipMemcpyAsync(w.st, h_st, sizeof(RoundState), hipMemcpyHostToDevice, stream), "state upload");
}

int ceil_log2_host(int64_t n) {
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

}  // namespace lc

using namespace lc;

namespace lc {

// an error that ends the current solve (later calls return it until cc_reset)
cc_status fail(cc_ctx *c, cc_status s, const char *msg) {
    if (c) {
        c->err = msg;
        c->failed_status = s;
    }
    return s;
}

// a rejected call: the context is unchanged
cc_status reject(cc_ctx *c, cc_status s, const char *msg) {
    if (c) c->err = msg;
    return s;
}

cc_status hip_status(cc_ctx *c) { return c->failed_status ? c->failed_status : CC_E_HIP; }

}  // namespace lc

namespace {

uint32_t ws_extras(uint32_t flags) {
    return ((flags & CC_EXPLICIT_PRIO) ? (uint32_t)kWsExplicit : 0u) | ((flags & CC_RECORD_ROUNDS) ? (uint32_t)kWsRecord : 0u) |
           ((flags & CC_MERGE_TO_LARGE) ? (uint32_t)kWsMerge : 0u);
}

cc_status reset_solve(cc_ctx *c, uint64_t seed) {
    c->o.seed = seed;
    c->stats.clear();
    c->rounds = 0;
    c->next_round = 0;
    c->ran_first = false;
    c->labels_ready = false;
    c->done = c->g.n_edges == 0;
    c->host_levels = 0;
    c->host_map_used = 0;
    c->n_cur = c->g.n_vertices;
    c->m_cur = c->g.n_edges;
    c->last_graph_round = -1;
    c->finished = false;
    c->failed_status = 0;
    c->err.clear();
    c->recs.clear();
    c->rec_used = 0;
    c->inv_for = nullptr;
    for (int i = 0; i < kFamilies; ++i) {
        c->fam_ms[i] = 0.0;
        c->fam_launches[i] = 0;
    }
    if (!c->write_initial_state(c->n_cur, c->m_cur, seed)) return hip_status(c);
    return CC_OK;
}

}  // namespace

namespace lc {

// The explicit priority table of round r: the one set for the latest round <= r (null: hash).
const uint32_t *table_for(const cc_ctx *c, int32_t r) {
    const uint32_t *t = nullptr;
    int32_t best = -1;
    for (const auto &e : c->prio_tabs)
        if (e.first <= r && e.first > best) {
            best = e.first;
            t = e.second;
        }
    return t;
}

// Enqueue round `next_round` and the asynchronous readback of the device state (no wait).
// *launched is 0 when nothing was enqueued (solve finished, or an error was returned).
cc_status ctx_round_enqueue(cc_ctx *c, int *launched) {
    *launched = 0;
    if (c->failed_status) return c->failed_status;
    if (!c->ws) return reject(c, CC_E_NOMEM, "no workspace: call cc_set_workspace first");
    if (c->done) return CC_DONE;
    const int r = c->next_round;
    const int64_t N = r == 0 ? c->g.n_vertices : c->n_cur;
    const int64_t M = r == 0 ? c->g.n_edges : c->m_cur;
    // MergeToLarge: even rounds are LocalContraction steps, odd rounds the step after each.
    // An LC step keeps room for its own map level and the step's, because the step reads the
    // sizes and priorities that the LC step left, and a fold between them must not intervene.
    const bool mtl = (c->o.flags & CC_MERGE_TO_LARGE) != 0;
    const int levels_needed = mtl ? 2 : 1;
    if (r > 0 && !(mtl && (r & 1)) &&
        (c->host_levels + levels_needed > kMaxLevels ||
         c->host_map_used + levels_needed * N > std::max<int64_t>(c->g.n_vertices, 1))) {
        if (!c->flatten()) return hip_status(c);
    }
    c->mtl_mode = !mtl ? 0 : (r & 1) ? 2 : 1;
    if (mtl) {
        const size_t ph = (size_t)(r / 2);
        c->mtl_alpha = (uint64_t)c->mtl_alphas[std::min(ph, c->mtl_alphas.size() - 1)];
    }
    PrioCtx pc{};
    pc.key = round_key(c->o.seed, r);
    pc.tab = table_for(c, r);
    if (pc.tab) {
        pc.inv = c->w.pinv;
        if (c->inv_for != pc.tab) {   // a new table: build (and check) its inverse first
            if (!c->hip_ok(launch_prio_inverse(c->w, pc.tab, c->grid_for(c->g.n_vertices), c->stream),
                           "priority inverse"))
                return hip_status(c);
            c->inv_for = pc.tab;
        }
    }
    if (!c->enqueue_round(r, N, M, pc)) return hip_status(c);
    if (c->w.rec) {   // CC_RECORD_ROUNDS: copy the parents before the next round overwrites them
        const int64_t count = r == 0 ? c->g.n_vertices : N;
        const int64_t need = r == 0 ? count : 2 * count;
        if ((int64_t)c->recs.size() <= r) c->recs.resize((size_t)r + 1, cc_ctx::Rec{-1, 0});
        if (c->rec_used + need <= c->w.rec_cap) {
            if (!c->hip_ok(launch_record_parents(c->w, r, c->w.rec + c->rec_used, c->grid_for(count), c->stream),
                           "record parents"))
                return hip_status(c);
            c->recs[r] = cc_ctx::Rec{c->rec_used, count};
            c->rec_used += need;
        }
    }
    if (!c->hip_ok(hipMemcpyAsync(c->h_st, c->w.st, sizeof(RoundState), hipMemcpyDeviceToHost, c->stream),
                   "state readback"))
        return hip_status(c);
    c->pending_N = N;
    c->pending_M = M;
    *launched = 1;
    return CC_OK;
}

// Consume the state of the round enqueued last (its readback must have completed).
cc_status ctx_round_complete(cc_ctx *c, cc_round_stats *out) {
    c->ev_collect();
    const RoundState &st = *c->h_st;
    const int r = c->next_round;
    const int64_t N = c->pending_N, M = c->pending_M;
    if (st.err & 1u) return fail(c, CC_E_INPUT, "an edge record names a vertex outside [0, n_vertices)");
    if (st.err & 8u) return fail(c, CC_E_INPUT, "an explicit priority table is not a permutation of [0, n_vertices)");
    if (st.err & ~1u) return fail(c, CC_E_STATE, "internal consistency check failed on the device");
    if (r == 0) c->ran_first = true;
    if (r > 0) {
        c->host_levels += 1;
        c->host_map_used += N;
    }
    c->next_round = r + 1;
    c->n_cur = (int64_t)st.n_cur;
    c->m_cur = (int64_t)st.m_cur;
    c->done = st.m_cur == 0;
    if (r == 0 && st.n_active == 0) {   // no loop-free record: zero rounds, labels are the ids
        return CC_DONE;
    }
    cc_round_stats s{};
    s.round = r;
    s.n_active = (int64_t)st.n_active;
    s.m_in = M;
    s.m_survive = (int64_t)st.s_count;
    s.m_out = (int64_t)st.m_next;
    s.n_finalised = (int64_t)st.n_final;
    s.m_sorted = (int64_t)st.s_keys;
    c->stats.push_back(s);
    c->rounds = r + 1;
    if (out) *out = s;
    return CC_OK;
}

cc_status ctx_labels_enqueue(cc_ctx *c, void *d_labels) {
    if (c->g.n_vertices == 0) return CC_OK;
    // with several levels, fold them first: compose then takes one lookup per vertex
    if (c->host_levels >= 2 && !c->flatten()) return hip_status(c);
    const bool out64 = c->g.layout == CC_EDGES_SOA_I64;
    const int grid = c->grid_for(c->g.n_vertices);
    const bool ev = c->ev_begin(kCompose);
    hipError_t e = launch_compose(c->w, !c->ran_first, c->next_round, d_labels, out64, false, nullptr, grid, c->stream);
    c->ev_end(ev);
    if (!c->hip_ok(e, "compose")) return CC_E_HIP;
    if (c->o.flags & CC_CANONICAL) {
        e = launch_canonical(c->w, d_labels, out64, false, nullptr, grid, c->stream);
        if (!c->hip_ok(e, "canonical labels")) return CC_E_HIP;
    }
    return CC_OK;
}

}  // namespace lc

namespace {

cc_status round_once(cc_ctx *c, cc_round_stats *out);
cc_status adopt_device_rounds(cc_ctx *c, int in_graph);

constexpr int kTailRounds = 8;                 // rounds per captured tail
constexpr int64_t kTailMaxRecords = 1 << 22;   // remaining graph small enough for a tail

int64_t pow2_ceil(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

constexpr size_t kTailCache = 6;               // captured tails kept per context

void drop_tails(cc_ctx *c) {
    for (auto &t : c->tails) (void)hipGraphExecDestroy(t.exec);
    c->tails.clear();
}

// A capture costs far more than a few small rounds: a context captures only once it has
// finished an earlier solve, i.e. when it is being reused.
bool tail_wanted(const cc_ctx *c) {
    return !(c->o.flags & (CC_EAGER | CC_EXPLICIT_PRIO | CC_RECORD_ROUNDS | CC_MERGE_TO_LARGE)) && c->o.max_rounds == 0 &&
           c->finish_edges == 0 && c->solves_done > 0 &&
           c->next_round >= 1 &&
           !c->done && c->m_cur > 0 && c->m_cur <= kTailMaxRecords;
}

// Capture kTailRounds rounds sized for (Nb, Mb) on a private stream.  The kernels read
// every count and the round's priority key from the device state, so the graph serves any
// solve whose remaining sizes round up to the same bounds and whose next round has the
// same parity (names and gids alternate between two buffers).
hipGraphExec_t capture_tail(cc_ctx *c, int64_t Nb, int64_t Mb) {
    if (!c->cap_stream && !c->hip_ok(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream"))
        return nullptr;
    hipStream_t user = c->stream;
    const bool prof = c->profile;
    c->stream = c->cap_stream;
    c->profile = false;   // no events inside a captured graph
    bool ok = c->hip_ok(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    PrioCtx pc{};
    for (int i = 0; ok && i < kTailRounds; ++i) ok = c->enqueue_round(c->next_round + i, Nb, Mb, pc);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    c->profile = prof;
    hipGraphExec_t exec = nullptr;
    if (ok) ok = c->hip_ok(e, "end capture");
    if (ok) ok = c->hip_ok(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "graph instantiate");
    if (g) (void)hipGraphDestroy(g);
    return ok ? exec : nullptr;
}

hipGraphExec_t tail_for(cc_ctx *c, int64_t Nb, int64_t Mb) {
    const int parity = c->next_round & 1;
    for (auto &t : c->tails) {
        if (t.N == Nb && t.M == Mb && t.parity == parity && t.ws == c->ws) {
            t.used = ++c->tail_clock;
            return t.exec;
        }
    }
    hipGraphExec_t exec = capture_tail(c, Nb, Mb);
    if (!exec) return nullptr;
    if (c->tails.size() >= kTailCache) {   // replace the least recently used
        size_t victim = 0;
        for (size_t i = 1; i < c->tails.size(); ++i)
            if (c->tails[i].used < c->tails[victim].used) victim = i;
        (void)hipGraphExecDestroy(c->tails[victim].exec);
        c->tails.erase(c->tails.begin() + (long)victim);
    }
    c->tails.push_back({exec, Nb, Mb, parity, c->ws, ++c->tail_clock});
    return exec;
}

// Up to kTailRounds rounds from one captured graph and one readback.
cc_status run_tail(cc_ctx *c) {
    const int64_t Nb = pow2_ceil(std::max<int64_t>(c->n_cur, 2));
    const int64_t Mb = pow2_ceil(std::max<int64_t>(c->m_cur, 2));
    const int64_t cap = std::max<int64_t>(c->g.n_vertices, 1);
    auto room = [&]() {
        return std::min<int64_t>((cap - c->host_map_used) / Nb, (int64_t)(kMaxLevels - c->host_levels));
    };
    if (room() < kTailRounds && !c->flatten()) return hip_status(c);
    if (room() < kTailRounds || c->next_round + kTailRounds > kStatRounds) return round_once(c, nullptr);
    hipGraphExec_t exec = tail_for(c, Nb, Mb);
    if (!exec) return hip_status(c);
    const bool ev = c->ev_begin(kTailGraph);
    const hipError_t e = hipGraphLaunch(exec, c->stream);
    c->ev_end(ev);
    if (!c->hip_ok(e, "graph launch")) return hip_status(c);
    if (!c->read_state()) return hip_status(c);
    return adopt_device_rounds(c, 1);
}

// Statistics of the rounds [c->next_round, st.rounds_active) that ran on the device without
// a readback of their own (a captured tail or the persistent launch), and the host's view of
// the state after them.
cc_status adopt_device_rounds(cc_ctx *c, int in_graph) {
    const RoundState &st = *c->h_st;
    if (st.err & 1u) return fail(c, CC_E_INPUT, "an edge record names a vertex outside [0, n_vertices)");
    if (st.err & ~1u) return fail(c, CC_E_STATE, "internal consistency check failed on the device");
    const int end = st.rounds_active;
    for (int r = c->next_round; r < end; ++r) {
        cc_round_stats s{};
        s.round = r;
        s.in_graph = in_graph;
        s.n_active = (int64_t)st.rstats[r][1];
        s.m_in = (int64_t)st.rstats[r][2];
        s.m_survive = (int64_t)st.rstats[r][3];
        s.m_out = (int64_t)st.rstats[r][4];
        s.n_finalised = (int64_t)st.rstats[r][5];
        s.m_sorted = (int64_t)st.rstats[r][6];
        c->stats.push_back(s);
    }
    c->rounds = end;
    c->next_round = end;
    c->last_graph_round = end - 1;
    c->host_levels = st.levels;
    c->host_map_used = (int64_t)st.map_off;
    c->n_cur = (int64_t)st.n_cur;
    c->m_cur = (int64_t)st.m_cur;
    c->done = st.m_cur == 0;
    return c->done ? CC_DONE : CC_OK;
}

bool fused_wanted(const cc_ctx *c) {
    return c->tail >= 2 && !c->fused_unavailable &&
           !(c->o.flags & (CC_EAGER | CC_EXPLICIT_PRIO | CC_RECORD_ROUNDS)) &&
           (c->o.max_rounds == 0 || c->next_round < c->o.max_rounds) && c->m_cur > c->finish_edges &&
           c->next_round >= 1 && c->next_round < kStatRounds &&
           !c->done && c->m_cur > 0 && c->m_cur <= kHashMaxRecords && 2 * c->m_cur + 1 <= c->w.kcap;
}

// The remaining small rounds in one persistent launch and one readback.  Its rounds end when
// the graph is empty or the next round does not fit the launch (then the loop of cc_run goes
// on with the other paths); a device that cannot keep the grid resident turns the launch off
// for this context.
cc_status run_fused(cc_ctx *c) {
    const int64_t cap = std::max<int64_t>(c->g.n_vertices, 1);
    // room for the next round's map (with MergeToLarge, a LocalContraction step's and its
    // step's; no fold between the two, so none before a step)
    const bool mtl = (c->o.flags & CC_MERGE_TO_LARGE) != 0;
    const int levels = mtl ? ((c->next_round & 1) ? 0 : 2) : 1;
    if (levels && (c->host_levels + levels > kMaxLevels || c->host_map_used + levels * c->n_cur > cap) &&
        !c->flatten())
        return hip_status(c);
    const int rule = mtl                       ? kFusedMerge
                     : c->variant == kVarTree   ? kFusedTree
                     : c->variant == kVarOneHop ? kFusedOneHop
                                                : kFusedLocal;
    const int grid = fused_rounds_grid(rule, 1 << (c->tail - 2), c->cus);
    if (grid <= 0) {
        c->fused_unavailable = true;
        return round_once(c, nullptr);
    }
    const int before = c->next_round;
    const bool ev = c->ev_begin(kFusedRounds);
    FusedLimits lim{};
    lim.round_limit = c->o.max_rounds > 0 ? c->o.max_rounds : kStatRounds;
    lim.finish_edges = c->finish_edges;
    if (mtl) {   // the phases' alphas; phases past what the launch carries are left to the host
        const size_t na = c->mtl_alphas.size();
        lim.n_alphas = (int32_t)std::min<size_t>(na, kFusedAlphas);
        for (int i = 0; i < lim.n_alphas; ++i) lim.alphas[i] = (uint64_t)c->mtl_alphas[(size_t)i];
        if (na > (size_t)kFusedAlphas) lim.round_limit = std::min(lim.round_limit, 2 * kFusedAlphas);
    }
    const hipError_t e = launch_fused_rounds(c->w, rule, grid, lim, c->stream);
    c->ev_end(ev);
    if (e == hipErrorCooperativeLaunchTooLarge) {   // the runtime disagrees with the occupancy query
        (void)hipGetLastError();
        c->fused_unavailable = true;
        return round_once(c, nullptr);
    }
    if (!c->hip_ok(e, "persistent rounds")) return hip_status(c);
    if (!c->read_state()) return hip_status(c);
    const cc_status s = adopt_device_rounds(c, 2);
    if (s == CC_OK && c->next_round == before) return round_once(c, nullptr);   // nothing fitted
    return s;
}

// one round, synchronously; returns CC_OK, CC_DONE or an error
cc_status round_once(cc_ctx *c, cc_round_stats *out) {
    int launched = 0;
    cc_status s = ctx_round_enqueue(c, &launched);
    if (!launched) return s;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return hip_status(c);
    return ctx_round_complete(c, out);
}

bool finish_wanted(const cc_ctx *c) {
    return c->finish_edges > 0 && c->next_round >= 1 && !c->done && c->m_cur > 0 && c->m_cur <= c->finish_edges;
}

// The union-find finish of the current graph (Section 6); ends the solve.
cc_status run_finish(cc_ctx *c) {
    if (c->failed_status) return c->failed_status;
    const int r = c->next_round;
    const int64_t N = c->n_cur, M = c->m_cur;
    if (c->host_levels >= kMaxLevels || c->host_map_used + N > std::max<int64_t>(c->g.n_vertices, 1)) {
        if (!c->flatten()) return hip_status(c);
    }
    const bool ev = c->ev_begin(kUfFinish);
    const hipError_t e = launch_uf_finish(c->w, r, c->grid_for(N), c->grid_for(ceil_div(M, 2)), c->stream);
    c->ev_end(ev);
    if (!c->hip_ok(e, "union-find finish")) return hip_status(c);
    if (!c->read_state()) return hip_status(c);
    const RoundState &st = *c->h_st;
    if (st.err & ~1u) return fail(c, CC_E_STATE, "internal consistency check failed on the device");
    c->host_levels += 1;
    c->host_map_used += N;
    c->n_cur = 0;
    c->m_cur = 0;
    c->done = true;
    c->finished = true;
    return CC_DONE;
}

// Pinned host mirrors of the round state, kept for reuse by later contexts.  Freeing pinned
// memory synchronises the whole device (hipHostFree waits for all work on it), so a context
// that ends while others still run must not free its mirror; it returns it here instead.  The
// pool holds at most as many mirrors (a few KB each) as contexts ever existed at once.
std::mutex g_mirror_mu;
std::vector<RoundState *> g_mirrors;

RoundState *mirror_take() {
    {
        std::lock_guard<std::mutex> lk(g_mirror_mu);
        if (!g_mirrors.empty()) {
            RoundState *m = g_mirrors.back();
            g_mirrors.pop_back();
            return m;
        }
    }
    RoundState *m = nullptr;
    if (hipHostMalloc((void **)&m, sizeof(RoundState), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return m;
}

void mirror_give(RoundState *m) {
    std::lock_guard<std::mutex> lk(g_mirror_mu);
    g_mirrors.push_back(m);
}

}  // namespace

namespace lc {

cc_status ctx_create(const cc_graph_desc *graph, const cc_options *opts, RoundState *mirror, cc_ctx **out) {
    if (!out) return CC_E_ARG;
    *out = nullptr;
    if (!graph || !opts) return CC_E_ARG;
    const cc_graph_desc &g = *graph;
    if (g.n_vertices < 0 || g.n_vertices > 0x7FFFFFFFLL || g.n_edges < 0 || g.n_edges > 0xFFFFFFFELL) return CC_E_ARG;
    if (g.layout < CC_EDGES_SOA_I32 || g.layout > CC_EDGES_PACKED_U64 || g.reserved != 0) return CC_E_ARG;
    if (g.n_edges > 0 && (!g.src || (g.layout != CC_EDGES_PACKED_U64 && !g.dst))) return CC_E_ARG;
    if (opts->max_rounds < 0) return CC_E_ARG;
    if ((opts->flags & CC_ROUND0_DIRECT) && (opts->flags & CC_ROUND0_TILED)) return CC_E_ARG;
    if ((opts->flags & CC_ROUND0_TILED) && g.n_vertices > 0 && !tiled_fits(g.n_vertices)) return CC_E_ARG;
    if ((opts->flags & CC_TREE) && (opts->flags & CC_ONE_HOP)) return CC_E_ARG;
    if ((opts->flags & CC_EXPLICIT_PRIO) && (opts->flags & CC_ROUND0_TILED)) return CC_E_ARG;
    if ((opts->flags & CC_MERGE_TO_LARGE) && (opts->flags & (CC_TREE | CC_ONE_HOP))) return CC_E_ARG;
    cc_ctx *c = new (std::nothrow) cc_ctx();
    if (!c) return CC_E_NOMEM;
    c->g = g;
    c->o = *opts;
    c->stream = (hipStream_t)opts->stream;
    c->profile = (opts->flags & CC_PROFILE) != 0;
    c->batch = false;
    c->in.s = g.src;
    c->in.d = g.dst;
    c->in.m = g.n_edges;
    c->in.n = (uint32_t)g.n_vertices;
    c->in.layout = g.layout == CC_EDGES_SOA_I32 ? kSoa32 : g.layout == CC_EDGES_SOA_I64 ? kSoa64 : kPacked;
    const bool aligned = ((uintptr_t)g.src % 16 == 0) && (g.layout == CC_EDGES_PACKED_U64 || (uintptr_t)g.dst % 16 == 0);
    c->in.vec = aligned ? 1 : 0;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    c->cus = std::max(cus, 1);
    c->grid_cap = c->cus * 8;
    if (mirror) {
        c->h_st = mirror;
        c->h_st_borrowed = true;
    } else if ((c->h_st = mirror_take()) != nullptr) {
        c->h_st_pooled = true;
    } else {
        // no usable device yet: a pageable mirror still works for every later copy
        c->h_st = (RoundState *)calloc(1, sizeof(RoundState));
        c->h_st_pageable = true;
        if (!c->h_st) {
            delete c;
            return CC_E_NOMEM;
        }
    }
    c->tiled = !(opts->flags & CC_EXPLICIT_PRIO) && choose_tiled(g.n_vertices, g.n_edges, opts->flags);
    c->variant = (opts->flags & CC_TREE) ? kVarTree : (opts->flags & CC_ONE_HOP) ? kVarOneHop : kVarLocal;
    c->tp = tiled_plan(g.n_vertices, g.n_edges);
    c->ws_need = plan_workspace(g.n_vertices, g.n_edges, false, c->tiled, nullptr, nullptr, ws_extras(opts->flags));
    {   // default MergeToLarge parameter: max(2, ceil(ln n))
        int64_t a = 2;
        while ((double)a < std::log((double)std::max<int64_t>(g.n_vertices, 2))) ++a;
        c->mtl_alphas.assign(1, a);
    }
    *out = c;
    return CC_OK;
}

}  // namespace lc

extern "C" {

cc_status cc_create(const cc_graph_desc *graph, const cc_options *opts, cc_ctx **out) {
    return lc::ctx_create(graph, opts, nullptr, out);
}

cc_status cc_workspace_size(const cc_ctx *c, size_t *bytes) {
    if (!c || !bytes) return CC_E_ARG;
    *bytes = c->ws_need;
    return CC_OK;
}

cc_status cc_set_workspace(cc_ctx *c, void *d_ws, size_t bytes) {
    if (!c || !d_ws) return CC_E_ARG;
    if (bytes < c->ws_need) return reject(c, CC_E_NOMEM, "workspace smaller than cc_workspace_size()");
    if ((uintptr_t)d_ws % 256 != 0) return reject(c, CC_E_ARG, "workspace must be 256-byte aligned");
    c->ws = d_ws;
    c->ws_bytes = bytes;
    plan_workspace(c->g.n_vertices, c->g.n_edges, false, c->tiled, (char *)d_ws, &c->w, ws_extras(c->o.flags));
    c->w.round0_sets_off = c->round0_sets_off ? 1 : 0;
    drop_tails(c);   // captured tails hold pointers into the previous workspace
    return reset_solve(c, c->o.seed);
}

cc_status cc_set_tuning(cc_ctx *c, const cc_tuning *t) {
    if (!c || !t) return CC_E_ARG;
    auto one_of = [](int v, int a, int b, int d) { return v == 0 || v == a || v == b || v == d; };
    if (t->round0 < 0 || t->round0 > 3 || t->blocks_per_cu < 0 || t->blocks_per_cu > 64 ||
        (t->round0_key_sets != 0 && t->round0_key_sets != 1) || !one_of(t->scatter_waves, 2, 3, 4) ||
        !one_of(t->row_pairs, 2, 4, 8) || !one_of(t->relabel_pairs, 1, 2, 4) || t->row_generation < -1 ||
        t->row_generation > 8 || t->round0_sort < 0 || t->round0_sort > 2 || t->tail < 0 || t->tail > 4 ||
        t->radix_form < 0 || t->radix_form > 2)
        return reject(c, CC_E_ARG, "tuning value out of range");
    const bool tiled = t->round0 == 0 ? c->tiled : t->round0 >= 2;
    const bool rows = t->round0 == 0 ? c->tiled_rows : t->round0 == 3;
    if (tiled && (!tiled_fits(c->g.n_vertices) || (c->o.flags & CC_EXPLICIT_PRIO)))
        return reject(c, CC_E_ARG, "the tiled round 0 does not apply to this context");
    const size_t need =
        plan_workspace(c->g.n_vertices, c->g.n_edges, false, tiled, nullptr, nullptr, ws_extras(c->o.flags));
    if (c->ws && c->ws_bytes < need) return reject(c, CC_E_NOMEM, "the workspace is too small for that round-0 form");
    c->tiled = tiled;
    c->tiled_rows = tiled && rows;
    c->ws_need = need;
    c->blocks_per_cu = t->blocks_per_cu ? t->blocks_per_cu : 8;
    c->grid_cap = c->cus * c->blocks_per_cu;
    c->round0_sets_off = t->round0_key_sets == 0;
    c->scatter_waves = t->scatter_waves ? t->scatter_waves : LC_SCATTER_WAVES;
    c->row_pairs = t->row_pairs ? t->row_pairs : LC_TMIN2_PAIRS;
    c->relabel_pairs = t->relabel_pairs ? t->relabel_pairs : LC_TRELABEL_PAIRS;
    c->row_generation = t->row_generation ? t->row_generation : 1;
    c->round0_sort = t->round0_sort ? t->round0_sort : 1;
    c->tail = t->tail ? t->tail : 1;
    c->radix_form = t->radix_form ? t->radix_form : 1;
    drop_tails(c);   // captured with the previous grid sizes and layout
    if (!c->ws) return CC_OK;
    plan_workspace(c->g.n_vertices, c->g.n_edges, false, c->tiled, (char *)c->ws, &c->w, ws_extras(c->o.flags));
    c->w.round0_sets_off = c->round0_sets_off ? 1 : 0;
    return reset_solve(c, c->o.seed);
}

cc_status cc_get_tuning(const cc_ctx *c, cc_tuning *t) {
    if (!c || !t) return CC_E_ARG;
    t->round0 = c->tiled ? (c->tiled_rows ? 3 : 2) : 1;
    t->blocks_per_cu = c->blocks_per_cu;
    t->round0_key_sets = c->round0_sets_off ? 0 : 1;
    t->scatter_waves = c->scatter_waves;
    t->row_pairs = c->row_pairs;
    t->relabel_pairs = c->relabel_pairs;
    t->row_generation = c->row_generation;
    t->round0_sort = c->round0_sort;
    t->tail = c->tail;
    t->radix_form = c->radix_form;
    return CC_OK;
}

cc_status cc_reset(cc_ctx *c, uint64_t seed) {
    if (!c) return CC_E_ARG;
    if (!c->ws) return reject(c, CC_E_NOMEM, "no workspace: call cc_set_workspace first");
    return reset_solve(c, seed);
}

cc_status cc_contract_round(cc_ctx *c, cc_round_stats *out) {
    if (!c) return CC_E_ARG;
    cc_status s = round_once(c, out);
    if (s == CC_DONE) c->labels_ready = true;
    return s;
}

cc_status cc_run(cc_ctx *c, int32_t *rounds) {
    if (!c) return CC_E_ARG;
    for (;;) {
        if (c->o.max_rounds > 0 && c->next_round >= c->o.max_rounds) break;
        cc_status s = finish_wanted(c)  ? run_finish(c)
                      : fused_wanted(c) ? run_fused(c)
                      : tail_wanted(c)  ? run_tail(c)
                                        : round_once(c, nullptr);
        if (s == CC_DONE) break;
        if (s != CC_OK) return s;
    }
    if (c->failed_status) return c->failed_status;
    c->labels_ready = true;
    c->solves_done += 1;
    if (rounds) *rounds = c->rounds;
    return CC_OK;
}

cc_status cc_labels(cc_ctx *c, void *d_labels) {
    if (!c || !d_labels) return CC_E_ARG;
    if (c->failed_status) return c->failed_status;
    if (!c->labels_ready) return reject(c, CC_E_STATE, "labels requested before cc_run or CC_DONE");
    return ctx_labels_enqueue(c, d_labels);
}

cc_status cc_round_parents(cc_ctx *c, int32_t r, int32_t *d_parents, int64_t *n_nodes) {
    if (!c || !d_parents) return CC_E_ARG;
    if (c->failed_status) return c->failed_status;
    if (!c->ran_first || c->next_round == 0) return reject(c, CC_E_STATE, "no round has run");
    const int last = c->next_round - 1;
    if (r < 0) r = last;
    if (r > last) return reject(c, CC_E_STATE, "that round has not run");
    const int grid = c->grid_for(c->g.n_vertices);
    hipError_t e;
    if (r < (int)c->recs.size() && c->recs[r].off >= 0) {   // recorded (CC_RECORD_ROUNDS)
        e = launch_expand_record(c->w, r, c->w.rec + c->recs[r].off, c->recs[r].count, d_parents, grid, c->stream);
    } else {
        if (r != last) return reject(c, CC_E_STATE, "only the most recent round is kept (use CC_RECORD_ROUNDS)");
        if (last == c->last_graph_round)
            return reject(c, CC_E_STATE, "the last round ran inside a captured tail (use CC_EAGER)");
        if (c->finished) return reject(c, CC_E_STATE, "the solve ended with the union-find finish");
        e = launch_dump_parents(c->w, d_parents, last, grid, c->stream);
    }
    if (!c->hip_ok(e, "dump parents")) return CC_E_HIP;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return CC_E_HIP;
    if (n_nodes) *n_nodes = r < (int)c->stats.size() ? c->stats[r].n_active : 0;
    return CC_OK;
}

cc_status cc_debug_round_arrays(cc_ctx *c, uint32_t *d_m1, uint32_t *d_l) {
    if (!c || !d_m1 || !d_l) return CC_E_ARG;
    if (c->failed_status) return c->failed_status;
    if (c->variant != kVarLocal) return reject(c, CC_E_STATE, "the minima are kept for LocalContraction only");
    if (!c->ran_first || c->next_round == 0) return reject(c, CC_E_STATE, "no round has run");
    const int last = c->next_round - 1;
    if ((c->o.flags & CC_MERGE_TO_LARGE) && (last & 1))
        return reject(c, CC_E_STATE, "the last round was a MergeToLarge step (no minima)");
    if (last == c->last_graph_round)
        return reject(c, CC_E_STATE, "the last round ran inside a captured tail (use CC_EAGER)");
    if (c->finished) return reject(c, CC_E_STATE, "the solve ended with the union-find finish");
    PrioCtx pc{};
    pc.tab = table_for(c, last);
    pc.inv = c->w.pinv;
    hipError_t e = launch_dump_minima(c->w, last, last == 0 && c->tiled, pc, d_m1, d_l, c->grid_for(c->g.n_vertices),
                                      c->stream);
    if (!c->hip_ok(e, "dump minima")) return CC_E_HIP;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return CC_E_HIP;
    return CC_OK;
}

cc_status cc_set_merge_to_large(cc_ctx *c, const int64_t *h_alphas, int32_t count) {
    if (!c || !h_alphas || count < 1) return CC_E_ARG;
    if (!(c->o.flags & CC_MERGE_TO_LARGE)) return reject(c, CC_E_STATE, "the context was created without CC_MERGE_TO_LARGE");
    for (int32_t i = 0; i < count; ++i)
        if (h_alphas[i] < 1 || h_alphas[i] > 0xFFFFFFFFLL) return reject(c, CC_E_ARG, "alpha must be in [1, 2^32 - 1]");
    c->mtl_alphas.assign(h_alphas, h_alphas + count);
    return CC_OK;
}

cc_status cc_set_explicit_priorities(cc_ctx *c, int32_t r, const uint32_t *d_prio) {
    if (!c || r < 0 || !d_prio) return CC_E_ARG;
    if (!(c->o.flags & CC_EXPLICIT_PRIO)) return reject(c, CC_E_STATE, "the context was created without CC_EXPLICIT_PRIO");
    bool replaced = false;
    for (auto &e : c->prio_tabs)
        if (e.first == r) {
            e.second = d_prio;
            replaced = true;
        }
    if (!replaced) c->prio_tabs.push_back({r, d_prio});
    c->inv_for = nullptr;   // the next round rebuilds the inverse of its table
    return CC_OK;
}

cc_status cc_round_edges(cc_ctx *c, uint64_t *d_edges, int64_t cap, int64_t *n_edges) {
    if (!c || !n_edges) return CC_E_ARG;
    if (c->failed_status) return c->failed_status;
    if (!c->ran_first || c->next_round == 0) return reject(c, CC_E_STATE, "no round has run");
    if (c->next_round - 1 == c->last_graph_round)
        return reject(c, CC_E_STATE, "the last round ran inside a captured tail (use CC_EAGER)");
    if (c->finished) return reject(c, CC_E_STATE, "the solve ended with the union-find finish");
    const int64_t m = c->m_cur;   // records of the graph the last round left (its readback)
    *n_edges = m;
    if (m == 0 || !d_edges) return CC_OK;   // no edge left, or the count only
    if (cap < m) return reject(c, CC_E_ARG, "edge buffer smaller than the edge count");
    hipError_t e = launch_dump_edges(c->w, d_edges, c->next_round, c->grid_for(m), c->stream);
    if (!c->hip_ok(e, "dump edges")) return CC_E_HIP;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return CC_E_HIP;
    return CC_OK;
}

cc_status cc_get_round_stats(const cc_ctx *c, int32_t r, cc_round_stats *out) {
    if (!c || !out || r < 0 || r >= (int32_t)c->stats.size()) return CC_E_ARG;
    *out = c->stats[r];
    return CC_OK;
}

int32_t cc_kernel_family_count(void) { return kFamilies; }

const char *cc_kernel_family_name(int32_t i) { return (i >= 0 && i < kFamilies) ? kFamilyNames[i] : nullptr; }

cc_status cc_set_finish(cc_ctx *c, int64_t max_edges) {
    if (!c || max_edges < 0) return CC_E_ARG;
    c->finish_edges = max_edges;
    return CC_OK;
}

cc_status cc_get_finished(const cc_ctx *c, int32_t *finished) {
    if (!c || !finished) return CC_E_ARG;
    *finished = c->finished ? 1 : 0;
    return CC_OK;
}

cc_status cc_set_profile_mask(cc_ctx *c, uint64_t family_mask) {
    if (!c) return CC_E_ARG;
    c->prof_mask = family_mask;
    return CC_OK;
}

cc_status cc_kernel_times(const cc_ctx *c, double *ms, int64_t *launches, int32_t cap) {
    if (!c) return CC_E_ARG;
    for (int i = 0; i < kFamilies && i < cap; ++i) {
        if (ms) ms[i] = c->fam_ms[i];
        if (launches) launches[i] = c->fam_launches[i];
    }
    return CC_OK;
}

// ---- round checkpoints --------------------------------------------------------------------
//
// Layout: CkptHeader, then the statistics so far, the device round state, the current edge
// records (8 bytes each, in the buffer the state names), the names of the current nodes, the
// name -> index array, map0 and the used part of the map arena.  Between rounds nothing else
// on the device is read by a later round.

namespace {

constexpr uint64_t kCkptMagic = 0x31304B43504B434CULL;   // "LCKPCK01"
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    uint64_t magic;
    uint32_t version, rule;   // rule: CC_TREE | CC_ONE_HOP bits of the context
    int64_t n0, m0;
    int32_t layout, next_round, rounds, ran_first;
    int32_t done, host_levels, finished, n_stats;
    int64_t host_map_used, n_cur, m_cur, map_used;
    uint64_t seed;
    int32_t e_sel, state_bytes;
    int64_t total_bytes;
};

struct CkptSizes {
    size_t stats, state, edges, names, idx, map0, maps, mtl, total;
};

CkptSizes ckpt_sizes(int64_t n0, int n_stats, int64_t m_cur, int64_t n_cur, int64_t map_used, bool mtl) {
    CkptSizes z{};
    z.mtl = mtl ? 4 * (size_t)n_cur : 0;
    z.stats = sizeof(cc_round_stats) * (size_t)n_stats;
    z.state = sizeof(RoundState);
    z.edges = 8 * (size_t)m_cur;
    z.names = 4 * (size_t)n_cur;
    z.idx = 4 * (size_t)n0;
    z.map0 = 4 * (size_t)n0;
    z.maps = 4 * (size_t)map_used;
    z.total = sizeof(CkptHeader) + z.stats + z.state + z.edges + z.names + z.idx + z.map0 + z.maps + 2 * z.mtl;
    return z;
}

uint32_t rule_bits(uint32_t flags) { return flags & (CC_TREE | CC_ONE_HOP | CC_MERGE_TO_LARGE); }

// After a LocalContraction step of a MergeToLarge solve, the sizes and priorities of the next
// graph's classes are part of the state (the step reads them).
bool ckpt_has_mtl(uint32_t flags, int32_t next_round) { return (flags & CC_MERGE_TO_LARGE) && (next_round & 1); }

}  // namespace

cc_status cc_save_state(cc_ctx *c, void *h_buf, size_t *bytes) {
    if (!c || !bytes) return CC_E_ARG;
    if (c->failed_status) return reject(c, CC_E_STATE, "the solve has failed");
    if (!c->ws) return reject(c, CC_E_NOMEM, "no workspace: call cc_set_workspace first");
    RoundState st;
    if (!c->hip_ok(hipMemcpyAsync(&st, c->w.st, sizeof st, hipMemcpyDeviceToHost, c->stream), "state readback") ||
        !c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize"))
        return CC_E_HIP;
    const int64_t n0 = c->g.n_vertices;
    const int64_t m_cur = c->next_round == 0 ? 0 : (int64_t)st.m_cur;
    const int64_t n_cur = c->next_round == 0 ? 0 : (int64_t)st.n_cur;
    const int64_t map_used = (int64_t)st.map_off;
    const CkptSizes z = ckpt_sizes(n0, (int)c->stats.size(), m_cur, n_cur, map_used, ckpt_has_mtl(c->o.flags, c->next_round));
    if (!h_buf) {
        *bytes = z.total;
        return CC_OK;
    }
    if (*bytes < z.total) return reject(c, CC_E_ARG, "checkpoint buffer smaller than the size cc_save_state reports");
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.version = kCkptVersion;
    h.rule = rule_bits(c->o.flags);
    h.n0 = n0;
    h.m0 = c->g.n_edges;
    h.layout = c->g.layout;
    h.next_round = c->next_round;
    h.rounds = c->rounds;
    h.ran_first = c->ran_first ? 1 : 0;
    h.done = c->done ? 1 : 0;
    h.host_levels = c->host_levels;
    h.finished = c->finished ? 1 : 0;
    h.n_stats = (int32_t)c->stats.size();
    h.host_map_used = c->host_map_used;
    h.n_cur = c->n_cur;
    h.m_cur = c->m_cur;
    h.map_used = map_used;
    h.seed = c->o.seed;
    h.e_sel = st.e_sel;
    h.state_bytes = (int32_t)sizeof(RoundState);
    h.total_bytes = (int64_t)z.total;
    char *p = (char *)h_buf;
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    if (z.stats) memcpy(p, c->stats.data(), z.stats);
    p += z.stats;
    memcpy(p, &st, z.state);
    p += z.state;
    struct Piece {
        const void *src;
        size_t n;
    } pieces[] = {{c->w.keys[st.e_sel & 1], z.edges},
                  {c->w.names[c->next_round & 1], z.names},
                  {c->w.idx_of, z.idx},
                  {c->w.map0, z.map0},
                  {c->w.maps, z.maps},
                  {c->w.mtl_size, z.mtl},
                  {c->w.mtl_v, z.mtl}};
    for (const Piece &q : pieces) {
        if (q.n && !c->hip_ok(hipMemcpyAsync(p, q.src, q.n, hipMemcpyDeviceToHost, c->stream), "checkpoint copy"))
            return CC_E_HIP;
        p += q.n;
    }
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return CC_E_HIP;
    *bytes = z.total;
    return CC_OK;
}

cc_status cc_load_state(cc_ctx *c, const void *h_buf, size_t bytes) {
    if (!c || !h_buf) return CC_E_ARG;
    if (!c->ws) return reject(c, CC_E_NOMEM, "no workspace: call cc_set_workspace first");
    CkptHeader h;
    if (bytes < sizeof h) return reject(c, CC_E_ARG, "not a checkpoint");
    memcpy(&h, h_buf, sizeof h);
    if (h.magic != kCkptMagic || h.version != kCkptVersion || h.state_bytes != (int32_t)sizeof(RoundState))
        return reject(c, CC_E_ARG, "not a checkpoint of this library version");
    if (h.n0 != c->g.n_vertices || h.m0 != c->g.n_edges || h.layout != c->g.layout || h.rule != rule_bits(c->o.flags))
        return reject(c, CC_E_ARG, "the checkpoint belongs to another graph or label rule");
    const int64_t n0 = c->g.n_vertices;
    const int64_t m_cur = h.next_round == 0 ? 0 : h.m_cur, n_cur = h.next_round == 0 ? 0 : h.n_cur;
    if (h.n_stats < 0 || h.n_stats > kStatRounds || h.next_round < 0 || h.rounds < 0 || h.rounds > h.next_round ||
        m_cur < 0 || m_cur > c->w.kcap || n_cur < 0 || n_cur > n0 || h.map_used < 0 || h.map_used > std::max<int64_t>(n0, 1) ||
        h.e_sel < 0 || h.e_sel > 1 || h.host_levels < 0 || h.host_levels > kMaxLevels)
        return reject(c, CC_E_ARG, "inconsistent checkpoint");
    const CkptSizes z = ckpt_sizes(n0, h.n_stats, m_cur, n_cur, h.map_used, ckpt_has_mtl(h.rule, h.next_round));
    if ((int64_t)z.total != h.total_bytes || bytes < z.total) return reject(c, CC_E_ARG, "truncated checkpoint");
    const char *p = (const char *)h_buf + sizeof h;
    std::vector<cc_round_stats> stats((size_t)h.n_stats);
    if (z.stats) memcpy(stats.data(), p, z.stats);
    p += z.stats;
    RoundState st;
    memcpy(&st, p, z.state);
    p += z.state;
    // The device state must agree with the header and keep later rounds inside the workspace:
    // they index the edge buffers, the names and the map arena with these fields.
    bool consistent = st.e_sel == h.e_sel && (int64_t)st.map_off == h.map_used && st.levels >= 0 &&
                      st.levels <= kMaxLevels && (int64_t)st.map_cap == std::max<int64_t>(n0, 1);
    if (h.next_round > 0) consistent = consistent && (int64_t)st.m_cur == m_cur && (int64_t)st.n_cur == n_cur;
    for (int l = 0; consistent && l < st.levels; ++l) consistent = (int64_t)st.level_off[l] <= h.map_used;
    if (!consistent) return reject(c, CC_E_ARG, "inconsistent checkpoint");
    // every copy below is ordered before the next round on the stream; the host buffer is
    // read before this call returns (synchronised)
    struct Piece {
        void *dst;
        const void *src;
        size_t n;
    } pieces[] = {{c->w.st, &st, z.state},
                  {c->w.keys[h.e_sel], nullptr, z.edges},
                  {c->w.names[h.next_round & 1], nullptr, z.names},
                  {c->w.idx_of, nullptr, z.idx},
                  {c->w.map0, nullptr, z.map0},
                  {c->w.maps, nullptr, z.maps},
                  {c->w.mtl_size, nullptr, z.mtl},
                  {c->w.mtl_v, nullptr, z.mtl}};
    for (Piece &q : pieces) {
        const void *src = q.src ? q.src : (const void *)p;
        if (q.n && !c->hip_ok(hipMemcpyAsync(q.dst, src, q.n, hipMemcpyHostToDevice, c->stream), "checkpoint copy"))
            return fail(c, CC_E_HIP, "checkpoint copy failed");
        if (!q.src) p += q.n;
    }
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "stream synchronize")) return fail(c, CC_E_HIP, "checkpoint copy failed");
    memcpy(c->h_st, &st, sizeof st);
    c->o.seed = h.seed;
    c->stats = std::move(stats);
    c->rounds = h.rounds;
    c->next_round = h.next_round;
    c->ran_first = h.ran_first != 0;
    c->done = h.done != 0;
    c->labels_ready = c->done;
    c->finished = h.finished != 0;
    c->host_levels = h.host_levels;
    c->host_map_used = h.host_map_used;
    c->n_cur = h.n_cur;
    c->m_cur = h.m_cur;
    c->last_graph_round = -1;
    c->failed_status = 0;
    c->err.clear();
    c->recs.clear();
    c->rec_used = 0;
    c->inv_for = nullptr;
    for (int i = 0; i < kFamilies; ++i) {
        c->fam_ms[i] = 0.0;
        c->fam_launches[i] = 0;
    }
    return CC_OK;
}

cc_status cc_destroy(cc_ctx *c) {
    if (!c) return CC_E_ARG;
    (void)hipStreamSynchronize(c->stream);
    for (auto e : c->events) (void)hipEventDestroy(e);
    drop_tails(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_st_pooled)
        mirror_give(c->h_st);   // the stream is idle: no copy to or from it is pending
    else if (c->h_st_pageable)
        free(c->h_st);
    delete c;
    return CC_OK;
}

const char *cc_last_error(const cc_ctx *c) { return c ? c->err.c_str() : "null context"; }

const char *cc_version(void) { return "lc-mi355x 0.1 (gfx950)"; }

}  // extern "C"
