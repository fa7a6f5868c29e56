// Host round engine shared by the plain solve and the batched solve.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "cc.h"
#include "lc_internal.hpp"

namespace lc {

enum Family {
    kRoundBegin = 0, kMin1In, kMin1, kMin2In, kMin2, kParent, kLabelRanks, kRelabelIn, kRelabel, kSortHist,
    kSortScan, kSortScatter, kUnique, kNodeScan, kNodes, kMap, kRoundEnd, kCompose, kFlatten,
    kPartAHist, kPartAScatter, kPartBHist, kPartBScatter, kPartScan, kMin1Tiled, kMin2Tiled, kRelabelTiled,
    kTailGraph, kUfFinish, kHashDedup, kMergeLarge, kPartRowsHist, kPartRowsScatter, kBucketSort, kFusedRounds, kFamilies
};

// how a round chooses its labels (cc_options.flags CC_TREE, CC_ONE_HOP)
enum Variant { kVarLocal = 0, kVarTree = 1, kVarOneHop = 2 };
extern const char *const kFamilyNames[kFamilies];

// Lays the workspace out from `base` (or only sizes it when base is null).  `tiled`: round 0
// runs over the tiled record layout, whose two key buffers hold twice the input records.
// `extras`: kWsExplicit adds the inverse of an explicit priority table, kWsRecord the round
// record area (CC_EXPLICIT_PRIO, CC_RECORD_ROUNDS).
enum { kWsExplicit = 1, kWsRecord = 2, kWsMerge = 4 };
constexpr int64_t kRecordPerVertex = 5;   // 4-byte record entries per vertex (20 bytes)
size_t plan_workspace(int64_t n0, int64_t m0, bool batch, bool tiled, char *base, Work *w, uint32_t extras = 0);
// Guard gaps for bounds-checking builds.  A host build of the library under AddressSanitizer
// (device memory is then host memory) sets LC_WS_GUARD to a multiple of 256: every buffer
// carved from a workspace is followed by that many bytes, marked as not addressable together
// with the buffer's alignment slack, so that an access past a buffer's declared size is
// reported where it happens instead of landing in the next buffer.  GPU builds keep 0.
#ifndef LC_WS_GUARD
#define LC_WS_GUARD 0
#endif
static_assert(LC_WS_GUARD % 256 == 0, "guard gaps keep the 256-byte alignment of workspace buffers");
// Marks [p, p + bytes) addressable and the `gap` bytes after it not (bounds-checking builds
// only; otherwise nothing).
void ws_mark(char *p, size_t bytes, size_t gap);
// Whether a plain solve of this size with these cc_options flags runs round 0 tiled.
bool choose_tiled(int64_t n0, int64_t m0, uint32_t flags);
int ceil_log2_host(int64_t n);

struct Engine {
    hipStream_t stream = nullptr;
    Work w{};
    EdgeIn in{};
    bool batch = false;
    bool tiled = false;           // round 0 over the tiled record layout
    bool tiled_rows = false;      // ... partitioned by row in one pass (no column order in a row)
    int variant = kVarLocal;
    TPlan tp{};
    bool profile = false;
    uint64_t prof_mask = ~0ull;   // families timed under CC_PROFILE (bit i: family i)
    bool done = false;
    int grid_cap = 2048;          // workgroups of the grid-stride kernels (CUs x blocks per CU)
    int cus = 256;                // compute units (row generations, resident scatter grid)
    int blocks_per_cu = 8;        // tuning: grid_cap = cus * blocks_per_cu
    bool round0_sets_off = false; // tuning: round 0's relabel without key sets
    int scatter_waves = LC_SCATTER_WAVES;  // tuning: radix scatter build (waves per SIMD)
    int row_pairs = LC_TMIN2_PAIRS;        // tuning: tiled two-hop pass, record pairs per thread
    int relabel_pairs = LC_TRELABEL_PAIRS; // tuning: tiled relabel, record pairs per thread
    int row_generation = 1;                // tuning: gathering row passes, rows per CU a launch (-1 all)
    int round0_sort = 1;                   // tuning: round 0's duplicate drop, 1 radix passes, 2 sampled buckets
    int tail = 1;                          // tuning: small rounds, 1 a launch sequence each, 2..4 one
                                           // persistent launch of 1 << (tail - 2) workgroups per CU
    int radix_form = 1;                    // tuning: radix passes, 1 count/scan/scatter a digit, 2 one sweep
    void *ws = nullptr;
    size_t ws_bytes = 0, ws_need = 0;
    RoundState *h_st = nullptr;   // pinned host mirror of the device round state
    bool h_st_pageable = false;
    bool h_st_borrowed = false;   // the mirror belongs to the caller (a server slot)
    bool h_st_pooled = false;     // the mirror returns to the library's pool on destroy
    // batch of independent graphs (union path)
    RoundKey *d_keys = nullptr;         // [G] per-graph round keys (device)
    const uint64_t *d_seeds = nullptr;  // [G] per-graph seeds (device)
    const uint32_t *d_voff = nullptr;   // [G+1] first union id of each graph (device)
    int32_t n_graphs = 0;
    // MergeToLarge: 0 off; 1 this round is a LocalContraction step whose next-round classes
    // get their sizes and priorities; 2 this round is the MergeToLarge step
    int mtl_mode = 0;
    uint64_t mtl_alpha = 0;
    int host_levels = 0;          // per-round maps currently kept in the arena
    int64_t host_map_used = 0;
    std::string err;
    int failed_status = 0;

    // kernel timing (CC_PROFILE)
    std::vector<hipEvent_t> events;
    std::vector<std::pair<int, int>> pending;
    int ev_used = 0;
    double fam_ms[kFamilies] = {};
    int64_t fam_launches[kFamilies] = {};

    int grid_for(int64_t units) const;
    int grid_tiles(int64_t keys) const;
    bool hip_ok(hipError_t e, const char *what);
    bool ev_begin(int family);   // true when an event pair was opened for this launch
    void ev_end(bool open);
    void ev_collect();
    // Enqueue round r (only r == 0 and the parity of r matter to the launch sequence).
    // N and M bound the round's nodes and records (exact in eager mode); passes bounds the
    // radix passes (computed from N when negative).
    bool enqueue_round(int r, int64_t N, int64_t M, const PrioCtx &pc, int passes = -1);
    bool flatten();
    bool read_state();
    bool write_initial_state(int64_t n_cur, int64_t m_cur, uint64_t seed = 0);
};

}  // namespace lc

// A single-graph solve behind the C ABI (cc_ctx of include/cc.h).
struct cc_ctx : public lc::Engine {
    cc_graph_desc g{};
    cc_options o{};
    std::vector<cc_round_stats> stats;
    int32_t rounds = 0;       // rounds of this solve that had nodes
    int32_t next_round = 0;   // index of the next round to enqueue
    bool ran_first = false;   // round 0's kernels ran (map0 is valid)
    bool labels_ready = false;
    int64_t n_cur = 0, m_cur = 0;
    int64_t pending_N = 0, pending_M = 0;   // bounds of the round in flight
    int32_t last_graph_round = -1;          // last round run inside a captured tail
    int64_t solves_done = 0;                // solves that cc_run finished on this context
    int64_t finish_edges = 0;               // union-find finish threshold (0: off)
    bool fused_unavailable = false;         // the device cannot keep the persistent grid resident
    bool finished = false;                  // this solve ended with the union-find finish
    // captured tails of rounds (cc_run), replayed while the rounded-up sizes match
    struct Tail {
        hipGraphExec_t exec;
        int64_t N, M;
        int parity;
        void *ws;
        uint64_t used;   // last use, for replacement
    };
    hipStream_t cap_stream = nullptr;
    std::vector<Tail> tails;
    uint64_t tail_clock = 0;
    // explicit priority tables (CC_EXPLICIT_PRIO): (first round, table), and the table whose
    // inverse the workspace holds
    std::vector<std::pair<int32_t, const uint32_t *>> prio_tabs;
    const uint32_t *inv_for = nullptr;
    // recorded parents (CC_RECORD_ROUNDS): per round, its first record entry (-1: not
    // recorded) and its node count in the record
    struct Rec {
        int64_t off, count;
    };
    std::vector<Rec> recs;
    int64_t rec_used = 0;
    // MergeToLarge parameters of phases 0, 1, ... (the last one repeats)
    std::vector<int64_t> mtl_alphas;
};

namespace lc {
cc_status fail(cc_ctx *c, cc_status s, const char *msg);
cc_status reject(cc_ctx *c, cc_status s, const char *msg);
cc_status hip_status(cc_ctx *c);
// cc_create with the host mirror of the round state supplied by the caller (non-null: kept
// until cc_destroy, never freed by it).  The serving scheduler gives each slot one for good:
// freeing pinned host memory synchronises the whole device, which would stall every other
// request in flight each time one completes.
cc_status ctx_create(const cc_graph_desc *graph, const cc_options *opts, RoundState *mirror, cc_ctx **out);
// Cohorts of the serving scheduler (lc_batch.hip): G graphs of int32 local ids whose records
// and labels stay at per-graph device pointers, solved as one disjoint union (the batch's union
// path), every round of all of them one launch sequence on `stream`.  cohort_begin enqueues the
// union input and round 0, cohort_advance (after the previous call's state readback into
// `mirror` has completed) the next round or the labels, and sets *finished once the labels
// and the rounds (h_rounds: G entries, pinned) are written.  Workspace as for a batch
// (cc_batch_workspace_size / cc_batch_set_workspace); cc_batch_destroy ends it.
cc_status cohort_create(int32_t G, const int64_t *h_voff, const int64_t *h_eoff, const uint64_t *h_seeds,
                        const int32_t *const *h_src, const int32_t *const *h_dst, int32_t *const *h_labels,
                        hipStream_t stream, RoundState *mirror, cc_batch **out);
cc_status cohort_begin(cc_batch *b, int32_t *h_rounds);
cc_status cohort_advance(cc_batch *b, int32_t *h_rounds, bool *finished);
// asynchronous round interface (used by the serving scheduler)
cc_status ctx_round_enqueue(cc_ctx *c, int *launched);
cc_status ctx_round_complete(cc_ctx *c, cc_round_stats *out);
cc_status ctx_labels_enqueue(cc_ctx *c, void *d_labels);
}  // namespace lc
