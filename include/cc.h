/*
 * cc.h -- LocalContraction connected components on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Lacki, Mirrokni, Wlodarczyk, "Connected Components at Scale via
 * Local Contractions" (arXiv 1807.10727), Section 3, paragraph
 * "LocalContraction".  Each phase ("round" below) draws a random ordering rho
 * of the current nodes, gives every node v the vertex of smallest priority in
 * its closed two-hop neighbourhood N(N(v)) (N(v) contains v, Section 2) as its
 * parent, merges nodes with equal parents, and keeps one copy of every edge
 * between different parents (the contraction step, proof of the lemma in
 * Section 3).  The run ends when no edge is left (Section 3); nodes left
 * without edges are final (Section 6 drops isolated nodes after each phase).
 *
 * Specification shared with any independent implementation:
 *   - a merged node is named by the original vertex id of its parent;
 *   - the priority of node name x in round r (r = 0 on the input graph) is
 *       fmix32(fmix32(x ^ k0) ^ k1),   (k1 << 32 | k0) = sm64(seed ^ sm64(r)),
 *     where sm64 is SplitMix64's output function (Steele, Lea, Flood 2014:
 *     z = x + 0x9E3779B97F4A7C15, then the two xor-shift-multiply steps and a
 *     final xor-shift) and fmix32 is MurmurHash3's 32-bit finaliser; priorities
 *     are compared as unsigned 32-bit integers.  Both steps are bijections, so
 *     no two nodes tie.
 *   - records are undirected pairs; loops and repeated records are allowed in
 *     the input and never change a closed neighbourhood.
 *   - the label of an original vertex is the name of the final node it ended
 *     in (an original vertex id of its component), or, with CC_CANONICAL, the
 *     smallest original id of its component.
 *
 * Memory: every pointer argument named d_* is device memory.  The library
 * never allocates device memory: the caller sizes a workspace with
 * cc_workspace_size() and hands it over with cc_set_workspace().  Input edge
 * buffers are borrowed (read only) until cc_destroy(); the caller must keep
 * them alive and unchanged.  All device work is enqueued on the stream given
 * in cc_options; calls that return statistics synchronise that stream.
 *
 * Errors: every entry point returns a cc_status.  No C++ exception crosses
 * this interface.  cc_last_error() describes the most recent failure of a
 * context (including the HIP error string when one is involved).
 *
 * Threading: a context is used by one thread at a time; distinct contexts
 * are independent.
 */
#ifndef CC_H_
#define CC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cc_status;
enum {
    CC_OK = 0,        /* success */
    CC_DONE = 1,      /* cc_contract_round: no edge was left, nothing was done */
    CC_E_ARG = -1,    /* invalid argument (null pointer, size, layout, alignment) */
    CC_E_INPUT = -2,  /* an edge record names a vertex outside [0, n_vertices) */
    CC_E_NOMEM = -3,  /* workspace missing or smaller than cc_workspace_size() */
    CC_E_HIP = -4,    /* a HIP runtime call failed (see cc_last_error) */
    CC_E_STATE = -5,  /* call not valid in the context's current state */
    CC_E_BUDGET = -6  /* a request does not fit the serving memory budget */
};

/* Edge record layouts.  Vertex ids must lie in [0, n_vertices), n_vertices <= 2^31 - 1. */
typedef enum {
    CC_EDGES_SOA_I32 = 0,    /* src: int32[n_edges], dst: int32[n_edges] */
    CC_EDGES_SOA_I64 = 1,    /* src: int64[n_edges], dst: int64[n_edges] */
    CC_EDGES_PACKED_U64 = 2  /* src: uint64[n_edges], record = (a << 32) | b; dst unused (NULL) */
} cc_edge_layout;

typedef struct {
    int64_t n_vertices;  /* vertex ids are 0 .. n_vertices-1 */
    int64_t n_edges;     /* number of records (int64: may exceed 2^31) */
    int32_t layout;      /* cc_edge_layout */
    int32_t reserved;    /* must be 0 */
    const void *src;     /* d_: see cc_edge_layout */
    const void *dst;     /* d_: see cc_edge_layout */
} cc_graph_desc;

/* cc_options.flags
 *
 * Round 0 reads the caller's records in one of two ways, with identical results.  Direct:
 * the min and relabel passes read the input records as they are.  Tiled: the input is first
 * partitioned into directed records grouped by blocks of their endpoints, so that those
 * passes touch node values that stay on chip; the key buffers then hold twice the records
 * (cc_workspace_size grows by 16 bytes per record) and n_vertices must be at most 2^26.
 * Without either flag, a solve runs tiled when n_vertices and n_edges are both at least
 * 2^20 and n_vertices is at most 2^26.  Setting both flags, or CC_ROUND0_TILED with more
 * than 2^26 vertices, makes cc_create return CC_E_ARG. */
enum {
    CC_CANONICAL = 1u << 0,     /* cc_labels writes the smallest original id of each component */
    CC_PROFILE = 1u << 1,       /* time every kernel with HIP events (see cc_kernel_times) */
    CC_ROUND0_DIRECT = 1u << 2, /* round 0 reads the input records directly */
    CC_ROUND0_TILED = 1u << 3,  /* round 0 over the tiled record layout */
    CC_EAGER = 1u << 4,         /* cc_run enqueues every round on its own (no captured tail) */
    CC_TREE = 1u << 5,          /* TreeContraction phases (see below) */
    CC_ONE_HOP = 1u << 6,       /* one-hop labels (see below) */
    CC_EXPLICIT_PRIO = 1u << 7, /* priorities from caller tables (cc_set_explicit_priorities) */
    CC_RECORD_ROUNDS = 1u << 8, /* keep every round's parents (cc_round_parents of any round) */
    CC_MERGE_TO_LARGE = 1u << 9 /* each phase followed by a MergeToLarge step (see below) */
};

/* Label rule of a phase.  Default: LocalContraction (Section 3), the vertex of smallest
 * priority within distance two (closed neighbourhoods).  CC_TREE: TreeContraction (Section 3):
 * every node points to its neighbour of smallest priority other than itself, and the nodes of
 * each weakly connected component of those pointers are merged, under the name of the
 * component's node of smallest priority (the smaller of the two nodes the pointers end in);
 * each phase at least halves the nodes and merged nodes are always connected.  CC_ONE_HOP: the
 * vertex of smallest priority in the closed neighbourhood (the rule of Section 6's Cracker
 * comparison, without its edge rewiring); more phases than LocalContraction.  Setting both
 * makes cc_create return CC_E_ARG.  Either runs round 0 directly or tiled like the default
 * rule.  Priorities, statistics, naming and the labels' meaning are as for LocalContraction. */

/* MergeToLarge (Section 5, paragraph "MergeToLarge step"; the step behind the O(log log n)
 * bound on random graphs): with CC_MERGE_TO_LARGE every LocalContraction phase is followed by a
 * step on the graph the phase left.  A node of that graph is large when its class (the nodes
 * of the phase whose parent it is) holds at least alpha_i nodes, alpha_i being the parameter of
 * phase i (cc_set_merge_to_large); its priority is the alpha_i-th largest priority of its class
 * in that phase.  Every node then takes as its parent the large node of largest priority within
 * distance 2 (itself included), or keeps itself, and nodes with equal parents merge, as in a
 * LocalContraction phase.  In the statistics and in cc_round_parents, phase i is round 2i (its
 * priorities are those of round 2i) and its step is round 2i + 1.  LocalContraction rule only
 * (with CC_TREE or CC_ONE_HOP cc_create returns CC_E_ARG); cc_run runs every round eagerly, and
 * the workspace grows by 28 bytes per vertex. */

/* cc_run and captured tails.  On a context that has already finished a solve, once the
 * remaining graph has at most 2^22 records, cc_run replays a hipGraph of up to 8 rounds
 * (captured on first use, kept per context and reused while the rounded-up sizes match)
 * instead of enqueuing each round and reading its state back: small rounds are otherwise
 * bound by launch overhead.  Results are
 * identical; rounds run this way have in_graph = 1 in their statistics, their kernels are
 * timed together as the family "tail_graph", and cc_round_parents is not available for
 * them.  CC_EAGER turns this off (cc_contract_round never uses it).  With cc_tuning.tail >= 2
 * the rounds that fit the hashed duplicate drop run instead in one persistent cooperative
 * launch (fresh contexts too), timed as "fused_rounds", with in_graph = 2 and the same
 * conditions. */

typedef struct {
    uint64_t seed;       /* priority seed (round keys derive from it as specified above) */
    int32_t max_rounds;  /* 0: run until no edge is left; k > 0: cc_run stops after k rounds */
    uint32_t flags;      /* CC_CANONICAL | CC_PROFILE | CC_ROUND0_DIRECT | CC_ROUND0_TILED | CC_EAGER |
                            CC_TREE | CC_ONE_HOP | CC_EXPLICIT_PRIO | CC_RECORD_ROUNDS | CC_MERGE_TO_LARGE */
    void *stream;        /* hipStream_t for all work of this context; NULL = null stream */
} cc_options;

/* Statistics of one round (all counts exact). */
typedef struct {
    int32_t round;        /* r, from 0 */
    int32_t in_graph;     /* 1 when the round ran inside a captured tail (see cc_run), 2 inside the
                             persistent launch (cc_tuning.tail) */
    int64_t n_active;     /* nodes with at least one loop-free edge in this round */
    int64_t m_in;         /* records read: the raw input count in round 0, |E_r| after */
    int64_t m_survive;    /* records whose two endpoints get different parents (repeats counted) */
    int64_t m_out;        /* distinct loop-free edges of the next graph, |E_{r+1}| */
    int64_t n_finalised;  /* distinct parents of this round that keep no edge */
    int64_t m_sorted;     /* keys this round's duplicate drop processed (a radix sort, or from
                             round 1 on a hashed key set when at most 2^22 of them): m_survive
                             less the repeats each relabel workgroup recognised itself (an LDS
                             key set per workgroup; launch-dependent, not a property of the
                             method) */
} cc_round_stats;

typedef struct cc_ctx cc_ctx;

/*
 * Create a context for one graph.  Validates the descriptor (layout, sizes,
 * 16-byte alignment is NOT required).  Records are read only from round 0 on;
 * an out-of-range id is detected on the device and reported as CC_E_INPUT by
 * the first round (such records are skipped, never dereferenced).
 * *out receives the context (NULL on failure).
 */
cc_status cc_create(const cc_graph_desc *graph, const cc_options *opts, cc_ctx **out);

/* Bytes of device workspace this context needs (depends on n_vertices and n_edges only). */
cc_status cc_workspace_size(const cc_ctx *ctx, size_t *bytes);

/*
 * Hand over the device workspace (caller-owned, >= cc_workspace_size bytes,
 * 256-byte aligned).  Must precede the first round; resets the solve.
 */
cc_status cc_set_workspace(cc_ctx *ctx, void *d_workspace, size_t bytes);

/*
 * Restart the solve on the same borrowed input with a new seed (the
 * workspace is kept).  Used to repeat solves without re-creating contexts.
 */
cc_status cc_reset(cc_ctx *ctx, uint64_t seed);

/*
 * Tuning knobs of a single-graph solve (picked by the autotuner; every setting gives identical
 * results, since none of them changes what a round computes, Section 3).
 */
typedef struct {
    int32_t round0;           /* 0: keep the current form; 1: round 0 reads the records directly;
                                 2: round 0 over the tiled layout (needs n_vertices <= 2^26, no
                                 CC_EXPLICIT_PRIO, and a workspace sized for it); 3: as 2, but the
                                 records reach their rows in one partition pass, unordered inside
                                 a row (two passes over the records fewer, less L2 locality in the
                                 row kernels' gathers; same conditions) */
    int32_t blocks_per_cu;    /* workgroups per compute unit of the grid-stride kernels (1..64); 0: 8 */
    int32_t round0_key_sets;  /* 1 (default): round 0's relabel workgroups drop the repeated keys they
                                 see through an LDS set; 0: they write every survivor */
    int32_t scatter_waves;    /* waves per SIMD the radix scatter is built for: 2, 3 or 4; 0: 3 */
    int32_t row_pairs;        /* tiled round 0, two-hop row pass: record pairs in flight per thread
                                 (2, 4 or 8); 0: 4 */
    int32_t relabel_pairs;    /* tiled round 0, relabel row pass: the same (1, 2 or 4); 0: 2 */
    int32_t row_generation;   /* tiled round 0: rows of the two gathering row passes launched
                                 together, per compute unit (1..8); 0: 1; -1: every row in one
                                 launch */
    int32_t round0_sort;      /* how round 0 orders its keys for the duplicate drop: 1 (0: default)
                                 LSD radix passes; 2 two levels of buckets cut at splitters drawn
                                 from the keys, then each bucket sorted in LDS */
    int32_t tail;             /* cc_run's rounds >= 1 once at most 2^22 records remain: 1 (0: default)
                                 a launch sequence per round (replayed from a captured graph on a
                                 reused context); 2, 3, 4: all of them in one persistent cooperative
                                 launch of 1, 2 or 4 workgroups per compute unit (at most what
                                 stays resident), the steps of a round separated by grid-wide
                                 barriers, one readback in all; its rounds report in_graph = 2.
                                 Every label rule and MergeToLarge (TreeContraction's pointer
                                 jumping and MergeToLarge's class priorities inside the launch
                                 too), without CC_EAGER, CC_EXPLICIT_PRIO or CC_RECORD_ROUNDS
                                 (otherwise the default applies); it stops at opts.max_rounds and
                                 where the union-find finish takes over */
    int32_t radix_form;       /* the duplicate drop's LSD radix sorts: 1 (0: default) per digit a count
                                 pass, a scan of the count table and a scatter; 2 one sweep: one
                                 count pass for every digit at once, then per digit only the
                                 scatter, each tile finding how many keys of each digit precede
                                 it by decoupled look-back over the tiles before it */
} cc_tuning;

/*
 * Apply tuning knobs (host struct, copied).  Resets the current solve as cc_reset with the
 * current seed does, and drops captured tails.  CC_E_ARG for a value out of range or a tiled
 * round 0 the context cannot take; CC_E_NOMEM when a workspace is set and is smaller than the
 * new form needs (cc_workspace_size reports the size for the current form).  cc_get_tuning
 * reports the knobs in force (round0 1, 2 or 3; every 0 "default" resolved to its value).
 */
cc_status cc_set_tuning(cc_ctx *ctx, const cc_tuning *t);
cc_status cc_get_tuning(const cc_ctx *ctx, cc_tuning *t);

/*
 * Run one round (Section 3, one phase of LocalContraction) and synchronise
 * the stream.  Returns CC_DONE without work once no edge is left.  `out`
 * (nullable, host) receives the round's statistics.
 */
cc_status cc_contract_round(cc_ctx *ctx, cc_round_stats *out);

/*
 * Run rounds until no edge is left (or opts.max_rounds rounds ran), then
 * compose the per-round maps into final labels on the device.  *rounds
 * (nullable, host) receives the number of rounds of this solve so far.
 */
cc_status cc_run(cc_ctx *ctx, int32_t *rounds);

/*
 * Write the label of every original vertex into d_labels (int32[n_vertices]
 * for CC_EDGES_SOA_I32 and CC_EDGES_PACKED_U64, int64[n_vertices] for
 * CC_EDGES_SOA_I64).  Asynchronous on the context's stream.  Valid after
 * cc_run, or after cc_contract_round returned CC_DONE; CC_E_STATE otherwise.
 */
cc_status cc_labels(cc_ctx *ctx, void *d_labels);

/*
 * Parents of round r (Section 3: the vertex of smallest priority in N(N(x)) of every node x),
 * a test and inspection aid, not on the measured path.  d_parents (int32[n_vertices])
 * receives, for every name x that was a node of round r, the name of its parent, and -1 for
 * every other name.  *n_nodes (nullable, host) receives the round's node count.
 * Synchronises.  r < 0 means the most recent round, which is always available unless it ran
 * inside a captured tail or the union-find finish ended the solve.  Earlier rounds need
 * CC_RECORD_ROUNDS: the context then copies every round's parents into a record area of the
 * workspace (4 bytes per vertex for round 0, 8 bytes per node for later rounds, at most 20
 * bytes per vertex in all; cc_workspace_size grows by that much) and runs every round
 * eagerly.  CC_E_STATE for a round that has not run, was not recorded (no CC_RECORD_ROUNDS,
 * or the record area was full), or is unavailable as above; CC_E_ARG for a null pointer.
 */
cc_status cc_round_parents(cc_ctx *ctx, int32_t r, int32_t *d_parents, int64_t *n_nodes);

/*
 * One-hop and two-hop minima of the most recent round (test and inspection aid, not on the
 * measured path): for every name x that was a node of that round, d_m1[x] = the smallest
 * priority in the closed neighbourhood N(x) and d_l[x] = the smallest priority in N(N(x))
 * (Section 3: the parent is the vertex with that priority; Section 2: N(x) contains x), and
 * 0xFFFFFFFF for every other name (both uint32[n_vertices], device).  After a round 0 that
 * ran over the tiled layout the two-hop minimum is not kept, and d_l[x] is then the priority
 * of x's parent, which equals it by definition.  LocalContraction only: CC_E_STATE with
 * CC_TREE or CC_ONE_HOP, before the first round, after a round inside a captured tail, or
 * after the union-find finish.  Synchronises.
 */
cc_status cc_debug_round_arrays(cc_ctx *ctx, uint32_t *d_m1, uint32_t *d_l);

/*
 * MergeToLarge parameters (needs CC_MERGE_TO_LARGE at cc_create): phase i uses
 * h_alphas[min(i, count - 1)] (host array, copied).  Without a call every phase uses
 * max(2, ceil(ln n_vertices)).  Applies from the next round enqueued.  CC_E_STATE without
 * CC_MERGE_TO_LARGE; CC_E_ARG for a null array, count < 1 or an alpha outside [1, 2^32 - 1].
 */
cc_status cc_set_merge_to_large(cc_ctx *ctx, const int64_t *h_alphas, int32_t count);

/*
 * Explicit priorities (needs CC_EXPLICIT_PRIO at cc_create).  A test hook for the
 * definition, under which the ordering may be any one-to-one map (Section 3): from round
 * r on, until a later round has a table of its own, the priority of node name x is d_prio[x]
 * instead of the seeded hash; rounds before the first table use the hash.  d_prio is
 * uint32[n_vertices], device memory borrowed until cc_destroy or a replacing call for the
 * same r, and must be a permutation of 0 .. n_vertices-1 (an ordering of all names; the
 * parent is found through its inverse, which the library builds in the workspace: 4 bytes
 * per vertex more).  A table that is not a permutation makes the round that first uses it
 * fail with CC_E_INPUT.  With CC_EXPLICIT_PRIO round 0 reads the records directly
 * (CC_ROUND0_TILED is CC_E_ARG) and cc_run runs every round eagerly.  CC_E_STATE without
 * CC_EXPLICIT_PRIO; CC_E_ARG for r < 0 or a null table.
 */
cc_status cc_set_explicit_priorities(cc_ctx *ctx, int32_t r, const uint32_t *d_prio);

/*
 * Round checkpoint in host memory.  Between rounds a solve is its current edge set, the
 * names of its nodes and the per-round maps that compose the labels (Section 3: a phase reads
 * only the graph the previous one left).  cc_save_state writes that state and the statistics
 * so far into h_buf (host); with h_buf NULL it only sets *bytes to the size needed, and a
 * *bytes smaller than that is CC_E_ARG.  cc_load_state restores it into a context created for
 * the same graph (same n_vertices, n_edges, layout and label rule; CC_E_ARG otherwise, and for
 * a buffer that is not a checkpoint) that has its workspace; cc_run or cc_contract_round then
 * continue with the next round, and every later round, the statistics and the labels equal
 * those of the uninterrupted solve.  Explicit priority tables and recorded parents are not
 * part of a checkpoint (set the tables again after loading).  Both synchronise.  CC_E_NOMEM
 * without a workspace; CC_E_STATE on a context whose solve has failed.
 */
cc_status cc_save_state(cc_ctx *ctx, void *h_buf, size_t *bytes);
cc_status cc_load_state(cc_ctx *ctx, const void *h_buf, size_t bytes);

/*
 * Edges of the graph the most recent round left (test and inspection aid, not on the
 * measured path): the distinct loop-free edges between that round's parents (the
 * contraction step, proof of the lemma in Section 3), each once, written to d_edges
 * (uint64[cap]) as (a << 32) | b with a < b the two endpoints' names, in no particular
 * order.  *n_edges (host) receives their number; d_edges NULL asks for the number only, and
 * a d_edges of fewer than that many entries gets nothing (CC_E_ARG).  Synchronises when it
 * writes.  CC_E_STATE like cc_round_parents (no round yet, a round inside a captured tail,
 * the union-find finish).
 */
cc_status cc_round_edges(cc_ctx *ctx, uint64_t *d_edges, int64_t cap, int64_t *n_edges);

/*
 * Union-find finish (Section 6): from round 1 on, once the graph left by a round has at most
 * max_edges edges (0, the default, turns this off), cc_run ends the solve by finding the
 * components of that graph with a union-find on the device instead of running more rounds.
 * Every remaining node then becomes final under the smallest name in its component, so the
 * raw labels differ from a solve without the finish (CC_CANONICAL labels do not).  The rounds
 * before the switch are unchanged; cc_run's round count and the statistics cover only them,
 * and cc_round_parents returns CC_E_STATE afterwards.  cc_contract_round never finishes.
 * Applies from the next cc_run; CC_E_ARG for a null context or a negative count.
 * cc_get_finished reports (1/0) whether the current solve ended this way.
 */
cc_status cc_set_finish(cc_ctx *ctx, int64_t max_edges);
cc_status cc_get_finished(const cc_ctx *ctx, int32_t *finished);

/* Statistics of round r of the current solve (host copy kept by the library). */
cc_status cc_get_round_stats(const cc_ctx *ctx, int32_t r, cc_round_stats *out);

/*
 * Kernel timing (CC_PROFILE): per kernel family, the summed event time in ms
 * and the number of launches since the last cc_set_workspace/cc_reset.
 * Families are listed by cc_kernel_family_name(i) for i < cc_kernel_family_count().
 */
int32_t cc_kernel_family_count(void);
const char *cc_kernel_family_name(int32_t i);
cc_status cc_kernel_times(const cc_ctx *ctx, double *ms, int64_t *launches, int32_t cap);

/*
 * Restrict CC_PROFILE's events to some families: bit i of family_mask enables family i
 * (default: all).  Each timed launch costs two event records on the stream, so timing one
 * family keeps the stream almost as fast as an untimed run.  Applies to launches enqueued
 * after the call; CC_E_ARG for a null context.
 */
cc_status cc_set_profile_mask(cc_ctx *ctx, uint64_t family_mask);

cc_status cc_destroy(cc_ctx *ctx);
const char *cc_last_error(const cc_ctx *ctx);

/* ------------------------------------------------------------------------------------
 * Batched solve of many independent graphs (one launch sequence, captured in a hipGraph).
 *
 * Graph g has vertices 0 .. n_g-1 (n_g = h_vtx_off[g+1] - h_vtx_off[g]) and the records
 * d_src[i], d_dst[i] (int32 local ids) for i in [h_edge_off[g], h_edge_off[g+1]).  Its
 * priorities come from h_seeds[g] exactly as in a solo solve with that seed, and components
 * of different graphs never interact (Section 3: only priorities inside a component are
 * compared), so every graph's labels equal its solo cc_run + cc_labels.  Offsets and seeds
 * are copied at creation; device arrays are borrowed until cc_batch_destroy.
 * ------------------------------------------------------------------------------------ */
typedef struct cc_batch cc_batch;

/* Tuning knobs (picked by the autotuner; every setting gives identical labels). */
typedef struct {
    int32_t blocks_per_cu;        /* workgroups per CU of the grid-stride kernels (1..64) */
    int32_t small_variant;        /* LDS solver limits: 0 none, 1 (512 vertices, 4096 records),
                                     2 (1024, 8192), 3 (2048, 16384) */
    int32_t small_threads;        /* workgroup size of the LDS solver: 256 or 512 */
    int32_t small_blocks_per_cu;  /* persistent LDS workgroups per CU (1..16) */
    int32_t rounds_per_graph;     /* union rounds captured in the graph (1..64); more run eagerly */
    int32_t use_graph;            /* 1: capture once and replay; 0: eager launches */
    int32_t radix_form;           /* the union's radix sorts: 1 (0: default) count, scan and scatter
                                     per digit; 2 one sweep, as cc_tuning.radix_form */
} cc_batch_config;

cc_status cc_batch_create(int32_t n_graphs, const int64_t *h_vtx_off, const int64_t *h_edge_off,
                          const uint64_t *h_seeds, const void *d_src, const void *d_dst, const cc_options *opts,
                          cc_batch **out);
cc_status cc_batch_workspace_size(const cc_batch *batch, size_t *bytes);
cc_status cc_batch_set_workspace(cc_batch *batch, void *d_workspace, size_t bytes);
cc_status cc_batch_set_config(cc_batch *batch, const cc_batch_config *config);
cc_status cc_batch_get_config(const cc_batch *batch, cc_batch_config *config);
/* Solve every graph: d_labels int32[h_vtx_off[G]] receives local labels (slot h_vtx_off[g] + v
 * for vertex v of graph g); h_rounds (nullable, host int32[G]) the rounds of each graph.
 * Synchronises the stream. */
cc_status cc_batch_run(cc_batch *batch, int32_t *d_labels, int32_t *h_rounds);
/* How the current configuration split the batch: graphs on the LDS solver, union records. */
cc_status cc_batch_split(const cc_batch *batch, int32_t *n_small, int64_t *union_records);
cc_status cc_batch_destroy(cc_batch *batch);
const char *cc_batch_last_error(const cc_batch *batch);

/* ------------------------------------------------------------------------------------
 * Serving: continuous batching of requests on one GPU.
 *
 * A scheduler thread admits requests while a slot and device memory are free and keeps
 * their state on the device; requests that arrive while others run are admitted as
 * slots and memory free up, and their work overlaps on the device.  Waiting small
 * requests (CC_EDGES_SOA_I32 within the LDS limits of small_variant) are fused into one
 * launch of the LDS solver; every other request gets a slot stream and a workspace from
 * the arena and advances one round (Section 3, one phase) per scheduler step.  With
 * cohort_max > 1, waiting large requests of at most cohort_max_vertices vertices (int32 SoA)
 * share a slot as one cohort: their graphs form one disjoint union, and each scheduler step
 * runs one round of all of them as one launch sequence (each graph keeps its own priorities
 * and round count, so its labels are its solo solve's); a request of a cohort whose records
 * name a vertex out of range fails alone (CC_E_INPUT).
 * A request's labels equal its solo solve with the same seed, whatever else is in flight.
 *
 * The arena is caller-owned device memory of budget_bytes (256-byte aligned); request
 * workspaces are carved from it and returned when the request completes, so the budget
 * caps the device memory in use.  A request whose own workspace exceeds the whole budget
 * is refused (CC_E_BUDGET); one that only waits for memory is deferred, never failed.
 * A request's edge arrays and label array are caller-owned device memory that must stay
 * valid until the request completes.  All entry points are thread-safe.
 * ------------------------------------------------------------------------------------ */
typedef struct cc_server cc_server;

typedef struct {
    int32_t n_slots;               /* large requests in flight at once (1..64), one stream each */
    int32_t small_variant;         /* LDS limits for small requests as in cc_batch_config; 0 = none */
    int32_t small_threads;         /* 256 or 512 */
    int32_t small_blocks_per_cu;   /* 1..16 */
    int32_t max_small_per_launch;  /* small requests fused into one launch (1..65536) */
    int32_t small_launches;        /* small launches in flight at once (1..8) */
    int32_t cohort_max;            /* up to this many waiting large requests (int32 SoA, at most
                                      cohort_max_vertices vertices each) start together as one
                                      cohort: one disjoint union whose every round is one launch
                                      sequence for all of them (0 or 1: none; at most 64) */
    int32_t cohort_max_vertices;   /* 0: 2^20 */
} cc_server_config;

typedef struct {
    uint64_t id;
    cc_status status;      /* CC_OK; CC_E_INPUT for an id out of range; CC_E_STATE if cancelled */
    int32_t rounds;
    int32_t small_path;    /* 1 if solved by the fused LDS launch */
    int32_t cohort;        /* requests of the cohort it was solved in (0: solved on its own) */
    double t_submit;       /* seconds on the server clock (cc_server_info().now) */
    double t_admit;
    double t_done;         /* labels written */
} cc_request_result;

typedef struct {
    double now;            /* server clock, seconds since creation */
    int64_t pending;       /* submitted, not admitted */
    int64_t active;        /* admitted, not completed */
    int64_t bytes_in_use;  /* arena bytes held by admitted requests */
    int64_t peak_bytes;
    int64_t small_launches;
} cc_server_info_t;

cc_status cc_server_create(void *d_arena, size_t budget_bytes, const cc_server_config *config, cc_server **out);
/* Queue one graph (described as for cc_create) with its priority seed; labels (int32, or
 * int64 for CC_EDGES_SOA_I64) go to d_labels.  *req_id identifies the request. */
cc_status cc_server_submit(cc_server *server, const cc_graph_desc *graph, uint64_t seed, void *d_labels,
                           uint64_t *req_id);
/* Completed requests (non-blocking): up to cap results into out, count in *n. */
cc_status cc_server_poll(cc_server *server, cc_request_result *out, int32_t cap, int32_t *n);
/* Like cc_server_poll, but waits up to timeout_s seconds for at least one completion. */
cc_status cc_server_wait(cc_server *server, cc_request_result *out, int32_t cap, int32_t *n, double timeout_s);
/* Cancel a request that has not completed (it completes with CC_E_STATE). */
cc_status cc_server_cancel(cc_server *server, uint64_t req_id);
/* paused != 0: admit no new request until called again with 0 (requests in flight continue,
 * submissions wait), for instance to release a burst of requests together. */
cc_status cc_server_pause(cc_server *server, int32_t paused);
cc_status cc_server_info(cc_server *server, cc_server_info_t *info);
/* Finishes every admitted request, cancels the waiting ones, stops the scheduler. */
cc_status cc_server_destroy(cc_server *server);
const char *cc_server_last_error(const cc_server *server);

/* Library version string and the offload target it was built for. */
const char *cc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CC_H_ */
