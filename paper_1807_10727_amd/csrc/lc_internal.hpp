// Internal interface between the round engine (host) and the kernels (device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_device.hpp"

namespace lc {

typedef unsigned long long u64c;  // type of 64-bit device atomics

constexpr int kMaxLevels = 64;    // per-round maps kept before they are folded into map0
constexpr int kStatRounds = 128;  // rounds whose statistics the device keeps (plain solve)

// Device-resident state of the current round.  Every kernel reads its element counts
// from here, so a sequence of rounds can be enqueued (or captured in a graph) without
// host round trips; the eager driver reads it back once per round.  Fields that kernels
// update with atomics sit on cache lines of their own, away from the fields every
// thread reads.
struct RoundState {
    // written only between rounds (single-thread kernels) or by one thread of a kernel
    u64c n_cur;        // N_r: nodes of this round (round 0: the whole id space n0)
    u64c m_cur;        // M_r: records of this round
    u64c n_prev;       // N of the round that just ended
    u64c aux_n;        // element count handed from one kernel to the next (scans)
    u64c map_off;      // next free entry of the map arena
    u64c map_cap;      // entries of the map arena
    u64c n_slabs;      // relabel output slabs of this round (slab layout)
    int32_t round;     // r
    int32_t nbits;     // key bits of this round's sort: 2 * ceil(log2 N_r)
    int32_t e_sel;     // key buffer that holds E_r (rounds >= 1)
    int32_t done;      // no edge left
    int32_t levels;    // per-round maps in the arena
    int32_t kb;        // bits per endpoint in this round's sort keys: ceil(log2 N_r)
    int32_t hb_shift;  // next-round block of an endpoint: index >> hb_shift (kb: one block)
    int32_t keys_dense;  // the relabel wrote its keys packed at [0, s_keys) (else: in slabs)
    u64c t_count;      // round 0, tiled layout: directed records (twice the loop-free inputs)
    u64c t_tiles;      // round 0, tiled layout: tiles of the row partition (its count table's columns)
    uint64_t seed;     // priority seed of a plain solve
    RoundKey key;      // this round's priority key, round_key(seed, round) (plain solve)
    int32_t rounds_active;   // rounds so far that read at least one record
    int32_t hash_slots;      // slots of the hashed duplicate drop (rounds that use it)
    u64c b_tiles1;           // sampled buckets: tiles of the first level
    u64c b_tiles2;           // sampled buckets: tiles of the second level (within first-level buckets)
    alignas(128) u64c n_active;   // nodes with a loop-free edge (atomics)
    alignas(128) u64c s_count;    // records surviving relabelling, repeats counted (atomics)
    alignas(128) u64c s_keys;     // sort keys written by the relabel: the survivors less the
                                  // repeats a workgroup recognised itself (atomics)
    alignas(128) u64c n_final;    // parents of this round that keep no edge (atomics)
    alignas(128) u64c n_labels;   // distinct parents of this round (atomics)
    alignas(128) uint32_t jflag[3];   // TreeContraction: pointer-jumping passes that changed a pointer
    uint32_t jdone;                   // TreeContraction: a pass found every pointer on its cycle
    alignas(128) uint32_t err;    // bit 0: input id out of range; bit 1: map arena overflow;
                                  // bit 2: internal consistency; bit 3: an explicit priority
                                  // table that is not a permutation of [0, n0) (atomics)
    alignas(128) u64c m_next;     // distinct edges of the next graph (one workgroup)
    u64c n_next;                  // nodes of the next graph (one workgroup)
    alignas(128) u64c level_off[kMaxLevels];
    // statistics of every round that read records (round, n_active, m_in, survivors, m_out,
    // n_final, sort keys), so that rounds enqueued back to back need a single readback
    u64c rstats[kStatRounds][7];
};

enum Layout { kSoa32 = 0, kSoa64 = 1, kPacked = 2 };

// Input edge records (round 0 only).
struct EdgeIn {
    const void *s;
    const void *d;
    int64_t m;      // records
    uint32_t n;     // valid ids are [0, n)
    int32_t layout;
    int32_t vec;    // 1: both arrays 16-byte aligned, vector loads allowed
};

// Priority context.  Plain graph: one round key.  Batch of independent graphs packed in
// one id space: graph g owns ids voff[g] .. voff[g+1]-1 and hashes its local ids with its
// own per-round key keys[g].
// An explicit ordering (cc_set_explicit_priorities) replaces the hash in a plain solve:
// tab[name] is the node's priority, a permutation of [0, n0), and inv its inverse.
struct PrioCtx {
    RoundKey key;
    const RoundKey *keys;   // [G] (batch)
    const uint32_t *voff;   // [G+1] (batch)
    const uint32_t *tab;    // [n0] explicit priorities, or null (hashed)
    const uint32_t *inv;    // [n0] inverse of tab
};

// Priority of a name in a plain solve, and the name that has a given priority.
__device__ inline uint32_t rho_of(const PrioCtx &pc, uint32_t name) {
    return pc.tab ? pc.tab[name] : prio(pc.key, name);
}
__device__ inline uint32_t rho_name(const PrioCtx &pc, uint32_t p, int64_t n0) {
    if (pc.tab) return (int64_t)p < n0 ? pc.inv[p] : 0xFFFFFFFFu;
    return prio_inv(pc.key, p);
}

// Splitters of one level of the sampled-bucket duplicate drop (lc_bucket.hip): up to 255
// distinct sample values u[0] < u[1] < ... cut the keys into at most 256 buckets in key order.
// A value that several splitter ranks of the sample fell on ("heavy") gets a bucket of its
// own, holding only keys equal to it; the open bucket open_id[i] holds the keys above u[i-1]
// and up to u[i] (below u[i] when u[i] is heavy), open_id[m] those above u[m-1].
struct alignas(16) BucketTab {
    uint64_t u[255];
    uint8_t heavy[255];
    uint8_t eq_id[255];     // bucket of the keys equal to a heavy u[i]
    uint8_t open_id[256];
    uint8_t eqb[256];       // bucket b holds a single key value
    int32_t m;              // distinct splitters
    int32_t nb;             // buckets (<= 256)
};
static_assert(sizeof(BucketTab) % 16 == 0, "bucket tables are copied in 16-byte words");

// Workspace arrays of one solve (device pointers).
struct Work {
    RoundState *st;
    uint32_t *ml;        // [2 n0] node word: ml[2x] one-hop minimum, ml[2x+1] two-hop minimum
    uint32_t *par;       // [n0] parent of each node: its index in this round, then (after
                         // the label scan) its rank among the labels, or kNoParent
    uint8_t *has_edge;   // [n0] label keeps an edge (byte stores by the unique count pass)
    uint32_t *nmap;      // [2 ceil(n0 / 32)] the same as bits: next-graph node map (nmap_rank)
    uint8_t *is_label;   // [n0] node of this round is somebody's parent (byte stores: many
                         // nodes name the same parent, which bit atomics would serialise)
    uint32_t *lmap;      // [2 ceil(n0 / 32)] the same as bits (nmap format): a label's
                         // rank among them is the index its edges use in the sort keys
    uint32_t *lab_at;    // [n0] node of this round that is the label of each rank
    uint32_t *newidx;    // [n0] scratch of the canonical relabelling
    uint32_t *names[2];  // [n0] node names, rounds >= 1 (round r uses names[r & 1])
    uint32_t *gids[2];   // [n0] batch: graph of each node, rounds >= 1
    uint32_t *gid0;      // [n0] batch: graph of each vertex (round 0)
    uint32_t *idx_of;    // [n0] compact index of a name in the current round
    uint32_t *map0;      // [n0] vertex -> node of the first kept level (or kFinal | name)
    uint32_t *maps;      // [n0] arena of the per-round maps of rounds >= 1
    uint64_t *keys[2];   // [m0] edge / sort key ping-pong buffers (E_r is keys[e_sel])
    uint32_t *counts;    // [kRadixMax * sort tiles] digit counts of one sort pass
    uint32_t *partials;  // scan partial sums
    int64_t kcap;        // records each key buffer holds
    uint32_t *tile_cnt;  // [sort tiles] unique: heads per tile
    uint32_t *pinv;      // [n0] inverse of an explicit priority table (CC_EXPLICIT_PRIO), else null
    uint32_t *rec;       // round record arena (CC_RECORD_ROUNDS), else null
    int64_t rec_cap;     // 4-byte entries of the record arena
    // MergeToLarge (CC_MERGE_TO_LARGE), per node of the graph a LocalContraction step left:
    // class size, the alpha-th largest member priority, a count; the two best-candidate passes
    uint32_t *mtl_size, *mtl_v, *mtl_cnt;   // [n0] each
    uint64_t *mtl_acc[2];                    // [n0] each
    uint32_t *slab_cnt;  // [slabs] relabel survivors per output slab
    // one-sweep radix passes (single solves): digit totals of every pass, then a tile counter
    // per pass ([kSweepWords]); the odd passes' look-back words ([kRadixMax * sort tiles]; the
    // even passes use counts)
    uint32_t *sweep;
    uint32_t *sweep_desc;
    // sampled-bucket duplicate drop (single solves): the first level's table and one table per
    // first-level bucket; first-level bucket starts ([257], the last = keys) and first tiles of
    // the second level ([257], the last = its tile count)
    BucketTab *btab;     // [257]
    uint64_t *bseg;      // [257]
    uint32_t *btile;     // [257]
    int32_t *g_rounds;   // batch: [G] rounds in which each graph still had an edge
    int64_t n0, m0;
    int32_t round0_sets_off;   // 1: round 0's relabel workgroups keep no key set (tuning)
};

constexpr int kThreads = 256;                      // workgroup size of the streaming kernels
#ifndef LC_SORT_THREADS
#define LC_SORT_THREADS 256
#endif
constexpr int kSortThreads = LC_SORT_THREADS;          // workgroup of the sort and unique kernels
constexpr int kSortItems = 16;                         // keys per thread in a sort tile
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per sort tile
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;   // elements per block of the generic scan
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
// Widest sort digit: a pass may take up to kRadixMaxBits bits when that saves a pass (see
// npasses and pass_digit).  9-bit digits measured slower than the pass they save (twice the
// bins halve the runs each tile writes), so the default keeps 8.
#ifndef LC_SORT_MAX_BITS
#define LC_SORT_MAX_BITS 8
#endif
constexpr int kRadixMaxBits = LC_SORT_MAX_BITS;
constexpr int kRadixMax = 1 << kRadixMaxBits;
constexpr int kMaxPasses = 8;                      // 64-bit keys
// One-sweep radix passes: a look-back word is empty, a tile's own count of a digit (below
// 2^31), or kSweepPrefix with the count of that digit in the tile and all before it.
constexpr uint32_t kSweepEmpty = 0xFFFFFFFFu;
constexpr uint32_t kSweepPrefix = 0x80000000u;
constexpr int kSweepWords = kMaxPasses * kRadixMax + kMaxPasses;
// A one-sweep sort of this many keys or more is flagged instead of run (its prefix words
// could not hold the counts); the host gives such rounds (more records than that) the other form.
constexpr uint64_t kSweepMaxKeys = 0x7FFFFFFFu;
// Polls of one look-back word before a tile gives up on it (seconds, where a tile takes
// microseconds): a word that is never published, which a correct run cannot produce, then
// fails the solve as an internal error instead of holding the GPU.  The offsets the tile
// uses stay below the true ones, so its writes stay inside the key buffer.
constexpr uint32_t kSweepMaxPolls = 1u << 22;
constexpr int kSlab = 2 * kSortTile;               // records per relabel workgroup slab
constexpr int64_t kSmallScanEntries = 1 << 15;    // count tables scanned by one workgroup
constexpr int64_t kSmallFlagNodes = 1 << 18;      // flag maps built by one workgroup
// Rounds >= 1 with at most kHashMaxRecords records (and a key buffer of at least 2 M + 1
// records) drop repeated edges through an open-addressing key set of 2 K + 1 slots instead of
// the radix passes, whose launches dominate such rounds.  The set lives in the round's own
// edge buffer, which the relabel has consumed.
#ifndef LC_HASH_DEDUP
#define LC_HASH_DEDUP 1
#endif
constexpr int64_t kHashMaxRecords = 1 << 22;   // as large as a captured tail's record bound
// A round of more records hashes when its keys (known on the device after the relabel, often
// far fewer than its records) do: the hashing kernels and the sort are both enqueued, gated.
enum Dedup { kDedupSort = 0, kDedupHash = 1, kDedupDevice = 2 };
#ifndef LC_SCATTER_WAVES
#define LC_SCATTER_WAVES 3   // default waves per SIMD of the radix scatter (2, 3 or 4 are built)
#endif
static_assert(LC_SCATTER_WAVES >= 2 && LC_SCATTER_WAVES <= 4, "the radix scatter is built for 2, 3 or 4 waves");
// Record pairs each thread keeps in flight in the gathering row kernels of the tiled round 0
// (defaults; the tuner may pick others).  A row sweeps the whole column id space once, so
// the ids its workgroup gathers in one step span (pairs * 2 * 1024 / row records) of that
// space: few enough pairs keep the span of the rows running together on an XCD inside its L2.
#ifndef LC_TMIN2_PAIRS
#define LC_TMIN2_PAIRS 4
#endif
#ifndef LC_TRELABEL_PAIRS
#define LC_TRELABEL_PAIRS 2
#endif
#ifndef LC_SCATTER_GRID
#define LC_SCATTER_GRID 1
#endif
#ifndef LC_DEDUP_LOG2
#define LC_DEDUP_LOG2 12   // slots of the relabel's workgroup key set (8 B each)
#endif
// Sort keys (edge_key) order edges by the block of hi, then lo, then hi, so the next round
// reads its edges grouped by the block of their larger endpoint.  A block spans about
// kBlockNodes next-round nodes, and lo is swept in increasing order within the block.  Wider
// blocks mean fewer sweeps over lo (better for the min passes), narrower ones keep hi's node
// state in L2 (better for the next-node marks); 2^19 measured best on the bench graph.
#ifndef LC_BLOCK_NODES_LOG2
#define LC_BLOCK_NODES_LOG2 19
#endif
constexpr int64_t kBlockNodes = 1 << LC_BLOCK_NODES_LOG2;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A round-0 id without a loop-free record has no parent and is nobody's parent (its rank).
constexpr uint32_t kNoParent = 0xFFFFFFFFu;

// Bit maps with prefix counts (the label map over a round's nodes, the next-graph node map
// over its labels).  Word pair i covers entries 32 i .. 32 i + 31: map[2 i] has a bit for each
// entry that is set, map[2 i + 1] counts the set entries before 32 i.  An entry's rank among
// the set ones is then one 8-byte load and a popcount away, and the map of N entries takes
// N / 4 bytes, small enough to stay in cache while sorted edges sweep over it.  The maps are
// built by a scan over byte flags: many threads set the same entry, which plain byte stores
// absorb and bit atomics would serialise.
__device__ inline bool nmap_has(const uint32_t *nmap, uint64_t x) {
    return (nmap[2 * (x >> 5)] >> (x & 31)) & 1u;
}
__device__ inline uint32_t nmap_rank(const uint32_t *nmap, uint64_t x) {
    const uint2 e = *(const uint2 *)(nmap + 2 * (x >> 5));
    return e.y + (uint32_t)__popc(e.x & ((1u << (x & 31)) - 1u));
}

// Sort key of an edge lo < hi between indices of a round with b = ceil(log2 N) bits per
// index: hi's block (hi >> s), then lo, then hi's s bits below the block.  The block number
// is hi's top b - s bits, so the key has 2 b bits whatever the block width; s = b when the
// round has a single block.
__host__ __device__ inline uint64_t edge_key(uint32_t lo, uint32_t hi, int kb, int s) {
    return ((uint64_t)(hi >> s) << (kb + s)) | ((uint64_t)lo << s) | (uint64_t)(hi & ((1u << s) - 1u));
}
__host__ __device__ inline void edge_key_split(uint64_t k, int kb, int s, uint64_t &lo, uint64_t &hi) {
    lo = (k >> s) & ((1ull << kb) - 1ull);
    hi = ((k >> (kb + s)) << s) | (k & ((1ull << s) - 1ull));
}

// Which key buffer each step uses, from the device state (identical on host and device).
// Radix passes for nbits-bit keys: 8-bit digits, or up to kRadixMaxBits-bit digits when
// that takes fewer passes.  pass_digit spreads the bits evenly, earlier passes taking the
// spare bit.
__host__ __device__ inline int npasses(int nbits) {
    if (nbits <= 0) return 0;
    const int p8 = (nbits + kRadixBits - 1) / kRadixBits;
    const int pw = (nbits + kRadixMaxBits - 1) / kRadixMaxBits;
    return pw < p8 ? pw : p8;
}
__host__ __device__ inline void pass_digit(int nbits, int pass, int &shift, int &width) {
    const int P = npasses(nbits);
    const int base = nbits / P, extra = nbits % P;
    width = base + (pass < extra ? 1 : 0);
    shift = pass * base + (pass < extra ? pass : extra);
}
__host__ __device__ inline int sort_src(int round, int e_sel) { return round == 0 ? 0 : 1 - e_sel; }
__host__ __device__ inline int sorted_sel(int round, int e_sel, int nbits) {
    return sort_src(round, e_sel) ^ (npasses(nbits) & 1);
}

// Round 0 over the tiled record layout (lc_tiled.hip).  The input is partitioned once into
// directed records (x << 32 | y), two per loop-free input record, grouped by the row block
// x >> xs and, within a row, by the column block y >> ys.  One workgroup owns a row: the
// row's node values live in LDS, and the rows that run at the same time sweep the column
// blocks in the same order, so the values gathered at y stay resident in L2.
struct TPlan {
    int32_t xs, ys;      // row / column block shifts
    int32_t rows, cols;  // row blocks (<= kTRowsMax), column blocks (<= 256)
    int64_t tiles_a;     // partition pass A: tiles of kTaIn input records
    int64_t tiles_b;     // partition pass B: upper bound of its kTbTile-record tiles
    int64_t tiles_r;     // the one-pass row partition: tiles of kTrIn input records
};
constexpr int kTxShiftMax = 15;            // 2^15 four-byte node values: 128 KiB of LDS
constexpr int kTRowsMax = 2048;            // row digit of at most 11 bits
constexpr int kTaIn = 2048;                // input records per pass-A tile
constexpr int kTbThreads = 512;
constexpr int kTbTile = 16 * kTbThreads;   // directed records per pass-B tile
constexpr int kTrIn = kTbTile / 2;         // input records per tile of the one-pass row partition
constexpr int kTRowThreads = 1024;         // workgroup of the per-row kernels
constexpr int64_t kTiledMinVertices = 1 << 20;   // default: tiled round 0 from 2^20 ids and records

__host__ __device__ inline int ceil_log2_i64(int64_t n) {
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

inline TPlan tiled_plan(int64_t n, int64_t m) {
    TPlan p{};
    const int lg = ceil_log2_i64(n < 2 ? 2 : n);
    p.xs = lg - 8 < 0 ? 0 : (lg - 8 > kTxShiftMax ? kTxShiftMax : lg - 8);
    p.ys = lg - 8 < 0 ? 0 : lg - 8;
    p.rows = (int32_t)ceil_div(n < 1 ? 1 : n, (int64_t)1 << p.xs);
    p.cols = (int32_t)ceil_div(n < 1 ? 1 : n, (int64_t)1 << p.ys);
    p.tiles_a = ceil_div(m < 1 ? 1 : m, kTaIn);
    p.tiles_b = ceil_div(2 * (m < 1 ? 1 : m), kTbTile);
    p.tiles_r = ceil_div(m < 1 ? 1 : m, kTrIn);
    return p;
}

inline bool tiled_fits(int64_t n) { return n >= 1 && tiled_plan(n, 1).rows <= kTRowsMax; }

// ---- launchers (lc_kernels.hip, lc_sort.hip, lc_tiled.hip) ------------------------------------------
// `grid` arguments are workgroup counts chosen by the host (grid-stride loops cover the
// rest); every kernel reads its true element count from RoundState.

// seeded: plain solve, rounds >= 1 (node words start at the own priority)
hipError_t launch_round_begin(const Work &w, bool seeded, int round, int grid, hipStream_t s,
                              const uint32_t *tab = nullptr);
// explicit priorities: inv[tab[x]] = x, and err bit 3 when tab is not a permutation of [0, n0)
hipError_t launch_prio_inverse(const Work &w, const uint32_t *tab, int grid, hipStream_t s);
// the parents of the round that just ended, recorded at rec: round 0 as one entry per id (the
// parent's name or kNoParent), later rounds as (name, parent name) pairs of its nodes
hipError_t launch_record_parents(const Work &w, int round, uint32_t *rec, int grid, hipStream_t s);
// expand a record into out[name] = parent name, -1 for names that were not nodes
hipError_t launch_expand_record(const Work &w, int round, const uint32_t *rec, int64_t count, int32_t *out,
                                int grid, hipStream_t s);
// one-hop and two-hop minima of the round that just ended, by name (kInf for other names);
// dense_m1: the tiled round 0's row pass left m1 one value per id and no two-hop word, whose
// value is then the priority of the node's parent (the definition of the parent)
hipError_t launch_dump_minima(const Work &w, int last_round, bool dense_m1, const PrioCtx &p, uint32_t *m1,
                              uint32_t *l2, int grid, hipStream_t s);
hipError_t launch_min1(const Work &w, const EdgeIn *in, const PrioCtx &p, bool batch, int round, int grid,
                       hipStream_t s);
hipError_t launch_min2(const Work &w, const EdgeIn *in, int grid, hipStream_t s);
// one_hop: the parent is the argmin of the one-hop minimum (the one-hop label variant)
hipError_t launch_parent(const Work &w, const PrioCtx &p, bool batch, int round, int grid, hipStream_t s,
                         bool one_hop = false);
// TreeContraction (lc_variants.hip): open one-hop minimum; then f, pointer jumping over at most
// ceil(log2 n_bound) + 2 passes, and the labels
hipError_t launch_min1_open(const Work &w, const EdgeIn *in, const PrioCtx &p, int round, int grid, hipStream_t s);
// dense: after the tiled round 0's row pass (m1 dense, f kept in lab_at)
hipError_t launch_tree_labels(const Work &w, const PrioCtx &p, int round, int64_t n_bound, int grid, hipStream_t s,
                              bool dense = false);
// MergeToLarge (lc_variants.hip): after the LocalContraction step of round `round` (its node
// map built), the class size and priority of every next-round node; then, in the next round,
// the parents of the step (the best large node within two hops)
hipError_t launch_mtl_prep(const Work &w, const PrioCtx &p, int round, uint64_t alpha, int grid_cur, int grid_next,
                           hipStream_t s);
hipError_t launch_mtl_labels(const Work &w, uint64_t alpha, int grid_nodes, int grid_edges, hipStream_t s);
// union-find finish of the graph of round `round` (lc_variants.hip)
hipError_t launch_uf_finish(const Work &w, int round, int grid_nodes, int grid_edges, hipStream_t s);
hipError_t launch_relabel(const Work &w, const EdgeIn *in, int grid, hipStream_t s);
// Tiles of one pass.  Pass 0 reads the relabel output in place: either packed (the tiled
// round 0), or in slabs, where tile t is the (t % 2)-th half of slab t / 2,
// filled from its start with that slab's survivors.  Later passes read a compact array of S
// keys.  In every case the keys of tile t are the first valid(t) positions of
// [t * kSortTile, (t + 1) * kSortTile).
struct Tiles {
    int64_t ntiles;
    int64_t S;
    const uint32_t *slab_cnt;
    bool slab;
    __device__ int valid(int64_t t) const {
        constexpr int kPer = kSlab / kSortTile;
        const int64_t c = slab ? (int64_t)slab_cnt[t / kPer] - (t % kPer) * kSortTile : S - t * kSortTile;
        return c <= 0 ? 0 : (c >= kSortTile ? kSortTile : (int)c);
    }
};

__device__ inline Tiles tiles_of(const Work &w, int pass) {
    const RoundState *st = w.st;
    Tiles t;
    t.S = (int64_t)st->s_keys;
    t.slab = pass == 0 && !st->keys_dense;
    t.slab_cnt = w.slab_cnt;
    t.ntiles = t.slab ? (int64_t)st->n_slabs * (kSlab / kSortTile) : ceil_div(t.S, kSortTile);
    return t;
}

// Sampled-bucket duplicate drop of round 0 (lc_bucket.hip), in place of the radix passes:
// stage 0 first-level splitters (one workgroup), 1 first-level counts, 2 first-level scatter,
// 3 first-level bucket starts and second-level tiles (one workgroup), 4 second-level
// splitters, 5 second-level counts, 6 second-level scatter, 7 sort of each final bucket into
// the buffer the radix passes would have left the keys in.  The count tables are scanned
// between stages 1 and 2 and between 5 and 6 (launch_sort_pass stages 1-3).
constexpr int kBucketLevel2Tiles = 256;   // extra count-table tiles of the second level
hipError_t launch_bucket(const Work &w, int stage, int grid, hipStream_t s);
// Rounds >= 1 that fit the hashed duplicate drop, one after another in one cooperative launch
// (lc_fused.hip).  fused_rounds_grid: cus * min(per_cu, workgroups of the kernel that stay
// resident on a CU), or 0 when not even one does.
enum FusedRule { kFusedLocal = 0, kFusedOneHop = 1, kFusedTree = 2, kFusedMerge = 3 };
int fused_rounds_grid(int rule, int per_cu, int cus);
constexpr int kFusedAlphas = 16;   // MergeToLarge phases whose alpha the persistent launch carries
struct FusedLimits {
    int32_t round_limit;    // rounds from this one on are left to the host
    int32_t n_alphas;       // MergeToLarge: alphas[i] is phase i's, the last repeating
    int64_t finish_edges;   // a graph of at most this many records is left to the union-find finish
    uint64_t alphas[kFusedAlphas];
};
hipError_t launch_fused_rounds(const Work &w, int rule, int grid, FusedLimits lim, hipStream_t s);
// parents -> label ranks, the label of each rank, and the key width of the sort (grid_scan 0:
// the label scan in one workgroup)
hipError_t launch_rank_parents(const Work &w, int grid, int grid_scan, hipStream_t s);
// stage 0 count pass, 1-3 scan of the count table (5: in one workgroup), 4 scatter; the
// one-sweep form: 6 totals and tile counters zeroed (one workgroup), 7 the digit totals of
// every pass, 8 the scatter of pass `pass` with its offsets found by look-back.
// gated (this and the unique): skipped when the round's device-side choice was to hash
// scatter_waves: the radix scatter build to launch (2, 3 or 4 waves per SIMD)
hipError_t launch_sort_pass(const Work &w, int pass, int grid, hipStream_t s, int stage, bool gated = false,
                            int scatter_waves = LC_SCATTER_WAVES);
// prefix counts of the label map (total -> n_labels) or of the next-graph node map over the
// labels (total -> n_next)
hipError_t launch_map_scan(const Work &w, bool labels, int grid, hipStream_t s, int stage);
hipError_t launch_scan_u32(uint32_t *data, uint32_t *partials, const u64c *n, u64c *total, int grid,
                           hipStream_t s, int stage);
hipError_t launch_unique(const Work &w, int grid, hipStream_t s, int stage, bool gated = false);
// duplicate drop by hashing: stage 1 size and clear the table (decide: or choose to sort;
// before a gated sort), 2 insert the relabel's keys, 3 count the kept keys per table tile and
// mark the next graph's nodes, 4 write them renamed into the relabel's buffer (after the tile
// counts and the node map are scanned)
hipError_t launch_hash_dedup(const Work &w, int grid, hipStream_t s, int stage, bool decide = false);
hipError_t launch_nodes(const Work &w, bool batch, int round, int grid, hipStream_t s);
hipError_t launch_map(const Work &w, int round, int grid, hipStream_t s);
// dedup: how the round dropped repeats: kDedupSort, kDedupHash (its edges are then in the
// relabel's buffer) or kDedupDevice (the device chose; hash_slots nonzero: it hashed)
hipError_t launch_round_end(const Work &w, int round, int dedup, hipStream_t s);
// the current graph's edges by name (the graph round `next_round` reads)
hipError_t launch_dump_edges(const Work &w, uint64_t *out, int next_round, int grid, hipStream_t s);
hipError_t launch_compose(const Work &w, bool identity, int cur_round, void *labels, bool out64, bool batch,
                          const uint32_t *voff, int grid, hipStream_t s);
// fold the host-known `levels` per-round maps into map0 and empty the arena
hipError_t launch_flatten(const Work &w, int levels, int grid, hipStream_t s);
hipError_t launch_canonical(const Work &w, void *labels, bool out64, bool batch, const uint32_t *voff, int grid,
                            hipStream_t s);
hipError_t launch_dump_parents(const Work &w, int32_t *out, int last_round, int grid, hipStream_t s);
hipError_t launch_batch_keys(const Work &w, RoundKey *keys, const uint64_t *seeds, int32_t n_graphs, hipStream_t s);
hipError_t launch_fill_gid(uint32_t *gid0, const uint32_t *voff, int32_t n_graphs, int grid, hipStream_t s);
// Tiled round 0.  Partition stages: 0 = pass-A counts, 1..3 = their scan (total ->
// t_count), 4 = pass-A scatter, 5 = pass-B counts, 6..8 = their scan, 9 = pass-B scatter.
// The one-pass row form (no column order inside a row): 10 = counts by row of both directed
// records of every input record, 11..13 = their scan (total -> t_count), 14 = scatter.
hipError_t launch_tiled_partition(const Work &w, const EdgeIn &in, const TPlan &tp, int grid, hipStream_t s,
                                  int stage);
// open: TreeContraction's one-hop minimum without the node's own priority
hipError_t launch_tiled_min1(const Work &w, const PrioCtx &p, const TPlan &tp, hipStream_t s, bool open = false);
// the one-hop label's parents from the row pass's one-hop minima
hipError_t launch_tiled_parent1(const Work &w, const PrioCtx &p, int grid, hipStream_t s);
// gen: rows per launch (the CU count: one 1024-thread, 128 KiB-LDS workgroup each)
// gen: rows launched together (<= 0: all rows in one launch); pairs: record pairs in flight
// per thread (two-hop pass 2, 4 or 8; relabel 1, 2 or 4; other values take the default)
hipError_t launch_tiled_min2(const Work &w, const PrioCtx &p, const TPlan &tp, hipStream_t s, int gen, int pairs);
hipError_t launch_tiled_relabel(const Work &w, const TPlan &tp, hipStream_t s, int gen, int pairs);

// Scan stages: 0 = block sums, 1 = scan of the sums (one workgroup), 2 = block downsweep.
// Sort stages: 0 = digit counts, 1..3 = scan of the counts (or 5: the whole scan in one
// workgroup), 4 = scatter.  Map scans: 0..2 as the generic scan, 3 = all in one workgroup.
// Unique stages: 0 = heads per tile + next-node marks, 1 = scan (one workgroup), 2 = ordered
// write of the heads renamed into the next round's indices (after the node scan and map).

}  // namespace lc
