/*
 * CPU oracle for LocalContraction (Lacki, Mirrokni, Wlodarczyk, "Connected
 * Components at Scale via Local Contractions", arXiv 1807.10727).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never does.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * What it computes, phase by phase (Section 3, paragraph "LocalContraction";
 * Section 2 for the closed neighbourhood N(v) that contains v):
 *   1. a random ordering rho of the current nodes is drawn (a keyed hash of
 *      the node name, or a caller-given table);
 *   2. every node v gets the label l(v) = the vertex of smallest priority in
 *      N(N(v)), found here as an argmin over the closed neighbourhood taken
 *      twice;
 *   3. nodes with equal labels are merged; the merged graph keeps an edge
 *      between two different labels and drops loops and duplicates (proof of
 *      the contraction-step lemma in Section 3);
 *   4. the loop ends when no edge is left (each component is one node).
 * Nodes that end up with no edge are final (Section 6 drops isolated nodes
 * after each phase).  The labels of the original vertices are the composition
 * of the per-phase maps.
 *
 * Two other ways to choose the labels of step 2 share steps 1, 3 and 4:
 *   - TreeContraction (Section 3, paragraph "TreeContraction"): every node v
 *     points to f(v), the vertex of smallest priority in N(v) \ {v}; nodes in
 *     the same weakly connected component of the graph of f are merged.  The
 *     merged node is named by the component's vertex of smallest priority
 *     (a reading: the paper names no representative);
 *   - the one-hop label (Section 6, the Cracker-equivalent rule without its
 *     edge rewiring): the vertex of smallest priority in the closed N(v).
 *   - MergeToLarge (Section 5, paragraph "MergeToLarge step"): every
 *     LocalContraction phase is followed by a step on the graph it left.  A node
 *     of that graph is large when its class had at least alpha_i nodes (alpha_i
 *     given per phase i); its priority is the alpha_i-th largest priority of its
 *     members in that phase.  Each node takes as its label the large node of
 *     largest priority within distance 2 (itself included), or keeps itself when
 *     there is none, and nodes with equal labels merge.  In the statistics, phase
 *     i is round 2i (LocalContraction, priorities of round 2i) and its step is
 *     round 2i+1 (reading: merging means equal labels, as in LocalContraction; a
 *     large node may itself move to another large node).
 * And an optional finish (Section 6): once a phase leaves at most
 * `finish_edges` edges, the components of what is left are found by
 * union-find, and each is named by its smallest name.
 *
 * Readings of points the paper leaves open (all shared with the GPU library
 * by specification only, never by code):
 *   - a merged node is named by the original id of its label vertex;
 *   - the priority of node x in phase r is
 *       fmix32(fmix32(x ^ k0) ^ k1),  (k1:k0) = sm64(seed ^ sm64(r)),
 *     with SplitMix64's output function sm64 (Steele, Lea, Flood 2014) and
 *     MurmurHash3's 32-bit finaliser fmix32 (Appleby), compared as unsigned;
 *   - records are undirected pairs; round-0 loops and duplicates are allowed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t round;
    int32_t pad_;
    int64_t n_active;    /* nodes with at least one loop-free edge in this phase */
    int64_t m_in;        /* records read: raw input count in phase 0, |E_r| after */
    int64_t m_survive;   /* records whose endpoints get different labels (repeats counted) */
    int64_t m_out;       /* distinct loop-free edges of the next graph */
    int64_t n_finalised; /* distinct labels of this phase that keep no edge */
} lco_round_stats;

/* ---- priority specification ------------------------------------------- */

static uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

uint64_t lco_sm64(uint64_t x) { return sm64(x); }
uint32_t lco_fmix32(uint32_t x) { return fmix32(x); }

uint32_t lco_priority(uint64_t seed, int32_t round, uint32_t name) {
    uint64_t k = sm64(seed ^ sm64((uint64_t)(uint32_t)round));
    return fmix32(fmix32(name ^ (uint32_t)k) ^ (uint32_t)(k >> 32));
}

/* ---- helpers ------------------------------------------------------------ */

static int cmp_u64(const void *x, const void *y) {
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

static uint64_t edge_key(uint32_t a, uint32_t b) {
    uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    return ((uint64_t)lo << 32) | hi;
}

/* sort and drop repeats; returns the new length */
static int64_t sort_unique(uint64_t *k, int64_t n) {
    if (n == 0) return 0;
    qsort(k, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t w = 1;
    for (int64_t i = 1; i < n; ++i)
        if (k[i] != k[w - 1]) k[w++] = k[i];
    return w;
}

#define LCO_LOCAL 0     /* LocalContraction */
#define LCO_TREE 1      /* TreeContraction */
#define LCO_ONE_HOP 2   /* one-hop label */
#define LCO_MTL 3       /* LocalContraction phases, each followed by a MergeToLarge step */

/* union-find over names (path halving), for the TreeContraction components and the finish */
static uint32_t uf_find(uint32_t *up, uint32_t x) {
    while (up[x] != x) {
        up[x] = up[up[x]];
        x = up[x];
    }
    return x;
}

static void uf_union(uint32_t *up, uint32_t a, uint32_t b) {
    a = uf_find(up, a);
    b = uf_find(up, b);
    if (a != b) up[a < b ? b : a] = a < b ? a : b;
}

/*
 * Run LocalContraction (or a variant) on n0 vertices and m0 records (src[i], dst[i]).
 *
 *   explicit_prio  optional [prio_rows][n0] table; phase r uses row
 *                  min(r, prio_rows-1); values must be distinct on the nodes
 *                  of each phase.  NULL means the hashed priority above.
 *   max_rounds     0 = until no edge is left, else stop after that many.
 *   labels         out [n0]: name of the node each vertex belongs to.
 *   stats          out [stats_cap] per-phase statistics (may be NULL).
 *   parents        out [parents_cap][n0]: label vertex of every node of the
 *                  phase, 0xFFFFFFFF for names that are not nodes of it
 *                  (may be NULL).
 *   variant        LCO_LOCAL, LCO_TREE, LCO_ONE_HOP or LCO_MTL.
 *   finish_edges   0, or: before every phase after the first, if at most this
 *                  many edges are left, finish with union-find instead.
 *   finished       out (may be NULL): 1 when the finish ran.
 *   m1_rows, l_rows  out (may be NULL): [minima_cap][n0] one-hop and two-hop
 *                  minimum priorities of every node of each phase (not for
 *                  TreeContraction; the one-hop label's two-hop row repeats the
 *                  one-hop row), 0xFFFFFFFF for names that are not nodes.
 * Returns the number of phases run, or -1 on bad input / out of memory.
 */
int32_t lco_run_full(int64_t n0, int64_t m0, const uint32_t *src, const uint32_t *dst, uint64_t seed,
                     const uint32_t *explicit_prio, int32_t prio_rows, int32_t max_rounds,
                     uint32_t *labels, lco_round_stats *stats, int32_t stats_cap, uint32_t *parents,
                     int32_t parents_cap, int32_t variant, int64_t finish_edges, int32_t *finished,
                     uint32_t *m1_rows, uint32_t *l_rows, int32_t minima_cap, const int64_t *alphas,
                     int32_t n_alphas) {
    if (variant < LCO_LOCAL || variant > LCO_MTL) return -1;
    if (variant == LCO_MTL && (!alphas || n_alphas < 1)) return -1;
    if (finished) *finished = 0;
    if (n0 < 0 || m0 < 0 || n0 > 0xFFFFFFFFLL) return -1;
    for (int64_t i = 0; i < m0; ++i)
        if ((int64_t)src[i] >= n0 || (int64_t)dst[i] >= n0) return -1;

    const size_t nn = (size_t)(n0 > 0 ? n0 : 1);
    uint64_t *E = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m0 > 0 ? m0 : 1));
    uint64_t *E2 = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m0 > 0 ? m0 : 1));
    uint8_t *in_v = (uint8_t *)malloc(nn);
    uint8_t *is_label = (uint8_t *)malloc(nn);
    uint8_t *in_next = (uint8_t *)malloc(nn);
    uint32_t *rho = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    uint32_t *m1_val = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    uint32_t *m1_arg = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    uint32_t *l_val = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    uint32_t *l_arg = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    uint32_t *up = (uint32_t *)malloc(sizeof(uint32_t) * nn);
    /* MergeToLarge: class size, priority and "large" of each name, and (class, priority) pairs */
    const int mtl = variant == LCO_MTL;
    uint32_t *mtl_prio = (uint32_t *)malloc(mtl ? sizeof(uint32_t) * nn : 1);
    uint8_t *mtl_large = (uint8_t *)malloc(mtl ? nn : 1);
    uint64_t *mtl_pairs = (uint64_t *)malloc(mtl ? sizeof(uint64_t) * nn : 1);
    if (!E || !E2 || !in_v || !is_label || !in_next || !rho || !m1_val || !m1_arg || !l_val || !l_arg || !up ||
        !mtl_prio || !mtl_large || !mtl_pairs) {
        free(E); free(E2); free(in_v); free(is_label); free(in_next);
        free(rho); free(m1_val); free(m1_arg); free(l_val); free(l_arg); free(up);
        free(mtl_prio); free(mtl_large); free(mtl_pairs);
        return -1;
    }

    for (int64_t v = 0; v < n0; ++v) labels[v] = (uint32_t)v;

    /* E_0: the set of unordered loop-free pairs of the input */
    int64_t mE = 0;
    for (int64_t i = 0; i < m0; ++i)
        if (src[i] != dst[i]) E[mE++] = edge_key(src[i], dst[i]);
    mE = sort_unique(E, mE);

    int32_t r = 0;
    while (mE > 0 && (max_rounds <= 0 || r < max_rounds)) {
        if (finish_edges > 0 && r > 0 && mE <= finish_edges) {
            /* Section 6: the small remaining graph's components by union-find; a
               component is named by its smallest name */
            for (int64_t x = 0; x < n0; ++x) up[x] = (uint32_t)x;
            for (int64_t i = 0; i < mE; ++i) uf_union(up, (uint32_t)(E[i] >> 32), (uint32_t)E[i]);
            memset(in_v, 0, nn);
            for (int64_t i = 0; i < mE; ++i) {
                in_v[E[i] >> 32] = 1;
                in_v[(uint32_t)E[i]] = 1;
            }
            /* linking the larger root under the smaller keeps every root the smallest
               name of its component */
            for (int64_t v = 0; v < n0; ++v)
                if (in_v[labels[v]]) labels[v] = uf_find(up, labels[v]);
            if (finished) *finished = 1;
            mE = 0;
            break;
        }
        /* V_r: endpoints of the current edges */
        memset(in_v, 0, nn);
        for (int64_t i = 0; i < mE; ++i) {
            in_v[E[i] >> 32] = 1;
            in_v[(uint32_t)E[i]] = 1;
        }
        int64_t n_active = 0;
        for (int64_t x = 0; x < n0; ++x) {
            if (!in_v[x]) continue;
            ++n_active;
            if (explicit_prio) {
                int32_t row = r < prio_rows ? r : prio_rows - 1;
                rho[x] = explicit_prio[(int64_t)row * n0 + x];
            } else {
                rho[x] = lco_priority(seed, r, (uint32_t)x);
            }
        }

        const int mtl_step = mtl && (r & 1);
        if (mtl_step) {
            /* MergeToLarge step (Section 5, run at the end of the previous LocalContraction
               step on the graph it left): a node takes as its label the large node of largest
               priority within distance 2, or keeps itself when there is none.  m1: best
               candidate in the closed N(x) (in_next flags "has one"); l: best over N(N(x))
               (is_label flags "has one"). */
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) {
                    in_next[x] = mtl_large[x];
                    m1_val[x] = mtl_prio[x];
                    m1_arg[x] = (uint32_t)x;
                }
            for (int64_t i = 0; i < mE; ++i) {
                uint32_t a = (uint32_t)(E[i] >> 32), b = (uint32_t)E[i];
                if (mtl_large[b] && (!in_next[a] || mtl_prio[b] > m1_val[a])) {
                    in_next[a] = 1; m1_val[a] = mtl_prio[b]; m1_arg[a] = b;
                }
                if (mtl_large[a] && (!in_next[b] || mtl_prio[a] > m1_val[b])) {
                    in_next[b] = 1; m1_val[b] = mtl_prio[a]; m1_arg[b] = a;
                }
            }
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) {
                    is_label[x] = in_next[x];
                    l_val[x] = m1_val[x];
                    l_arg[x] = m1_arg[x];
                }
            for (int64_t i = 0; i < mE; ++i) {
                uint32_t a = (uint32_t)(E[i] >> 32), b = (uint32_t)E[i];
                if (in_next[b] && (!is_label[a] || m1_val[b] > l_val[a])) {
                    is_label[a] = 1; l_val[a] = m1_val[b]; l_arg[a] = m1_arg[b];
                }
                if (in_next[a] && (!is_label[b] || m1_val[a] > l_val[b])) {
                    is_label[b] = 1; l_val[b] = m1_val[a]; l_arg[b] = m1_arg[a];
                }
            }
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x] && !is_label[x]) l_arg[x] = (uint32_t)x;
        } else if (variant == LCO_TREE) {
            /* f(v): argmin of rho over the neighbours other than v (every node of
               the phase has one: the edges are loop-free) */
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) { m1_val[x] = 0xFFFFFFFFu; m1_arg[x] = (uint32_t)x; }
            for (int64_t i = 0; i < mE; ++i) {
                uint32_t a = (uint32_t)(E[i] >> 32), b = (uint32_t)E[i];
                if (m1_arg[a] == (uint32_t)a || rho[b] < m1_val[a]) { m1_val[a] = rho[b]; m1_arg[a] = b; }
                if (m1_arg[b] == (uint32_t)b || rho[a] < m1_val[b]) { m1_val[b] = rho[a]; m1_arg[b] = a; }
            }
            /* weakly connected components of the graph v -> f(v) */
            for (int64_t x = 0; x < n0; ++x) up[x] = (uint32_t)x;
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) uf_union(up, (uint32_t)x, m1_arg[x]);
            /* each component's vertex of smallest priority names it */
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) l_val[x] = 0xFFFFFFFFu;
            for (int64_t x = 0; x < n0; ++x) {
                if (!in_v[x]) continue;
                uint32_t c = uf_find(up, (uint32_t)x);
                if (l_val[c] == 0xFFFFFFFFu || rho[x] < rho[l_arg[c]]) { l_val[c] = 0; l_arg[c] = (uint32_t)x; }
            }
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) m1_val[x] = l_arg[uf_find(up, (uint32_t)x)];
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) l_arg[x] = m1_val[x];
        } else {
            /* closed one-hop argmin: v itself, then every neighbour */
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) { m1_val[x] = rho[x]; m1_arg[x] = (uint32_t)x; }
            for (int64_t i = 0; i < mE; ++i) {
                uint32_t a = (uint32_t)(E[i] >> 32), b = (uint32_t)E[i];
                if (rho[b] < m1_val[a]) { m1_val[a] = rho[b]; m1_arg[a] = b; }
                if (rho[a] < m1_val[b]) { m1_val[b] = rho[a]; m1_arg[b] = a; }
            }
            /* LocalContraction: the same over the one-hop results, argmin of rho
               over N(N(v)); the one-hop label stops here */
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) { l_val[x] = m1_val[x]; l_arg[x] = m1_arg[x]; }
            if (variant == LCO_LOCAL || variant == LCO_MTL) {
                for (int64_t i = 0; i < mE; ++i) {
                    uint32_t a = (uint32_t)(E[i] >> 32), b = (uint32_t)E[i];
                    if (m1_val[b] < l_val[a]) { l_val[a] = m1_val[b]; l_arg[a] = m1_arg[b]; }
                    if (m1_val[a] < l_val[b]) { l_val[b] = m1_val[a]; l_arg[b] = m1_arg[a]; }
                }
            }
        }
        /* l_arg[x] is now the label vertex (parent) of node x */

        /* optional: the one-hop and two-hop minimum priorities of every node (the values
           whose argmin the labels are), 0xFFFFFFFF for names that are not nodes */
        if (m1_rows && l_rows && variant != LCO_TREE && !mtl_step && r < minima_cap) {
            uint32_t *row1 = m1_rows + (int64_t)r * n0, *row2 = l_rows + (int64_t)r * n0;
            for (int64_t x = 0; x < n0; ++x) {
                row1[x] = in_v[x] ? m1_val[x] : 0xFFFFFFFFu;
                row2[x] = in_v[x] ? l_val[x] : 0xFFFFFFFFu;
            }
        }

        if (parents && r < parents_cap) {
            uint32_t *row = parents + (int64_t)r * n0;
            for (int64_t x = 0; x < n0; ++x) row[x] = in_v[x] ? l_arg[x] : 0xFFFFFFFFu;
        }

        /* records that survive relabelling (repeats counted) */
        int64_t m_in, survive = 0;
        if (r == 0) {
            m_in = m0;
            for (int64_t i = 0; i < m0; ++i)
                if (src[i] != dst[i] && l_arg[src[i]] != l_arg[dst[i]]) ++survive;
        } else {
            m_in = mE;
            for (int64_t i = 0; i < mE; ++i)
                if (l_arg[E[i] >> 32] != l_arg[(uint32_t)E[i]]) ++survive;
        }

        /* next graph: relabel endpoints, drop loops and duplicates */
        int64_t m2 = 0;
        for (int64_t i = 0; i < mE; ++i) {
            uint32_t pa = l_arg[E[i] >> 32], pb = l_arg[(uint32_t)E[i]];
            if (pa != pb) E2[m2++] = edge_key(pa, pb);
        }
        m2 = sort_unique(E2, m2);

        /* labels that keep no edge are final */
        memset(is_label, 0, nn);
        memset(in_next, 0, nn);
        for (int64_t x = 0; x < n0; ++x)
            if (in_v[x]) is_label[l_arg[x]] = 1;
        for (int64_t i = 0; i < m2; ++i) {
            in_next[E2[i] >> 32] = 1;
            in_next[(uint32_t)E2[i]] = 1;
        }
        int64_t n_labels = 0, n_next = 0;
        for (int64_t x = 0; x < n0; ++x) {
            n_labels += is_label[x];
            n_next += in_next[x];
        }

        /* MergeToLarge, after a LocalContraction step: the nodes this step created are the
           classes of equal labels; a class of at least alpha nodes is large, and its priority
           is the alpha-th largest priority of its members in this step (Section 5).  The
           pairs (label, complement of the priority) sort each class by falling priority. */
        if (mtl && !mtl_step) {
            const int32_t ph = r / 2;
            const int64_t alpha = alphas[ph < n_alphas ? ph : n_alphas - 1];
            int64_t np = 0;
            for (int64_t x = 0; x < n0; ++x)
                if (in_v[x]) mtl_pairs[np++] = ((uint64_t)l_arg[x] << 32) | (uint64_t)(uint32_t)~rho[x];
            qsort(mtl_pairs, (size_t)np, sizeof(uint64_t), cmp_u64);
            memset(mtl_large, 0, nn);
            for (int64_t i = 0; i < np;) {
                int64_t j = i;
                while (j < np && (mtl_pairs[j] >> 32) == (mtl_pairs[i] >> 32)) ++j;
                const uint32_t y = (uint32_t)(mtl_pairs[i] >> 32);
                if (alpha >= 1 && j - i >= alpha) {
                    mtl_large[y] = 1;
                    mtl_prio[y] = ~(uint32_t)mtl_pairs[i + alpha - 1];
                }
                i = j;
            }
        }

        /* compose: a vertex whose node took part in this phase moves to its label */
        for (int64_t v = 0; v < n0; ++v)
            if (in_v[labels[v]]) labels[v] = l_arg[labels[v]];

        if (stats && r < stats_cap) {
            lco_round_stats *s = &stats[r];
            s->round = r;
            s->pad_ = 0;
            s->n_active = n_active;
            s->m_in = m_in;
            s->m_survive = survive;
            s->m_out = m2;
            s->n_finalised = n_labels - n_next;
        }

        uint64_t *t = E; E = E2; E2 = t;
        mE = m2;
        ++r;
    }

    free(E); free(E2); free(in_v); free(is_label); free(in_next);
    free(rho); free(m1_val); free(m1_arg); free(l_val); free(l_arg); free(up);
    free(mtl_prio); free(mtl_large); free(mtl_pairs);
    return r;
}

int32_t lco_run_variant(int64_t n0, int64_t m0, const uint32_t *src, const uint32_t *dst, uint64_t seed,
                        const uint32_t *explicit_prio, int32_t prio_rows, int32_t max_rounds,
                        uint32_t *labels, lco_round_stats *stats, int32_t stats_cap, uint32_t *parents,
                        int32_t parents_cap, int32_t variant, int64_t finish_edges, int32_t *finished) {
    return lco_run_full(n0, m0, src, dst, seed, explicit_prio, prio_rows, max_rounds, labels, stats, stats_cap,
                        parents, parents_cap, variant, finish_edges, finished, NULL, NULL, 0, NULL, 0);
}

int32_t lco_run(int64_t n0, int64_t m0, const uint32_t *src, const uint32_t *dst, uint64_t seed,
                const uint32_t *explicit_prio, int32_t prio_rows, int32_t max_rounds,
                uint32_t *labels, lco_round_stats *stats, int32_t stats_cap, uint32_t *parents,
                int32_t parents_cap) {
    return lco_run_variant(n0, m0, src, dst, seed, explicit_prio, prio_rows, max_rounds, labels, stats, stats_cap,
                           parents, parents_cap, LCO_LOCAL, 0, NULL);
}

/*
 * Independent graphs packed in one arena (local ids per graph), each run on
 * its own with its own seed: graph g has n = voff[g+1]-voff[g] vertices and
 * records eoff[g] .. eoff[g+1]-1.  labels and rounds are written per graph;
 * parents (optional) as [parents_cap][n_g] blocks starting at
 * voff[g]*parents_cap.  Returns 0, or -1 if any graph failed.
 */
int32_t lco_run_batch(int64_t n_graphs, const int64_t *voff, const int64_t *eoff, const uint32_t *src,
                      const uint32_t *dst, const uint64_t *seeds, uint32_t *labels, int32_t *rounds,
                      uint32_t *parents, int32_t parents_cap) {
    int32_t status = 0;
    for (int64_t g = 0; g < n_graphs; ++g) {
        int64_t n = voff[g + 1] - voff[g];
        int64_t m = eoff[g + 1] - eoff[g];
        int32_t rr = lco_run(n, m, src + eoff[g], dst + eoff[g], seeds[g], NULL, 0, 0, labels + voff[g], NULL, 0,
                             parents ? parents + voff[g] * parents_cap : NULL, parents_cap);
        if (rr < 0) status = -1;
        rounds[g] = rr;
    }
    return status;
}

/*
 * Textbook union-find (union by size, path halving) over the records: writes
 * for every vertex the smallest vertex id of its connected component.  Used to
 * check the partition of large runs, where the phase-by-phase oracle is slow.
 */
int32_t lco_components_min_id(int64_t n, int64_t m, const uint32_t *src, const uint32_t *dst, uint32_t *out) {
    uint32_t *parent = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *size = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    if (!parent || !size) {
        free(parent);
        free(size);
        return -1;
    }
    for (int64_t v = 0; v < n; ++v) {
        parent[v] = (uint32_t)v;
        size[v] = 1;
    }
    for (int64_t i = 0; i < m; ++i) {
        if ((int64_t)src[i] >= n || (int64_t)dst[i] >= n) {
            free(parent);
            free(size);
            return -1;
        }
        uint32_t a = src[i], b = dst[i];
        while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
        while (parent[b] != b) { parent[b] = parent[parent[b]]; b = parent[b]; }
        if (a == b) continue;
        if (size[a] < size[b]) { uint32_t t = a; a = b; b = t; }
        parent[b] = a;
        size[a] += size[b];
    }
    /* smallest id per root: vertices are visited in increasing order */
    for (int64_t v = 0; v < n; ++v) out[v] = 0xFFFFFFFFu;
    for (int64_t v = 0; v < n; ++v) {
        uint32_t r = (uint32_t)v;
        while (parent[r] != r) r = parent[r];
        if (out[r] == 0xFFFFFFFFu) out[r] = (uint32_t)v;
        out[v] = out[r];
    }
    free(parent);
    free(size);
    return 0;
}
