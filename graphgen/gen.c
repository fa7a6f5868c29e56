/*
 * Seeded synthetic graph generators (harness input only).
 *
 * This file holds no part of the connected-components method: it only draws
 * edge lists.  Both the oracle side and the GPU side consume its output, so it
 * must stay free of any contraction arithmetic.
 *
 * Randomness is counter based.  A stream key is
 *     key(seed, stream) = sm64(seed ^ sm64(stream))
 * and the i-th draw of a stream is sm64(key + i * GOLDEN), i.e. the (i+1)-th
 * output of a SplitMix64 generator (Steele, Lea and Flood, OOPSLA 2014) whose
 * state starts at key.  Integers in [0, n) use the multiply-high reduction of
 * Lemire (2019) on the top 32 bits of a draw (bias at most n / 2^32).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64(uint64_t x) {
    uint64_t z = x + GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gg_sm64(uint64_t x) { return sm64(x); }

uint64_t gg_key(uint64_t seed, uint64_t stream) { return sm64(seed ^ sm64(stream)); }

static inline uint64_t draw(uint64_t key, uint64_t i) { return sm64(key + i * GOLDEN); }

/* uniform integer in [0, n), n <= 2^32 */
static inline uint32_t below(uint64_t x, uint64_t n) {
    return (uint32_t)(((x >> 32) * n) >> 32);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

enum { ST_GNM = 1, ST_PERM = 2, ST_RMAT_NOISE = 3, ST_RMAT_BITS = 4, ST_RMAT_PERM = 5 };

/*
 * Erdos-Renyi G(n, m) records: both endpoints uniform in [0, n) from the
 * seed; duplicates and self-loops are kept.  Writes m records into
 * (src[i], dst[i]) shifted by `id_base`.
 */
void gg_gnm(uint64_t seed, int64_t n, int64_t m, uint32_t id_base, uint32_t *src, uint32_t *dst) {
    const uint64_t key = gg_key(seed, ST_GNM);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        src[i] = id_base + below(draw(key, 2 * (uint64_t)i), (uint64_t)n);
        dst[i] = id_base + below(draw(key, 2 * (uint64_t)i + 1), (uint64_t)n);
    }
}

/* Fisher-Yates permutation of [0, n) driven by stream `stream` of `seed`. */
void gg_permutation(uint64_t seed, uint64_t stream, int64_t n, uint32_t *perm) {
    const uint64_t key = gg_key(seed, stream);
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = below(draw(key, (uint64_t)i), (uint64_t)(i + 1));
        uint32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

/*
 * `count` disjoint paths of `length` vertices on fresh ids
 * [id_base, id_base + count*length).  The fresh ids are shuffled by a seeded
 * permutation and path j visits perm[j*length .. j*length+length-1] in order.
 * Writes count*(length-1) records.
 */
void gg_paths(uint64_t seed, int64_t count, int64_t length, uint32_t id_base, uint32_t *src,
              uint32_t *dst) {
    const int64_t nv = count * length;
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
    gg_permutation(seed, ST_PERM, nv, perm);
    const int64_t per = length - 1;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < count; ++j) {
        for (int64_t k = 0; k < per; ++k) {
            src[j * per + k] = id_base + perm[j * length + k];
            dst[j * per + k] = id_base + perm[j * length + k + 1];
        }
    }
    free(perm);
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with 2^scale vertices and
 * m records.  Quadrant probabilities (a, b, c, d) are perturbed once per level
 * per graph: each is multiplied by (1 + u), u uniform in [-noise, noise], and
 * the four are renormalised.  Each record descends `scale` levels, one 32-bit
 * uniform per level.  Finally ids are relabelled by a seeded Fisher-Yates
 * permutation when `permute` is set.  Duplicates and self-loops are kept.
 */
void gg_rmat(uint64_t seed, int32_t scale, int64_t m, double a, double b, double c, double d,
             double noise, int32_t permute, uint32_t id_base, uint32_t *src, uint32_t *dst) {
    double ca[64], cb[64], cc[64]; /* cumulative thresholds per level */
    const uint64_t nkey = gg_key(seed, ST_RMAT_NOISE);
    for (int l = 0; l < scale; ++l) {
        double q[4] = {a, b, c, d};
        double s = 0.0;
        for (int k = 0; k < 4; ++k) {
            double u = (2.0 * unit(draw(nkey, (uint64_t)(4 * l + k))) - 1.0) * noise;
            q[k] *= 1.0 + u;
            s += q[k];
        }
        ca[l] = q[0] / s;
        cb[l] = (q[0] + q[1]) / s;
        cc[l] = (q[0] + q[1] + q[2]) / s;
    }
    const uint64_t bkey = gg_key(seed, ST_RMAT_BITS);
    const int draws = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint32_t u = 0, v = 0;
        for (int k = 0; k < draws; ++k) {
            uint64_t x = draw(bkey, (uint64_t)i * (uint64_t)draws + (uint64_t)k);
            for (int h = 0; h < 2; ++h) {
                int l = 2 * k + h;
                if (l >= scale) break;
                double r = (double)(uint32_t)(x >> (32 * h)) * (1.0 / 4294967296.0);
                uint32_t bit = 1u << (scale - 1 - l);
                if (r < ca[l]) {
                } else if (r < cb[l]) {
                    v |= bit;
                } else if (r < cc[l]) {
                    u |= bit;
                } else {
                    u |= bit;
                    v |= bit;
                }
            }
        }
        src[i] = u;
        dst[i] = v;
    }
    if (permute) {
        int64_t n = (int64_t)1 << scale;
        uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
        gg_permutation(seed, ST_RMAT_PERM, n, perm);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            src[i] = id_base + perm[src[i]];
            dst[i] = id_base + perm[dst[i]];
        }
        free(perm);
    } else if (id_base) {
        for (int64_t i = 0; i < m; ++i) {
            src[i] += id_base;
            dst[i] += id_base;
        }
    }
}

/* Raw draws of a stream, for the Python side (batch mixes, traces). */
void gg_draws(uint64_t seed, uint64_t stream, int64_t start, int64_t count, uint64_t *out) {
    const uint64_t key = gg_key(seed, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = draw(key, (uint64_t)(start + i));
}

/* Pack SoA int32 records into u64 keys (src << 32 | dst). */
void gg_pack(int64_t m, const uint32_t *src, const uint32_t *dst, uint64_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) out[i] = ((uint64_t)src[i] << 32) | dst[i];
}
