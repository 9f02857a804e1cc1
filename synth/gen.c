/*
 * Seeded synthetic workload generators for MAP accepting-cycle detection.
 *
 * This module produces input graphs only: edge lists (s -> d of the generated
 * state graph G, ids 1..n, 0 meaning "none") and accepting flags.  It contains
 * none of the MAP arithmetic; the CPU oracle and the HIP library both consume
 * the arrays it writes.
 *
 * The paper measures on DVE models that are not available here, and gives no
 * graph sizes (Section 3, Table 1).  These generators stand in for them:
 *   config 1  uniform random digraph, out-degree U{1..4}, 5% accepting;
 *             variant "dag" keeps only edges from a higher to a lower id.
 *   config 2  state-space-shaped graph in BFS order: out-degree 1+Poisson(3),
 *             80% local (offset <= 1024) / 20% uniform edges, 90% forward /
 *             10% back, 1% accepting.  Back edges never span an accepting id,
 *             so variant B has no accepting cycle; variant A adds one planted
 *             accepting 64-cycle.
 *   config 3  large DAG: vertex v >= 2 draws U{1..7} edges to U[1, v-1],
 *             0.1% accepting (no accepting cycle by construction).
 *   config 4  one graph of a batch: log-uniform n in [1e3, 1e6], config-1
 *             draw in DAG form, 5% accepting, odd graph indices get a planted
 *             accepting 64-cycle.
 *   config 5  one query of a serving stream: log-uniform n in [1e4, 4e6],
 *             accepting ratio U[0.1%, 5%], config-4 recipe.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), bounded
 * integers by Lemire's multiply-shift with rejection (ACM TOMACS 2019),
 * Poisson by sequential inversion of the CDF, k-of-n sampling by Floyd's
 * algorithm.  Every purpose draws from its own stream derived from the seed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct {
    int32_t n;
    int64_t m;
    int32_t *src;
    int32_t *dst;
    uint8_t *acc;
    int32_t n_acc;
    int32_t n_planted;
    int32_t planted[64];
} synth_graph;

/* ---------------------------------------------------------------- RNG --- */

typedef struct { uint64_t s; } rng_t;

static uint64_t sm_next(rng_t *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* One stream per (seed, purpose): the state is the seed mixed with a tag. */
static rng_t stream(uint64_t seed, uint64_t tag) {
    rng_t r = { seed * 0xD1B54A32D192ED03ull + tag * 0x8CB92BA72F3D8DD7ull + 1 };
    sm_next(&r);
    return r;
}

/* Uniform integer in [0, range), range >= 1 (Lemire). */
static uint64_t below(rng_t *r, uint64_t range) {
    uint64_t x = sm_next(r);
    __uint128_t mm = (__uint128_t)x * range;
    uint64_t lo = (uint64_t)mm;
    if (lo < range) {
        uint64_t t = (0 - range) % range;
        while (lo < t) {
            x = sm_next(r);
            mm = (__uint128_t)x * range;
            lo = (uint64_t)mm;
        }
    }
    return (uint64_t)(mm >> 64);
}

/* Uniform integer in [lo, hi], lo <= hi. */
static int64_t uni(rng_t *r, int64_t lo, int64_t hi) {
    return lo + (int64_t)below(r, (uint64_t)(hi - lo + 1));
}

static double unit(rng_t *r) { return (double)(sm_next(r) >> 11) * (1.0 / 9007199254740992.0); }

static int poisson(rng_t *r, double lambda) {
    double u = unit(r), p = exp(-lambda), f = p;
    int k = 0;
    while (u > f && k < 200) {
        k++;
        p *= lambda / k;
        f += p;
    }
    return k;
}

/* Floyd: mark exactly k distinct ids of [lo, hi] in mark[id - lo]. */
static void floyd(rng_t *r, int64_t lo, int64_t hi, int64_t k, uint8_t *mark) {
    int64_t n = hi - lo + 1;
    for (int64_t j = n - k; j < n; ++j) {
        int64_t t = (int64_t)below(r, (uint64_t)(j + 1));
        if (mark[t]) mark[j] = 1; else mark[t] = 1;
    }
}

/* ------------------------------------------------------- edge buffer --- */

typedef struct { int32_t *s, *d; int64_t m, cap; } ebuf;

static int eb_push(ebuf *b, int32_t s, int32_t d) {
    if (b->m == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        int32_t *ns = (int32_t *)realloc(b->s, (size_t)nc * 4);
        if (!ns) return -1;
        b->s = ns;
        int32_t *nd = (int32_t *)realloc(b->d, (size_t)nc * 4);
        if (!nd) return -1;
        b->d = nd;
        b->cap = nc;
    }
    b->s[b->m] = s;
    b->d[b->m] = d;
    b->m++;
    return 0;
}

static int eb_reserve(ebuf *b, int64_t cap) {
    if (cap <= b->cap) return 0;
    int32_t *ns = (int32_t *)realloc(b->s, (size_t)cap * 4);
    if (!ns) return -1;
    b->s = ns;
    int32_t *nd = (int32_t *)realloc(b->d, (size_t)cap * 4);
    if (!nd) return -1;
    b->d = nd;
    b->cap = cap;
    return 0;
}

static void finish(synth_graph *g, ebuf *b, int32_t n, uint8_t *acc) {
    g->n = n;
    g->m = b->m;
    g->src = b->s;
    g->dst = b->d;
    g->acc = acc;
    int32_t c = 0;
    for (int32_t i = 0; i < n; ++i) c += acc[i];
    g->n_acc = c;
}

void synth_free(synth_graph *g) {
    free(g->src);
    free(g->dst);
    free(g->acc);
    memset(g, 0, sizeof(*g));
}

enum { TAG_ACC = 1, TAG_EDGES = 2, TAG_PLANT = 3, TAG_SIZE = 4, TAG_RATIO = 5 };

/* Accepting set with exactly k members, acc[i] for id i+1. */
static uint8_t *draw_accepting(uint64_t seed, int32_t n, int64_t k) {
    uint8_t *acc = (uint8_t *)calloc((size_t)n, 1);
    if (!acc) return NULL;
    if (k > n) k = n;
    if (k > 0) {
        rng_t r = stream(seed, TAG_ACC);
        floyd(&r, 1, n, k, acc);
    }
    return acc;
}

/* A planted 64-cycle through one accepting vertex: c0 drawn from the accepting
 * set, 63 further distinct ids drawn from the rest, in random order. */
static int plant_random_cycle(uint64_t seed, int32_t n, const uint8_t *acc, ebuf *b, synth_graph *g) {
    g->n_planted = 0;
    if (n < 64) return 0;
    int32_t nacc = 0;
    for (int32_t i = 0; i < n; ++i) nacc += acc[i];
    if (nacc == 0) return 0;
    rng_t r = stream(seed, TAG_PLANT);
    int64_t pick = (int64_t)below(&r, (uint64_t)nacc);
    int32_t c0 = 0;
    for (int32_t i = 0; i < n; ++i)
        if (acc[i] && pick-- == 0) { c0 = i + 1; break; }
    int32_t cyc[64];
    cyc[0] = c0;
    int k = 1;
    while (k < 64) {
        int32_t c = (int32_t)uni(&r, 1, n);
        int dup = 0;
        for (int j = 0; j < k; ++j) dup |= (cyc[j] == c);
        if (!dup) cyc[k++] = c;
    }
    for (int i = 0; i < 64; ++i) {
        if (eb_push(b, cyc[i], cyc[(i + 1) & 63])) return -1;
        g->planted[i] = cyc[i];
    }
    g->n_planted = 64;
    return 0;
}

/* ---------------------------------------------------------- config 1 --- */

/* Config-1 draw: every v in 1..n gets U{dmin..dmax} edges to U[1, n].
 * dag != 0 keeps only edges with s > d (the same draw, filtered). */
static int config1_edges(uint64_t seed, int32_t n, int dmin, int dmax, int dag, ebuf *b) {
    rng_t r = stream(seed, TAG_EDGES);
    if (eb_reserve(b, (int64_t)n * (dmin + dmax) / (dag ? 4 : 2) + 16)) return -1;
    for (int32_t v = 1; v <= n; ++v) {
        int d = (int)uni(&r, dmin, dmax);
        for (int j = 0; j < d; ++j) {
            int32_t t = (int32_t)uni(&r, 1, n);
            if (dag && !(v > t)) continue;
            if (eb_push(b, v, t)) return -1;
        }
    }
    return 0;
}

int synth_config1(uint64_t seed, int32_t n, int dag, synth_graph *g) {
    memset(g, 0, sizeof(*g));
    if (n < 1) return -1;
    uint8_t *acc = draw_accepting(seed, n, (int64_t)n * 5 / 100);
    if (!acc) return -1;
    ebuf b = {0};
    if (config1_edges(seed, n, 1, 4, dag, &b)) { free(acc); free(b.s); free(b.d); return -1; }
    finish(g, &b, n, acc);
    return 0;
}

/* ---------------------------------------------------------- config 2 --- */

int synth_config2(uint64_t seed, int32_t n, int planted, synth_graph *g) {
    memset(g, 0, sizeof(*g));
    if (n < 2) return -1;
    const int32_t W = 1024;
    uint8_t *acc = draw_accepting(seed, n, (int64_t)n / 100);
    if (!acc) return -1;
    /* prev[v-1] = largest accepting id < v (0 if none) */
    int32_t *prev = (int32_t *)malloc((size_t)n * 4);
    if (!prev) { free(acc); return -1; }
    int32_t last = 0;
    for (int32_t v = 1; v <= n; ++v) {
        prev[v - 1] = last;
        if (acc[v - 1]) last = v;
    }
    ebuf b = {0};
    if (eb_reserve(&b, (int64_t)n * 4 + n / 8 + 1024)) { free(acc); free(prev); return -1; }
    rng_t r = stream(seed, TAG_EDGES);
    for (int32_t v = 1; v <= n; ++v) {
        int d = 1 + poisson(&r, 3.0);
        int32_t gap_lo = prev[v - 1] + 1; /* back targets must lie in [gap_lo, v-1] */
        for (int j = 0; j < d; ++j) {
            int local = below(&r, 5) < 4;   /* p = 0.8 */
            int fwd = below(&r, 10) < 9;    /* p = 0.9 */
            int can_fwd = v < n;
            int32_t blo = local ? (gap_lo > v - W ? gap_lo : v - W) : gap_lo;
            int can_back = !acc[v - 1] && blo <= v - 1;
            if (fwd && !can_fwd) fwd = 0;
            if (!fwd && !can_back) fwd = 1;
            if (fwd && !can_fwd) continue; /* neither direction possible */
            int32_t t;
            if (fwd) {
                if (local) {
                    int64_t x = (int64_t)v + uni(&r, 1, W);
                    t = (int32_t)(x > n ? n : x);
                } else {
                    t = (int32_t)uni(&r, (int64_t)v + 1, n);
                }
            } else {
                t = (int32_t)uni(&r, blo, (int64_t)v - 1);
            }
            if (eb_push(&b, v, t)) { free(acc); free(prev); free(b.s); free(b.d); return -1; }
        }
    }
    free(prev);
    g->n_planted = 0;
    if (planted && n >= 1024) {
        /* Window [s, s+1023]; c0 = smallest accepting id in it; 63 more
         * distinct ids from (c0, s+1023]; cycle c0 -> c1 -> ... -> c63 -> c0. */
        rng_t pr = stream(seed, TAG_PLANT);
        int32_t c0 = 0, s = 0;
        for (int tries = 0; tries < 100000 && !c0; ++tries) {
            s = (int32_t)uni(&pr, 1, (int64_t)n - (W - 1));
            for (int32_t x = s; x <= s + W - 1; ++x)
                if (acc[x - 1]) { c0 = x; break; }
            if (c0 && (s + W - 1) - c0 < 63) c0 = 0;
        }
        if (c0) {
            int32_t hi = s + W - 1;
            uint8_t mark[1024];
            memset(mark, 0, sizeof(mark));
            floyd(&pr, (int64_t)c0 + 1, hi, 63, mark);
            int32_t cyc[64];
            int k = 0;
            cyc[k++] = c0;
            for (int32_t x = c0 + 1; x <= hi; ++x)
                if (mark[x - (c0 + 1)]) cyc[k++] = x;
            for (int i = 0; i < 64; ++i) {
                if (eb_push(&b, cyc[i], cyc[(i + 1) & 63])) { free(acc); free(b.s); free(b.d); return -1; }
                g->planted[i] = cyc[i];
            }
            g->n_planted = 64;
        }
    }
    finish(g, &b, n, acc);
    return 0;
}

/* ---------------------------------------------------------- config 3 --- */

int synth_config3(uint64_t seed, int32_t n, synth_graph *g) {
    memset(g, 0, sizeof(*g));
    if (n < 1) return -1;
    int64_t k = (int64_t)n / 1000;
    if (k < 1) k = 1;
    uint8_t *acc = draw_accepting(seed, n, k);
    if (!acc) return -1;
    ebuf b = {0};
    if (eb_reserve(&b, (int64_t)n * 4 + (int64_t)n / 16 + 1024)) { free(acc); return -1; }
    rng_t r = stream(seed, TAG_EDGES);
    for (int32_t v = 2; v <= n; ++v) {
        int d = (int)uni(&r, 1, 7);
        for (int j = 0; j < d; ++j) {
            int32_t t = (int32_t)uni(&r, 1, (int64_t)v - 1);
            if (eb_push(&b, v, t)) { free(acc); free(b.s); free(b.d); return -1; }
        }
    }
    finish(g, &b, n, acc);
    return 0;
}

/* ------------------------------------------------------ configs 4, 5 --- */

static uint64_t sub_seed(uint64_t seed, uint64_t index) {
    rng_t r = stream(seed, 0x100000000ull + index);
    return sm_next(&r);
}

static int32_t log_uniform(rng_t *r, double lo, double hi) {
    double x = exp(log(lo) + unit(r) * (log(hi) - log(lo)));
    int32_t v = (int32_t)floor(x);
    return v < 1 ? 1 : v;
}

static int batch_graph(uint64_t gseed, int32_t n, double ratio, int plant, synth_graph *g) {
    int64_t k = (int64_t)floor(ratio * n);
    if (k < 1) k = 1;
    uint8_t *acc = draw_accepting(gseed, n, k);
    if (!acc) return -1;
    ebuf b = {0};
    if (config1_edges(gseed, n, 1, 4, 1, &b)) { free(acc); free(b.s); free(b.d); return -1; }
    if (plant && plant_random_cycle(gseed, n, acc, &b, g)) { free(acc); free(b.s); free(b.d); return -1; }
    int32_t np = g->n_planted;
    int32_t pl[64];
    memcpy(pl, g->planted, sizeof(pl));
    finish(g, &b, n, acc);
    g->n_planted = np;
    memcpy(g->planted, pl, sizeof(pl));
    return 0;
}

/* Graph `index` of the config-4 batch drawn from `seed`. */
int synth_config4(uint64_t seed, int32_t index, synth_graph *g) {
    memset(g, 0, sizeof(*g));
    uint64_t gs = sub_seed(seed, (uint64_t)index);
    rng_t r = stream(gs, TAG_SIZE);
    int32_t n = log_uniform(&r, 1e3, 1e6);
    return batch_graph(gs, n, 0.05, index & 1, g);
}

/* Size of graph `index` of the config-4 batch, without building it. */
int32_t synth_config4_n(uint64_t seed, int32_t index) {
    uint64_t gs = sub_seed(seed, (uint64_t)index);
    rng_t r = stream(gs, TAG_SIZE);
    return log_uniform(&r, 1e3, 1e6);
}

/* Query `index` of the config-5 stream: size, accepting ratio and the gap to
 * the previous arrival (exponential, mean 1; the caller scales it by 1/QPS). */
int synth_config5_meta(uint64_t seed, int32_t index, int32_t *n, double *ratio, double *gap) {
    uint64_t gs = sub_seed(seed ^ 0x5555555555555555ull, (uint64_t)index);
    rng_t r = stream(gs, TAG_SIZE);
    *n = log_uniform(&r, 1e4, 4e6);
    rng_t q = stream(gs, TAG_RATIO);
    *ratio = 0.001 + unit(&q) * (0.05 - 0.001);
    *gap = -log(1.0 - unit(&q));
    return 0;
}

int synth_config5(uint64_t seed, int32_t index, synth_graph *g) {
    memset(g, 0, sizeof(*g));
    int32_t n;
    double ratio, gap;
    synth_config5_meta(seed, index, &n, &ratio, &gap);
    uint64_t gs = sub_seed(seed ^ 0x5555555555555555ull, (uint64_t)index);
    return batch_graph(gs, n, ratio, index & 1, g);
}
