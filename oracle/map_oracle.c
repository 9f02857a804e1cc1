/*
 * CPU oracle for MAP accepting-cycle detection.  TEST INFRASTRUCTURE ONLY:
 * the GPU library is checked against it; nothing on the product path links,
 * loads or calls it.  It shares no code with the HIP library.
 *
 * Problem (paper, Section 2 "DiVinE CUDA Algorithmics"): given a directed
 * graph with accepting vertices, decide whether some cycle passes through an
 * accepting vertex.  Method MAP, as the paper states it:
 *   - order the accepting vertices (here: by numeric id, larger wins; id 0
 *     means "no vertex");
 *   - compute for every vertex its maximal accepting predecessor map(u);
 *   - if an accepting u has map(u) == u, u lies on an accepting cycle: stop;
 *   - otherwise every accepting vertex that is the map value of some vertex
 *     loses its accepting flag, and the computation restarts;
 *   - stop when a cycle is found or no accepting vertex is left.
 * The paper runs MAP on the transposed graph; predecessors in the transposed
 * graph are successors in the generated graph G.  So, on the edge list s -> d
 * of G that this oracle takes,
 *
 *   map(v) = max { a in A : v reaches a along >= 1 edge of G }   (0 if none).
 *
 * map is computed as the fixpoint of value propagation (paper, Section 2:
 * every vertex keeps the largest value propagated into it; the maximum over
 * incoming values and its own value is forwarded; stop when nothing improves).
 * A vertex w sends max(map(w), w if w is accepting); v keeps the maximum of
 * what its successors send.  Readings taken where the paper is silent:
 *   - the predecessor is proper (path of >= 1 edge), otherwise every maximal
 *     accepting vertex would trivially be its own predecessor;
 *   - the values stripped are the nonzero map values of all vertices;
 *   - map is reset to 0 at each restart;
 *   - a third exit: when no value is stripped (every map value is 0) there is
 *     no accepting cycle, and the loop stops;
 *   - the test map(u) == u is made at the fixpoint only; the witness is the
 *     largest such u;
 *   - the iteration count K is the number of fixpoint computations.
 *
 * Three independent routes to the same fixpoint (they must agree exactly):
 *   jacobi  the value propagation as stated, all vertices updated at once
 *           from the previous vector, repeated until nothing changes;
 *   reach   the definition: a graph search from every vertex (tiny graphs);
 *   desc    the definition taken in decreasing order of accepting id: the
 *           vertices that reach a and have no value yet get value a (a
 *           backward search over unlabelled vertices).  Labelled sets stay
 *           closed under predecessors, so a search never needs to pass through
 *           a labelled vertex, and an accepting vertex that already holds a
 *           value reaches a larger one, so its search adds nothing.
 *           O(n + m) per fixpoint: used for the large goldens and baselines.
 * Plus two textbook deciders of the verdict alone: Tarjan's strongly
 * connected components (accepting vertex in a nontrivial component or on a
 * self-loop) and the nested depth-first search of Courcoubetis, Vardi,
 * Wolper and Yannakakis.
 *
 * Build flavours (same source, same arithmetic): the plain single-threaded
 * build every test uses; with -fopenmp -DORACLE_OPENMP the edge loop of a
 * jacobi pass is shared among the host's threads (used only to time the
 * jacobi route on all host cores); and sanitizer builds for the CPU tests.
 *
 * All ids are int32, 1..n; edges are (src[i] -> dst[i]); acc[i] flags id i+1.
 * Per-iteration digest: sum over v of mix64((v << 32) | map(v)) mod 2^64, with
 * mix64 the SplitMix64 finalizer (Steele, Lea & Flood, OOPSLA 2014).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef ORACLE_OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3
#define OR_ENOTCONVERGED -5

enum { MODE_JACOBI = 0, MODE_REACH = 1, MODE_DESC = 2 };

/* ------------------------------------------------------- adjacency --- */

/* Lists of neighbours per vertex, vertex index 1..n: off[v]..off[v+1]. */
typedef struct { int32_t n; int64_t *off; int32_t *nb; } adj_t;

static void adj_free(adj_t *a) { free(a->off); free(a->nb); }

/* forward != 0: successors (s -> d gives d in list of s); else predecessors. */
static int adj_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int forward, adj_t *a) {
    a->n = n;
    a->off = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    a->nb = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!a->off || !a->nb) { adj_free(a); return OR_ENOMEM; }
    for (int64_t i = 0; i < m; ++i) a->off[(forward ? src[i] : dst[i]) + 1]++;
    for (int32_t v = 1; v <= n + 1; ++v) a->off[v] += a->off[v - 1];
    int64_t *fill = (int64_t *)malloc(((size_t)n + 2) * sizeof(int64_t));
    if (!fill) { adj_free(a); return OR_ENOMEM; }
    memcpy(fill, a->off, ((size_t)n + 2) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        int32_t key = forward ? src[i] : dst[i];
        int32_t val = forward ? dst[i] : src[i];
        a->nb[fill[key]++] = val;
    }
    free(fill);
    return OR_OK;
}

static int check_ids(int32_t n, int64_t m, const int32_t *src, const int32_t *dst) {
    if (n < 1 || m < 0) return OR_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        if (src[i] < 1 || src[i] > n || dst[i] < 1 || dst[i] > n) return OR_EINVAL;
    return OR_OK;
}

/* -------------------------------------------------------- fixpoints --- */

/* What w sends along an edge: its kept value, or itself if larger and accepting. */
static int32_t sent(int32_t w, const int32_t *val, const uint8_t *acc) {
    int32_t x = val[w - 1];
    if (acc[w - 1] && w > x) x = w;
    return x;
}

#ifdef ORACLE_OPENMP
/* next[v] = max(next[v], x), for edges of one source handled by different
 * threads in the same pass. */
static void raise_to(int32_t *p, int32_t x) {
    int32_t cur = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (x > cur && !__atomic_compare_exchange_n(p, &cur, x, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
}
#endif

/* Threads the jacobi route uses (1 in the plain build). */
int oracle_threads(void) {
#ifdef ORACLE_OPENMP
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
#else
    return 1;
#endif
}

/* jacobi: m_{t+1}(v) = max(m_t(v), max over edges v->w of sent_t(w)), from
 * m_0 = 0, until m_{t+1} == m_t.  *sweeps counts every pass made, including
 * the final pass that changes nothing. */
static int fix_jacobi(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc,
                      int32_t *map, int64_t *sweeps) {
    int32_t *next = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!next) return OR_ENOMEM;
    memset(map, 0, (size_t)n * sizeof(int32_t));
    int64_t t = 0;
    for (;;) {
        memcpy(next, map, (size_t)n * sizeof(int32_t));
#ifdef ORACLE_OPENMP
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) raise_to(&next[src[i] - 1], sent(dst[i], map, acc));
#else
        for (int64_t i = 0; i < m; ++i) {
            int32_t x = sent(dst[i], map, acc);
            if (x > next[src[i] - 1]) next[src[i] - 1] = x;
        }
#endif
        t++;
        if (memcmp(next, map, (size_t)n * sizeof(int32_t)) == 0) break;
        memcpy(map, next, (size_t)n * sizeof(int32_t));
    }
    free(next);
    if (sweeps) *sweeps = t;
    return OR_OK;
}

/* reach: for every v, search G from the successors of v; map(v) is the
 * largest accepting id found. */
static int fix_reach(int32_t n, const adj_t *succ, const uint8_t *acc, int32_t *map) {
    int32_t *stack = (int32_t *)malloc(((size_t)succ->off[n + 1] + 1) * sizeof(int32_t));
    int32_t *seen = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t)); /* seen[x] == v: visited in v's search */
    if (!stack || !seen) { free(stack); free(seen); return OR_ENOMEM; }
    for (int32_t v = 1; v <= n; ++v) {
        int32_t best = 0;
        int64_t sp = 0;
        for (int64_t j = succ->off[v]; j < succ->off[v + 1]; ++j) {
            int32_t w = succ->nb[j];
            if (seen[w] != v) { seen[w] = v; stack[sp++] = w; }
        }
        while (sp > 0) {
            int32_t x = stack[--sp];
            if (acc[x - 1] && x > best) best = x;
            for (int64_t j = succ->off[x]; j < succ->off[x + 1]; ++j) {
                int32_t w = succ->nb[j];
                if (seen[w] != v) { seen[w] = v; stack[sp++] = w; }
            }
        }
        map[v - 1] = best;
    }
    free(stack);
    free(seen);
    return OR_OK;
}

/* desc: accepting ids a in decreasing order; if a holds no value yet, every
 * unlabelled vertex with a path of >= 1 edge to a gets value a, found by a
 * breadth-first search over predecessors that enters unlabelled vertices only. */
static int fix_desc(int32_t n, const adj_t *pred, const uint8_t *acc, int32_t *map) {
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return OR_ENOMEM;
    memset(map, 0, (size_t)n * sizeof(int32_t));
    for (int32_t a = n; a >= 1; --a) {
        if (!acc[a - 1] || map[a - 1] != 0) continue;
        int64_t head = 0, tail = 0;
        for (int64_t j = pred->off[a]; j < pred->off[a + 1]; ++j) {
            int32_t u = pred->nb[j];
            if (map[u - 1] == 0) { map[u - 1] = a; queue[tail++] = u; }
        }
        while (head < tail) {
            int32_t x = queue[head++];
            for (int64_t j = pred->off[x]; j < pred->off[x + 1]; ++j) {
                int32_t u = pred->nb[j];
                if (map[u - 1] == 0) { map[u - 1] = a; queue[tail++] = u; }
            }
        }
    }
    free(queue);
    return OR_OK;
}

int oracle_fixpoint(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc,
                    int32_t mode, int32_t *map, int64_t *sweeps) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    if (sweeps) *sweeps = 0;
    if (mode == MODE_JACOBI) return fix_jacobi(n, m, src, dst, acc, map, sweeps);
    adj_t a;
    rc = adj_build(n, m, src, dst, mode == MODE_REACH, &a);
    if (rc) return rc;
    rc = (mode == MODE_REACH) ? fix_reach(n, &a, acc, map) : (mode == MODE_DESC) ? fix_desc(n, &a, acc, map)
                                                                                : OR_EINVAL;
    adj_free(&a);
    return rc;
}

/* The vectors m_1, m_2, ... of the jacobi propagation, one row of n per pass,
 * up to steps_cap rows; returns the number of passes made (the last one
 * changes nothing), or < 0 on error. */
int64_t oracle_jacobi_steps(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc,
                            int32_t *steps, int64_t steps_cap) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    int32_t *cur = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int32_t *next = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!cur || !next) { free(cur); free(next); return OR_ENOMEM; }
    int64_t t = 0;
    for (;;) {
        memcpy(next, cur, (size_t)n * sizeof(int32_t));
        for (int64_t i = 0; i < m; ++i) {
            int32_t x = sent(dst[i], cur, acc);
            if (x > next[src[i] - 1]) next[src[i] - 1] = x;
        }
        if (t < steps_cap) memcpy(steps + (size_t)t * n, next, (size_t)n * sizeof(int32_t));
        t++;
        if (memcmp(next, cur, (size_t)n * sizeof(int32_t)) == 0) break;
        memcpy(cur, next, (size_t)n * sizeof(int32_t));
    }
    free(cur);
    free(next);
    return t;
}

/* ---------------------------------------------------------- digest --- */

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_digest(int32_t n, const int32_t *map) {
    uint64_t s = 0;
    for (int32_t v = 1; v <= n; ++v) s += mix64(((uint64_t)(uint32_t)v << 32) | (uint32_t)map[v - 1]);
    return s;
}

/* ------------------------------------------------------- MAP loop --- */

/*
 * The MAP outer loop.  result[0..3] = found, witness, K, |A| at exit.
 * trace (may be NULL): row k-1 = { |Del_k| (0 when iteration k found a cycle
 * or stripped nothing), sweeps of iteration k (jacobi only, else 0), digest of
 * map_k }.  maps (may be NULL): map_k for k <= maps_cap, row-major [k-1][n].
 * acc_out (may be NULL): the accepting set at exit.  max_iter <= 0: no cap.
 * Returns OR_ENOTCONVERGED when the cap stops the loop.
 */
int oracle_map_detect(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc0,
                      int32_t mode, int32_t max_iter, int32_t *result, int64_t *sweeps_total,
                      uint64_t *trace, int32_t trace_cap, int32_t *maps, int32_t maps_cap, uint8_t *acc_out) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    uint8_t *acc = (uint8_t *)malloc((size_t)n);
    int32_t *map = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!acc || !map) { free(acc); free(map); return OR_ENOMEM; }
    for (int32_t i = 0; i < n; ++i) acc[i] = acc0[i] ? 1 : 0;
    adj_t a = {0};
    if (mode == MODE_REACH || mode == MODE_DESC) {
        rc = adj_build(n, m, src, dst, mode == MODE_REACH, &a);
        if (rc) { free(acc); free(map); return rc; }
    } else if (mode != MODE_JACOBI) {
        free(acc); free(map);
        return OR_EINVAL;
    }
    int32_t found = 0, witness = 0, k = 0;
    int64_t total = 0;
    rc = OR_OK;
    for (;;) {
        int32_t left = 0;
        for (int32_t i = 0; i < n; ++i) left += acc[i];
        if (left == 0) break;                                   /* no accepting vertex left */
        if (max_iter > 0 && k >= max_iter) { rc = OR_ENOTCONVERGED; break; }
        k++;
        int64_t sw = 0;
        if (mode == MODE_JACOBI) rc = fix_jacobi(n, m, src, dst, acc, map, &sw);
        else if (mode == MODE_REACH) rc = fix_reach(n, &a, acc, map);
        else rc = fix_desc(n, &a, acc, map);
        if (rc) break;
        total += sw;
        if (maps && k <= maps_cap) memcpy(maps + (size_t)(k - 1) * n, map, (size_t)n * sizeof(int32_t));
        uint64_t *row = (trace && k <= trace_cap) ? trace + (size_t)(k - 1) * 3 : NULL;
        if (row) { row[0] = 0; row[1] = (uint64_t)sw; row[2] = oracle_digest(n, map); }
        for (int32_t v = n; v >= 1; --v)                          /* own maximal accepting predecessor */
            if (map[v - 1] == v) { found = 1; witness = v; break; }
        if (found) break;
        int64_t del = 0;                                          /* strip every nonzero map value */
        for (int32_t v = 1; v <= n; ++v) {
            int32_t x = map[v - 1];
            if (x != 0 && acc[x - 1]) { acc[x - 1] = 0; del++; }
        }
        if (row) row[0] = (uint64_t)del;
        if (del == 0) break;                                      /* nothing stripped: no cycle */
    }
    int32_t left = 0;
    for (int32_t i = 0; i < n; ++i) left += acc[i];
    if (acc_out) memcpy(acc_out, acc, (size_t)n);
    result[0] = found;
    result[1] = witness;
    result[2] = k;
    result[3] = left;
    if (sweeps_total) *sweeps_total = total;
    if (mode != MODE_JACOBI) adj_free(&a);
    free(acc);
    free(map);
    return rc;
}

/* ---------------------------------------------------------- Tarjan --- */

/*
 * Strongly connected components (Tarjan 1972), iterative.  Returns 1 if some
 * accepting vertex lies in a component of >= 2 vertices or has a self-loop,
 * 0 if not, < 0 on error.  comp (may be NULL) receives a component id per
 * vertex.
 */
int oracle_tarjan(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc,
                  int32_t *comp) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    adj_t s;
    rc = adj_build(n, m, src, dst, 1, &s);
    if (rc) return rc;
    int32_t *index = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *low = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *cid = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *stk = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *call = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t *it = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    uint8_t *on = (uint8_t *)calloc((size_t)n + 1, 1);
    int32_t *csize = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!index || !low || !cid || !stk || !call || !it || !on || !csize) {
        rc = OR_ENOMEM;
        goto done;
    }
    for (int32_t v = 0; v <= n; ++v) index[v] = -1;
    int32_t counter = 0, sp = 0, ncomp = 0;
    for (int32_t root = 1; root <= n; ++root) {
        if (index[root] >= 0) continue;
        int32_t csp = 0;
        call[csp++] = root;
        index[root] = low[root] = counter++;
        stk[sp++] = root;
        on[root] = 1;
        it[root] = s.off[root];
        while (csp > 0) {
            int32_t v = call[csp - 1];
            if (it[v] < s.off[v + 1]) {
                int32_t w = s.nb[it[v]++];
                if (index[w] < 0) {
                    index[w] = low[w] = counter++;
                    stk[sp++] = w;
                    on[w] = 1;
                    it[w] = s.off[w];
                    call[csp++] = w;
                } else if (on[w] && index[w] < low[v]) {
                    low[v] = index[w];
                }
            } else {
                if (low[v] == index[v]) {
                    int32_t w;
                    do {
                        w = stk[--sp];
                        on[w] = 0;
                        cid[w] = ncomp;
                        csize[ncomp]++;
                    } while (w != v);
                    ncomp++;
                }
                csp--;
                if (csp > 0) {
                    int32_t p = call[csp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
            }
        }
    }
    rc = 0;
    for (int32_t v = 1; v <= n && !rc; ++v)
        if (acc[v - 1] && csize[cid[v]] >= 2) rc = 1;
    for (int64_t i = 0; i < m && !rc; ++i)
        if (src[i] == dst[i] && acc[src[i] - 1]) rc = 1;
    if (comp)
        for (int32_t v = 1; v <= n; ++v) comp[v - 1] = cid[v];
done:
    free(index); free(low); free(cid); free(stk); free(call); free(it); free(on); free(csize);
    adj_free(&s);
    return rc;
}

/* ------------------------------------------------------ nested DFS --- */

/*
 * Nested depth-first search (Courcoubetis, Vardi, Wolper, Yannakakis 1992).
 * The outer (blue) search covers every vertex, roots in id order; when an
 * accepting vertex s finishes, an inner (red) search from s looks for an edge
 * back into s, over vertices not yet red.  Recursive: small graphs only.
 */
typedef struct { const adj_t *s; const uint8_t *acc; uint8_t *blue, *red; int32_t seed; } ndfs_t;

static int red_dfs(ndfs_t *c, int32_t v) {
    c->red[v] = 1;
    for (int64_t j = c->s->off[v]; j < c->s->off[v + 1]; ++j) {
        int32_t w = c->s->nb[j];
        if (w == c->seed) return 1;
        if (!c->red[w] && red_dfs(c, w)) return 1;
    }
    return 0;
}

static int blue_dfs(ndfs_t *c, int32_t v) {
    c->blue[v] = 1;
    for (int64_t j = c->s->off[v]; j < c->s->off[v + 1]; ++j) {
        int32_t w = c->s->nb[j];
        if (!c->blue[w] && blue_dfs(c, w)) return 1;
    }
    if (c->acc[v - 1]) {
        c->seed = v;
        if (red_dfs(c, v)) return 1;
    }
    return 0;
}

int oracle_ndfs(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    if (n > 100000) return OR_EINVAL;
    adj_t s;
    rc = adj_build(n, m, src, dst, 1, &s);
    if (rc) return rc;
    ndfs_t c = { &s, acc, (uint8_t *)calloc((size_t)n + 1, 1), (uint8_t *)calloc((size_t)n + 1, 1), 0 };
    if (!c.blue || !c.red) rc = OR_ENOMEM;
    else {
        rc = 0;
        for (int32_t v = 1; v <= n && !rc; ++v)
            if (!c.blue[v]) rc = blue_dfs(&c, v);
    }
    free(c.blue);
    free(c.red);
    adj_free(&s);
    return rc;
}

/* -------------------------------------------------- counterexample --- */
/*
 * A counterexample for a reported cycle (the paper lists counterexample
 * generation as missing from the tool, Section 5): a lasso made of a shortest
 * path from an initial vertex `init` to the witness w and a shortest cycle
 * through w, both along edges of G, found by breadth-first search over
 * successors.  Their lengths are unique.  The paper fixes no choice among
 * several shortest paths; this one takes, walking back from the end, the
 * smallest vertex of each breadth-first level that has an edge to the vertex
 * after it: of all shortest paths, the one whose vertices read backwards are
 * lexicographically smallest (so the path depends on the edge set alone, not
 * on the order of the edge list).
 *
 * path receives init = s_0, ..., s_S = w, c_1, ..., c_L = w (S + L + 1 ids);
 * without an initial vertex (init == 0) or with init == w, S = 0.
 * Returns OR_OK; OR_ENOPATH when init does not reach w or w lies on no cycle
 * (a length not found is -1); OR_ENOSPC when cap is below S + L + 1 (both
 * lengths set, path untouched); OR_EINVAL on bad input, OR_ENOMEM.
 */
#define OR_ENOPATH -8
#define OR_ENOSPC -9

static int cmp_i32(const void *a, const void *b) {
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Breadth-first search from `from`, one level at a time, until an edge enters
 * `to`.  Each level is expanded in increasing vertex order, so parent[v] is
 * the smallest vertex of the level before v's with an edge to v (0: not
 * reached) and *last the smallest vertex of the final level with an edge to
 * `to`.  `from` itself is not marked, so from == to finds a shortest cycle.
 * Returns the number of edges of a shortest path of >= 1 edge, or -1. */
static int32_t bfs_to(const adj_t *s, int32_t from, int32_t to, int32_t *parent, int32_t *queue,
                      int32_t *last) {
    memset(parent, 0, ((size_t)s->n + 1) * sizeof(int32_t));
    int64_t head = 0, tail = 0;
    queue[tail++] = from;
    for (int32_t dist = 0; head < tail; ++dist) {
        const int64_t level_end = tail;
        qsort(queue + head, (size_t)(level_end - head), sizeof(int32_t), cmp_i32);
        for (; head < level_end; ++head) {
            const int32_t u = queue[head];
            for (int64_t j = s->off[u]; j < s->off[u + 1]; ++j) {
                const int32_t v = s->nb[j];
                if (v == to) { *last = u; return dist + 1; }
                if (v != from && parent[v] == 0) {
                    parent[v] = u;
                    queue[tail++] = v;
                }
            }
        }
    }
    return -1;
}

int oracle_lasso(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t w, int32_t init,
                 int32_t *stem_len, int32_t *cycle_len, int32_t *path, int32_t cap) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    if (w < 1 || w > n || init < 0 || init > n || cap < 0 || !stem_len || !cycle_len) return OR_EINVAL;
    adj_t s;
    rc = adj_build(n, m, src, dst, 1, &s);
    if (rc) return rc;
    int32_t *parent = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *stem = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!parent || !queue || !stem) { rc = OR_ENOMEM; goto out; }
    int32_t S = 0, L, last = 0;
    *stem_len = *cycle_len = -1;
    if (init != 0 && init != w) {
        S = bfs_to(&s, init, w, parent, queue, &last);
        if (S < 0) { rc = OR_ENOPATH; goto out; }
        /* s_S = w, s_{S-1} = last, s_{i-1} = parent[s_i]; parent[init] stays 0 */
        stem[S] = w;
        for (int32_t i = S - 1, x = last; i >= 0; --i) { stem[i] = x; x = parent[x]; }
    } else {
        stem[0] = w;
    }
    *stem_len = S;
    L = bfs_to(&s, w, w, parent, queue, &last);
    if (L < 0) { rc = OR_ENOPATH; goto out; }
    *cycle_len = L;
    if ((int64_t)S + L + 1 > cap) { rc = OR_ENOSPC; goto out; }
    for (int32_t i = 0; i <= S; ++i) path[i] = stem[i];
    path[S + L] = w;
    for (int32_t i = S + L - 1, x = last; i > S; --i) { path[i] = x; x = parent[x]; }
    rc = OR_OK;
out:
    free(parent);
    free(queue);
    free(stem);
    adj_free(&s);
    return rc;
}

/* --------------------------------------------------------- pruning --- */
/*
 * Relevance pruning for detection on a growing graph.  The paper's tool keeps
 * in its matrix only the states of components that contain accepting states,
 * and a second thread repeatedly runs the detection on the part of the graph
 * built so far (Section 2).  That component reduction needs the property
 * automaton; its stand-in on a bare graph is the trim of cycle-free vertices:
 * while some vertex has no remaining predecessor or no remaining successor,
 * remove it.  What remains is the largest vertex set in which every vertex has
 * a predecessor and a successor inside the set.  Every cycle lies inside it,
 * so clearing the accepting flag of every vertex outside it leaves the
 * verdict unchanged (K and the witness follow the reduced accepting set).
 *
 * keep[i] = 1 if id i+1 remains; acc_out (may be NULL) = acc & keep.
 * Queue-based peeling with per-vertex counts of remaining in- and out-edges
 * (parallel edges counted with multiplicity), O(n + m).  Returns the number of
 * vertices kept, or a negative error.
 */
int64_t oracle_trim(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *acc,
                    uint8_t *keep, uint8_t *acc_out) {
    int rc = check_ids(n, m, src, dst);
    if (rc) return rc;
    if (!keep) return OR_EINVAL;
    adj_t s, p;
    rc = adj_build(n, m, src, dst, 1, &s);
    if (rc) return rc;
    rc = adj_build(n, m, src, dst, 0, &p);
    if (rc) { adj_free(&s); return rc; }
    int64_t *indeg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t *outdeg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    int32_t *queue = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t kept = 0;
    if (!indeg || !outdeg || !queue) { kept = OR_ENOMEM; goto out; }
    int64_t head = 0, tail = 0;
    for (int32_t v = 1; v <= n; ++v) {
        indeg[v] = p.off[v + 1] - p.off[v];
        outdeg[v] = s.off[v + 1] - s.off[v];
        keep[v - 1] = 1;
        if (indeg[v] == 0 || outdeg[v] == 0) { keep[v - 1] = 0; queue[tail++] = v; }
    }
    while (head < tail) {
        int32_t v = queue[head++];
        for (int64_t j = s.off[v]; j < s.off[v + 1]; ++j) {      /* v's out-edges leave */
            int32_t w = s.nb[j];
            if (--indeg[w] == 0 && keep[w - 1]) { keep[w - 1] = 0; queue[tail++] = w; }
        }
        for (int64_t j = p.off[v]; j < p.off[v + 1]; ++j) {      /* v's in-edges leave */
            int32_t u = p.nb[j];
            if (--outdeg[u] == 0 && keep[u - 1]) { keep[u - 1] = 0; queue[tail++] = u; }
        }
    }
    for (int32_t v = 1; v <= n; ++v) {
        kept += keep[v - 1];
        if (acc_out) acc_out[v - 1] = (uint8_t)(acc && acc[v - 1] && keep[v - 1] ? 1 : 0);
    }
out:
    free(indeg);
    free(outdeg);
    free(queue);
    adj_free(&s);
    adj_free(&p);
    return kept;
}
