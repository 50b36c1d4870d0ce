/*
 * CPU oracle for the 16-class directed triad census.  TEST INFRASTRUCTURE ONLY:
 * this file is built into liboracle.so, which only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load.  The GPU library shares
 * no code with it.
 *
 * What it computes (Nagpal 2013, section "Triad Census Algorithm"):
 *   for a strict digraph G = [V, E] with E a set of ordered pairs, the number
 *   of unordered vertex triples whose induced 3-vertex digraph falls in each
 *   of the 16 isomorphism classes, numbered in the thesis's order
 *   003, 012, 102, 021D, 021U, 021C, 111D, 111U, 030T, 030C, 201, 120D, 120U,
 *   120C, 210, 300 (here 0-based: class 0 is 003, class 15 is 300).
 *
 * Functions and the passages they follow:
 *   oracle_table          the 64 -> 16 isomorphism map (TriadTable).  The thesis
 *                         describes it but does not print it; it is derived here
 *                         from the class definitions by canonical forms under
 *                         the six vertex relabellings.
 *   oracle_census*        the subquadratic census (figure "Subquadratic Triad
 *                         Census Algorithm") with the pre-computed (u, v) dyad
 *                         type of the v0.4 change (figure "Modified TriadCode"),
 *                         IsEdge / IsNeighbour as binary searches in sorted
 *                         out-lists / neighbour lists, S built explicitly.
 *   oracle_census_range   the same loop restricted to canonical dyads whose
 *                         first vertex u lies in [u0, u1): the local census of
 *                         one task queue in the task-queue formulation (figure
 *                         "Subquadratic Triad Census Algorithm based on
 *                         distributed task queues"); class 003 is left at 0.
 *   oracle_census_mt      multithreaded timing variant: canonical dyads split
 *                         into contiguous task queues of equal |N(u)|+|N(v)|-2
 *                         (figure "Canonical Dyad (uniform distr.)" task-queue
 *                         generation), one local census per thread, summed after
 *                         the join (section v0.6, "local census array per thread").
 *   oracle_brute          the naive O(n^3) census the section on the algorithm
 *                         mentions: every triple classified through TriadCode.
 *   oracle_census64       the 64-class labelled census the section on the
 *                         TriadCode describes before the table folds it into
 *                         16 classes: the same loop, histogramming the raw
 *                         6-bit code of (u, v, w) in the roles the loop gives
 *                         them; the dyadic term n - |S| - 2 goes to the code of
 *                         the (u, v) pair alone (w joined to neither), and code
 *                         0 is C(n, 3) minus the rest.
 *
 * Input handling (reading of the thesis's "strict digraph, E a set"): arcs
 * (u, u) are dropped and repeated arcs are merged; ids must lie in [0, n).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* TriadTable: 64 -> 16 from the class definitions                     */
/* ------------------------------------------------------------------ */

/* Code bits as in TriadCode: 1 u->v, 2 v->u, 4 u->w, 8 w->u, 16 v->w, 32 w->v,
 * with vertices u = 0, v = 1, w = 2. */
static int bit_of_arc(int x, int y)
{
    if (x == 0 && y == 1) return 1;
    if (x == 1 && y == 0) return 2;
    if (x == 0 && y == 2) return 4;
    if (x == 2 && y == 0) return 8;
    if (x == 1 && y == 2) return 16;
    if (x == 2 && y == 1) return 32;
    return 0;
}

static int relabel_code(int code, const int p[3])
{
    int out = 0;
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y)
            if (x != y && (code & bit_of_arc(x, y)))
                out |= bit_of_arc(p[x], p[y]);
    return out;
}

static int canonical_code(int code)
{
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                    {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int best = 64;
    for (int i = 0; i < 6; ++i) {
        int c = relabel_code(code, perms[i]);
        if (c < best) best = c;
    }
    return best;
}

/* One representative digraph per class, vertices a = 0, b = 1, c = 2, written
 * from the MAN naming convention (M mutual, A asymmetric, N null dyads) and the
 * D(own) / U(p) / C(yclic) / T(ransitive) letters.  Each row lists arcs as
 * (tail, head) pairs; -1 ends a row. */
static const int class_rep[16][13] = {
    /* 003  */ {-1},
    /* 012  */ {0, 1, -1},
    /* 102  */ {0, 1, 1, 0, -1},
    /* 021D */ {1, 0, 1, 2, -1},                       /* b->a, b->c          */
    /* 021U */ {0, 1, 2, 1, -1},                       /* a->b, c->b          */
    /* 021C */ {0, 1, 1, 2, -1},                       /* a->b->c             */
    /* 111D */ {0, 1, 1, 0, 2, 1, -1},                 /* a<->b, c->b         */
    /* 111U */ {0, 1, 1, 0, 1, 2, -1},                 /* a<->b, b->c         */
    /* 030T */ {0, 1, 1, 2, 0, 2, -1},                 /* a->b->c, a->c       */
    /* 030C */ {0, 1, 1, 2, 2, 0, -1},                 /* a->b->c->a          */
    /* 201  */ {0, 1, 1, 0, 1, 2, 2, 1, -1},           /* a<->b<->c           */
    /* 120D */ {1, 0, 1, 2, 0, 2, 2, 0, -1},           /* b->a, b->c, a<->c   */
    /* 120U */ {0, 1, 2, 1, 0, 2, 2, 0, -1},           /* a->b, c->b, a<->c   */
    /* 120C */ {0, 1, 1, 2, 0, 2, 2, 0, -1},           /* a->b->c, a<->c      */
    /* 210  */ {0, 1, 1, 2, 2, 1, 0, 2, 2, 0, -1},     /* a->b, b<->c, a<->c  */
    /* 300  */ {0, 1, 1, 0, 0, 2, 2, 0, 1, 2, 2, 1, -1},
};

/* Fills T[64]; returns 0 on success, -1 if the definitions do not partition the
 * 64 codes into 16 classes (two representatives isomorphic, or a code left out). */
int oracle_table(uint8_t T[64])
{
    int rep_canon[16];
    for (int k = 0; k < 16; ++k) {
        int code = 0;
        for (int i = 0; class_rep[k][i] >= 0; i += 2)
            code |= bit_of_arc(class_rep[k][i], class_rep[k][i + 1]);
        rep_canon[k] = canonical_code(code);
        for (int j = 0; j < k; ++j)
            if (rep_canon[j] == rep_canon[k]) return -1;
    }
    for (int code = 0; code < 64; ++code) {
        int c = canonical_code(code), found = -1;
        for (int k = 0; k < 16; ++k)
            if (rep_canon[k] == c) found = k;
        if (found < 0) return -1;
        T[code] = (uint8_t)found;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Graph: sorted out-lists (IsEdge) and sorted neighbour lists (N)     */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t arcs;          /* distinct arcs kept */
    int64_t *out_ptr;      /* n + 1 */
    int32_t *out;          /* sorted heads per tail */
    int64_t *nb_ptr;       /* n + 1 */
    int32_t *nb;           /* sorted undirected neighbours per vertex */
    uint8_t T[64];
} og_t;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Builds the oracle's own adjacency.  Returns NULL on a bad id or no memory. */
void *oracle_graph_new(int32_t n, int64_t m, const int32_t *src, const int32_t *dst)
{
    if (n < 0 || m < 0) return NULL;
    og_t *g = (og_t *)calloc(1, sizeof(og_t));
    if (!g) return NULL;
    g->n = n;
    if (oracle_table(g->T) != 0) { free(g); return NULL; }
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(key); free(g); return NULL; }
        if (src[i] == dst[i]) continue;                       /* no loops */
        key[k++] = (int64_t)src[i] * n + dst[i];
    }
    qsort(key, (size_t)k, sizeof(int64_t), cmp_i64);
    int64_t a = 0;
    for (int64_t i = 0; i < k; ++i)                           /* E is a set */
        if (i == 0 || key[i] != key[i - 1]) key[a++] = key[i];
    g->arcs = a;
    g->out_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(a > 0 ? a : 1));
    for (int64_t i = 0; i < a; ++i) {
        g->out_ptr[key[i] / n + 1]++;
        g->out[i] = (int32_t)(key[i] % n);   /* keys sorted: rows and heads in order */
    }
    for (int32_t u = 0; u < n; ++u) g->out_ptr[u + 1] += g->out_ptr[u];

    /* undirected neighbour sets: both orientations of every arc, sorted, unique */
    int64_t *ukey = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * a > 0 ? 2 * a : 1));
    for (int64_t i = 0; i < a; ++i) {
        int64_t u = key[i] / n, v = key[i] % n;
        ukey[2 * i] = u * n + v;
        ukey[2 * i + 1] = v * n + u;
    }
    qsort(ukey, (size_t)(2 * a), sizeof(int64_t), cmp_i64);
    int64_t b = 0;
    for (int64_t i = 0; i < 2 * a; ++i)
        if (i == 0 || ukey[i] != ukey[i - 1]) ukey[b++] = ukey[i];
    g->nb_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b > 0 ? b : 1));
    for (int64_t i = 0; i < b; ++i) {
        g->nb_ptr[ukey[i] / n + 1]++;
        g->nb[i] = (int32_t)(ukey[i] % n);
    }
    for (int32_t u = 0; u < n; ++u) g->nb_ptr[u + 1] += g->nb_ptr[u];
    free(key);
    free(ukey);
    return g;
}

void oracle_graph_free(void *h)
{
    og_t *g = (og_t *)h;
    if (!g) return;
    free(g->out_ptr); free(g->out); free(g->nb_ptr); free(g->nb); free(g);
}

int64_t oracle_graph_arcs(void *h) { return ((og_t *)h)->arcs; }

/* degree of u in the undirected sense, |N(u)| */
int64_t oracle_graph_degree(void *h, int32_t u)
{
    og_t *g = (og_t *)h;
    return g->nb_ptr[u + 1] - g->nb_ptr[u];
}

static int in_sorted(const int32_t *a, int64_t len, int32_t x)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < len && a[lo] == x;
}

/* IsEdge(x, y): is the arc x -> y in E? */
static int is_edge(const og_t *g, int32_t x, int32_t y)
{
    return in_sorted(g->out + g->out_ptr[x], g->out_ptr[x + 1] - g->out_ptr[x], y);
}

/* IsNeighbour(x, y): are x and y joined in either direction? */
static int is_neighbour(const og_t *g, int32_t x, int32_t y)
{
    return in_sorted(g->nb + g->nb_ptr[x], g->nb_ptr[x + 1] - g->nb_ptr[x], y);
}

/* S = N(u) u N(v) \ {u, v}, written sorted into buf; returns |S|. */
static int64_t build_S(const og_t *g, int32_t u, int32_t v, int32_t *buf)
{
    const int32_t *a = g->nb + g->nb_ptr[u], *b = g->nb + g->nb_ptr[v];
    int64_t la = g->nb_ptr[u + 1] - g->nb_ptr[u], lb = g->nb_ptr[v + 1] - g->nb_ptr[v];
    int64_t i = 0, j = 0, s = 0;
    while (i < la || j < lb) {
        int32_t x;
        if (j >= lb || (i < la && a[i] < b[j])) x = a[i++];
        else if (i >= la || b[j] < a[i]) x = b[j++];
        else { x = a[i]; ++i; ++j; }
        if (x != u && x != v) buf[s++] = x;
    }
    return s;
}

/* The per-dyad body: dyad (u, v), u < v, joined in at least one direction. */
static void census_dyad(const og_t *g, int32_t u, int32_t v, int32_t *buf, uint64_t c[16])
{
    int64_t n = g->n;
    int64_t s = build_S(g, u, v, buf);
    int e0 = is_edge(g, u, v), e1 = is_edge(g, v, u);
    int pre = e0 + 2 * e1;                         /* v0.4: (u, v) part of the code */
    int type = (e0 && e1) ? 2 : 1;                 /* 102 if mutual, else 012 */
    c[type] += (uint64_t)(n - s - 2);
    for (int64_t k = 0; k < s; ++k) {
        int32_t w = buf[k];
        if (v < w || (w < v && u < w && !is_neighbour(g, u, w))) {
            int code = pre + 4 * is_edge(g, u, w) + 8 * is_edge(g, w, u)
                     + 16 * is_edge(g, v, w) + 32 * is_edge(g, w, v);
            c[g->T[code]] += 1;
        }
    }
}

static int64_t max_degree(const og_t *g)
{
    int64_t d = 0;
    for (int32_t u = 0; u < g->n; ++u) {
        int64_t x = g->nb_ptr[u + 1] - g->nb_ptr[u];
        if (x > d) d = x;
    }
    return d;
}

/* canonical dyads with u in [u0, u1); classes 1..15 accumulated into c */
static void census_vertices(const og_t *g, int32_t u0, int32_t u1, int32_t *buf, uint64_t c[16])
{
    for (int32_t u = u0; u < u1; ++u)
        for (int64_t p = g->nb_ptr[u]; p < g->nb_ptr[u + 1]; ++p) {
            int32_t v = g->nb[p];
            if (u < v) census_dyad(g, u, v, buf, c);
        }
}

/* C(n, 3) - sum of the other 15 classes, with a 128-bit product. */
static void finish_null(int64_t n, uint64_t c[16])
{
    u128 total = n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
    u128 sum = 0;
    for (int k = 1; k < 16; ++k) sum += c[k];
    c[0] = (uint64_t)(total - sum);
}

int oracle_census(void *h, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    uint64_t c[16] = {0};
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * max_degree(g) + 1));
    if (!buf) return -1;
    census_vertices(g, 0, g->n, buf, c);
    free(buf);
    finish_null(g->n, c);
    memcpy(out, c, sizeof(c));
    return 0;
}

/* The per-dyad body again, counting raw codes instead of classes. */
static void census64_dyad(const og_t *g, int32_t u, int32_t v, int32_t *buf, uint64_t c[64])
{
    int64_t n = g->n;
    int64_t s = build_S(g, u, v, buf);
    int e0 = is_edge(g, u, v), e1 = is_edge(g, v, u);
    int pre = e0 + 2 * e1;
    c[pre] += (uint64_t)(n - s - 2);
    for (int64_t k = 0; k < s; ++k) {
        int32_t w = buf[k];
        if (v < w || (w < v && u < w && !is_neighbour(g, u, w))) {
            int code = pre + 4 * is_edge(g, u, w) + 8 * is_edge(g, w, u)
                     + 16 * is_edge(g, v, w) + 32 * is_edge(g, w, v);
            c[code] += 1;
        }
    }
}

int oracle_census64(void *h, uint64_t out[64])
{
    og_t *g = (og_t *)h;
    uint64_t c[64] = {0};
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * max_degree(g) + 1));
    if (!buf) return -1;
    for (int32_t u = 0; u < g->n; ++u)
        for (int64_t p = g->nb_ptr[u]; p < g->nb_ptr[u + 1]; ++p) {
            int32_t v = g->nb[p];
            if (u < v) census64_dyad(g, u, v, buf, c);
        }
    free(buf);
    int64_t n = g->n;
    u128 total = n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
    u128 sum = 0;
    for (int k = 1; k < 64; ++k) sum += c[k];
    c[0] = (uint64_t)(total - sum);
    memcpy(out, c, sizeof(c));
    return 0;
}

int oracle_census_range(void *h, int32_t u0, int32_t u1, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    if (u0 < 0) u0 = 0;
    if (u1 > g->n) u1 = g->n;
    uint64_t c[16] = {0};
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * max_degree(g) + 1));
    if (!buf) return -1;
    if (u0 < u1) census_vertices(g, u0, u1, buf, c);
    free(buf);
    memcpy(out, c, sizeof(c));
    return 0;
}

/* ---- multithreaded variant: task queues of equal |N(u)|+|N(v)|-2 ---- */

typedef struct {
    const og_t *g;
    int32_t u_begin, u_end;     /* vertex range of the first dyad's u .. */
    int64_t p_begin, p_end;     /* .. and the neighbour-entry range it spans */
    uint64_t c[16];
} task_t;

static void *task_run(void *arg)
{
    task_t *t = (task_t *)arg;
    const og_t *g = t->g;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * max_degree(g) + 1));
    if (!buf) return (void *)1;
    memset(t->c, 0, sizeof(t->c));
    /* dyads are the neighbour entries p of u with u < nb[p], taken in order */
    int32_t u = t->u_begin;
    for (int64_t p = t->p_begin; p < t->p_end; ++p) {
        while (p >= g->nb_ptr[u + 1]) ++u;
        int32_t v = g->nb[p];
        if (u < v) census_dyad(g, u, v, buf, t->c);
    }
    free(buf);
    return NULL;
}

int oracle_census_mt(void *h, int threads, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    if (threads < 1) threads = 1;
    /* total uniform-distribution workload */
    int64_t total = 0;
    for (int32_t u = 0; u < g->n; ++u)
        for (int64_t p = g->nb_ptr[u]; p < g->nb_ptr[u + 1]; ++p) {
            int32_t v = g->nb[p];
            if (u < v) total += (g->nb_ptr[u + 1] - g->nb_ptr[u]) + (g->nb_ptr[v + 1] - g->nb_ptr[v]) - 2;
        }
    int64_t quota = total / threads + 1;
    task_t *tasks = (task_t *)calloc((size_t)threads, sizeof(task_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    int q = 0;
    int64_t load = 0;
    tasks[0].g = g; tasks[0].u_begin = 0; tasks[0].p_begin = 0;
    for (int32_t u = 0; u < g->n; ++u)
        for (int64_t p = g->nb_ptr[u]; p < g->nb_ptr[u + 1]; ++p) {
            int32_t v = g->nb[p];
            if (!(u < v)) continue;
            load += (g->nb_ptr[u + 1] - g->nb_ptr[u]) + (g->nb_ptr[v + 1] - g->nb_ptr[v]) - 2;
            if (load > quota && q + 1 < threads) {     /* close this queue after dyad p */
                tasks[q].p_end = p + 1;
                ++q;
                tasks[q].g = g;
                tasks[q].u_begin = u;
                tasks[q].p_begin = p + 1;
                load = 0;
            }
        }
    tasks[q].p_end = g->nb_ptr[g->n];
    int nq = q + 1;
    for (int i = 0; i < nq; ++i) pthread_create(&tid[i], NULL, task_run, &tasks[i]);
    int err = 0;
    uint64_t c[16] = {0};
    for (int i = 0; i < nq; ++i) {
        void *r = NULL;
        pthread_join(tid[i], &r);
        if (r) err = 1;
        for (int k = 0; k < 16; ++k) c[k] += tasks[i].c[k];
    }
    free(tasks);
    free(tid);
    if (err) return -1;
    finish_null(g->n, c);
    memcpy(out, c, sizeof(c));
    return nq;
}

/* ---- naive O(n^3) census over an n x n bit matrix ---- */

typedef struct {
    const uint64_t *adj;
    int64_t words, n;
    int32_t a_begin, a_step;
    const uint8_t *T;
    uint64_t c[16];
} brute_t;

static int bit(const uint64_t *adj, int64_t words, int64_t x, int64_t y)
{
    return (int)((adj[x * words + (y >> 6)] >> (y & 63)) & 1u);
}

static void *brute_run(void *arg)
{
    brute_t *t = (brute_t *)arg;
    memset(t->c, 0, sizeof(t->c));
    for (int64_t a = t->a_begin; a < t->n; a += t->a_step)
        for (int64_t b = a + 1; b < t->n; ++b)
            for (int64_t c = b + 1; c < t->n; ++c) {
                /* TriadCode with u = a, v = b, w = c */
                int code = bit(t->adj, t->words, a, b) + 2 * bit(t->adj, t->words, b, a)
                         + 4 * bit(t->adj, t->words, a, c) + 8 * bit(t->adj, t->words, c, a)
                         + 16 * bit(t->adj, t->words, b, c) + 32 * bit(t->adj, t->words, c, b);
                t->c[t->T[code]] += 1;
            }
    return NULL;
}

int oracle_brute(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int threads,
                 uint64_t out[16])
{
    uint8_t T[64];
    if (oracle_table(T) != 0 || n < 0) return -1;
    if (threads < 1) threads = 1;
    int64_t words = ((int64_t)n + 63) / 64;
    uint64_t *adj = (uint64_t *)calloc((size_t)(words * (n > 0 ? n : 1)), sizeof(uint64_t));
    if (!adj) return -1;
    for (int64_t i = 0; i < m; ++i) {
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(adj); return -1; }
        if (src[i] != dst[i]) adj[(int64_t)src[i] * words + (dst[i] >> 6)] |= 1ull << (dst[i] & 63);
    }
    brute_t *t = (brute_t *)calloc((size_t)threads, sizeof(brute_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    for (int i = 0; i < threads; ++i) {
        t[i].adj = adj; t[i].words = words; t[i].n = n;
        t[i].a_begin = i; t[i].a_step = threads; t[i].T = T;
        pthread_create(&tid[i], NULL, brute_run, &t[i]);
    }
    uint64_t c[16] = {0};
    for (int i = 0; i < threads; ++i) {
        pthread_join(tid[i], NULL);
        for (int k = 0; k < 16; ++k) c[k] += t[i].c[k];
    }
    free(t); free(tid); free(adj);
    memcpy(out, c, sizeof(c));
    return 0;
}
