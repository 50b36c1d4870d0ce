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
 * The census is computed from that definition, not by the thesis's algorithm:
 * every triple with at least one joined pair is classified once, anchored at
 * its smallest vertex (triples with one joined pair in bulk per pair), and
 * class 003 takes the rest of C(n, 3).  It shares no step with the GPU path,
 * which follows the thesis's per-dyad loop.
 *
 * Functions and the passages they follow:
 *   oracle_table          the 64 -> 16 isomorphism map (TriadTable).  The thesis
 *                         describes it but does not print it; it is derived here
 *                         from the class definitions by canonical forms under
 *                         the six vertex relabellings.
 *   oracle_census         the 16-class census (section "Triad Census
 *                         Algorithm", the problem statement and the count of
 *                         null triads as C(n, 3) minus the others).
 *   oracle_census64       the 64-class labelled census the section on the
 *                         TriadCode describes before the table folds it into
 *                         16 classes: the histogram of the 6-bit code of every
 *                         triple, read in the roles in which the thesis's loop
 *                         counts it (u the smallest vertex, v the smaller of the
 *                         vertices joined to u, w the third; a triple with one
 *                         joined pair takes the code of that pair alone), and
 *                         code 0 is C(n, 3) minus the rest.
 *   oracle_census_range   classes 1..15 of the triples whose smallest vertex
 *                         (for one joined pair: the pair's smaller vertex) lies
 *                         in [x0, x1): what one task queue of canonical dyads
 *                         with first vertex in that range counts in the
 *                         task-queue formulation (figure "Subquadratic Triad
 *                         Census Algorithm based on distributed task queues");
 *                         class 003 is left at 0.
 *   oracle_census_mt      the same census with threads taking chunks of
 *                         smallest vertices, one local histogram per thread,
 *                         summed after the join (timing variant).
 *   oracle_brute          the naive O(n^3) census the section on the algorithm
 *                         mentions: every triple classified through TriadCode
 *                         over an n x n bit matrix.
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
/* Graph: sorted out-lists (arcs) and sorted neighbour lists with the  */
/* direction of every joined pair                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t arcs;          /* distinct arcs kept */
    int64_t *out_ptr;      /* n + 1 */
    int32_t *out;          /* sorted heads per tail */
    int64_t *nb_ptr;       /* n + 1 */
    int32_t *nb;           /* sorted undirected neighbours per vertex */
    uint8_t *nb_dir;       /* per neighbour entry w of x: bit0 x->w, bit1 w->x */
    uint8_t T[64];
} og_t;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
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

/* is the arc x -> y in E? */
static int arc(const og_t *g, int32_t x, int32_t y)
{
    return in_sorted(g->out + g->out_ptr[x], g->out_ptr[x + 1] - g->out_ptr[x], y);
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
    g->nb_dir = (uint8_t *)malloc((size_t)(b > 0 ? b : 1));
    for (int64_t i = 0; i < b; ++i) {
        int32_t x = (int32_t)(ukey[i] / n), w = (int32_t)(ukey[i] % n);
        g->nb_ptr[x + 1]++;
        g->nb[i] = w;
        g->nb_dir[i] = (uint8_t)(arc(g, x, w) | (arc(g, w, x) << 1));
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
    free(g->out_ptr); free(g->out); free(g->nb_ptr); free(g->nb); free(g->nb_dir); free(g);
}

int64_t oracle_graph_arcs(void *h) { return ((og_t *)h)->arcs; }

/* degree of u in the undirected sense, |N(u)| */
int64_t oracle_graph_degree(void *h, int32_t u)
{
    og_t *g = (og_t *)h;
    return g->nb_ptr[u + 1] - g->nb_ptr[u];
}

/* ------------------------------------------------------------------ */
/* The census by its definition: every triple classified once          */
/* ------------------------------------------------------------------ */

/* Per-thread look-up tables over the vertices.  in_x[w] == x + 1 exactly when
 * w is joined to x, and then dir_x[w] holds the arcs between them (bit0 x->w,
 * bit1 w->x); in_p / dir_p do the same for the second vertex p of the current
 * pair, keyed by that pair's entry position + 1 so no table is ever cleared. */
typedef struct {
    int64_t *in_x, *in_p;
    uint8_t *dir_x, *dir_p;
} ws_t;

static int ws_init(ws_t *ws, int32_t n)
{
    size_t len = (size_t)(n > 0 ? n : 1);
    ws->in_x = (int64_t *)calloc(len, sizeof(int64_t));
    ws->in_p = (int64_t *)calloc(len, sizeof(int64_t));
    ws->dir_x = (uint8_t *)calloc(len, 1);
    ws->dir_p = (uint8_t *)calloc(len, 1);
    return ws->in_x && ws->in_p && ws->dir_x && ws->dir_p ? 0 : -1;
}

static void ws_free(ws_t *ws)
{
    free(ws->in_x); free(ws->in_p); free(ws->dir_x); free(ws->dir_p);
}

/*
 * Every unordered triple {x, p, q} of distinct vertices with x its smallest
 * vertex, classified by the 6-bit TriadCode of its induced digraph, read in the
 * roles u = x, v = p, w = q (bits 1 u->v, 2 v->u, 4 u->w, 8 w->u, 16 v->w,
 * 32 w->v).  A triple with no joined pair is not visited (code 0 is filled in
 * by subtraction from C(n, 3)).  The others are met exactly once:
 *
 *   one joined pair {x, p}, x < p:  counted in bulk per pair, as the number of
 *       third vertices joined to neither, n - 2 - |(N(x) u N(p)) \ {x, p}|;
 *   x joined to both others:        p < q, both in N(x);
 *   x joined to exactly one other:  p that one, q in N(p) \ N(x), q > x.
 *
 * In the last two cases v is the smaller of the vertices joined to u and w
 * the remaining one, which are the roles in which the subquadratic loop of
 * section "Triad Census Algorithm" counts the triple (its canonical condition
 * gives a triple a < b < c to the dyad (a, b) when a, b are joined, else to
 * (a, c)); a pair's bulk count goes to the code of the pair alone.  The codes
 * are added into hist[64].
 */
static void triples_at(const og_t *g, int32_t x, ws_t *ws, uint64_t hist[64])
{
    const int64_t n = g->n;
    const int64_t xb = g->nb_ptr[x], xe = g->nb_ptr[x + 1];
    for (int64_t i = xb; i < xe; ++i) {
        ws->in_x[g->nb[i]] = (int64_t)x + 1;
        ws->dir_x[g->nb[i]] = g->nb_dir[i];
    }
    for (int64_t i = xb; i < xe; ++i) {
        const int32_t p = g->nb[i];
        if (p < x) continue;
        const int64_t key = i + 1;
        const int64_t pb = g->nb_ptr[p], pe = g->nb_ptr[p + 1];
        for (int64_t j = pb; j < pe; ++j) {
            ws->in_p[g->nb[j]] = key;
            ws->dir_p[g->nb[j]] = g->nb_dir[j];
        }
        const int uv = ws->dir_x[p];                  /* bit0 x->p, bit1 p->x */

        /* one joined pair: the third vertices joined to x or to p */
        int64_t touched = 0;
        for (int64_t j = xb; j < xe; ++j)
            if (g->nb[j] != p) ++touched;
        for (int64_t j = pb; j < pe; ++j) {
            const int32_t w = g->nb[j];
            if (w != x && ws->in_x[w] != (int64_t)x + 1) ++touched;
        }
        hist[uv] += (uint64_t)(n - 2 - touched);

        /* x joined to p and to q, p < q */
        for (int64_t j = xb; j < xe; ++j) {
            const int32_t q = g->nb[j];
            if (q <= p) continue;
            const int pq = ws->in_p[q] == key ? ws->dir_p[q] : 0;
            hist[uv | ws->dir_x[q] << 2 | pq << 4] += 1;
        }

        /* x joined to p only; q joined to p, not to x, q > x */
        for (int64_t j = pb; j < pe; ++j) {
            const int32_t q = g->nb[j];
            if (q <= x || ws->in_x[q] == (int64_t)x + 1) continue;
            hist[uv | ws->dir_p[q] << 4] += 1;
        }
    }
}

static u128 choose3(int64_t n)
{
    return n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
}

/* 16-class census from the code histogram: class T[code] takes every code;
 * class 003 is C(n, 3) minus the other classes when `null` is set, else 0. */
static void fold(const og_t *g, const uint64_t hist[64], int null, uint64_t out[16])
{
    uint64_t c[16] = {0};
    u128 sum = 0;
    for (int code = 1; code < 64; ++code) {
        c[g->T[code]] += hist[code];
        sum += hist[code];
    }
    c[0] = null ? (uint64_t)(choose3(g->n) - sum) : 0;
    memcpy(out, c, sizeof(c));
}

static int hist_range(const og_t *g, int32_t x0, int32_t x1, uint64_t hist[64])
{
    ws_t ws;
    if (ws_init(&ws, g->n) != 0) { ws_free(&ws); return -1; }
    for (int32_t x = x0; x < x1; ++x) triples_at(g, x, &ws, hist);
    ws_free(&ws);
    return 0;
}

int oracle_census(void *h, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    uint64_t hist[64] = {0};
    if (hist_range(g, 0, g->n, hist) != 0) return -1;
    fold(g, hist, 1, out);
    return 0;
}

/* 64-class labelled census: the code histogram itself, code 0 (no joined pair)
 * being C(n, 3) minus the rest. */
int oracle_census64(void *h, uint64_t out[64])
{
    og_t *g = (og_t *)h;
    uint64_t hist[64] = {0};
    if (hist_range(g, 0, g->n, hist) != 0) return -1;
    u128 sum = 0;
    for (int code = 1; code < 64; ++code) sum += hist[code];
    hist[0] = (uint64_t)(choose3(g->n) - sum);
    memcpy(out, hist, sizeof(hist));
    return 0;
}

/* Classes 1..15 of the triples whose smallest vertex lies in [x0, x1) (a
 * triple with one joined pair: the smaller vertex of that pair); class 003
 * is left at 0.  The parts of a partition of [0, n) add up to the census. */
int oracle_census_range(void *h, int32_t x0, int32_t x1, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    if (x0 < 0) x0 = 0;
    if (x1 > g->n) x1 = g->n;
    uint64_t hist[64] = {0};
    if (x0 < x1 && hist_range(g, x0, x1, hist) != 0) return -1;
    fold(g, hist, 0, out);
    return 0;
}

/* ---- multithreaded variant: threads take chunks of smallest vertices ---- */

typedef struct {
    const og_t *g;
    int32_t *next;              /* shared: first vertex of the next chunk */
    int32_t chunk;
    int err;
    uint64_t hist[64];
} mt_t;

static void *mt_run(void *arg)
{
    mt_t *t = (mt_t *)arg;
    ws_t ws;
    if (ws_init(&ws, t->g->n) != 0) { ws_free(&ws); t->err = 1; return NULL; }
    for (;;) {
        int32_t x0 = __atomic_fetch_add(t->next, t->chunk, __ATOMIC_RELAXED);
        if (x0 >= t->g->n) break;
        int32_t x1 = x0 + t->chunk < t->g->n ? x0 + t->chunk : t->g->n;
        for (int32_t x = x0; x < x1; ++x) triples_at(t->g, x, &ws, t->hist);
    }
    ws_free(&ws);
    return NULL;
}

/* Same result as oracle_census; returns the number of threads used. */
int oracle_census_mt(void *h, int threads, uint64_t out[16])
{
    og_t *g = (og_t *)h;
    if (threads < 1) threads = 1;
    int32_t next = 0;
    mt_t *t = (mt_t *)calloc((size_t)threads, sizeof(mt_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!t || !tid) { free(t); free(tid); return -1; }
    for (int i = 0; i < threads; ++i) {
        t[i].g = g; t[i].next = &next; t[i].chunk = 64;
        pthread_create(&tid[i], NULL, mt_run, &t[i]);
    }
    uint64_t hist[64] = {0};
    int err = 0;
    for (int i = 0; i < threads; ++i) {
        pthread_join(tid[i], NULL);
        err |= t[i].err;
        for (int k = 0; k < 64; ++k) hist[k] += t[i].hist[k];
    }
    free(t);
    free(tid);
    if (err) return -1;
    fold(g, hist, 1, out);
    return threads;
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
