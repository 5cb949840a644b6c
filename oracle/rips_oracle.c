/*
 * rips_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct CPU computation of Vietoris-Rips
 * persistence pairs and barcodes, written from the paper's definitions.
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may build, load or call it.  It shares no code with the HIP
 * library.
 *
 * What it computes (paper sections "Background", "Computation" and
 * "The Coboundary Matrix"):
 *   - simplices: every vertex set {v_p > ... > v_0} whose diameter (largest
 *     pairwise distance, vertices have diameter 0) is <= threshold;
 *   - combinatorial index cidx = sum_i C(v_i, i+1) (combinatorial number
 *     system section);
 *   - simplex-wise filtration order: diameter ascending, then dimension
 *     ascending, then cidx descending (section on the simplex-wise
 *     refinement);
 *   - the dimension-p coboundary matrix: one column per p-simplex, ordered
 *     in reverse filtration order (diameter descending, cidx ascending); the
 *     nonzero rows of a column are the simplex's cofacets inside the
 *     filtered complex; the "lowest" row (Algorithm 1's low) is the row that
 *     comes last in the anti-transposed matrix, i.e. the cofacet that is
 *     OLDEST in the filtration (smallest diameter, then largest cidx);
 *   - Algorithm 1 (standard reduction over Z/2): for each column j in order,
 *     while some earlier column k has the same low, add reduced column k to
 *     column j; a nonzero result gives the persistence pair (column, low).
 *
 * Every dimension is reduced on its own, over ALL its columns: no clearing,
 * no apparent pairs, no emergent pairs, no enclosing-radius truncation.
 * A reduced column R_k is kept in memory only when it differs from the
 * original coboundary; otherwise it is regenerated when needed.  This
 * changes memory use only, never a result.
 *
 * A second entry point lists apparent pairs by their literal definition
 * (section "The Apparent Pairs Lemma", the definition of an apparent pair):
 * sigma's oldest cofacet tau whose youngest facet is sigma, found by full
 * minimum / maximum over all cofacets and facets, without the lemma.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_DIM 6

typedef struct {
    float diam;
    uint64_t cidx;
} simplex_t;

typedef struct {
    /* all persistence pairs (sigma = column simplex, tau = its pivot row) */
    int64_t n_pairs;
    uint64_t *pair_sigma;
    uint64_t *pair_tau;
    float *pair_birth; /* diam(sigma) */
    float *pair_death; /* diam(tau)   */
    /* columns that reduced to zero (essential unless they are the tau of a
     * pair one dimension lower; the caller classifies) */
    int64_t n_zero;
    uint64_t *zero_sigma;
    float *zero_birth;
    /* number of p-simplices with diameter <= threshold */
    int64_t n_simplices;
    /* column additions performed (statistics only) */
    int64_t n_additions;
    /* columns skipped by the clearing lemma (clearing mode only) */
    int64_t n_cleared;
} oracle_dim_t;

/* ------------------------------------------------------------------ */
/* problem description shared by all threads (read only)             */
/* ------------------------------------------------------------------ */
typedef struct {
    const float *dist; /* condensed lower triangle, edge-cidx order */
    int n;
    float thr;
    uint64_t *binom; /* (ORACLE_MAX_DIM + 3) rows of (n + 1) entries */
    int **nbr;       /* nbr[v] = vertices u != v with d(u,v) <= thr, ascending */
    int *nbr_len;
} problem_t;

static float dist_of(const problem_t *P, int a, int b)
{
    if (a == b)
        return 0.0f;
    if (a < b) {
        int t = a;
        a = b;
        b = t;
    }
    return P->dist[(int64_t)a * (a - 1) / 2 + b];
}

static uint64_t binom(const problem_t *P, int v, int k)
{
    return P->binom[(int64_t)k * (P->n + 1) + v];
}

/* cidx of a vertex set given in DECREASING order: sum_i C(v_i, i+1) where
 * v_0 is the smallest vertex. */
static uint64_t cidx_of(const problem_t *P, const int *dec, int len)
{
    uint64_t c = 0;
    for (int pos = 0; pos < len; ++pos) {
        int i = len - 1 - pos; /* rank from the bottom */
        c += binom(P, dec[pos], i + 1);
    }
    return c;
}

/* filtration order: a is older than b */
static int older(const simplex_t *a, const simplex_t *b)
{
    if (a->diam != b->diam)
        return a->diam < b->diam;
    return a->cidx > b->cidx;
}

static int cmp_row_order(const void *x, const void *y)
{
    const simplex_t *a = x, *b = y;
    if (older(a, b))
        return -1;
    if (older(b, a))
        return 1;
    return 0;
}

/* coboundary-matrix column order: diameter descending, cidx ascending */
static int cmp_col_order(const void *x, const void *y)
{
    const simplex_t *a = x, *b = y;
    if (a->diam != b->diam)
        return a->diam > b->diam ? -1 : 1;
    if (a->cidx != b->cidx)
        return a->cidx < b->cidx ? -1 : 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* growable arrays                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    simplex_t *a;
    int64_t len, cap;
} svec_t;

static int svec_push(svec_t *v, simplex_t s)
{
    if (v->len == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 64;
        simplex_t *na = realloc(v->a, (size_t)nc * sizeof(simplex_t));
        if (!na)
            return -1;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->len++] = s;
    return 0;
}

/* ------------------------------------------------------------------ */
/* vertices of a simplex from its cidx (largest v with C(v,k) <= c)    */
/* ------------------------------------------------------------------ */
static void vertices_of(const problem_t *P, uint64_t c, int p, int *dec)
{
    int hi = P->n; /* vertices are < hi */
    for (int pos = 0; pos <= p; ++pos) {
        int k = p + 1 - pos;
        int v = hi - 1;
        while (binom(P, v, k) > c)
            --v;
        dec[pos] = v;
        c -= binom(P, v, k);
        hi = v;
    }
}

/* ------------------------------------------------------------------ */
/* enumeration of all p-simplices with diameter <= thr                 */
/* ------------------------------------------------------------------ */
typedef struct {
    const problem_t *P;
    int p;
    int dec[ORACLE_MAX_DIM + 2];
    svec_t *out;
    int err;
} enum_ctx_t;

static void enum_rec(enum_ctx_t *E, int depth, float diam)
{
    const problem_t *P = E->P;
    if (depth == E->p + 1) {
        simplex_t s = {diam, cidx_of(P, E->dec, E->p + 1)};
        if (svec_push(E->out, s))
            E->err = 1;
        return;
    }
    int upper = depth == 0 ? P->n : E->dec[depth - 1];
    for (int v = 0; v < upper; ++v) {
        float nd = diam;
        int ok = 1;
        for (int i = 0; i < depth; ++i) {
            float d = dist_of(P, v, E->dec[i]);
            if (!(d <= P->thr)) {
                ok = 0;
                break;
            }
            if (d > nd)
                nd = d;
        }
        if (!ok)
            continue;
        E->dec[depth] = v;
        enum_rec(E, depth + 1, nd);
    }
}

/* ------------------------------------------------------------------ */
/* coboundary of a p-simplex: all cofacets with diameter <= thr,       */
/* sorted oldest first (so element 0 is Algorithm 1's low)             */
/* ------------------------------------------------------------------ */
static int coboundary(const problem_t *P, int p, const simplex_t *s, svec_t *out)
{
    int dec[ORACLE_MAX_DIM + 2], tdec[ORACLE_MAX_DIM + 3];
    vertices_of(P, s->cidx, p, dec);
    out->len = 0;
    /* a cofacet vertex must be a neighbour of every vertex; scan the
     * neighbours of the smallest vertex */
    int anchor = dec[p];
    for (int t = 0; t < P->nbr_len[anchor]; ++t) {
        int v = P->nbr[anchor][t];
        int in = 0, ok = 1;
        float nd = s->diam;
        for (int i = 0; i <= p; ++i) {
            if (dec[i] == v) {
                in = 1;
                break;
            }
            float d = dist_of(P, v, dec[i]);
            if (!(d <= P->thr)) {
                ok = 0;
                break;
            }
            if (d > nd)
                nd = d;
        }
        if (in || !ok)
            continue;
        /* insert v into the decreasing vertex list */
        int q = 0, placed = 0;
        for (int i = 0; i <= p; ++i) {
            if (!placed && v > dec[i]) {
                tdec[q++] = v;
                placed = 1;
            }
            tdec[q++] = dec[i];
        }
        if (!placed)
            tdec[q++] = v;
        simplex_t c = {nd, cidx_of(P, tdec, p + 2)};
        if (svec_push(out, c))
            return -1;
    }
    qsort(out->a, (size_t)out->len, sizeof(simplex_t), cmp_row_order);
    return 0;
}

/* oldest cofacet (Algorithm 1's low of the unreduced column) by a linear
 * minimum over all cofacets; returns 0 when the coboundary is empty */
static int oldest_cofacet(const problem_t *P, int p, const simplex_t *s, simplex_t *low)
{
    int dec[ORACLE_MAX_DIM + 2], tdec[ORACLE_MAX_DIM + 3];
    vertices_of(P, s->cidx, p, dec);
    int anchor = dec[p], have = 0;
    for (int t = 0; t < P->nbr_len[anchor]; ++t) {
        int v = P->nbr[anchor][t];
        int in = 0, ok = 1;
        float nd = s->diam;
        for (int i = 0; i <= p; ++i) {
            if (dec[i] == v) {
                in = 1;
                break;
            }
            float d = dist_of(P, v, dec[i]);
            if (!(d <= P->thr)) {
                ok = 0;
                break;
            }
            if (d > nd)
                nd = d;
        }
        if (in || !ok)
            continue;
        if (have && nd > low->diam)
            continue;
        int q = 0, placed = 0;
        for (int i = 0; i <= p; ++i) {
            if (!placed && v > dec[i]) {
                tdec[q++] = v;
                placed = 1;
            }
            tdec[q++] = dec[i];
        }
        if (!placed)
            tdec[q++] = v;
        simplex_t c = {nd, cidx_of(P, tdec, p + 2)};
        if (!have || older(&c, low)) {
            *low = c;
            have = 1;
        }
    }
    return have;
}

/* symmetric difference of two row-ordered columns (Z/2 addition) */
static int symdiff(const svec_t *a, const simplex_t *b, int64_t blen, svec_t *out)
{
    out->len = 0;
    int64_t i = 0, j = 0;
    while (i < a->len || j < blen) {
        if (j >= blen || (i < a->len && older(&a->a[i], &b[j]))) {
            if (svec_push(out, a->a[i++]))
                return -1;
        } else if (i >= a->len || older(&b[j], &a->a[i])) {
            if (svec_push(out, b[j++]))
                return -1;
        } else { /* same simplex: 1 + 1 = 0 over Z/2 */
            ++i;
            ++j;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* pivot table: row cidx -> column index (open addressing)             */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t *key; /* cidx + 1, 0 = empty */
    int64_t *val;
    uint64_t mask;
} ptab_t;

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

static int ptab_init(ptab_t *t, int64_t n)
{
    uint64_t cap = 16;
    while (cap < (uint64_t)n * 2 + 16)
        cap <<= 1;
    t->key = calloc(cap, sizeof(uint64_t));
    t->val = malloc(cap * sizeof(int64_t));
    t->mask = cap - 1;
    return (t->key && t->val) ? 0 : -1;
}

static int64_t ptab_get(const ptab_t *t, uint64_t k)
{
    uint64_t h = mix64(k) & t->mask;
    while (t->key[h]) {
        if (t->key[h] == k + 1)
            return t->val[h];
        h = (h + 1) & t->mask;
    }
    return -1;
}

static void ptab_put(ptab_t *t, uint64_t k, int64_t v)
{
    uint64_t h = mix64(k) & t->mask;
    while (t->key[h] && t->key[h] != k + 1)
        h = (h + 1) & t->mask;
    t->key[h] = k + 1;
    t->val[h] = v;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 on the dimension-p coboundary matrix                    */
/* ------------------------------------------------------------------ */
typedef struct {
    const problem_t *P;
    int p;
    oracle_dim_t *out;
    const ptab_t *skip; /* clearing mode: tau's of dimension p-1, or NULL */
    int err;
} dim_job_t;

static void *reduce_dimension(void *arg)
{
    dim_job_t *J = arg;
    const problem_t *P = J->P;
    int p = J->p;
    oracle_dim_t *O = J->out;
    memset(O, 0, sizeof(*O));

    svec_t cols = {0};
    enum_ctx_t E = {.P = P, .p = p, .out = &cols, .err = 0};
    enum_rec(&E, 0, 0.0f);
    if (E.err) {
        J->err = 1;
        return NULL;
    }
    O->n_simplices = cols.len;
    if (J->skip) {
        /* clearing lemma: a column whose simplex is the tau of a pair one
         * dimension lower reduces to zero; leave it out of the matrix */
        int64_t m = 0;
        for (int64_t i = 0; i < cols.len; ++i)
            if (ptab_get(J->skip, cols.a[i].cidx) < 0)
                cols.a[m++] = cols.a[i];
        O->n_cleared = cols.len - m;
        cols.len = m;
    }
    qsort(cols.a, (size_t)cols.len, sizeof(simplex_t), cmp_col_order);

    simplex_t **stored = calloc((size_t)cols.len + 1, sizeof(simplex_t *));
    int64_t *stored_len = calloc((size_t)cols.len + 1, sizeof(int64_t));
    ptab_t piv;
    svec_t col = {0}, tmp = {0}, other = {0};
    svec_t ps = {0}, pt = {0}, zs = {0};
    if (!stored || !stored_len || ptab_init(&piv, cols.len)) {
        J->err = 1;
        return NULL;
    }

    for (int64_t j = 0; j < cols.len; ++j) {
        /* Most columns need no addition: their low is not yet a pivot.
         * Find the low by a minimum scan and materialise the sorted column
         * only when an addition is due.  Results are unchanged. */
        simplex_t low0;
        if (!oldest_cofacet(P, p, &cols.a[j], &low0)) {
            if (svec_push(&zs, cols.a[j])) {
                J->err = 1;
                break;
            }
            continue;
        }
        if (ptab_get(&piv, low0.cidx) < 0) {
            ptab_put(&piv, low0.cidx, j);
            if (svec_push(&ps, cols.a[j]) || svec_push(&pt, low0)) {
                J->err = 1;
                break;
            }
            continue;
        }
        if (coboundary(P, p, &cols.a[j], &col)) {
            J->err = 1;
            break;
        }
        int modified = 0;
        while (col.len > 0) {
            int64_t k = ptab_get(&piv, col.a[0].cidx);
            if (k < 0)
                break;
            const simplex_t *kb;
            int64_t kl;
            if (stored[k]) {
                kb = stored[k];
                kl = stored_len[k];
            } else {
                if (coboundary(P, p, &cols.a[k], &other)) {
                    J->err = 1;
                    break;
                }
                kb = other.a;
                kl = other.len;
            }
            if (symdiff(&col, kb, kl, &tmp)) {
                J->err = 1;
                break;
            }
            svec_t sw = col;
            col = tmp;
            tmp = sw;
            modified = 1;
            ++O->n_additions;
        }
        if (J->err)
            break;
        if (col.len > 0) {
            ptab_put(&piv, col.a[0].cidx, j);
            simplex_t s_sigma = cols.a[j];
            if (svec_push(&ps, s_sigma) || svec_push(&pt, col.a[0])) {
                J->err = 1;
                break;
            }
            if (modified) {
                stored[j] = malloc((size_t)col.len * sizeof(simplex_t));
                if (!stored[j]) {
                    J->err = 1;
                    break;
                }
                memcpy(stored[j], col.a, (size_t)col.len * sizeof(simplex_t));
                stored_len[j] = col.len;
            }
        } else {
            if (svec_push(&zs, cols.a[j])) {
                J->err = 1;
                break;
            }
        }
    }

    if (!J->err) {
        O->n_pairs = ps.len;
        O->pair_sigma = malloc((size_t)(ps.len + 1) * sizeof(uint64_t));
        O->pair_tau = malloc((size_t)(ps.len + 1) * sizeof(uint64_t));
        O->pair_birth = malloc((size_t)(ps.len + 1) * sizeof(float));
        O->pair_death = malloc((size_t)(ps.len + 1) * sizeof(float));
        O->n_zero = zs.len;
        O->zero_sigma = malloc((size_t)(zs.len + 1) * sizeof(uint64_t));
        O->zero_birth = malloc((size_t)(zs.len + 1) * sizeof(float));
        if (!O->pair_sigma || !O->pair_tau || !O->pair_birth || !O->pair_death ||
            !O->zero_sigma || !O->zero_birth) {
            J->err = 1;
        } else {
            for (int64_t i = 0; i < ps.len; ++i) {
                O->pair_sigma[i] = ps.a[i].cidx;
                O->pair_birth[i] = ps.a[i].diam;
                O->pair_tau[i] = pt.a[i].cidx;
                O->pair_death[i] = pt.a[i].diam;
            }
            for (int64_t i = 0; i < zs.len; ++i) {
                O->zero_sigma[i] = zs.a[i].cidx;
                O->zero_birth[i] = zs.a[i].diam;
            }
        }
    }

    for (int64_t j = 0; j < cols.len; ++j)
        free(stored[j]);
    free(stored);
    free(stored_len);
    free(piv.key);
    free(piv.val);
    free(col.a);
    free(tmp.a);
    free(other.a);
    free(ps.a);
    free(pt.a);
    free(zs.a);
    free(cols.a);
    return NULL;
}

/* ------------------------------------------------------------------ */
/* problem set-up                                                      */
/* ------------------------------------------------------------------ */
static int problem_init(problem_t *P, const float *dist, int n, float thr)
{
    memset(P, 0, sizeof(*P));
    P->dist = dist;
    P->n = n;
    P->thr = thr;
    int K = ORACLE_MAX_DIM + 3;
    P->binom = calloc((size_t)K * (n + 1), sizeof(uint64_t));
    if (!P->binom)
        return -1;
    /* Pascal's rule, saturating at UINT64_MAX */
    for (int v = 0; v <= n; ++v) {
        for (int k = 0; k < K; ++k) {
            uint64_t val;
            if (k == 0)
                val = 1;
            else if (v == 0)
                val = 0;
            else {
                uint64_t a = P->binom[(int64_t)(k - 1) * (n + 1) + v - 1];
                uint64_t b = P->binom[(int64_t)k * (n + 1) + v - 1];
                val = (a > UINT64_MAX - b) ? UINT64_MAX : a + b;
            }
            P->binom[(int64_t)k * (n + 1) + v] = val;
        }
    }
    P->nbr = calloc((size_t)n, sizeof(int *));
    P->nbr_len = calloc((size_t)n, sizeof(int));
    if (!P->nbr || !P->nbr_len)
        return -1;
    for (int v = 0; v < n; ++v) {
        P->nbr[v] = malloc((size_t)(n > 1 ? n : 1) * sizeof(int));
        if (!P->nbr[v])
            return -1;
        int m = 0;
        for (int u = 0; u < n; ++u)
            if (u != v && dist_of(P, u, v) <= thr)
                P->nbr[v][m++] = u;
        P->nbr_len[v] = m;
    }
    return 0;
}

static void problem_free(problem_t *P)
{
    if (P->nbr)
        for (int v = 0; v < P->n; ++v)
            free(P->nbr[v]);
    free(P->nbr);
    free(P->nbr_len);
    free(P->binom);
}

/* ------------------------------------------------------------------ */
/* public entry points                                                 */
/* ------------------------------------------------------------------ */

/* Persistence pairs and zero columns for dimensions 0..maxdim.
 * dist: condensed lower triangle (n*(n-1)/2 floats, edge-cidx order).
 * clearing == 0: every dimension is reduced over all its columns,
 *   independently (one thread each when threads > 1).
 * clearing != 0: dimensions are reduced in increasing order and the columns
 *   of dimension p that are the tau of a dimension-(p-1) pair are left out
 *   (paper, section "Clearing Lemma"); results are identical, the zero
 *   columns then list only the columns that were actually reduced.
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_reduce(const float *dist, int n, int maxdim, float thr, int threads,
                  int clearing, oracle_dim_t *out)
{
    if (!dist && n > 1)
        return -1;
    if (n < 1 || maxdim < 0 || maxdim > ORACLE_MAX_DIM - 1 || !(thr >= 0.0f))
        return -1;
    problem_t P;
    if (problem_init(&P, dist, n, thr)) {
        problem_free(&P);
        return -2;
    }
    dim_job_t jobs[ORACLE_MAX_DIM];
    pthread_t tids[ORACLE_MAX_DIM];
    int started[ORACLE_MAX_DIM] = {0};
    for (int p = 0; p <= maxdim; ++p) {
        jobs[p].P = &P;
        jobs[p].p = p;
        jobs[p].out = &out[p];
        jobs[p].skip = NULL;
        jobs[p].err = 0;
    }
    if (clearing) {
        int err = 0;
        for (int p = 0; p <= maxdim && !err; ++p) {
            ptab_t skip = {0};
            if (p > 0) {
                if (ptab_init(&skip, out[p - 1].n_pairs)) {
                    err = 1;
                    break;
                }
                for (int64_t i = 0; i < out[p - 1].n_pairs; ++i)
                    ptab_put(&skip, out[p - 1].pair_tau[i], i);
                jobs[p].skip = &skip;
            }
            reduce_dimension(&jobs[p]);
            err |= jobs[p].err;
            free(skip.key);
            free(skip.val);
        }
        problem_free(&P);
        return err ? -2 : 0;
    }
    if (threads > 1) {
        for (int p = maxdim; p >= 0; --p)
            started[p] = pthread_create(&tids[p], NULL, reduce_dimension, &jobs[p]) == 0;
    }
    for (int p = 0; p <= maxdim; ++p)
        if (!started[p])
            reduce_dimension(&jobs[p]);
    for (int p = 0; p <= maxdim; ++p)
        if (started[p])
            pthread_join(tids[p], NULL);
    problem_free(&P);
    int err = 0;
    for (int p = 0; p <= maxdim; ++p)
        err |= jobs[p].err;
    return err ? -2 : 0;
}

void oracle_free(oracle_dim_t *out, int maxdim)
{
    for (int p = 0; p <= maxdim; ++p) {
        free(out[p].pair_sigma);
        free(out[p].pair_tau);
        free(out[p].pair_birth);
        free(out[p].pair_death);
        free(out[p].zero_sigma);
        free(out[p].zero_birth);
        memset(&out[p], 0, sizeof(out[p]));
    }
}

/* Apparent pairs of dimension (p, p+1) by the definition: tau is the oldest
 * cofacet of sigma (full minimum over all cofacets in the filtered complex)
 * and sigma is the youngest facet of tau (full maximum over tau's facets).
 * Considers every p-simplex with diameter <= thr.  Writes at most cap pairs;
 * returns the number of apparent pairs (which may exceed cap), or a negative
 * value on error. */
int64_t oracle_apparent_pairs(const float *dist, int n, int p, float thr,
                              uint64_t *sigma_out, uint64_t *tau_out, int64_t cap)
{
    if (n < 1 || p < 0 || p > ORACLE_MAX_DIM - 1 || !(thr >= 0.0f))
        return -1;
    problem_t P;
    if (problem_init(&P, dist, n, thr)) {
        problem_free(&P);
        return -2;
    }
    svec_t cols = {0}, cob = {0};
    enum_ctx_t E = {.P = &P, .p = p, .out = &cols, .err = 0};
    enum_rec(&E, 0, 0.0f);
    int64_t count = 0;
    int tdec[ORACLE_MAX_DIM + 3], fdec[ORACLE_MAX_DIM + 2];
    for (int64_t j = 0; j < cols.len && !E.err; ++j) {
        const simplex_t *s = &cols.a[j];
        if (coboundary(&P, p, s, &cob)) {
            E.err = 1;
            break;
        }
        if (cob.len == 0)
            continue;
        /* oldest cofacet: explicit minimum in filtration order */
        simplex_t tau = cob.a[0];
        for (int64_t i = 1; i < cob.len; ++i)
            if (older(&cob.a[i], &tau))
                tau = cob.a[i];
        /* youngest facet of tau: explicit maximum in filtration order */
        vertices_of(&P, tau.cidx, p + 1, tdec);
        simplex_t young = {0.0f, 0};
        int have = 0;
        for (int drop = 0; drop <= p + 1; ++drop) {
            int q = 0;
            for (int i = 0; i <= p + 1; ++i)
                if (i != drop)
                    fdec[q++] = tdec[i];
            float d = 0.0f;
            for (int a = 0; a <= p; ++a)
                for (int b = a + 1; b <= p; ++b) {
                    float e = dist_of(&P, fdec[a], fdec[b]);
                    if (e > d)
                        d = e;
                }
            simplex_t f = {d, cidx_of(&P, fdec, p + 1)};
            if (!have || older(&young, &f)) {
                young = f;
                have = 1;
            }
        }
        if (young.cidx == s->cidx) {
            if (count < cap) {
                sigma_out[count] = s->cidx;
                tau_out[count] = tau.cidx;
            }
            ++count;
        }
    }
    int err = E.err;
    free(cols.a);
    free(cob.a);
    problem_free(&P);
    return err ? -2 : count;
}

/* Number of p-simplices with diameter <= thr (for accounting checks). */
int64_t oracle_count_simplices(const float *dist, int n, int p, float thr)
{
    if (n < 1 || p < 0 || p > ORACLE_MAX_DIM - 1 || !(thr >= 0.0f))
        return -1;
    problem_t P;
    if (problem_init(&P, dist, n, thr)) {
        problem_free(&P);
        return -2;
    }
    svec_t cols = {0};
    enum_ctx_t E = {.P = &P, .p = p, .out = &cols, .err = 0};
    enum_rec(&E, 0, 0.0f);
    int64_t c = E.err ? -2 : cols.len;
    free(cols.a);
    problem_free(&P);
    return c;
}
