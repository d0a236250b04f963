/*
 * bt_oracle.c - plain CPU oracle for butterfly supports and bitruss numbers.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with
 * the GPU path, uses no vertex priority, no BE-Index and no blooms, and is
 * written from the plain definitions of the paper's Section II:
 *   - a butterfly is a (2,2)-biclique (Definition 2); the support of an
 *     edge is the number of butterflies that contain it;
 *   - the k-bitruss is the maximal subgraph in which every edge lies in at
 *     least k butterflies (Definition 4), and the bitruss number of an edge
 *     is the largest such k (Definition 5).
 *
 * Graph format: upper-major CSR.  row_ptr int64[n_upper+1], col int32[m]
 * (lower ids, strictly increasing per row).  Edge e is CSR position e.
 * All integer arithmetic is int64; there is no floating point.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int32_t n_upper, n_lower;
    int64_t m;
    const int64_t *row_ptr; /* upper rows */
    const int32_t *col;
    int64_t *lptr;          /* lower rows (transpose) */
    int32_t *ladj;          /* upper endpoint of each lower-row entry */
    int64_t *leid;          /* edge id of each lower-row entry */
} graph_t;

static int graph_init(graph_t *g, int32_t nu, int32_t nl, int64_t m,
                      const int64_t *row_ptr, const int32_t *col) {
    g->n_upper = nu; g->n_lower = nl; g->m = m;
    g->row_ptr = row_ptr; g->col = col;
    g->lptr = (int64_t *)calloc((size_t)nl + 1, sizeof(int64_t));
    g->ladj = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    g->leid = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc(((size_t)nl + 1) * sizeof(int64_t));
    if (!g->lptr || !g->ladj || !g->leid || !cur) { free(cur); return -1; }
    for (int64_t e = 0; e < m; ++e) g->lptr[col[e] + 1]++;
    for (int32_t v = 0; v < nl; ++v) g->lptr[v + 1] += g->lptr[v];
    memcpy(cur, g->lptr, ((size_t)nl + 1) * sizeof(int64_t));
    /* Rows are visited in increasing upper id, so each lower row lists its
     * upper neighbours in increasing id order. */
    for (int32_t u = 0; u < nu; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t p = cur[col[e]]++;
            g->ladj[p] = u;
            g->leid[p] = e;
        }
    free(cur);
    return 0;
}

static void graph_free(graph_t *g) {
    free(g->lptr); free(g->ladj); free(g->leid);
}

/* One side of the graph seen as "rows": for a vertex a of side A, its
 * neighbours in side B with the id of each edge.  Upper side: CSR rows,
 * edge id = position.  Lower side: transpose rows with stored edge ids. */
typedef struct {
    int32_t n;
    const int64_t *ptr;
    const int32_t *adj;
    const int64_t *eid; /* NULL means eid = position */
} side_t;

static side_t upper_side(const graph_t *g) {
    side_t s = {g->n_upper, g->row_ptr, g->col, NULL};
    return s;
}
static side_t lower_side(const graph_t *g) {
    side_t s = {g->n_lower, g->lptr, g->ladj, g->leid};
    return s;
}
static inline int64_t side_eid(const side_t *s, int64_t p) {
    return s->eid ? s->eid[p] : p;
}

static int64_t sum_sq_deg(const side_t *s) {
    int64_t t = 0;
    for (int32_t a = 0; a < s->n; ++a) {
        int64_t d = s->ptr[a + 1] - s->ptr[a];
        t += d * d;
    }
    return t;
}

/*
 * Per-edge butterfly support from its definition.  For an edge (a, v) with
 * a in side A and v in side B, every butterfly through it is fixed by a
 * second A-vertex w adjacent to v and a second B-vertex adjacent to both a
 * and w, so
 *     support(a, v) = sum over w in N(v), w != a, of (|N(a) & N(w)| - 1).
 * |N(a) & N(w)| is counted for all w at once by walking every path
 * a - v' - w.  The total butterfly count is obtained independently as
 * sum over pairs {a, w} of C(|N(a) & N(w)|, 2): a butterfly is a pair of
 * A-vertices together with a pair of their common neighbours.
 */
static void support_side(const side_t *A, const side_t *B, int64_t *sup,
                         int64_t *pair_total) {
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int32_t *cnt = (int32_t *)calloc((size_t)A->n + 1, sizeof(int32_t));
        int32_t *touched = (int32_t *)malloc(((size_t)A->n + 1) * sizeof(int32_t));
#pragma omp for schedule(dynamic, 16)
        for (int32_t a = 0; a < A->n; ++a) {
            int32_t nt = 0;
            for (int64_t p = A->ptr[a]; p < A->ptr[a + 1]; ++p) {
                int32_t v = A->adj[p];
                for (int64_t q = B->ptr[v]; q < B->ptr[v + 1]; ++q) {
                    int32_t w = B->adj[q];
                    if (w == a) continue;
                    if (cnt[w]++ == 0) touched[nt++] = w;
                }
            }
            for (int64_t p = A->ptr[a]; p < A->ptr[a + 1]; ++p) {
                int32_t v = A->adj[p];
                int64_t s = 0;
                for (int64_t q = B->ptr[v]; q < B->ptr[v + 1]; ++q) {
                    int32_t w = B->adj[q];
                    if (w == a) continue;
                    s += (int64_t)cnt[w] - 1;
                }
                sup[side_eid(A, p)] = s;
            }
            for (int32_t i = 0; i < nt; ++i) {
                int32_t w = touched[i];
                int64_t c = cnt[w];
                if (w > a) total += c * (c - 1) / 2;
                cnt[w] = 0;
            }
        }
        free(cnt);
        free(touched);
    }
    *pair_total = total;
}

/*
 * Support of every edge.  butterflies_out = (sum of supports) / 4, since a
 * butterfly has four edges; pairs_out = the independent pair count above.
 * The start side is the one whose middle layer has the smaller sum of
 * squared degrees (the number of paths walked).  Returns 0 on success.
 */
int bto_support(int32_t n_upper, int32_t n_lower, int64_t m,
                const int64_t *row_ptr, const int32_t *col,
                int64_t *sup_out, int64_t *butterflies_out, int64_t *pairs_out,
                int orientation, int nthreads) {
    graph_t g;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    if (graph_init(&g, n_upper, n_lower, m, row_ptr, col)) return -1;
    side_t U = upper_side(&g), L = lower_side(&g);
    /* orientation: 0 = automatic, 1 = start from upper, 2 = start from lower */
    int from_upper = orientation == 1 ||
                     (orientation == 0 && sum_sq_deg(&L) <= sum_sq_deg(&U));
    int64_t pairs = 0;
    if (from_upper) support_side(&U, &L, sup_out, &pairs);
    else support_side(&L, &U, sup_out, &pairs);
    int64_t s = 0;
    for (int64_t e = 0; e < m; ++e) s += sup_out[e];
    if (butterflies_out) *butterflies_out = s / 4;
    if (pairs_out) *pairs_out = pairs;
    graph_free(&g);
    return 0;
}

/* Support of one edge (u, v) straight from the definition, for sampled
 * checks on graphs too large to count whole: pairs w in N(v) \ {u} with the
 * size of N(u) & N(w) found by merging the two sorted upper rows. */
int64_t bto_edge_support(int32_t n_upper, const int64_t *row_ptr, const int32_t *col,
                         const int64_t *lptr, const int32_t *ladj, int64_t e) {
    (void)n_upper;
    int32_t u = 0;
    {   /* row containing position e */
        int32_t lo = 0, hi = n_upper;
        while (hi - lo > 1) {
            int32_t mid = lo + (hi - lo) / 2;
            if (row_ptr[mid] <= e) lo = mid; else hi = mid;
        }
        u = lo;
    }
    int32_t v = col[e];
    int64_t s = 0;
    for (int64_t q = lptr[v]; q < lptr[v + 1]; ++q) {
        int32_t w = ladj[q];
        if (w == u) continue;
        int64_t i = row_ptr[u], ie = row_ptr[u + 1], j = row_ptr[w], je = row_ptr[w + 1];
        int64_t common = 0;
        while (i < ie && j < je) {
            if (col[i] < col[j]) ++i;
            else if (col[i] > col[j]) ++j;
            else { ++common; ++i; ++j; }
        }
        s += common - 1;
    }
    return s;
}

/*
 * Rows of the remaining graph.  Each vertex keeps the edges it still has at
 * the front of its row, in no particular order: nbr[p] is the other
 * endpoint and eid[p] the edge at place p, len[x] the number of remaining
 * edges of x, and pos[e] the place of edge e in its row.  Removing an edge
 * moves the last remaining entry of the row into its place, so walks over
 * the remaining graph never visit removed edges.
 */
typedef struct {
    const int64_t *ptr;
    int32_t *len;
    int32_t *nbr;
    int64_t *eid;
    int64_t *pos;
} rows_t;

static int rows_init(rows_t *r, const side_t *s, int64_t m) {
    r->ptr = s->ptr;
    r->len = (int32_t *)malloc(((size_t)s->n + 1) * sizeof(int32_t));
    r->nbr = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    r->eid = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    r->pos = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!r->len || !r->nbr || !r->eid || !r->pos) return -1;
    for (int32_t a = 0; a < s->n; ++a) {
        r->len[a] = (int32_t)(s->ptr[a + 1] - s->ptr[a]);
        for (int64_t p = s->ptr[a]; p < s->ptr[a + 1]; ++p) {
            int64_t e = side_eid(s, p);
            r->nbr[p] = s->adj[p];
            r->eid[p] = e;
            r->pos[e] = p;
        }
    }
    return 0;
}

static void rows_remove(rows_t *r, int32_t a, int64_t e) {
    int64_t p = r->pos[e];
    int64_t last = r->ptr[a] + r->len[a] - 1;
    r->nbr[p] = r->nbr[last];
    r->eid[p] = r->eid[last];
    r->pos[r->eid[p]] = p;
    r->len[a]--;
}

static void rows_free(rows_t *r) {
    free(r->len); free(r->nbr); free(r->eid); free(r->pos);
}

/* A frontier edge with the vertex whose row its enumeration marks. */
typedef struct {
    int32_t side;  /* 0: marks the upper endpoint's row, 1: the lower one's */
    int32_t vtx;
    int64_t e;
} fkey_t;

static int fkey_cmp(const void *pa, const void *pb) {
    const fkey_t *a = (const fkey_t *)pa, *b = (const fkey_t *)pb;
    if (a->side != b->side) return a->side < b->side ? -1 : 1;
    if (a->vtx != b->vtx) return a->vtx < b->vtx ? -1 : 1;
    return a->e < b->e ? -1 : (a->e > b->e);
}

enum { kGroup = 64 };

/*
 * The butterfly made of the frontier edge e and the edges f[0..2] of the
 * remaining graph.  Only the frontier edge of smallest id in it destroys it
 * (so it is destroyed once), lowering the support of each of its edges
 * outside the frontier by one; an edge whose support thereby falls from
 * above the level to the level joins the next frontier.  Returns 1 if e
 * destroyed it.
 */
static inline int destroy(int64_t e, const int64_t f[3], const uint8_t *in_f, int64_t *s,
                          int64_t level, int64_t *next, int64_t *n_next) {
    for (int j = 0; j < 3; ++j)
        if (in_f[f[j]] && f[j] < e) return 0;
    for (int j = 0; j < 3; ++j) {
        if (in_f[f[j]]) continue;
        int64_t old = __atomic_fetch_sub(&s[f[j]], 1, __ATOMIC_RELAXED);
        if (old > level && old - 1 <= level) {
            int64_t slot = __atomic_fetch_add(n_next, 1, __ATOMIC_RELAXED);
            next[slot] = f[j];
        }
    }
    return 1;
}

/*
 * Bitruss numbers by level-synchronous bottom-up peeling with explicit
 * butterfly enumeration.
 *
 * The current level L starts at 0.  Each round takes the frontier F = the
 * remaining edges with support <= L; when it is empty L rises to the
 * minimum remaining support.  Every edge of F gets bitruss number L.  Every
 * butterfly of the remaining graph that contains an edge of F is found by
 * enumeration from that edge and is destroyed once: it is handled by the
 * F-edge of smallest id it contains, which lowers the support of each of
 * its edges outside F by one.  Then F is removed.  An edge whose support
 * drops from above L to at most L during a round forms part of the next
 * frontier.
 *
 * Why this is the bitruss number: while level L is processed, the remaining
 * graph contains the L-bitruss (only edges with fewer than L butterflies
 * in a supergraph of it were removed before), and any remaining edge whose
 * support is at most L in a supergraph of the (L+1)-bitruss is not in the
 * (L+1)-bitruss.  Removing all of F at once is the same as removing its
 * edges one by one at this level (the paper's batch-edge lemma in Section
 * V-B): supports that fall to or below L only cause removal at this level.
 *
 * sup_in may be NULL (supports are then counted first).  stats_out (may be
 * NULL) receives {levels, rounds, butterflies destroyed, max phi}.
 */
int bto_bitruss(int32_t n_upper, int32_t n_lower, int64_t m,
                const int64_t *row_ptr, const int32_t *col,
                const int64_t *sup_in, int64_t *phi_out, int64_t *stats_out,
                int nthreads) {
    graph_t g;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    if (graph_init(&g, n_upper, n_lower, m, row_ptr, col)) return -1;
    side_t U = upper_side(&g), Ls = lower_side(&g);
    rows_t RU, RL;
    int64_t *s = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    uint8_t *in_f = (uint8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
    int64_t *front = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *rest = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int32_t *urow = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int64_t *hop_u = (int64_t *)calloc((size_t)n_upper + 1, sizeof(int64_t));
    int64_t *hop_l = (int64_t *)calloc((size_t)n_lower + 1, sizeof(int64_t));
    fkey_t *fkey = (fkey_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(fkey_t));
    int64_t *gstart = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    if (!s || !alive || !in_f || !front || !next || !rest || !urow || !hop_u || !hop_l ||
        !fkey || !gstart ||
        rows_init(&RU, &U, m) || rows_init(&RL, &Ls, m)) {
        graph_free(&g);
        return -1;
    }
    if (sup_in) {
        memcpy(s, sup_in, (size_t)m * sizeof(int64_t));
    } else {
        int64_t b, p;
        bto_support(n_upper, n_lower, m, row_ptr, col, s, &b, &p, 0, nthreads);
    }
    for (int32_t u = 0; u < n_upper; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) urow[e] = u;
    /* hop(x) = sum of the degrees of x's neighbours: the number of entries
     * an enumeration from x's side walks in the whole graph.  Used only to
     * pick the cheaper of the two symmetric enumerations. */
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = urow[e], v = col[e];
        hop_u[u] += Ls.ptr[v + 1] - Ls.ptr[v];
        hop_l[v] += U.ptr[u + 1] - U.ptr[u];
    }
    for (int64_t e = 0; e < m; ++e) { alive[e] = 1; rest[e] = e; }
    /* rest lists every remaining edge and possibly removed ones; it is
     * compacted whenever more than half of its entries are removed. */
    int64_t n_rest = m, n_alive = m, n_front = 0, level = 0;
    int64_t levels = 0, rounds = 0, destroyed = 0, max_phi = 0;

    int nthr = omp_get_max_threads();
    int32_t **mark_u = (int32_t **)calloc((size_t)nthr, sizeof(int32_t *));
    int32_t **mark_l = (int32_t **)calloc((size_t)nthr, sizeof(int32_t *));
    int64_t **meid_u = (int64_t **)calloc((size_t)nthr, sizeof(int64_t *));
    int64_t **meid_l = (int64_t **)calloc((size_t)nthr, sizeof(int64_t *));
    for (int t = 0; t < nthr; ++t) {
        mark_u[t] = (int32_t *)malloc(((size_t)n_upper + 1) * sizeof(int32_t));
        mark_l[t] = (int32_t *)malloc(((size_t)n_lower + 1) * sizeof(int32_t));
        meid_u[t] = (int64_t *)malloc(((size_t)n_upper + 1) * sizeof(int64_t));
        meid_l[t] = (int64_t *)malloc(((size_t)n_lower + 1) * sizeof(int64_t));
        for (int32_t i = 0; i <= n_upper; ++i) mark_u[t][i] = -1;
        for (int32_t i = 0; i <= n_lower; ++i) mark_l[t][i] = -1;
    }

    while (n_alive > 0) {
        if (n_front == 0) {
            /* New level: the minimum remaining support, then its edges. */
            if (n_rest > 2 * n_alive) {
                int64_t k = 0;
                for (int64_t i = 0; i < n_rest; ++i)
                    if (alive[rest[i]]) rest[k++] = rest[i];
                n_rest = k;
            }
            int64_t mn = INT64_MAX;
#pragma omp parallel for reduction(min : mn) schedule(static)
            for (int64_t i = 0; i < n_rest; ++i) {
                int64_t e = rest[i];
                if (alive[e] && s[e] < mn) mn = s[e];
            }
            if (mn > level) level = mn;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n_rest; ++i) {
                int64_t e = rest[i];
                if (alive[e] && s[e] <= level) {
                    int64_t slot = __atomic_fetch_add(&n_front, 1, __ATOMIC_RELAXED);
                    front[slot] = e;
                }
            }
            ++levels;
        }
        ++rounds;
        for (int64_t i = 0; i < n_front; ++i) {
            in_f[front[i]] = 1;
            phi_out[front[i]] = level;
        }
        if (level > max_phi) max_phi = level;
        /* Each F-edge (u,v) enumerates from the side whose walk is shorter:
         * side 0 marks N(u) and walks N(v) then N(w), side 1 the mirror.
         * F-edges that mark the same vertex are taken in groups of at most
         * kGroup, so a row is marked once per group. */
        for (int64_t i = 0; i < n_front; ++i) {
            int64_t e = front[i];
            int32_t u = urow[e], v = col[e];
            fkey[i].side = hop_l[v] <= hop_u[u] ? 0 : 1;
            fkey[i].vtx = fkey[i].side == 0 ? u : v;
            fkey[i].e = e;
        }
        qsort(fkey, (size_t)n_front, sizeof(fkey_t), fkey_cmp);
        int64_t n_groups = 0;
        for (int64_t i = 0; i < n_front; ++i)
            if (i == 0 || fkey[i].side != fkey[i - 1].side || fkey[i].vtx != fkey[i - 1].vtx ||
                i - gstart[n_groups - 1] == kGroup)
                gstart[n_groups++] = i;
        gstart[n_groups] = n_front;
        int64_t n_next = 0;
#pragma omp parallel reduction(+ : destroyed)
        {
            int t = omp_get_thread_num();
            int32_t *mu = mark_u[t], *ml = mark_l[t];
            int64_t *eu = meid_u[t], *el = meid_l[t];
#pragma omp for schedule(dynamic, 1)
            for (int64_t gi = 0; gi < n_groups; ++gi) {
                const int32_t stamp = (int32_t)gi;
                const int32_t a = fkey[gstart[gi]].vtx;
                int64_t f[3];
                if (fkey[gstart[gi]].side == 0) {
                    /* Mark the remaining neighbours x of u = a; for each
                     * F-edge (u,v) walk the remaining w in N(v) and x in
                     * N(w): (w,x) closes [u,v,w,x]. */
                    for (int64_t p = RU.ptr[a]; p < RU.ptr[a] + RU.len[a]; ++p) {
                        ml[RU.nbr[p]] = stamp;
                        el[RU.nbr[p]] = RU.eid[p];
                    }
                    for (int64_t j = gstart[gi]; j < gstart[gi + 1]; ++j) {
                        int64_t e = fkey[j].e;
                        int32_t u = a, v = col[e];
                        for (int64_t q = RL.ptr[v]; q < RL.ptr[v] + RL.len[v]; ++q) {
                            int32_t w = RL.nbr[q];
                            if (w == u) continue;
                            for (int64_t r = RU.ptr[w]; r < RU.ptr[w] + RU.len[w]; ++r) {
                                int32_t x = RU.nbr[r];
                                if (x == v || ml[x] != stamp) continue;
                                f[0] = RL.eid[q]; f[1] = el[x]; f[2] = RU.eid[r];
                                destroyed += destroy(e, f, in_f, s, level, next, &n_next);
                            }
                        }
                    }
                    for (int64_t p = RU.ptr[a]; p < RU.ptr[a] + RU.len[a]; ++p) ml[RU.nbr[p]] = -1;
                } else {
                    /* Mirror: mark the remaining neighbours w of v = a; for
                     * each F-edge (u,v) walk the remaining x in N(u) and w
                     * in N(x). */
                    for (int64_t q = RL.ptr[a]; q < RL.ptr[a] + RL.len[a]; ++q) {
                        mu[RL.nbr[q]] = stamp;
                        eu[RL.nbr[q]] = RL.eid[q];
                    }
                    for (int64_t j = gstart[gi]; j < gstart[gi + 1]; ++j) {
                        int64_t e = fkey[j].e;
                        int32_t u = urow[e], v = a;
                        for (int64_t p = RU.ptr[u]; p < RU.ptr[u] + RU.len[u]; ++p) {
                            int32_t x = RU.nbr[p];
                            if (x == v) continue;
                            for (int64_t q = RL.ptr[x]; q < RL.ptr[x] + RL.len[x]; ++q) {
                                int32_t w = RL.nbr[q];
                                if (w == u || mu[w] != stamp) continue;
                                f[0] = eu[w]; f[1] = RU.eid[p]; f[2] = RL.eid[q];
                                destroyed += destroy(e, f, in_f, s, level, next, &n_next);
                            }
                        }
                    }
                    for (int64_t q = RL.ptr[a]; q < RL.ptr[a] + RL.len[a]; ++q) mu[RL.nbr[q]] = -1;
                }
            }
        }
        /* Remove F from the graph. */
        for (int64_t i = 0; i < n_front; ++i) {
            int64_t e = front[i];
            alive[e] = 0;
            in_f[e] = 0;
            rows_remove(&RU, urow[e], e);
            rows_remove(&RL, col[e], e);
        }
        n_alive -= n_front;
        int64_t *tmp = front; front = next; next = tmp;
        n_front = n_next;
    }
    if (stats_out) {
        stats_out[0] = levels;
        stats_out[1] = rounds;
        stats_out[2] = destroyed;
        stats_out[3] = max_phi;
    }
    for (int t = 0; t < nthr; ++t) {
        free(mark_u[t]); free(mark_l[t]); free(meid_u[t]); free(meid_l[t]);
    }
    free(mark_u); free(mark_l); free(meid_u); free(meid_l);
    free(s); free(alive); free(in_f); free(front); free(next); free(rest);
    free(urow); free(hop_u); free(hop_l); free(fkey); free(gstart);
    rows_free(&RU); rows_free(&RL);
    graph_free(&g);
    return 0;
}

int bto_max_threads(void) { return omp_get_max_threads(); }
