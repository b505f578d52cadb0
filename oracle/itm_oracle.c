/*
 * CPU oracle for Interval Tree Matching (ITM) -- TEST INFRASTRUCTURE ONLY.
 *
 * Marzolla, D'Angelo, Mandrioli, "A Parallel Data Distribution Management
 * Algorithm", DS-RT 2013.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it; the GPU
 * library never does, and the two share no source.
 *
 * What it computes (Sec. III, problem statement): for subscription extents
 * S_1..S_n and update extents U_1..U_m in d dimensions, every pair (j, i)
 * with S_i and U_j intersecting.  Ids are 0-based here.  Two extents
 * intersect iff their projections intersect in every dimension (Sec. III-A).
 * The result is returned as ascending 64-bit keys (j << 32) | i, i.e. the
 * nonzeros of the intersection matrix M listed column (update) by column.
 *
 * Segment predicate.  Algorithm 1 prints a strict test while the text writes
 * closed segments [low, high]; this oracle follows the closed reading
 * (x.low <= y.high and y.low <= x.high).  The strict form is kept behind a
 * flag as a diagnostic only.
 *
 * Functions and the passage each follows:
 *   itree_create      Sec. IV: interval tree as a balanced search tree ordered
 *                     by lower bound (ties by upper bound; the id breaks the
 *                     remaining ties), each node holding maxupper and
 *                     minlower of its subtree.  Built statically by taking
 *                     the median as the root (a perfectly balanced BST).
 *   itree_query       the query of Sec. IV (Algorithm 4), closed form, as a
 *                     search over a stack of pending subtrees: a subtree is
 *                     skipped when maxupper < q.lower or minlower > q.upper;
 *                     otherwise its root is tested and its parts examined,
 *                     the right part only while the root's lower bound is
 *                     <= q.upper (the closed counterpart of the printed
 *                     strict condition).
 *   oracle_itm        Algorithm 5 per dimension, then the d-way combine of
 *                     Sec. III-A written literally: per update, sort the d
 *                     per-dimension lists and intersect them.  The parallel
 *                     form splits updates into contiguous blocks, one per
 *                     thread (Sec. IV, "Parallelizing ITM"), and concatenates
 *                     the blocks in order.
 *   oracle_brute      Algorithm 2 (Brute Force) with the closed predicate.
 *   oracle_sbm_1d     Algorithm 3 (Sort-Based Matching, Sec. III-D), d = 1:
 *                     endpoints sorted, sweep with active sets; at equal
 *                     coordinates lower endpoints come first (closed reading).
 *   oracle_itm_1d_visits  Algorithm 4 per query with a visit counter, for the
 *                     O(min{n, (k+1) log n}) cost bound of Sec. IV.
 *   oracle_pst_1d     the alternative Sec. IV names: a priority search tree
 *                     (McCreight) over the points (lower, upper), queried
 *                     with lower <= q.upper and upper >= q.lower (closed), in
 *                     O(log n + k); returns the pairs, or per query the
 *                     nodes visited and the hits, to compare with Algorithm 4.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_INPUT (-2)
#define OR_E_NOMEM (-4)

/* ------------------------------------------------------------------ */
/* growable vectors                                                    */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t* v; size_t n, cap; int oom; } vec32;
typedef struct { uint64_t* v; size_t n, cap; int oom; } vec64;

static void v32_push(vec32* a, uint32_t x) {
    if (a->n == a->cap) {
        size_t nc = a->cap ? a->cap * 2 : 64;
        uint32_t* p = (uint32_t*)realloc(a->v, nc * sizeof(uint32_t));
        if (!p) { a->oom = 1; return; }
        a->v = p; a->cap = nc;
    }
    a->v[a->n++] = x;
}

static void v64_push(vec64* a, uint64_t x) {
    if (a->n == a->cap) {
        size_t nc = a->cap ? a->cap * 2 : 256;
        uint64_t* p = (uint64_t*)realloc(a->v, nc * sizeof(uint64_t));
        if (!p) { a->oom = 1; return; }
        a->v = p; a->cap = nc;
    }
    a->v[a->n++] = x;
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ */
/* the segment predicate (Algorithm 1)                                 */
/* ------------------------------------------------------------------ */
static int intersect_1d(float xl, float xh, float yl, float yh, int strict) {
    if (strict) return xl < yh && yl < xh;
    return xl <= yh && yl <= xh;
}

/* ------------------------------------------------------------------ */
/* interval tree (Sec. IV)                                             */
/* ------------------------------------------------------------------ */
typedef struct { float lo, hi; uint32_t id; } seg_t;
typedef struct {
    seg_t in;
    float maxupper, minlower;
    int32_t left, right;
} node_t;
typedef struct { node_t* nodes; int32_t root; uint32_t n; } itree_t;

static int cmp_seg(const void* a, const void* b) {
    const seg_t* x = (const seg_t*)a;
    const seg_t* y = (const seg_t*)b;
    if (x->lo < y->lo) return -1;
    if (x->lo > y->lo) return 1;
    if (x->hi < y->hi) return -1;
    if (x->hi > y->hi) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Subtree over sorted[lo, hi): the median is the node, halves are children. */
static int32_t build_rec(node_t* nodes, const seg_t* sorted, int32_t lo, int32_t hi) {
    if (lo >= hi) return -1;
    int32_t mid = lo + (hi - lo) / 2;
    node_t* x = &nodes[mid];
    x->in = sorted[mid];
    x->left = build_rec(nodes, sorted, lo, mid);
    x->right = build_rec(nodes, sorted, mid + 1, hi);
    x->maxupper = x->in.hi;
    x->minlower = x->in.lo;
    if (x->left >= 0) {
        const node_t* l = &nodes[x->left];
        if (l->maxupper > x->maxupper) x->maxupper = l->maxupper;
        if (l->minlower < x->minlower) x->minlower = l->minlower;
    }
    if (x->right >= 0) {
        const node_t* r = &nodes[x->right];
        if (r->maxupper > x->maxupper) x->maxupper = r->maxupper;
        if (r->minlower < x->minlower) x->minlower = r->minlower;
    }
    return mid;
}

static int itree_create(itree_t* t, const float* lo, const float* hi, uint32_t n) {
    t->n = n;
    t->root = -1;
    t->nodes = NULL;
    if (n == 0) return OR_OK;
    seg_t* s = (seg_t*)malloc((size_t)n * sizeof(seg_t));
    t->nodes = (node_t*)malloc((size_t)n * sizeof(node_t));
    if (!s || !t->nodes) { free(s); free(t->nodes); t->nodes = NULL; return OR_E_NOMEM; }
    for (uint32_t i = 0; i < n; ++i) { s[i].lo = lo[i]; s[i].hi = hi[i]; s[i].id = i; }
    qsort(s, n, sizeof(seg_t), cmp_seg);
    t->root = build_rec(t->nodes, s, 0, (int32_t)n);
    free(s);
    return OR_OK;
}

static void itree_free(itree_t* t) { free(t->nodes); t->nodes = NULL; }

/* The subscriptions of a tree meeting q (Sec. IV, the query of an interval
 * tree), closed form; the strict form only under the diagnostic flag.
 *
 * Facts of Sec. IV this rests on: (1) no interval of a subtree meets q when
 * the subtree's largest upper bound lies below q.lower or its smallest lower
 * bound lies above q.upper; (2) the tree is ordered by lower bound, so every
 * interval in the right part of a node has a lower bound at least the node's,
 * and once that bound lies beyond q.upper no interval there can meet q.
 * Every other subtree is examined: its root is tested, and its two parts are
 * put on a stack of subtrees still to examine.  Which order the stack gives
 * does not matter: the caller sorts the ids.  `visits` counts the subtrees
 * examined (each non-empty one taken from the stack), the quantity bounded by
 * O(min{n, (k+1) log n}) in Sec. IV.  The stack never holds more than one
 * pending part per level of the tree plus the one being examined. */
#define ORACLE_STACK 128
static void itree_query(const itree_t* t, float ql, float qh, int strict, vec32* out,
                        uint64_t* visits) {
    int32_t pending[ORACLE_STACK];
    int top = 0;
    pending[top++] = t->root;
    while (top > 0) {
        int32_t xi = pending[--top];
        if (xi < 0) continue;
        const node_t* x = &t->nodes[xi];
        if (visits) ++*visits;
        int none_inside = x->maxupper < ql || x->minlower > qh;      /* fact (1) */
        if (none_inside) continue;
        if (intersect_1d(x->in.lo, x->in.hi, ql, qh, strict)) v32_push(out, x->in.id);
        int right_may_meet = strict ? (x->in.lo < qh) : (x->in.lo <= qh);  /* fact (2) */
        if (right_may_meet) pending[top++] = x->right;
        pending[top++] = x->left;
    }
}

static int tree_height(const itree_t* t, int32_t xi) {
    if (xi < 0) return 0;
    int a = tree_height(t, t->nodes[xi].left);
    int b = tree_height(t, t->nodes[xi].right);
    return 1 + (a > b ? a : b);
}

/* ------------------------------------------------------------------ */
/* input checks                                                        */
/* ------------------------------------------------------------------ */
static int check_set(const float* lo, const float* hi, uint64_t cnt) {
    for (uint64_t i = 0; i < cnt; ++i) {
        if (!isfinite(lo[i]) || !isfinite(hi[i]) || lo[i] > hi[i]) return OR_E_INPUT;
    }
    return OR_OK;
}

static int check_args(const float* s_lo, const float* s_hi, uint32_t n,
                      const float* u_lo, const float* u_hi, uint32_t m, uint32_t d) {
    if (d < 1 || d > 8) return OR_E_ARG;
    if ((n && (!s_lo || !s_hi)) || (m && (!u_lo || !u_hi))) return OR_E_ARG;
    if (check_set(s_lo, s_hi, (uint64_t)n * d) != OR_OK) return OR_E_INPUT;
    if (check_set(u_lo, u_hi, (uint64_t)m * d) != OR_OK) return OR_E_INPUT;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* ITM, d dimensions, literal per-update intersection of the d lists   */
/* ------------------------------------------------------------------ */
static void itm_block(const itree_t* trees, const float* u_lo, const float* u_hi,
                      uint32_t m, uint32_t d, uint32_t j0, uint32_t j1, int strict,
                      vec64* out) {
    vec32 lists[8];
    memset(lists, 0, sizeof(lists));
    size_t pos[8];
    for (uint32_t j = j0; j < j1; ++j) {
        for (uint32_t k = 0; k < d; ++k) {
            lists[k].n = 0;
            float ql = u_lo[(size_t)k * m + j], qh = u_hi[(size_t)k * m + j];
            itree_query(&trees[k], ql, qh, strict, &lists[k], NULL);
            qsort(lists[k].v, lists[k].n, sizeof(uint32_t), cmp_u32);
            pos[k] = 0;
        }
        /* intersect the sorted lists: walk list 0, advance the others */
        for (size_t a = 0; a < lists[0].n; ++a) {
            uint32_t s = lists[0].v[a];
            int all = 1;
            for (uint32_t k = 1; k < d && all; ++k) {
                while (pos[k] < lists[k].n && lists[k].v[pos[k]] < s) ++pos[k];
                if (pos[k] >= lists[k].n || lists[k].v[pos[k]] != s) all = 0;
            }
            if (all) v64_push(out, ((uint64_t)j << 32) | s);
        }
    }
    for (uint32_t k = 0; k < d; ++k) { if (lists[k].oom) out->oom = 1; free(lists[k].v); }
}

int oracle_itm(const float* s_lo, const float* s_hi, uint32_t n,
               const float* u_lo, const float* u_hi, uint32_t m, uint32_t d,
               int threads, int strict, uint64_t** out_keys, uint64_t* out_count) {
    if (!out_keys || !out_count) return OR_E_ARG;
    *out_keys = NULL;
    *out_count = 0;
    int rc = check_args(s_lo, s_hi, n, u_lo, u_hi, m, d);
    if (rc != OR_OK) return rc;
    if (n == 0 || m == 0) return OR_OK;
    itree_t trees[8];
    memset(trees, 0, sizeof(trees));
    for (uint32_t k = 0; k < d; ++k) {
        rc = itree_create(&trees[k], s_lo + (size_t)k * n, s_hi + (size_t)k * n, n);
        if (rc != OR_OK) { for (uint32_t q = 0; q < d; ++q) itree_free(&trees[q]); return rc; }
    }
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > m) threads = (int)m;
    vec64* parts = (vec64*)calloc((size_t)threads, sizeof(vec64));
    if (!parts) { for (uint32_t q = 0; q < d; ++q) itree_free(&trees[q]); return OR_E_NOMEM; }
#ifdef _OPENMP
#pragma omp parallel for num_threads(threads) schedule(static, 1)
#endif
    for (int t = 0; t < threads; ++t) {
        uint32_t j0 = (uint32_t)(((uint64_t)m * t) / threads);
        uint32_t j1 = (uint32_t)(((uint64_t)m * (t + 1)) / threads);
        itm_block(trees, u_lo, u_hi, m, d, j0, j1, strict, &parts[t]);
    }
    uint64_t total = 0;
    int oom = 0;
    for (int t = 0; t < threads; ++t) { total += parts[t].n; oom |= parts[t].oom; }
    uint64_t* keys = NULL;
    if (!oom && total) {
        keys = (uint64_t*)malloc(total * sizeof(uint64_t));
        if (!keys) oom = 1;
    }
    if (!oom) {
        uint64_t at = 0;
        for (int t = 0; t < threads; ++t) {
            if (parts[t].n) memcpy(keys + at, parts[t].v, parts[t].n * sizeof(uint64_t));
            at += parts[t].n;
        }
    }
    for (int t = 0; t < threads; ++t) free(parts[t].v);
    free(parts);
    for (uint32_t q = 0; q < d; ++q) itree_free(&trees[q]);
    if (oom) { free(keys); return OR_E_NOMEM; }
    *out_keys = keys;
    *out_count = total;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2, brute force                                            */
/* ------------------------------------------------------------------ */
int oracle_brute(const float* s_lo, const float* s_hi, uint32_t n,
                 const float* u_lo, const float* u_hi, uint32_t m, uint32_t d,
                 int strict, uint64_t** out_keys, uint64_t* out_count) {
    if (!out_keys || !out_count) return OR_E_ARG;
    *out_keys = NULL;
    *out_count = 0;
    int rc = check_args(s_lo, s_hi, n, u_lo, u_hi, m, d);
    if (rc != OR_OK) return rc;
    vec64 out = {0};
    for (uint32_t j = 0; j < m; ++j) {
        for (uint32_t i = 0; i < n; ++i) {
            int all = 1;
            for (uint32_t k = 0; k < d && all; ++k) {
                all = intersect_1d(s_lo[(size_t)k * n + i], s_hi[(size_t)k * n + i],
                                   u_lo[(size_t)k * m + j], u_hi[(size_t)k * m + j], strict);
            }
            if (all) v64_push(&out, ((uint64_t)j << 32) | i);
        }
    }
    if (out.oom) { free(out.v); return OR_E_NOMEM; }
    *out_keys = out.v;
    *out_count = out.n;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Sort-Based Matching, d = 1 (Sec. III-D)                             */
/* ------------------------------------------------------------------ */
typedef struct { float x; uint32_t tag; } endpoint_t; /* tag: id<<2 | upper<<1 | isupdate */

static int cmp_endpoint(const void* a, const void* b) {
    const endpoint_t* p = (const endpoint_t*)a;
    const endpoint_t* q = (const endpoint_t*)b;
    if (p->x < q->x) return -1;
    if (p->x > q->x) return 1;
    /* closed segments: at an equal coordinate every lower endpoint is
       processed before any upper endpoint, so touching segments meet */
    uint32_t pu = (p->tag >> 1) & 1u, qu = (q->tag >> 1) & 1u;
    if (pu != qu) return (int)pu - (int)qu;
    return (p->tag > q->tag) - (p->tag < q->tag);
}

typedef struct { uint32_t* ids; uint32_t* where; uint32_t n; } active_t;

static void act_add(active_t* a, uint32_t id) { a->where[id] = a->n; a->ids[a->n++] = id; }
static void act_del(active_t* a, uint32_t id) {
    uint32_t w = a->where[id], last = a->ids[--a->n];
    a->ids[w] = last;
    a->where[last] = w;
}

int oracle_sbm_1d(const float* s_lo, const float* s_hi, uint32_t n,
                  const float* u_lo, const float* u_hi, uint32_t m,
                  uint64_t** out_keys, uint64_t* out_count) {
    if (!out_keys || !out_count) return OR_E_ARG;
    *out_keys = NULL;
    *out_count = 0;
    int rc = check_args(s_lo, s_hi, n, u_lo, u_hi, m, 1);
    if (rc != OR_OK) return rc;
    if (n >= (1u << 30) || m >= (1u << 30)) return OR_E_ARG;
    size_t E = 2 * ((size_t)n + m);
    endpoint_t* L = (endpoint_t*)malloc((E ? E : 1) * sizeof(endpoint_t));
    active_t subs = {(uint32_t*)malloc((n + 1) * sizeof(uint32_t)),
                     (uint32_t*)malloc((n + 1) * sizeof(uint32_t)), 0};
    active_t upds = {(uint32_t*)malloc((m + 1) * sizeof(uint32_t)),
                     (uint32_t*)malloc((m + 1) * sizeof(uint32_t)), 0};
    vec64 out = {0};
    if (!L || !subs.ids || !subs.where || !upds.ids || !upds.where) { rc = OR_E_NOMEM; goto done; }
    size_t e = 0;
    for (uint32_t i = 0; i < n; ++i) {
        L[e].x = s_lo[i]; L[e++].tag = (i << 2) | 0u;
        L[e].x = s_hi[i]; L[e++].tag = (i << 2) | 2u;
    }
    for (uint32_t j = 0; j < m; ++j) {
        L[e].x = u_lo[j]; L[e++].tag = (j << 2) | 1u;
        L[e].x = u_hi[j]; L[e++].tag = (j << 2) | 3u;
    }
    qsort(L, E, sizeof(endpoint_t), cmp_endpoint);
    for (size_t p = 0; p < E; ++p) {
        uint32_t id = L[p].tag >> 2;
        int upper = (L[p].tag >> 1) & 1, isupd = L[p].tag & 1;
        if (!isupd) {
            if (!upper) act_add(&subs, id);
            else {
                act_del(&subs, id);
                for (uint32_t a = 0; a < upds.n; ++a) v64_push(&out, ((uint64_t)upds.ids[a] << 32) | id);
            }
        } else {
            if (!upper) act_add(&upds, id);
            else {
                act_del(&upds, id);
                for (uint32_t a = 0; a < subs.n; ++a) v64_push(&out, ((uint64_t)id << 32) | subs.ids[a]);
            }
        }
    }
    if (out.oom) { rc = OR_E_NOMEM; goto done; }
    qsort(out.v, out.n, sizeof(uint64_t), cmp_u64);
    *out_keys = out.v;
    *out_count = out.n;
    out.v = NULL;
    rc = OR_OK;
done:
    free(L); free(subs.ids); free(subs.where); free(upds.ids); free(upds.where); free(out.v);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Algorithm 4 with visit counts, one dimension (cost bound, Sec. IV)  */
/* ------------------------------------------------------------------ */
int oracle_itm_1d_visits(const float* s_lo, const float* s_hi, uint32_t n,
                         const float* u_lo, const float* u_hi, uint32_t m,
                         uint64_t* visits, uint32_t* hits, uint32_t* height) {
    int rc = check_args(s_lo, s_hi, n, u_lo, u_hi, m, 1);
    if (rc != OR_OK) return rc;
    itree_t t;
    rc = itree_create(&t, s_lo, s_hi, n);
    if (rc != OR_OK) return rc;
    if (height) *height = (uint32_t)tree_height(&t, t.root);
    vec32 lst = {0};
    for (uint32_t j = 0; j < m; ++j) {
        uint64_t v = 0;
        lst.n = 0;
        itree_query(&t, u_lo[j], u_hi[j], 0, &lst, &v);
        visits[j] = v;
        hits[j] = (uint32_t)lst.n;
    }
    free(lst.v);
    itree_free(&t);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Priority search tree (Sec. IV names it as a drop-in alternative)    */
/* ------------------------------------------------------------------ */
/* Every node holds the point of largest upper bound among the points of its
 * subtree; the other points, in lower-bound order, are split at the median
 * into the two subtrees (left: smaller lower bounds).  min_lo is the smallest
 * lower bound in the node's subtree (the node's point included). */
typedef struct { seg_t pt; float min_lo; int32_t left, right; } pnode_t;
typedef struct { pnode_t* nodes; int32_t count; int32_t root; } pst_t;

/* Subtree over the lower-bound-sorted points seg[lo, hi). */
static int32_t pst_build_rec(pst_t* t, seg_t* seg, int32_t lo, int32_t hi) {
    if (lo >= hi) return -1;
    int32_t best = lo;
    for (int32_t i = lo + 1; i < hi; ++i) {
        if (seg[i].hi > seg[best].hi) best = i;  /* first of equal uppers */
    }
    seg_t top = seg[best];
    const float min_lo = seg[lo].lo;
    /* remove it, keeping the others in lower-bound order */
    memmove(&seg[lo + 1], &seg[lo], (size_t)(best - lo) * sizeof(seg_t));
    int32_t v = t->count++;
    t->nodes[v].pt = top;
    t->nodes[v].min_lo = min_lo;
    int32_t rest = lo + 1, mid = rest + (hi - rest) / 2;
    int32_t l = pst_build_rec(t, seg, rest, mid);
    int32_t r = pst_build_rec(t, seg, mid, hi);
    t->nodes[v].left = l;
    t->nodes[v].right = r;
    return v;
}

static int pst_create(pst_t* t, const float* lo, const float* hi, uint32_t n) {
    t->count = 0;
    t->root = -1;
    t->nodes = NULL;
    if (n == 0) return OR_OK;
    seg_t* s = (seg_t*)malloc((size_t)n * sizeof(seg_t));
    t->nodes = (pnode_t*)malloc((size_t)n * sizeof(pnode_t));
    if (!s || !t->nodes) { free(s); free(t->nodes); t->nodes = NULL; return OR_E_NOMEM; }
    for (uint32_t i = 0; i < n; ++i) { s[i].lo = lo[i]; s[i].hi = hi[i]; s[i].id = i; }
    qsort(s, n, sizeof(seg_t), cmp_seg);
    t->root = pst_build_rec(t, s, 0, (int32_t)n);
    free(s);
    return OR_OK;
}

/* Points with lower <= qh and upper >= ql (the closed segments meeting q):
 * a subtree is left as soon as its node's upper is below ql (no point below
 * it has a larger upper) or its smallest lower bound is above qh (no point
 * in it starts early enough); otherwise the node's point is reported if it
 * starts early enough, and both subtrees are searched. */
static void pst_query(const pst_t* t, int32_t v, float ql, float qh, vec32* out,
                      uint64_t* visits) {
    if (v < 0) return;
    const pnode_t* x = &t->nodes[v];
    if (visits) ++*visits;
    if (x->pt.hi < ql || x->min_lo > qh) return;
    if (x->pt.lo <= qh) v32_push(out, x->pt.id);
    pst_query(t, x->left, ql, qh, out, visits);
    pst_query(t, x->right, ql, qh, out, visits);
}

int oracle_pst_1d(const float* s_lo, const float* s_hi, uint32_t n,
                  const float* u_lo, const float* u_hi, uint32_t m,
                  uint64_t** out_keys, uint64_t* out_count,
                  uint64_t* visits, uint32_t* hits) {
    if (out_keys) *out_keys = NULL;
    if (out_count) *out_count = 0;
    int rc = check_args(s_lo, s_hi, n, u_lo, u_hi, m, 1);
    if (rc != OR_OK) return rc;
    pst_t t;
    rc = pst_create(&t, s_lo, s_hi, n);
    if (rc != OR_OK) return rc;
    vec32 lst = {0};
    vec64 keys = {0};
    for (uint32_t j = 0; j < m; ++j) {
        uint64_t v = 0;
        lst.n = 0;
        pst_query(&t, t.root, u_lo[j], u_hi[j], &lst, &v);
        if (visits) visits[j] = v;
        if (hits) hits[j] = (uint32_t)lst.n;
        if (out_keys) {
            qsort(lst.v, lst.n, sizeof(uint32_t), cmp_u32);
            for (size_t a = 0; a < lst.n; ++a) v64_push(&keys, ((uint64_t)j << 32) | lst.v[a]);
        }
    }
    int oom = lst.oom || keys.oom;
    free(lst.v);
    free(t.nodes);
    if (oom) { free(keys.v); return OR_E_NOMEM; }
    if (out_keys) { *out_keys = keys.v; *out_count = keys.n; } else { free(keys.v); }
    return OR_OK;
}

void oracle_free(void* p) { free(p); }

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
