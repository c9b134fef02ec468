/*
 * Broad-phase contact candidate generation for the synthetic scenes.
 *
 * Input generator shared by the oracle-side tests and the GPU path.  It holds
 * none of the barrier method's arithmetic: it only compares axis-aligned
 * bounding boxes.  A candidate is emitted when the box of one primitive,
 * inflated by dhat, overlaps the box of the other primitive and the two
 * primitives belong to different objects.  Whether a candidate is actually
 * closer than dhat (and of which sub-type it is) is decided downstream by
 * the pair evaluation itself.
 *
 * Output tuples use the paper's sign encoding of contact pairs (Sec. 7.2,
 * "Data structures"):
 *   point-triangle candidate  [-(p+1), t0, t1, t2]
 *   edge-edge candidate       [a0, a1, b0, b1]
 * The list is sorted lexicographically on the decoded vertex ids so the
 * result does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { int64_t key; int32_t prim; } cell_entry;

static int cmp_cell_entry(const void* a, const void* b) {
    const cell_entry* x = (const cell_entry*)a;
    const cell_entry* y = (const cell_entry*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->prim > y->prim) - (x->prim < y->prim);
}

static int64_t cell_key(int64_t ix, int64_t iy, int64_t iz) {
    /* 21 bits per axis, offset so small negatives stay ordered */
    const int64_t off = 1 << 20;
    return ((ix + off) << 42) | ((iy + off) << 21) | (iz + off);
}

typedef struct { double lo[3], hi[3]; } box3;

static void prim_box(const double* x, const int32_t* v, int n, box3* b) {
    for (int d = 0; d < 3; ++d) { b->lo[d] = INFINITY; b->hi[d] = -INFINITY; }
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) {
            double c = x[3 * (int64_t)v[k] + d];
            if (c < b->lo[d]) b->lo[d] = c;
            if (c > b->hi[d]) b->hi[d] = c;
        }
}

static int boxes_overlap(const box3* a, double infl, const box3* b) {
    for (int d = 0; d < 3; ++d)
        if (a->lo[d] - infl > b->hi[d] || b->lo[d] > a->hi[d] + infl) return 0;
    return 1;
}

/* Sorted (cell, primitive) table of the raw boxes of n primitives. */
static cell_entry* build_table(const double* x, const int32_t* prims, int nper, int64_t n,
                               double h, const double* org, int64_t* out_len) {
    int64_t cap = n * 8 + 16, len = 0;
    cell_entry* t = (cell_entry*)malloc(sizeof(cell_entry) * cap);
    for (int64_t i = 0; i < n; ++i) {
        box3 b; prim_box(x, prims + nper * i, nper, &b);
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = (int64_t)floor((b.lo[d] - org[d]) / h);
            hi[d] = (int64_t)floor((b.hi[d] - org[d]) / h);
        }
        for (int64_t a = lo[0]; a <= hi[0]; ++a)
            for (int64_t c = lo[1]; c <= hi[1]; ++c)
                for (int64_t e = lo[2]; e <= hi[2]; ++e) {
                    if (len == cap) { cap *= 2; t = (cell_entry*)realloc(t, sizeof(cell_entry) * cap); }
                    t[len].key = cell_key(a, c, e); t[len].prim = (int32_t)i; ++len;
                }
    }
    qsort(t, len, sizeof(cell_entry), cmp_cell_entry);
    *out_len = len;
    return t;
}

static int64_t lower_bound(const cell_entry* t, int64_t n, int64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) { int64_t m = (lo + hi) / 2; if (t[m].key < key) lo = m + 1; else hi = m; }
    return lo;
}

typedef struct { int32_t* v; int64_t n, cap; } tuple_vec;

static void push4(tuple_vec* tv, int32_t a, int32_t b, int32_t c, int32_t d) {
    if (tv->n == tv->cap) {
        tv->cap = tv->cap ? tv->cap * 2 : 1024;
        tv->v = (int32_t*)realloc(tv->v, sizeof(int32_t) * 4 * tv->cap);
    }
    int32_t* o = tv->v + 4 * tv->n++;
    o[0] = a; o[1] = b; o[2] = c; o[3] = d;
}

static int64_t decoded0(const int32_t* t) { return t[0] < 0 ? -(int64_t)t[0] - 1 : t[0]; }

static int cmp_tuple(const void* a, const void* b) {
    const int32_t* x = (const int32_t*)a;
    const int32_t* y = (const int32_t*)b;
    /* point-triangle candidates first, then edge-edge; then by vertex ids */
    int kx = x[0] < 0 ? 0 : 1, ky = y[0] < 0 ? 0 : 1;
    if (kx != ky) return kx - ky;
    int64_t dx = decoded0(x), dy = decoded0(y);
    if (dx != dy) return dx < dy ? -1 : 1;
    for (int k = 1; k < 4; ++k)
        if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}

/*
 * Returns the number of tuples; *out receives a malloc'd int32[n][4] that the
 * caller releases with bp_free.  vobj[v] is the object id of vertex v.
 */
int64_t bp_candidates(int32_t V, const double* x, const int32_t* vobj,
                      int64_t F, const int32_t* tris, int64_t E, const int32_t* edges,
                      double dhat, int want_pt, int want_ee, int32_t** out) {
    double org[3] = {INFINITY, INFINITY, INFINITY}, ext = 0.0;
    for (int64_t v = 0; v < V; ++v)
        for (int d = 0; d < 3; ++d) if (x[3 * v + d] < org[d]) org[d] = x[3 * v + d];
    for (int d = 0; d < 3; ++d) org[d] -= 4 * dhat;
    for (int64_t i = 0; i < F; ++i) {
        box3 b; prim_box(x, tris + 3 * i, 3, &b);
        for (int d = 0; d < 3; ++d) if (b.hi[d] - b.lo[d] > ext) ext = b.hi[d] - b.lo[d];
    }
    for (int64_t i = 0; i < E; ++i) {
        box3 b; prim_box(x, edges + 2 * i, 2, &b);
        for (int d = 0; d < 3; ++d) if (b.hi[d] - b.lo[d] > ext) ext = b.hi[d] - b.lo[d];
    }
    double h = ext + dhat;
    if (h <= 0) h = dhat > 0 ? dhat : 1.0;

    tuple_vec all = {0, 0, 0};

    if (want_pt && F > 0) {
        int64_t tl; cell_entry* tt = build_table(x, tris, 3, F, h, org, &tl);
        int nth = 1;
#ifdef _OPENMP
        #pragma omp parallel
        { _Pragma("omp single") nth = omp_get_num_threads(); }
#endif
        tuple_vec* loc = (tuple_vec*)calloc(nth, sizeof(tuple_vec));
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t p = 0; p < V; ++p) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            box3 pb; int32_t pv = (int32_t)p; prim_box(x, &pv, 1, &pb);
            /* the point's inflated box may touch up to 2 cells per axis */
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = (int64_t)floor((pb.lo[d] - dhat - org[d]) / h);
                hi[d] = (int64_t)floor((pb.hi[d] + dhat - org[d]) / h);
            }
            for (int64_t a = lo[0]; a <= hi[0]; ++a)
                for (int64_t c = lo[1]; c <= hi[1]; ++c)
                    for (int64_t e = lo[2]; e <= hi[2]; ++e) {
                        int64_t key = cell_key(a, c, e);
                        for (int64_t k = lower_bound(tt, tl, key); k < tl && tt[k].key == key; ++k) {
                            const int32_t* t = tris + 3 * (int64_t)tt[k].prim;
                            if (vobj[t[0]] == vobj[p]) continue;
                            if (t[0] == p || t[1] == p || t[2] == p) continue;
                            box3 tb; prim_box(x, t, 3, &tb);
                            if (!boxes_overlap(&pb, dhat, &tb)) continue;
                            /* report once: in the cell holding the min corner of the overlap */
                            int own = 1;
                            for (int d = 0; d < 3 && own; ++d) {
                                double m = fmax(pb.lo[d] - dhat, tb.lo[d]);
                                int64_t cd = (int64_t)floor((m - org[d]) / h);
                                own = (d == 0 ? a : d == 1 ? c : e) == cd;
                            }
                            if (!own) continue;
                            push4(&loc[tid], -(p + 1), t[0], t[1], t[2]);
                        }
                    }
        }
        for (int i = 0; i < nth; ++i) {
            for (int64_t k = 0; k < loc[i].n; ++k)
                push4(&all, loc[i].v[4 * k], loc[i].v[4 * k + 1], loc[i].v[4 * k + 2], loc[i].v[4 * k + 3]);
            free(loc[i].v);
        }
        free(loc); free(tt);
    }

    if (want_ee && E > 0) {
        int64_t tl; cell_entry* tt = build_table(x, edges, 2, E, h, org, &tl);
        int nth = 1;
#ifdef _OPENMP
        #pragma omp parallel
        { _Pragma("omp single") nth = omp_get_num_threads(); }
#endif
        tuple_vec* loc = (tuple_vec*)calloc(nth, sizeof(tuple_vec));
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < E; ++i) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            const int32_t* ea = edges + 2 * i;
            box3 ab; prim_box(x, ea, 2, &ab);
            int64_t lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = (int64_t)floor((ab.lo[d] - dhat - org[d]) / h);
                hi[d] = (int64_t)floor((ab.hi[d] + dhat - org[d]) / h);
            }
            for (int64_t a = lo[0]; a <= hi[0]; ++a)
                for (int64_t c = lo[1]; c <= hi[1]; ++c)
                    for (int64_t e = lo[2]; e <= hi[2]; ++e) {
                        int64_t key = cell_key(a, c, e);
                        for (int64_t k = lower_bound(tt, tl, key); k < tl && tt[k].key == key; ++k) {
                            int64_t j = tt[k].prim;
                            if (j <= i) continue;
                            const int32_t* eb = edges + 2 * j;
                            if (vobj[ea[0]] == vobj[eb[0]]) continue;
                            if (ea[0] == eb[0] || ea[0] == eb[1] || ea[1] == eb[0] || ea[1] == eb[1]) continue;
                            box3 bb; prim_box(x, eb, 2, &bb);
                            if (!boxes_overlap(&ab, dhat, &bb)) continue;
                            int own = 1;
                            for (int d = 0; d < 3 && own; ++d) {
                                double m = fmax(ab.lo[d] - dhat, bb.lo[d]);
                                int64_t cd = (int64_t)floor((m - org[d]) / h);
                                own = (d == 0 ? a : d == 1 ? c : e) == cd;
                            }
                            if (!own) continue;
                            push4(&loc[tid], ea[0], ea[1], eb[0], eb[1]);
                        }
                    }
        }
        for (int i = 0; i < nth; ++i) {
            for (int64_t k = 0; k < loc[i].n; ++k)
                push4(&all, loc[i].v[4 * k], loc[i].v[4 * k + 1], loc[i].v[4 * k + 2], loc[i].v[4 * k + 3]);
            free(loc[i].v);
        }
        free(loc); free(tt);
    }

    qsort(all.v, all.n, sizeof(int32_t) * 4, cmp_tuple);
    *out = all.v;
    return all.n;
}

void bp_free(int32_t* p) { free(p); }
