// Contact candidates on the GPU: every point-triangle and edge-edge pair of
// different objects, sharing no vertex, whose axis-aligned boxes come within
// dhat (one box inflated by dhat, closed intervals) -- the pairs the sum of
// Eq. 3 ranges over, before the distance decides which are active.  A
// uniform grid stands in for the paper's LBVH (Sec. 7.2): along each axis
// the cell size is the largest primitive extent along that axis plus dhat,
// so every box spans at most two cells per axis, and thin stacks (sheets a
// fraction of dhat apart) are split along their normal; a pair is reported
// by the one cell holding the lower corner of its boxes' overlap, so each is
// found exactly once.
//
//  1. bounds: per-block minima / maxima of the positions and the largest
//     primitive extent (the host finishes the reduction and sizes the grid);
//  2. per primitive kind, a cell table: counts (integer atomics), scan,
//     fill, then each cell's list sorted by primitive id, so the table does
//     not depend on the order of the atomics;
//  3. one lane per query primitive (points against triangles, edges against
//     edges of larger index), a counting pass, a scan, an emitting pass that
//     walks the same cells in the same order.
// The output is deterministic: point-triangle candidates grouped by point in
// increasing order, then edge-edge candidates grouped by first edge, each
// group in cell order and primitive order within a cell.
#include "internal.hpp"

namespace gipc {
namespace {

struct Grid {
    double org[3];
    double h[3];
    int32_t n[3];
};

struct Box {
    d3 lo, hi;
};

// one 64-byte record per primitive for the queries: its box, its vertex
// ids (v[2] = v[1] for edges) and its object
struct __align__(64) PrimRec {
    double lo[3], hi[3];
    int32_t v[3];
    int32_t obj;
};

__device__ __forceinline__ Box prim_box(const double* __restrict__ X, const int32_t* v, int nper) {
    Box b{ld3(X, v[0]), ld3(X, v[0])};
    for (int k = 1; k < nper; ++k) {
        const d3 p = ld3(X, v[k]);
        b.lo = mk(fmin(b.lo.x, p.x), fmin(b.lo.y, p.y), fmin(b.lo.z, p.z));
        b.hi = mk(fmax(b.hi.x, p.x), fmax(b.hi.y, p.y), fmax(b.hi.z, p.z));
    }
    return b;
}

__device__ __forceinline__ int cell_of(double c, double org, double h, int32_t n) {
    const int i = (int)floor((c - org) / h);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ double get(const d3& v, int d) { return d == 0 ? v.x : (d == 1 ? v.y : v.z); }

// box a inflated by dhat overlaps box b
__device__ __forceinline__ bool overlap(const Box& a, double dhat, const Box& b) {
    return !(a.lo.x - dhat > b.hi.x || b.lo.x > a.hi.x + dhat || a.lo.y - dhat > b.hi.y || b.lo.y > a.hi.y + dhat ||
             a.lo.z - dhat > b.hi.z || b.lo.z > a.hi.z + dhat);
}

// per block: min x,y,z, max x,y,z of the positions, largest primitive
// extent along x, y, z
__global__ void __launch_bounds__(kBlock) k_cand_bounds(const double* __restrict__ X, int32_t V,
                                                        const int32_t* __restrict__ tris, int64_t F,
                                                        const int32_t* __restrict__ edges, int64_t E,
                                                        double* __restrict__ part) {
    __shared__ double lds[kBlock / 64][9];
    double r[9] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < V; i += stride) {
        const d3 p = ld3(X, (int)i);
        r[0] = fmin(r[0], p.x); r[1] = fmin(r[1], p.y); r[2] = fmin(r[2], p.z);
        r[3] = fmax(r[3], p.x); r[4] = fmax(r[4], p.y); r[5] = fmax(r[5], p.z);
    }
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < F + E; i += stride) {
        const Box b = i < F ? prim_box(X, tris + 3 * i, 3) : prim_box(X, edges + 2 * (i - F), 2);
        r[6] = fmax(r[6], b.hi.x - b.lo.x);
        r[7] = fmax(r[7], b.hi.y - b.lo.y);
        r[8] = fmax(r[8], b.hi.z - b.lo.z);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) r[q] = fmin(r[q], __shfl_xor(r[q], o, 64));
#pragma unroll
        for (int q = 3; q < 9; ++q) r[q] = fmax(r[q], __shfl_xor(r[q], o, 64));
    }
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 9; ++q) lds[threadIdx.x >> 6][q] = r[q];
    __syncthreads();
    if (threadIdx.x < 9) {
        const int q = threadIdx.x;
        double v = lds[0][q];
        for (int w = 1; w < kBlock / 64; ++w) v = q < 3 ? fmin(v, lds[w][q]) : fmax(v, lds[w][q]);
        part[9 * blockIdx.x + q] = v;
    }
}

// invalid vertex ids of the topology -> counters[0], the first one -> counters[1]
__global__ void __launch_bounds__(kBlock) k_cand_check(int32_t V, const int32_t* __restrict__ vobj,
                                                       const int32_t* __restrict__ tris, int64_t F,
                                                       const int32_t* __restrict__ edges, int64_t E,
                                                       unsigned long long* __restrict__ counters) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= F + E) return;
    const int32_t* v = i < F ? tris + 3 * i : edges + 2 * (i - F);
    const int n = i < F ? 3 : 2;
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        ok = ok && v[k] >= 0 && v[k] < V;
        for (int l = 0; l < k; ++l) ok = ok && v[l] != v[k];
    }
    if (!ok) {
        atomicAdd(&counters[0], 1ull);
        atomicMin(&counters[1], (unsigned long long)i);
    }
}

template <int NPER>
__global__ void __launch_bounds__(kBlock) k_cell_count_prims(const double* __restrict__ X,
                                                             const int32_t* __restrict__ prims, int64_t n, Grid g,
                                                             int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Box b = prim_box(X, prims + NPER * i, NPER);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(b.lo, d), g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(b.hi, d), g.org[d], g.h[d], g.n[d]);
    }
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int c = lo[1]; c <= hi[1]; ++c)
            for (int e = lo[2]; e <= hi[2]; ++e) atomicAdd(&count[((int64_t)a * g.n[1] + c) * g.n[2] + e], 1);
}

template <int NPER>
__global__ void __launch_bounds__(kBlock) k_cell_fill_prims(const double* __restrict__ X,
                                                            const int32_t* __restrict__ prims, int64_t n, Grid g,
                                                            const int64_t* __restrict__ off,
                                                            int32_t* __restrict__ fill, int32_t* __restrict__ ent) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Box b = prim_box(X, prims + NPER * i, NPER);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(b.lo, d), g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(b.hi, d), g.org[d], g.h[d], g.n[d]);
    }
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int c = lo[1]; c <= hi[1]; ++c)
            for (int e = lo[2]; e <= hi[2]; ++e) {
                const int64_t cell = ((int64_t)a * g.n[1] + c) * g.n[2] + e;
                ent[off[cell] + atomicAdd(&fill[cell], 1)] = (int32_t)i;
            }
}

template <int NPER>
__global__ void __launch_bounds__(kBlock) k_prim_records(const double* __restrict__ X,
                                                         const int32_t* __restrict__ prims, int64_t n,
                                                         const int32_t* __restrict__ vobj,
                                                         PrimRec* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t* v = prims + NPER * i;
    const Box b = prim_box(X, v, NPER);
    PrimRec r;
    r.lo[0] = b.lo.x; r.lo[1] = b.lo.y; r.lo[2] = b.lo.z;
    r.hi[0] = b.hi.x; r.hi[1] = b.hi.y; r.hi[2] = b.hi.z;
    r.v[0] = v[0]; r.v[1] = v[1]; r.v[2] = NPER == 3 ? v[2] : v[1];
    r.obj = vobj[v[0]];
    rec[i] = r;
}

// each cell's list in increasing primitive id (insertion sort: lists are short)
__global__ void __launch_bounds__(kBlock) k_cell_sort(int64_t ncell, const int64_t* __restrict__ off,
                                                      int32_t* __restrict__ ent) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    const int64_t b = off[c], e = off[c + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t v = ent[i];
        int64_t j = i - 1;
        while (j >= b && ent[j] > v) {
            ent[j + 1] = ent[j];
            --j;
        }
        ent[j + 1] = v;
    }
}

// queries: KIND 0 = points against triangles, 1 = edges against edges of
// larger index; EMIT = 0 counts per query, 1 writes at out + off[q].
// Candidate primitives are read from their 64-byte records.
template <int KIND, bool EMIT>
__global__ void __launch_bounds__(kBlock) k_cand_query(const double* __restrict__ X, int64_t nq,
                                                       const int32_t* __restrict__ vobj,
                                                       const PrimRec* __restrict__ qrec,
                                                       const PrimRec* __restrict__ trec, Grid g, double dhat,
                                                       const int64_t* __restrict__ coff,
                                                       const int32_t* __restrict__ cent, int32_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ qoff, int4* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= nq) return;
    Box qb;
    int32_t q0, q1, qo;
    if (KIND == 0) {
        qb.lo = qb.hi = ld3(X, (int)q);
        q0 = q1 = (int32_t)q;
        qo = vobj[q];
    } else {
        const PrimRec r = qrec[q];
        qb.lo = mk(r.lo[0], r.lo[1], r.lo[2]);
        qb.hi = mk(r.hi[0], r.hi[1], r.hi[2]);
        q0 = r.v[0]; q1 = r.v[1]; qo = r.obj;
    }
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(qb.lo, d) - dhat, g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(qb.hi, d) + dhat, g.org[d], g.h[d], g.n[d]);
    }
    int64_t w = EMIT ? qoff[q] : 0;
    int32_t found = 0;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int c = lo[1]; c <= hi[1]; ++c)
            for (int e = lo[2]; e <= hi[2]; ++e) {
                const int64_t cell = ((int64_t)a * g.n[1] + c) * g.n[2] + e;
                const int cc[3] = {a, c, e};
                int64_t t = coff[cell];
                const int64_t t1 = coff[cell + 1];
                if (KIND == 1) {
                    // entries are sorted by edge id: skip those not above q
                    while (t < t1 && (int64_t)cent[t] <= q) ++t;
                }
                for (; t < t1; ++t) {
                    const PrimRec r = trec[cent[t]];
                    if (r.obj == qo) continue;
                    if (KIND == 0) {
                        if (r.v[0] == q0 || r.v[1] == q0 || r.v[2] == q0) continue;
                    } else {
                        if (r.v[0] == q0 || r.v[0] == q1 || r.v[1] == q0 || r.v[1] == q1) continue;
                    }
                    const Box tb{mk(r.lo[0], r.lo[1], r.lo[2]), mk(r.hi[0], r.hi[1], r.hi[2])};
                    if (!overlap(qb, dhat, tb)) continue;
                    // the cell of the overlap's lower corner reports the pair
                    bool own = true;
                    for (int d = 0; d < 3 && own; ++d) {
                        const double m = fmax(get(qb.lo, d) - dhat, get(tb.lo, d));
                        own = cell_of(m, g.org[d], g.h[d], g.n[d]) == cc[d];
                    }
                    if (!own) continue;
                    if (EMIT) {
                        out[w++] = KIND == 0 ? make_int4(-(q0 + 1), r.v[0], r.v[1], r.v[2])
                                             : make_int4(q0, q1, r.v[0], r.v[1]);
                    } else {
                        ++found;
                    }
                }
            }
    if (!EMIT) cnt[q] = found;
}

unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int32_t cand_bound_blocks(int64_t V, int64_t FE) {
    const int64_t n = V > FE ? V : FE;
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int32_t)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_cand_bounds(const double* x, int32_t V, const int32_t* tris, int64_t F, const int32_t* edges,
                              int64_t E, double* part, int32_t nb, hipStream_t s) {
    k_cand_bounds<<<(unsigned)nb, kBlock, 0, s>>>(x, V, tris, F, edges, E, part);
    return hipGetLastError();
}

hipError_t launch_cand_check(int32_t V, const int32_t* vobj, const int32_t* tris, int64_t F, const int32_t* edges,
                             int64_t E, int64_t* counters, hipStream_t s) {
    if (F + E == 0) return hipSuccess;
    k_cand_check<<<grid1(F + E), kBlock, 0, s>>>(V, vobj, tris, F, edges, E,
                                                 reinterpret_cast<unsigned long long*>(counters));
    return hipGetLastError();
}

hipError_t launch_cell_count(gipc_ctx* ctx, const double* x, const int32_t* prims, int nper, int64_t n,
                             const CandGrid& cg, int32_t* count, int32_t* fill, int64_t* off, hipStream_t s) {
    Grid g;
    for (int d = 0; d < 3; ++d) { g.org[d] = cg.org[d]; g.n[d] = cg.n[d]; g.h[d] = cg.h[d]; }
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    hipError_t e;
    if ((e = hipMemsetAsync(count, 0, sizeof(int32_t) * ncell, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(fill, 0, sizeof(int32_t) * ncell, s)) != hipSuccess) return e;
    if (n > 0) {
        if (nper == 3) k_cell_count_prims<3><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, count);
        else k_cell_count_prims<2><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, count);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return exclusive_scan<int32_t, int64_t>(count, ncell, off, ctx, s);
}

hipError_t launch_cell_fill(const double* x, const int32_t* prims, int nper, int64_t n, const CandGrid& cg,
                            int32_t* fill, const int64_t* off, int32_t* ent, hipStream_t s) {
    Grid g;
    for (int d = 0; d < 3; ++d) { g.org[d] = cg.org[d]; g.n[d] = cg.n[d]; g.h[d] = cg.h[d]; }
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (n > 0) {
        if (nper == 3) k_cell_fill_prims<3><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, off, fill, ent);
        else k_cell_fill_prims<2><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, off, fill, ent);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_cell_sort<<<grid1(ncell), kBlock, 0, s>>>(ncell, off, const_cast<int32_t*>(ent));
    return hipGetLastError();
}

hipError_t launch_prim_records(const double* x, const int32_t* prims, int nper, int64_t n, const int32_t* vobj,
                               void* rec, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (nper == 3)
        k_prim_records<3><<<grid1(n), kBlock, 0, s>>>(x, prims, n, vobj, static_cast<PrimRec*>(rec));
    else
        k_prim_records<2><<<grid1(n), kBlock, 0, s>>>(x, prims, n, vobj, static_cast<PrimRec*>(rec));
    return hipGetLastError();
}

hipError_t launch_cand_query(int kind, bool emit, const double* x, int64_t nq, const int32_t* vobj,
                             const void* qrec, const void* trec, const CandGrid& cg, double dhat,
                             const int64_t* coff, const int32_t* cent, int32_t* cnt, const int64_t* qoff,
                             int32_t* out, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    Grid g;
    for (int d = 0; d < 3; ++d) { g.org[d] = cg.org[d]; g.n[d] = cg.n[d]; g.h[d] = cg.h[d]; }
    int4* o = reinterpret_cast<int4*>(out);
    const PrimRec* qr = static_cast<const PrimRec*>(qrec);
    const PrimRec* tr = static_cast<const PrimRec*>(trec);
    if (kind == 0) {
        if (emit) k_cand_query<0, true><<<grid1(nq), kBlock, 0, s>>>(x, nq, vobj, qr, tr, g, dhat, coff, cent, cnt, qoff, o);
        else k_cand_query<0, false><<<grid1(nq), kBlock, 0, s>>>(x, nq, vobj, qr, tr, g, dhat, coff, cent, cnt, qoff, o);
    } else {
        if (emit) k_cand_query<1, true><<<grid1(nq), kBlock, 0, s>>>(x, nq, vobj, qr, tr, g, dhat, coff, cent, cnt, qoff, o);
        else k_cand_query<1, false><<<grid1(nq), kBlock, 0, s>>>(x, nq, vobj, qr, tr, g, dhat, coff, cent, cnt, qoff, o);
    }
    return hipGetLastError();
}

}  // namespace gipc
