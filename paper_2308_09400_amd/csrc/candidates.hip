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
//  3. per query kind (points, edges), a cell table of the queries whose
//     box inflated by dhat covers the cell, in any order;
//  4. one wave per cell pairing its queries with its primitives (points
//     against triangles, edges against edges of larger index): a counting
//     pass that also keeps the hit masks, a scan over the queries' visits
//     of cells, and an emitting pass that replays the masks.
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

// the item of a lane, -1 past the end
__device__ __forceinline__ int64_t item_of(int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    return i < n ? i : -1;
}

// A wave's visits of cells flattened: each lane's cells lo..hi (x slowest,
// z fastest) are numbered after those of the lanes below it, and the wave
// takes them 64 at a time, so that lanes covering few cells do not idle
// while others walk up to 27.  f(cell, item) for every visit; the owner of
// visit v is the last lane whose first number is at most v (a lane covering
// no cell shares its first number with the next lane and is never last).
template <typename C, typename F>
__device__ __forceinline__ void wave_visits(const int lo[3], const int hi[3], bool valid, int32_t item, C vcell, F f) {
    __shared__ int4 vbox[kBlock / 64][64];
    __shared__ int2 vnum[kBlock / 64][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int sy = hi[1] - lo[1] + 1, sz = hi[2] - lo[2] + 1;
    const int n = valid ? (hi[0] - lo[0] + 1) * sy * sz : 0;
    int inc = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    const int total = __builtin_amdgcn_readlane(inc, 63);
    vbox[w][lane] = make_int4(lo[0], lo[1], lo[2], (sy << 8) | sz);
    vnum[w][lane] = make_int2(inc - n, item);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int base = 0; base < total; base += 64) {
        const int v = base + lane;
        if (v < total) {
            int l = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (vnum[w][l + step].x <= v) l += step;
            const int4 b = vbox[w][l];
            const int2 nm = vnum[w][l];
            const int bz = b.w & 255, byz = (b.w >> 8) * bz;
            const int j = v - nm.x;
            const int da = j / byz, rem = j - da * byz;
            const int dc = rem / bz, de = rem - dc * bz;
            f(vcell(b.x + da, b.y + dc, b.z + de), nm.y);
        }
    }
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
    const int64_t i0 = item_of(n);
    const bool valid = i0 >= 0;
    const int64_t i = valid ? i0 : 0;
    const Box b = prim_box(X, prims + NPER * i, NPER);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(b.lo, d), g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(b.hi, d), g.org[d], g.h[d], g.n[d]);
    }
    const auto vcell = [&](int a, int c, int e) { return ((int64_t)a * g.n[1] + c) * g.n[2] + e; };
    wave_visits(lo, hi, valid, (int32_t)i, vcell, [&](int64_t cell, int32_t) { atomicAdd(&count[cell], 1); });
}

template <int NPER>
__global__ void __launch_bounds__(kBlock) k_cell_fill_prims(const double* __restrict__ X,
                                                            const int32_t* __restrict__ prims, int64_t n, Grid g,
                                                            const int64_t* __restrict__ off,
                                                            int32_t* __restrict__ fill, int32_t* __restrict__ ent) {
    const int64_t i0 = item_of(n);
    const bool valid = i0 >= 0;
    const int64_t i = valid ? i0 : 0;
    const Box b = prim_box(X, prims + NPER * i, NPER);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(b.lo, d), g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(b.hi, d), g.org[d], g.h[d], g.n[d]);
    }
    const auto vcell = [&](int a, int c, int e) { return ((int64_t)a * g.n[1] + c) * g.n[2] + e; };
    wave_visits(lo, hi, valid, (int32_t)i, vcell, [&](int64_t cell, int32_t item) {
        ent[off[cell] + atomicAdd(&fill[cell], 1)] = item;
    });
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

// each cell's list in increasing primitive id, one wave per cell: an entry's
// place is the number of entries of the cell below it (the ids of a cell
// are distinct), counted against the others handed over by lane reads;
// raw -> ent
__global__ void __launch_bounds__(kBlock) k_cell_sort(int64_t ncell, const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ raw,
                                                      int32_t* __restrict__ ent) {
    const int lane = threadIdx.x & 63;
    const int64_t c =
        (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (c >= ncell) return;
    const int64_t b = off[c], n = off[c + 1] - b;
    for (int64_t c0 = 0; c0 < n; c0 += 64) {
        const bool mine_ok = c0 + lane < n;
        const int32_t mine = mine_ok ? raw[b + c0 + lane] : 0;
        int64_t rank = 0;
        for (int64_t c1 = 0; c1 < n; c1 += 64) {
            const int32_t other = c1 + lane < n ? raw[b + c1 + lane] : 0;
            const int m = (int)(n - c1 < 64 ? n - c1 : 64);
            for (int k = 0; k < m; ++k) rank += __builtin_amdgcn_readlane(other, k) < mine;
        }
        if (mine_ok) ent[b + rank] = mine;
    }
}

// The queries' side, one record per query primitive: KIND 0 = points (their
// position, a zero-size box), 1 = edges (their 64-byte record).
template <int KIND>
__device__ __forceinline__ void query_of(int64_t q, const double* __restrict__ X, const int32_t* __restrict__ vobj,
                                         const PrimRec* __restrict__ qrec, Box& qb, int32_t& q0, int32_t& q1,
                                         int32_t& qo) {
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
}

// the cells covered by a query's box inflated by dhat
__device__ __forceinline__ void query_cells(const Box& qb, const Grid& g, double dhat, int lo[3], int hi[3]) {
    for (int d = 0; d < 3; ++d) {
        lo[d] = cell_of(get(qb.lo, d) - dhat, g.org[d], g.h[d], g.n[d]);
        hi[d] = cell_of(get(qb.hi, d) + dhat, g.org[d], g.h[d], g.n[d]);
    }
}

// query table, counting: span[q] = cells the query covers, count[cell] +=
// queries covering the cell
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_qcells_count(const double* __restrict__ X, int64_t nq,
                                                         const PrimRec* __restrict__ qrec, Grid g, double dhat,
                                                         int32_t* __restrict__ span, int32_t* __restrict__ count) {
    const int64_t qi = item_of(nq);
    const bool valid = qi >= 0;
    const int64_t q = valid ? qi : 0;
    Box qb;
    int32_t q0, q1, qo;
    query_of<KIND>(q, X, nullptr, qrec, qb, q0, q1, qo);
    int lo[3], hi[3];
    query_cells(qb, g, dhat, lo, hi);
    if (valid) span[q] = (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
    const auto vcell = [&](int a, int c, int e) { return ((int64_t)a * g.n[1] + c) * g.n[2] + e; };
    wave_visits(lo, hi, valid, (int32_t)q, vcell, [&](int64_t cell, int32_t) { atomicAdd(&count[cell], 1); });
}

// query table, filling: the queries covering each cell, in no particular
// order (the output positions come from the query and the cell, not from
// this order)
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_qcells_fill(const double* __restrict__ X, int64_t nq,
                                                        const PrimRec* __restrict__ qrec, Grid g, double dhat,
                                                        const int64_t* __restrict__ off, int32_t* __restrict__ fill,
                                                        int32_t* __restrict__ ent) {
    const int64_t qi = item_of(nq);
    const bool valid = qi >= 0;
    const int64_t q = valid ? qi : 0;
    Box qb;
    int32_t q0, q1, qo;
    query_of<KIND>(q, X, nullptr, qrec, qb, q0, q1, qo);
    int lo[3], hi[3];
    query_cells(qb, g, dhat, lo, hi);
    const auto vcell = [&](int a, int c, int e) { return ((int64_t)a * g.n[1] + c) * g.n[2] + e; };
    wave_visits(lo, hi, valid, (int32_t)q, vcell, [&](int64_t cell, int32_t item) {
        ent[off[cell] + atomicAdd(&fill[cell], 1)] = item;
    });
}

// a lane's 64-bit value, read by every lane (k wave-uniform)
__device__ __forceinline__ unsigned long long read_lane_u64(unsigned long long v, int k) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), k);
    return ((unsigned long long)hi << 32) | lo;
}

// a lane's double, read by every lane (k wave-uniform)
__device__ __forceinline__ double read_lane(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Edge-edge pairs, one wave per cell: its lanes take the edge queries
// covering the cell, 64 at a time, and the cell's edge list 64 records at a
// time, one record per lane; each record is then handed to every lane from
// the lane holding it (a lane read, no memory access), so the records are
// read once per 64 queries.  The query q's visit of the cell is entry e = qeoff[q] + j, j the
// cell's rank in the query's walk (x slowest, z fastest): EMIT = false
// stores the entry's candidate count in cnt[e], EMIT = true writes its
// candidates at out + eoff[e], in list order.  Only edges of larger index
// than the query are taken.  The counting pass also stores, per record
// and chunk of queries, the 64-lane mask of the queries it pairs with
// (bal, from boff[cell]); the emitting pass replays those masks instead of
// testing again, reading only the records' vertex ids, and writes query by
// query so that a store covers consecutive slots of one query.  The
// counting pass also leaves each visit's entry e in evis (by position in
// the cell's query list), so the emitting pass needs no query boxes.
//
// The cell reporting a pair holds the lower corner of the overlap, whose
// coordinate along d is the larger of the inflated query's and the
// primitive's lower bounds; the cell index is monotonic in the coordinate,
// so that cell is, per axis, the larger of the two lower bounds' cells, and
// both are at most the current cell's (both boxes cover it): the pair is
// this cell's when, along every axis, one of the two lower cells is this
// cell's.
//
// (Seven waves per SIMD asked for: the compiler then keeps the counting
// pass at 66 registers instead of 84, without spills; the point-triangle
// pass below at 68.)
template <bool EMIT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) k_cell_pairs_ee(const double* __restrict__ X,
                                                       const int32_t* __restrict__ vobj,
                                                       const PrimRec* __restrict__ qrec,
                                                       const PrimRec* __restrict__ trec, Grid g, double dhat,
                                                       int64_t ncell, const int64_t* __restrict__ qtoff,
                                                       const int32_t* __restrict__ qent,
                                                       const int64_t* __restrict__ qeoff,
                                                       const int64_t* __restrict__ coff,
                                                       const int32_t* __restrict__ cent, int32_t* __restrict__ cnt,
                                                       const int64_t* __restrict__ eoff,
                                                       const int64_t* __restrict__ boff,
                                                       unsigned long long* __restrict__ bal,
                                                       int64_t* __restrict__ evis, int4* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t cell =
        (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (cell >= ncell) return;
    const int64_t qa = qtoff[cell], qz = qtoff[cell + 1];
    const int64_t ta = coff[cell], tz = coff[cell + 1];
    if (qa == qz || (EMIT && ta == tz)) return;
    const int cc[3] = {(int)(cell / ((int64_t)g.n[1] * g.n[2])), (int)((cell / g.n[2]) % g.n[1]),
                       (int)(cell % g.n[2])};
    for (int64_t qb0 = qa; qb0 < qz; qb0 += 64) {
        const int64_t i = qb0 + lane;
        const bool act = i < qz;
        const int64_t q = qent[act ? i : qa];
        Box qb{};
        int32_t q0 = 0, q1 = 0, qo = 0;
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        int64_t e, w = 0, wz = 0;
        if (EMIT) {
            // the counting pass left the visit's entry; only the query's ids
            // are needed
            e = act ? evis[i] : 0;
            const int4 qv = *reinterpret_cast<const int4*>(&qrec[q].v[0]);
            q0 = qv.x;
            q1 = qv.y;
            w = act ? eoff[e] : 0;
            wz = act ? eoff[e + 1] : 0;
            if (__ballot(w < wz) == 0) continue;
        } else {
            query_of<1>(q, X, vobj, qrec, qb, q0, q1, qo);
            query_cells(qb, g, dhat, lo, hi);
            e = qeoff[q] + ((int64_t)(cc[0] - lo[0]) * (hi[1] - lo[1] + 1) + (cc[1] - lo[1])) *
                               (hi[2] - lo[2] + 1) + (cc[2] - lo[2]);
            if (act) evis[i] = e;
        }
        const bool own0 = lo[0] == cc[0], own1 = lo[1] == cc[1], own2 = lo[2] == cc[2];
        const double qlx = qb.lo.x - dhat, qly = qb.lo.y - dhat, qlz = qb.lo.z - dhat;
        const double qhx = qb.hi.x + dhat, qhy = qb.hi.y + dhat, qhz = qb.hi.z + dhat;
        int64_t t0 = ta;
        // the list is in increasing edge id: skip what no lane takes
        int64_t qmin = act ? q : INT64_MAX;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int64_t v = __shfl_xor(qmin, o, 64);
            qmin = v < qmin ? v : qmin;
        }
        qmin = __builtin_amdgcn_readfirstlane((int)qmin);
        // (64 entries a step: they form a prefix of each window)
        for (;;) {
            const int64_t j = t0 + lane;
            const unsigned long long m = __ballot(j < tz && (int64_t)cent[j] <= qmin);
            t0 += __popcll(m);
            if (m != ~0ull) break;
        }
        int32_t found = 0;
        // this chunk's hit masks: slot (chunk of queries, record) of the cell
        const int64_t bslot = boff[cell] + ((qb0 - qa) >> 6) * (tz - ta);
        for (int64_t tb0 = t0; tb0 < tz; tb0 += 64) {
            // this lane's record of the chunk
            const int64_t j = tb0 + lane;
            const int32_t id = cent[j < tz ? j : tb0];
            const int nk = (int)(tz - tb0 < 64 ? tz - tb0 : 64);
            if (EMIT) {
                // replay the counting pass's masks, query by query (only
                // the queries with a hit in this chunk): the hit records'
                // lanes write the query's next candidates side by side
                const int4 rv = *reinterpret_cast<const int4*>(&trec[id].v[0]);
                const unsigned long long mine = lane < nk ? bal[bslot + (tb0 - ta) + lane] : 0ull;
                unsigned long long any = mine;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) any |= __shfl_xor(any, o, 64);
                any = read_lane_u64(any, 0);
                const unsigned long long below = (1ull << lane) - 1ull;
                while (any) {
                    const int jq = __builtin_ctzll(any);
                    any &= any - 1ull;
                    const bool bit = (mine >> jq) & 1ull;
                    const unsigned long long bm = __ballot(bit);
                    const int64_t base = (int64_t)read_lane_u64((unsigned long long)w, jq);
                    const int32_t a0 = __builtin_amdgcn_readlane(q0, jq), a1 = __builtin_amdgcn_readlane(q1, jq);
                    if (bit)
                        out[base + __popcll(bm & below)] =
                            make_int4(a0, a1, rv.x, rv.y);
                    if (lane == jq) w += __popcll(bm);
                }
                if (__ballot(w < wz) == 0) break;
                continue;
            }
            const PrimRec r = trec[id];
            int tsel = 0;
            for (int d = 0; d < 3; ++d)
                tsel |= (cell_of(r.lo[d], g.org[d], g.h[d], g.n[d]) == cc[d]) << d;
            unsigned long long mine = 0;
            for (int k = 0; k < nk; ++k) {
                const double lx = read_lane(r.lo[0], k), ly = read_lane(r.lo[1], k), lz = read_lane(r.lo[2], k);
                const double hx = read_lane(r.hi[0], k), hy = read_lane(r.hi[1], k), hz = read_lane(r.hi[2], k);
                const int32_t v0 = __builtin_amdgcn_readlane(r.v[0], k), v1 = __builtin_amdgcn_readlane(r.v[1], k);
                const int32_t ob = __builtin_amdgcn_readlane(r.obj, k), tid = __builtin_amdgcn_readlane(id, k);
                const int ts = __builtin_amdgcn_readlane(tsel, k);
                bool hit = act && ob != qo && (int64_t)tid > q && v0 != q0 && v0 != q1 && v1 != q0 && v1 != q1;
                hit = hit && !(qlx > hx || lx > qhx || qly > hy || ly > qhy || qlz > hz || lz > qhz);
                hit = hit && (own0 || (ts & 1)) && (own1 || (ts & 2)) && (own2 || (ts & 4));
                const unsigned long long m = __ballot(hit);
                if (lane == k) mine = m;
                found += hit;
            }
            if (lane < nk) bal[bslot + (tb0 - ta) + lane] = mine;
        }
        if (!EMIT && act) cnt[e] = found;
    }
}

// Point-triangle pairs of a cell the other way round: the cell's triangles
// in the lanes, 64 at a time, and its points (a cell holds tens of them,
// fewer than triangles) handed to every lane by lane reads, so a wave step
// tests one point against 64 triangles.  The points' setup (entry e,
// reporting-cell flags) is done with the points in the lanes, 64 at a
// time.  A pair is taken when the point and the triangle belong to
// different objects, the point is none of the triangle's vertices, the
// point's box inflated by dhat overlaps the triangle's box and the cell
// reports it (as for the edges); the counting pass stores each point's
// 64-bit mask over a chunk of triangles at bal + boff[cell] + (triangle
// chunk) * (points of the cell) + (point's place in the cell's list), and
// the emitting pass replays them, writing at out + eoff[e] in list order.
template <bool EMIT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_cell_pairs_pt(const double* __restrict__ X, const int32_t* __restrict__ vobj, const PrimRec* __restrict__ trec,
                Grid g, double dhat, int64_t ncell, const int64_t* __restrict__ qtoff,
                const int32_t* __restrict__ qent, const int64_t* __restrict__ qeoff,
                const int64_t* __restrict__ coff, const int32_t* __restrict__ cent, int32_t* __restrict__ cnt,
                const int64_t* __restrict__ eoff, const int64_t* __restrict__ boff,
                unsigned long long* __restrict__ bal, int64_t* __restrict__ evis, int4* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t cell =
        (int64_t)blockIdx.x * (kBlock / 64) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (cell >= ncell) return;
    const int64_t qa = qtoff[cell], qz = qtoff[cell + 1];
    const int64_t ta = coff[cell], tz = coff[cell + 1];
    if (qa == qz || (EMIT && ta == tz)) return;
    const int cc[3] = {(int)(cell / ((int64_t)g.n[1] * g.n[2])), (int)((cell / g.n[2]) % g.n[1]),
                       (int)(cell % g.n[2])};
    const int64_t nq = qz - qa;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int64_t qb0 = qa; qb0 < qz; qb0 += 64) {
        const int64_t i = qb0 + lane;
        const bool act = i < qz;
        const int32_t q = qent[act ? i : qa];
        const int nqk = (int)(qz - qb0 < 64 ? qz - qb0 : 64);
        d3 pq = mk(0.0, 0.0, 0.0);
        int32_t qo = 0, own = 0;
        int64_t e, w = 0, wz = 0;
        if (EMIT) {
            e = act ? evis[i] : 0;
            w = act ? eoff[e] : 0;
            wz = act ? eoff[e + 1] : 0;
            if (__ballot(w < wz) == 0) continue;
        } else {
            Box qb;
            int32_t q0, q1;
            query_of<0>(q, X, vobj, nullptr, qb, q0, q1, qo);
            pq = qb.lo;
            int lo[3], hi[3];
            query_cells(qb, g, dhat, lo, hi);
            e = qeoff[q] + ((int64_t)(cc[0] - lo[0]) * (hi[1] - lo[1] + 1) + (cc[1] - lo[1])) *
                               (hi[2] - lo[2] + 1) + (cc[2] - lo[2]);
            if (act) evis[i] = e;
            own = (lo[0] == cc[0]) | ((lo[1] == cc[1]) << 1) | ((lo[2] == cc[2]) << 2);
        }
        int32_t found = 0;
        for (int64_t tb0 = ta; tb0 < tz; tb0 += 64) {
            const int64_t j = tb0 + lane;
            const bool tact = j < tz;
            const int32_t id = cent[tact ? j : tb0];
            const int64_t slot = boff[cell] + ((tb0 - ta) >> 6) * nq + (qb0 - qa);
            if (EMIT) {
                const int4 rv = *reinterpret_cast<const int4*>(&trec[id].v[0]);
                const unsigned long long mq = lane < nqk ? bal[slot + lane] : 0ull;
                for (int k = 0; k < nqk; ++k) {
                    const unsigned long long m = read_lane_u64(mq, k);
                    if (m == 0) continue;
                    const int64_t base = (int64_t)read_lane_u64((unsigned long long)w, k);
                    const int32_t a0 = __builtin_amdgcn_readlane(q, k);
                    if ((m >> lane) & 1ull) out[base + __popcll(m & below)] = make_int4(-(a0 + 1), rv.x, rv.y, rv.z);
                    if (lane == k) w += __popcll(m);
                }
                if (__ballot(w < wz) == 0) break;
                continue;
            }
            const PrimRec r = trec[id];
            int tsel = 0;
            for (int d = 0; d < 3; ++d)
                tsel |= (cell_of(r.lo[d], g.org[d], g.h[d], g.n[d]) == cc[d]) << d;
            unsigned long long mine = 0;
            for (int k = 0; k < nqk; ++k) {
                const double px = read_lane(pq.x, k), py = read_lane(pq.y, k), pz = read_lane(pq.z, k);
                const int32_t a0 = __builtin_amdgcn_readlane(q, k), ob = __builtin_amdgcn_readlane(qo, k);
                const int ow = __builtin_amdgcn_readlane(own, k) | tsel;
                bool hit = tact && r.obj != ob && r.v[0] != a0 && r.v[1] != a0 && r.v[2] != a0;
                hit = hit && !(px - dhat > r.hi[0] || r.lo[0] > px + dhat || py - dhat > r.hi[1] ||
                               r.lo[1] > py + dhat || pz - dhat > r.hi[2] || r.lo[2] > pz + dhat);
                hit = hit && ow == 7;
                const unsigned long long m = __ballot(hit);
                if (lane == k) {
                    mine = m;
                    found += __popcll(m);
                }
            }
            if (lane < nqk) bal[slot + lane] = mine;
        }
        if (!EMIT && act) cnt[e] = found;
    }
}

// per cell, the hit-mask slots of its pairs pass: one per chunk of 64
// queries and primitive of the cell, or (by_points, the point-triangle
// pass) one per chunk of 64 triangles and point of the cell
__global__ void __launch_bounds__(kBlock) k_cell_slots(int64_t ncell, int by_points, const int64_t* __restrict__ qtoff,
                                                       const int64_t* __restrict__ coff, int64_t* __restrict__ n) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    const int64_t nq = qtoff[c + 1] - qtoff[c], nt = coff[c + 1] - coff[c];
    n[c] = by_points ? ((nt + 63) >> 6) * nq : ((nq + 63) >> 6) * nt;
}

unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

Grid to_grid(const CandGrid& cg) {
    Grid g;
    for (int d = 0; d < 3; ++d) { g.org[d] = cg.org[d]; g.n[d] = cg.n[d]; g.h[d] = cg.h[d]; }
    return g;
}

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
    const Grid g = to_grid(cg);
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
                            int32_t* fill, const int64_t* off, int32_t* raw, int32_t* ent, hipStream_t s) {
    const Grid g = to_grid(cg);
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (n > 0) {
        if (nper == 3) k_cell_fill_prims<3><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, off, fill, raw);
        else k_cell_fill_prims<2><<<grid1(n), kBlock, 0, s>>>(x, prims, n, g, off, fill, raw);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_cell_sort<<<(unsigned)((ncell + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, s>>>(ncell, off, raw, ent);
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

hipError_t launch_qcells_count(int kind, const double* x, int64_t nq, const void* qrec, const CandGrid& cg,
                               double dhat, int32_t* span, int32_t* count, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const Grid g = to_grid(cg);
    const PrimRec* qr = static_cast<const PrimRec*>(qrec);
    if (kind == 0) k_qcells_count<0><<<grid1(nq), kBlock, 0, s>>>(x, nq, qr, g, dhat, span, count);
    else k_qcells_count<1><<<grid1(nq), kBlock, 0, s>>>(x, nq, qr, g, dhat, span, count);
    return hipGetLastError();
}

hipError_t launch_qcells_fill(int kind, const double* x, int64_t nq, const void* qrec, const CandGrid& cg,
                              double dhat, const int64_t* off, int32_t* fill, int32_t* ent, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const Grid g = to_grid(cg);
    const PrimRec* qr = static_cast<const PrimRec*>(qrec);
    if (kind == 0) k_qcells_fill<0><<<grid1(nq), kBlock, 0, s>>>(x, nq, qr, g, dhat, off, fill, ent);
    else k_qcells_fill<1><<<grid1(nq), kBlock, 0, s>>>(x, nq, qr, g, dhat, off, fill, ent);
    return hipGetLastError();
}

hipError_t launch_cell_slots(int kind, const CandGrid& cg, const int64_t* qtoff, const int64_t* coff, int64_t* n,
                             hipStream_t s) {
    const int64_t ncell = (int64_t)cg.n[0] * cg.n[1] * cg.n[2];
    k_cell_slots<<<grid1(ncell), kBlock, 0, s>>>(ncell, kind == 0, qtoff, coff, n);
    return hipGetLastError();
}

hipError_t launch_cell_pairs(int kind, bool emit, const double* x, const int32_t* vobj, const void* qrec,
                             const void* trec, const CandGrid& cg, double dhat, const int64_t* qtoff,
                             const int32_t* qent, const int64_t* qeoff, const int64_t* coff, const int32_t* cent,
                             int32_t* cnt, const int64_t* eoff, const int64_t* boff, uint64_t* bal,
                             int64_t* evis, int32_t* out, hipStream_t s) {
    const Grid g = to_grid(cg);
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const unsigned nb = (unsigned)((ncell + kBlock / 64 - 1) / (kBlock / 64));
    int4* o = reinterpret_cast<int4*>(out);
    const PrimRec* qr = static_cast<const PrimRec*>(qrec);
    const PrimRec* tr = static_cast<const PrimRec*>(trec);
    unsigned long long* b = reinterpret_cast<unsigned long long*>(bal);
    if (kind == 0) {
        if (emit)
            k_cell_pairs_pt<true><<<nb, kBlock, 0, s>>>(x, vobj, tr, g, dhat, ncell, qtoff, qent, qeoff, coff, cent,
                                                        cnt, eoff, boff, b, evis, o);
        else
            k_cell_pairs_pt<false><<<nb, kBlock, 0, s>>>(x, vobj, tr, g, dhat, ncell, qtoff, qent, qeoff, coff, cent,
                                                         cnt, eoff, boff, b, evis, o);
    } else {
        if (emit)
            k_cell_pairs_ee<true><<<nb, kBlock, 0, s>>>(x, vobj, qr, tr, g, dhat, ncell, qtoff, qent, qeoff, coff, cent,
                                                        cnt, eoff, boff, b, evis, o);
        else
            k_cell_pairs_ee<false><<<nb, kBlock, 0, s>>>(x, vobj, qr, tr, g, dhat, ncell, qtoff, qent, qeoff, coff,
                                                         cent, cnt, eoff, boff, b, evis, o);
    }
    return hipGetLastError();
}

}  // namespace gipc
