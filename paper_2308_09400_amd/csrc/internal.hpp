// Host-side internals shared by the translation units of libgipc: the
// context, device buffers and the kernel launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>

#include "../../include/gipc.h"
#include "device_math.hpp"

namespace gipc {

constexpr int kBlock = 256;          // threads per workgroup (4 waves of 64)
constexpr int kScanItems = 8;        // elements per thread in the scans
constexpr int kMaxRowPairs = 2048;   // pairs touching one vertex (LDS sort capacity, 64 KiB)
constexpr int kEnergyPiece = 8192;   // vertices per energy piece

// Grow-only device buffer, from hipMalloc or from the caller's allocator
// (al non-null; device = the context's device).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    const gipc_allocator* al = nullptr;
    int device = 0;
};

hipError_t ensure(DevBuf& b, size_t bytes);
void release(DevBuf& b);

template <typename T>
inline T* as(DevBuf& b) { return static_cast<T*>(b.p); }

// Workgroups go to the chip's 8 XCDs in turn (workgroup b runs on XCD
// b mod 8), and every XCD has an L2 of its own.  xcd_block() renumbers the
// launch so that each XCD takes one contiguous run of logical workgroups:
// the neighbouring rows of a gather kernel then read the records they share
// through the same L2.  It is a permutation of 0 .. gridDim.x-1.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t b = blockIdx.x, n = gridDim.x;
    const int64_t q = n / kXcds, r = n % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Ranges of staged pairs per sub-type: pairs of type t occupy [off[t], off[t+1]).
struct TypeRanges {
    int64_t off[9];
};

__device__ __forceinline__ int type_of(int64_t k, const TypeRanges& tr) {
    int t = 1;
    while (t < 7 && k >= tr.off[t + 1]) ++t;
    return t;
}

__device__ __forceinline__ int vslot(const int4& v, int j) {
    return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// One tuple in the paper's sign encoding (Sec. 7.2, "Data structures"),
// negative ids as -(i+1), decoded with ~i:
//   [a0, a1, b0, b1]            edge-edge (a1 negative: close to parallel)
//   [-p, t0, t1, t2]            point-triangle
//   [-p, e0, e1, -1]            point-edge
//   [-p, q, -1, -1]             point-point
//   [-p, -o, e0, -e1]           point-edge cut from a close-to-parallel
//                               edge-edge pair (p's edge is (p, o))
//   [-p, -o, -q, -r]            point-point cut from one (q's edge is (q, r))
// Returns the kind (0 EE, 1 PT, 2 PE, 3 PP, 4 PE cut from EE, 5 PP cut
// from EE) with the vertex ids in v (nv of them), or -1 for a malformed
// tuple: a pattern not above, an id outside [0, V) or a repeated id.
__device__ __forceinline__ int decode_tuple(const int4 t, int32_t V, int v[4], int& nv) {
    int kind = -1;
    v[0] = v[1] = v[2] = v[3] = -1;
    nv = 0;
    if (t.x >= 0) {
        if (t.z >= 0 && t.w >= 0) {
            kind = 0; nv = 4;
            v[0] = t.x; v[1] = t.y >= 0 ? t.y : ~t.y; v[2] = t.z; v[3] = t.w;
        }
    } else if (t.y >= 0) {
        v[0] = ~t.x; v[1] = t.y;
        if (t.z >= 0 && t.w >= 0) { kind = 1; nv = 4; v[2] = t.z; v[3] = t.w; }
        else if (t.z >= 0 && t.w == -1) { kind = 2; nv = 3; v[2] = t.z; }
        else if (t.z == -1 && t.w == -1) { kind = 3; nv = 2; }
    } else if (t.w < 0) {
        v[0] = ~t.x; v[1] = ~t.y; v[3] = ~t.w; nv = 4;
        if (t.z >= 0) { kind = 4; v[2] = t.z; }
        else { kind = 5; v[2] = ~t.z; }
    }
    bool ok = kind >= 0;
    for (int k = 0; k < nv && ok; ++k) {
        ok = v[k] >= 0 && v[k] < V;
        for (int l = 0; l < k && ok; ++l) ok = v[l] != v[k];
    }
    return ok ? kind : -1;
}

// wave64 sum by a fixed butterfly, then the block's waves in order: the
// result does not depend on scheduling.  NT = threads of the workgroup.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double* lds /*[NT/64]*/) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += lds[w];
    __syncthreads();
    return s;  // valid in thread 0
}

__device__ __forceinline__ double block_sum(double v, double* lds /*[kBlock/64]*/) {
    return block_sum_n<kBlock>(v, lds);
}

struct PcgScalars {  // device-resident scalars of the PCG loop
    double rz, pq, rr, bb, alpha, beta, rtol2, rz0;
    int iters, done, breakdown, maxit;
    int delta;  // stopping test: 0 r.r <= rtol2 b.b, 1 r.z <= rtol2 r0.z0
    int conv;   // the stopping test held
};

}  // namespace gipc

struct gipc_ctx {
    int device = 0;
    std::string err;
    gipc_allocator alloc{};  // the caller's allocator (alloc.alloc null: hipMalloc)

    // staging (per candidate)
    gipc::DevBuf cand_ft, cand_vid, bcount, boff, counters;
    // staged pairs, sorted by sub-type; mult = multiplicity of merged
    // duplicates (valid when merged)
    gipc::DevBuf st_vid, st_src, mult;
    bool merged = false;
    // merge scratch
    gipc::DevBuf mkeys, mrep_of, mcount, mbcount, mpos, st_vid2, st_src2;
    gipc::TypeRanges ranges{};
    int64_t Ps = 0;
    int32_t V = 0;
    // symbolic
    gipc::DevBuf deg, kcount, fill, inc_ptr, kptr, contrib, kcol, kbeg, ncols, row_ptr, col_idx, cptr, slot_row,
        diag_slot, maxbuf, bigrows, tslot, incr;
    // per 64 blocks of the pattern: head bits of row starts, row of the first block
    gipc::DevBuf whead, wrow;
    // visiting order of the block rows in the assembly (spatial cells)
    gipc::DevBuf order, obox, ocell, ohist, ooff, ofill;
    int64_t nnzb = 0, K = 0;
    int32_t max_deg = 0;
    // scenes of the build: scene id per vertex (batches only), energy pieces
    // (vertex ranges of at most kEnergyPiece inside one scene) and the
    // scenes' piece offsets
    gipc::DevBuf vscene, pieces, poff;
    int32_t S = 1, npieces = 0;
    bool batched = false;
    // factors of the last eval; per-vertex energy shares and piece sums
    gipc::DevBuf rec_main, rec_extra, rec_a1, ev, epart;
    // matrix-free operator: the c_i w~_k vectors of every incidence, row by
    // row (built at the first use after an eval), and (alpha, beta) per pair
    gipc::DevBuf mfg, mfab;
    // lagged friction: per-pair lag and eval records, energy shares and
    // pieces; the build it was lagged for and eps_v dt
    gipc::DevBuf flag, ffr, fev, fpart;
    // contact candidates: bounds partials, counters, cell tables (points
    // against triangles, edges against edges), per-query counts and offsets
    gipc::DevBuf cpart, ccnt, ccount, cfill, coff_t, cent_t, coff_e, cent_e, qcnt, qoff_p, qoff_e, crec_t, crec_e;
    gipc::DevBuf qtoff_p, qtoff_e, qent_p, qent_e, ecnt_p, ecnt_e, eoff_p, eoff_e, craw, bslot, boff_p, boff_e, bal_p, bal_e, evis_p, evis_e;
    uint64_t fric_gen = 0;
    double fric_sv = 0.0;
    uint64_t eval_gen = 0;   // bumped by every eval
    uint64_t mfg_gen = 0;    // eval_gen the vectors in mfg belong to
    int64_t ninc = 0;  // incidences (k, i) of the build: sum of the stencil sizes
    // launch shapes (gipc_tune)
    gipc_tune tune{4, 16, 4, 0};
    // PCG workspace
    gipc::DevBuf r, z, p, q, p32, minv, part, scal;
    // scan scratch; counters of gipc_pairs_check
    gipc::DevBuf scan_tmp, scan_tmp2, chk;
    gipc::DevBuf accd_cnt;

    gipc_info info{};
    bool built = false;
    bool evaluated = false;
    uint64_t build_gen = 0;  // bumped by every gipc_pairs_build (graphs check it)
};

namespace gipc {

// ---- scan.hip
// out[i] = sum_{j<i} in[j] for i <= n (out has n+1 entries); *total_dev
// (device int64, nullable) receives the sum without narrowing.
// TIn: int32/int64, TOut: int32/int64.
template <typename TIn, typename TOut>
hipError_t exclusive_scan(const TIn* in, int64_t n, TOut* out, gipc_ctx* ctx, hipStream_t s,
                          int64_t* total_dev = nullptr);
// zeroes a[0..n), and b and c when not null, in one launch
hipError_t zero_i32(int32_t* a, int32_t* b, int32_t* c, int64_t n, hipStream_t s);
hipError_t reduce_max_i32(const int32_t* in, int64_t n, int32_t* out_dev, hipStream_t s);

// ---- stage.hip
hipError_t launch_vertex_scene(const int32_t* vert_off, int32_t S, int32_t V, int32_t* vscene, hipStream_t s);
hipError_t launch_stage_classify(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* xr,
                                 const DevParams& pm, uint8_t* ft, int4* vid, int32_t* bcount, int64_t* counters,
                                 hipStream_t s);
hipError_t launch_stage_scatter(const uint8_t* ft, const int4* vid, int64_t P, const int64_t* boff, int4* st_vid,
                                int32_t* st_src, hipStream_t s);
// the build's classification (ft_b, vid_b) against the one at x; counters
// (device int64 [6], zeroed, [5] = INT64_MAX): entered, left, changed,
// degenerate, malformed, first changed tuple
hipError_t launch_stage_check(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* xr,
                              const DevParams& pm, const uint8_t* ft_b, const int4* vid_b, int64_t* counters,
                              hipStream_t s);
hipError_t launch_stage_offsets(const int64_t* boff, int64_t nb, int64_t* out, hipStream_t s);

// ---- merge.hip
// merge duplicate PE / PP constraints of ctx->ranges (vertex ids < V) into
// one staged pair with a multiplicity (ctx->mult); swaps the staged arrays
// and writes the merged type offsets (9 int64) to new_off_dev
hipError_t merge_duplicates(gipc_ctx* ctx, int32_t V, hipStream_t s, int64_t* new_off_dev);

// ---- order.hip
// ctx->order = the vertices sorted into Morton cells of their bounding cube
// (scene-major with each scene's own cube when S > 1: vert_off device int32
// [S+1] and ctx->vscene must be set)
hipError_t build_row_order(gipc_ctx* ctx, const double* x, int32_t V, const int32_t* vert_off, int32_t S,
                           hipStream_t s);

// ---- symbolic.hip
hipError_t launch_sym_count(const int4* st_vid, TypeRanges tr, int32_t* deg, int32_t* kcount, hipStream_t s);
// incr: one record per incidence: k << 2 | i, then the vertices of the pair's other
// slots in slot order (-1 past the stencil)
hipError_t launch_sym_scatter(const int4* st_vid, TypeRanges tr, const int64_t* inc_ptr, int32_t* fill,
                              int4* incr, hipStream_t s);
// big: int32 [V] scratch for the rows sorted by whole workgroups, nbig: a
// device counter that must be zero on entry
// contrib: each row's sorted contribution codes; kcol / kbeg: the row's
// distinct columns and the offset of each one's first contribution, written
// compactly from the row's contribution offset; ncols: their count
hipError_t launch_sym_rowsort(int32_t V, int32_t max_deg, const int64_t* inc_ptr, const int4* incr,
                              TypeRanges tr, const int64_t* kptr, uint32_t* contrib,
                              int32_t* kcol, int32_t* kbeg, int32_t* ncols, int32_t* big, int64_t* nbig,
                              hipStream_t s);
hipError_t launch_sym_fill(int32_t V, const int64_t* kptr, const int32_t* kcol, const int32_t* kbeg,
                           const int32_t* row_ptr, int32_t* col_idx, int64_t* cptr, int32_t* slot_row,
                           int32_t* diag_slot, unsigned long long* whead, int32_t* wrow, int64_t nnzb,
                           hipStream_t s);
// tslot[s] = slot of (c, r) for every block s = (r, c) with c > r, else -1
hipError_t launch_sym_transpose(int64_t nnzb, const int32_t* slot_row, const int32_t* col_idx,
                                const int32_t* row_ptr, int32_t* tslot, hipStream_t s);

// ---- eval.hip
// waves: workgroup size in wavefronts (1, 2, 4 or 8)
// mult: multiplicity per staged pair, nullable (all 1)
hipError_t launch_eval(const int4* st_vid, const int32_t* mult, TypeRanges tr, const double* x, const double* xr,
                       const DevParams& pm, double* rec_main, double* rec_extra, double* rec_a1, int waves,
                       hipStream_t s);
// per-scene energies from the per-vertex shares: pieces, then scenes
hipError_t launch_energy(const double* ev, const int2* pieces, int32_t npieces, const int32_t* poff, int32_t S,
                         double* part, double* energy, hipStream_t s);

// ---- assemble.hip
// mode bit 1: gradient and per-vertex energy shares, bit 2: diagonal block
// values; lanes per row: 4, 8, 16 or 32
// rows are visited in the order `order` (a permutation of 0..V-1; null: 0..V-1)
hipError_t launch_rows_diag(int mode, int32_t V, const int32_t* order, const int32_t* diag_slot, const int64_t* cptr,
                            const uint32_t* contrib, const double* rec_main, const double* rec_extra,
                            const double* rec_a1, int64_t e0,
                            int64_t m0, const double* diag, double* grad, double* ev, void* val, int dtype,
                            int64_t nnzb, int lanes, hipStream_t s);
// blocks above the diagonal are summed once and stored with their
// transpose at tslot, row by row in the order `order` (null: storage order); waves: workgroup size
// in wavefronts (1, 2, 4 or 8)
hipError_t launch_offdiag(int32_t V, const int32_t* order, const int32_t* row_ptr, const int32_t* diag_slot,
                          int64_t nnzb, const int32_t* col_idx, const int32_t* tslot,
                          const int64_t* cptr, const uint32_t* contrib, const double* rec_main,
                          const double* rec_extra, int64_t e0, int64_t m0, void* val, int dtype, int waves,
                          hipStream_t s);
hipError_t launch_pair_inspect(const int4* st_vid, const int32_t* st_src, const int32_t* smult, TypeRanges tr,
                               const double* rec_main, const double* rec_extra, const double* rec_a1, const double* x,
                               const double* xr,
                               const DevParams& pm, int32_t* src, int32_t* type, int32_t* vid, int32_t* mult,
                               double* energy, double* grad, double* hess, hipStream_t s);

// matrix-free operator (assemble.hip): everything the two passes read
struct MfView {
    int32_t V;
    TypeRanges tr;
    const int4* st_vid;
    const int32_t* order;
    const int32_t* diag_slot;
    const int64_t* cptr;
    const uint32_t* contrib;
    const double* rec_main;
    const double* rec_extra;
    const int64_t* inc_ptr;  // per-vertex incidence offsets of the build
    const double* diag;      // per-vertex diagonal term, nullable = 0
    const double* g;         // [incidences][3] c_i w~_k, row by row (per eval)
    double2* ab;             // [Ps] (alpha, beta) of the current product (scratch)
    // dense local Hessians [Ps][12][12] (gipc_proxy_dense) instead of the
    // factors when non-null, multiplied by dense_scheme (dense.hip)
    const double* dense;
    int dense_scheme;
};
// y = (diag (x) I3 + H) x; with part, one partial of x . y per workgroup
// (mf_num_parts of them); kernels return at once when sc->done (nullable)
hipError_t launch_mf_apply(const MfView& m, const double* x, double* y, double* part, const PcgScalars* sc,
                           hipStream_t s);
hipError_t launch_mf_diag_inverse(const MfView& m, double* minv, hipStream_t s);
hipError_t launch_mf_coef(const MfView& m, double* g, hipStream_t s);
// the same product and preconditioner from m.dense (dense.hip)
hipError_t launch_dense_apply(const MfView& m, const double* x, double* y, double* part, const PcgScalars* sc,
                              hipStream_t s);
hipError_t launch_dense_diag_inverse(const MfView& m, double* minv, hipStream_t s);
int64_t mf_num_parts(int32_t V);

// dense projected proxy Hessians per staged pair, analytic or numeric
// (numeric.hip); hess [Ps][12][12]
hipError_t launch_proxy_dense(int method, const int4* st_vid, const int32_t* mult, const TypeRanges& tr,
                              const double* x, const double* xr, const DevParams& pm, double* hess, hipStream_t s);

// lagged friction (friction.hip): lag [Ps][9] at x^n; eval writes fr [Ps][16],
// grad [V][3], energy shares ev [V] and, with val, adds the blocks
hipError_t launch_fric_lag(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, const double* x,
                           const double* xr, const DevParams& pm, double mu, double* lag, hipStream_t s);
hipError_t launch_fric_eval(int32_t V, const int4* st_vid, const TypeRanges& tr, const double* lag, const double* x,
                            double sv, double* fr, const int32_t* row_ptr, const int32_t* diag_slot,
                            const int64_t* cptr, const uint32_t* contrib, double* grad, double* ev, void* val,
                            int dtype, int64_t nnzb, hipStream_t s);

// contact candidates (candidates.hip)
struct CandGrid {
    double org[3];
    double h[3];
    int32_t n[3];
};
int32_t cand_bound_blocks(int64_t V, int64_t FE);
// part [nb][9]: min x y z, max x y z, largest primitive extent along x y z
hipError_t launch_cand_bounds(const double* x, int32_t V, const int32_t* tris, int64_t F, const int32_t* edges,
                              int64_t E, double* part, int32_t nb, hipStream_t s);
hipError_t launch_cand_check(int32_t V, const int32_t* vobj, const int32_t* tris, int64_t F, const int32_t* edges,
                             int64_t E, int64_t* counters, hipStream_t s);
// cell table of n primitives of nper vertices: counts and offsets off
// [ncell+1] (off[ncell] = entries), then the entries ent [off[ncell]],
// each cell's in increasing id (raw [off[ncell]]: unsorted, scratch)
hipError_t launch_cell_count(gipc_ctx* ctx, const double* x, const int32_t* prims, int nper, int64_t n,
                             const CandGrid& g, int32_t* count, int32_t* fill, int64_t* off, hipStream_t s);
hipError_t launch_cell_fill(const double* x, const int32_t* prims, int nper, int64_t n, const CandGrid& g,
                            int32_t* fill, const int64_t* off, int32_t* raw, int32_t* ent, hipStream_t s);
// 64-byte query records of n primitives (box, vertex ids, object)
constexpr int kPrimRecBytes = 64;
hipError_t launch_prim_records(const double* x, const int32_t* prims, int nper, int64_t n, const int32_t* vobj,
                               void* rec, hipStream_t s);
// query tables, kind 0: points, 1: edge records (qrec): span[q] = cells
// the query's box inflated by dhat covers, count[cell] += queries covering
// it; then the queries of each cell at ent + off[cell]
hipError_t launch_qcells_count(int kind, const double* x, int64_t nq, const void* qrec, const CandGrid& g,
                               double dhat, int32_t* span, int32_t* count, hipStream_t s);
hipError_t launch_qcells_fill(int kind, const double* x, int64_t nq, const void* qrec, const CandGrid& g,
                              double dhat, const int64_t* off, int32_t* fill, int32_t* ent, hipStream_t s);
// n[cell] = hit-mask slots of the cell's pairs pass (kind 1: chunks of 64
// queries times primitives; kind 0: chunks of 64 triangles times points)
hipError_t launch_cell_slots(int kind, const CandGrid& g, const int64_t* qtoff, const int64_t* coff, int64_t* n,
                             hipStream_t s);
// per cell, its queries (qtoff/qent) against its primitives (coff/cent,
// records trec): kind 0 points vs triangles, 1 edges vs edges of larger
// index; per visit e = qeoff[q] + rank of the cell in q's walk, counts into
// cnt[e] and hit masks into bal + boff[cell] (emit = false), or int32 [4]
// tuples at out + 4 eoff[e] from those masks (emit = true); evis (one per
// query-table entry) carries each visit's e from the first to the second
hipError_t launch_cell_pairs(int kind, bool emit, const double* x, const int32_t* vobj, const void* qrec,
                             const void* trec, const CandGrid& g, double dhat, const int64_t* qtoff,
                             const int32_t* qent, const int64_t* qeoff, const int64_t* coff, const int32_t* cent,
                             int32_t* cnt, const int64_t* eoff, const int64_t* boff, uint64_t* bal,
                             int64_t* evis, int32_t* out, hipStream_t s);

// ---- accd.hip
// additive CCD of P tuples moving by disp; counters [6] (see k_accd_reset)
hipError_t launch_accd(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* disp, double s,
                       double tc, int32_t max_iter, double* toi, unsigned long long* counters, hipStream_t st);

// ---- solve.hip
hipError_t launch_spmv(const gipc_bsr& A, const void* x, void* y, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);
// streaming read of bytes / 16 aligned 16-byte words (sink: device uint32, written only by chance)
hipError_t launch_read(const void* src, int64_t bytes, uint32_t* sink, hipStream_t s);
// with mf set, the operator is matrix-free (A is not read)
// delta = 1: stop when r.z <= rtol r0.z0 instead of ||r|| <= rtol ||b||;
// *conv (nullable) receives whether the stopping test held
hipError_t pcg_run(gipc_ctx* ctx, const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                   int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf = nullptr,
                   int delta = 0, int* conv = nullptr);
// the same on buffers carved from one device range ws of at least
// pcg_workspace_bytes(A, mf) bytes (no allocation)
size_t pcg_workspace_bytes(const gipc_bsr& A, const MfView* mf);
hipError_t pcg_run_in(void* ws, const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                      int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf = nullptr);

}  // namespace gipc
