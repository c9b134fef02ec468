/*
 * gipc.h -- C ABI of the MI355X (gfx950) implementation of the GIPC barrier
 * hot path (Huang, Chitalu, Lin, Komura: "GIPC: Fast and stable Gauss-Newton
 * optimization of IPC barrier energy").
 *
 * Per contact pair the library evaluates the rewritten barrier energy
 * (Eq. 24, optionally mollified by Eq. 25-29 for edge-edge pairs), its
 * gradient (Eq. 13-14, Eq. 30) and its analytically projected Gauss-Newton
 * proxy Hessian (Eq. 18-23 and Eq. 32-36), assembles the local Hessians
 * into a 3x3 block-sparse (BSR) matrix, and solves with it by block-Jacobi
 * preconditioned conjugate gradients (Sec. 7.2).
 *
 * Conventions for every entry point:
 *  - Pointers documented as "device" are HIP device pointers; the caller
 *    owns them.  Buffers the library needs internally live in the context.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it and the call returns; outputs are valid once
 *    the stream has completed, unless a function states that it
 *    synchronises.
 *  - Functions return gipc_status and never throw or exit.  On an error the
 *    context keeps a message (gipc_ctx_last_error).
 *  - A context is bound to the device that was current at creation and must
 *    not be used from two host threads at once.
 */
#ifndef GIPC_H
#define GIPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GIPC_OK = 0,
    GIPC_ERR_INVALID_ARG = -1,   /* NULL pointer, negative size, bad flag */
    GIPC_ERR_INDEX = -2,         /* malformed tuple, vertex id out of range, repeated vertex,
                                    tuple spanning two scenes of a batch */
    GIPC_ERR_DEGENERATE = -3,    /* reported by gipc_get_info: pairs with d = 0 or non-finite d */
    GIPC_ERR_HIP = -4,           /* a HIP runtime call failed */
    GIPC_ERR_WORKSPACE = -5,     /* allocation failed or a documented capacity limit was exceeded */
    GIPC_ERR_BREAKDOWN = -6,     /* PCG: p^T A p <= 0 (A not positive definite) */
    GIPC_ERR_STATE = -7,         /* call order violated (e.g. eval before build) */
    GIPC_WARN_NOT_CONVERGED = 1, /* PCG stopped at maxit above the tolerance */
    GIPC_WARN_STALE = 2          /* gipc_pairs_check: the staged pairs no longer match the tuples at x;
                                    rebuild with gipc_pairs_build before evaluating there */
} gipc_status;

/* parameter flags */
#define GIPC_FLAG_FILTER 0x1u        /* eigenvalue filter of Eq. 23 */
#define GIPC_FLAG_MOLLIFY 0x2u       /* nearly-parallel edge-edge mollifier, Eq. 25-36 */
#define GIPC_FLAG_BARRIER_EQ12 0x4u  /* non-stiffened barrier Eq. 12 instead of Eq. 24 (test mode) */
#define GIPC_FLAG_NO_MERGE 0x8u      /* gipc_pairs_build: keep duplicate reduced constraints apart */
#define GIPC_FLAGS_DEFAULT (GIPC_FLAG_FILTER | GIPC_FLAG_MOLLIFY)

/* A batch of independent scenes concatenated into one mesh and one tuple
 * list (an extension: the paper evaluates one scene at a time).  Scene s
 * owns the vertices [vert_off[s], vert_off[s+1]); every tuple's vertices
 * must lie in one scene.  Device arrays:
 *   vert_off  int32 [S+1]  non-decreasing, vert_off[0] = 0, vert_off[S] = V
 *   dhat      double [S]   > 0, the scene's dhat (replaces params->dhat)
 *   kappa     double [S]   >= 0, the scene's kappa (replaces params->kappa)
 * gipc_pairs_build reads and checks all three (INVALID_ARG) and keeps the
 * scene of every vertex; later calls on that build must pass a batch with
 * the same S and the same dhat and kappa values (they are read again on
 * the device, not re-checked). */
typedef struct {
    int32_t S;
    const int32_t* vert_off;
    const double* dhat;
    const double* kappa;
} gipc_batch;

typedef struct {
    double dhat;        /* computational accuracy target (Eq. 6, Eq. 9) */
    double kappa;       /* barrier stiffness multiplying every pair's energy */
    double dthr_ratio;  /* d_thr / dhat of the filter, Eq. 23 (paper: 0.1) */
    double epsx_ratio;  /* eps_x = epsx_ratio |x12-x11|^2 |x22-x21|^2 at rest, Eq. 25 (paper: 1e-3) */
    uint32_t flags;     /* GIPC_FLAG_* */
    const gipc_batch* batch;  /* host struct, NULL for one scene (dhat, kappa above) */
} gipc_params;

/* Vertex positions (the x of Eq. 1).  Both arrays: device, float64 [V][3]
 * (AoS, 24 bytes per vertex).  x_rest (the reference positions of Eq. 25)
 * may be NULL, meaning x. */
typedef struct {
    int32_t V;
    const double* x;
    const double* x_rest;
} gipc_mesh;

/* Contact tuples of vertex ids with the type in the signs (Sec. 7.2,
 * "Data structures"; a negative entry -(i+1) stands for vertex i); device,
 * int32 [P][4]:
 *   [a0, a1, b0, b1]            edge-edge pair
 *   [-(p+1), t0, t1, t2]        point-triangle pair
 *   [-(p+1), e0, e1, -1]        point-edge pair
 *   [-(p+1), q, -1, -1]         point-point pair
 * and the close-to-parallel encodings (second entry negative):
 *   [a0, -(a1+1), b0, b1]       edge-edge pair
 *   [-(p+1), -(o+1), e0, -(e1+1)]   point p of edge (p, o) against edge (e0, e1)
 *   [-(p+1), -(o+1), -(q+1), -(r+1)] point p of edge (p, o) against point q of edge (q, r)
 * Every pair's distance is the constrained minimum over its primitives
 * (Eq. 4 / Eq. 5; the last two are the point-segment and point-point
 * sub-problems of Eq. 5); the library reduces it to its sub-type itself.
 * Whether the mollifier of Eq. 25 applies is decided from the two edges
 * (c = |a x b|^2 against eps_x) for every edge-edge family tuple, whatever
 * its encoding says. */
typedef struct {
    int64_t P;
    const int32_t* tuples;
} gipc_pairs;

enum { GIPC_F64 = 0, GIPC_F32 = 1 };

/* Block-sparse matrix with 3x3 blocks.  row_ptr: device int32 [nbrows+1];
 * col_idx: device int32 [nnzb], columns ascending within a row, every row
 * holding its diagonal block; val: device, component-major [9][nnzb]
 * (component 3a+b of block s at val[(3a+b)*nnzb + s]) of float64 (GIPC_F64)
 * or float32 (GIPC_F32).  Vectors multiplied with it are [nbrows][3] of the
 * same dtype.
 * wave_head, wave_row: optional row-start map of the blocks in groups of 64,
 * filled by gipc_bsr_pattern from the context's pattern (owned by the
 * context, valid until the next build): for group g = 0 .. ceil(nnzb/64)-1,
 * bit l of wave_head[g] (device uint64) is set when block 64g+l is the first
 * block of its row, and wave_row[g] (device int32) is the row of block 64g.
 * With both set (which requires every row to hold a block) an FP64 product
 * runs one block per lane; with either NULL, as in a descriptor made by the
 * caller, it runs row by row.  Results agree to rounding order. */
typedef struct {
    int32_t nbrows;
    int64_t nnzb;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    void* val;
    int32_t dtype;
    const uint64_t* wave_head;
    const int32_t* wave_row;
} gipc_bsr;

/* Counts of the last gipc_pairs_build (host struct). */
typedef struct {
    int64_t n_candidates;   /* tuples given */
    int64_t n_active;       /* pairs closer than dhat after classification */
    int64_t n_by_type[8];   /* active pairs by sub-type: [1] PT, [2] PE, [3] PP, [4] EE,
                               [5] EE, [6] PE, [7] PP cut from mollified edge-edge pairs */
    int64_t n_staged;       /* staged pairs after merging duplicate PE / PP constraints */
    int64_t n_staged_by_type[8]; /* staged pairs by sub-type (as n_by_type) */
    int64_t n_degenerate;   /* pairs at distance 0 or with non-finite positions (skipped) */
    int64_t first_degenerate; /* tuple index of the first one, -1 if none */
    int64_t nnzb;           /* blocks of the assembled matrix */
    int64_t n_contrib;      /* local-block contributions gathered by the assembly */
    int32_t max_row_pairs;  /* largest number of pairs touching one vertex */
    int64_t n_degenerate_prims;  /* tuples with an edge of zero length or a triangle of zero area whose
                                    distance is positive: evaluated by the remaining sub-problems of
                                    Eq. 4 / Eq. 5 (the smallest over the triangle's edges, or over the
                                    endpoints), counted here */
    int64_t first_degenerate_prim; /* tuple index of the first one, -1 if none */
} gipc_info;

typedef struct gipc_ctx gipc_ctx;

/* Status name ("GIPC_OK", ...). */
const char* gipc_status_string(int status);

/* Create a context on the current HIP device.  Allocates only a few small
 * buffers; larger ones grow on demand (hipMalloc).  *out is NULL on failure. */
gipc_status gipc_ctx_create(gipc_ctx** out);

/* Device memory from the caller, e.g. a framework's caching allocator:
 * alloc returns a pointer to at least `bytes` bytes of device memory on
 * `device`, 256-byte aligned, or NULL (the call needing it then fails with
 * WORKSPACE); free takes back a pointer alloc returned, with the same size.
 * The library calls them from the host thread that calls it; it hands a
 * block back only when nothing queued on the device can still use it (it
 * synchronises the device first: buffers grow rarely, and on destroy). */
typedef struct {
    void* (*alloc)(void* user, size_t bytes, int device);
    void (*free)(void* user, void* ptr, size_t bytes, int device);
    void* user;
} gipc_allocator;

/* gipc_ctx_create with every buffer of the context taken from `al` (host
 * struct, copied; NULL = hipMalloc).  INVALID_ARG if a callback is NULL. */
gipc_status gipc_ctx_create_with_allocator(const gipc_allocator* al, gipc_ctx** out);
/* Free every buffer the context holds (synchronises its device).  NULL ok. */
void gipc_ctx_destroy(gipc_ctx* ctx);
/* Message of the last error on this context ("" if none). */
const char* gipc_ctx_last_error(const gipc_ctx* ctx);

/*
 * Stage a pair list and build the block pattern (Sec. 7.2 "Data
 * structures"; matrix decomposition of supplement Sec. 6).
 * Classifies every tuple at positions mesh->x by the active constraints of
 * Eq. 4 / Eq. 5, drops pairs at distance >= dhat, sorts the active ones by
 * sub-type (the four type buffers of supplement Sec. 6) and builds the BSR
 * pattern of diag + sum_k S_k^T H_k S_k over the vertices each pair's
 * distance depends on (all four for mollified edge-edge pairs).
 * With params->batch, each tuple is tested against its own scene's dhat.
 * Active point-edge and point-point constraints with the same vertices
 * (the point and the unordered edge, or the unordered vertex pair) are
 * merged into one staged pair with an integer multiplicity that scales its
 * energy, gradient and Hessian: the sum of Eq. 3 over the candidates is
 * unchanged (up to rounding order).  GIPC_FLAG_NO_MERGE keeps them apart.
 * Synchronises `stream` (three times, four with a batch) to size the
 * pattern; `info` (host, nullable) receives the counts.  Errors:
 * INVALID_ARG, INDEX (no state is kept), WORKSPACE (a vertex touched by
 * more than 2048 active pairs), HIP.
 */
gipc_status gipc_pairs_build(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_pairs* pairs,
                             const gipc_params* params, void* stream, gipc_info* info);

/* Result of gipc_pairs_check (host struct). */
typedef struct {
    int64_t n_entered;     /* tuples closer than dhat at x that were not at the build */
    int64_t n_left;        /* tuples active at the build, at or beyond dhat at x, whose staged sub-type
                              formula also gives d >= dhat there (the evaluation drops them: harmless) */
    int64_t n_changed;     /* tuples active at the build whose sub-type, stencil or mollifier decision
                              differs at x, or that left dhat while their staged formula did not */
    int64_t n_degenerate;  /* tuples at distance 0 or non-finite at x */
    int64_t first;         /* index of the first tuple counted in n_entered or n_changed, -1 if none */
} gipc_check;

/*
 * Whether the staged pairs of the last build still describe the tuples at
 * positions mesh->x.  The evaluation entry points evaluate each staged pair
 * with the sub-type formula fixed at the build (Eq. 4 / Eq. 5 reduced to the
 * active constraints there): exact at the build's positions and wherever
 * the constrained minimum keeps the same active set, but not once a point
 * slides off a triangle or edge, a pair comes within dhat, or an edge pair
 * crosses the mollifier threshold of Eq. 25.  This call classifies the same
 * tuples (pairs: the build's list, unchanged; params as at the build) at
 * mesh->x and compares tuple by tuple.  Returns GIPC_OK when the build still
 * holds (n_entered = n_changed = 0), GIPC_WARN_STALE when it must be rebuilt
 * before an evaluation at x, or an error: INVALID_ARG, STATE (no build, V,
 * P or the batch differ from the build), INDEX (malformed tuples), HIP.
 * out (host, nullable) receives the counts.  Synchronises `stream`.
 */
gipc_status gipc_pairs_check(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_pairs* pairs,
                             const gipc_params* params, gipc_check* out, void* stream);

/* Counts of the last successful build (host copy, no synchronisation). */
gipc_status gipc_get_info(const gipc_ctx* ctx, gipc_info* info);

/* Pattern of the last build: fills nbrows, nnzb, row_ptr, col_idx,
 * wave_head and wave_row (device pointers owned by the context, valid until
 * the next build); leaves val and dtype untouched. */
gipc_status gipc_bsr_pattern(const gipc_ctx* ctx, gipc_bsr* A);

/*
 * Barrier energy and gradient of the staged pairs at mesh->x (Eq. 24 / 29,
 * Eq. 13-14 / 30): energy (device, double [S], S = 1 without a batch)
 * receives kappa_s * sum_{k in scene s} e_k b_k per scene; grad (device,
 * double [V][3], overwritten).  Also stores each pair's compact
 * proxy-Hessian factors (Eq. 18-23, 32-36) in the context for
 * gipc_assemble_bsr.  Deterministic for a given gipc_tune (no
 * floating-point atomics; sums in fixed orders).
 * Errors: INVALID_ARG, STATE (no build, V or the batch differs from the
 * build).
 */
gipc_status gipc_barrier_eval(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params,
                              double* energy, double* grad, void* stream);

/*
 * Assemble the proxy Hessians of the last gipc_barrier_eval plus
 * diag(d_v) (x) I3 into A->val (device, [9][nnzb] of A->dtype; FP32 values
 * are rounded once from FP64 sums).  A->row_ptr / col_idx / nnzb / nbrows
 * must be the context's pattern (gipc_bsr_pattern).  diag: device double
 * [V] (e.g. mass / dt^2), nullable = 0.  Errors: INVALID_ARG, STATE.
 */
gipc_status gipc_assemble_bsr(gipc_ctx* ctx, const double* diag, const gipc_bsr* A, void* stream);

/* gipc_barrier_eval followed by gipc_assemble_bsr, with the gradient and
 * the diagonal blocks produced by one kernel. */
gipc_status gipc_eval_assemble(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params,
                               double* energy, double* grad, const double* diag, const gipc_bsr* A,
                               void* stream);

/* y = A x (device vectors of A's dtype, [nbrows][3]); any BSR in the layout
 * above.  Deterministic.  Errors: INVALID_ARG. */
gipc_status gipc_bsr_spmv(const gipc_bsr* A, const void* x, void* y, void* stream);

/*
 * Solve A x = b by conjugate gradients preconditioned with the inverses of
 * A's 3x3 diagonal blocks (Sec. 7.2; Saad Alg. 9.1).  b, x: device double
 * [nbrows][3]; x holds x0 on entry and the result on return.  A may be FP64
 * or FP32; with FP32 blocks the product A p reads an FP32 copy of p and
 * accumulates in FP32, while vectors, dot products and the preconditioner
 * (inverted in FP64 from the FP32 blocks) stay FP64.  A batch is solved as
 * one block-diagonal system.  Stops when ||r||_2 <= rtol ||b||_2 (checked every
 * iteration on the device; the host polls every 16 iterations) or after
 * maxit iterations; rtol = 0 runs exactly maxit iterations.  Synchronises
 * `stream`; *iters and *relres (host, nullable) receive the iterations run
 * and ||r||/||b||.  Returns OK, WARN_NOT_CONVERGED (rtol > 0 not reached),
 * BREAKDOWN, INVALID_ARG or HIP.
 */
gipc_status gipc_pcg(gipc_ctx* ctx, const gipc_bsr* A, const double* b, double* x, double rtol, int32_t maxit,
                     int32_t* iters, double* relres, void* stream);

/*
 * gipc_pcg stopped by the paper's own termination (its PCG in the
 * implementation section, tolerance 1e-4 there): after iteration k when
 * r_k . z_k <= eps r_0 . z_0, z = M^-1 r the preconditioned residual
 * (checked before the first iteration too), or after maxit iterations.
 * Same arguments, layouts, kernels and synchronisation as gipc_pcg;
 * *relres still receives ||r||/||b||.  Returns OK when the test held,
 * WARN_NOT_CONVERGED when eps > 0 and maxit came first, BREAKDOWN,
 * INVALID_ARG (eps < 0, maxit < 0, bad matrix) or HIP.
 */
gipc_status gipc_pcg_delta(gipc_ctx* ctx, const gipc_bsr* A, const double* b, double* x, double eps,
                           int32_t maxit, int32_t* iters, double* relres, void* stream);

/*
 * gipc_pcg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, kernels and launch sequence as gipc_pcg, with its work
 * vectors, inverted diagonal blocks, reduction partials and scalars in a
 * fixed area of GIPC_PCG_STATIC_SCRATCH_BYTES bytes that the library's code
 * object holds on every GPU it is loaded on (kept until the process ends).
 * No context; calls no hipMalloc or hipFree.  The caller passes the matrix
 * and the vectors (b, x: device double [nbrows][3], x holds x0 on entry) as
 * for gipc_pcg, and gets the same results.  The area needs about
 * 168 bytes per block row (180 with FP32 blocks) plus 24 bytes per
 * workgroup of the product, so it holds systems of up to about 390,000
 * block rows (370,000 with FP32 blocks); larger ones return WORKSPACE with
 * nothing launched.  Every
 * call on a GPU uses that GPU's one area, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * GPU -- from two host threads, or on two streams without ordering -- race
 * and give wrong results.  Synchronises `stream`, except with rtol = 0 and
 * both iters and relres NULL: the call then only enqueues its kernels (no
 * read-back, no synchronisation, no memset, so it can be recorded in a HIP
 * graph) and cannot report a breakdown (the kernels stop iterating at one).
 * Returns as gipc_pcg (BREAKDOWN, WARN_NOT_CONVERGED, INVALID_ARG, WORKSPACE,
 * HIP).
 */
#define GIPC_PCG_STATIC_SCRATCH_BYTES (64u << 20)
gipc_status gipc_pcg_static(const gipc_bsr* A, const double* b, double* x, double rtol, int32_t maxit,
                            int32_t* iters, double* relres, void* stream);

/*
 * Matrix-free operator: y = (diag (x) I3 + sum_k S_k^T H_k S_k) x with the
 * proxy Hessians H_k of the last eval (Eq. 20-23 and Eq. 32-36, in the factor
 * form of Eq. 15-17), applied pair by pair from their compact factors without forming a
 * matrix; this is the operator of the paper's matrix-free PCG (supplement,
 * Sec. 6).  It equals gipc_bsr_spmv with the matrix gipc_assemble_bsr would
 * produce in FP64 (same products, summed in another order).  x, y: device
 * double [V][3], must not alias; diag: device double [V], nullable = 0.  The
 * context's pattern and records are read; the first call after an eval
 * also lays out 24 bytes per incidence (pair, vertex) of that eval's
 * factors, and every call writes 16 bytes of scratch per staged pair, so
 * calls on one context must not overlap.
 * Deterministic.  Errors: INVALID_ARG, STATE (no build + eval), HIP.
 */
gipc_status gipc_mf_apply(gipc_ctx* ctx, const double* diag, const double* x, double* y, void* stream);

/*
 * gipc_pcg on the matrix-free operator above (FP64 throughout): the
 * preconditioner inverts the 3x3 diagonal blocks summed from the same
 * factors.  Same arguments, stopping rule, synchronisation and returns as
 * gipc_pcg, with the matrix replaced by the last eval and diag.
 */
gipc_status gipc_pcg_mf(gipc_ctx* ctx, const double* diag, const double* b, double* x, double rtol, int32_t maxit,
                        int32_t* iters, double* relres, void* stream);

/* schemes of gipc_dense_apply / gipc_pcg_dense */
#define GIPC_DENSE_THREAD 0  /* one lane per pair computes its whole local product */
#define GIPC_DENSE_ENTRY 1   /* one lane per matrix entry, rows summed by a wavefront segmented reduction */

/*
 * The matrix-free product of the paper's PCG from dense local Hessians, in
 * the two parallel schemes its Table 2 compares (supplement Sec. 6,
 * "Parallel local matrix-vector multiplication"):
 * y = (diag (x) I3 + sum_k S_k^T H_k S_k) x with H_k read from hess (device
 * double [info.n_staged][12][12] as gipc_proxy_dense writes it on the
 * current build: the leading 3n x 3n block of pair k, n its stencil
 * vertices, times its multiplicity), one launch per stencil size (the
 * paper's type buffers).  GIPC_DENSE_THREAD gives each pair one lane, which
 * forms its 3n local rows; GIPC_DENSE_ENTRY gives each matrix entry one lane
 * and sums the 3n lanes of a local row inside the wavefront (a segmented
 * reduction; rows cut by a wavefront boundary are summed in two parts).
 * Both add the local rows to y with FP64 atomics, as the paper does, so the
 * result varies from run to run in its last bits (the summation order is
 * not fixed).  x, y: device double [V][3], must not alias; diag: device
 * double [V], nullable = 0.  Errors: INVALID_ARG (bad scheme, NULL),
 * STATE (no build), HIP.
 */
gipc_status gipc_dense_apply(gipc_ctx* ctx, const double* hess, int32_t scheme, const double* diag, const double* x,
                             double* y, void* stream);

/*
 * gipc_pcg with the product of gipc_dense_apply (FP64 throughout): the
 * preconditioner inverts diag + the 3x3 diagonal blocks of the local
 * Hessians, summed per vertex in a fixed order.  Same arguments, stopping
 * rule, synchronisation and returns as gipc_pcg.
 */
gipc_status gipc_pcg_dense(gipc_ctx* ctx, const double* hess, int32_t scheme, const double* diag, const double* b,
                           double* x, double rtol, int32_t maxit, int32_t* iters, double* relres, void* stream);

/* Surface topology for candidate generation (device arrays): the object
 * id of every vertex (candidates only pair different objects; a triangle or
 * edge belongs to the object of its first vertex), triangles int32 [F][3]
 * and edges int32 [E][2]. */
typedef struct {
    const int32_t* vobj;
    const int32_t* tris;
    int64_t F;
    const int32_t* edges;
    int64_t E;
} gipc_topology;

/*
 * Contact candidates on the GPU: every (point p, triangle t) with p not a
 * vertex of t and every pair of edges i < j sharing no vertex, of different
 * objects, whose axis-aligned boxes come within dhat (one box inflated by
 * dhat, closed intervals): the pairs the sum of Eq. 3 ranges over before
 * the distance decides which are active.  A uniform grid stands in for the
 * paper's BVH (Sec. 7.2).  Output tuples in the encoding above, int32
 * [count][4] device: point-triangle [-(p+1), t0, t1, t2] grouped by point
 * in increasing p, then edge-edge [a0, a1, b0, b1] grouped by first edge;
 * deterministic.  *count (host) receives the number of candidates; tuples
 * are written only when tuples is non-NULL and cap >= count (else
 * WORKSPACE with *count set, nothing written; tuples = NULL only counts).
 * Synchronises `stream`.  Errors: INVALID_ARG (NULL, dhat < 0 or
 * non-finite, non-finite positions), INDEX (topology ids out of range or
 * repeated within a primitive), WORKSPACE (grid above 2^28 cells, cap), HIP.
 */
gipc_status gipc_candidates(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_topology* topo, double dhat,
                            int32_t* tuples, int64_t cap, int64_t* count, void* stream);

/* Result of gipc_accd (host struct). */
typedef struct {
    double step;          /* smallest time over the tuples (tc when P = 0): the largest feasible step */
    int64_t n_capped;     /* tuples whose search max_iter stopped (their time is the one accumulated) */
    int64_t n_touching;   /* tuples at distance 0 (or non-finite) at t = 0: time 0 */
    int32_t max_steps;    /* most trial steps any tuple took */
} gipc_accd_info;

/*
 * Step bound of the line search (maxFeasibleStepSize in Algorithm 1) by
 * additive CCD, which the paper adopts (Related Work, "Collision
 * Detection"): every tuple (the encoding of gipc_pairs, distance the
 * constrained minimum of Eq. 4 / Eq. 5) moves as x(t) = x + t disp over
 * t in [0, tc].  With the mean displacement of the tuple's vertices removed
 * and l_p the largest displacement norm over its first primitive plus the
 * largest over its second, the distance falls at most at rate l_p; from
 * d0 = d(0) the search takes a first sub-step (1 - s) d0 / l_p, then
 * 0.9 d / l_p from each accepted point (d the distance there), and stops at
 * the first trial point whose distance is below s d0, returning the time
 * accumulated before it, or returns tc once the time passes tc; no relative
 * motion gives tc and d0 = 0 gives 0.  The time is a lower bound on the
 * time of impact (the distance stays above s d0 up to it).
 * mesh->x: positions at t = 0 (device double [V][3]); disp: device double
 * [V][3]; toi: device double [P], nullable (the time of each tuple);
 * s in (0, 1): the separation kept (e.g. 0.1); tc >= 0 finite: the largest
 * step (1 for alpha <= 1); max_iter >= 1: trial steps per tuple.
 * Synchronises `stream` and fills info (host, nullable).  Errors:
 * INVALID_ARG, INDEX (a malformed tuple; info is not filled), HIP.
 */
gipc_status gipc_accd(gipc_ctx* ctx, const gipc_mesh* mesh, const double* disp, const gipc_pairs* pairs, double s,
                      double tc, int32_t max_iter, double* toi, gipc_accd_info* info, void* stream);

/* Lagged friction parameters (supplement Sec. 5): friction coefficient mu,
 * the velocity threshold eps_v of the transition f1 and the time step dt
 * (f1 reaches 1 at |u| = eps_v dt). */
typedef struct {
    double mu;
    double eps_v;
    double dt;
} gipc_friction;

/*
 * Lag the friction of the staged pairs of the last build at the previous
 * positions mesh->x (x^n; mesh->x_rest as for the barrier): per pair the
 * closest-point coefficients c of its constrained distance, the contact
 * normal n, the normal force lambda = kappa e |db/dd| (distance derivative
 * of the pair's barrier energy with its mollifier; per-scene dhat / kappa
 * of params) times mu and the multiplicity, and the anchor
 * (I - n n^T) sum_i c_i x_i^n.  Pairs inactive at x^n get no friction.
 * Stored in the context until the next gipc_pairs_build.  Errors:
 * INVALID_ARG (NULL, mu < 0, eps_v <= 0, dt <= 0, non-finite), STATE (no
 * build, V differs), HIP.
 */
gipc_status gipc_friction_lag(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params,
                              const gipc_friction* fr, void* stream);

/*
 * Lagged friction at the current positions x (device double [V][3]):
 * energy (device double [S], one per scene) = sum_k mu lambda_k f0(|u_k|),
 * grad (device double [V][3], overwritten) = its gradient, and, with A
 * non-NULL (the pattern of the last build, FP64 or FP32), the PSD-projected
 * friction Hessian blocks c_i c_j S_k ADDED to A's values; u_k is the
 * tangential sliding of the pair since x^n in the lagged basis and S_k the
 * 3x3 form of the projected 2x2 block (eigenvalues f1'(|u|) along u and
 * f1(|u|)/|u| across it, clamped at 0).  Deterministic.  Errors:
 * INVALID_ARG, STATE (no lag since the last build), HIP.
 */
gipc_status gipc_friction_eval(gipc_ctx* ctx, const double* x, double* energy, double* grad, const gipc_bsr* A,
                               void* stream);

/* methods of gipc_proxy_dense */
#define GIPC_PROJ_ANALYTIC 0
#define GIPC_PROJ_NUMERIC 1
#define GIPC_PROJ_EXACT 2

/*
 * Dense projected proxy Hessian of every staged pair of the last build at
 * positions mesh->x, for the comparison the paper makes in Table 1 (time
 * to construct and project a pair's 3n x 3n barrier Hessian).
 * GIPC_PROJ_ANALYTIC expands the factors of the analytic eigensystems
 * (Sec. 5.2-5.3, Eq. 18-21; Sec. 6.2, Eq. 32-36); GIPC_PROJ_NUMERIC builds
 * kappa D^T H D with the unprojected inner Hessian (Eq. 16-17, 31) and
 * projects it in x-space by cyclic Jacobi rotations (negative eigenvalues
 * clamped).  Non-mollified pairs give the same matrix both ways (rank one);
 * mollified pairs differ where the inner 2x2 block is indefinite.
 * GIPC_PROJ_EXACT is the traditional route the paper's table compares
 * against: the exact Hessian of the pair's energy kappa e(c) b(g(x)) -- Eq. 15
 * with the d^2 J / dx^2 term, i.e. Eq. 22 without dropping b_d grad^2 d, for
 * the sub-problem staged at the build (no filter) -- projected onto the PSD
 * cone by cyclic Jacobi rotations, on the complement of rigid translations
 * (where that matrix has its whole range: it vanishes on translations).
 * hess: device double [info.n_staged][12][12],
 * row-major, the leading 3n x 3n block filled (n = stencil vertices in
 * slot order, as gipc_pair_inspect reports them), the rest zero, times the
 * pair's multiplicity.  Does not touch the eval state.  Errors:
 * INVALID_ARG (bad method, NULL), STATE (no build, V differs), HIP.
 */
gipc_status gipc_proxy_dense(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, int32_t method,
                             double* hess, void* stream);

/*
 * Inspection of the staged pairs of the last build and the factors of the
 * last eval, expanded per pair (for tests and tooling).  Device buffers sized
 * for info.n_staged pairs, each nullable:
 *   src [Pa] int32        tuple index each staged pair came from (the first
 *                         tuple of a merged group)
 *   type [Pa] int32       sub-type code as in gipc_info.n_by_type
 *   vid [Pa][4] int32     vertex ids of the staged stencil (-1 unused)
 *   mult [Pa] int32       number of candidate tuples the staged pair stands for
 *   energy [Pa] double    mult * kappa e b of the pair, evaluated at mesh->x
 *   grad [Pa][12] double  local gradient over the 4 stencil slots, times mult  (needs an eval)
 *   hess [Pa][144] double local proxy Hessian, 12x12 row-major, times mult (needs an eval)
 * Errors: INVALID_ARG, STATE.
 */
gipc_status gipc_pair_inspect(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, int32_t* src,
                              int32_t* type, int32_t* vid, int32_t* mult, double* energy, double* grad,
                              double* hess, void* stream);

/* Plain device-to-device copy of `bytes` bytes with the library's own
 * streaming kernel (bandwidth reference for roofline fractions). */
gipc_status gipc_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* Streaming read of the first bytes - bytes % 16 bytes of src (device,
 * 16-byte aligned) with the library's own read kernel: the read-bandwidth
 * reference for roofline fractions.  sink: device, 4 bytes, written only if
 * the xor of all words read equals 0x9e3779b9 (so that no load is
 * dropped).  Errors: INVALID_ARG (negative size, NULL, misaligned src), HIP. */
gipc_status gipc_read(const void* src, int64_t bytes, void* sink, void* stream);

/*
 * Launch shapes of the evaluation and assembly kernels (per context).
 *   eval_waves     wavefronts per workgroup of the pair evaluation: 1, 2, 4, 8
 *   row_lanes      lanes per block row of the gradient / diagonal-block
 *                  gather: 4, 8, 16, 32 (changes the summation order of
 *                  those sums, hence their last bits)
 *   offdiag_waves  wavefronts per workgroup of the off-diagonal blocks: 1, 2, 4, 8
 *   row_order      order in which those two passes visit the block rows:
 *                  0 = spatial cells of the build's positions, 1 = storage
 *                  order (same results; 1 assembles faster but leaves more
 *                  of the matrix to be written back during the next kernel)
 * Default {4, 16, 4, 0}.  Set: INVALID_ARG for other values.
 */
typedef struct {
    int32_t eval_waves;
    int32_t row_lanes;
    int32_t offdiag_waves;
    int32_t row_order;
} gipc_tune;

gipc_status gipc_get_tune(const gipc_ctx* ctx, gipc_tune* tune);
gipc_status gipc_set_tune(gipc_ctx* ctx, const gipc_tune* tune);

/*
 * Autotuner: with the arguments of gipc_eval_assemble on the current build,
 * time every eval_waves, row_lanes and offdiag_waves choice (each kernel
 * alone, `reps` launches after one warm-up, HIP events on `stream`), then
 * both row orders (the two assembly passes together), keep
 * the fastest of each in the context and in *best (host, nullable).  The
 * outputs hold the result of the last timed launch of each kernel, which
 * equals a gipc_eval_assemble with the chosen shapes only up to summation
 * order: call gipc_eval_assemble afterwards.  Synchronises.  Errors as
 * gipc_eval_assemble, INVALID_ARG for reps < 1.
 */
gipc_status gipc_autotune(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                          double* grad, const double* diag, const gipc_bsr* A, int32_t reps, gipc_tune* best,
                          void* stream);

/*
 * The launch sequence of gipc_eval_assemble (pair evaluation, gradient and
 * diagonal blocks, off-diagonal blocks, per-scene energies) captured once
 * into a HIP graph for the given argument pointers; replays read whatever
 * those buffers hold then (e.g. positions updated in place) and run no
 * allocation, memset or synchronisation.  Capture uses a private stream and
 * sizes the context's buffers first (it may allocate).  A graph stays valid
 * until the next gipc_pairs_build on its context, or until
 * the context is destroyed (launch returns STATE after a rebuild).
 * Errors: as gipc_eval_assemble; HIP if capture or instantiation fails.
 */
typedef struct gipc_graph gipc_graph;

gipc_status gipc_graph_create(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                              double* grad, const double* diag, const gipc_bsr* A, gipc_graph** out);
gipc_status gipc_graph_launch(gipc_graph* graph, void* stream);
void gipc_graph_destroy(gipc_graph* graph);

#ifdef __cplusplus
}
#endif
#endif /* GIPC_H */
