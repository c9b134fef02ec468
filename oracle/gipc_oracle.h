/*
 * CPU FP64 oracle for the GIPC barrier hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow reference of what the path computes (Huang et al., "GIPC: Fast
 * and stable Gauss-Newton optimization of IPC barrier energy").  It shares no
 * code with the HIP library.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.
 *
 * Contact tuples use the paper's sign encoding (Sec. 7.2, "Data structures"):
 *   [a0, a1, b0, b1]          edge-edge pair (a1 may be -(v+1): close to parallel)
 *   [-(p+1), t0, t1, t2]      point-triangle pair
 *   [-(p+1), e0, e1, -1]      point-edge pair
 *   [-(p+1), q, -1, -1]       point-point pair
 *   [-(p+1), -(o+1), e0, -(e1+1)]     point p of edge (p, o) vs edge (e0, e1),
 *   [-(p+1), -(o+1), -(q+1), -(r+1)]  point p of edge (p, o) vs point q of
 *                             edge (q, r): the close-to-parallel encodings
 * Every pair's distance is the constrained minimum over its primitives
 * (Eq. 4 / Eq. 5, point-edge as the segment sub-problem of Eq. 4, the last
 * two as the point-segment / point-point sub-problems of Eq. 5).  The
 * mollifier applies to the kinds built on two edges (edge-edge and the last
 * two).  Other sign patterns are rejected.
 */
#ifndef GIPC_ORACLE_H
#define GIPC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double dhat;        /* computational accuracy target */
    double kappa;       /* barrier stiffness */
    double dthr_ratio;  /* filter threshold d_thr / dhat (Eq. 23), 0.1 */
    double epsx_ratio;  /* mollifier tolerance factor (Eq. 25), 1e-3 */
    int filter;         /* apply Eq. 23 */
    int mollify;        /* apply Eq. 25-36 to edge-edge families */
    int eq12;           /* use the non-stiffened barrier Eq. 12 instead of Eq. 24 */
} orc_params;

/* lagged friction (supplement Sec. 5): coefficient, the velocity threshold
 * eps_v of f1 and the time step h */
typedef struct {
    double mu;
    double eps_v;
    double dt;
} orc_fparams;

/* sub-type codes reported per pair */
enum { ORC_INACTIVE = 0, ORC_PT = 1, ORC_PE = 2, ORC_PP = 3, ORC_EE = 4, ORC_DEGENERATE = 7 };

/* barrier b(g) and its first two derivatives in g (Eq. 24, or Eq. 12) */
void orc_barrier(double g, double dhat, int eq12, double* b, double* db, double* d2b);
/* mollifier e(c) and derivatives (Eq. 25) */
void orc_mollifier(double c, double epsx, double* e, double* de, double* d2e);

/* Cyclic Jacobi eigen-decomposition of a symmetric n x n row-major matrix.
 * lam[n] receives eigenvalues, vec (n x n row-major) eigenvectors in columns. */
int orc_jacobi_eig(int n, const double* A, double* lam, double* vec);

/*
 * One contact pair.  xs / xr hold the stencil's current / rest positions as
 * [4][3] (unused rows ignored).  Outputs: energy, gradient [12] and proxy
 * Hessian [12][12] over the stencil's 4 vertex slots (slots the tuple does
 * not use stay zero), the sub-type, whether the mollifier applied and d^2.
 * Optional debug outputs (nullable): the inner Hessian in vec(J) space
 * before projection [9*9], its projection [9*9], vec(db/dJ) [9] and m.
 */
int orc_pair_local(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm,
                   double* E, double* grad12, double* hess144, int* subtype, int* mollified, double* dist2,
                   double* innerH, double* innerHp, double* dbdJ, int* m_out);

/*
 * The traditional route for the same pair: Kx = kappa D^T H D, the proxy
 * Hessian with the unprojected inner Hessian, [12][12], and Px, its
 * projection onto the PSD cone computed in x-space (3n x 3n, padded to 12)
 * by cyclic Jacobi rotations.  For non-mollified pairs Px equals the proxy
 * Hessian of orc_pair_local (a rank-one matrix); for mollified pairs it
 * differs when the inner 2x2 block is indefinite.  Both nullable.
 */
int orc_pair_xproj(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm, double* Kx,
                   double* Px);

/* orc_pair_xproj's Px for every tuple of a list, pairPx [P][12][12]. */
int orc_eval_xproj(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                   const orc_params* prm, int nthreads, double* pairPx);

/*
 * The traditional route of the paper's Table 1 comparison for one pair: H,
 * the exact Hessian of the pair's energy kappa e(c) b(g(x)) (Eq. 15 with the
 * d^2 J / dx^2 term, equivalently Eq. 22 without dropping b_d grad^2 d), for
 * the sub-problem of Eq. 4 / Eq. 5 active at x, by second-order forward
 * differentiation of closed-form distances; and Hp, its projection onto the
 * PSD cone by cyclic Jacobi rotations (negative eigenvalues clamped).  No
 * filter (Eq. 23 belongs to the proxy).  [12][12] over the stencil slots,
 * both nullable; inactive or degenerate pairs give zeros.  Returns -1 on a
 * malformed tuple.
 */
int orc_pair_exact(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm, double* H,
                   double* Hp);

/* orc_pair_exact for every tuple of a list: pairH, pairHp [P][12][12]
 * (nullable).  Returns -1 on a malformed tuple or index. */
int orc_eval_exact(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                   const orc_params* prm, int nthreads, double* pairH, double* pairHp);

/*
 * Additive CCD of one tuple moving as x(t) = xs + t ps (both [4][3]): the
 * accumulated safe time *toi (lower bound on the time of impact, at most tc;
 * tc without relative motion; 0 at distance 0), with the minimum
 * separation fraction s.  *iters (nullable) = trial steps, -1 if max_iter
 * stopped it.  Returns -2 on a malformed tuple, 1 at distance 0, else 0.
 */
int orc_accd(const int32_t tuple[4], const double* xs, const double* ps, double s, double tc, int max_iter,
             double* toi, int* iters);

/* orc_accd for every tuple of a list (positions x, displacements disp, both
 * [V][3]): toi [P].  Returns the number stopped by max_iter, -1 on a
 * malformed tuple or index. */
int64_t orc_accd_scene(int32_t V, const double* x, const double* disp, int64_t P, const int32_t* tuples, double s,
                       double tc, int max_iter, int nthreads, double* toi);

/* f0, f1 and f1' of the friction transition at y (h = dt). */
void orc_friction_f(double y, double eps_v, double dt, double* f0, double* f1, double* df1);

/*
 * Lagged friction of one pair: basis, normal force and closest-point
 * coefficients at xs_n [4][3], sliding from xs_n to xs; outputs D, gradient
 * [12] and PSD-projected Hessian [12][12] over the tuple's slots; info
 * (nullable, 10 doubles): lambda, normal[3], c[4], u[2].
 */
int orc_friction_pair(const int32_t tuple[4], const double* xs_n, const double* xr, const double* xs,
                      const orc_params* prm, const orc_fparams* fp, double* D, double* grad12, double* hess144,
                      double* info);

/* Friction of a list of tuples (per-pair outputs nullable). */
int64_t orc_friction_eval(int32_t V, const double* x_n, const double* x, const double* x_rest, int64_t P,
                          const int32_t* tuples, const orc_params* prm, const orc_fparams* fp, int nthreads,
                          double* energy, double* grad, double* pairE, double* pairG, double* pairH);

/* Contact candidates by brute force (every point-triangle and edge-edge
 * pair of different objects, no shared vertex, boxes within dhat); returns
 * the count and writes at most cap sign-encoded tuples to out (nullable). */
int64_t orc_candidates(int32_t V, const double* x, const int32_t* vobj, int64_t F, const int32_t* tris, int64_t E,
                       const int32_t* edges, double dhat, int32_t* out, int64_t cap);

/* Number of OpenMP threads the scene-level functions use. */
int orc_num_threads(void);

/* Stencil of a tuple: returns the vertex count (2..4, or -1 if malformed);
 * vid[4] receives decoded vertex ids in slot order (-1 unused). */
int orc_stencil(const int32_t tuple[4], int32_t vid[4]);

/*
 * Whole scene.  x, x_rest: [V][3] (x_rest nullable -> x).  Writes the total
 * energy and grad[3V] (overwritten).  Per-pair outputs are optional.
 * Returns the number of degenerate pairs, or -1 on a malformed tuple / index
 * out of range.
 */
int64_t orc_eval(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                 const orc_params* prm, int nthreads, double* energy, double* grad,
                 double* pairE, double* pairG, double* pairH, int32_t* subtype, int32_t* mollified);

/*
 * Assemble A = diag(d_v I3) + sum_k S_k^T H_k S_k as a sorted, duplicate-free
 * list of 3x3 blocks (row-major values).  Every stencil block of every pair
 * is listed (zero or not) and every vertex gets a diagonal block.  Returns
 * the block count; with rows == NULL only counts.  diag nullable (0).
 */
int64_t orc_assemble(int32_t V, int64_t P, const int32_t* tuples, const double* pairH, const double* diag,
                     int32_t* rows, int32_t* cols, double* vals, int64_t cap);

/* y = (diag (x) I3 + sum_k S_k^T H_k S_k) x by local mat-vecs on the dense
 * 12x12 local Hessians (pairH [P][12][12], the leading 3nv x 3nv used),
 * without a global matrix.  Returns -1 on a malformed tuple or a vertex
 * outside [0, V), else 0. */
int orc_matfree(int32_t V, int64_t P, const int32_t* tuples, const double* pairH, const double* diag,
                const double* x, double* y);

/* y = A x for a block list produced by orc_assemble. */
void orc_spmv(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
              const double* x, double* y);

/*
 * Block-Jacobi preconditioned CG on A x = b (textbook PCG) with the 3x3
 * diagonal blocks of A as preconditioner.  x holds x0 on entry.  Stops when
 * ||r||_2 <= rtol ||b||_2 or after maxit iterations.  Returns iterations;
 * *relres receives ||r||/||b||.
 */
int orc_pcg(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
            const double* b, double* x, double rtol, int maxit, double* relres);
/* the same PCG stopped by the paper's termination: r.z <= eps r0.z0 (z the
 * preconditioned residual), checked before each iteration */
int orc_pcg_delta(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
                  const double* b, double* x, double eps, int maxit, double* relres);

#ifdef __cplusplus
}
#endif
#endif
