/*
 * CPU FP64 oracle for the GIPC barrier hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow reference.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path
 * never does.  It shares no code with the HIP library.
 *
 * Per contact pair it follows the paper's construction step by step:
 *   1. distance as the constrained minimum of Eq. 4 (point-triangle) or
 *      Eq. 5 (edge-edge), found by enumerating the interior stationary point
 *      and every boundary sub-problem, keeping the smallest;
 *   2. gap function g = f^2, f = d / dhat (Eq. 9-11);
 *   3. barrier b(g) of Eq. 24 (or Eq. 12 in test mode);
 *   4. for edge-edge pairs with c = |(x12-x11) x (x22-x21)|^2 below eps_x, the
 *      mollifier of Eq. 25 with J = diag(1, sqrt(c), f) (Eq. 28-29);
 *   5. gradient by the chain rule through J (Eq. 13-14, Eq. 30);
 *   6. inner Hessian in vec(J) space (Eq. 16-17, or the four-term Eq. 31),
 *      built from Kronecker products, evaluated at the filtered Jacobian
 *      (Eq. 23, reading: f -> max(f, d_thr / dhat) inside the inner Hessian);
 *   7. PSD projection of that inner Hessian by cyclic Jacobi rotations with
 *      negative eigenvalues clamped to zero -- the numerical route the paper's
 *      analytic eigensystems (Eq. 18-21, 32-36) replace;
 *   8. contraction with the change-of-basis dJ/dx, whose only non-zero rows
 *      belong to the varying diagonal entries of J (Sec. 4, supplement Sec. 2);
 *      the d^2 J / dx^2 term is dropped as in the paper (Eq. 15, 22).
 * Tuples follow the paper's sign encoding (Sec. 7.2), including the
 * close-to-parallel point-edge / point-point encodings, whose distance is
 * the point-segment / point-point sub-problem of Eq. 5 and whose mollifier
 * is decided from their two edges like an edge-edge pair's.
 * Readings of points the paper leaves open are listed with the project's
 * design notes; every function below cites the passage it implements.
 */
#include "gipc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* interior stationary point used only when the Gram determinant exceeds
 * ORC_TOL times the product of the squared lengths (non-degenerate
 * triangle / non-parallel edges); otherwise the boundary sub-problems
 * decide (reading of Eq. 4-5 for degenerate primitives). */
#define ORC_TOL 1e-10

/* tuple kinds: edge-edge, point-triangle, point-edge, point-point, and the
 * point-edge / point-point pairs cut from a close-to-parallel edge-edge pair
 * (the paper's encodings with a negative second entry, Sec. 7.2) */
enum { K_EE = 0, K_PT = 1, K_PE = 2, K_PP = 3, K_PE_PAR = 4, K_PP_PAR = 5 };

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
/* p*q - r*s within 1.5 ulp of the exact value (Kahan's difference of
 * products: fma recovers the rounding error of r*s).  Used for the cross
 * product that defines the parallelness c of Eq. 25: for edges parallel up to
 * the rounding of their coordinates, the plain formula returns cancellation
 * noise, and the direction of a x b sets grad sqrt(c) (Eq. 28-29). */
static double diff_prod(double p, double q, double r, double s) {
    double w = r * s;
    double err = fma(-r, s, w);
    return fma(p, q, -w) + err;
}
static void cross3_acc(const double* a, const double* b, double* o) {
    o[0] = diff_prod(a[1], b[2], a[2], b[1]);
    o[1] = diff_prod(a[2], b[0], a[0], b[2]);
    o[2] = diff_prod(a[0], b[1], a[1], b[0]);
}

/* ---------------------------------------------------------------- scalars */

/* Eq. 24: b = dhat^4 (1-g)^2 ln^2 g.  Eq. 12: b = -dhat^4 (1-g)^2 ln g.
 * Derivatives in g by the product rule. */
void orc_barrier(double g, double dhat, int eq12, double* b, double* db, double* d2b) {
    const double s = dhat * dhat * dhat * dhat;
    const double L = log(g), u = 1.0 - g;
    /* u^2 and its derivatives: (u^2)' = -2u, (u^2)'' = 2 */
    const double q = u * u, dq = -2.0 * u, d2q = 2.0;
    double h, dh, d2h; /* the log factor */
    if (eq12) { h = -L; dh = -1.0 / g; d2h = 1.0 / (g * g); }
    else { h = L * L; dh = 2.0 * L / g; d2h = (2.0 - 2.0 * L) / (g * g); }
    *b = s * q * h;
    *db = s * (dq * h + q * dh);
    *d2b = s * (d2q * h + 2.0 * dq * dh + q * d2h);
}

/* Eq. 25: e = -c^2/eps^2 + 2c/eps for c < eps, else 1. */
void orc_mollifier(double c, double epsx, double* e, double* de, double* d2e) {
    if (c < epsx) {
        *e = -(c * c) / (epsx * epsx) + 2.0 * c / epsx;
        *de = -2.0 * c / (epsx * epsx) + 2.0 / epsx;
        *d2e = -2.0 / (epsx * epsx);
    } else {
        *e = 1.0; *de = 0.0; *d2e = 0.0;
    }
}

/* ------------------------------------------------------------ eigen solver */

/* Cyclic-by-row Jacobi method for the symmetric eigenproblem (Golub & Van
 * Loan, "Matrix Computations", Sec. 8.5): repeatedly zero each off-diagonal
 * pair with a plane rotation until the off-diagonal norm falls below 1e-15
 * of the Frobenius norm. */
int orc_jacobi_eig(int n, const double* A0, double* lam, double* vec) {
    double A[144];
    if (n > 12) return -1;
    memcpy(A, A0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) vec[i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweep = 0;
    for (; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) off += A[i * n + j] * A[i * n + j];
        if (sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                /* 2x2 symmetric Schur decomposition */
                double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) { /* A <- A J */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* A <- J^T A */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) { /* V <- V J */
                    double vkp = vec[k * n + p], vkq = vec[k * n + q];
                    vec[k * n + p] = c * vkp - s * vkq;
                    vec[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
    return sweep;
}

/* ------------------------------------------------------------- distances */

typedef struct {
    double d2;      /* squared distance */
    double coef[4]; /* closest points: p* - q* = sum_k coef[k] x_k */
    double w[3];    /* p* - q* */
    int sub;        /* ORC_PT / PE / PP / EE */
    int sp[4];      /* slots of the winning sub-problem: PT, EE all four; PE
                       (point, segment end, segment end, -1); PP (point, point, -1, -1) */
} orc_dist;

/* point P against segment AB, parameter clamped to [0, 1] */
static double seg_closest(const double* P, const double* A, const double* B, double* alpha, double* w) {
    double ab[3], ap[3];
    sub3(B, A, ab); sub3(P, A, ap);
    double l2 = dot3(ab, ab);
    double a = l2 > 0.0 ? dot3(ap, ab) / l2 : 0.0;
    if (a < 0.0) a = 0.0;
    if (a > 1.0) a = 1.0;
    for (int d = 0; d < 3; ++d) w[d] = P[d] - (A[d] + a * ab[d]);
    *alpha = a;
    return dot3(w, w);
}

/* keep candidate if strictly closer (first candidate wins ties: the fixed
 * enumeration order is the tie-break) */
static void keep(orc_dist* best, double d2, const double coef[4], const double w[3], int sub, int s0, int s1,
                 int s2, int s3) {
    if (d2 < best->d2) {
        best->d2 = d2;
        memcpy(best->coef, coef, sizeof(double) * 4);
        memcpy(best->w, w, sizeof(double) * 3);
        best->sub = sub;
        best->sp[0] = s0; best->sp[1] = s1; best->sp[2] = s2; best->sp[3] = s3;
    }
}

/* point slot P against segment slots A B with clamped parameter a: the
 * sub-problem kept, point-edge inside the segment, point-point at an end */
static void keep_seg(orc_dist* best, double d2, const double coef[4], const double w[3], double a, int P, int A,
                     int B) {
    if (a > 0.0 && a < 1.0) keep(best, d2, coef, w, ORC_PE, P, A, B, -1);
    else keep(best, d2, coef, w, ORC_PP, P, a <= 0.0 ? A : B, -1, -1);
}

/* Eq. 4: point p = X[0] against triangle X[1], X[2], X[3]. */
static void dist_pt(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    const double *p = X[0], *t0 = X[1], *t1 = X[2], *t2 = X[3];
    double e1[3], e2[3], r[3];
    sub3(t1, t0, e1); sub3(t2, t0, e2); sub3(p, t0, r);
    double a11 = dot3(e1, e1), a12 = dot3(e1, e2), a22 = dot3(e2, e2);
    double b1 = dot3(e1, r), b2 = dot3(e2, r);
    double det = a11 * a22 - a12 * a12;
    if (det > ORC_TOL * a11 * a22) {
        double be1 = (a22 * b1 - a12 * b2) / det, be2 = (a11 * b2 - a12 * b1) / det;
        if (be1 >= 0.0 && be2 >= 0.0 && be1 + be2 <= 1.0) {
            double w[3];
            for (int d = 0; d < 3; ++d) w[d] = p[d] - (t0[d] + be1 * e1[d] + be2 * e2[d]);
            double coef[4] = {1.0, -(1.0 - be1 - be2), -be1, -be2};
            keep(o, dot3(w, w), coef, w, ORC_PT, 0, 1, 2, 3);
        }
    }
    static const int segs[3][2] = {{1, 2}, {2, 3}, {3, 1}};
    for (int s = 0; s < 3; ++s) {
        int ia = segs[s][0], ib = segs[s][1];
        double a, w[3];
        double d2 = seg_closest(p, X[ia], X[ib], &a, w);
        double coef[4] = {1.0, 0.0, 0.0, 0.0};
        coef[ia] = -(1.0 - a); coef[ib] = -a;
        keep_seg(o, d2, coef, w, a, 0, ia, ib);
    }
}

/* point p = X[0] against segment X[1] X[2] (point-edge pair) */
static void dist_pe(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    double a, w[3];
    double d2 = seg_closest(X[0], X[1], X[2], &a, w);
    double coef[4] = {1.0, -(1.0 - a), -a, 0.0};
    keep_seg(o, d2, coef, w, a, 0, 1, 2);
}

static void dist_pp(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    double w[3];
    sub3(X[0], X[1], w);
    double coef[4] = {1.0, -1.0, 0.0, 0.0};
    keep(o, dot3(w, w), coef, w, ORC_PP, 0, 1, -1, -1);
}

/* Eq. 5 restricted to one boundary sub-problem: point X[0] (an endpoint of
 * edge X[0]X[1]) against segment X[2]X[3] -- the point-edge pair of a
 * close-to-parallel edge-edge pair (Sec. 7.2 encodings). */
static void dist_pe_par(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    double a, w[3];
    double d2 = seg_closest(X[0], X[2], X[3], &a, w);
    double coef[4] = {1.0, 0.0, -(1.0 - a), -a};
    keep_seg(o, d2, coef, w, a, 0, 2, 3);
}

/* point X[0] against point X[2] (endpoints of edges X[0]X[1] and X[2]X[3]) */
static void dist_pp_par(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    double w[3];
    sub3(X[0], X[2], w);
    double coef[4] = {1.0, 0.0, -1.0, 0.0};
    keep(o, dot3(w, w), coef, w, ORC_PP, 0, 2, -1, -1);
}

/* Eq. 5: edge X[0]X[1] against edge X[2]X[3]. */
static void dist_ee(const double X[4][3], orc_dist* o) {
    o->d2 = INFINITY; o->sub = ORC_INACTIVE;
    double a[3], b[3], r[3];
    sub3(X[1], X[0], a); sub3(X[3], X[2], b); sub3(X[0], X[2], r);
    double aa = dot3(a, a), bb = dot3(b, b), ab = dot3(a, b), ar = dot3(a, r), br = dot3(b, r);
    double det = aa * bb - ab * ab;
    if (det > ORC_TOL * aa * bb) {
        /* stationarity of |r + g1 a - g2 b|^2 */
        double g1 = (ab * br - bb * ar) / det, g2 = (aa * br - ab * ar) / det;
        if (g1 >= 0.0 && g1 <= 1.0 && g2 >= 0.0 && g2 <= 1.0) {
            double w[3];
            for (int d = 0; d < 3; ++d) w[d] = (X[0][d] + g1 * a[d]) - (X[2][d] + g2 * b[d]);
            double coef[4] = {1.0 - g1, g1, -(1.0 - g2), -g2};
            keep(o, dot3(w, w), coef, w, ORC_EE, 0, 1, 2, 3);
        }
    }
    /* boundary: an endpoint of one edge against the other edge */
    for (int s = 0; s < 4; ++s) {
        double al, w[3], coef[4] = {0, 0, 0, 0}, d2;
        if (s < 2) { /* X[s] against segment X[2]X[3]: w = X[s] - q */
            d2 = seg_closest(X[s], X[2], X[3], &al, w);
            coef[s] = 1.0; coef[2] = -(1.0 - al); coef[3] = -al;
        } else {     /* X[s] against segment X[0]X[1]: w = q - X[s] */
            double wq[3];
            d2 = seg_closest(X[s], X[0], X[1], &al, wq);
            for (int d = 0; d < 3; ++d) w[d] = -wq[d];
            coef[0] = 1.0 - al; coef[1] = al; coef[s] = -1.0;
        }
        if (s < 2) keep_seg(o, d2, coef, w, al, s, 2, 3);
        else keep_seg(o, d2, coef, w, al, s, 0, 1);
    }
}

/* ----------------------------------------------------------- tuple decode */

static int decode(const int32_t t[4], int32_t vid[4], int* kind) {
    vid[0] = vid[1] = vid[2] = vid[3] = -1;
    if (t[0] == INT32_MIN || t[1] == INT32_MIN) return -1;
    if (t[0] >= 0) { /* edge-edge; a negative i1 is the paper's nearly-parallel flag */
        if (t[2] < 0 || t[3] < 0) return -1;
        vid[0] = t[0]; vid[1] = t[1] >= 0 ? t[1] : -t[1] - 1; vid[2] = t[2]; vid[3] = t[3];
        *kind = K_EE;
        return 4;
    }
    vid[0] = -t[0] - 1;
    if (t[1] < 0) { /* close to parallel: [-p, -o, e0, -e1] or [-p, -o, -q, -r] */
        if (t[3] >= 0 || t[2] == INT32_MIN || t[3] == INT32_MIN) return -1;
        vid[1] = -t[1] - 1;
        vid[3] = -t[3] - 1;
        if (t[2] >= 0) { vid[2] = t[2]; *kind = K_PE_PAR; }
        else { vid[2] = -t[2] - 1; *kind = K_PP_PAR; }
        return 4;
    }
    vid[1] = t[1];
    if (t[2] >= 0 && t[3] >= 0) { vid[2] = t[2]; vid[3] = t[3]; *kind = K_PT; return 4; }
    if (t[2] >= 0 && t[3] == -1) { vid[2] = t[2]; *kind = K_PE; return 3; }
    if (t[2] == -1 && t[3] == -1) { *kind = K_PP; return 2; }
    return -1;
}

/* distance of a decoded tuple: its constrained minimum (Eq. 4 / Eq. 5) */
static void dist_of(int kind, const double X[4][3], orc_dist* D) {
    if (kind == K_PT) dist_pt(X, D);
    else if (kind == K_EE) dist_ee(X, D);
    else if (kind == K_PE) dist_pe(X, D);
    else if (kind == K_PE_PAR) dist_pe_par(X, D);
    else if (kind == K_PP_PAR) dist_pp_par(X, D);
    else dist_pp(X, D);
}

/* the kinds built on two edges X[0]X[1], X[2]X[3]: the mollifier applies */
static int edge_family(int kind) { return kind == K_EE || kind == K_PE_PAR || kind == K_PP_PAR; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_stencil(const int32_t tuple[4], int32_t vid[4]) {
    int kind;
    return decode(tuple, vid, &kind);
}

/* ------------------------------------------------------------ one pair */

/* column-major vec index of entry (i, j) of an m x m matrix */
static int vidx(int i, int j, int m) { return i + m * j; }

/* Kronecker-form Hessian of ||J n||^2 with respect to vec(J): 2 (N (x) I_m),
 * N = n n^T (derivative of Eq. 14), added with weight s into H (m^2 x m^2). */
static void add_d2g(double* H, int m, int nsel, double s) {
    const int M = m * m;
    for (int i = 0; i < m; ++i) /* N = e_nsel e_nsel^T: only (nsel, nsel) */
        H[vidx(i, nsel, m) * M + vidx(i, nsel, m)] += 2.0 * s;
}

/* vec(2 J N) for diagonal J (given by its diagonal) and N = e_n e_n^T (Eq. 14) */
static void dg_dJ(const double* Jdiag, int m, int nsel, double* out) {
    for (int i = 0; i < m * m; ++i) out[i] = 0.0;
    /* (J N)_{ij} = J_{i,nsel} delta_{j,nsel}; J diagonal */
    out[vidx(nsel, nsel, m)] = 2.0 * Jdiag[nsel];
}

/* Kx / Px (nullable, [12][12]): the proxy Hessian before projection,
 * kappa D^T H D with the unprojected inner Hessian, and its projection onto
 * the PSD cone computed in x-space by the same Jacobi routine (the
 * traditional route of projecting the 3n x 3n matrix numerically). */
static int pair_local_impl(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm,
                           double* E, double* grad12, double* hess144, int* subtype, int* mollified,
                           double* dist2, double* innerH, double* innerHp, double* dbdJ, int* m_out, double* Kx,
                           double* Px) {
    int32_t vid[4];
    int kind;
    int nv = decode(tuple, vid, &kind);
    *E = 0.0;
    memset(grad12, 0, sizeof(double) * 12);
    memset(hess144, 0, sizeof(double) * 144);
    if (Kx) memset(Kx, 0, sizeof(double) * 144);
    if (Px) memset(Px, 0, sizeof(double) * 144);
    *subtype = ORC_INACTIVE; *mollified = 0; *dist2 = NAN;
    if (m_out) *m_out = 0;
    if (nv < 0) return -1;

    double X[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) X[k][d] = (k < nv) ? xs[3 * k + d] : 0.0;

    orc_dist D;
    dist_of(kind, X, &D);
    *dist2 = D.d2;

    const double dhat = prm->dhat, kappa = prm->kappa;
    if (!(D.d2 > 0.0) || !isfinite(D.d2)) { *subtype = ORC_DEGENERATE; return 1; }
    const double g = D.d2 / (dhat * dhat);
    if (g >= 1.0) return 0;
    *subtype = D.sub;

    const double d = sqrt(D.d2), f = d / dhat;
    /* grad f = grad d^2 / (2 dhat d); grad_k d^2 = 2 coef_k (p* - q*) because
     * the constrained minimiser is stationary in its free parameters */
    double gf[12];
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) gf[3 * k + c] = D.coef[k] * D.w[c] / (dhat * d);

    /* mollifier (Eq. 25-28) for the edge-edge family */
    int moll = 0;
    double cpar = 0.0, e = 1.0, de = 0.0, d2e = 0.0, gsc[12];
    memset(gsc, 0, sizeof(gsc));
    if (edge_family(kind) && prm->mollify) {
        double a[3], b[3], n[3], ar[3], br[3];
        sub3(X[1], X[0], a); sub3(X[3], X[2], b); cross3_acc(a, b, n);
        cpar = dot3(n, n);
        const double* R = xr ? xr : xs;
        sub3(R + 3, R + 0, ar); sub3(R + 9, R + 6, br);
        double epsx = prm->epsx_ratio * dot3(ar, ar) * dot3(br, br);
        if (cpar < epsx) {
            moll = 1;
            orc_mollifier(cpar, epsx, &e, &de, &d2e);
            /* dc = 2 n . (da x b + a x db): partials along each unit axis */
            double dcda[3], dcdb[3];
            for (int j = 0; j < 3; ++j) {
                double ej[3] = {0, 0, 0}, t1[3], t2[3];
                ej[j] = 1.0;
                cross3(ej, b, t1); cross3(a, ej, t2);
                dcda[j] = 2.0 * dot3(n, t1);
                dcdb[j] = 2.0 * dot3(n, t2);
            }
            /* grad sqrt(c) = grad c / (2 sqrt c); zero at c = 0 (sqrt not differentiable there) */
            double sc = sqrt(cpar);
            double k = sc > 0.0 ? 1.0 / (2.0 * sc) : 0.0;
            for (int j = 0; j < 3; ++j) {
                gsc[0 + j] = -dcda[j] * k; gsc[3 + j] = dcda[j] * k;
                gsc[6 + j] = -dcdb[j] * k; gsc[9 + j] = dcdb[j] * k;
            }
        }
    }
    *mollified = moll;

    double b, db, d2b;
    orc_barrier(g, dhat, prm->eq12, &b, &db, &d2b);
    *E = kappa * e * b;

    /* filtered Jacobian for the Hessian (Eq. 23) */
    const double ff = prm->filter ? fmax(f, prm->dthr_ratio) : f;
    const double gfl = ff * ff;
    double bf, dbf, d2bf;
    orc_barrier(gfl, dhat, prm->eq12, &bf, &dbf, &d2bf);

    int m;
    double Jd[3], Jfd[3];
    int ng, nga = -1; /* selected columns: distance normal, mollifier normal */
    if (moll) {
        m = 3;
        Jd[0] = 1.0; Jd[1] = sqrt(cpar); Jd[2] = f;
        Jfd[0] = 1.0; Jfd[1] = sqrt(cpar); Jfd[2] = ff;
        ng = 2; nga = 1;
    } else {
        m = (D.sub == ORC_PE) ? 2 : (D.sub == ORC_PP) ? 1 : 3; /* Eq. 10 */
        for (int i = 0; i < m; ++i) { Jd[i] = 1.0; Jfd[i] = 1.0; }
        Jd[m - 1] = f; Jfd[m - 1] = ff;
        ng = m - 1;
    }
    const int M = m * m;
    if (m_out) *m_out = m;

    /* change of basis dvec(J)/dx: M x 12, rows of the varying diagonal entries */
    double Dm[9][12];
    memset(Dm, 0, sizeof(Dm));
    for (int i = 0; i < 12; ++i) Dm[vidx(ng, ng, m)][i] = gf[i];
    if (moll)
        for (int i = 0; i < 12; ++i) Dm[vidx(nga, nga, m)][i] = gsc[i];

    /* db/dJ (Eq. 13-14, 30), at the actual J */
    double vg[9], va[9], bJ[9];
    dg_dJ(Jd, m, ng, vg);
    for (int i = 0; i < M; ++i) bJ[i] = e * db * vg[i];
    if (moll) {
        dg_dJ(Jd, m, nga, va);
        for (int i = 0; i < M; ++i) bJ[i] += de * b * va[i];
    }
    if (dbdJ) { memset(dbdJ, 0, sizeof(double) * 9); memcpy(dbdJ, bJ, sizeof(double) * M); }
    for (int i = 0; i < 12; ++i) {
        double s = 0.0;
        for (int r = 0; r < M; ++r) s += Dm[r][i] * bJ[r];
        grad12[i] = kappa * s;
    }

    /* inner Hessian at the filtered J (Eq. 16-17; four-term Eq. 31) */
    double H[81];
    memset(H, 0, sizeof(H));
    double vgf[9], vaf[9];
    dg_dJ(Jfd, m, ng, vgf);
    add_d2g(H, m, ng, e * dbf);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) H[i * M + j] += e * d2bf * vgf[i] * vgf[j];
    if (moll) {
        dg_dJ(Jfd, m, nga, vaf);
        add_d2g(H, m, nga, de * bf);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                H[i * M + j] += d2e * bf * vaf[i] * vaf[j];
                H[i * M + j] += de * dbf * (vgf[i] * vaf[j] + vaf[i] * vgf[j]);
            }
    }
    if (innerH) { memset(innerH, 0, sizeof(double) * 81); memcpy(innerH, H, sizeof(double) * M * M); }

    /* numerical PSD projection */
    double lam[9], Q[81], Hp[81];
    orc_jacobi_eig(M, H, lam, Q);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k)
                if (lam[k] > 0.0) s += Q[i * M + k] * lam[k] * Q[j * M + k];
            Hp[i * M + j] = s;
        }
    if (innerHp) { memset(innerHp, 0, sizeof(double) * 81); memcpy(innerHp, Hp, sizeof(double) * M * M); }

    /* H_x = kappa D^T Hp D */
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            double s = 0.0;
            for (int r = 0; r < M; ++r) {
                if (Dm[r][i] == 0.0) continue;
                for (int c = 0; c < M; ++c) s += Dm[r][i] * Hp[r * M + c] * Dm[c][j];
            }
            hess144[i * 12 + j] = kappa * s;
        }

    /* x-space route: project kappa D^T H D itself */
    if (Kx || Px) {
        double K[144], lamx[12], Qx[144];
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) {
                double s = 0.0;
                for (int r = 0; r < M; ++r) {
                    if (Dm[r][i] == 0.0) continue;
                    for (int c = 0; c < M; ++c) s += Dm[r][i] * H[r * M + c] * Dm[c][j];
                }
                K[i * 12 + j] = kappa * s;
            }
        if (Kx) memcpy(Kx, K, sizeof(K));
        if (Px) {
            orc_jacobi_eig(12, K, lamx, Qx);
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < 12; ++k)
                        if (lamx[k] > 0.0) s += Qx[i * 12 + k] * lamx[k] * Qx[j * 12 + k];
                    Px[i * 12 + j] = s;
                }
        }
    }
    return 0;
}

int orc_pair_local(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm,
                   double* E, double* grad12, double* hess144, int* subtype, int* mollified, double* dist2,
                   double* innerH, double* innerHp, double* dbdJ, int* m_out) {
    return pair_local_impl(tuple, xs, xr, prm, E, grad12, hess144, subtype, mollified, dist2, innerH, innerHp,
                           dbdJ, m_out, NULL, NULL);
}

int orc_pair_xproj(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm, double* Kx,
                   double* Px) {
    double E, g[12], h[144], d2;
    int st, mo;
    return pair_local_impl(tuple, xs, xr, prm, &E, g, h, &st, &mo, &d2, NULL, NULL, NULL, NULL, Kx, Px);
}

/* ------------------------------------------------------------ whole scene */

int64_t orc_eval(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                 const orc_params* prm, int nthreads, double* energy, double* grad,
                 double* pairE, double* pairG, double* pairH, int32_t* subtype, int32_t* mollified) {
    /* validate first */
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k) {
            if (vid[k] < 0 || vid[k] >= V) return -1;
            for (int l = 0; l < k; ++l) if (vid[l] == vid[k]) return -1;
        }
    }
    double* lE = pairE ? pairE : (double*)malloc(sizeof(double) * (P > 0 ? P : 1));
    double* lG = pairG ? pairG : (double*)malloc(sizeof(double) * 12 * (P > 0 ? P : 1));
    int64_t ndeg = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static) reduction(+ : ndeg)
    for (int64_t p = 0; p < P; ++p) {
        const int32_t* t = tuples + 4 * p;
        int32_t vid[4];
        int nv = orc_stencil(t, vid);
        double xs[12] = {0}, xr[12] = {0}, H[144];
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) {
                xs[3 * k + d] = x[3 * (int64_t)vid[k] + d];
                xr[3 * k + d] = (x_rest ? x_rest : x)[3 * (int64_t)vid[k] + d];
            }
        int st, mo;
        double d2;
        orc_pair_local(t, xs, xr, prm, &lE[p], lG + 12 * p, pairH ? pairH + 144 * p : H, &st, &mo, &d2,
                       NULL, NULL, NULL, NULL);
        if (st == ORC_DEGENERATE) ndeg += 1;
        if (subtype) subtype[p] = st;
        if (mollified) mollified[p] = mo;
    }
    /* sums in pair order */
    double Es = 0.0;
    memset(grad, 0, sizeof(double) * 3 * (size_t)V);
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        Es += lE[p];
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) grad[3 * (int64_t)vid[k] + d] += lG[12 * p + 3 * k + d];
    }
    *energy = Es;
    if (!pairE) free(lE);
    if (!pairG) free(lG);
    return ndeg;
}

/* Per pair, the x-space projection of the unprojected proxy Hessian
 * (orc_pair_xproj) into pairPx [P][12][12].  Returns -1 on a malformed
 * tuple or a vertex outside [0, V). */
int orc_eval_xproj(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                   const orc_params* prm, int nthreads, double* pairPx) {
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k)
            if (vid[k] < 0 || vid[k] >= V) return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        const int32_t* t = tuples + 4 * p;
        int32_t vid[4];
        int nv = orc_stencil(t, vid);
        double xs[12] = {0}, xr[12] = {0};
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) {
                xs[3 * k + d] = x[3 * (int64_t)vid[k] + d];
                xr[3 * k + d] = (x_rest ? x_rest : x)[3 * (int64_t)vid[k] + d];
            }
        orc_pair_xproj(t, xs, xr, prm, NULL, pairPx + 144 * p);
    }
    return 0;
}

/* ------------------------------------------------- exact local Hessian */

/* The traditional route the paper's Table 1 compares against ("construct,
 * then numerically project"): the exact Hessian of one pair's energy
 * kappa e(c) b(g(x)), g = d^2 / dhat^2, with d^2 the squared distance of the
 * pair's sub-problem (Eq. 4 / Eq. 5 at the active set found at x) -- Eq. 15
 * with the d^2 J / dx^2 term kept, or Eq. 22 without dropping b_d grad^2 d
 * -- projected onto the PSD cone by the cyclic Jacobi routine above.  It is
 * obtained by second-order forward differentiation: every quantity carries
 * its value, gradient and Hessian in the 12 stencil coordinates, and the
 * sub-type's distance is written as a closed form in the coordinates:
 *   point-triangle  ((p - t0) . n)^2 / |n|^2,  n = (t1 - t0) x (t2 - t0)
 *   edge-edge       ((a0 - b0) . n)^2 / |n|^2,  n = (a1 - a0) x (b1 - b0)
 *   point-edge      |p - a|^2 - ((p - a) . (b - a))^2 / |b - a|^2
 *   point-point     |p - q|^2
 * and the parallelness c = |(x1 - x0) x (x3 - x2)|^2 of the mollifier. */

typedef struct {
    double v, g[12], h[144];
} jet;

static void j_const(jet* o, double c) {
    memset(o, 0, sizeof(jet));
    o->v = c;
}
static void j_var(jet* o, double c, int i) {
    j_const(o, c);
    o->g[i] = 1.0;
}
static void j_add(jet* o, const jet* a, const jet* b) {
    o->v = a->v + b->v;
    for (int i = 0; i < 12; ++i) o->g[i] = a->g[i] + b->g[i];
    for (int i = 0; i < 144; ++i) o->h[i] = a->h[i] + b->h[i];
}
static void j_sub(jet* o, const jet* a, const jet* b) {
    o->v = a->v - b->v;
    for (int i = 0; i < 12; ++i) o->g[i] = a->g[i] - b->g[i];
    for (int i = 0; i < 144; ++i) o->h[i] = a->h[i] - b->h[i];
}
/* product rule, to second order */
static void j_mul(jet* o, const jet* a, const jet* b) {
    jet r;
    r.v = a->v * b->v;
    for (int i = 0; i < 12; ++i) r.g[i] = a->g[i] * b->v + a->v * b->g[i];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j)
            r.h[12 * i + j] = a->h[12 * i + j] * b->v + a->v * b->h[12 * i + j] + a->g[i] * b->g[j] +
                              b->g[i] * a->g[j];
    *o = r;
}
/* f(a) with f, f', f'' at a->v: chain rule to second order */
static void j_apply(jet* o, const jet* a, double f, double fp, double fpp) {
    jet r;
    r.v = f;
    for (int i = 0; i < 12; ++i) r.g[i] = fp * a->g[i];
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) r.h[12 * i + j] = fp * a->h[12 * i + j] + fpp * a->g[i] * a->g[j];
    *o = r;
}
static void j_div(jet* o, const jet* a, const jet* b) {
    jet inv;
    const double y = b->v;
    j_apply(&inv, b, 1.0 / y, -1.0 / (y * y), 2.0 / (y * y * y));
    j_mul(o, a, &inv);
}
static void j3_sub(jet* o, const jet* a, const jet* b) {
    for (int d = 0; d < 3; ++d) j_sub(&o[d], &a[d], &b[d]);
}
static void j3_dot(jet* o, const jet* a, const jet* b) {
    jet t;
    j_mul(o, &a[0], &b[0]);
    j_mul(&t, &a[1], &b[1]);
    j_add(o, o, &t);
    j_mul(&t, &a[2], &b[2]);
    j_add(o, o, &t);
}
static void j3_cross(jet* o, const jet* a, const jet* b) {
    jet t, u;
    for (int d = 0; d < 3; ++d) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        j_mul(&t, &a[d1], &b[d2]);
        j_mul(&u, &a[d2], &b[d1]);
        j_sub(&o[d], &t, &u);
    }
}
/* (r . n)^2 / |n|^2 with n = e x f */
static void j_plane_d2(jet* o, const jet* r, const jet* e, const jet* f) {
    jet n[3], rn, nn;
    j3_cross(n, e, f);
    j3_dot(&rn, r, n);
    j3_dot(&nn, n, n);
    j_mul(&rn, &rn, &rn);
    j_div(o, &rn, &nn);
}

/* exact Hessian H and its projection Hp ([12][12] over the stencil slots;
 * nullable) of one pair; returns -1 on a malformed tuple, 0 otherwise
 * (inactive or degenerate pairs give zeros) */
int orc_pair_exact(const int32_t tuple[4], const double* xs, const double* xr, const orc_params* prm, double* H,
                   double* Hp) {
    int32_t vid[4];
    int kind;
    const int nv = decode(tuple, vid, &kind);
    if (H) memset(H, 0, sizeof(double) * 144);
    if (Hp) memset(Hp, 0, sizeof(double) * 144);
    if (nv < 0) return -1;
    double X[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) X[k][d] = (k < nv) ? xs[3 * k + d] : 0.0;
    orc_dist D;
    dist_of(kind, X, &D);
    const double dhat = prm->dhat, kappa = prm->kappa;
    if (!(D.d2 > 0.0) || !isfinite(D.d2)) return 0;
    const double g0 = D.d2 / (dhat * dhat);
    if (g0 >= 1.0) return 0;

    jet x[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) j_var(&x[k][d], X[k][d], 3 * k + d);
    /* squared distance of the winning sub-problem */
    jet d2;
    if (D.sub == ORC_PT || D.sub == ORC_EE) {
        jet r[3], e[3], f[3];
        if (D.sub == ORC_PT) {
            j3_sub(r, x[0], x[1]); j3_sub(e, x[2], x[1]); j3_sub(f, x[3], x[1]);
        } else {
            j3_sub(r, x[0], x[2]); j3_sub(e, x[1], x[0]); j3_sub(f, x[3], x[2]);
        }
        j_plane_d2(&d2, r, e, f);
    } else if (D.sub == ORC_PE) {
        jet r[3], e[3], rr, re, ee, t;
        j3_sub(r, x[D.sp[0]], x[D.sp[1]]);
        j3_sub(e, x[D.sp[2]], x[D.sp[1]]);
        j3_dot(&rr, r, r); j3_dot(&re, r, e); j3_dot(&ee, e, e);
        j_mul(&re, &re, &re);
        j_div(&t, &re, &ee);
        j_sub(&d2, &rr, &t);
    } else {
        jet r[3];
        j3_sub(r, x[D.sp[0]], x[D.sp[1]]);
        j3_dot(&d2, r, r);
    }
    /* barrier of the gap g = d^2 / dhat^2 */
    jet gj, E;
    j_apply(&gj, &d2, d2.v / (dhat * dhat), 1.0 / (dhat * dhat), 0.0);
    double b, db, d2b;
    orc_barrier(gj.v, dhat, prm->eq12, &b, &db, &d2b);
    j_apply(&E, &gj, b, db, d2b);
    /* mollifier of the edge-edge family (Eq. 25) */
    if (edge_family(kind) && prm->mollify) {
        const double* R = xr ? xr : xs;
        double ar[3], br[3];
        sub3(R + 3, R + 0, ar); sub3(R + 9, R + 6, br);
        const double epsx = prm->epsx_ratio * dot3(ar, ar) * dot3(br, br);
        jet a[3], bb[3], n[3], c, ej;
        j3_sub(a, x[1], x[0]); j3_sub(bb, x[3], x[2]);
        j3_cross(n, a, bb);
        j3_dot(&c, n, n);
        if (c.v < epsx) {
            double e, de, d2e;
            orc_mollifier(c.v, epsx, &e, &de, &d2e);
            j_apply(&ej, &c, e, de, d2e);
            j_mul(&E, &E, &ej);
        }
    }
    for (int i = 0; i < 144; ++i) E.h[i] *= kappa;
    /* exactly symmetric (the jets carry both orders of every product) */
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < i; ++j) {
            const double m = 0.5 * (E.h[12 * i + j] + E.h[12 * j + i]);
            E.h[12 * i + j] = E.h[12 * j + i] = m;
        }
    if (H) memcpy(H, E.h, sizeof(double) * 144);
    if (Hp) {
        /* PSD projection of the stencil's 3 nv x 3 nv block by Jacobi */
        const int n = 3 * nv;
        double A[144], lam[12], V[144];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) A[n * i + j] = E.h[12 * i + j];
        orc_jacobi_eig(n, A, lam, V);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k)
                    if (lam[k] > 0.0) acc += V[n * i + k] * lam[k] * V[n * j + k];
                Hp[12 * i + j] = acc;
            }
    }
    return 0;
}

int orc_eval_exact(int32_t V, const double* x, const double* x_rest, int64_t P, const int32_t* tuples,
                   const orc_params* prm, int nthreads, double* pairH, double* pairHp) {
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k)
            if (vid[k] < 0 || vid[k] >= V) return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        const int32_t* t = tuples + 4 * p;
        int32_t vid[4];
        int nv = orc_stencil(t, vid);
        double xs[12] = {0}, xr[12] = {0};
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) {
                xs[3 * k + d] = x[3 * (int64_t)vid[k] + d];
                xr[3 * k + d] = (x_rest ? x_rest : x)[3 * (int64_t)vid[k] + d];
            }
        orc_pair_exact(t, xs, xr, prm, pairH ? pairH + 144 * p : NULL, pairHp ? pairHp + 144 * p : NULL);
    }
    return 0;
}

/* ------------------------------------------------------------------ ACCD */

/* Additive CCD (the line search's step bound, maxFeasibleStepSize of
 * Algorithm 1; the paper adopts the additive CCD of Li et al., Codimensional
 * IPC, 2021, as its Related Work says), restated: the pair moves as
 * x(t) = x + t p.  The common translation is removed from p (the mean over
 * the vertices the distance involves); l_p is the largest |p_i| over the
 * first primitive plus the largest over the second, a bound on how fast the
 * distance can fall.  With d0 the distance at t = 0 and the gap g = s d0:
 *   t = 0, t_l = (1 - s) d0 / l_p
 *   repeat: d = distance at t + t_l; if t > 0 and d < g stop;
 *           t = t + t_l; if t > t_c return t_c; t_l = 0.9 d / l_p
 * and t is returned.  The trial positions are x + (t + t_l) p, formed from
 * x each time.  l_p = 0 (no relative motion) returns t_c; d0 = 0 returns 0.
 * *iters receives the trial steps taken; a search stopped by max_iter
 * returns the t accumulated so far and -1. */
int orc_accd(const int32_t tuple[4], const double* xs, const double* ps, double s, double tc, int max_iter,
             double* toi, int* iters) {
    int32_t vid[4];
    int kind;
    const int nv = decode(tuple, vid, &kind);
    *toi = 0.0;
    if (iters) *iters = 0;
    if (nv < 0) return -2;
    double X[4][3], Pd[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) {
            X[k][d] = k < nv ? xs[3 * k + d] : 0.0;
            Pd[k][d] = k < nv ? ps[3 * k + d] : 0.0;
        }
    /* the two primitives of the kind, as slot lists */
    int first[2], nf, second[3], ns;
    switch (kind) {
        case K_EE: first[0] = 0; first[1] = 1; nf = 2; second[0] = 2; second[1] = 3; ns = 2; break;
        case K_PT: first[0] = 0; nf = 1; second[0] = 1; second[1] = 2; second[2] = 3; ns = 3; break;
        case K_PE: first[0] = 0; nf = 1; second[0] = 1; second[1] = 2; ns = 2; break;
        case K_PP: first[0] = 0; nf = 1; second[0] = 1; ns = 1; break;
        case K_PE_PAR: first[0] = 0; nf = 1; second[0] = 2; second[1] = 3; ns = 2; break;
        default: first[0] = 0; nf = 1; second[0] = 2; ns = 1; break;
    }
    double mean[3] = {0, 0, 0};
    for (int a = 0; a < nf; ++a)
        for (int d = 0; d < 3; ++d) mean[d] += Pd[first[a]][d];
    for (int a = 0; a < ns; ++a)
        for (int d = 0; d < 3; ++d) mean[d] += Pd[second[a]][d];
    for (int d = 0; d < 3; ++d) mean[d] /= (double)(nf + ns);
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) Pd[k][d] -= mean[d];
    double l1 = 0.0, l2 = 0.0;
    for (int a = 0; a < nf; ++a) l1 = fmax(l1, sqrt(dot3(Pd[first[a]], Pd[first[a]])));
    for (int a = 0; a < ns; ++a) l2 = fmax(l2, sqrt(dot3(Pd[second[a]], Pd[second[a]])));
    const double lp = l1 + l2;
    orc_dist D;
    dist_of(kind, X, &D);
    if (!(D.d2 > 0.0) || !isfinite(D.d2)) return 1;   /* touching: no step */
    if (!(lp > 0.0)) { *toi = tc; return 0; }
    const double d0 = sqrt(D.d2), g = s * d0;
    double t = 0.0, tl = (1.0 - s) * d0 / lp;
    for (int it = 1; it <= max_iter; ++it) {
        double Xt[4][3];
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) Xt[k][d] = X[k][d] + (t + tl) * Pd[k][d];
        orc_dist Dt;
        dist_of(kind, Xt, &Dt);
        const double dd = sqrt(Dt.d2);
        if (iters) *iters = it;
        if (t > 0.0 && dd < g) { *toi = t; return 0; }
        t = t + tl;
        if (t > tc) { *toi = tc; return 0; }
        tl = 0.9 * dd / lp;
    }
    *toi = t;
    if (iters) *iters = -1;
    return 0;
}

int64_t orc_accd_scene(int32_t V, const double* x, const double* disp, int64_t P, const int32_t* tuples, double s,
                       double tc, int max_iter, int nthreads, double* toi) {
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k)
            if (vid[k] < 0 || vid[k] >= V) return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t capped = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(+:capped)
    for (int64_t p = 0; p < P; ++p) {
        const int32_t* t = tuples + 4 * p;
        int32_t vid[4];
        int nv = orc_stencil(t, vid);
        double xs[12] = {0}, ps[12] = {0};
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) {
                xs[3 * k + d] = x[3 * (int64_t)vid[k] + d];
                ps[3 * k + d] = disp[3 * (int64_t)vid[k] + d];
            }
        int it = 0;
        orc_accd(t, xs, ps, s, tc, max_iter, toi + p, &it);
        if (it < 0) ++capped;
    }
    return capped;
}

/* ------------------------------------------------------------- friction */

/* f0, f1 = f0' and f1' of the smooth static-to-dynamic transition
 * (supplement Sec. 5; h = dt): f1(y) = -y^2/(eps h)^2 + 2y/(eps h) below
 * eps h, 1 above; f0 its antiderivative with f0(eps h) = eps h. */
void orc_friction_f(double y, double eps_v, double dt, double* f0, double* f1, double* df1) {
    const double s = eps_v * dt;
    if (y < s) {
        *f0 = -y * y * y / (3.0 * s * s) + y * y / s + s / 3.0;
        *f1 = -y * y / (s * s) + 2.0 * y / s;
        *df1 = -2.0 * y / (s * s) + 2.0 / s;
    } else {
        *f0 = y;
        *f1 = 1.0;
        *df1 = 0.0;
    }
}

/* One pair's lagged friction (supplement Sec. 5).  At the previous
 * positions xs_n: the closest-point coefficients c and direction w of the
 * pair's constrained distance, the normal force lambda = kappa e |db/dd|
 * (the distance derivative of the pair's barrier energy, with its
 * mollifier e), and the sliding basis T = c (x) P (12 x 2) with P an
 * orthonormal basis of the plane normal to w.  At the current positions
 * xs: u = T^T (xs - xs_n), D = mu lambda f0(|u|), grad = mu lambda
 * f1(|u|)/|u| T u and the Hessian mu lambda T M T^T with the 2x2
 * M = (f1'|u| - f1)/|u|^3 u u^T + f1/|u| I projected to PSD (Jacobi on the
 * 2x2).  info (nullable, 10): lambda, n[3], c[4], u[2].  Returns -1 on a
 * malformed tuple; pairs inactive or degenerate at xs_n give zeros. */
int orc_friction_pair(const int32_t tuple[4], const double* xs_n, const double* xr, const double* xs,
                      const orc_params* prm, const orc_fparams* fp, double* Dout, double* grad12, double* hess144,
                      double* info) {
    int32_t vid[4];
    int kind;
    int nv = decode(tuple, vid, &kind);
    *Dout = 0.0;
    memset(grad12, 0, sizeof(double) * 12);
    memset(hess144, 0, sizeof(double) * 144);
    if (info) memset(info, 0, sizeof(double) * 10);
    if (nv < 0) return -1;
    double X[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) X[k][d] = (k < nv) ? xs_n[3 * k + d] : 0.0;
    orc_dist Dd;
    dist_of(kind, X, &Dd);
    const double dhat = prm->dhat, kappa = prm->kappa;
    if (!(Dd.d2 > 0.0) || !isfinite(Dd.d2)) return 0;
    const double g = Dd.d2 / (dhat * dhat);
    if (g >= 1.0) return 0;
    const double d = sqrt(Dd.d2);
    double e = 1.0;
    if (edge_family(kind) && prm->mollify) {
        double a[3], b[3], n[3], ar[3], br[3];
        sub3(X[1], X[0], a); sub3(X[3], X[2], b); cross3_acc(a, b, n);
        const double cpar = dot3(n, n);
        const double* R = xr ? xr : xs_n;
        sub3(R + 3, R + 0, ar); sub3(R + 9, R + 6, br);
        const double epsx = prm->epsx_ratio * dot3(ar, ar) * dot3(br, br);
        if (cpar < epsx) {
            double de, d2e;
            orc_mollifier(cpar, epsx, &e, &de, &d2e);
        }
    }
    double b, db, d2b;
    orc_barrier(g, dhat, prm->eq12, &b, &db, &d2b);
    const double lam = kappa * e * fabs(db * 2.0 * d / (dhat * dhat));
    /* normal and an orthonormal basis of its plane */
    double nrm[3] = {Dd.w[0] / d, Dd.w[1] / d, Dd.w[2] / d};
    double ax[3] = {1.0, 0.0, 0.0};
    if (fabs(nrm[0]) > 0.9) { ax[0] = 0.0; ax[1] = 1.0; }
    double p1[3], p2[3];
    const double an = dot3(ax, nrm);
    for (int r = 0; r < 3; ++r) p1[r] = ax[r] - an * nrm[r];
    const double l1 = sqrt(dot3(p1, p1));
    for (int r = 0; r < 3; ++r) p1[r] /= l1;
    cross3(nrm, p1, p2);
    double T[12][2];
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < 3; ++r) {
            T[3 * k + r][0] = Dd.coef[k] * p1[r];
            T[3 * k + r][1] = Dd.coef[k] * p2[r];
        }
    double u[2] = {0.0, 0.0};
    for (int i = 0; i < 12; ++i) {
        const int k = i / 3;
        const double dx = k < nv ? xs[i] - xs_n[i] : 0.0;
        u[0] += T[i][0] * dx;
        u[1] += T[i][1] * dx;
    }
    const double y = sqrt(u[0] * u[0] + u[1] * u[1]);
    double f0, f1, df1;
    orc_friction_f(y, fp->eps_v, fp->dt, &f0, &f1, &df1);
    const double ml = fp->mu * lam;
    *Dout = ml * f0;
    const double s = fp->eps_v * fp->dt;
    /* f1(y)/y and (f1'(y) y - f1(y)) / y^3, in closed form below eps h */
    double f1y, cuu;
    if (y < s) {
        f1y = 2.0 / s - y / (s * s);
        cuu = y > 0.0 ? -1.0 / (s * s * y) : 0.0;
    } else {
        f1y = 1.0 / y;
        cuu = -1.0 / (y * y * y);
    }
    for (int i = 0; i < 12; ++i) grad12[i] = ml * f1y * (T[i][0] * u[0] + T[i][1] * u[1]);
    double M[4] = {cuu * u[0] * u[0] + f1y, cuu * u[0] * u[1], cuu * u[1] * u[0], cuu * u[1] * u[1] + f1y};
    double lm[2], Q[4];
    orc_jacobi_eig(2, M, lm, Q);
    double Mp[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k)
                if (lm[k] > 0.0) acc += Q[i * 2 + k] * lm[k] * Q[j * 2 + k];
            Mp[i * 2 + j] = acc;
        }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
            double acc = 0.0;
            for (int a2 = 0; a2 < 2; ++a2)
                for (int b2 = 0; b2 < 2; ++b2) acc += T[i][a2] * Mp[a2 * 2 + b2] * T[j][b2];
            hess144[i * 12 + j] = ml * acc;
        }
    if (info) {
        info[0] = lam;
        for (int r = 0; r < 3; ++r) info[1 + r] = nrm[r];
        for (int k = 0; k < 4; ++k) info[4 + k] = Dd.coef[k];
        info[8] = u[0]; info[9] = u[1];
    }
    return 0;
}

/* Friction of a whole list: energy and gradient sums in pair order, and per
 * pair D, gradient and Hessian on request (nullable). */
int64_t orc_friction_eval(int32_t V, const double* x_n, const double* x, const double* x_rest, int64_t P,
                          const int32_t* tuples, const orc_params* prm, const orc_fparams* fp, int nthreads,
                          double* energy, double* grad, double* pairE, double* pairG, double* pairH) {
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k)
            if (vid[k] < 0 || vid[k] >= V) return -1;
    }
    double* lE = pairE ? pairE : (double*)malloc(sizeof(double) * (P > 0 ? P : 1));
    double* lG = pairG ? pairG : (double*)malloc(sizeof(double) * 12 * (P > 0 ? P : 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        const int32_t* t = tuples + 4 * p;
        int32_t vid[4];
        int nv = orc_stencil(t, vid);
        double xn[12] = {0}, xc[12] = {0}, xr[12] = {0}, H[144];
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) {
                xn[3 * k + d] = x_n[3 * (int64_t)vid[k] + d];
                xc[3 * k + d] = x[3 * (int64_t)vid[k] + d];
                xr[3 * k + d] = (x_rest ? x_rest : x_n)[3 * (int64_t)vid[k] + d];
            }
        orc_friction_pair(t, xn, xr, xc, prm, fp, &lE[p], lG + 12 * p, pairH ? pairH + 144 * p : H, NULL);
    }
    double Es = 0.0;
    memset(grad, 0, sizeof(double) * 3 * (size_t)V);
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        Es += lE[p];
        for (int k = 0; k < nv; ++k)
            for (int d = 0; d < 3; ++d) grad[3 * (int64_t)vid[k] + d] += lG[12 * p + 3 * k + d];
    }
    *energy = Es;
    if (!pairE) free(lE);
    if (!pairG) free(lG);
    return 0;
}

/* ----------------------------------------------------------- candidates */

/* axis-aligned box of n vertices */
static void cand_box(const double* x, const int32_t* v, int n, double lo[3], double hi[3]) {
    for (int d = 0; d < 3; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) {
            const double c = x[3 * (int64_t)v[k] + d];
            if (c < lo[d]) lo[d] = c;
            if (c > hi[d]) hi[d] = c;
        }
}

/* box a inflated by dhat overlaps box b (closed intervals) */
static int cand_overlap(const double alo[3], const double ahi[3], double dhat, const double blo[3],
                        const double bhi[3]) {
    for (int d = 0; d < 3; ++d)
        if (alo[d] - dhat > bhi[d] || blo[d] > ahi[d] + dhat) return 0;
    return 1;
}

/* Contact candidates by brute force over all point-triangle and edge-edge
 * pairs (the pairs the barrier sum of Eq. 3 ranges over, restricted to
 * those whose bounding boxes come within dhat): a point p and a triangle t
 * of another object (vobj), p not a vertex of t, with p's box inflated by
 * dhat overlapping t's box -> [-(p+1), t0, t1, t2]; edges i < j of
 * different objects sharing no vertex, i's box inflated by dhat overlapping
 * j's -> [a0, a1, b0, b1].  Point-triangle first, in (p, t) order, then
 * edge-edge in (i, j) order.  Returns the count; writes at most cap tuples
 * to out (nullable). */
int64_t orc_candidates(int32_t V, const double* x, const int32_t* vobj, int64_t F, const int32_t* tris, int64_t E,
                       const int32_t* edges, double dhat, int32_t* out, int64_t cap) {
    int64_t n = 0;
    for (int32_t p = 0; p < V; ++p) {
        double plo[3], phi[3];
        cand_box(x, &p, 1, plo, phi);
        for (int64_t f = 0; f < F; ++f) {
            const int32_t* t = tris + 3 * f;
            if (vobj[t[0]] == vobj[p] || t[0] == p || t[1] == p || t[2] == p) continue;
            double tlo[3], thi[3];
            cand_box(x, t, 3, tlo, thi);
            if (!cand_overlap(plo, phi, dhat, tlo, thi)) continue;
            if (out && n < cap) { out[4 * n] = -(p + 1); out[4 * n + 1] = t[0]; out[4 * n + 2] = t[1]; out[4 * n + 3] = t[2]; }
            ++n;
        }
    }
    for (int64_t i = 0; i < E; ++i) {
        const int32_t* a = edges + 2 * i;
        double alo[3], ahi[3];
        cand_box(x, a, 2, alo, ahi);
        for (int64_t j = i + 1; j < E; ++j) {
            const int32_t* b = edges + 2 * j;
            if (vobj[a[0]] == vobj[b[0]] || a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
            double blo[3], bhi[3];
            cand_box(x, b, 2, blo, bhi);
            if (!cand_overlap(alo, ahi, dhat, blo, bhi)) continue;
            if (out && n < cap) { out[4 * n] = a[0]; out[4 * n + 1] = a[1]; out[4 * n + 2] = b[0]; out[4 * n + 3] = b[1]; }
            ++n;
        }
    }
    return n;
}

/* --------------------------------------------------------------- assembly */

typedef struct { int32_t r, c; int64_t seq; } blk_key;

static int cmp_blk(const void* a, const void* b) {
    const blk_key* x = (const blk_key*)a;
    const blk_key* y = (const blk_key*)b;
    if (x->r != y->r) return x->r < y->r ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return (x->seq > y->seq) - (x->seq < y->seq);
}

/* Global matrix as the sum of the local matrices placed by the
 * local-to-global vertex map (supplement Sec. 6, matrix decomposition). */
int64_t orc_assemble(int32_t V, int64_t P, const int32_t* tuples, const double* pairH, const double* diag,
                     int32_t* rows, int32_t* cols, double* vals, int64_t cap) {
    int64_t n = V;
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        n += (int64_t)nv * nv;
    }
    blk_key* keys = (blk_key*)malloc(sizeof(blk_key) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int32_t v = 0; v < V; ++v) { keys[m].r = v; keys[m].c = v; keys[m].seq = -1 - (int64_t)v; ++m; }
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        for (int k = 0; k < nv; ++k)
            for (int l = 0; l < nv; ++l) {
                keys[m].r = vid[k]; keys[m].c = vid[l]; keys[m].seq = p * 16 + k * 4 + l; ++m;
            }
    }
    qsort(keys, (size_t)m, sizeof(blk_key), cmp_blk);
    int64_t nb = 0;
    for (int64_t i = 0; i < m; ++i) {
        int start = (i == 0) || keys[i].r != keys[i - 1].r || keys[i].c != keys[i - 1].c;
        if (start) {
            if (rows && nb < cap) {
                rows[nb] = keys[i].r; cols[nb] = keys[i].c;
                memset(vals + 9 * nb, 0, sizeof(double) * 9);
            }
            ++nb;
        }
        if (!rows || nb - 1 >= cap) continue;
        double* B = vals + 9 * (nb - 1);
        if (keys[i].seq < 0) {
            double dv = diag ? diag[keys[i].r] : 0.0;
            B[0] += dv; B[4] += dv; B[8] += dv;
        } else {
            int64_t p = keys[i].seq / 16;
            int k = (int)((keys[i].seq / 4) % 4), l = (int)(keys[i].seq % 4);
            const double* H = pairH + 144 * p;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) B[3 * a + c] += H[(3 * k + a) * 12 + 3 * l + c];
        }
    }
    free(keys);
    return nb;
}

void orc_spmv(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
              const double* x, double* y) {
    memset(y, 0, sizeof(double) * 3 * (size_t)V);
    for (int64_t i = 0; i < nb; ++i) {
        const double* B = vals + 9 * i;
        const double* xc = x + 3 * (int64_t)cols[i];
        double* yr = y + 3 * (int64_t)rows[i];
        for (int a = 0; a < 3; ++a) yr[a] += B[3 * a] * xc[0] + B[3 * a + 1] * xc[1] + B[3 * a + 2] * xc[2];
    }
}

/* y = (diag (x) I3 + sum_k S_k^T H_k S_k) x without forming the global
 * matrix: each pair gathers its stencil's entries of x, multiplies them by
 * its dense local Hessian and adds the product back at the same vertices
 * (supplement Sec. 6, decomposition of the system mat-vec into local
 * mat-vecs).  Returns -1 on a malformed tuple or a vertex outside [0, V). */
int orc_matfree(int32_t V, int64_t P, const int32_t* tuples, const double* pairH, const double* diag,
                const double* x, double* y) {
    for (int32_t v = 0; v < V; ++v) {
        double dv = diag ? diag[v] : 0.0;
        for (int a = 0; a < 3; ++a) y[3 * (int64_t)v + a] = dv * x[3 * (int64_t)v + a];
    }
    for (int64_t p = 0; p < P; ++p) {
        int32_t vid[4];
        int nv = orc_stencil(tuples + 4 * p, vid);
        if (nv < 0) return -1;
        for (int k = 0; k < nv; ++k)
            if (vid[k] < 0 || vid[k] >= V) return -1;
        double xl[12], yl[12];
        for (int k = 0; k < nv; ++k)
            for (int a = 0; a < 3; ++a) xl[3 * k + a] = x[3 * (int64_t)vid[k] + a];
        const double* H = pairH + 144 * p;
        for (int i = 0; i < 3 * nv; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 3 * nv; ++j) acc += H[12 * i + j] * xl[j];
            yl[i] = acc;
        }
        for (int k = 0; k < nv; ++k)
            for (int a = 0; a < 3; ++a) y[3 * (int64_t)vid[k] + a] += yl[3 * k + a];
    }
    return 0;
}

/* inverse of a 3x3 matrix by cofactors; identity if singular */
static void inv3(const double* A, double* R) {
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(fabs(det) > 0.0)) { memset(R, 0, sizeof(double) * 9); R[0] = R[4] = R[8] = 1.0; return; }
    double id = 1.0 / det;
    R[0] = c00 * id; R[1] = (A[2] * A[7] - A[1] * A[8]) * id; R[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    R[3] = c01 * id; R[4] = (A[0] * A[8] - A[2] * A[6]) * id; R[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    R[6] = c02 * id; R[7] = (A[1] * A[6] - A[0] * A[7]) * id; R[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

static double vdot(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Preconditioned conjugate gradients (Saad, "Iterative Methods for Sparse
 * Linear Systems", Alg. 9.1) with the 3x3 block diagonal as preconditioner,
 * the paper's simple block preconditioner (Sec. 7.2).  Stopping test at the
 * top of each iteration: delta = 0, ||r|| <= tol ||b||; delta = 1, the
 * paper's termination (its PCG in the implementation section), r.z <= tol
 * r0.z0 with z = M^-1 r. */
static int pcg_core(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
                    const double* b, double* x, double tol, int maxit, double* relres, int delta) {
    const int64_t n = 3 * (int64_t)V;
    double* Minv = (double*)calloc((size_t)V * 9, sizeof(double));
    for (int32_t v = 0; v < V; ++v) { Minv[9 * v] = Minv[9 * v + 4] = Minv[9 * v + 8] = 1.0; }
    for (int64_t i = 0; i < nb; ++i)
        if (rows[i] == cols[i]) inv3(vals + 9 * i, Minv + 9 * (int64_t)rows[i]);
    double* r = (double*)malloc(sizeof(double) * n);
    double* z = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    orc_spmv(V, nb, rows, cols, vals, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double bn = sqrt(vdot(n, b, b));
    for (int32_t v = 0; v < V; ++v)
        for (int a = 0; a < 3; ++a) {
            const double* M = Minv + 9 * v;
            z[3 * v + a] = M[3 * a] * r[3 * v] + M[3 * a + 1] * r[3 * v + 1] + M[3 * a + 2] * r[3 * v + 2];
        }
    memcpy(p, z, sizeof(double) * n);
    double rz = vdot(n, r, z);
    const double rz0 = rz;
    int it = 0;
    for (; it < maxit; ++it) {
        if (delta) {
            if (rz <= tol * rz0) break;
        } else {
            double rn = sqrt(vdot(n, r, r));
            if (rn <= tol * bn) break;
        }
        orc_spmv(V, nb, rows, cols, vals, p, q);
        double pq = vdot(n, p, q);
        double alpha = rz / pq;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        for (int32_t v = 0; v < V; ++v)
            for (int a = 0; a < 3; ++a) {
                const double* M = Minv + 9 * v;
                z[3 * v + a] = M[3 * a] * r[3 * v] + M[3 * a + 1] * r[3 * v + 1] + M[3 * a + 2] * r[3 * v + 2];
            }
        double rz2 = vdot(n, r, z);
        double beta = rz2 / rz;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz2;
    }
    *relres = bn > 0.0 ? sqrt(vdot(n, r, r)) / bn : 0.0;
    free(Minv); free(r); free(z); free(p); free(q);
    return it;
}

int orc_pcg(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
            const double* b, double* x, double rtol, int maxit, double* relres) {
    return pcg_core(V, nb, rows, cols, vals, b, x, rtol, maxit, relres, 0);
}

int orc_pcg_delta(int32_t V, int64_t nb, const int32_t* rows, const int32_t* cols, const double* vals,
                  const double* b, double* x, double eps, int maxit, double* relres) {
    return pcg_core(V, nb, rows, cols, vals, b, x, eps, maxit, relres, 1);
}
