// Dense projected proxy Hessians, two ways, for the comparison of Table 1:
// the time to construct a pair's barrier Hessian and project it to PSD.
//
//  analytic: the compact factors of the analytic eigensystems (Eq. 18-21,
//            32-36) expanded into the 3n x 3n matrix;
//  numeric:  the same matrix built with the unprojected inner Hessian,
//            kappa D^T H D, and projected in x-space by cyclic Jacobi
//            rotations (Golub & Van Loan, Sec. 8.5), negative eigenvalues
//            clamped to zero: the traditional route, on matrices of the
//            sizes the paper's table times (12 x 12, 9 x 9, 6 x 6).
// For non-mollified pairs the proxy Hessian is rank one, lambda g g^T, so
// both give max(lambda, 0) g g^T; for mollified pairs the x-space projection
// of the rank-two matrix differs from the inner-space one whenever the
// inner 2x2 block is indefinite.
//
// One lane per staged pair; the symmetric matrix (upper triangle) and the
// accumulated rotations live in registers, every index is a compile-time
// constant after unrolling.  Output [Ps][12][12] row-major, FP64, the
// leading 3n x 3n filled and the rest zero, times the multiplicity.
#include "internal.hpp"

namespace gipc {
namespace {

// index of (i, j), i <= j, in the packed upper triangle of an N x N matrix
template <int N>
__device__ constexpr int ut(int i, int j) {
    return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

constexpr int kMaxSweeps = 20;

// A (packed upper, N(N+1)/2) <- its projection onto the PSD cone
template <int N>
__device__ __forceinline__ void jacobi_project(double* A) {
    double Q[N * N];
#pragma unroll
    for (int i = 0; i < N * N; ++i) Q[i] = (i % (N + 1) == 0) ? 1.0 : 0.0;
    double fro2 = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j) fro2 += (i == j ? 1.0 : 2.0) * A[ut<N>(i, j)] * A[ut<N>(i, j)];
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        double off2 = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = i + 1; j < N; ++j) off2 += A[ut<N>(i, j)] * A[ut<N>(i, j)];
        if (!(off2 > 1e-30 * fro2)) break;
#pragma unroll
        for (int p = 0; p < N - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < N; ++q) {
                // 2x2 symmetric Schur decomposition zeroing A(p, q)
                const double apq = A[ut<N>(p, q)], app = A[ut<N>(p, p)], aqq = A[ut<N>(q, q)];
                const bool rot = apq != 0.0;
                const double tau = (aqq - app) / (rot ? 2.0 * apq : 1.0);
                const double t = rot ? (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau)) : 0.0;
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (k == p || k == q) continue;
                    const double akp = A[ut<N>(k, p)], akq = A[ut<N>(k, q)];
                    A[ut<N>(k, p)] = c * akp - s * akq;
                    A[ut<N>(k, q)] = s * akp + c * akq;
                }
                A[ut<N>(p, p)] = app - t * apq;
                A[ut<N>(q, q)] = aqq + t * apq;
                A[ut<N>(p, q)] = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const double qkp = Q[k * N + p], qkq = Q[k * N + q];
                    Q[k * N + p] = c * qkp - s * qkq;
                    Q[k * N + q] = s * qkp + c * qkq;
                }
            }
        }
    }
    double lam[N];
#pragma unroll
    for (int k = 0; k < N; ++k) lam[k] = fmax(A[ut<N>(k, k)], 0.0);
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a; b < N; ++b) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) s += Q[a * N + k] * lam[k] * Q[b * N + k];
            A[ut<N>(a, b)] = s;
        }
}

template <int NV, bool NUMERIC>
__global__ void __launch_bounds__(64) k_proxy_dense(const int4* __restrict__ st_vid, const int32_t* __restrict__ mult,
                                                    TypeRanges tr, int64_t k0, int64_t k1,
                                                    const double* __restrict__ X, const double* __restrict__ XR,
                                                    DevParams pm, double* __restrict__ hess) {
    constexpr int N = 3 * NV;
    const int64_t k = k0 + (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (k >= k1) return;
    const int ft = type_of(k, tr);
    const int4 v4 = st_vid[k];
    const int v[4] = {v4.x, v4.y, v4.z, v4.w};
    PairFactors o;
    eval_typed(ft, v, X, XR, pm, o);
    const double w = mult ? (double)mult[k] : 1.0;
    double gf[N], gs[N];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const d3 g = o.c[i] * o.wt;
        const d3 h = i < 2 ? o.u : o.v;
        const double sg = (i & 1) ? 1.0 : -1.0;
        gf[3 * i] = g.x; gf[3 * i + 1] = g.y; gf[3 * i + 2] = g.z;
        gs[3 * i] = sg * h.x; gs[3 * i + 1] = sg * h.y; gs[3 * i + 2] = sg * h.z;
    }
    const double h22 = w * (NUMERIC ? o.H22r : o.P22), h12 = w * (NUMERIC ? o.H12r : o.P12),
                 h11 = w * (NUMERIC ? o.H11r : o.P11);
    double A[N * (N + 1) / 2];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a; b < N; ++b)
            A[ut<N>(a, b)] = h22 * gf[a] * gf[b] + h12 * (gf[a] * gs[b] + gs[a] * gf[b]) + h11 * gs[a] * gs[b];
    if (NUMERIC) jacobi_project<N>(A);
    double* out = hess + 144 * k;
#pragma unroll
    for (int a = 0; a < 12; ++a)
#pragma unroll
        for (int b = 0; b < 12; ++b) out[12 * a + b] = (a < N && b < N) ? A[ut<N>(a, b)] : 0.0;
}

// ------------------------------------------------------------------------
// The exact local Hessian, projected numerically: the traditional route of
// Table 1 ("construct, then project"), on the matrix IPC builds -- Eq. 15
// with the d^2 J / dx^2 term, equivalently Eq. 22 without dropping
// b_d grad^2 d -- for the pair's energy kappa m e(c) b(g), g = d^2 / dhat^2:
//   H = a G G^T + b2 Hd + g2 (C G^T + G C^T) + d2c Hc + e2 C C^T
// with G = grad d^2, Hd = grad^2 d^2, C = grad c, Hc = grad^2 c and
//   a = k e b'' / dhat^4, b2 = k e b' / dhat^2, g2 = k e' b' / dhat^2,
//   d2c = k e' b, e2 = k e'' b   (k = kappa m; e = 1, e' = e'' = 0 unless
//   the mollifier of Eq. 25 applies).
// The distance is the pair's sub-problem, d^2 = min over its free
// parameters beta of |w(x, beta)|^2 with w = sum_i c_i(beta) x_i affine in
// beta; at the minimiser (Danskin; implicit differentiation of the
// stationarity condition):
//   Hd = 2 (c c^T) (x) I3 - 2 Z (T^T T)^-1 Z^T,
//   T = [dw/dbeta_m] (3 x m),  Z = [z_m],  (z_m)_i = (dc_i/dbeta_m) w + c_i t_m,
// m = 2 (point-triangle, edge-edge), 1 (point-edge), 0 (point-point).  With
// a = x1 - x0, b = x3 - x2 and n = a x b, c = |n|^2 has
//   grad_a c = 2 b x n,  grad_b c = 2 n x a,
//   d2c/da2 = 2 (|b|^2 I - b b^T),  d2c/db2 = 2 (|a|^2 I - a a^T),
//   d2c/da db = 4 a b^T - 2 b a^T - 2 (a.b) I.
// Every term is invariant under rigid translations, so H vanishes on them:
// the kernel builds H on the orthogonal complement (Helmert basis of the
// stencil, Q = Hm (x) I3, size 3n - 3), projects that matrix by the cyclic
// Jacobi rotations above (negative eigenvalues clamped) and writes
// Q^T P Q.  The translation block it skips is zero; the projection is the
// one of the whole 3n x 3n matrix.

// Helmert row k of an n-point stencil: (1, .., 1, -(k+1), 0, ..) over
// sqrt((k+1)(k+2)), orthogonal to (1, .., 1)
__device__ constexpr double helm(int k, int i) {
    const double inv = k == 0 ? 0.70710678118654752440 : (k == 1 ? 0.40824829046386301637 : 0.28867513459481288225);
    return i <= k ? inv : (i == k + 1 ? -(k + 1) * inv : 0.0);
}

// Cyclic Jacobi on the packed symmetric M x M matrix A, as jacobi_project,
// with the accumulated rotations split over L lanes: every lane of a pair
// rotates the whole of A (the same arithmetic, so the same bits and the same
// sweep decisions) and its own R rows of V (rows h R .. h R + R - 1; rows past
// M are padding).  On return A holds the eigenvalues on its diagonal.
template <int M, int L>
__device__ __forceinline__ void jacobi_split(double* A, double (*Vl)[M], int h) {
    constexpr int R = (M + L - 1) / L;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) Vl[r][c] = (h * R + r == c) ? 1.0 : 0.0;
    double fro2 = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = i; j < M; ++j) fro2 += (i == j ? 1.0 : 2.0) * A[ut<M>(i, j)] * A[ut<M>(i, j)];
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        double off2 = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = i + 1; j < M; ++j) off2 += A[ut<M>(i, j)] * A[ut<M>(i, j)];
        if (!(off2 > 1e-30 * fro2)) break;
#pragma unroll
        for (int p = 0; p < M - 1; ++p) {
#pragma unroll
            for (int q = p + 1; q < M; ++q) {
                const double apq = A[ut<M>(p, q)], app = A[ut<M>(p, p)], aqq = A[ut<M>(q, q)];
                const bool rot = apq != 0.0;
                const double tau = (aqq - app) / (rot ? 2.0 * apq : 1.0);
                const double t = rot ? (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau)) : 0.0;
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    if (k == p || k == q) continue;
                    const double akp = A[ut<M>(k, p)], akq = A[ut<M>(k, q)];
                    A[ut<M>(k, p)] = c * akp - s * akq;
                    A[ut<M>(k, q)] = s * akp + c * akq;
                }
                A[ut<M>(p, p)] = app - t * apq;
                A[ut<M>(q, q)] = aqq + t * apq;
                A[ut<M>(p, q)] = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double vp = Vl[r][p], vq = Vl[r][q];
                    Vl[r][p] = c * vp - s * vq;
                    Vl[r][q] = s * vp + c * vq;
                }
            }
        }
    }
}

template <int NV>
__global__ void __launch_bounds__(64) k_exact_dense(const int4* __restrict__ st_vid, const int32_t* __restrict__ mult,
                                                    TypeRanges tr, int64_t k0, int64_t k1,
                                                    const double* __restrict__ X, const double* __restrict__ XR,
                                                    DevParams pm, double* __restrict__ hess) {
    constexpr int NK = NV - 1, M = 3 * NK;
    constexpr int L = NV == 4 ? 2 : 1;   // lanes per pair (splitting the rotations of the 9 x 9 case)
    const int64_t k = k0 + ((int64_t)blockIdx.x * 64 + threadIdx.x) / L;
    const int h = (int)(threadIdx.x % L);
    if (k >= k1) return;
    const int ft = type_of(k, tr);
    const int4 v4 = st_vid[k];
    const int vv[4] = {v4.x, v4.y, v4.z, v4.w};
    d3 x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = i < NV ? ld3(X, vv[i]) : mk(0, 0, 0);
    // the sub-problem: coefficients c, dc / dbeta (Cp), dw / dbeta (t), m
    double c[4] = {0, 0, 0, 0}, Cp[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    d3 t[2] = {mk(0, 0, 0), mk(0, 0, 0)};
    int m = 0;
    // (slot indices below are compile-time constants in every branch, so the
    // small arrays stay in registers)
    if (ft == FT_PP) {
        c[0] = 1.0; c[1] = -1.0;
    } else if (ft == FT_PPM) {
        c[0] = 1.0; c[2] = -1.0;
    } else if (ft == FT_PE) {
        const d3 e = x[2] - x[1], r = x[0] - x[1];
        const double al = dot(r, e) / dot(e, e);
        c[0] = 1.0; c[1] = -(1.0 - al); c[2] = -al;
        Cp[0][1] = 1.0; Cp[0][2] = -1.0;
        t[0] = x[1] - x[2];
        m = 1;
    } else if (ft == FT_PEM) {
        const d3 e = x[3] - x[2], r = x[0] - x[2];
        const double al = dot(r, e) / dot(e, e);
        c[0] = 1.0; c[2] = -(1.0 - al); c[3] = -al;
        Cp[0][2] = 1.0; Cp[0][3] = -1.0;
        t[0] = x[2] - x[3];
        m = 1;
    } else if (ft == FT_PT) {
        const d3 e1 = x[2] - x[1], e2 = x[3] - x[1], r = x[0] - x[1];
        const d3 n = cross(e1, e2);
        const double nn = dot(n, n), a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
        const double b1 = dot(e1, r), b2 = dot(e2, r);
        const double be1 = (a22 * b1 - a12 * b2) / nn, be2 = (a11 * b2 - a12 * b1) / nn;
        c[0] = 1.0; c[1] = -(1.0 - be1 - be2); c[2] = -be1; c[3] = -be2;
        Cp[0][1] = 1.0; Cp[0][2] = -1.0;
        Cp[1][1] = 1.0; Cp[1][3] = -1.0;
        t[0] = x[1] - x[2]; t[1] = x[1] - x[3];
        m = 2;
    } else {  // edge-edge
        const d3 a = x[1] - x[0], b = x[3] - x[2], r = x[0] - x[2];
        const d3 n = cross(a, b);
        const double cc = dot(n, n), aa = dot(a, a), bb = dot(b, b), ab = dot(a, b), ar = dot(a, r), br = dot(b, r);
        const double g1 = (ab * br - bb * ar) / cc, g2 = (aa * br - ab * ar) / cc;
        c[0] = 1.0 - g1; c[1] = g1; c[2] = -(1.0 - g2); c[3] = -g2;
        Cp[0][0] = -1.0; Cp[0][1] = 1.0;
        Cp[1][2] = 1.0; Cp[1][3] = -1.0;
        t[0] = a; t[1] = x[2] - x[3];
        m = 2;
    }
    d3 w = mk(0, 0, 0);
#pragma unroll
    for (int i = 0; i < NV; ++i) w = w + c[i] * x[i];
    double dhat, kappa;
    scene_params(pm, vv[0], dhat, kappa);
    const double d2 = dot(w, w);
    double* out = hess + 144 * k;
    if (!(d2 > 0.0) || !(d2 < dhat * dhat)) {
        for (int i = h; i < 144; i += L) out[i] = 0.0;
        return;
    }
    const double km = kappa * (mult ? (double)mult[k] : 1.0);
    double b, db, d2b;
    barrier(d2 / (dhat * dhat), dhat, pm.eq12, b, db, d2b);
    // mollifier of the edge-edge family
    double e = 1.0, de = 0.0, d2e = 0.0;
    d3 A = mk(0, 0, 0), B = mk(0, 0, 0), nAB = mk(0, 0, 0);
    bool moll = false;
    if (NV == 4 && ft >= FT_EEM && pm.mollify) {
        A = x[1] - x[0];
        B = x[3] - x[2];
        nAB = cross_acc(A, B);
        const double cpar = dot(nAB, nAB);
        const double ex = eps_x(XR, vv[0], vv[1], vv[2], vv[3], pm.epsx_ratio);
        if (cpar < ex) {
            moll = true;
            const double iex = 1.0 / ex;
            e = cpar * iex * (2.0 - cpar * iex);
            de = 2.0 * iex * (1.0 - cpar * iex);
            d2e = -2.0 * iex * iex;
        }
    }
    const double ih2 = 1.0 / (dhat * dhat);
    const double sa = km * e * d2b * ih2 * ih2, sb = km * e * db * ih2, sg = km * de * db * ih2, sd = km * de * b,
                 se = km * d2e * b;
    // vectors in the translation-free basis: component (k, a) at 3k + a
    double qG[M], qz[2][M], qC[M], hc[NK], ha[NK], hb[NK];
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
        double sc = 0.0;
        d3 gk = mk(0, 0, 0), z0 = mk(0, 0, 0), z1 = mk(0, 0, 0);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double h = helm(kk, i);
            sc += h * c[i];
            gk = gk + (2.0 * h * c[i]) * w;
            z0 = z0 + h * (Cp[0][i] * w + c[i] * t[0]);
            z1 = z1 + h * (Cp[1][i] * w + c[i] * t[1]);
        }
        hc[kk] = sc;
        qG[3 * kk] = gk.x; qG[3 * kk + 1] = gk.y; qG[3 * kk + 2] = gk.z;
        qz[0][3 * kk] = z0.x; qz[0][3 * kk + 1] = z0.y; qz[0][3 * kk + 2] = z0.z;
        qz[1][3 * kk] = z1.x; qz[1][3 * kk + 1] = z1.y; qz[1][3 * kk + 2] = z1.z;
        // grad c over the stencil is (-gA, gA, -gB, gB): its Helmert coordinates
        ha[kk] = NV == 4 ? helm(kk, 1) - helm(kk, 0) : 0.0;
        hb[kk] = NV == 4 ? helm(kk, 3) - helm(kk, 2) : 0.0;
    }
    const d3 gA = 2.0 * cross(B, nAB), gB = 2.0 * cross(nAB, A);
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
        const d3 q = ha[kk] * gA + hb[kk] * gB;
        qC[3 * kk] = q.x; qC[3 * kk + 1] = q.y; qC[3 * kk + 2] = q.z;
    }
    // (T^T T)^-1, m <= 2
    double i00 = 0.0, i01 = 0.0, i11 = 0.0;
    if (m == 1) {
        i00 = 1.0 / dot(t[0], t[0]);
    } else if (m == 2) {
        const double m00 = dot(t[0], t[0]), m01 = dot(t[0], t[1]), m11 = dot(t[1], t[1]);
        const double id = 1.0 / (m00 * m11 - m01 * m01);
        i00 = m11 * id; i01 = -m01 * id; i11 = m00 * id;
    }
    const double aa = dot(A, A), bb = dot(B, B), ab = dot(A, B);
    const double Av[3] = {A.x, A.y, A.z}, Bv[3] = {B.x, B.y, B.z};
    double H[M * (M + 1) / 2];
#pragma unroll
    for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = p; q < M; ++q) {
            const int kp = p / 3, ap = p % 3, kq = q / 3, aq = q % 3;
            double hd = (ap == aq ? 2.0 * hc[kp] * hc[kq] : 0.0) -
                        2.0 * (qz[0][p] * (i00 * qz[0][q] + i01 * qz[1][q]) +
                               qz[1][p] * (i01 * qz[0][q] + i11 * qz[1][q]));
            double v = sa * qG[p] * qG[q] + sb * hd;
            if (moll) {
                const double del = ap == aq ? 1.0 : 0.0;
                const double kaa = 2.0 * (bb * del - Bv[ap] * Bv[aq]);
                const double kbb = 2.0 * (aa * del - Av[ap] * Av[aq]);
                const double kab = 4.0 * Av[ap] * Bv[aq] - 2.0 * Bv[ap] * Av[aq] - 2.0 * ab * del;
                const double kba = 4.0 * Av[aq] * Bv[ap] - 2.0 * Bv[aq] * Av[ap] - 2.0 * ab * del;
                const double hcc = ha[kp] * ha[kq] * kaa + ha[kp] * hb[kq] * kab + hb[kp] * ha[kq] * kba +
                                   hb[kp] * hb[kq] * kbb;
                v += sg * (qC[p] * qG[q] + qG[p] * qC[q]) + sd * hcc + se * qC[p] * qC[q];
            }
            H[ut<M>(p, q)] = v;
        }
    constexpr int R = (M + L - 1) / L;
    double Vl[R][M];
    jacobi_split<M, L>(H, Vl, h);
    double lam[M];
#pragma unroll
    for (int j = 0; j < M; ++j) lam[j] = fmax(H[ut<M>(j, j)], 0.0);
    // P' = V diag(lam+) V^T, packed into H: lane h holds rows h R .. h R + R
    // - 1 of V; it forms P'(r, s) for its rows r against its own rows s and,
    // one row at a time, the partner's rows, then the lanes swap the entries
    // each formed, so both hold all of P'
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int r2 = 0; r2 < R; ++r2) {
            // own rows: (h R + r, h R + r2)
            double acc = 0.0;
#pragma unroll
            for (int mm = 0; mm < M; ++mm) acc += Vl[r][mm] * lam[mm] * Vl[r2][mm];
            if (L == 1) {
                if (r <= r2 && r2 < M) H[ut<M>(r, r2)] = acc;
            } else {
                const double accp = __shfl_xor(acc, 1, 64);  // the partner's (h' R + r, h' R + r2)
                const int i0 = r, j0 = r2, i1 = R + r, j1 = R + r2;   // lane 0's and lane 1's blocks
                const double v0 = h == 0 ? acc : accp, v1 = h == 0 ? accp : acc;
                if (i0 <= j0 && j0 < M) H[ut<M>(i0, j0)] = v0;
                if (i1 <= j1 && j1 < M) H[ut<M>(i1, j1)] = v1;
            }
        }
    if (L > 1) {
        // mixed blocks (lane 0's rows against lane 1's rows): lane 0 forms
        // row r against the partner's row r2, received one at a time
#pragma unroll
        for (int r2 = 0; r2 < R; ++r2) {
            double vs[M];
#pragma unroll
            for (int mm = 0; mm < M; ++mm) vs[mm] = __shfl_xor(Vl[r2][mm], 1, 64);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int mm = 0; mm < M; ++mm) acc += Vl[r][mm] * lam[mm] * vs[mm];
                // lane 0: (r, R + r2); lane 1: (R + r, r2), the transpose
                const double accp = __shfl_xor(acc, 1, 64);
                const double v = h == 0 ? acc : accp;   // entry (r, R + r2) from lane 0
                if (R + r2 < M) H[ut<M>(r, R + r2)] = v;
            }
        }
    }
    // x-space rows of P = Q^T P' Q that this lane writes: vertices
    // i = h NV / L .. (h + 1) NV / L - 1 of the stencil
    constexpr int NI = NV / L;
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
        const int i = h * NI + ii;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double* row = out + 12 * (3 * i + a);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int bq = 0; bq < 3; ++bq) {
                    double v = 0.0;
                    if (j < NV) {
#pragma unroll
                        for (int ka = 0; ka < NK; ++ka) {
                            const double hi = helm(ka, i);
#pragma unroll
                            for (int kb = 0; kb < NK; ++kb)
                                v += hi * helm(kb, j) * H[ut<M>(3 * ka + a, 3 * kb + bq)];
                        }
                    }
                    row[3 * j + bq] = v;
                }
        }
    }
    // rows of stencil slots the pair does not use
    for (int i = NV + h; i < 4; i += L)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int j = 0; j < 12; ++j) out[12 * (3 * i + a) + j] = 0.0;
}

template <int NV>
hipError_t launch_exact_range(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, int64_t k0, int64_t k1,
                              const double* x, const double* xr, const DevParams& pm, double* hess, hipStream_t s) {
    if (k1 <= k0) return hipSuccess;
    constexpr int L = NV == 4 ? 2 : 1;
    k_exact_dense<NV><<<(unsigned)(((k1 - k0) * L + 63) / 64), 64, 0, s>>>(st_vid, mult, tr, k0, k1, x, xr, pm,
                                                                          hess);
    return hipGetLastError();
}

hipError_t launch_exact_all(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, const double* x,
                            const double* xr, const DevParams& pm, double* hess, hipStream_t s) {
    hipError_t e;
    if ((e = launch_exact_range<4>(st_vid, mult, tr, tr.off[FT_PT], tr.off[FT_PT + 1], x, xr, pm, hess, s))) return e;
    if ((e = launch_exact_range<3>(st_vid, mult, tr, tr.off[FT_PE], tr.off[FT_PE + 1], x, xr, pm, hess, s))) return e;
    if ((e = launch_exact_range<2>(st_vid, mult, tr, tr.off[FT_PP], tr.off[FT_PP + 1], x, xr, pm, hess, s))) return e;
    return launch_exact_range<4>(st_vid, mult, tr, tr.off[FT_EE], tr.off[8], x, xr, pm, hess, s);
}

template <int NV, bool NUMERIC>
hipError_t launch_range(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, int64_t k0, int64_t k1,
                        const double* x, const double* xr, const DevParams& pm, double* hess, hipStream_t s) {
    if (k1 <= k0) return hipSuccess;
    k_proxy_dense<NV, NUMERIC><<<(unsigned)((k1 - k0 + 63) / 64), 64, 0, s>>>(st_vid, mult, tr, k0, k1, x, xr, pm,
                                                                              hess);
    return hipGetLastError();
}

template <bool NUMERIC>
hipError_t launch_all(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, const double* x,
                      const double* xr, const DevParams& pm, double* hess, hipStream_t s) {
    hipError_t e;
    // staged order: PT (4 vertices), PE (3), PP (2), then the edge-edge family (4)
    if ((e = launch_range<4, NUMERIC>(st_vid, mult, tr, tr.off[FT_PT], tr.off[FT_PT + 1], x, xr, pm, hess, s)))
        return e;
    if ((e = launch_range<3, NUMERIC>(st_vid, mult, tr, tr.off[FT_PE], tr.off[FT_PE + 1], x, xr, pm, hess, s)))
        return e;
    if ((e = launch_range<2, NUMERIC>(st_vid, mult, tr, tr.off[FT_PP], tr.off[FT_PP + 1], x, xr, pm, hess, s)))
        return e;
    return launch_range<4, NUMERIC>(st_vid, mult, tr, tr.off[FT_EE], tr.off[8], x, xr, pm, hess, s);
}

}  // namespace

hipError_t launch_proxy_dense(int method, const int4* st_vid, const int32_t* mult, const TypeRanges& tr,
                              const double* x, const double* xr, const DevParams& pm, double* hess, hipStream_t s) {
    if (method == GIPC_PROJ_EXACT) return launch_exact_all(st_vid, mult, tr, x, xr, pm, hess, s);
    return method == GIPC_PROJ_NUMERIC ? launch_all<true>(st_vid, mult, tr, x, xr, pm, hess, s)
                                       : launch_all<false>(st_vid, mult, tr, x, xr, pm, hess, s);
}

}  // namespace gipc
