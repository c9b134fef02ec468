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
    return method == GIPC_PROJ_NUMERIC ? launch_all<true>(st_vid, mult, tr, x, xr, pm, hess, s)
                                       : launch_all<false>(st_vid, mult, tr, x, xr, pm, hess, s);
}

}  // namespace gipc
