// Lagged friction (supplement Sec. 5) on the staged contact pairs.
//
// Lag (once per time step, at the previous positions x^n): per pair the
// closest-point coefficients c of its constrained distance, the contact
// normal n = w / |w|, the normal force lambda = kappa e |db/dd| (the
// distance derivative of the pair's barrier energy, with its mollifier)
// times mu and the multiplicity, and the anchor a = P sum_i c_i x_i^n with
// P = I - n n^T.  The sliding basis of the paper is T = c (x) B with B an
// orthonormal basis of n's plane, so u = T^T (x - x^n) has the length of
//   t = P sum_i c_i x_i - a,
// and T M T^T = (c c^T) (x) (B M B^T): every quantity below is written with
// t and P, which makes it independent of how B is chosen.
//
// Eval (per Newton iterate x): per pair
//   D = mu lambda f0(|t|),   grad_i = mu lambda f1(|t|)/|t| c_i t,
//   S = mu lambda [ max(f1'(|t|), 0) t^ t^T + max(f1(|t|)/|t|, 0) (P - t^ t^T) ],
// the eigen-decomposition of the 2x2 M (eigenvalue f1' along u, f1/|u|
// across it) clamped to PSD; the Hessian block (i, j) is c_i c_j S.  A row
// pass then gathers the gradient, per-vertex energy shares and, on request,
// adds c_i c_j S to every BSR block, each block summing its contribution
// list in the order of the symbolic phase.
#include "internal.hpp"

namespace gipc {
namespace {

constexpr int kFrLanes = 16;

// lag record [c1, c2, nx, ny, nz, mu lambda m, ax, ay, az]
__global__ void __launch_bounds__(kBlock) k_fric_lag(const int4* __restrict__ st_vid,
                                                     const int32_t* __restrict__ mult, TypeRanges tr,
                                                     const double* __restrict__ X, const double* __restrict__ XR,
                                                     DevParams pm, double mu, double* __restrict__ lag) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tr.off[8]) return;
    const int ft = type_of(k, tr);
    const int4 v4 = st_vid[k];
    const int v[4] = {v4.x, v4.y, v4.z, v4.w};
    PairFactors o;
    eval_typed(ft, v, X, XR, pm, o);
    double dhat, kappa;
    scene_params(pm, v[0], dhat, kappa);
    const double w = mult ? (double)mult[k] : 1.0;
    // dE/dd = a2 / dhat (a2 is the derivative along grad f, f = d / dhat)
    const double ml = mu * w * fabs(o.a2) / dhat;
    const double nw = sqrt(dot(o.wt, o.wt));
    const d3 n = nw > 0.0 ? (1.0 / nw) * o.wt : mk(0, 0, 0);
    const int nv = ft_nverts(ft);
    d3 s = mk(0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i < nv) s = s + o.c[i] * ld3(X, v[i]);
    const d3 a = s - dot(n, s) * n;
    double* r = lag + 9 * k;
    r[0] = o.c[1]; r[1] = o.c[2];
    r[2] = n.x; r[3] = n.y; r[4] = n.z;
    r[5] = ml;
    r[6] = a.x; r[7] = a.y; r[8] = a.z;
}

// friction record [D, gx, gy, gz, S00, S01, S02, S11, S12, S22]
__global__ void __launch_bounds__(kBlock) k_fric_pair(const int4* __restrict__ st_vid, TypeRanges tr,
                                                      const double* __restrict__ lag, const double* __restrict__ X,
                                                      double sv, double* __restrict__ fr) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tr.off[8]) return;
    const int ft = type_of(k, tr);
    const int nv = ft_nverts(ft);
    const int4 v4 = st_vid[k];
    const double* L = lag + 9 * k;
    const double m[8] = {L[0], L[1], 0, 0, 0, 0, 0, 0};
    const bool ee = k >= tr.off[FT_EE];
    d3 s = mk(0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (i < nv) s = s + rec_coef(m, i, ee) * ld3(X, vslot(v4, i));
    const d3 n = mk(L[2], L[3], L[4]);
    const double ml = L[5];
    const d3 t = (s - dot(n, s) * n) - mk(L[6], L[7], L[8]);
    const double y = sqrt(dot(t, t));
    // f0, f1 / y and f1' of the transition, s_v = eps_v dt
    double f0, f1y, df1;
    if (y < sv) {
        f0 = -y * y * y / (3.0 * sv * sv) + y * y / sv + sv / 3.0;
        f1y = 2.0 / sv - y / (sv * sv);
        df1 = -2.0 * y / (sv * sv) + 2.0 / sv;
    } else {
        f0 = y;
        f1y = 1.0 / y;
        df1 = 0.0;
    }
    const double be = ml * fmax(f1y, 0.0);
    const double al = y > 0.0 ? (ml * fmax(df1, 0.0) - be) / (y * y) : 0.0;
    const d3 g = (ml * f1y) * t;
    double* r = fr + 10 * k;
    r[0] = ml * f0;
    r[1] = g.x; r[2] = g.y; r[3] = g.z;
    // S = be (I - n n^T) + al t t^T
    r[4] = be * (1.0 - n.x * n.x) + al * t.x * t.x;
    r[5] = -be * n.x * n.y + al * t.x * t.y;
    r[6] = -be * n.x * n.z + al * t.x * t.z;
    r[7] = be * (1.0 - n.y * n.y) + al * t.y * t.y;
    r[8] = -be * n.y * n.z + al * t.y * t.z;
    r[9] = be * (1.0 - n.z * n.z) + al * t.z * t.z;
}

__device__ __forceinline__ double lag_coef(const double* __restrict__ lag, uint32_t k, int i, int64_t e0) {
    const double m[8] = {lag[9 * (int64_t)k], lag[9 * (int64_t)k + 1], 0, 0, 0, 0, 0, 0};
    return rec_coef(m, i, (int64_t)k >= e0);
}

// kFrLanes lanes per row; each lane sums whole blocks of the row in their
// contribution order; the diagonal block also gives the gradient and the
// energy shares (pairs whose slot 0 is the row)
__global__ void __launch_bounds__(kBlock) k_fric_rows(int32_t V, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ diag_slot,
                                                      const int64_t* __restrict__ cptr,
                                                      const uint32_t* __restrict__ contrib,
                                                      const double* __restrict__ lag, const double* __restrict__ fr,
                                                      int64_t e0, double* __restrict__ grad, double* __restrict__ ev,
                                                      void* __restrict__ val, int dtype, int64_t nnzb) {
    const int64_t r = (int64_t)blockIdx.x * (kBlock / kFrLanes) + threadIdx.x / kFrLanes;
    const int lg = threadIdx.x % kFrLanes;
    if (r >= V) return;
    const int32_t ds = diag_slot[r];
    for (int32_t sl = row_ptr[r] + lg; sl < row_ptr[r + 1]; sl += kFrLanes) {
        const bool dg = sl == ds;
        if (!val && !dg) continue;
        double B[6] = {0, 0, 0, 0, 0, 0};
        d3 gsum = mk(0, 0, 0);
        double es = 0.0;
        for (int64_t t = cptr[sl]; t < cptr[sl + 1]; ++t) {
            const uint32_t code = contrib[t];
            const uint32_t k = code >> 4;
            const int i = (int)((code >> 2) & 3u), j = (int)(code & 3u);
            const double ci = lag_coef(lag, k, i, e0), cj = i == j ? ci : lag_coef(lag, k, j, e0);
            const double* f = fr + 10 * (int64_t)k;
            if (val) {
                const double cc = ci * cj;
#pragma unroll
                for (int q = 0; q < 6; ++q) B[q] += cc * f[4 + q];
            }
            if (dg) {
                gsum = gsum + ci * mk(f[1], f[2], f[3]);
                if (i == 0) es += f[0];
            }
        }
        if (dg) {
            grad[3 * r] = gsum.x;
            grad[3 * r + 1] = gsum.y;
            grad[3 * r + 2] = gsum.z;
            ev[r] = es;
        }
        if (val) {
            // symmetric 3x3 from its upper triangle, added to the stored block
            const double F[9] = {B[0], B[1], B[2], B[1], B[3], B[4], B[2], B[4], B[5]};
            if (dtype == GIPC_F64) {
                double* vv = static_cast<double*>(val);
#pragma unroll
                for (int c = 0; c < 9; ++c) vv[c * nnzb + sl] += F[c];
            } else {
                float* vv = static_cast<float*>(val);
#pragma unroll
                for (int c = 0; c < 9; ++c) vv[c * nnzb + sl] = (float)((double)vv[c * nnzb + sl] + F[c]);
            }
        }
    }
}

unsigned grid(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fric_lag(const int4* st_vid, const int32_t* mult, const TypeRanges& tr, const double* x,
                           const double* xr, const DevParams& pm, double mu, double* lag, hipStream_t s) {
    if (tr.off[8] == 0) return hipSuccess;
    k_fric_lag<<<grid(tr.off[8]), kBlock, 0, s>>>(st_vid, mult, tr, x, xr, pm, mu, lag);
    return hipGetLastError();
}

hipError_t launch_fric_eval(int32_t V, const int4* st_vid, const TypeRanges& tr, const double* lag, const double* x,
                            double sv, double* fr, const int32_t* row_ptr, const int32_t* diag_slot,
                            const int64_t* cptr, const uint32_t* contrib, double* grad, double* ev, void* val,
                            int dtype, int64_t nnzb, hipStream_t s) {
    if (tr.off[8] > 0) {
        k_fric_pair<<<grid(tr.off[8]), kBlock, 0, s>>>(st_vid, tr, lag, x, sv, fr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (V == 0) return hipSuccess;
    const int64_t nb = ((int64_t)V * kFrLanes + kBlock - 1) / kBlock;
    k_fric_rows<<<(unsigned)nb, kBlock, 0, s>>>(V, row_ptr, diag_slot, cptr, contrib, lag, fr, tr.off[FT_EE], grad,
                                                ev, val, dtype, nnzb);
    return hipGetLastError();
}

}  // namespace gipc
