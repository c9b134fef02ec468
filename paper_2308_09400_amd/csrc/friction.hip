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
// the diagonal blocks; a second pass adds c_i c_j S to every off-diagonal
// BSR block, each block summing its contribution list in the order of the
// symbolic phase.
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

// friction record, 16 doubles (one 128-byte line per pair for the row pass):
// [D, gx, gy, gz, S00, S01, S02, S11, S12, S22, c1, c2, -, -, -, -]
constexpr int kFr = 16;
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
    double* r = fr + kFr * k;
    r[10] = L[0];
    r[11] = L[1];
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

// c_i of pair k from its friction record
__device__ __forceinline__ double fr_coef(const double* f, uint32_t k, int i, int64_t e0) {
    const double m[8] = {f[10], f[11], 0, 0, 0, 0, 0, 0};
    return rec_coef(m, i, (int64_t)k >= e0);
}

// adds the symmetric 3x3 given by its upper triangle U to stored block sl
__device__ __forceinline__ void add_block_sym(void* val, int dtype, int64_t nnzb, int64_t sl, const double* U) {
    const double F[9] = {U[0], U[1], U[2], U[1], U[3], U[4], U[2], U[4], U[5]};
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

// kFrLanes lanes per row.  The diagonal list (the row's incidences) is
// split over the lanes and reduced by a fixed butterfly: gradient, energy
// share (pairs whose slot 0 is the row) and, with val, the diagonal block.
__global__ void __launch_bounds__(kBlock) k_fric_rows(int32_t V, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ diag_slot,
                                                      const int64_t* __restrict__ cptr,
                                                      const uint32_t* __restrict__ contrib,
                                                      const double* __restrict__ fr, int64_t e0,
                                                      double* __restrict__ grad, double* __restrict__ ev,
                                                      void* __restrict__ val, int dtype, int64_t nnzb) {
    const int64_t r = xcd_block() * (kBlock / kFrLanes) + threadIdx.x / kFrLanes;
    const int lg = threadIdx.x % kFrLanes;
    const bool valid = r < V;
    const int32_t ds = valid ? diag_slot[r] : 0;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // gradient, energy, diagonal block
    if (valid) {
        for (int64_t t = cptr[ds] + lg; t < cptr[ds + 1]; t += kFrLanes) {
            const uint32_t code = contrib[t];
            const uint32_t k = code >> 4;
            const int i = (int)((code >> 2) & 3u);
            const double* f = fr + kFr * (int64_t)k;
            const double ci = fr_coef(f, k, i, e0);
            acc[0] += ci * f[1];
            acc[1] += ci * f[2];
            acc[2] += ci * f[3];
            if (i == 0) acc[3] += f[0];
            const double cc = ci * ci;
#pragma unroll
            for (int q = 0; q < 6; ++q) acc[4 + q] += cc * f[4 + q];
        }
    }
#pragma unroll
    for (int o = kFrLanes / 2; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] += __shfl_xor(acc[q], o, kFrLanes);
    if (!valid) return;
    if (lg == 0) {
        grad[3 * r] = acc[0];
        grad[3 * r + 1] = acc[1];
        grad[3 * r + 2] = acc[2];
        ev[r] = acc[3];
    }
    if (val && lg == 0) add_block_sym(val, dtype, nnzb, ds, acc + 4);
}

// Off-diagonal blocks, kFoLanes lanes per row: the row's blocks below and
// above the diagonal are taken kFoLanes at a time (a window of consecutive
// slots, whose contribution lists are contiguous), the window's
// contributions dealt evenly to the lanes, kFoLanes x kFoGroup per step; each
// lane writes its terms c_i c_j S (upper triangles) to LDS and the owner of
// each block adds its own in list order.  Block (c, r) sums the same pairs
// as (r, c) in the same order with the same products c_i c_j, so the two
// are equal, as S is symmetric.
constexpr int kFoLanes = 32, kFoGroup = 2;

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_fric_offdiag(int32_t V, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ diag_slot,
                                                        const int64_t* __restrict__ cptr,
                                                        const uint32_t* __restrict__ contrib,
                                                        const double* __restrict__ fr, int64_t e0,
                                                        void* __restrict__ val, int dtype, int64_t nnzb) {
    constexpr int L = kFoLanes, G = kFoGroup, C = L * G;
    __shared__ double lds[BLOCK / L][C][6];
    const int64_t r = xcd_block() * (BLOCK / L) + threadIdx.x / L;
    if (r >= V) return;  // the whole lane group (L divides the wavefront)
    const int lg = threadIdx.x % L;
    double(*T)[6] = lds[threadIdx.x / L];
    const int32_t ds = diag_slot[r];
    // the two runs of off-diagonal slots: [row start, ds) and (ds, row end)
    const int32_t lo[2] = {row_ptr[r], ds + 1}, hi[2] = {ds, row_ptr[r + 1]};
    for (int h = 0; h < 2; ++h) {
        for (int32_t w0 = lo[h]; w0 < hi[h]; w0 += L) {
            const int32_t w1 = min(w0 + L, hi[h]);
            const int32_t sl = w0 + lg;
            const bool own = sl < w1;
            int64_t o0 = 0, o1 = 0;
            if (own) {
                o0 = cptr[sl];
                o1 = cptr[sl + 1];
            }
            const int64_t W0 = cptr[w0], W1 = cptr[w1];
            double B[6] = {0, 0, 0, 0, 0, 0};
            for (int64_t c0 = W0; c0 < W1; c0 += C) {
                uint32_t code[G];
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int64_t t = c0 + u * L + lg;
                    code[u] = t < W1 ? contrib[t] : 0u;
                }
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    if (c0 + u * L + lg < W1) {
                        const uint32_t k = code[u] >> 4;
                        const int i = (int)((code[u] >> 2) & 3u), j = (int)(code[u] & 3u);
                        const double* f = fr + kFr * (int64_t)k;
                        const double cc = fr_coef(f, k, i, e0) * fr_coef(f, k, j, e0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) T[u * L + lg][c] = cc * f[4 + c];
                    }
                }
                // the lane group lies in one wavefront: its LDS writes are
                // visible to its reads once the compiler keeps their order
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (own) {
                    const int64_t a = o0 > c0 ? o0 : c0, z = o1 < c0 + C ? o1 : c0 + C;
                    for (int64_t t = a; t < z; ++t) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) B[c] += T[t - c0][c];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (own) add_block_sym(val, dtype, nnzb, sl, B);
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
    k_fric_rows<<<(unsigned)nb, kBlock, 0, s>>>(V, row_ptr, diag_slot, cptr, contrib, fr, tr.off[FT_EE], grad, ev,
                                                val, dtype, nnzb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !val) return e;
    const int64_t nbo = ((int64_t)V * kFoLanes + kBlock - 1) / kBlock;
    k_fric_offdiag<kBlock><<<(unsigned)nbo, kBlock, 0, s>>>(V, row_ptr, diag_slot, cptr, contrib, fr, tr.off[FT_EE],
                                                            val, dtype, nnzb);
    return hipGetLastError();
}

}  // namespace gipc
