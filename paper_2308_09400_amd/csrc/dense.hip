// The matrix-free product from dense local Hessians, in the two schemes the
// paper compares in Table 2 (supplement Sec. 6, "Parallel local
// matrix-vector multiplication"): y = diag (x) I3 x + sum_k S_k^T H_k S_k x
// with every H_k stored dense (the [3n][3n] leading block of a 12 x 12 slot,
// n = 4, 3, 2 stencil vertices; gipc_proxy_dense writes them), each pair's
// local product added to y without forming a global matrix.
//   thread scheme: one lane per pair computes its whole local product
//     H_k x_k (3n rows of 3n entries) and adds each row to y;
//   entry scheme: one lane per matrix entry multiplies it with its x
//     component; the lanes of one local row (3n consecutive lanes, which may
//     straddle two wavefronts) are summed by a segmented reduction inside the
//     wavefront and only the first lane of each segment adds it to y.
// Both run one launch per stencil size (the paper's per-type buffers) and
// add to y with FP64 atomics, as the paper's scheme does, so the summation
// order, and the last bits of y, vary from run to run.
#include "internal.hpp"

namespace gipc {
namespace {

constexpr int kDenseDotBlock = 1024;   // must match the partial count of the PCG (mf_num_parts)
constexpr int kDenseDotRows = 64;      // rows per workgroup of the dot kernel (1024 / 16 lanes per row)

__global__ void __launch_bounds__(kBlock) k_dense_init(int32_t V, const double* __restrict__ diag,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 3ll * V) return;
    y[i] = diag ? diag[i / 3] * x[i] : 0.0;
}

// one lane per pair of [k0, k1), N stencil vertices
template <int N>
__global__ void __launch_bounds__(kBlock) k_dense_thread(int64_t k0, int64_t k1, const int4* __restrict__ st_vid,
                                                         const double* __restrict__ hess,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    constexpr int D = 3 * N;
    const int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= k1) return;
    const int4 v4 = st_vid[k];
    const int v[4] = {v4.x, v4.y, v4.z, v4.w};
    double xl[D];
#pragma unroll
    for (int c = 0; c < D; ++c) xl[c] = x[3ll * v[c / 3] + c % 3];
    const double* H = hess + 144 * k;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) acc += H[12 * r + c] * xl[c];
        atomicAdd(&y[3ll * v[r / 3] + r % 3], acc);
    }
}

// one lane per entry of the pairs of [k0, k1): entry e = (pair, row, col)
// in row-major order of the local matrices.  The wavefront's first entry is
// split into (pair, offset) once, on the scalar unit; each lane then needs
// only 32-bit divisions by the constants D*D and D.
template <int N>
__global__ void __launch_bounds__(kBlock) k_dense_entry(int64_t k0, int64_t k1, const int4* __restrict__ st_vid,
                                                        const double* __restrict__ hess,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    constexpr int D = 3 * N;
    constexpr uint32_t D2 = D * D;
    const int64_t ne = (k1 - k0) * (int64_t)D2;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    const int64_t wave0 = (int64_t)wv * 64;
    const int64_t kw = wave0 / D2;                                // pair of the wavefront's first entry
    const uint32_t off = (uint32_t)(wave0 - kw * D2) + (uint32_t)lane;  // < D2 + 64
    const uint32_t q = off / D2, rem = off - q * D2;
    const uint32_t r = rem / D, c = rem - r * D;
    const int64_t e = wave0 + lane;
    const bool in = e < ne;
    const int64_t k = k0 + kw + q;
    double v = 0.0;
    int4 v4 = make_int4(0, 0, 0, 0);
    if (in) {
        v4 = st_vid[k];
        const int vc = vslot(v4, (int)(c / 3));
        v = hess[144 * k + 12 * r + c] * x[3ll * vc + c % 3];
    }
    // the segment of this lane: its local row, clipped to the wavefront;
    // seg_beg / seg_end = first / last lane of the segment here
    const int seg_beg = max(0, lane - (int)c);
    const int seg_end = min(63, lane + (D - 1 - (int)c));
    // inclusive suffix sums inside the segment (Hillis-Steele on shfl_down);
    // a segment spans at most D <= 12 lanes, so distances 1, 2, 4, 8 reach
    // its end
#pragma unroll
    for (int o = 1; o < D; o <<= 1) {
        const double t = __shfl_down(v, o, 64);
        if (lane + o <= seg_end) v += t;
    }
    if (in && lane == seg_beg) atomicAdd(&y[3ll * vslot(v4, (int)(r / 3)) + r % 3], v);
}

// partial sums of x . y over kDenseDotRows rows per workgroup (the partial
// layout the PCG's alpha step reads)
__global__ void __launch_bounds__(kDenseDotBlock) k_dense_dot(int32_t V, const double* __restrict__ x,
                                                              const double* __restrict__ y, double* __restrict__ part,
                                                              const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    __shared__ double lds[kDenseDotBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * (3 * kDenseDotRows) + threadIdx.x;
    double d = 0.0;
    if (threadIdx.x < 3 * kDenseDotRows && i < 3ll * V) d = x[i] * y[i];
    d = block_sum_n<kDenseDotBlock>(d, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
}

// inverses of the 3x3 diagonal blocks: diag + the (i, i) blocks of the
// row's pairs, summed over the row's diagonal contribution list in order
__global__ void __launch_bounds__(kBlock) k_dense_diag_inverse(int32_t V, const int32_t* __restrict__ diag_slot,
                                                               const int64_t* __restrict__ cptr,
                                                               const uint32_t* __restrict__ contrib,
                                                               const double* __restrict__ hess,
                                                               const double* __restrict__ diag,
                                                               double* __restrict__ minv) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= V) return;
    double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int32_t sl = diag_slot[r];
    for (int64_t t = cptr[sl]; t < cptr[sl + 1]; ++t) {
        const uint32_t code = contrib[t];
        const int64_t k = code >> 4;
        const int i = (int)((code >> 2) & 3u);
        const double* H = hess + 144 * k + (3 * i) * 12 + 3 * i;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) B[3 * a + b] += H[12 * a + b];
    }
    const double dv = diag ? diag[r] : 0.0;
    B[0] += dv; B[4] += dv; B[8] += dv;
    const double c00 = B[4] * B[8] - B[5] * B[7], c01 = B[5] * B[6] - B[3] * B[8], c02 = B[3] * B[7] - B[4] * B[6];
    const double det = B[0] * c00 + B[1] * c01 + B[2] * c02;
    double* M = minv + 9 * r;
    if (!(fabs(det) > 0.0) || !isfinite(det)) {
        for (int c = 0; c < 9; ++c) M[c] = (c % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const double id = 1.0 / det;
    M[0] = c00 * id; M[1] = (B[2] * B[7] - B[1] * B[8]) * id; M[2] = (B[1] * B[5] - B[2] * B[4]) * id;
    M[3] = c01 * id; M[4] = (B[0] * B[8] - B[2] * B[6]) * id; M[5] = (B[2] * B[3] - B[0] * B[5]) * id;
    M[6] = c02 * id; M[7] = (B[1] * B[6] - B[0] * B[7]) * id; M[8] = (B[0] * B[4] - B[1] * B[3]) * id;
}

template <int N>
hipError_t dense_range(int scheme, int64_t k0, int64_t k1, const int4* st_vid, const double* hess, const double* x,
                       double* y, const PcgScalars* sc, hipStream_t s) {
    if (k1 <= k0) return hipSuccess;
    if (scheme == GIPC_DENSE_THREAD) {
        const int64_t nb = (k1 - k0 + kBlock - 1) / kBlock;
        k_dense_thread<N><<<(unsigned)nb, kBlock, 0, s>>>(k0, k1, st_vid, hess, x, y, sc);
    } else {
        const int64_t ne = (k1 - k0) * (int64_t)(9 * N * N);
        const int64_t nb = (ne + kBlock - 1) / kBlock;
        k_dense_entry<N><<<(unsigned)nb, kBlock, 0, s>>>(k0, k1, st_vid, hess, x, y, sc);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense_apply(const MfView& m, const double* x, double* y, double* part, const PcgScalars* sc,
                              hipStream_t s) {
    if (m.V == 0) return hipSuccess;
    const int64_t n3 = 3ll * m.V;
    k_dense_init<<<(unsigned)((n3 + kBlock - 1) / kBlock), kBlock, 0, s>>>(m.V, m.diag, x, y, sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const TypeRanges& tr = m.tr;
    // per stencil size: 4 vertices (PT, EE and the mollified kinds), 3 (PE), 2 (PP)
    const int64_t r4[3][2] = {{tr.off[FT_PT], tr.off[FT_PT + 1]}, {tr.off[FT_EE], tr.off[FT_EE + 1]},
                              {tr.off[FT_EEM], tr.off[8]}};
    for (int q = 0; q < 3; ++q)
        if ((e = dense_range<4>(m.dense_scheme, r4[q][0], r4[q][1], m.st_vid, m.dense, x, y, sc, s)) != hipSuccess)
            return e;
    if ((e = dense_range<3>(m.dense_scheme, tr.off[FT_PE], tr.off[FT_PE + 1], m.st_vid, m.dense, x, y, sc, s)) !=
        hipSuccess)
        return e;
    if ((e = dense_range<2>(m.dense_scheme, tr.off[FT_PP], tr.off[FT_PP + 1], m.st_vid, m.dense, x, y, sc, s)) !=
        hipSuccess)
        return e;
    if (part) {
        k_dense_dot<<<(unsigned)mf_num_parts(m.V), kDenseDotBlock, 0, s>>>(m.V, x, y, part, sc);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_dense_diag_inverse(const MfView& m, double* minv, hipStream_t s) {
    if (m.V == 0) return hipSuccess;
    k_dense_diag_inverse<<<(unsigned)((m.V + kBlock - 1) / kBlock), kBlock, 0, s>>>(m.V, m.diag_slot, m.cptr,
                                                                                   m.contrib, m.dense, m.diag, minv);
    return hipGetLastError();
}

}  // namespace gipc
