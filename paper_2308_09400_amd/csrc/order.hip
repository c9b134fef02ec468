// Processing order of the block rows for the assembly gathers.  A pair's
// record is read by every row of its stencil; in the caller's vertex order
// those rows can be far apart (the same grid point on two stacked sheets),
// so each read misses the caches.  Rows are visited instead in the order of
// a counting sort of the vertices into Morton-ordered cells of the bounding
// cube (one scale for all axes, so vertices within contact distance share
// or neighbour a cell): 128^3 cells for one scene; for a batch, scene-major
// buckets with cells of each scene's own cube (fewer per scene).  Only the
// visiting order changes: every row's sums are the same, so results do not
// depend on it (the order inside a cell, set by atomics, is arbitrary).
#include "internal.hpp"

namespace gipc {
namespace {

constexpr int kCellBits = 7;                       // cells per axis: 128

// per-workgroup min / max of each coordinate
__global__ void __launch_bounds__(kBlock) k_bbox_part(const double* __restrict__ X, int32_t V,
                                                      double* __restrict__ part) {
    __shared__ double lds[6][kBlock / 64];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < V; v += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double c = X[3 * v + a];
            lo[a] = fmin(lo[a], c);
            hi[a] = fmax(hi[a], c);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, 64));
        }
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            lds[a][threadIdx.x >> 6] = lo[a];
            lds[3 + a][threadIdx.x >> 6] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double m = lds[a][0];
        for (int w = 1; w < kBlock / 64; ++w) m = a < 3 ? fmin(m, lds[a][w]) : fmax(m, lds[a][w]);
        part[6 * blockIdx.x + a] = m;
    }
}

// 10-bit spread for Morton interleaving (bits i -> 3i)
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// the box over all partial boxes: box[0..2] = min, box[3..5] = max; one
// wavefront per coordinate bound
__global__ void __launch_bounds__(384) k_bbox_final(const double* __restrict__ part, int32_t nparts,
                                                    double* __restrict__ box) {
    const int a = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool mn = a < 3;
    double m = mn ? INFINITY : -INFINITY;
    for (int p = lane; p < nparts; p += 64) m = mn ? fmin(m, part[6 * p + a]) : fmax(m, part[6 * p + a]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o, 64);
        m = mn ? fmin(m, t) : fmax(m, t);
    }
    if (lane == 0) box[a] = m;
}

// one workgroup per scene: the box of its vertex range (batches)
__global__ void __launch_bounds__(kBlock) k_bbox_scene(const double* __restrict__ X,
                                                       const int32_t* __restrict__ vert_off,
                                                       double* __restrict__ box) {
    __shared__ double lds[6][kBlock / 64];
    const int sc = blockIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = vert_off[sc] + (int64_t)threadIdx.x; v < vert_off[sc + 1]; v += kBlock) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double c = X[3 * v + a];
            lo[a] = fmin(lo[a], c);
            hi[a] = fmax(hi[a], c);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, 64));
        }
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            lds[a][threadIdx.x >> 6] = lo[a];
            lds[3 + a][threadIdx.x >> 6] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double m = lds[a][0];
        for (int w = 1; w < kBlock / 64; ++w) m = a < 3 ? fmin(m, lds[a][w]) : fmax(m, lds[a][w]);
        box[6 * sc + a] = m;
    }
}

// bucket of every vertex (scene-major, then the Morton cell with `bits`
// bits per axis inside the scene's cube) and the bucket histogram
__global__ void __launch_bounds__(kBlock) k_cell_count(const double* __restrict__ X, int32_t V,
                                                       const int32_t* __restrict__ vscene,
                                                       const double* __restrict__ box, int bits,
                                                       int32_t* __restrict__ cell, int32_t* __restrict__ hist) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= V) return;
    const int sc = vscene ? vscene[v] : 0;
    const double* b = box + 6 * sc;
    const double lo[3] = {b[0], b[1], b[2]};
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, b[3 + a] - lo[a]);
    const int n = 1 << bits;
    const double scale = ext > 0.0 && isfinite(ext) ? (double)n / ext : 0.0;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        double t = (X[3 * v + a] - lo[a]) * scale;
        t = t >= 0.0 ? t : 0.0;  // also maps NaN to 0
        q[a] = t < (double)(n - 1) ? (uint32_t)t : (uint32_t)(n - 1);
    }
    const int32_t c = (int32_t)(((uint32_t)sc << (3 * bits)) | spread3(q[0]) | (spread3(q[1]) << 1) |
                                (spread3(q[2]) << 2));
    cell[v] = c;
    atomicAdd(&hist[c], 1);
}

__global__ void __launch_bounds__(kBlock) k_cell_scatter(int32_t V, const int32_t* __restrict__ cell,
                                                         const int32_t* __restrict__ cell_off,
                                                         int32_t* __restrict__ fill, int32_t* __restrict__ order) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= V) return;
    const int32_t c = cell[v];
    order[cell_off[c] + atomicAdd(&fill[c], 1)] = (int32_t)v;
}

}  // namespace

hipError_t build_row_order(gipc_ctx* ctx, const double* x, int32_t V, const int32_t* vert_off, int32_t S,
                           hipStream_t s) {
    hipError_t e;
#define TRY(x_)                                   \
    do {                                          \
        if ((e = (x_)) != hipSuccess) return e;   \
    } while (0)
    TRY(ensure(ctx->order, sizeof(int32_t) * (size_t)(V > 0 ? V : 1)));
    if (V == 0) return hipSuccess;
    const int32_t nparts = 512;
    // bits per axis: at most 7, and at most about 4 V buckets in all (S
    // scenes share them), so small builds do not pay for a large histogram
    int bits = kCellBits;
    while (bits > 0 && ((int64_t)S << (3 * bits)) > 4 * (int64_t)V) --bits;
    const int64_t nbuckets = (int64_t)S << (3 * bits);
    if (nbuckets > ((int64_t)1 << 31) - 2) return hipErrorInvalidValue;
    TRY(ensure(ctx->obox, sizeof(double) * 6 * (size_t)(S > 1 ? S : nparts + 1)));
    TRY(ensure(ctx->ocell, sizeof(int32_t) * (size_t)V));
    TRY(ensure(ctx->ohist, sizeof(int32_t) * (size_t)nbuckets));
    TRY(ensure(ctx->ooff, sizeof(int32_t) * (size_t)(nbuckets + 1)));
    TRY(ensure(ctx->ofill, sizeof(int32_t) * (size_t)nbuckets));
    double* box;
    if (S > 1) {
        box = as<double>(ctx->obox);
        k_bbox_scene<<<(unsigned)S, kBlock, 0, s>>>(x, vert_off, box);
        TRY(hipGetLastError());
    } else {
        box = as<double>(ctx->obox) + 6 * nparts;
        k_bbox_part<<<nparts, kBlock, 0, s>>>(x, V, as<double>(ctx->obox));
        TRY(hipGetLastError());
        k_bbox_final<<<1, 384, 0, s>>>(as<double>(ctx->obox), nparts, box);
        TRY(hipGetLastError());
    }
    TRY(zero_i32(as<int32_t>(ctx->ohist), as<int32_t>(ctx->ofill), nullptr, nbuckets, s));
    const unsigned nb = (unsigned)(((int64_t)V + kBlock - 1) / kBlock);
    k_cell_count<<<nb, kBlock, 0, s>>>(x, V, S > 1 ? as<int32_t>(ctx->vscene) : nullptr, box, bits,
                                      as<int32_t>(ctx->ocell), as<int32_t>(ctx->ohist));
    TRY(hipGetLastError());
    TRY((exclusive_scan<int32_t, int32_t>(as<int32_t>(ctx->ohist), nbuckets, as<int32_t>(ctx->ooff), ctx, s)));
    k_cell_scatter<<<nb, kBlock, 0, s>>>(V, as<int32_t>(ctx->ocell), as<int32_t>(ctx->ooff), as<int32_t>(ctx->ofill),
                                        as<int32_t>(ctx->order));
    TRY(hipGetLastError());
#undef TRY
    return hipSuccess;
}

}  // namespace gipc
