// Device-wide exclusive scan (three passes: block sums, scan of the block
// sums in one workgroup, block-local scans plus carry) and an integer max.
// Integer arithmetic only, so the results are deterministic.
#include "internal.hpp"

namespace gipc {
namespace {

constexpr int kChunk = kBlock * kScanItems;  // elements per workgroup

template <typename T>
__device__ T block_exscan(T v, T* lds, T& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T n = __shfl_up(inc, o, 64);
        if (lane >= o) inc += n;
    }
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            T t = lds[w];
            lds[w] = s;
            s += t;
        }
        lds[kBlock / 64] = s;
    }
    __syncthreads();
    T ex = lds[wid] + inc - v;
    total = lds[kBlock / 64];
    __syncthreads();
    return ex;
}

template <typename TIn>
__global__ void __launch_bounds__(kBlock) k_scan_partial(const TIn* __restrict__ in, int64_t n,
                                                         int64_t* __restrict__ bsum) {
    __shared__ int64_t lds[kBlock / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) s += (int64_t)in[i];
    }
    int64_t tot;
    block_exscan<int64_t>(s, lds, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of bsum[0..nb) in place by one workgroup; out[n] = total
template <typename TOut>
__global__ void __launch_bounds__(kBlock) k_scan_top(int64_t* __restrict__ bsum, int64_t nb, TOut* __restrict__ out,
                                                     int64_t n, int64_t* __restrict__ total) {
    __shared__ int64_t lds[kBlock / 64 + 1];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kChunk) {
        int64_t base = c0 + (int64_t)threadIdx.x * kScanItems;
        int64_t v[kScanItems];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = base + k;
            v[k] = i < nb ? bsum[i] : 0;
            s += v[k];
        }
        int64_t tot;
        int64_t ex = block_exscan<int64_t>(s, lds, tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            int64_t i = base + k;
            if (i < nb) bsum[i] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        out[n] = (TOut)carry;
        if (total) *total = carry;
    }
}

template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kBlock) k_scan_final(const TIn* __restrict__ in, int64_t n,
                                                       const int64_t* __restrict__ bsum, TOut* __restrict__ out) {
    __shared__ int64_t lds[kBlock / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? (int64_t)in[i] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t ex = block_exscan<int64_t>(s, lds, tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = (TOut)ex;
        ex += v[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_max_i32(const int32_t* __restrict__ in, int64_t n, int32_t* out) {
    __shared__ int32_t lds[kBlock / 64];
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        m = max(m, in[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, lds[w]);
        atomicMax(out, m);
    }
}

}  // namespace

template <typename TIn, typename TOut>
hipError_t exclusive_scan(const TIn* in, int64_t n, TOut* out, gipc_ctx* ctx, hipStream_t s, int64_t* total_dev) {
    int64_t nb = (n + kChunk - 1) / kChunk;
    if (nb < 1) nb = 1;
    hipError_t e = ensure(ctx->scan_tmp, sizeof(int64_t) * (nb + 1));
    if (e != hipSuccess) return e;
    int64_t* bsum = as<int64_t>(ctx->scan_tmp);
    if (n > 0) k_scan_partial<TIn><<<(unsigned)nb, kBlock, 0, s>>>(in, n, bsum);
    else {
        e = hipMemsetAsync(bsum, 0, sizeof(int64_t), s);
        if (e != hipSuccess) return e;
    }
    k_scan_top<TOut><<<1, kBlock, 0, s>>>(bsum, n > 0 ? nb : 0, out, n, total_dev);
    if (n > 0) k_scan_final<TIn, TOut><<<(unsigned)nb, kBlock, 0, s>>>(in, n, bsum, out);
    return hipGetLastError();
}

template hipError_t exclusive_scan<int32_t, int64_t>(const int32_t*, int64_t, int64_t*, gipc_ctx*, hipStream_t,
                                                     int64_t*);
template hipError_t exclusive_scan<int32_t, int32_t>(const int32_t*, int64_t, int32_t*, gipc_ctx*, hipStream_t,
                                                     int64_t*);
template hipError_t exclusive_scan<int64_t, int64_t>(const int64_t*, int64_t, int64_t*, gipc_ctx*, hipStream_t,
                                                     int64_t*);

namespace {
// zeroes up to three int32 arrays of n entries in one launch (b, c nullable)
__global__ void __launch_bounds__(kBlock) k_zero_i32(int32_t* __restrict__ a, int32_t* __restrict__ b,
                                                     int32_t* __restrict__ c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    a[i] = 0;
    if (b) b[i] = 0;
    if (c) c[i] = 0;
}
}  // namespace

hipError_t zero_i32(int32_t* a, int32_t* b, int32_t* c, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zero_i32<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(a, b, c, n);
    return hipGetLastError();
}

hipError_t reduce_max_i32(const int32_t* in, int64_t n, int32_t* out_dev, hipStream_t s) {
    hipError_t e = hipMemsetAsync(out_dev, 0, sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    if (n <= 0) return hipSuccess;
    // one atomic per workgroup on the same word: few workgroups, each
    // striding over many elements
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 256) blocks = 256;
    k_max_i32<<<(unsigned)blocks, kBlock, 0, s>>>(in, n, out_dev);
    return hipGetLastError();
}

}  // namespace gipc
