// Pair staging: classification of every tuple by the active constraints of
// its constrained distance (Eq. 4 / Eq. 5), dropping of pairs at distance
// >= dhat, and a stable counting sort of the active pairs by sub-type (the
// per-type pair buffers of Sec. 6.2 / supplement Sec. 6).  Two passes over
// the candidates (classify + per-workgroup type histogram, then scatter) with
// an exclusive scan of the [type][workgroup] histogram in between; the order
// within a type is the tuple order, so the result is deterministic.
#include "internal.hpp"

namespace gipc {
namespace {

// counters (relative to the pointer the kernel gets): [0] malformed tuples,
// [1] first malformed index, [2] degenerate pairs, [3] first degenerate
// index, [20] tuples whose vertices lie in different scenes, [21] the first
__device__ __forceinline__ void flag_index(unsigned long long* cnt, unsigned long long* first, int64_t p) {
    atomicAdd(cnt, 1ull);
    atomicMin(first, (unsigned long long)p);
}

__global__ void __launch_bounds__(kBlock) k_stage_classify(const int4* __restrict__ tuples, int64_t P, int32_t V,
                                                           const double* __restrict__ X, const double* __restrict__ XR,
                                                           DevParams pm, uint8_t* __restrict__ ft_out,
                                                           int4* __restrict__ vid_out, int32_t* __restrict__ bcount,
                                                           unsigned long long* __restrict__ counters) {
    __shared__ int32_t cnt[kBlock / 64][8];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int ft = FT_NONE;
    int4 vo = make_int4(-1, -1, -1, -1);
    if (p < P) {
        const int4 t = tuples[p];
        int kind = -1;  // 0 EE, 1 PT, 2 PE, 3 PP
        int v[4] = {-1, -1, -1, -1};
        int nv = 0;
        if (t.x != INT32_MIN && t.y != INT32_MIN) {
            if (t.x >= 0) {
                if (t.z >= 0 && t.w >= 0) {
                    kind = 0; nv = 4;
                    v[0] = t.x; v[1] = t.y >= 0 ? t.y : -t.y - 1; v[2] = t.z; v[3] = t.w;
                }
            } else if (t.y >= 0) {
                v[0] = -t.x - 1; v[1] = t.y;
                if (t.z >= 0 && t.w >= 0) { kind = 1; nv = 4; v[2] = t.z; v[3] = t.w; }
                else if (t.z >= 0 && t.w == -1) { kind = 2; nv = 3; v[2] = t.z; }
                else if (t.z == -1 && t.w == -1) { kind = 3; nv = 2; }
            }
        }
        bool ok = kind >= 0;
        for (int k = 0; k < nv && ok; ++k) {
            ok = v[k] >= 0 && v[k] < V;
            for (int l = 0; l < k && ok; ++l) ok = v[l] != v[k];
        }
        bool same_scene = true;
        if (ok && pm.vscene) {
            const int s0 = pm.vscene[v[0]];
            for (int k = 1; k < nv; ++k) same_scene = same_scene && pm.vscene[v[k]] == s0;
        }
        if (!ok) {
            flag_index(&counters[0], &counters[1], p);
        } else if (!same_scene) {
            flag_index(&counters[20], &counters[21], p);
        } else {
            double d2;
            Staged s;
            if (kind == 0) s = classify_ee(X, XR, v[0], v[1], v[2], v[3], pm, d2);
            else if (kind == 1) s = classify_pt(X, v[0], v[1], v[2], v[3], d2);
            else if (kind == 2) s = classify_pe(X, v[0], v[1], v[2], d2);
            else {
                d3 w = ld3(X, v[0]) - ld3(X, v[1]);
                d2 = dot(w, w);
                s = Staged{FT_PP, {v[0], v[1], -1, -1}};
            }
            double dhat, kappa;
            scene_params(pm, v[0], dhat, kappa);
            if (!(d2 > 0.0) || !(d2 < INFINITY)) {
                flag_index(&counters[2], &counters[3], p);
            } else if (d2 < dhat * dhat) {
                ft = s.ft;
                vo = make_int4(s.v[0], s.v[1], s.v[2], s.v[3]);
            }
        }
        ft_out[p] = (uint8_t)ft;
        if (ft != FT_NONE) vid_out[p] = vo;  // read back for active tuples only
    }
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        unsigned long long m = __ballot(ft == t);
        if (lane == 0) cnt[wid][t] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x < 8) {
        int s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += cnt[w][threadIdx.x];
        bcount[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
    if (threadIdx.x == 0) bcount[blockIdx.x] = 0;
}

__global__ void __launch_bounds__(kBlock) k_stage_scatter(const uint8_t* __restrict__ ft_in,
                                                          const int4* __restrict__ vid_in, int64_t P,
                                                          const int64_t* __restrict__ boff, int4* __restrict__ st_vid,
                                                          int32_t* __restrict__ st_src) {
    __shared__ int32_t cnt[kBlock / 64][8];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int ft = p < P ? (int)ft_in[p] : FT_NONE;
    unsigned long long mine = 0;
#pragma unroll
    for (int t = 1; t < 8; ++t) {
        unsigned long long m = __ballot(ft == t);
        if (ft == t) mine = m;
        if (lane == 0) cnt[wid][t] = __popcll(m);
    }
    __syncthreads();
    if (ft != FT_NONE) {
        int64_t pos = boff[(int64_t)ft * gridDim.x + blockIdx.x];
        for (int w = 0; w < wid; ++w) pos += cnt[w][ft];
        pos += __popcll(mine & __lanemask_lt());
        st_vid[pos] = vid_in[p];
        st_src[pos] = (int32_t)p;
    }
}

}  // namespace

hipError_t launch_stage_classify(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* xr,
                                 const DevParams& pm, uint8_t* ft, int4* vid, int32_t* bcount, int64_t* counters,
                                 hipStream_t s) {
    int64_t nb = (P + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_stage_classify<<<(unsigned)nb, kBlock, 0, s>>>(reinterpret_cast<const int4*>(tuples), P, V, x, xr, pm, ft, vid,
                                                     bcount, reinterpret_cast<unsigned long long*>(counters));
    return hipGetLastError();
}

hipError_t launch_stage_scatter(const uint8_t* ft, const int4* vid, int64_t P, const int64_t* boff, int4* st_vid,
                                int32_t* st_src, hipStream_t s) {
    int64_t nb = (P + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_stage_scatter<<<(unsigned)nb, kBlock, 0, s>>>(ft, vid, P, boff, st_vid, st_src);
    return hipGetLastError();
}

}  // namespace gipc

namespace gipc {
namespace {
// type offsets: out[t] = boff[t * nb] for t = 0..8 (boff[8 nb] is the total)
__global__ void k_stage_offsets(const int64_t* __restrict__ boff, int64_t nb, int64_t* __restrict__ out) {
    int t = threadIdx.x;
    if (t < 9) out[t] = boff[t * nb];
}
}  // namespace

hipError_t launch_stage_offsets(const int64_t* boff, int64_t nb, int64_t* out, hipStream_t s) {
    k_stage_offsets<<<1, 64, 0, s>>>(boff, nb, out);
    return hipGetLastError();
}

namespace {
// scene of every vertex: the last s with vert_off[s] <= v (vert_off is
// non-decreasing with vert_off[0] = 0 and vert_off[S] = V, checked on the host)
__global__ void __launch_bounds__(kBlock) k_vertex_scene(const int32_t* __restrict__ vert_off, int32_t S, int32_t V,
                                                         int32_t* __restrict__ vscene) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= V) return;
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vert_off[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    vscene[v] = lo;
}
}  // namespace

hipError_t launch_vertex_scene(const int32_t* vert_off, int32_t S, int32_t V, int32_t* vscene, hipStream_t s) {
    if (V == 0) return hipSuccess;
    k_vertex_scene<<<(unsigned)((V + kBlock - 1) / kBlock), kBlock, 0, s>>>(vert_off, S, V, vscene);
    return hipGetLastError();
}
}  // namespace gipc
