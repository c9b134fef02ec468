// Pair staging: classification of every tuple by the active constraints of
// its constrained distance (Eq. 4 / Eq. 5), dropping of pairs at distance
// >= dhat, and a stable counting sort of the active pairs by sub-type (the
// per-type pair buffers of Sec. 7.2 / supplement Sec. 6).  Two passes over
// the candidates (classify + per-workgroup type histogram, then scatter) with
// an exclusive scan of the [type][workgroup] histogram in between; the order
// within a type is the tuple order, so the result is deterministic.
#include "internal.hpp"

namespace gipc {
namespace {

// counters (relative to the pointer the kernel gets): [0] malformed tuples,
// [1] first malformed index, [2] degenerate pairs, [3] first degenerate
// index, [14] tuples with a degenerate primitive, [15] the first, [20]
// tuples whose vertices lie in different scenes, [21] the first
__device__ __forceinline__ void flag_index(unsigned long long* cnt, unsigned long long* first, int64_t p) {
    atomicAdd(cnt, 1ull);
    atomicMin(first, (unsigned long long)p);
}

enum TupleStatus { TS_OK = 0, TS_BAD = 1, TS_SPAN = 2, TS_DEGEN = 3 };

// One tuple (decode_tuple): the vertex ids are checked, then the tuple is
// classified at X: ft is its
// sub-type if it is closer than its scene's dhat (else FT_NONE), vo its
// staged stencil, dprim whether a primitive is degenerate (an edge of zero
// length, a triangle of zero area) while the distance is still positive.
__device__ inline int classify_tuple(const int4 t, int32_t V, const double* __restrict__ X,
                                     const double* __restrict__ XR, const DevParams& pm, int& ft, int4& vo,
                                     bool& dprim) {
    ft = FT_NONE;
    vo = make_int4(-1, -1, -1, -1);
    dprim = false;
    int v[4], nv;
    const int kind = decode_tuple(t, V, v, nv);
    if (kind < 0) return TS_BAD;
    if (pm.vscene) {
        const int s0 = pm.vscene[v[0]];
        for (int k = 1; k < nv; ++k)
            if (pm.vscene[v[k]] != s0) return TS_SPAN;
    }
    double d2;
    bool degen = false;
    Staged s;
    if (kind == 0) s = classify_ee(X, XR, v[0], v[1], v[2], v[3], pm, d2, degen);
    else if (kind == 1) s = classify_pt(X, v[0], v[1], v[2], v[3], d2, degen);
    else if (kind == 2) s = classify_pe(X, v[0], v[1], v[2], d2, degen);
    else if (kind == 3) {
        d3 w = ld3(X, v[0]) - ld3(X, v[1]);
        d2 = dot(w, w);
        s = Staged{FT_PP, {v[0], v[1], -1, -1}};
    } else {
        s = classify_par(X, XR, v[0], v[1], v[2], v[3], kind == 4, pm, d2, degen);
    }
    if (!(d2 > 0.0) || !(d2 < INFINITY)) return TS_DEGEN;
    dprim = degen;
    double dhat, kappa;
    scene_params(pm, v[0], dhat, kappa);
    if (d2 < dhat * dhat) {
        ft = s.ft;
        vo = make_int4(s.v[0], s.v[1], s.v[2], s.v[3]);
    }
    return TS_OK;
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
    if (p < P) {
        int4 vo;
        bool dprim;
        const int st = classify_tuple(tuples[p], V, X, XR, pm, ft, vo, dprim);
        if (st == TS_BAD) flag_index(&counters[0], &counters[1], p);
        else if (st == TS_SPAN) flag_index(&counters[20], &counters[21], p);
        else if (st == TS_DEGEN) flag_index(&counters[2], &counters[3], p);
        else if (dprim) flag_index(&counters[14], &counters[15], p);
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

// The build's classification against the one at X, tuple by tuple (the
// build's sub-types in ft_b, stencils of its active tuples in vid_b):
// counters [0] tuples closer than dhat now but not at the build, [1] active
// at the build but not now (the build's sub-type formula also puts them at
// or beyond dhat, so the evaluation drops them), [2] active at the build
// with another sub-type or stencil now, or inactive now while the build's
// formula still finds them within dhat, [3] degenerate now (distance 0 or
// not finite), [4] malformed or spanning two scenes, [5] the first tuple
// counted in [0] or [2].
__global__ void __launch_bounds__(kBlock) k_stage_check(const int4* __restrict__ tuples, int64_t P, int32_t V,
                                                        const double* __restrict__ X, const double* __restrict__ XR,
                                                        DevParams pm, const uint8_t* __restrict__ ft_b,
                                                        const int4* __restrict__ vid_b,
                                                        unsigned long long* __restrict__ counters) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= P) return;
    int ft;
    int4 vo;
    bool dprim;
    const int st = classify_tuple(tuples[p], V, X, XR, pm, ft, vo, dprim);
    if (st == TS_BAD || st == TS_SPAN) {
        atomicAdd(&counters[4], 1ull);
        return;
    }
    if (st == TS_DEGEN) {
        atomicAdd(&counters[3], 1ull);
        ft = FT_NONE;
    }
    const int fb = ft_b[p];
    int which = -1;
    if (fb == FT_NONE && ft != FT_NONE) {
        which = 0;
    } else if (fb != FT_NONE && ft == FT_NONE) {
        // harmless if the build's sub-type formula, which the evaluation
        // uses, also puts the pair at or beyond dhat
        const int4 b = vid_b[p];
        const int bv[4] = {b.x, b.y, b.z, b.w};
        PairFactors o;
        eval_typed(fb, bv, X, XR, pm, o);
        which = (o.E != 0.0 || o.a2 != 0.0 || o.P22 != 0.0) ? 2 : 1;
    } else if (fb != FT_NONE) {
        const int4 b = vid_b[p];
        if (fb != ft || b.x != vo.x || b.y != vo.y || b.z != vo.z || b.w != vo.w) which = 2;
    }
    if (which == 1) atomicAdd(&counters[1], 1ull);
    else if (which >= 0) flag_index(&counters[which], &counters[5], p);
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

hipError_t launch_stage_check(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* xr,
                              const DevParams& pm, const uint8_t* ft_b, const int4* vid_b, int64_t* counters,
                              hipStream_t s) {
    int64_t nb = (P + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_stage_check<<<(unsigned)nb, kBlock, 0, s>>>(reinterpret_cast<const int4*>(tuples), P, V, x, xr, pm, ft_b, vid_b,
                                                  reinterpret_cast<unsigned long long*>(counters));
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
