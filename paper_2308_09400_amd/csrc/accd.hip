// Additive CCD: the step bound of the line search (maxFeasibleStepSize in
// the implementation overview, Algorithm 1).  The paper adopts the additive
// CCD of Codimensional IPC (Li et al. 2021; Related Work, "Collision
// Detection"): a lower bound on the time of impact accumulated from safe
// sub-steps, each no longer than the current distance over a bound on how
// fast the distance can shrink.
//
// One lane per tuple.  The tuple moves as x(t) = x + t p over t in [0, tc].
// With the common translation removed from p (the mean over the vertices the
// distance involves) and l_p the largest |p_i| over the first primitive plus
// the largest over the second, the distance falls at most at rate l_p.  From
// d0 = d(0) and the stop gap s d0 the lane takes a first sub-step
// (1 - s) d0 / l_p, then 0.9 d / l_p from each accepted point, until the
// distance at a trial point would fall below s d0 (the accumulated time is
// returned) or the time passes tc (tc is returned).  Distances are the
// constrained minimum of the tuple's primitives (Eq. 4 / Eq. 5), evaluated
// at each trial point from x, not accumulated.
#include "internal.hpp"

namespace gipc {
namespace {

// constrained squared distance of a decoded tuple whose four slots are the
// local positions L[0..11] (slot k at L[3k])
__device__ __forceinline__ double local_dist2(int kind, const double* L) {
    DevParams pm{};  // no mollifier decision: only the distance is wanted
    double d2 = 0.0;
    bool degen;
    if (kind == 0) (void)classify_ee(L, nullptr, 0, 1, 2, 3, pm, d2, degen);
    else if (kind == 1) (void)classify_pt(L, 0, 1, 2, 3, d2, degen);
    else if (kind == 2) (void)classify_pe(L, 0, 1, 2, d2, degen);
    else if (kind == 3) {
        const d3 w = ld3(L, 0) - ld3(L, 1);
        d2 = dot(w, w);
    } else {
        (void)classify_par(L, nullptr, 0, 1, 2, 3, kind == 4, pm, d2, degen);
    }
    return d2;
}

// counters: [0] malformed tuples, [1] first malformed index, [2] tuples
// stopped by max_iter, [3] tuples at distance 0, [4] bits of the smallest
// time (non-negative doubles order as their bit patterns), [5] largest
// number of trial steps
__global__ void k_accd_reset(unsigned long long* c, double tc) {
    if (threadIdx.x == 0) {
        c[0] = 0ull;
        c[1] = ~0ull;
        c[2] = 0ull;
        c[3] = 0ull;
        c[4] = (unsigned long long)__double_as_longlong(tc);
        c[5] = 0ull;
    }
}

// per-tuple search; returns the time and the trial steps taken (max_iter
// when the cap stopped it, flagged in capped)
__device__ inline double accd_one(int kind, const double* x0, double* dp, int nv, double s, double tc,
                                  int32_t max_iter, int& it, bool& capped, bool& touching) {
    (void)nv;
    // slots of the two primitives: first [0, nf), second [sb, sb + ns)
    int nf = 1, sb = 1, ns = 1;
    switch (kind) {
        case 0: nf = 2; sb = 2; ns = 2; break;  // edge-edge
        case 1: ns = 3; break;                  // point-triangle
        case 2: ns = 2; break;                  // point-edge
        case 3: break;                          // point-point
        case 4: sb = 2; ns = 2; break;          // point vs edge (e0, e1) in slots 2, 3
        default: sb = 2; break;                 // point vs point in slot 2
    }
    // remove the mean displacement of the slots the distance involves
    double m[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = k < nf || (k >= sb && k < sb + ns);
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] += in ? dp[3 * k + d] : 0.0;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) m[d] /= (double)(nf + ns);
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) dp[3 * k + d] -= m[d];
    double l1 = 0.0, l2 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double n = sqrt(dp[3 * k] * dp[3 * k] + dp[3 * k + 1] * dp[3 * k + 1] + dp[3 * k + 2] * dp[3 * k + 2]);
        if (k < nf) l1 = fmax(l1, n);
        else if (k >= sb && k < sb + ns) l2 = fmax(l2, n);
    }
    const double lp = l1 + l2;
    const double dd0 = local_dist2(kind, x0);
    it = 0;
    capped = false;
    touching = false;
    if (!(dd0 > 0.0) || !(dd0 < INFINITY)) {
        touching = true;  // no step
        return 0.0;
    }
    if (!(lp > 0.0)) return tc;  // no relative motion
    const double d0 = sqrt(dd0), g = s * d0;
    double t = 0.0, tl = (1.0 - s) * d0 / lp;
    for (it = 1; it <= max_iter; ++it) {
        double xt[12];
        const double tt = t + tl;
#pragma unroll
        for (int j = 0; j < 12; ++j) xt[j] = x0[j] + tt * dp[j];
        const double dd = sqrt(local_dist2(kind, xt));
        if (t > 0.0 && dd < g) return t;
        t = t + tl;
        if (t > tc) return tc;
        tl = 0.9 * dd / lp;
    }
    it = max_iter;
    capped = true;
    return t;
}

__global__ void __launch_bounds__(kBlock) k_accd(const int4* __restrict__ tuples, int64_t P, int32_t V,
                                                 const double* __restrict__ X, const double* __restrict__ D,
                                                 double s, double tc, int32_t max_iter, double* __restrict__ toi_out,
                                                 unsigned long long* __restrict__ c) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double t = tc;  // neutral for the minimum
    int it = 0;
    if (p < P) {
        int v[4], nv;
        const int kind = decode_tuple(tuples[p], V, v, nv);
        if (kind < 0) {
            atomicAdd(&c[0], 1ull);
            atomicMin(&c[1], (unsigned long long)p);
            t = 0.0;
        } else {
            double x0[12], dp[12];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool use = k < nv;
                const int vk = use ? v[k] : 0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x0[3 * k + d] = use ? X[3ll * vk + d] : 0.0;
                    dp[3 * k + d] = use ? D[3ll * vk + d] : 0.0;
                }
            }
            bool capped, touching;
            t = accd_one(kind, x0, dp, nv, s, tc, max_iter, it, capped, touching);
            if (capped) atomicAdd(&c[2], 1ull);
            if (touching) atomicAdd(&c[3], 1ull);
        }
        if (toi_out) toi_out[p] = t;
    }
    // one atomic per wavefront for the smallest time and the most steps
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        t = fmin(t, __shfl_xor(t, o, 64));
        it = max(it, __shfl_xor(it, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&c[4], (unsigned long long)__double_as_longlong(t));
        atomicMax(&c[5], (unsigned long long)it);
    }
}

}  // namespace

hipError_t launch_accd(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* disp, double s,
                       double tc, int32_t max_iter, double* toi, unsigned long long* counters, hipStream_t st) {
    k_accd_reset<<<1, 64, 0, st>>>(counters, tc);
    if (P > 0) {
        const unsigned nb = (unsigned)((P + kBlock - 1) / kBlock);
        k_accd<<<nb, kBlock, 0, st>>>(reinterpret_cast<const int4*>(tuples), P, V, x, disp, s, tc, max_iter, toi,
                                      counters);
    }
    return hipGetLastError();
}

}  // namespace gipc
