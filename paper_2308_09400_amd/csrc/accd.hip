// Additive CCD: the step bound of the line search (maxFeasibleStepSize in
// the implementation overview, Algorithm 1).  The paper adopts the additive
// CCD of Codimensional IPC (Li et al. 2021; Related Work, "Collision
// Detection"): a lower bound on the time of impact accumulated from safe
// sub-steps, each no longer than the current distance over a bound on how
// fast the distance can shrink.
//
// The tuple moves as x(t) = x + t p over t in [0, tc].
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
// number of trial steps, [6] head of the tuple queue
__global__ void k_accd_reset(unsigned long long* c, double tc) {
    if (threadIdx.x == 0) {
        c[0] = 0ull;
        c[1] = ~0ull;
        c[2] = 0ull;
        c[3] = 0ull;
        c[4] = (unsigned long long)__double_as_longlong(tc);
        c[5] = 0ull;
        c[6] = 0ull;
    }
}

// Every lane keeps one tuple's search state and takes the next tuple from a
// queue as soon as its search ends (a wavefront takes kAccdChunk queue
// entries at a time with one atomic), so a wavefront does not wait on its
// slowest lane: on the ten-sheet candidates the searches take 1 to 766
// trial steps, and one lane per tuple took 18.1 ms against 3.2 ms here.
// The grid is a fixed number of workgroups that run until the queue is
// empty; every search ends within max_iter steps, so every wavefront does.
constexpr int kAccdChunk = 256;
constexpr int kAccdGrid = 2048;  // workgroups: more than the chip holds at once

__global__ void __launch_bounds__(kBlock) k_accd_queue(const int4* __restrict__ tuples, int64_t P, int32_t V,
                                                       const double* __restrict__ X, const double* __restrict__ D,
                                                       double s, double tc, int32_t max_iter,
                                                       double* __restrict__ toi_out,
                                                       unsigned long long* __restrict__ c) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t cb = 0, ce = 0;   // the wavefront's current chunk [cb, ce)
    bool exhausted = false;
    bool act = false;
    int64_t p = 0;
    int kind = 0, it = 0, itmax = 0;
    double x0[12], dp[12];
    double lp = 0.0, g = 0.0, t = 0.0, tl = 0.0, tmin = tc;
    while (true) {
        unsigned long long idle = __ballot(!act);
        while (idle != 0ull && !exhausted) {
            if (cb >= ce) {
                unsigned long long b = 0ull;
                if (lane == 0) b = atomicAdd(&c[6], (unsigned long long)kAccdChunk);
                cb = (int64_t)__shfl(b, 0, 64);
                ce = cb + kAccdChunk < P ? cb + kAccdChunk : P;
                if (cb >= P) {
                    exhausted = true;
                    break;
                }
            }
            const int64_t take = (int64_t)__popcll(idle) < ce - cb ? (int64_t)__popcll(idle) : ce - cb;
            const int64_t rank = __popcll(idle & below);
            const bool got = !act && rank < take;
            if (got) p = cb + rank;
            cb += take;
            if (got) {
                int v[4], nv;
                kind = decode_tuple(tuples[p], V, v, nv);
                double res = tc;
                bool done = true;
                if (kind < 0) {
                    atomicAdd(&c[0], 1ull);
                    atomicMin(&c[1], (unsigned long long)p);
                    res = 0.0;
                } else {
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
                    int nf = 1, sb = 1, ns = 1;
                    switch (kind) {
                        case 0: nf = 2; sb = 2; ns = 2; break;
                        case 1: ns = 3; break;
                        case 2: ns = 2; break;
                        case 3: break;
                        case 4: sb = 2; ns = 2; break;
                        default: sb = 2; break;
                    }
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
                        const double n = sqrt(dp[3 * k] * dp[3 * k] + dp[3 * k + 1] * dp[3 * k + 1] +
                                              dp[3 * k + 2] * dp[3 * k + 2]);
                        if (k < nf) l1 = fmax(l1, n);
                        else if (k >= sb && k < sb + ns) l2 = fmax(l2, n);
                    }
                    lp = l1 + l2;
                    const double dd0 = local_dist2(kind, x0);
                    if (!(dd0 > 0.0) || !(dd0 < INFINITY)) {
                        atomicAdd(&c[3], 1ull);
                        res = 0.0;
                    } else if (lp > 0.0) {
                        const double d0 = sqrt(dd0);
                        g = s * d0;
                        t = 0.0;
                        tl = (1.0 - s) * d0 / lp;
                        it = 0;
                        done = false;
                    }
                }
                if (done) {
                    if (toi_out) toi_out[p] = res;
                    tmin = fmin(tmin, res);
                } else {
                    act = true;
                }
            }
            idle = __ballot(!act);
        }
        if (__ballot(act) == 0ull) break;  // the queue is empty and every search has ended
        if (act) {
            ++it;
            double xt[12];
            const double tt = t + tl;
#pragma unroll
            for (int j = 0; j < 12; ++j) xt[j] = x0[j] + tt * dp[j];
            const double dd = sqrt(local_dist2(kind, xt));
            bool fin = false;
            double res = 0.0;
            if (t > 0.0 && dd < g) {
                res = t;
                fin = true;
            } else {
                t = t + tl;
                if (t > tc) {
                    res = tc;
                    fin = true;
                } else {
                    tl = 0.9 * dd / lp;
                    if (it >= max_iter) {
                        atomicAdd(&c[2], 1ull);
                        res = t;
                        fin = true;
                    }
                }
            }
            if (fin) {
                if (toi_out) toi_out[p] = res;
                tmin = fmin(tmin, res);
                itmax = max(itmax, it);
                act = false;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tmin = fmin(tmin, __shfl_xor(tmin, o, 64));
        itmax = max(itmax, __shfl_xor(itmax, o, 64));
    }
    if (lane == 0) {
        atomicMin(&c[4], (unsigned long long)__double_as_longlong(tmin));
        atomicMax(&c[5], (unsigned long long)itmax);
    }
}

}  // namespace

hipError_t launch_accd(const int32_t* tuples, int64_t P, int32_t V, const double* x, const double* disp, double s,
                       double tc, int32_t max_iter, double* toi, unsigned long long* counters, hipStream_t st) {
    k_accd_reset<<<1, 64, 0, st>>>(counters, tc);
    if (P > 0) {
        int64_t nb = (P + kBlock - 1) / kBlock;
        if (nb > kAccdGrid) nb = kAccdGrid;
        k_accd_queue<<<(unsigned)nb, kBlock, 0, st>>>(reinterpret_cast<const int4*>(tuples), P, V, x, disp, s, tc,
                                                      max_iter, toi, counters);
    }
    return hipGetLastError();
}

}  // namespace gipc
