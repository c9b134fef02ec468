// Per-pair evaluation (Algorithm 2 of the paper, one lane per staged pair):
// distance of the pair's sub-type, barrier energy, gradient factors and the
// analytically projected proxy Hessian, stored as compact factors:
//   main  [Ps][8]  = c0 c1 c2 w~x w~y w~z P22 a2     (c3 = -(c0+c1+c2))
//   extra [Pm][9]  = u v P11 P12 a1                   (mollified kinds only)
// The energy is reduced per workgroup in a fixed order and then summed by
// one workgroup, so it is bit-reproducible.
#include "internal.hpp"

namespace gipc {
namespace {

__global__ void __launch_bounds__(kBlock) k_eval(const int4* __restrict__ st_vid, TypeRanges tr,
                                                 const double* __restrict__ X, const double* __restrict__ XR,
                                                 DevParams pm, double* __restrict__ rec_main,
                                                 double* __restrict__ rec_extra, double* __restrict__ e_part) {
    __shared__ double lds[kBlock / 64];
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double E = 0.0;
    if (k < tr.off[8]) {
        const int ft = type_of(k, tr);
        const int4 v4 = st_vid[k];
        const int v[4] = {v4.x, v4.y, v4.z, v4.w};
        PairFactors o;
        eval_typed(ft, v, X, XR, pm, o);
        E = o.E;
        double2* m = reinterpret_cast<double2*>(rec_main + 8 * k);
        m[0] = make_double2(o.c[0], o.c[1]);
        m[1] = make_double2(o.c[2], o.wt.x);
        m[2] = make_double2(o.wt.y, o.wt.z);
        m[3] = make_double2(o.P22, o.a2);
        if (ft >= FT_EEM) {
            double* x = rec_extra + 9 * (k - tr.off[FT_EEM]);
            x[0] = o.u.x; x[1] = o.u.y; x[2] = o.u.z;
            x[3] = o.v.x; x[4] = o.v.y; x[5] = o.v.z;
            x[6] = o.P11; x[7] = o.P12; x[8] = o.a1;
        }
    }
    double s = block_sum(E, lds);
    if (threadIdx.x == 0) e_part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_energy_final(const double* __restrict__ e_part, int64_t n,
                                                         double* __restrict__ energy) {
    __shared__ double lds[kBlock / 64];
    // 8 independent accumulators per lane keep loads in flight; fixed order
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = threadIdx.x;
    for (; i + 7 * kBlock < n; i += 8 * kBlock) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += e_part[i + u * kBlock];
    }
    for (int u = 0; i < n; i += kBlock, ++u) a[u & 7] += e_part[i];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = block_sum(s, lds);
    if (threadIdx.x == 0) *energy = s;
}

}  // namespace

int64_t eval_num_parts(int64_t Ps) { return Ps > 0 ? (Ps + kBlock - 1) / kBlock : 0; }

hipError_t launch_eval(const int4* st_vid, TypeRanges tr, const double* x, const double* xr, const DevParams& pm,
                       double* rec_main, double* rec_extra, double* e_part, hipStream_t s) {
    int64_t nb = eval_num_parts(tr.off[8]);
    if (nb == 0) return hipSuccess;
    k_eval<<<(unsigned)nb, kBlock, 0, s>>>(st_vid, tr, x, xr, pm, rec_main, rec_extra, e_part);
    return hipGetLastError();
}

hipError_t launch_energy_final(const double* e_part, int64_t nparts, double* energy, hipStream_t s) {
    k_energy_final<<<1, kBlock, 0, s>>>(e_part, nparts, energy);
    return hipGetLastError();
}

}  // namespace gipc
