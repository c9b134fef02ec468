// Per-pair evaluation (Algorithm 2 of the paper, one lane per staged pair):
// distance of the pair's sub-type, barrier energy, gradient factors and the
// analytically projected proxy Hessian, stored as compact factors:
//   main  [Ps][8]  = c1 c2 w~x w~y w~z P22 a2 E     (c0, c3 from the family)
//   extra [Pm][8]  = u v P11 P12, a1 [Pm]            (mollified kinds only)
// The energy is not reduced here: the row pass gathers each pair's E into
// the vertex in its slot 0, and the per-scene sums below run over fixed
// vertex pieces, so the result does not depend on how pairs map to lanes.
#include "internal.hpp"

namespace gipc {
namespace {

// a merged pair stands for `mult` identical constraints: its energy, its
// gradient factors and its Hessian factors are scaled by that count
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_eval(const int4* __restrict__ st_vid, const int32_t* __restrict__ mult,
                                                TypeRanges tr, const double* __restrict__ X,
                                                const double* __restrict__ XR, DevParams pm,
                                                double* __restrict__ rec_main, double* __restrict__ rec_extra,
                                                double* __restrict__ rec_a1) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= tr.off[8]) return;
    const int ft = type_of(k, tr);
    const int4 v4 = st_vid[k];
    const int v[4] = {v4.x, v4.y, v4.z, v4.w};
    const double w = mult ? (double)mult[k] : 1.0;
    PairFactors o;
    eval_typed(ft, v, X, XR, pm, o);
    double2* m = reinterpret_cast<double2*>(rec_main + 8 * k);
    m[0] = make_double2(o.c[1], o.c[2]);
    m[1] = make_double2(o.wt.x, o.wt.y);
    m[2] = make_double2(o.wt.z, w * o.P22);
    m[3] = make_double2(w * o.a2, w * o.E);
    if (ft >= FT_EEM) {
        double2* x = reinterpret_cast<double2*>(rec_extra + 8 * (k - tr.off[FT_EEM]));
        x[0] = make_double2(o.u.x, o.u.y);
        x[1] = make_double2(o.u.z, o.v.x);
        x[2] = make_double2(o.v.y, o.v.z);
        x[3] = make_double2(w * o.P11, w * o.P12);
        rec_a1[k - tr.off[FT_EEM]] = w * o.a1;
    }
}

// one workgroup per vertex piece: fixed strided order, four accumulators,
// then the fixed block reduction
__global__ void __launch_bounds__(kBlock) k_energy_pieces(const double* __restrict__ ev,
                                                          const int2* __restrict__ piece,
                                                          double* __restrict__ part) {
    __shared__ double lds[kBlock / 64];
    const int2 pc = piece[blockIdx.x];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int u = 0;
    for (int v = pc.x + (int)threadIdx.x; v < pc.y; v += kBlock, ++u) a[u & 3] += ev[v];
    double s = block_sum((a[0] + a[1]) + (a[2] + a[3]), lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one workgroup per scene: its pieces' partial sums in order
__global__ void __launch_bounds__(kBlock) k_energy_scenes(const double* __restrict__ part,
                                                          const int32_t* __restrict__ poff,
                                                          double* __restrict__ energy) {
    __shared__ double lds[kBlock / 64];
    const int s = blockIdx.x;
    const int p0 = poff[s], p1 = poff[s + 1];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int u = 0;
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kBlock, ++u) a[u & 3] += part[p];
    double e = block_sum((a[0] + a[1]) + (a[2] + a[3]), lds);
    if (threadIdx.x == 0) energy[s] = e;
}

template <int BLOCK>
hipError_t eval_launch(const int4* st_vid, const int32_t* mult, TypeRanges tr, const double* x, const double* xr,
                       const DevParams& pm, double* rec_main, double* rec_extra, double* rec_a1, hipStream_t s) {
    const int64_t nb = (tr.off[8] + BLOCK - 1) / BLOCK;
    k_eval<BLOCK><<<(unsigned)nb, BLOCK, 0, s>>>(st_vid, mult, tr, x, xr, pm, rec_main, rec_extra, rec_a1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_eval(const int4* st_vid, const int32_t* mult, TypeRanges tr, const double* x, const double* xr,
                       const DevParams& pm, double* rec_main, double* rec_extra, double* rec_a1, int waves,
                       hipStream_t s) {
    if (tr.off[8] == 0) return hipSuccess;
    switch (waves) {
        case 1: return eval_launch<64>(st_vid, mult, tr, x, xr, pm, rec_main, rec_extra, rec_a1, s);
        case 2: return eval_launch<128>(st_vid, mult, tr, x, xr, pm, rec_main, rec_extra, rec_a1, s);
        case 8: return eval_launch<512>(st_vid, mult, tr, x, xr, pm, rec_main, rec_extra, rec_a1, s);
        default: return eval_launch<256>(st_vid, mult, tr, x, xr, pm, rec_main, rec_extra, rec_a1, s);
    }
}

hipError_t launch_energy(const double* ev, const int2* pieces, int32_t npieces, const int32_t* poff, int32_t S,
                         double* part, double* energy, hipStream_t s) {
    if (npieces > 0) {
        k_energy_pieces<<<(unsigned)npieces, kBlock, 0, s>>>(ev, pieces, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (S > 0) k_energy_scenes<<<(unsigned)S, kBlock, 0, s>>>(part, poff, energy);
    return hipGetLastError();
}

}  // namespace gipc
