// Numeric assembly by gathering (no floating-point atomics): every BSR block
// sums its own contribution list, in the order fixed by the symbolic phase.
//   block(v_i, v_j) += P22 g_i g_j^T + P12 (s_i g_j^T + g_i s_j^T) + P11 s_i s_j^T
// with g_i = c_i w~ (slot i of grad f) and s_i = (-u, u, -v, v)_i (slot i of
// grad sqrt(c), mollified pairs only).  The gradient of vertex r gathers
// a2 g_i + a1 s_i over the contributions of its diagonal block, which are
// exactly its incidences (i = j); the same pass sums the energies of the
// pairs whose slot 0 is r.
#include "internal.hpp"

namespace gipc {
namespace {

__device__ __forceinline__ d3 sq_slot(const double* x, int i) {
    // (-u, u, -v, v)
    double sg = (i & 1) ? 1.0 : -1.0;
    return i < 2 ? mk(sg * x[0], sg * x[1], sg * x[2]) : mk(sg * x[3], sg * x[4], sg * x[5]);
}

__device__ __forceinline__ void add_outer(double* B, double s, d3 a, d3 b) {
    B[0] += s * a.x * b.x; B[1] += s * a.x * b.y; B[2] += s * a.x * b.z;
    B[3] += s * a.y * b.x; B[4] += s * a.y * b.y; B[5] += s * a.y * b.z;
    B[6] += s * a.z * b.x; B[7] += s * a.z * b.y; B[8] += s * a.z * b.z;
}

// one local block (i, j) of pair k added to B; pairs from e0 on are of the
// edge-edge family, from m0 on mollified
__device__ __forceinline__ void add_block(double* B, const double* __restrict__ rec_main,
                                          const double* __restrict__ rec_extra, int64_t e0, int64_t m0, uint32_t k,
                                          int i, int j) {
    const double* m = rec_main + 8 * (int64_t)k;
    const bool ee = (int64_t)k >= e0;
    d3 wt = mk(m[R_W], m[R_W + 1], m[R_W + 2]);
    d3 gi = rec_coef(m, i, ee) * wt, gj = rec_coef(m, j, ee) * wt;
    add_outer(B, m[R_P22], gi, gj);
    if ((int64_t)k >= m0) {
        const double* x = rec_extra + 8 * ((int64_t)k - m0);
        d3 si = sq_slot(x, i), sj = sq_slot(x, j);
        add_outer(B, x[6], si, sj);
        add_outer(B, x[7], si, gj);
        add_outer(B, x[7], gi, sj);
    }
}

// store B (tr = false) or its transpose (tr = true) into block slot s
// the main-record fields a block needs (c1, c2, w~, P22), loaded as three
// 16-byte words, so several contributions' loads can be in flight at once
struct MainRec {
    double2 a, b, c;  // (c1, c2), (w~x, w~y), (w~z, P22)
};

__device__ __forceinline__ MainRec load_main(const double* __restrict__ rec_main, uint32_t k) {
    const double2* m = reinterpret_cast<const double2*>(rec_main + 8 * (int64_t)k);
    return MainRec{m[0], m[1], m[2]};
}

// add_block with the main record already loaded; the extra record (64
// bytes, one line) is read as four 16-byte words
__device__ __forceinline__ void add_block_rec(double* B, const MainRec& mr, const double* __restrict__ rec_extra,
                                              int64_t e0, int64_t m0, uint32_t k, int i, int j) {
    const double m[8] = {mr.a.x, mr.a.y, mr.b.x, mr.b.y, mr.c.x, mr.c.y, 0.0, 0.0};
    const bool ee = (int64_t)k >= e0;
    d3 wt = mk(m[R_W], m[R_W + 1], m[R_W + 2]);
    d3 gi = rec_coef(m, i, ee) * wt, gj = rec_coef(m, j, ee) * wt;
    add_outer(B, m[R_P22], gi, gj);
    if ((int64_t)k >= m0) {
        const double2* xp = reinterpret_cast<const double2*>(rec_extra + 8 * ((int64_t)k - m0));
        const double2 x0 = xp[0], x1 = xp[1], x2 = xp[2], x3 = xp[3];
        const double x[8] = {x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, x3.x, x3.y};
        d3 si = sq_slot(x, i), sj = sq_slot(x, j);
        add_outer(B, x[6], si, sj);
        add_outer(B, x[7], si, gj);
        add_outer(B, x[7], gi, sj);
    }
}

__device__ __forceinline__ void store_block(void* val, int dtype, int64_t nnzb, int64_t s, const double* B,
                                            bool tr = false) {
    if (dtype == GIPC_F64) {
        double* v = static_cast<double*>(val);
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c * nnzb + s] = B[tr ? 3 * (c % 3) + c / 3 : c];
    } else {
        float* v = static_cast<float*>(val);
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c * nnzb + s] = (float)B[tr ? 3 * (c % 3) + c / 3 : c];
    }
}

// LANES lanes per block row: each lane sums every LANES-th contribution of
// the row's diagonal list, then a fixed xor butterfly combines the lanes
// (same order on every run for a given LANES).  Rows are visited in `order`,
// or in storage order when it is null.
template <int LANES>
__global__ void __launch_bounds__(kBlock) k_rows_diag(int mode, int32_t V, const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ diag_slot,
                                                      const int64_t* __restrict__ cptr,
                                                      const uint32_t* __restrict__ contrib,
                                                      const double* __restrict__ rec_main,
                                                      const double* __restrict__ rec_extra,
                                                      const double* __restrict__ rec_a1, int64_t e0, int64_t m0,
                                                      const double* __restrict__ diag, double* __restrict__ grad,
                                                      double* __restrict__ ev, void* val, int dtype, int64_t nnzb) {
    const int64_t gi = xcd_block() * (kBlock / LANES) + threadIdx.x / LANES;
    const int lg = threadIdx.x % LANES;
    const bool valid = gi < V;
    const int64_t r = valid ? (order ? order[gi] : gi) : 0;
    double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    d3 g = mk(0, 0, 0);
    double e = 0.0;
    int32_t s = 0;
    if (valid) {
        s = diag_slot[r];
        const int64_t t0 = cptr[s], t1 = cptr[s + 1];
        // two of the lane's contributions per step: codes, then the whole
        // records, then the sums in list order
        for (int64_t t = t0 + lg; t < t1; t += 2 * LANES) {
            const bool two = t + LANES < t1;
            const uint32_t code[2] = {contrib[t], two ? contrib[t + LANES] : 0u};
            double m[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 0 || two) {
                    const double2* p = reinterpret_cast<const double2*>(rec_main + 8 * (int64_t)(code[u] >> 4));
                    const double2 w0 = p[0], w1 = p[1], w2 = p[2], w3 = p[3];
                    m[u][0] = w0.x; m[u][1] = w0.y; m[u][2] = w1.x; m[u][3] = w1.y;
                    m[u][4] = w2.x; m[u][5] = w2.y; m[u][6] = w3.x; m[u][7] = w3.y;
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u == 1 && !two) break;
                const uint32_t k = code[u] >> 4;
                const int i = (int)((code[u] >> 2) & 3u);
                const bool ee = (int64_t)k >= e0;
                const d3 gi = rec_coef(m[u], i, ee) * mk(m[u][R_W], m[u][R_W + 1], m[u][R_W + 2]);
                const double* x = (int64_t)k >= m0 ? rec_extra + 8 * ((int64_t)k - m0) : nullptr;
                if (mode & 1) {
                    g = g + m[u][R_A2] * gi;
                    if (i == 0) e += m[u][R_E];
                    if (x) g = g + rec_a1[(int64_t)k - m0] * sq_slot(x, i);
                }
                if (mode & 2) {
                    add_outer(B, m[u][R_P22], gi, gi);
                    if (x) {
                        const d3 si = sq_slot(x, i);
                        add_outer(B, x[6], si, si);
                        add_outer(B, x[7], si, gi);
                        add_outer(B, x[7], gi, si);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) {
        g.x += __shfl_xor(g.x, o, LANES);
        g.y += __shfl_xor(g.y, o, LANES);
        g.z += __shfl_xor(g.z, o, LANES);
        e += __shfl_xor(e, o, LANES);
#pragma unroll
        for (int c = 0; c < 9; ++c) B[c] += __shfl_xor(B[c], o, LANES);
    }
    if (!valid || lg != 0) return;
    if (mode & 1) {
        grad[3 * r + 0] = g.x;
        grad[3 * r + 1] = g.y;
        grad[3 * r + 2] = g.z;
        ev[r] = e;
    }
    if (mode & 2) {
        double dv = diag ? diag[r] : 0.0;
        B[0] += dv; B[4] += dv; B[8] += dv;
        // symmetric up to rounding: keep the upper triangle on both sides
        B[3] = B[1]; B[6] = B[2]; B[7] = B[5];
        store_block(val, dtype, nnzb, s, B);
    }
}

// Off-diagonal blocks, kOffLanes lanes per block row, rows visited in
// `order` (storage order when null).  The row's blocks above the diagonal
// are taken kOffLanes at a time (a window; lane l owns block l of it), and
// the window's contribution lists, which are contiguous, are spread evenly
// over the lanes: kOffLanes x kOffGroup contributions per step, each lane
// gathering kOffGroup records at once and writing its local 3x3 terms to
// LDS, after which every owner adds its own block's terms in list order.
// A block's sum is thus in list order whatever the launch shape, and no
// lane waits on a long list while the others idle (the lists of one row
// run from 1 to about 40 contributions).  Each block is stored, and stored
// transposed in the mirrored slot (the (c, r) list holds the same pairs
// with i and j swapped, so its sum is the transpose up to rounding;
// storing the transpose makes A exactly symmetric).  Blocks without a
// mirror (tslot -2) are only stored.
constexpr int kOffLanes = 32;
constexpr int kOffGroup = 2;

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_offdiag(int32_t V, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ diag_slot,
                                                    const int32_t* __restrict__ tslot,
                                                    const int64_t* __restrict__ cptr,
                                                    const uint32_t* __restrict__ contrib,
                                                    const double* __restrict__ rec_main,
                                                    const double* __restrict__ rec_extra, int64_t e0, int64_t m0,
                                                    void* val, int dtype, int64_t nnzb) {
    constexpr int L = kOffLanes, G = kOffGroup, C = L * G;
    __shared__ double lds[BLOCK / L][C][9];
    const int64_t gi = xcd_block() * (BLOCK / L) + threadIdx.x / L;
    if (gi >= V) return;  // the whole lane group (L divides the wavefront)
    const int lg = threadIdx.x % L;
    double(*T)[9] = lds[threadIdx.x / L];
    const int32_t r = order ? order[gi] : (int32_t)gi;
    const int32_t dg = diag_slot[r], end = row_ptr[r + 1];
    const int nbk = end - dg - 1;  // blocks above the diagonal
    for (int w0 = 0; w0 < nbk; w0 += L) {
        const bool own = w0 + lg < nbk;
        const int32_t s = dg + 1 + w0 + lg;
        int64_t o0 = 0, o1 = 0;
        if (own) {
            o0 = cptr[s];
            o1 = cptr[s + 1];
        }
        // the window's contributions (slot end is the next row's first)
        const int64_t W0 = cptr[dg + 1 + w0], W1 = cptr[dg + 1 + min(w0 + L, nbk)];
        double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t c0 = W0; c0 < W1; c0 += C) {
            uint32_t code[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int64_t t = c0 + u * L + lg;
                code[u] = t < W1 ? contrib[t] : 0u;
            }
            MainRec mr[G];
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (c0 + u * L + lg < W1) mr[u] = load_main(rec_main, code[u] >> 4);
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (c0 + u * L + lg < W1) {
                    double tm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                    add_block_rec(tm, mr[u], rec_extra, e0, m0, code[u] >> 4, (int)((code[u] >> 2) & 3u),
                                  (int)(code[u] & 3u));
#pragma unroll
                    for (int c = 0; c < 9; ++c) T[u * L + lg][c] = tm[c];
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
                    const double* tm = T[t - c0];
#pragma unroll
                    for (int c = 0; c < 9; ++c) B[c] += tm[c];
                }
            }
            // every owner has read the step's terms before the next writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (own) {
            store_block(val, dtype, nnzb, s, B);
            const int32_t t = tslot[s];
            if (t >= 0) store_block(val, dtype, nnzb, t, B, true);
        }
    }
}

// Expanded per-pair view of the staged list and the stored factors.
__global__ void __launch_bounds__(kBlock) k_pair_inspect(const int4* __restrict__ st_vid,
                                                         const int32_t* __restrict__ st_src,
                                                         const int32_t* __restrict__ smult, TypeRanges tr,
                                                         const double* __restrict__ rec_main,
                                                         const double* __restrict__ rec_extra,
                                                         const double* __restrict__ rec_a1,
                                                         const double* __restrict__ X, const double* __restrict__ XR,
                                                         DevParams pm, int32_t* src, int32_t* type, int32_t* vid,
                                                         int32_t* mult, double* energy, double* grad,
                                                         double* hess) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tr.off[8]) return;
    const int ft = type_of(k, tr);
    const int4 v4 = st_vid[k];
    const int64_t m0 = tr.off[FT_EEM], e0 = tr.off[FT_EE];
    const int32_t w = smult ? smult[k] : 1;
    if (src) src[k] = st_src[k];
    if (type) type[k] = ft;
    if (mult) mult[k] = w;
    if (vid) {
        vid[4 * k + 0] = v4.x; vid[4 * k + 1] = v4.y; vid[4 * k + 2] = v4.z; vid[4 * k + 3] = v4.w;
    }
    if (energy) {
        const int v[4] = {v4.x, v4.y, v4.z, v4.w};
        PairFactors o;
        eval_typed(ft, v, X, XR, pm, o);
        energy[k] = (double)w * o.E;
    }
    const int nv = ft_nverts(ft);
    if (grad) {
        const double* m = rec_main + 8 * k;
        for (int i = 0; i < 4; ++i) {
            d3 g = mk(0, 0, 0);
            if (i < nv) {
                g = m[R_A2] * (rec_coef(m, i, k >= e0) * mk(m[R_W], m[R_W + 1], m[R_W + 2]));
                if (k >= m0) {
                    const double* x = rec_extra + 8 * (k - m0);
                    g = g + rec_a1[k - m0] * sq_slot(x, i);
                }
            }
            grad[12 * k + 3 * i + 0] = g.x;
            grad[12 * k + 3 * i + 1] = g.y;
            grad[12 * k + 3 * i + 2] = g.z;
        }
    }
    if (hess) {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                if (i < nv && j < nv) add_block(B, rec_main, rec_extra, e0, m0, (uint32_t)k, i, j);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) hess[144 * k + (3 * i + a) * 12 + 3 * j + b] = B[3 * a + b];
            }
    }
}

}  // namespace

namespace {
template <int LANES>
hipError_t rows_launch(int mode, int32_t V, const int32_t* order, const int32_t* diag_slot, const int64_t* cptr,
                       const uint32_t* contrib, const double* rec_main, const double* rec_extra,
                       const double* rec_a1, int64_t e0,
                       int64_t m0, const double* diag, double* grad, double* ev, void* val, int dtype, int64_t nnzb,
                       hipStream_t s) {
    const int64_t nb = ((int64_t)V * LANES + kBlock - 1) / kBlock;
    k_rows_diag<LANES><<<(unsigned)nb, kBlock, 0, s>>>(mode, V, order, diag_slot, cptr, contrib, rec_main, rec_extra,
                                                       rec_a1, e0, m0, diag, grad, ev, val, dtype, nnzb);
    return hipGetLastError();
}

template <int BLOCK>
hipError_t offdiag_launch(int32_t V, const int32_t* order, const int32_t* row_ptr, const int32_t* diag_slot,
                          int64_t nnzb, const int32_t* tslot, const int64_t* cptr, const uint32_t* contrib,
                          const double* rec_main, const double* rec_extra, int64_t e0, int64_t m0, void* val,
                          int dtype, hipStream_t s) {
    const int64_t nb = ((int64_t)V * kOffLanes + BLOCK - 1) / BLOCK;
    k_offdiag<BLOCK><<<(unsigned)nb, BLOCK, 0, s>>>(V, order, row_ptr, diag_slot, tslot, cptr, contrib, rec_main,
                                                    rec_extra, e0, m0, val, dtype, nnzb);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_rows_diag(int mode, int32_t V, const int32_t* order, const int32_t* diag_slot, const int64_t* cptr,
                            const uint32_t* contrib, const double* rec_main, const double* rec_extra,
                            const double* rec_a1, int64_t e0,
                            int64_t m0, const double* diag, double* grad, double* ev, void* val, int dtype,
                            int64_t nnzb, int lanes, hipStream_t s) {
    if (V == 0) return hipSuccess;
#define ROWS(L) rows_launch<L>(mode, V, order, diag_slot, cptr, contrib, rec_main, rec_extra, rec_a1, e0, m0, diag, \
                               grad, ev, val, dtype, nnzb, s)
    switch (lanes) {
        case 4: return ROWS(4);
        case 8: return ROWS(8);
        case 32: return ROWS(32);
        default: return ROWS(16);
    }
#undef ROWS
}

hipError_t launch_offdiag(int32_t V, const int32_t* order, const int32_t* row_ptr, const int32_t* diag_slot,
                          int64_t nnzb, const int32_t* col_idx, const int32_t* tslot, const int64_t* cptr,
                          const uint32_t* contrib, const double* rec_main, const double* rec_extra, int64_t e0,
                          int64_t m0, void* val, int dtype, int waves, hipStream_t s) {
    (void)col_idx;
    if (V == 0 || nnzb == 0) return hipSuccess;
#define OFF(B) offdiag_launch<B>(V, order, row_ptr, diag_slot, nnzb, tslot, cptr, contrib, rec_main, rec_extra, e0, \
                                 m0, val, dtype, s)
    switch (waves) {
        case 1: return OFF(64);
        case 2: return OFF(128);
        case 8: return OFF(512);
        default: return OFF(256);
    }
#undef OFF
}

hipError_t launch_pair_inspect(const int4* st_vid, const int32_t* st_src, const int32_t* smult, TypeRanges tr,
                               const double* rec_main, const double* rec_extra, const double* rec_a1, const double* x,
                               const double* xr,
                               const DevParams& pm, int32_t* src, int32_t* type, int32_t* vid, int32_t* mult,
                               double* energy, double* grad, double* hess, hipStream_t s) {
    int64_t nb = (tr.off[8] + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_pair_inspect<<<(unsigned)nb, kBlock, 0, s>>>(st_vid, st_src, smult, tr, rec_main, rec_extra, rec_a1, x, xr, pm, src,
                                                  type, vid, mult, energy, grad, hess);
    return hipGetLastError();
}

}  // namespace gipc

// ---------------------------------------------------------------- matrix-free operator
//
// y = (diag (x) I3 + sum_k S_k^T H_k S_k) x straight from the compact
// factors of the last eval, without a BSR matrix (the paper's own PCG
// operator, supplement Sec. 6, with its local mat-vec written in factor
// form).  With s_k = grad f . x_k and t_k = grad sqrt(c) . x_k over the
// pair's stencil, H_k x_k = grad f (P22 s + P12 t) + grad sqrt(c) (P12 s + P11 t),
// so incidence (k, i) adds alpha_k c_i w~_k + beta_k gs_i to row v_i, with
// alpha = P22 s + P12 t, beta = P12 s + P11 t and gs = (-u, u, -v, v).
//
// Once per eval the vectors c_i w~_k of all incidences are laid out row by
// row, in the order of each row's diagonal contribution list (which holds
// exactly the row's incidences); then every product runs
//   pass 1 (one lane per staged pair): (alpha_k, beta_k);
//   pass 2 (kMfLanes lanes per row, rows in the spatial order): the row's
//     vectors and list codes stream in, alpha (for mollified pairs also
//     beta and u or v) is gathered per incidence; sums run in list order.

namespace gipc {
namespace {

constexpr int kMfLanes = 16;
constexpr int kMfBlock = 1024;
constexpr int kMfUnroll = 4;

__device__ __forceinline__ d3 ld3_at(const double* __restrict__ p, int64_t i) {
    return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}

// the bounded end of row r's diagonal list: the list holds exactly the
// row's incidences (stencils have distinct vertices); the bound keeps every
// access inside the row's run of the incidence array
__device__ __forceinline__ int64_t diag_end(int64_t t0, const int64_t* cptr, int32_t sl, const int64_t* inc_ptr,
                                            int64_t r) {
    return min(cptr[sl + 1], t0 + (inc_ptr[r + 1] - inc_ptr[r]));
}

// g[inc_ptr[r] + q] = c_i w~_k for the q-th incidence (k, i) of row r
__global__ void __launch_bounds__(kBlock) k_mf_coef(int32_t V, const int32_t* __restrict__ diag_slot,
                                                    const int64_t* __restrict__ cptr,
                                                    const uint32_t* __restrict__ contrib,
                                                    const int64_t* __restrict__ inc_ptr,
                                                    const double* __restrict__ rec_main, int64_t e0,
                                                    double* __restrict__ g) {
    const int64_t r = xcd_block() * (kBlock / kMfLanes) + threadIdx.x / kMfLanes;
    const int lg = threadIdx.x % kMfLanes;
    if (r >= V) return;
    const int32_t sl = diag_slot[r];
    const int64_t t0 = cptr[sl], base = inc_ptr[r];
    const int64_t t1 = diag_end(t0, cptr, sl, inc_ptr, r);
    for (int64_t t = t0 + lg; t < t1; t += kMfLanes) {
        const uint32_t code = contrib[t];
        const uint32_t k = code >> 4;
        const MainRec mr = load_main(rec_main, k);
        const double m[8] = {mr.a.x, mr.a.y, mr.b.x, mr.b.y, mr.c.x, mr.c.y, 0.0, 0.0};
        const d3 v = rec_coef(m, (int)((code >> 2) & 3u), (int64_t)k >= e0) * mk(m[R_W], m[R_W + 1], m[R_W + 2]);
        double* o = g + 3 * (base + (t - t0));
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
    }
}

__global__ void __launch_bounds__(kBlock) k_mf_pair(const int4* __restrict__ st_vid, TypeRanges tr,
                                                    const double* __restrict__ rec_main,
                                                    const double* __restrict__ rec_extra,
                                                    const double* __restrict__ x, double2* __restrict__ ab,
                                                    const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= tr.off[8]) return;
    const int ft = type_of(k, tr);
    const int nv = ft_nverts(ft);
    const int4 v4 = st_vid[k];
    const MainRec mr = load_main(rec_main, (uint32_t)k);
    const double m[8] = {mr.a.x, mr.a.y, mr.b.x, mr.b.y, mr.c.x, mr.c.y, 0.0, 0.0};
    const bool ee = k >= tr.off[FT_EE];
    d3 y = mk(0, 0, 0);
    d3 xs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        xs[i] = i < nv ? ld3(x, vslot(v4, i)) : mk(0, 0, 0);
        if (i < nv) y = y + rec_coef(m, i, ee) * xs[i];
    }
    const double s = dot(mk(m[R_W], m[R_W + 1], m[R_W + 2]), y);
    double a = m[R_P22] * s, b = 0.0;
    if (k >= tr.off[FT_EEM]) {
        const double* e = rec_extra + 8 * (k - tr.off[FT_EEM]);
        const double t = dot(mk(e[0], e[1], e[2]), xs[1] - xs[0]) + dot(mk(e[3], e[4], e[5]), xs[3] - xs[2]);
        a += e[7] * t;
        b = e[7] * s + e[6] * t;
    }
    ab[k] = make_double2(a, b);
}

// pass 2; with part, also one partial of x . y per workgroup (the PCG's p.q)
__global__ void __launch_bounds__(kMfBlock) k_mf_rows(int32_t V, const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ diag_slot,
                                                      const int64_t* __restrict__ cptr,
                                                      const uint32_t* __restrict__ contrib,
                                                      const int64_t* __restrict__ inc_ptr,
                                                      const double* __restrict__ g,
                                                      const double* __restrict__ rec_extra, int64_t m0,
                                                      const double2* __restrict__ ab,
                                                      const double* __restrict__ diag, const double* __restrict__ x,
                                                      double* __restrict__ y, double* __restrict__ part,
                                                      const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    __shared__ double lds[kMfBlock / 64];
    const int64_t gi = xcd_block() * (kMfBlock / kMfLanes) + threadIdx.x / kMfLanes;
    const int lg = threadIdx.x % kMfLanes;
    const bool valid = gi < V;
    const int64_t r = valid ? order[gi] : 0;
    d3 acc = mk(0, 0, 0);
    if (valid) {
        const int32_t sl = diag_slot[r];
        const int64_t t0 = cptr[sl], base = inc_ptr[r];
        const int64_t t1 = diag_end(t0, cptr, sl, inc_ptr, r);
        // kMfUnroll incidences' loads in flight per lane, summed in list order
        for (int64_t t = t0 + lg; t < t1; t += kMfUnroll * kMfLanes) {
            uint32_t code[kMfUnroll];
            double2 w[kMfUnroll];
            d3 gv[kMfUnroll];
#pragma unroll
            for (int q = 0; q < kMfUnroll; ++q) code[q] = t + q * kMfLanes < t1 ? contrib[t + q * kMfLanes] : 0u;
#pragma unroll
            for (int q = 0; q < kMfUnroll; ++q) {
                const bool in = t + q * kMfLanes < t1;
                w[q] = in ? ab[code[q] >> 4] : make_double2(0.0, 0.0);
                gv[q] = in ? ld3_at(g, base + (t + q * kMfLanes - t0)) : mk(0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < kMfUnroll; ++q) {
                acc = acc + w[q].x * gv[q];
                const int64_t k = code[q] >> 4;
                if (k >= m0 && t + q * kMfLanes < t1) {
                    const int i = (int)((code[q] >> 2) & 3u);
                    const double* e = rec_extra + 8 * (k - m0) + (i < 2 ? 0 : 3);
                    const double sb = (i & 1) ? w[q].y : -w[q].y;
                    acc = acc + sb * mk(e[0], e[1], e[2]);
                }
            }
        }
    }
#pragma unroll
    for (int o = kMfLanes / 2; o > 0; o >>= 1) {
        acc.x += __shfl_xor(acc.x, o, kMfLanes);
        acc.y += __shfl_xor(acc.y, o, kMfLanes);
        acc.z += __shfl_xor(acc.z, o, kMfLanes);
    }
    double d = 0.0;
    if (valid && lg == 0) {
        const d3 xr = ld3(x, (int)r);
        const double dv = diag ? diag[r] : 0.0;
        const d3 yr = acc + dv * xr;
        y[3 * r] = yr.x;
        y[3 * r + 1] = yr.y;
        y[3 * r + 2] = yr.z;
        d = dot(xr, yr);
    }
    if (part) {
        d = block_sum_n<kMfBlock>(d, lds);
        if (threadIdx.x == 0) part[blockIdx.x] = d;
    }
}

// inverse of every diagonal block diag_r I3 + sum_k H_k(i, i), for the
// block-Jacobi preconditioner of the matrix-free PCG (identity if singular)
__global__ void __launch_bounds__(kBlock) k_mf_diag_inverse(int32_t V, const int32_t* __restrict__ diag_slot,
                                                            const int64_t* __restrict__ cptr,
                                                            const uint32_t* __restrict__ contrib,
                                                            const double* __restrict__ rec_main,
                                                            const double* __restrict__ rec_extra, int64_t e0,
                                                            int64_t m0, const double* __restrict__ diag,
                                                            double* __restrict__ minv) {
    const int64_t r = (int64_t)blockIdx.x * (kBlock / kMfLanes) + threadIdx.x / kMfLanes;
    const int lg = threadIdx.x % kMfLanes;
    const bool valid = r < V;
    double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        const int32_t sl = diag_slot[r];
        const int64_t t0 = cptr[sl], t1 = cptr[sl + 1];
        for (int64_t t = t0 + lg; t < t1; t += kMfLanes) {
            const uint32_t code = contrib[t];
            add_block(B, rec_main, rec_extra, e0, m0, code >> 4, (int)((code >> 2) & 3u), (int)((code >> 2) & 3u));
        }
    }
#pragma unroll
    for (int o = kMfLanes / 2; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 9; ++c) B[c] += __shfl_xor(B[c], o, kMfLanes);
    if (!valid || lg != 0) return;
    const double dv = diag ? diag[r] : 0.0;
    B[0] += dv; B[4] += dv; B[8] += dv;
    B[3] = B[1]; B[6] = B[2]; B[7] = B[5];
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

}  // namespace

int64_t mf_num_parts(int32_t V) { return ((int64_t)V * kMfLanes + kMfBlock - 1) / kMfBlock; }

hipError_t launch_mf_apply(const MfView& m, const double* x, double* y, double* part, const PcgScalars* sc,
                           hipStream_t s) {
    if (m.dense) return launch_dense_apply(m, x, y, part, sc, s);
    if (m.V == 0) return hipSuccess;
    if (m.tr.off[8] > 0) {
        k_mf_pair<<<(unsigned)((m.tr.off[8] + kBlock - 1) / kBlock), kBlock, 0, s>>>(m.st_vid, m.tr, m.rec_main,
                                                                                     m.rec_extra, x, m.ab, sc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_mf_rows<<<(unsigned)mf_num_parts(m.V), kMfBlock, 0, s>>>(m.V, m.order, m.diag_slot, m.cptr, m.contrib,
                                                               m.inc_ptr, m.g, m.rec_extra, m.tr.off[FT_EEM], m.ab,
                                                               m.diag, x, y, part, sc);
    return hipGetLastError();
}

hipError_t launch_mf_coef(const MfView& m, double* g, hipStream_t s) {
    if (m.V == 0) return hipSuccess;
    const int64_t nb = ((int64_t)m.V * kMfLanes + kBlock - 1) / kBlock;
    k_mf_coef<<<(unsigned)nb, kBlock, 0, s>>>(m.V, m.diag_slot, m.cptr, m.contrib, m.inc_ptr, m.rec_main,
                                              m.tr.off[FT_EE], g);
    return hipGetLastError();
}

hipError_t launch_mf_diag_inverse(const MfView& m, double* minv, hipStream_t s) {
    if (m.dense) return launch_dense_diag_inverse(m, minv, s);
    if (m.V == 0) return hipSuccess;
    const int64_t e0 = m.tr.off[FT_EE], m0 = m.tr.off[FT_EEM];
    const int64_t nb = ((int64_t)m.V * kMfLanes + kBlock - 1) / kBlock;
    k_mf_diag_inverse<<<(unsigned)nb, kBlock, 0, s>>>(m.V, m.diag_slot, m.cptr, m.contrib, m.rec_main, m.rec_extra,
                                                      e0, m0, m.diag, minv);
    return hipGetLastError();
}

}  // namespace gipc
