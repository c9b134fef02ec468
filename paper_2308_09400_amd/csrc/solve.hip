// BSR SpMV, block-Jacobi preconditioned CG and a plain copy kernel.
//
// SpMV, FP64 with the pattern's row-start map (k_spmv_ent): one lane per
// block.  Wavefront g takes blocks 64g .. 64g+63, so every value, column and
// head-bit load is a full, aligned 64-lane stream with no row-pointer load
// ahead of it.  Each lane forms its block's product A_s x_col; a segmented
// suffix scan over the wavefront (segments cut at the row-start bits) leaves
// each row's sum over the wavefront in the lane of its first block.  Rows
// that end inside the wavefront are stored at once; a row that runs on into
// the next wavefront of the workgroup is finished in LDS from the per-wave
// pieces in wavefront order; the row holding the workgroup's last block, if
// it runs on past the workgroup, gets its remaining blocks from the last
// wavefront (a loop over 64-block chunks and a butterfly).  Every sum is in
// a fixed order, so the product is deterministic.  Measured on the ten-sheet
// matrix (17.4M blocks): 260 us against 296 us for the row kernel below;
// non-temporal value loads gave 260 against 271 us (the values are read
// once; the gathered x lines then stay in L2 longer), 8 wavefronts per
// workgroup beat 4 and 16, issuing the tail with the main loads was slower
// (281 us), as were two or four 64-block chunks per wavefront (288 us), a
// second fix-up launch for rows that cross wavefronts (278 us),
// non-temporal column loads (264 us) and a contiguous eighth of the
// workgroups per XCD (259 against 257 us in that run).  For FP32 blocks the
// row kernel stays (161 us against 163 us), and a descriptor without the map
// uses it too.
//
// SpMV by rows (k_spmv): G = 32 lanes per block row (two rows per
// wavefront); each lane walks every 32nd block of the row (component-major
// values, so the lanes of a row read consecutive values of each component),
// gathers x[col] (mostly cache hits), and the 32 partial 3-vectors are
// combined by a fixed xor-butterfly inside the lane group.  Deterministic.
// Rows of the contact matrices hold about 27 blocks, so most lanes issue all
// their loads at once.  Measured on the ten-sheet matrix, FP64: 4 / 8 / 16 /
// 32 / 64 lanes = 815 / 373 / 311 / 296 / 383 us; FP32: 8 / 16 / 32 lanes =
// 228 / 178 / 163 us.  At 8 lanes, non-temporal value loads (573 us) and
// XCD-contiguous row chunks (405 us) were slower; at 32 lanes, two to four
// rows per lane group (315-340 us) were too.
//
// PCG (Saad Alg. 9.1 with the inverse 3x3 diagonal blocks as
// preconditioner, the paper's simple block preconditioner of Sec. 7.2):
// every scalar (alpha, beta, residual norms, the stopping test) lives in
// device memory, so an iteration is six kernel launches without host
// round trips (product, p.q partials, alpha, update with the r.z and r.r
// partials, beta, p update); the host polls the "done" flag every 16
// iterations (once when rtol = 0).  The p.q partials are a pass of their
// own over p and q: formed in the product's epilogue (a block reduction
// at the end of every product workgroup) they cost 355 against 327 us per
// FP64 iteration on the ten-sheet matrix, and 254 against 223 us in FP32.
#include "internal.hpp"

namespace gipc {
namespace {

constexpr int kG = 32;  // lanes per block row

template <typename T>
__global__ void __launch_bounds__(kBlock) k_spmv(int32_t nrows, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                 int64_t nnzb, const T* __restrict__ x, T* __restrict__ y) {
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kG;
    const int lg = threadIdx.x % kG;
    T a0 = 0, a1 = 0, a2 = 0;
    if (row < nrows) {
        const int32_t e = rp[row + 1];
        for (int32_t s = rp[row] + lg; s < e; s += kG) {
            const int64_t c = ci[s];
            const T x0 = x[3 * c], x1 = x[3 * c + 1], x2 = x[3 * c + 2];
            a0 += val[s] * x0 + val[nnzb + s] * x1 + val[2 * nnzb + s] * x2;
            a1 += val[3 * nnzb + s] * x0 + val[4 * nnzb + s] * x1 + val[5 * nnzb + s] * x2;
            a2 += val[6 * nnzb + s] * x0 + val[7 * nnzb + s] * x1 + val[8 * nnzb + s] * x2;
        }
    }
#pragma unroll
    for (int o = kG / 2; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, kG);
        a1 += __shfl_xor(a1, o, kG);
        a2 += __shfl_xor(a2, o, kG);
    }
    if (row < nrows && lg == 0) {
        y[3 * row] = a0;
        y[3 * row + 1] = a1;
        y[3 * row + 2] = a2;
    }
}

__device__ __forceinline__ d3 ldv(const double* a, int64_t r) { return mk(a[3 * r], a[3 * r + 1], a[3 * r + 2]); }
__device__ __forceinline__ void stv(double* a, int64_t r, d3 v) {
    a[3 * r] = v.x; a[3 * r + 1] = v.y; a[3 * r + 2] = v.z;
}

// entry-parallel FP64 product (see the top of the file); inside the PCG
// (sc not null) it does nothing once the solve has stopped
constexpr int kEntWaves = 8;
constexpr int kEntBlock = kEntWaves * 64;

__global__ void __launch_bounds__(kEntBlock) k_spmv_ent(int64_t nnzb, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const double* __restrict__ val,
                                                        const unsigned long long* __restrict__ hm,
                                                        const int32_t* __restrict__ wrow,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        const PcgScalars* __restrict__ sc) {
    if (sc && sc->done) return;
    __shared__ double sf[kEntWaves][3], sl[kEntWaves][3], stail[3];
    __shared__ unsigned long long sm[kEntWaves], smn[kEntWaves];
    __shared__ int32_t srow[kEntWaves];
    const int64_t W = (nnzb + 63) >> 6;
    const int wi = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t w = (int64_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * kEntWaves + wi));
    if (w < W) {
        const int64_t s = (w << 6) + l;
        const bool ok = s < nnzb;
        const int64_t se = ok ? s : nnzb - 1;
        const int64_t c = ci[se];
        double v[9];  // read once: non-temporal, so the x lines stay in L2
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = __builtin_nontemporal_load(val + k * nnzb + se);
        const unsigned long long m = hm[w];                         // row starts in this wavefront
        const unsigned long long mn = (w + 1 < W) ? hm[w + 1] : 1ull;  // bit 0: the next one starts a row
        const int32_t r0 = wrow[w];
        const double x0 = x[3 * c], x1 = x[3 * c + 1], x2 = x[3 * c + 2];
        double q0 = v[0] * x0 + v[1] * x1 + v[2] * x2;
        double q1 = v[3] * x0 + v[4] * x1 + v[5] * x2;
        double q2 = v[6] * x0 + v[7] * x1 + v[8] * x2;
        if (!ok) q0 = q1 = q2 = 0.0;
        // segmented suffix scan: lane l ends with the sum over [l, e), e = next row start
        const unsigned long long above = m & ~((2ull << l) - 1ull);
        const int e = above ? __builtin_ctzll(above) : 64;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const double t0 = __shfl_down(q0, dd), t1 = __shfl_down(q1, dd), t2 = __shfl_down(q2, dd);
            if (l + dd < e) {
                q0 += t0;
                q1 += t1;
                q2 += t2;
            }
        }
        if (l == 0) {  // lane 0: the piece before the first row start
            sf[wi][0] = q0;
            sf[wi][1] = q1;
            sf[wi][2] = q2;
            sm[wi] = m;
            smn[wi] = mn;
        }
        if ((m >> l) & 1ull) {
            const int last = 63 - __builtin_clzll(m);
            const int32_t r = r0 + __popcll(m & ((2ull << l) - 1ull) & ~1ull);
            if ((l != last) || (mn & 1ull)) {  // the row ends in this wavefront
                y[3 * r] = q0;
                y[3 * r + 1] = q1;
                y[3 * r + 2] = q2;
            } else {
                sl[wi][0] = q0;
                sl[wi][1] = q1;
                sl[wi][2] = q2;
                srow[wi] = r;
            }
        }
        // the row of the workgroup's last block runs on past the workgroup
        if (wi == kEntWaves - 1 && !(mn & 1ull)) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            const int64_t end = rp[r0 + __popcll(m & ~1ull) + 1];
            for (int64_t t = ((w + 1) << 6) + l; t < end; t += 64) {
                const int64_t cc = ci[t];
                const double y0 = x[3 * cc], y1 = x[3 * cc + 1], y2 = x[3 * cc + 2];
                a0 += val[t] * y0 + val[nnzb + t] * y1 + val[2 * nnzb + t] * y2;
                a1 += val[3 * nnzb + t] * y0 + val[4 * nnzb + t] * y1 + val[5 * nnzb + t] * y2;
                a2 += val[6 * nnzb + t] * y0 + val[7 * nnzb + t] * y1 + val[8 * nnzb + t] * y2;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                a0 += __shfl_xor(a0, o);
                a1 += __shfl_xor(a1, o);
                a2 += __shfl_xor(a2, o);
            }
            if (l == 0) {
                stail[0] = a0;
                stail[1] = a1;
                stail[2] = a2;
            }
        }
    } else if (l == 0) {
        sm[wi] = 1ull;
        smn[wi] = 1ull;
    }
    __syncthreads();
    // thread t finishes the row opened by wavefront t's last row start when
    // it runs on: the pieces of the following wavefronts in order, then the
    // tail past the workgroup if it reaches that far
    if (threadIdx.x < kEntWaves) {
        const int t = threadIdx.x;
        if (sm[t] != 0ull && !(smn[t] & 1ull)) {
            double a0 = sl[t][0], a1 = sl[t][1], a2 = sl[t][2];
            bool ended = false;
            for (int k = t + 1; k < kEntWaves; ++k) {
                a0 += sf[k][0];
                a1 += sf[k][1];
                a2 += sf[k][2];
                if (sm[k] != 0ull || (smn[k] & 1ull)) {
                    ended = true;
                    break;
                }
            }
            if (!ended) {
                a0 += stail[0];
                a1 += stail[1];
                a2 += stail[2];
            }
            const int32_t r = srow[t];
            y[3 * r] = a0;
            y[3 * r + 1] = a1;
            y[3 * r + 2] = a2;
        }
    }
}

// streaming copy, 4 independent 16-byte loads in flight per lane
__global__ void __launch_bounds__(kBlock) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// streaming read of n 16-byte words, 4 independent loads in flight per lane
// (the chip's read bandwidth for roofline fractions); the xor of all words
// is stored only if it equals a fixed constant, which keeps every load live
// while writing nothing in practice
__global__ void __launch_bounds__(kBlock) k_read16(const uint4* __restrict__ src, int64_t n,
                                                   uint32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        acc ^= (a.x ^ a.y ^ a.z ^ a.w) ^ (b.x ^ b.y ^ b.z ^ b.w) ^ (c.x ^ c.y ^ c.z ^ c.w) ^ (d.x ^ d.y ^ d.z ^ d.w);
    }
    for (; i < n; i += stride) {
        const uint4 a = src[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

__global__ void k_copy1(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------- PCG
//
// Per iteration: q = A p with per-workgroup partials of p.q; one workgroup
// sums them in index order and forms alpha; the vector update writes
// partials of r.z and r.r; one workgroup forms beta and the stopping test;
// p = z + beta p.  Every kernel reads the device "done" flag first, so the
// host can enqueue many iterations at once.  Sums are in a fixed order and
// therefore bit-reproducible.

// the single-workgroup reductions of the PCG scalars use 1024 threads
constexpr int kRed = 1024;

// sum of part[0..n) by one workgroup of kRed threads: 8 independent
// accumulators per lane (loads in flight), then a fixed combination and the
// block butterfly
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int64_t n, double* lds) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t i = threadIdx.x;
    for (; i + 7 * kRed < n; i += 8 * kRed) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[i + u * kRed];
    }
    for (int u = 0; i < n; i += kRed, ++u) a[u & 7] += part[i];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    return block_sum_n<kRed>(s, lds);
}

// inverse of each row's diagonal block (cofactors, FP64); identity if singular
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bj_inverse(int32_t V, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                       int64_t nnzb, double* __restrict__ minv) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= V) return;
    double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t s = rp[r]; s < rp[r + 1]; ++s)
        if (ci[s] == r) {
            for (int c = 0; c < 9; ++c) A[c] = (double)val[c * nnzb + s];
            break;
        }
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    double* M = minv + 9 * r;
    if (!(fabs(det) > 0.0) || !isfinite(det)) {
        for (int c = 0; c < 9; ++c) M[c] = (c % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    double id = 1.0 / det;
    M[0] = c00 * id; M[1] = (A[2] * A[7] - A[1] * A[8]) * id; M[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    M[3] = c01 * id; M[4] = (A[0] * A[8] - A[2] * A[6]) * id; M[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    M[6] = c02 * id; M[7] = (A[1] * A[6] - A[0] * A[7]) * id; M[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

__device__ __forceinline__ d3 apply3(const double* M, d3 v) {
    return mk(M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
              M[6] * v.x + M[7] * v.y + M[8] * v.z);
}


// q = A p (kG lanes per row).  T is the matrix type: for FP32 matrices the
// product runs in FP32 on the FP32 copy pm of p and is widened to FP64 when
// stored.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_spmv(int32_t nrows, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                     int64_t nnzb, const T* __restrict__ pm, double* __restrict__ q,
                                                     const PcgScalars* __restrict__ sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kG;
    const int lg = threadIdx.x % kG;
    T a0 = 0, a1 = 0, a2 = 0;
    if (row < nrows) {
        const int32_t e = rp[row + 1];
        for (int32_t s = rp[row] + lg; s < e; s += kG) {
            const int64_t c = ci[s];
            const T x0 = pm[3 * c], x1 = pm[3 * c + 1], x2 = pm[3 * c + 2];
            a0 += val[s] * x0 + val[nnzb + s] * x1 + val[2 * nnzb + s] * x2;
            a1 += val[3 * nnzb + s] * x0 + val[4 * nnzb + s] * x1 + val[5 * nnzb + s] * x2;
            a2 += val[6 * nnzb + s] * x0 + val[7 * nnzb + s] * x1 + val[8 * nnzb + s] * x2;
        }
    }
#pragma unroll
    for (int o = kG / 2; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, kG);
        a1 += __shfl_xor(a1, o, kG);
        a2 += __shfl_xor(a2, o, kG);
    }
    if (row < nrows && lg == 0) stv(q, row, mk((double)a0, (double)a1, (double)a2));
}

// partials of p.q, one per workgroup of kBlock rows
__global__ void __launch_bounds__(kBlock) k_pcg_pq(int32_t V, const double* __restrict__ p,
                                                   const double* __restrict__ q, double* __restrict__ part,
                                                   const PcgScalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ double lds[kBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d = 0.0;
    if (i < V) d = dot(ldv(p, i), ldv(q, i));
    d = block_sum(d, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
}

__global__ void __launch_bounds__(kRed) k_pcg_alpha(const double* __restrict__ part, int64_t nb, PcgScalars* sc) {
    if (sc->done) return;
    __shared__ double lds[kRed / 64];
    double pq = sum_parts(part, nb, lds);
    if (threadIdx.x == 0) {
        sc->pq = pq;
        if (!(pq > 0.0)) {
            sc->breakdown = 1;
            sc->done = 1;
        } else {
            sc->alpha = sc->rz / pq;
        }
    }
}

// first: r = b - q, z = M^-1 r, p = z, partials (r.z, r.r, b.b);
// otherwise: x += alpha p, r -= alpha q, z = M^-1 r, partials (r.z, r.r)
__global__ void __launch_bounds__(kBlock) k_pcg_update(int first, int32_t V, const double* __restrict__ b,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ z, double* __restrict__ p,
                                                       const double* __restrict__ q, const double* __restrict__ minv,
                                                       double* __restrict__ part, const PcgScalars* __restrict__ sc) {
    if (!first && sc->done) return;
    __shared__ double lds[kBlock / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const double al = first ? 0.0 : sc->alpha;
    double rz = 0, rr = 0, bb = 0;
    if (i < V) {
        d3 rv;
        if (first) {
            d3 bv = ldv(b, i);
            rv = bv - ldv(q, i);
            bb = dot(bv, bv);
        } else {
            stv(x, i, ldv(x, i) + al * ldv(p, i));
            rv = ldv(r, i) - al * ldv(q, i);
        }
        d3 zv = apply3(minv + 9 * i, rv);
        stv(r, i, rv);
        stv(z, i, zv);
        if (first) stv(p, i, zv);
        rz = dot(rv, zv);
        rr = dot(rv, rv);
    }
    rz = block_sum(rz, lds);
    rr = block_sum(rr, lds);
    if (first) bb = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[gridDim.x + blockIdx.x] = rr;
        part[2 * gridDim.x + blockIdx.x] = bb;
    }
}

// all scalars zero (a kernel, not a memset, so the sequence stays free of
// memset nodes wherever it is recorded)
__global__ void k_pcg_reset(PcgScalars* sc) {
    if (threadIdx.x == 0) *sc = PcgScalars{};
}

// first: initial scalars; otherwise beta, the new r.z and the stopping test
// (delta = 0: r.r <= rtol2 b.b; delta = 1: r.z <= rtol2 r0.z0, the paper's
// termination, rtol2 then holding its tolerance unsquared)
__global__ void __launch_bounds__(kRed) k_pcg_beta(int first, const double* __restrict__ part, int64_t nb,
                                                     PcgScalars* sc, double rtol2, int maxit, int delta) {
    if (!first && sc->done) return;
    __shared__ double lds[kRed / 64];
    const double RZ = sum_parts(part, nb, lds), RR = sum_parts(part + nb, nb, lds);
    const double BB = first ? sum_parts(part + 2 * nb, nb, lds) : 0.0;
    if (threadIdx.x != 0) return;
    if (first) {
        sc->rz = RZ; sc->rr = RR; sc->bb = BB; sc->rtol2 = rtol2; sc->rz0 = RZ;
        sc->pq = 0; sc->alpha = 0; sc->beta = 0;
        sc->iters = 0; sc->breakdown = 0; sc->maxit = maxit; sc->delta = delta;
        sc->conv = delta ? (RZ <= rtol2 * RZ) : (RR <= rtol2 * BB);
        sc->done = sc->conv || maxit <= 0;
    } else {
        sc->beta = RZ / sc->rz;
        sc->rz = RZ;
        sc->rr = RR;
        sc->iters += 1;
        sc->conv = sc->delta ? (RZ <= sc->rtol2 * sc->rz0) : (RR <= sc->rtol2 * sc->bb);
        sc->done = sc->conv || sc->iters >= sc->maxit;
    }
}

// p = z + beta p (beta = 0 and z = p on the first call: plain copy), and
// the FP32 copy of p when the matrix is FP32
__global__ void __launch_bounds__(kBlock) k_pupdate(int64_t n, const double* __restrict__ z, double* __restrict__ p,
                                                    float* __restrict__ p32, const PcgScalars* __restrict__ sc,
                                                    int first) {
    if (!first && sc->done) return;
    const double be = first ? 0.0 : sc->beta;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double v = first ? p[i] : z[i] + be * p[i];
        p[i] = v;
        if (p32) p32[i] = (float)v;
    }
}

}  // namespace

// the entry-parallel product needs FP64 blocks and the pattern's row-start map
static bool spmv_by_entry(const gipc_bsr& A) {
    return A.dtype == GIPC_F64 && A.wave_head != nullptr && A.wave_row != nullptr && A.nnzb > 0;
}

static int64_t spmv_ent_blocks(int64_t nnzb) { return ((nnzb + 63) / 64 + kEntWaves - 1) / kEntWaves; }

hipError_t launch_spmv(const gipc_bsr& A, const void* x, void* y, hipStream_t s) {
    if (A.nbrows == 0) return hipSuccess;
    if (spmv_by_entry(A)) {
        k_spmv_ent<<<(unsigned)spmv_ent_blocks(A.nnzb), kEntBlock, 0, s>>>(
            A.nnzb, A.row_ptr, A.col_idx, static_cast<const double*>(A.val),
            reinterpret_cast<const unsigned long long*>(A.wave_head), A.wave_row, static_cast<const double*>(x),
            static_cast<double*>(y), nullptr);
        return hipGetLastError();
    }
    const int64_t threads = (int64_t)A.nbrows * kG;
    const unsigned nb = (unsigned)((threads + kBlock - 1) / kBlock);
    if (A.dtype == GIPC_F64)
        k_spmv<double><<<nb, kBlock, 0, s>>>(A.nbrows, A.row_ptr, A.col_idx, static_cast<const double*>(A.val), A.nnzb,
                                             static_cast<const double*>(x), static_cast<double*>(y));
    else
        k_spmv<float><<<nb, kBlock, 0, s>>>(A.nbrows, A.row_ptr, A.col_idx, static_cast<const float*>(A.val), A.nnzb,
                                            static_cast<const float*>(x), static_cast<float*>(y));
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    int64_t n16 = aligned ? bytes / 16 : 0;
    if (n16 > 0) {
        int64_t blocks = (n16 + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        k_copy16<<<(unsigned)blocks, kBlock, 0, s>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    }
    int64_t rest = bytes - 16 * n16;
    if (rest > 0) {
        int64_t blocks = (rest + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        k_copy1<<<(unsigned)blocks, kBlock, 0, s>>>(static_cast<const uint8_t*>(src) + 16 * n16,
                                                    static_cast<uint8_t*>(dst) + 16 * n16, rest);
    }
    return hipGetLastError();
}

hipError_t launch_read(const void* src, int64_t bytes, uint32_t* sink, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return hipSuccess;
    int64_t blocks = (n16 + 4 * kBlock - 1) / (4 * kBlock);
    if (blocks > 16384) blocks = 16384;
    k_read16<<<(unsigned)blocks, kBlock, 0, s>>>(static_cast<const uint4*>(src), n16, sink);
    return hipGetLastError();
}

// work buffers of one PCG solve
struct PcgWork {
    double *r, *z, *p, *q, *minv, *part;
    float* p32;
    PcgScalars* sc;
};

// the partials the reductions need: one per workgroup of kBlock rows (the
// matrix-free operator forms its p.q partials in its own layout)
static int64_t pcg_num_parts(const gipc_bsr& A, const MfView* mf) {
    const int32_t V = mf ? mf->V : A.nbrows;
    const int64_t nbv = (V + kBlock - 1) / kBlock;
    const int64_t nbs = mf ? mf_num_parts(V) : nbv;
    return nbv > nbs ? nbv : nbs;
}

// bytes of every PCG buffer, each rounded up to 256
static size_t pcg_round(size_t b) { return (b + 255) & ~size_t(255); }

size_t pcg_workspace_bytes(const gipc_bsr& A, const MfView* mf) {
    const int32_t V = mf ? mf->V : A.nbrows;
    const size_t n3 = 3 * (size_t)V;
    const bool f32 = !mf && A.dtype == GIPC_F32;
    return 4 * pcg_round(sizeof(double) * n3) + pcg_round(sizeof(double) * 9 * (size_t)V) +
           pcg_round(sizeof(double) * 3 * (size_t)pcg_num_parts(A, mf)) + pcg_round(sizeof(PcgScalars)) +
           (f32 ? pcg_round(sizeof(float) * n3) : 0);
}

static hipError_t pcg_exec(const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                           int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf,
                           const PcgWork& w, int delta, int* conv);

// the buffers carved out of one device range of pcg_workspace_bytes bytes
hipError_t pcg_run_in(void* ws, const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                      int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf) {
    const int32_t V = mf ? mf->V : A.nbrows;
    const size_t n3 = 3 * (size_t)V;
    const bool f32 = !mf && A.dtype == GIPC_F32;
    char* c = static_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* p = c;
        c += pcg_round(bytes);
        return p;
    };
    PcgWork w;
    w.r = reinterpret_cast<double*>(take(sizeof(double) * n3));
    w.z = reinterpret_cast<double*>(take(sizeof(double) * n3));
    w.p = reinterpret_cast<double*>(take(sizeof(double) * n3));
    w.q = reinterpret_cast<double*>(take(sizeof(double) * n3));
    w.minv = reinterpret_cast<double*>(take(sizeof(double) * 9 * (size_t)V));
    w.part = reinterpret_cast<double*>(take(sizeof(double) * 3 * (size_t)pcg_num_parts(A, mf)));
    w.sc = reinterpret_cast<PcgScalars*>(take(sizeof(PcgScalars)));
    w.p32 = f32 ? reinterpret_cast<float*>(take(sizeof(float) * n3)) : nullptr;
    return pcg_exec(A, b, x, rtol, maxit, iters, relres, breakdown, s, mf, w, 0, nullptr);
}

hipError_t pcg_run(gipc_ctx* ctx, const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                   int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf, int delta,
                   int* conv) {
    const int32_t V = mf ? mf->V : A.nbrows;
    const size_t n3 = 3 * (size_t)V;
    hipError_t e;
#define GIPC_TRY(x)                            \
    do {                                       \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    GIPC_TRY(ensure(ctx->r, sizeof(double) * n3));
    GIPC_TRY(ensure(ctx->z, sizeof(double) * n3));
    GIPC_TRY(ensure(ctx->p, sizeof(double) * n3));
    GIPC_TRY(ensure(ctx->q, sizeof(double) * n3));
    GIPC_TRY(ensure(ctx->minv, sizeof(double) * 9 * (size_t)V));
    GIPC_TRY(ensure(ctx->part, sizeof(double) * 3 * (size_t)pcg_num_parts(A, mf)));
    GIPC_TRY(ensure(ctx->scal, sizeof(PcgScalars)));
    const bool f32 = !mf && A.dtype == GIPC_F32;
    if (f32) GIPC_TRY(ensure(ctx->p32, sizeof(float) * n3));
#undef GIPC_TRY
    PcgWork w{as<double>(ctx->r), as<double>(ctx->z), as<double>(ctx->p), as<double>(ctx->q),
              as<double>(ctx->minv), as<double>(ctx->part), f32 ? as<float>(ctx->p32) : nullptr,
              as<PcgScalars>(ctx->scal)};
    return pcg_exec(A, b, x, rtol, maxit, iters, relres, breakdown, s, mf, w, delta, conv);
}

static hipError_t pcg_exec(const gipc_bsr& A, const double* b, double* x, double rtol, int32_t maxit,
                           int32_t* iters, double* relres, int* breakdown, hipStream_t s, const MfView* mf,
                           const PcgWork& w, int delta, int* conv) {
    const int32_t V = mf ? mf->V : A.nbrows;
    const int64_t n3 = 3 * (int64_t)V;
    const int64_t nbv = (V + kBlock - 1) / kBlock;  // row-parallel kernels
    const bool ent = !mf && spmv_by_entry(A);       // entry-parallel FP64 product
    const int64_t nbs = mf ? mf_num_parts(V) : nbv;  // p.q partials
    const unsigned nbrow = (unsigned)(((int64_t)V * kG + kBlock - 1) / kBlock);  // kG lanes per row
    hipError_t e;
#define GIPC_TRY(x)                            \
    do {                                       \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    const bool f32 = !mf && A.dtype == GIPC_F32;
    double *r = w.r, *z = w.z, *p = w.p, *q = w.q;
    double *minv = w.minv, *part = w.part;
    float* p32 = w.p32;
    PcgScalars* sc = w.sc;
    const unsigned nbn = (unsigned)((n3 + kBlock - 1) / kBlock);

    k_pcg_reset<<<1, 64, 0, s>>>(sc);
    // r = b - A x0 (for FP32 matrices through an FP32 copy of x0)
    if (mf) {
        GIPC_TRY(launch_mf_diag_inverse(*mf, minv, s));
        GIPC_TRY(launch_mf_apply(*mf, x, q, nullptr, nullptr, s));
    } else if (f32) {
        k_bj_inverse<float><<<(unsigned)nbv, kBlock, 0, s>>>(V, A.row_ptr, A.col_idx,
                                                             static_cast<const float*>(A.val), A.nnzb, minv);
        k_pupdate<<<nbn, kBlock, 0, s>>>(n3, nullptr, x, p32, sc, 1);  // FP32 copy of x0 in p32
        k_pcg_spmv<float><<<nbrow, kBlock, 0, s>>>(V, A.row_ptr, A.col_idx, static_cast<const float*>(A.val),
                                                   A.nnzb, p32, q, sc);
    } else {
        k_bj_inverse<double><<<(unsigned)nbv, kBlock, 0, s>>>(V, A.row_ptr, A.col_idx,
                                                              static_cast<const double*>(A.val), A.nnzb, minv);
        GIPC_TRY(launch_spmv(A, x, q, s));
    }
    k_pcg_update<<<(unsigned)nbv, kBlock, 0, s>>>(1, V, b, x, r, z, p, q, minv, part, sc);
    k_pcg_beta<<<1, kRed, 0, s>>>(1, part, nbv, sc, delta ? rtol : rtol * rtol, maxit, delta);
    if (f32) k_pupdate<<<nbn, kBlock, 0, s>>>(n3, z, p, p32, sc, 1);  // FP32 copy of p0
    GIPC_TRY(hipGetLastError());

    PcgScalars hs{};
    // nothing read back (no synchronisation, so the launches can be
    // captured) when the stopping test needs no host poll and the caller
    // asked for no counts
    const bool host = rtol > 0.0 || iters || relres || breakdown;
    const int32_t chunk = rtol > 0.0 ? 16 : (maxit > 0 ? maxit : 1);
    int32_t launched = 0;
    while (launched < maxit) {
        int32_t m = maxit - launched < chunk ? maxit - launched : chunk;
        for (int32_t it = 0; it < m; ++it) {
            if (mf) {
                GIPC_TRY(launch_mf_apply(*mf, p, q, part, sc, s));
            } else {
                if (f32)
                    k_pcg_spmv<float><<<nbrow, kBlock, 0, s>>>(V, A.row_ptr, A.col_idx,
                                                               static_cast<const float*>(A.val), A.nnzb, p32, q, sc);
                else if (ent)
                    k_spmv_ent<<<(unsigned)spmv_ent_blocks(A.nnzb), kEntBlock, 0, s>>>(
                        A.nnzb, A.row_ptr, A.col_idx, static_cast<const double*>(A.val),
                        reinterpret_cast<const unsigned long long*>(A.wave_head), A.wave_row, p, q, sc);
                else
                    k_pcg_spmv<double><<<nbrow, kBlock, 0, s>>>(V, A.row_ptr, A.col_idx,
                                                                static_cast<const double*>(A.val), A.nnzb, p, q, sc);
                k_pcg_pq<<<(unsigned)nbv, kBlock, 0, s>>>(V, p, q, part, sc);
            }
            k_pcg_alpha<<<1, kRed, 0, s>>>(part, nbs, sc);
            k_pcg_update<<<(unsigned)nbv, kBlock, 0, s>>>(0, V, b, x, r, z, p, q, minv, part, sc);
            k_pcg_beta<<<1, kRed, 0, s>>>(0, part, nbv, sc, 0.0, 0, 0);
            k_pupdate<<<nbn, kBlock, 0, s>>>(n3, z, p, p32, sc, 0);
        }
        GIPC_TRY(hipGetLastError());
        launched += m;
        if (!host) break;  // rtol = 0: one chunk of maxit iterations
        GIPC_TRY(hipMemcpyAsync(&hs, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
        GIPC_TRY(hipStreamSynchronize(s));
        if (hs.done) break;
    }
    if (maxit <= 0 && host) {
        GIPC_TRY(hipMemcpyAsync(&hs, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
        GIPC_TRY(hipStreamSynchronize(s));
    }
#undef GIPC_TRY
    if (iters) *iters = hs.iters;
    if (relres) *relres = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : 0.0;
    if (breakdown) *breakdown = hs.breakdown;
    if (conv) *conv = hs.conv;
    return hipSuccess;
}

}  // namespace gipc
