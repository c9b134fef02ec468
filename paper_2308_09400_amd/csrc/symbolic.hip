// Symbolic assembly: the block pattern of diag + sum_k S_k^T H_k S_k (the
// matrix decomposition of supplement Sec. 6 read in reverse: every local
// block (i, j) of pair k lands in global block (v_i, v_j)).
//
//  1. incidence counts per vertex (integer atomics: counts are exact);
//  2. exclusive scans -> per-vertex incidence and contribution offsets;
//  3. incidence scatter (order inside a vertex is irrelevant: step 4 sorts):
//     one 16-byte record per incidence, (k << 2 | i, the vertices of the
//     pair's other slots in slot order, -1 past the stencil);
//  4. per block row, the keys (column, k, i, j) of all local blocks landing
//     in that row are sorted: one wavefront per row with the keys in
//     registers (bitonic network over cross-lane shuffles) for rows of up to
//     128 incidences, one workgroup per row with the keys in LDS for the
//     rest; the sorted codes are the row's contribution lists, grouped by
//     column, and the row's distinct columns with the offset of each one's
//     first contribution are written compactly at the row's start;
//  5. scan of the per-row column counts -> row_ptr;
//  6. per row, the compact column list gives col_idx and the start of each
//     block's contribution list.
// A contribution code is k << 4 | i << 2 | j (staged pair k, local block i, j).
#include "internal.hpp"

namespace gipc {
namespace {

// Lanes of the wavefront with equal keys (key, key2) form a group led by its
// lowest lane, wherever they sit in the wavefront: one atomic per group
// instead of one per lane.  The loop runs once per distinct key (the
// pending mask is the same in every lane).
struct WaveGroup {
    int leader;                  // -1 for lanes not in
    unsigned long long members;  // the group's lanes
};

__device__ __forceinline__ WaveGroup wave_group(int key, int key2, bool in) {
    WaveGroup g{-1, 0ull};
    unsigned long long pending = __ballot(in);
    while (pending) {
        const int l = __ffsll((long long)pending) - 1;
        const int a = __shfl(key, l, 64), b = __shfl(key2, l, 64);
        const bool same = in && key == a && key2 == b;
        const unsigned long long grp = __ballot(same);
        if (same) {
            g.leader = l;
            g.members = grp;
        }
        pending &= ~grp;
    }
    return g;
}

__global__ void __launch_bounds__(kBlock) k_sym_count(const int4* __restrict__ st_vid, TypeRanges tr,
                                                      int32_t* __restrict__ deg, int32_t* __restrict__ kcount) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = k < tr.off[8];
    const int nv = in ? ft_nverts(type_of(k, tr)) : 0;
    const int4 v = in ? st_vid[k] : make_int4(-1, -1, -1, -1);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int vi = vslot(v, i);
        const bool valid = i < nv;
        const WaveGroup g = wave_group(valid ? vi : -1, nv, valid);
        if (valid && g.leader == lane) {
            const int n = __popcll(g.members);
            atomicAdd(&deg[vi], n);
            atomicAdd(&kcount[vi], n * nv);
        }
    }
}

// every incidence carries the rest of its pair's stencil, so the row sort
// streams one record per incidence instead of gathering the staged list
__global__ void __launch_bounds__(kBlock) k_sym_scatter(const int4* __restrict__ st_vid, TypeRanges tr,
                                                        const int64_t* __restrict__ inc_ptr,
                                                        int32_t* __restrict__ fill, int4* __restrict__ incr) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = k < tr.off[8];
    const int nv = in ? ft_nverts(type_of(k, tr)) : 0;
    const int4 v = in ? st_vid[k] : make_int4(-1, -1, -1, -1);
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int vi = vslot(v, i);
        const bool valid = i < nv;
        const WaveGroup g = wave_group(valid ? vi : -1, 0, valid);
        int base = 0;
        if (valid && g.leader == lane) base = atomicAdd(&fill[vi], __popcll(g.members));
        base = __shfl(base, valid ? g.leader : lane, 64);
        if (valid) {
            const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const int64_t at = inc_ptr[vi] + base + __popcll(g.members & below);
            int o[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int j = m < i ? m : m + 1;
                o[m] = j < nv ? vslot(v, j) : -1;
            }
            incr[at] = make_int4((int)(((uint32_t)k << 2) | (uint32_t)i), o[0], o[1], o[2]);
        }
    }
}

// slot j != i of an incidence record: its m-th other slot
__device__ __forceinline__ int other_slot(int j, int i) { return j < i ? j : j - 1; }

__device__ __forceinline__ int rec_other(const int4& rec, int m) { return m == 0 ? rec.y : (m == 1 ? rec.z : rec.w); }

constexpr int kWaveM = 8;                    // keys per lane in the wavefront sort
constexpr int kWaveN = 64 * kWaveM;          // 512 keys per row
constexpr int kWaveIncidences = kWaveN / 4;  // 128 incidences of 4 key slots

// sort of one row's keys in LDS by a whole workgroup (rows with more than
// kWaveIncidences incidences)
__device__ void rowsort_lds(int r, const int64_t* __restrict__ inc_ptr, const int4* __restrict__ incr,
                            const TypeRanges& tr, const int64_t* __restrict__ kptr,
                            uint32_t* __restrict__ contrib, int32_t* __restrict__ kcol, int32_t* __restrict__ kbeg,
                            int32_t* __restrict__ ncols) {
    extern __shared__ unsigned long long keys[];
    __shared__ int32_t wcnt[kBlock / 64];
    const int64_t start = inc_ptr[r];
    const int n = (int)(inc_ptr[r + 1] - start);
    unsigned N = 1;
    while (N < 4u * (unsigned)n) N <<= 1;
    for (unsigned t = threadIdx.x; t < N; t += kBlock) keys[t] = ~0ull;
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += kBlock) {
        const int4 rec = incr[start + t];
        const uint32_t code = (uint32_t)rec.x;
        const uint32_t k = code >> 2, i = code & 3u;
        const int nv = ft_nverts(type_of(k, tr));
        for (int j = 0; j < nv; ++j) {
            const int col = j == (int)i ? r : rec_other(rec, other_slot(j, (int)i));
            keys[4 * t + j] = ((unsigned long long)(uint32_t)col << 32) | (unsigned long long)((k << 4) | (i << 2) | (uint32_t)j);
        }
    }
    __syncthreads();
    // bitonic sort, ascending
    for (unsigned kk = 2; kk <= N; kk <<= 1) {
        for (unsigned j = kk >> 1; j > 0; j >>= 1) {
            for (unsigned t = threadIdx.x; t < N / 2; t += kBlock) {
                unsigned i = (t / j) * (2 * j) + (t % j), l = i + j;
                unsigned long long a = keys[i], b = keys[l];
                bool up = (i & kk) == 0;
                if ((a > b) == up) {
                    keys[i] = b;
                    keys[l] = a;
                }
            }
            __syncthreads();
        }
    }
    const int64_t base = kptr[r];
    const int K = (int)(kptr[r + 1] - base);
    // the first contribution of every column, ranked in order (chunks of a
    // workgroup: wave ballots, then the waves' counts in order)
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int carry = 0;
    for (int c0 = 0; c0 < K; c0 += kBlock) {
        const int t = c0 + (int)threadIdx.x;
        bool first = false;
        int col = 0;
        if (t < K) {
            const unsigned long long key = keys[t];
            col = (int)(key >> 32);
            contrib[base + t] = (uint32_t)key;
            first = t == 0 || (int)(keys[t - 1] >> 32) != col;
        }
        const unsigned long long m = __ballot(first);
        if (lane == 0) wcnt[wid] = __popcll(m);
        __syncthreads();
        int before = carry, total = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wid) before += wcnt[w];
            total += wcnt[w];
        }
        if (first) {
            const int rank = before + __popcll(m & __lanemask_lt());
            kcol[base + rank] = col;
            kbeg[base + rank] = t;
        }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) ncols[r] = carry;
}

// value of lane (lane ^ D) for a compile-time lane distance D.  Distances 1
// and 2 are DPP quad permutations and 4 and 8 two DPP row shifts (lane
// i <- i + D and i <- i - D within its row of 16, picked by bit D of the
// lane), all plain VALU moves; 16 is an LDS swizzle in bitmask mode (no
// memory access); 32 goes through ds_bpermute.  The sort network is bound
// by these exchanges, and the crossbar form of all of them was its limit.
template <int D>
__device__ __forceinline__ int xor_lanes32(int v) {
    if constexpr (D == 1) {
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (D == 2) {
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (D == 4 || D == 8) {
        const int up = __builtin_amdgcn_mov_dpp(v, 0x100 + D, 0xF, 0xF, false);  // row_shl:D
        const int dn = __builtin_amdgcn_mov_dpp(v, 0x110 + D, 0xF, 0xF, false);  // row_shr:D
        return (__lane_id() & D) ? dn : up;
    } else if constexpr (D == 16) {
        return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // and 0x1f, or 0, xor 16
    } else {
        return __shfl_xor(v, D, 64);
    }
}

template <int D>
__device__ __forceinline__ unsigned long long xor_lanes64(unsigned long long v) {
    const int lo = xor_lanes32<D>((int)(uint32_t)v), hi = xor_lanes32<D>((int)(uint32_t)(v >> 32));
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ unsigned long long xor_lanes64(unsigned long long v, int d) {
    switch (d) {  // d is a constant once the network is unrolled
        case 1: return xor_lanes64<1>(v);
        case 2: return xor_lanes64<2>(v);
        case 4: return xor_lanes64<4>(v);
        case 8: return xor_lanes64<8>(v);
        case 16: return xor_lanes64<16>(v);
        default: return xor_lanes64<32>(v);
    }
}

__device__ __forceinline__ unsigned long long shfl_up64(unsigned long long v, int d) {
    const int lo = __shfl_up((int)(uint32_t)v, d, 64), hi = __shfl_up((int)(uint32_t)(v >> 32), d, 64);
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint32_t xor_lanes_any(uint32_t v, int d) {
    switch (d) {  // d is a constant once the network is unrolled
        case 1: return (uint32_t)xor_lanes32<1>((int)v);
        case 2: return (uint32_t)xor_lanes32<2>((int)v);
        case 4: return (uint32_t)xor_lanes32<4>((int)v);
        case 8: return (uint32_t)xor_lanes32<8>((int)v);
        case 16: return (uint32_t)xor_lanes32<16>((int)v);
        default: return (uint32_t)xor_lanes32<32>((int)v);
    }
}

__device__ __forceinline__ unsigned long long xor_lanes_any(unsigned long long v, int d) { return xor_lanes64(v, d); }

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Ascending bitonic sort of the 64 M elements e = M lane + q of a wavefront:
// shuffles across lanes for distances >= M, swaps inside the lane below.
template <int M, typename K>
__device__ __forceinline__ void bitonic_wave(K (&key)[M]) {
    constexpr int N = 64 * M;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int kk = 2; kk <= N; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= M) {
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const int e = M * lane + q;
                    const K o = xor_lanes_any(key[q], j / M);
                    // this element keeps the smaller key iff it is the lower
                    // one of an ascending pair or the upper one of a descending
                    const bool take_min = ((e & kk) == 0) == ((e & j) == 0);
                    if ((o < key[q]) == take_min) key[q] = o;
                }
            } else {
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    if ((q & j) == 0) {
                        const int l = q | j;
                        const int e = M * lane + q;
                        const bool up = (e & kk) == 0;
                        const K a = key[q], b = key[l];
                        if ((a > b) == up) {
                            key[q] = b;
                            key[l] = a;
                        }
                    }
                }
            }
        }
    }
}

// Second half of the wavefront row sort: the T keys (column << 32 | code) of
// the slots j != i, packed in lk, sorted with M keys per lane (64 M >= T),
// merged with the row's n own-column contributions (dsort: their codes
// sorted, element MD lane + q).  A single sort by (column, code) would put
// the own column r between the columns below and above it; that is the list
// written here: codes to contrib, each column's first offset to kbeg, the
// columns to kcol, all at the row's contribution offset.
template <int M>
__device__ __forceinline__ void rowsort_main(int64_t r, int n, int T, int MD, const uint32_t (&dsort)[2],
                                             const unsigned long long* lk, const int64_t* __restrict__ kptr,
                                             uint32_t* __restrict__ contrib, int32_t* __restrict__ kcol,
                                             int32_t* __restrict__ kbeg, int32_t* __restrict__ ncols) {
    const int lane = threadIdx.x & 63;
    unsigned long long key[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const int e = M * lane + q;
        key[q] = e < T ? lk[e] : ~0ull;
    }
    bitonic_wave<M>(key);
    const int64_t base = kptr[r];
    const int ri = (int)r;
    // L = keys with a column below r (a prefix, the keys being sorted)
    int lt = 0;
#pragma unroll
    for (int q = 0; q < M; ++q) lt += (M * lane + q < T && (int)(key[q] >> 32) < ri) ? 1 : 0;
    const int L = wave_sum_i(lt);
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const int e = M * lane + q;
        if (e < T) contrib[base + (e < L ? e : e + n)] = (uint32_t)key[q];
    }
    for (int q = 0; q < MD; ++q) {
        const int e = MD * lane + q;
        if (e < n) contrib[base + L + e] = dsort[q];
    }
    // the first key of every column: flags, this lane's count, its rank
    // among all (exclusive scan of the counts over the lanes)
    const unsigned long long prev_last = shfl_up64(key[M - 1], 1);
    bool first[M];
    int c = 0, cb = 0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        const int e = M * lane + q;
        first[q] = false;
        if (e < T) {
            const int col = (int)(key[q] >> 32);
            const unsigned long long pk = q == 0 ? prev_last : key[q > 0 ? q - 1 : 0];
            first[q] = e == 0 || (int)(pk >> 32) != col;
            c += first[q] ? 1 : 0;
            cb += (first[q] && col < ri) ? 1 : 0;
        }
    }
    int pre = c;  // inclusive scan over the lanes, then exclusive
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(pre, o, 64);
        if (lane >= o) pre += v;
    }
    const int total = __shfl(pre, 63, 64);
    const int below = wave_sum_i(cb);  // columns below r
    int rank = pre - c;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        if (first[q]) {
            const int e = M * lane + q;
            const int col = (int)(key[q] >> 32);
            const bool lo = col < ri;
            kcol[base + rank + (lo ? 0 : 1)] = col;
            kbeg[base + rank + (lo ? 0 : 1)] = lo ? e : e + n;
            ++rank;
        }
    }
    if (lane == 0) {
        kcol[base + below] = ri;
        kbeg[base + below] = L;
        ncols[r] = total + 1;
    }
}

// one wavefront per row, keys in registers.  The slot j = i of an incidence
// (k, i) is the row's own column, so those n keys are sorted as 32-bit codes
// apart from the rest, and only the other slots (sum of nv - 1 over the
// incidences, packed, not 4 slots per incidence) go through the 64-bit
// network: the ten-sheet rows (about 54 incidences, 2.2 other slots each)
// sort 128 keys instead of 256.  Rows with more than kWaveIncidences
// incidences are appended to `big` for the workgroup sort.
__global__ void __launch_bounds__(kBlock) k_sym_rowsort_wave(int32_t V, const int64_t* __restrict__ inc_ptr,
                                                             const int4* __restrict__ incr, TypeRanges tr,
                                                             const int64_t* __restrict__ kptr,
                                                             uint32_t* __restrict__ contrib,
                                                             int32_t* __restrict__ kcol, int32_t* __restrict__ kbeg,
                                                             int32_t* __restrict__ ncols,
                                                             int32_t* __restrict__ big,
                                                             unsigned long long* __restrict__ nbig) {
    __shared__ unsigned long long skeys[kBlock / 64][kWaveN];
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (r >= V) return;  // the whole wavefront
    const int64_t start = inc_ptr[r];
    const int n = (int)(inc_ptr[r + 1] - start);
    if (n == 0) {
        if (lane == 0) ncols[r] = 1;  // the diagonal block alone
        return;
    }
    if (n > kWaveIncidences) {
        if (lane == 0) big[atomicAdd(nbig, 1ull)] = (int32_t)r;
        return;
    }
    // incidences t = lane and lane + 64: the own-column code (slot j = i) as
    // a 32-bit key, the other nv - 1 slots as (column, code) keys packed in
    // incidence order into this wavefront's LDS row
    unsigned long long* lk = skeys[threadIdx.x >> 6];
    uint32_t dkey[2] = {~0u, ~0u};
    int o[2] = {0, 0};
    uint32_t kc[2] = {0u, 0u};
    int4 vv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        vv[h] = make_int4(0, -1, -1, -1);
        if (t < n) {
            vv[h] = incr[start + t];
            const uint32_t code = (uint32_t)vv[h].x;
            const uint32_t k = code >> 2, i = code & 3u;
            o[h] = ft_nverts(type_of(k, tr)) - 1;
            kc[h] = code;
            dkey[h] = (k << 4) | (i << 2) | i;
        }
    }
    int pos[2], T = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int sc = o[h];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(sc, d, 64);
            if (lane >= d) sc += v;
        }
        pos[h] = T + sc - o[h];
        T += __shfl(sc, 63, 64);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (o[h] > 0) {
            const uint32_t k = kc[h] >> 2, i = kc[h] & 3u;
            int p = pos[h];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j <= o[h] && j != (int)i)
                    lk[p++] = ((unsigned long long)(uint32_t)rec_other(vv[h], other_slot(j, (int)i)) << 32) |
                              (unsigned long long)((k << 4) | (i << 2) | (uint32_t)j);
        }
    }
    // the own-column codes, sorted while the LDS writes land
    uint32_t dsort[2] = {~0u, ~0u};
    int MD = 1;
    if (n <= 64) {
        uint32_t d1[1] = {dkey[0]};
        bitonic_wave<1>(d1);
        dsort[0] = d1[0];
    } else {
        uint32_t d2[2] = {dkey[0], dkey[1]};
        bitonic_wave<2>(d2);
        dsort[0] = d2[0];
        dsort[1] = d2[1];
        MD = 2;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the branch is uniform in the wavefront
    if (T <= 64) rowsort_main<1>(r, n, T, MD, dsort, lk, kptr, contrib, kcol, kbeg, ncols);
    else if (T <= 128) rowsort_main<2>(r, n, T, MD, dsort, lk, kptr, contrib, kcol, kbeg, ncols);
    else if (T <= 256) rowsort_main<4>(r, n, T, MD, dsort, lk, kptr, contrib, kcol, kbeg, ncols);
    else rowsort_main<8>(r, n, T, MD, dsort, lk, kptr, contrib, kcol, kbeg, ncols);
}

// one workgroup per listed row (grid-stride over the list of rows the
// wavefront kernel left: more than kWaveIncidences incidences)
__global__ void __launch_bounds__(kBlock) k_sym_rowsort(const int32_t* __restrict__ rows,
                                                        const unsigned long long* __restrict__ nrows,
                                                        const int64_t* __restrict__ inc_ptr,
                                                        const int4* __restrict__ incr, TypeRanges tr,
                                                        const int64_t* __restrict__ kptr,
                                                        uint32_t* __restrict__ contrib, int32_t* __restrict__ kcol,
                                                        int32_t* __restrict__ kbeg, int32_t* __restrict__ ncols) {
    const int64_t nr = (int64_t)*nrows;
    for (int64_t idx = blockIdx.x; idx < nr; idx += gridDim.x) {
        rowsort_lds(rows[idx], inc_ptr, incr, tr, kptr, contrib, kcol, kbeg, ncols);
        __syncthreads();
    }
}

// zeroes n 64-bit words (a kernel rather than a memset, so the build may be
// recorded in a graph)
__global__ void __launch_bounds__(kBlock) k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// one wavefront per row: the row's compact column list (written by the row
// sort at the row's contribution offset) gives col_idx, the start of each
// block's list (cptr), the block's row and the diagonal slot
__global__ void __launch_bounds__(kBlock) k_sym_fill(int32_t V, const int64_t* __restrict__ kptr,
                                                     const int32_t* __restrict__ kcol,
                                                     const int32_t* __restrict__ kbeg,
                                                     const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
                                                     int64_t* __restrict__ cptr, int32_t* __restrict__ slot_row,
                                                     int32_t* __restrict__ diag_slot,
                                                     unsigned long long* __restrict__ whead,
                                                     int32_t* __restrict__ wrow, int64_t nnzb) {
    const int lane = threadIdx.x & 63;
    const int64_t r64 = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (r64 >= V) return;  // the whole wavefront
    const int r = (int)r64;
    const int64_t base = kptr[r];
    const int K = (int)(kptr[r + 1] - base);
    const int rp = row_ptr[r];
    if (lane == 0 && r == V - 1) cptr[nnzb] = kptr[V];
    // per 64-block wave of the product: head bit of the row's first block,
    // row of every block whose index is a multiple of 64
    if (lane == 0) atomicOr(whead + (rp >> 6), 1ull << (rp & 63));
    if (K == 0) {
        if (lane == 0) {
            col_idx[rp] = r;
            cptr[rp] = base;
            slot_row[rp] = r;
            diag_slot[r] = rp;
            if ((rp & 63) == 0) wrow[rp >> 6] = r;
        }
        return;
    }
    const int nc = row_ptr[r + 1] - rp;
    for (int j = lane; j < nc; j += 64) {
        const int col = kcol[base + j];
        const int s = rp + j;
        col_idx[s] = col;
        cptr[s] = base + kbeg[base + j];
        slot_row[s] = r;
        if (col == r) diag_slot[r] = s;
        if ((s & 63) == 0) wrow[s >> 6] = r;
    }
}

}  // namespace

hipError_t launch_sym_count(const int4* st_vid, TypeRanges tr, int32_t* deg, int32_t* kcount, hipStream_t s) {
    int64_t nb = (tr.off[8] + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_sym_count<<<(unsigned)nb, kBlock, 0, s>>>(st_vid, tr, deg, kcount);
    return hipGetLastError();
}

hipError_t launch_sym_scatter(const int4* st_vid, TypeRanges tr, const int64_t* inc_ptr, int32_t* fill,
                              int4* incr, hipStream_t s) {
    int64_t nb = (tr.off[8] + kBlock - 1) / kBlock;
    if (nb == 0) return hipSuccess;
    k_sym_scatter<<<(unsigned)nb, kBlock, 0, s>>>(st_vid, tr, inc_ptr, fill, incr);
    return hipGetLastError();
}

hipError_t launch_sym_rowsort(int32_t V, int32_t max_deg, const int64_t* inc_ptr, const int4* incr,
                              TypeRanges tr, const int64_t* kptr, uint32_t* contrib,
                              int32_t* kcol, int32_t* kbeg, int32_t* ncols, int32_t* big, int64_t* nbig,
                              hipStream_t s) {
    if (V == 0) return hipSuccess;
    unsigned long long* nb = reinterpret_cast<unsigned long long*>(nbig);
    const unsigned blocks = (unsigned)(((int64_t)V + kBlock / 64 - 1) / (kBlock / 64));
    k_sym_rowsort_wave<<<blocks, kBlock, 0, s>>>(V, inc_ptr, incr, tr, kptr, contrib, kcol, kbeg, ncols, big, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || max_deg <= kWaveIncidences) return e;
    unsigned N = 64;
    while (N < 4u * (unsigned)max_deg) N <<= 1;
    const size_t lds = sizeof(unsigned long long) * N;
    const unsigned grid = (unsigned)(V < 2048 ? V : 2048);
    k_sym_rowsort<<<grid, kBlock, lds, s>>>(big, nb, inc_ptr, incr, tr, kptr, contrib, kcol, kbeg, ncols);
    return hipGetLastError();
}

namespace {
// slot of the transposed block (c, r) for every block (r, c) with c > r:
// binary search of r among the sorted columns of row c; -1 for diagonal and
// lower blocks.  The pattern is symmetric by construction (a pair's local
// blocks (i, j) and (j, i) both land in it); an upper block without mirror
// would get -2 and be summed on its own.
__global__ void __launch_bounds__(kBlock) k_sym_transpose(int64_t nnzb, const int32_t* __restrict__ slot_row,
                                                          const int32_t* __restrict__ col_idx,
                                                          const int32_t* __restrict__ row_ptr,
                                                          int32_t* __restrict__ tslot) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= nnzb) return;
    const int32_t r = slot_row[s], c = col_idx[s];
    int32_t t = -1;
    if (c > r) {
        int32_t lo = row_ptr[c], hi = row_ptr[c + 1] - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col_idx[mid] < r) lo = mid + 1;
            else hi = mid;
        }
        t = col_idx[lo] == r ? lo : -2;
    }
    tslot[s] = t;
}
}  // namespace

hipError_t launch_sym_transpose(int64_t nnzb, const int32_t* slot_row, const int32_t* col_idx,
                                const int32_t* row_ptr, int32_t* tslot, hipStream_t s) {
    if (nnzb == 0) return hipSuccess;
    k_sym_transpose<<<(unsigned)((nnzb + kBlock - 1) / kBlock), kBlock, 0, s>>>(nnzb, slot_row, col_idx, row_ptr,
                                                                                tslot);
    return hipGetLastError();
}

hipError_t launch_sym_fill(int32_t V, const int64_t* kptr, const int32_t* kcol, const int32_t* kbeg,
                           const int32_t* row_ptr, int32_t* col_idx, int64_t* cptr, int32_t* slot_row,
                           int32_t* diag_slot, unsigned long long* whead, int32_t* wrow, int64_t nnzb,
                           hipStream_t s) {
    if (V == 0) return hipSuccess;
    const int64_t W = (nnzb + 63) >> 6;
    k_zero_u64<<<(unsigned)((W + kBlock - 1) / kBlock), kBlock, 0, s>>>(whead, W);
    const unsigned blocks = (unsigned)(((int64_t)V + kBlock / 64 - 1) / (kBlock / 64));
    k_sym_fill<<<blocks, kBlock, 0, s>>>(V, kptr, kcol, kbeg, row_ptr, col_idx, cptr, slot_row, diag_slot, whead,
                                         wrow, nnzb);
    return hipGetLastError();
}

}  // namespace gipc
