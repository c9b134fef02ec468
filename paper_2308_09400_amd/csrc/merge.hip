// Merging of duplicate constraints after staging.  On aligned grids many
// candidate tuples reduce to the same point-edge or point-point constraint
// (a point over a shared edge or vertex is found through every triangle and
// edge pair around it).  The energy of Eq. 3 sums each candidate with its
// own constrained distance, so identical reduced constraints can be
// evaluated once and weighted by their count: that is exact.
//
// Duplicates are found with an open-addressing hash table on a 64-bit
// fingerprint of the canonical key (PP: the unordered vertex pair; PE: the
// point and the unordered edge).  The representative of a key is the
// smallest staged index carrying it (atomicMin), and a pair merges into it
// only if its full key equals the representative's, so a fingerprint
// collision can only leave duplicates unmerged, never merge different
// constraints.  Counts are integer atomics and the compaction keeps the
// staged order, so the result is deterministic.
//
// Layout: one 8-byte word per slot holding a 36-bit fingerprint above the
// 28-bit representative (staged indices are below 2^28), so a slot is
// claimed and its representative lowered with 64-bit atomics on one word
// (the minimum of two words with the same fingerprint is the one with the
// smaller representative).  A key's home slot is proportional to its first
// vertex plus a 16-slot offset from the fingerprint: staged pairs come in
// vertex-major order within each sub-type, so neighbouring lanes probe
// neighbouring lines.
#include "internal.hpp"

namespace gipc {
namespace {

// splitmix64 finalizer (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct Key {
    int a, b, c;
};

__device__ __forceinline__ Key canon(bool pp, int4 v) {
    if (pp) return Key{min(v.x, v.y), max(v.x, v.y), -1};
    return Key{v.x, min(v.y, v.z), max(v.y, v.z)};
}

constexpr int kRepBits = 28;
constexpr unsigned long long kRepMask = (1ull << kRepBits) - 1ull;

// 36-bit fingerprint in the high bits of a slot word, never 0 (0 = empty)
__device__ __forceinline__ unsigned long long fingerprint(const Key& k) {
    uint64_t x = ((uint64_t)(uint32_t)k.a << 32) | (uint32_t)k.b;
    uint64_t f = mix64(x ^ mix64((uint64_t)(uint32_t)k.c + 0x9e3779b97f4a7c15ull)) & ~kRepMask;
    return f ? f : (1ull << kRepBits);
}

__device__ __forceinline__ uint64_t home(const Key& k, unsigned long long f, double scale, uint64_t mask) {
    return ((uint64_t)((double)(uint32_t)k.a * scale) + ((f >> kRepBits) & 15ull)) & mask;
}

// Probes stop after kMaxProbe slots: a pair whose key finds neither its
// slot nor an empty one that close to home stays unmerged (exact, only
// slower); both passes walk the same sequence, so they agree.
constexpr int kMaxProbe = 4096;

// Lanes of a wavefront carrying the same key (same kind) form a group; its
// leader is its lowest lane, which holds the group's smallest staged index.
// Only leaders touch the table.  The loop runs once per distinct key of the
// wavefront (the mask of pending lanes is the same in every lane).
struct Group {
    int leader;                  // lane of this lane's leader (-1 if not in)
    unsigned long long members;  // lanes of this lane's group
};

__device__ __forceinline__ Group wave_group(const Key& key, bool pp, bool in) {
    Group g{-1, 0ull};
    unsigned long long pending = __ballot(in);
    while (pending) {
        const int l = __ffsll((long long)pending) - 1;
        const int ka = __shfl(key.a, l, 64), kb = __shfl(key.b, l, 64), kc = __shfl(key.c, l, 64);
        const int kp = __shfl((int)pp, l, 64);
        const bool same = in && key.a == ka && key.b == kb && key.c == kc && (int)pp == kp;
        const unsigned long long grp = __ballot(same);
        if (same) {
            g.leader = l;
            g.members = grp;
        }
        pending &= ~grp;
    }
    return g;
}

// pairs [k0, k1) are PE then PP from pp0 on
__global__ void __launch_bounds__(kBlock) k_merge_insert(const int4* __restrict__ st_vid, int64_t k0, int64_t k1,
                                                         int64_t pp0, unsigned long long* __restrict__ table,
                                                         double scale, uint64_t mask) {
    const int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = k < k1;
    const bool pp = k >= pp0;
    const Key key = in ? canon(pp, st_vid[k]) : Key{-1, -1, -1};
    // only the leader of each group of equal keys in the wavefront inserts
    const Group grp = wave_group(key, pp, in);
    if (!in || grp.leader != (int)(threadIdx.x & 63)) return;
    const unsigned long long f = fingerprint(key);
    const unsigned long long word = f | (unsigned long long)k;
    uint64_t h = home(key, f, scale, mask);
    for (int t = 0; t < kMaxProbe; ++t) {
        const unsigned long long prev = atomicCAS(&table[h], 0ull, word);
        if (prev == 0ull) return;
        if ((prev & ~kRepMask) == f) {
            if (word < prev) atomicMin(&table[h], word);
            return;
        }
        h = (h + 1) & mask;
    }
}

__global__ void __launch_bounds__(kBlock) k_merge_resolve(const int4* __restrict__ st_vid, int64_t k0, int64_t k1,
                                                          int64_t pp0, const unsigned long long* __restrict__ table,
                                                          double scale, uint64_t mask, int32_t* __restrict__ rep_of,
                                                          int32_t* __restrict__ mult) {
    const int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = k < k1;
    const bool pp = k >= pp0;
    const Key me = in ? canon(pp, st_vid[k]) : Key{-1, -1, -1};
    const Group grp = wave_group(me, pp, in);
    const int lane = threadIdx.x & 63;
    // the leader finds the representative of the group's key; a group whose
    // key is in no slot (probe bound) takes its leader
    int32_t my = (int32_t)k;
    if (in && grp.leader == lane) {
        const unsigned long long f = fingerprint(me);
        uint64_t h = home(me, f, scale, mask);
        for (int t = 0; t < kMaxProbe; ++t) {
            const unsigned long long w = table[h];
            if ((w & ~kRepMask) == f) {
                const int32_t r = (int32_t)(w & kRepMask);
                if (r != (int32_t)k) {  // another pair is the representative: compare full keys
                    const bool rpp = r >= pp0;
                    const Key o = canon(rpp, st_vid[r]);
                    if (rpp == pp && o.a == me.a && o.b == me.b && o.c == me.c) my = r;
                }
                break;
            }
            if (w == 0ull) break;  // not inserted (probe bound reached on insert)
            h = (h + 1) & mask;
        }
    }
    const int32_t rep = __shfl(my, grp.leader < 0 ? lane : grp.leader, 64);
    if (!in) return;
    rep_of[k - k0] = rep;
    if (grp.leader == lane) atomicAdd(&mult[rep - k0], __popcll(grp.members));
}

// the pairs the compaction keeps: those outside [k0, k1), and inside it
// the representatives
__device__ __forceinline__ bool survives(int64_t k, int64_t Ps, int64_t k0, int64_t k1,
                                         const int32_t* __restrict__ rep_of) {
    return k < Ps && (k < k0 || k >= k1 || rep_of[k - k0] == (int32_t)k);
}

// survivors per workgroup of kBlock staged pairs
__global__ void __launch_bounds__(kBlock) k_merge_count(int64_t Ps, int64_t k0, int64_t k1,
                                                        const int32_t* __restrict__ rep_of,
                                                        int32_t* __restrict__ bcnt) {
    __shared__ int32_t cnt[kBlock / 64];
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const unsigned long long m = __ballot(survives(k, Ps, k0, k1, rep_of));
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t c = 0;
        for (int w = 0; w < kBlock / 64; ++w) c += cnt[w];
        bcnt[blockIdx.x] = c;
    }
}

// stable compaction: a survivor's position is its workgroup's offset plus
// the survivors before it in the workgroup
__global__ void __launch_bounds__(kBlock) k_merge_scatter(int64_t Ps, int64_t k0, int64_t k1,
                                                          const int32_t* __restrict__ rep_of,
                                                          const int64_t* __restrict__ boff,
                                                          const int4* __restrict__ st_vid,
                                                          const int32_t* __restrict__ st_src,
                                                          const int32_t* __restrict__ mult_in,
                                                          int4* __restrict__ vid_out, int32_t* __restrict__ src_out,
                                                          int32_t* __restrict__ mult_out) {
    __shared__ int32_t cnt[kBlock / 64];
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int wid = threadIdx.x >> 6;
    const bool f = survives(k, Ps, k0, k1, rep_of);
    const unsigned long long m = __ballot(f);
    if ((threadIdx.x & 63) == 0) cnt[wid] = __popcll(m);
    __syncthreads();
    if (!f) return;
    int64_t n = boff[blockIdx.x];
    for (int w = 0; w < wid; ++w) n += cnt[w];
    n += __popcll(m & __lanemask_lt());
    vid_out[n] = st_vid[k];
    src_out[n] = st_src[k];
    mult_out[n] = (k >= k0 && k < k1) ? mult_in[k - k0] : 1;
}

// merged type offsets, one workgroup per t = 0..8: out[t] = the survivors
// before tr.off[t]
__global__ void __launch_bounds__(kBlock) k_merge_offsets(int64_t Ps, int64_t k0, int64_t k1,
                                                          const int32_t* __restrict__ rep_of,
                                                          const int64_t* __restrict__ boff, TypeRanges tr,
                                                          int64_t* __restrict__ out) {
    __shared__ int32_t cnt[kBlock / 64];
    const int64_t o = tr.off[blockIdx.x];
    const int64_t b = o / kBlock;
    const int64_t k = b * kBlock + threadIdx.x;
    const unsigned long long m = __ballot(k < o && survives(k, Ps, k0, k1, rep_of));
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t c = boff[b];
        for (int w = 0; w < kBlock / 64; ++w) c += cnt[w];
        out[blockIdx.x] = c;
    }
}

unsigned grid(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t merge_duplicates(gipc_ctx* ctx, int32_t V, hipStream_t s, int64_t* new_off_dev) {
    const TypeRanges& tr = ctx->ranges;
    const int64_t Ps = tr.off[8], k0 = tr.off[FT_PE], pp0 = tr.off[FT_PP], k1 = tr.off[FT_PP + 1];
    const int64_t n = k1 - k0;
    uint64_t H = 1024;
    while (H < (uint64_t)n + (uint64_t)n / 4) H <<= 1;
    // home slots spread over the whole table: V is the vertex count of the pair set
    const double scale = V > 0 ? (double)H / (double)V : 1.0;
    hipError_t e;
#define TRY(x)                          \
    do {                                \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    TRY(ensure(ctx->mkeys, sizeof(unsigned long long) * H));
    TRY(ensure(ctx->mrep_of, sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    TRY(ensure(ctx->mcount, sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    const int64_t nbk = (Ps + kBlock - 1) / kBlock;  // compaction workgroups
    TRY(ensure(ctx->mbcount, sizeof(int32_t) * (size_t)(nbk > 0 ? nbk : 1)));
    TRY(ensure(ctx->mpos, sizeof(int64_t) * (size_t)(nbk + 1)));
    TRY(ensure(ctx->st_vid2, sizeof(int4) * (size_t)(Ps > 0 ? Ps : 1)));
    TRY(ensure(ctx->st_src2, sizeof(int32_t) * (size_t)(Ps > 0 ? Ps : 1)));
    TRY(ensure(ctx->mult, sizeof(int32_t) * (size_t)(Ps > 0 ? Ps : 1)));
    if (n > 0) {
        TRY(hipMemsetAsync(ctx->mkeys.p, 0, sizeof(unsigned long long) * H, s));
        TRY(hipMemsetAsync(ctx->mcount.p, 0, sizeof(int32_t) * n, s));
        k_merge_insert<<<grid(n), kBlock, 0, s>>>(as<int4>(ctx->st_vid), k0, k1, pp0,
                                                  as<unsigned long long>(ctx->mkeys), scale, H - 1);
        TRY(hipGetLastError());
        k_merge_resolve<<<grid(n), kBlock, 0, s>>>(as<int4>(ctx->st_vid), k0, k1, pp0,
                                                   as<unsigned long long>(ctx->mkeys), scale, H - 1,
                                                   as<int32_t>(ctx->mrep_of), as<int32_t>(ctx->mcount));
        TRY(hipGetLastError());
    }
    const int32_t* rep = as<int32_t>(ctx->mrep_of);
    if (Ps > 0) {
        k_merge_count<<<(unsigned)nbk, kBlock, 0, s>>>(Ps, k0, k1, rep, as<int32_t>(ctx->mbcount));
        TRY(hipGetLastError());
    }
    TRY((exclusive_scan<int32_t, int64_t>(as<int32_t>(ctx->mbcount), nbk, as<int64_t>(ctx->mpos), ctx, s)));
    if (Ps > 0) {
        k_merge_scatter<<<(unsigned)nbk, kBlock, 0, s>>>(Ps, k0, k1, rep, as<int64_t>(ctx->mpos),
                                                         as<int4>(ctx->st_vid), as<int32_t>(ctx->st_src),
                                                         as<int32_t>(ctx->mcount), as<int4>(ctx->st_vid2),
                                                         as<int32_t>(ctx->st_src2), as<int32_t>(ctx->mult));
        TRY(hipGetLastError());
    }
    k_merge_offsets<<<9, kBlock, 0, s>>>(Ps, k0, k1, rep, as<int64_t>(ctx->mpos), tr, new_off_dev);
    TRY(hipGetLastError());
#undef TRY
    std::swap(ctx->st_vid, ctx->st_vid2);
    std::swap(ctx->st_src, ctx->st_src2);
    return hipSuccess;
}

}  // namespace gipc
