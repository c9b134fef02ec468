// C ABI of libgipc: argument checks, context state, buffer management and
// the launch sequences.  Every compute step runs in the kernels of the
// other translation units.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"

using namespace gipc;

namespace gipc {

hipError_t ensure(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes <= b.bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipSuccess;
        if (b.al) {
            // work queued on any stream may still read the old block: the
            // caller's allocator gets it back only once the device is idle
            e = hipDeviceSynchronize();
            if (e == hipSuccess) b.al->free(b.al->user, b.p, b.bytes, b.device);
        } else {
            e = hipFree(b.p);
        }
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t cap = bytes + bytes / 4;
    cap = (cap + 255) & ~size_t(255);
    void* p = nullptr;
    if (b.al) {
        p = b.al->alloc(b.al->user, cap, b.device);
        if (!p) return hipErrorOutOfMemory;
        if ((reinterpret_cast<uintptr_t>(p) & 255) != 0) {
            b.al->free(b.al->user, p, cap, b.device);
            return hipErrorInvalidValue;
        }
    } else {
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
    }
    b.p = p;
    b.bytes = cap;
    return hipSuccess;
}

void release(DevBuf& b) {
    if (b.p) {
        if (b.al) b.al->free(b.al->user, b.p, b.bytes, b.device);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
}

}  // namespace gipc

namespace {

std::vector<DevBuf*> ctx_buffers(gipc_ctx* ctx);

// counters layout (int64 slots of ctx->counters)
enum {
    C_NBAD = 0, C_FIRST_BAD = 1, C_NDEG = 2, C_FIRST_DEG = 3, C_ACTIVE = 4, C_OFF = 5,  // 5..13: type offsets
    C_INC = 16, C_K = 17, C_NNZB = 18, C_MAXDEG = 19, C_NSPAN = 20, C_FIRST_SPAN = 21, C_NBIG = 22,
    C_MOFF = 24,  // 24..32: merged type offsets
    C_NDPRIM = 14, C_FIRST_DPRIM = 15,
    C_NSLOTS = 40
};

// every build counter to zero, the "first index" slots to all ones (so an
// atomic minimum over the flagged indices gives the first one)
__global__ void k_reset_counters(int64_t* __restrict__ cnt) {
    const int i = threadIdx.x;
    if (i >= C_NSLOTS) return;
    const bool first = i == C_FIRST_BAD || i == C_FIRST_DEG || i == C_FIRST_DPRIM || i == C_FIRST_SPAN;
    cnt[i] = first ? -1 : 0;
}

gipc_status fail(gipc_ctx* ctx, gipc_status st, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

gipc_status hip_fail(gipc_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(ctx, GIPC_ERR_WORKSPACE, "%s: out of device memory (%s)", what, hipGetErrorString(e));
    return fail(ctx, GIPC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define CK(call, what)                                 \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

gipc_status check_device(gipc_ctx* ctx) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return fail(ctx, GIPC_ERR_HIP, "hipGetDevice failed");
    if (d != ctx->device)
        return fail(ctx, GIPC_ERR_INVALID_ARG, "context belongs to device %d but device %d is current", ctx->device, d);
    return GIPC_OK;
}

gipc_status to_dev_params(gipc_ctx* ctx, const gipc_params* p, DevParams& o) {
    if (!p) return fail(ctx, GIPC_ERR_INVALID_ARG, "params is NULL");
    if (!(p->dhat > 0.0) || !std::isfinite(p->dhat)) return fail(ctx, GIPC_ERR_INVALID_ARG, "dhat must be > 0");
    if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa)) return fail(ctx, GIPC_ERR_INVALID_ARG, "kappa must be >= 0");
    if (!(p->dthr_ratio >= 0.0) || !(p->dthr_ratio < 1.0))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "dthr_ratio must be in [0, 1)");
    if (!(p->epsx_ratio >= 0.0) || !std::isfinite(p->epsx_ratio))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "epsx_ratio must be >= 0");
    if (p->flags & ~(GIPC_FLAG_FILTER | GIPC_FLAG_MOLLIFY | GIPC_FLAG_BARRIER_EQ12 | GIPC_FLAG_NO_MERGE))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "unknown flag bits 0x%x", p->flags);
    o.dhat = p->dhat;
    o.kappa = p->kappa;
    o.dthr_ratio = p->dthr_ratio;
    o.epsx_ratio = p->epsx_ratio;
    o.filter = (p->flags & GIPC_FLAG_FILTER) ? 1 : 0;
    o.mollify = (p->flags & GIPC_FLAG_MOLLIFY) ? 1 : 0;
    o.eq12 = (p->flags & GIPC_FLAG_BARRIER_EQ12) ? 1 : 0;
    o.vscene = nullptr;
    o.dhat_s = nullptr;
    o.kappa_s = nullptr;
    if (p->batch) {
        const gipc_batch* b = p->batch;
        if (b->S < 1) return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->S must be >= 1");
        if (!b->vert_off || !b->dhat || !b->kappa)
            return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->vert_off, dhat and kappa must be device arrays");
        o.dhat_s = b->dhat;
        o.kappa_s = b->kappa;
    }
    return GIPC_OK;
}

// the batch of a call after the build: same presence and S as the build's
gipc_status bind_batch(gipc_ctx* ctx, const gipc_params* p, DevParams& pm) {
    const bool has = p->batch != nullptr;
    if (has != ctx->batched) return fail(ctx, GIPC_ERR_STATE, "the batch must be given iff the build had one");
    if (has) {
        if (p->batch->S != ctx->S)
            return fail(ctx, GIPC_ERR_STATE, "batch->S = %d differs from the build (%d)", p->batch->S, ctx->S);
        pm.vscene = static_cast<const int32_t*>(ctx->vscene.p);
    }
    return GIPC_OK;
}

gipc_status check_mesh(gipc_ctx* ctx, const gipc_mesh* m) {
    if (!m) return fail(ctx, GIPC_ERR_INVALID_ARG, "mesh is NULL");
    if (m->V < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "V < 0");
    if (m->V > 0 && !m->x) return fail(ctx, GIPC_ERR_INVALID_ARG, "mesh->x is NULL");
    return GIPC_OK;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

gipc_status read_counters(gipc_ctx* ctx, int64_t* host, int first, int n, hipStream_t s) {
    CK(hipMemcpyAsync(host + first, as<int64_t>(ctx->counters) + first, sizeof(int64_t) * n, hipMemcpyDeviceToHost,
                      s),
       "copy counters");
    CK(hipStreamSynchronize(s), "stream synchronize");
    return GIPC_OK;
}

bool same_pattern(const gipc_ctx* ctx, const gipc_bsr* A) {
    return A->nbrows == ctx->V && A->nnzb == ctx->nnzb && A->row_ptr == ctx->row_ptr.p &&
           A->col_idx == ctx->col_idx.p;
}

}  // namespace

extern "C" {

const char* gipc_status_string(int st) {
    switch (st) {
        case GIPC_OK: return "GIPC_OK";
        case GIPC_ERR_INVALID_ARG: return "GIPC_ERR_INVALID_ARG";
        case GIPC_ERR_INDEX: return "GIPC_ERR_INDEX";
        case GIPC_ERR_DEGENERATE: return "GIPC_ERR_DEGENERATE";
        case GIPC_ERR_HIP: return "GIPC_ERR_HIP";
        case GIPC_ERR_WORKSPACE: return "GIPC_ERR_WORKSPACE";
        case GIPC_ERR_BREAKDOWN: return "GIPC_ERR_BREAKDOWN";
        case GIPC_ERR_STATE: return "GIPC_ERR_STATE";
        case GIPC_WARN_NOT_CONVERGED: return "GIPC_WARN_NOT_CONVERGED";
        case GIPC_WARN_STALE: return "GIPC_WARN_STALE";
        default: return "GIPC_UNKNOWN_STATUS";
    }
}

gipc_status gipc_ctx_create_with_allocator(const gipc_allocator* al, gipc_ctx** out) {
    if (!out) return GIPC_ERR_INVALID_ARG;
    *out = nullptr;
    if (al && (!al->alloc || !al->free)) return GIPC_ERR_INVALID_ARG;
    gipc_ctx* ctx = new (std::nothrow) gipc_ctx();
    if (!ctx) return GIPC_ERR_WORKSPACE;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return GIPC_ERR_HIP;
    }
    if (al) {
        ctx->alloc = *al;
        for (DevBuf* b : ctx_buffers(ctx)) {
            b->al = &ctx->alloc;
            b->device = ctx->device;
        }
    }
    if (ensure(ctx->counters, sizeof(int64_t) * C_NSLOTS) != hipSuccess) {
        delete ctx;
        return GIPC_ERR_WORKSPACE;
    }
    *out = ctx;
    return GIPC_OK;
}

gipc_status gipc_ctx_create(gipc_ctx** out) { return gipc_ctx_create_with_allocator(nullptr, out); }

void gipc_ctx_destroy(gipc_ctx* ctx) {
    if (!ctx) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    if (ctx->alloc.alloc) (void)hipDeviceSynchronize();
    for (DevBuf* b : ctx_buffers(ctx)) release(*b);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete ctx;
}

}  // extern "C"

namespace {
// every device buffer the context holds
std::vector<DevBuf*> ctx_buffers(gipc_ctx* ctx) {
    return {&ctx->cand_ft, &ctx->cand_vid, &ctx->bcount, &ctx->boff, &ctx->counters, &ctx->st_vid,
                      &ctx->st_src, &ctx->mult, &ctx->mkeys, &ctx->mrep_of, &ctx->mcount,
                      &ctx->mbcount, &ctx->mpos, &ctx->st_vid2, &ctx->st_src2, &ctx->deg, &ctx->kcount, &ctx->fill, &ctx->inc_ptr, &ctx->kptr,
                      &ctx->contrib, &ctx->kcol, &ctx->kbeg, &ctx->ncols, &ctx->row_ptr, &ctx->col_idx, &ctx->cptr,
                      &ctx->slot_row, &ctx->diag_slot, &ctx->whead, &ctx->wrow, &ctx->maxbuf, &ctx->bigrows, &ctx->tslot, &ctx->incr, &ctx->order,
                      &ctx->obox, &ctx->ocell, &ctx->ohist, &ctx->ooff, &ctx->ofill, &ctx->rec_main, &ctx->rec_extra, &ctx->rec_a1, &ctx->ev,
                      &ctx->epart, &ctx->mfg, &ctx->mfab, &ctx->flag, &ctx->ffr, &ctx->fev, &ctx->fpart, &ctx->cpart, &ctx->ccnt, &ctx->ccount, &ctx->cfill, &ctx->coff_t, &ctx->cent_t, &ctx->coff_e, &ctx->cent_e, &ctx->qcnt, &ctx->qoff_p, &ctx->qoff_e, &ctx->crec_t, &ctx->crec_e, &ctx->qtoff_p, &ctx->qtoff_e, &ctx->qent_p, &ctx->qent_e, &ctx->ecnt_p, &ctx->ecnt_e, &ctx->eoff_p, &ctx->eoff_e, &ctx->craw, &ctx->bslot, &ctx->boff_p, &ctx->boff_e, &ctx->bal_p, &ctx->bal_e, &ctx->evis_p, &ctx->evis_e, &ctx->vscene, &ctx->pieces, &ctx->poff,
                      &ctx->r, &ctx->z, &ctx->p, &ctx->q, &ctx->p32, &ctx->minv, &ctx->part, &ctx->scal, &ctx->scan_tmp,
                      &ctx->scan_tmp2, &ctx->chk, &ctx->accd_cnt};
}
}  // namespace

extern "C" {

const char* gipc_ctx_last_error(const gipc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gipc_status gipc_pairs_build(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_pairs* pairs,
                             const gipc_params* params, void* stream, gipc_info* info) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    if (!pairs) return fail(ctx, GIPC_ERR_INVALID_ARG, "pairs is NULL");
    if (pairs->P < 0 || pairs->P >= (int64_t(1) << 31))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "P must be in [0, 2^31)");
    if (pairs->P > 0 && !pairs->tuples) return fail(ctx, GIPC_ERR_INVALID_ARG, "pairs->tuples is NULL");
    DevParams pm;
    if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;

    hipStream_t s = S(stream);
    const int64_t P = pairs->P;
    const int32_t V = mesh->V;
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    ctx->built = false;
    ctx->evaluated = false;
    ++ctx->build_gen;

    // ---- scenes: vertex ranges, energy pieces, scene of every vertex
    const gipc_batch* batch = params->batch;
    const int32_t Sc = batch ? batch->S : 1;
    std::vector<int32_t> voff(Sc + 1);
    if (batch) {
        std::vector<double> dh(Sc), ka(Sc);
        CK(hipMemcpyAsync(voff.data(), batch->vert_off, sizeof(int32_t) * (Sc + 1), hipMemcpyDeviceToHost, s),
           "copy batch");
        CK(hipMemcpyAsync(dh.data(), batch->dhat, sizeof(double) * Sc, hipMemcpyDeviceToHost, s), "copy batch");
        CK(hipMemcpyAsync(ka.data(), batch->kappa, sizeof(double) * Sc, hipMemcpyDeviceToHost, s), "copy batch");
        CK(hipStreamSynchronize(s), "stream synchronize");
        if (voff[0] != 0 || voff[Sc] != V)
            return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->vert_off must start at 0 and end at V = %d", V);
        for (int32_t k = 0; k < Sc; ++k) {
            if (voff[k + 1] < voff[k])
                return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->vert_off decreases at scene %d", k);
            if (!(dh[k] > 0.0) || !std::isfinite(dh[k]))
                return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->dhat[%d] must be > 0", k);
            if (!(ka[k] >= 0.0) || !std::isfinite(ka[k]))
                return fail(ctx, GIPC_ERR_INVALID_ARG, "batch->kappa[%d] must be >= 0", k);
        }
    } else {
        voff[0] = 0;
        voff[1] = V;
    }
    std::vector<int2> pcs;
    std::vector<int32_t> po(Sc + 1);
    for (int32_t k = 0; k < Sc; ++k) {
        po[k] = (int32_t)pcs.size();
        for (int64_t v = voff[k]; v < voff[k + 1]; v += kEnergyPiece)
            pcs.push_back(make_int2((int)v, (int)std::min<int64_t>(v + kEnergyPiece, voff[k + 1])));
    }
    po[Sc] = (int32_t)pcs.size();
    CK(ensure(ctx->pieces, sizeof(int2) * pcs.size()), "alloc energy pieces");
    CK(ensure(ctx->poff, sizeof(int32_t) * po.size()), "alloc energy pieces");
    if (!pcs.empty())
        CK(hipMemcpyAsync(ctx->pieces.p, pcs.data(), sizeof(int2) * pcs.size(), hipMemcpyHostToDevice, s),
           "upload energy pieces");
    CK(hipMemcpyAsync(ctx->poff.p, po.data(), sizeof(int32_t) * po.size(), hipMemcpyHostToDevice, s),
       "upload energy pieces");
    if (batch) {
        CK(ensure(ctx->vscene, sizeof(int32_t) * (size_t)(V > 0 ? V : 1)), "alloc vertex scenes");
        CK(launch_vertex_scene(batch->vert_off, Sc, V, as<int32_t>(ctx->vscene), s), "vertex scenes");
        pm.vscene = as<int32_t>(ctx->vscene);
    }
    CK(hipStreamSynchronize(s), "stream synchronize");  // the host tables above go out of scope
    ctx->S = Sc;
    ctx->batched = batch != nullptr;
    ctx->npieces = (int32_t)pcs.size();

    // ---- staging
    const int64_t nb = (P + kBlock - 1) / kBlock;
    CK(ensure(ctx->cand_ft, (size_t)P), "alloc staging");
    CK(ensure(ctx->cand_vid, sizeof(int4) * (size_t)P), "alloc staging");
    CK(ensure(ctx->bcount, sizeof(int32_t) * 8 * (size_t)(nb > 0 ? nb : 1)), "alloc staging");
    CK(ensure(ctx->boff, sizeof(int64_t) * (8 * (size_t)nb + 1)), "alloc staging");
    CK(ensure(ctx->st_vid, sizeof(int4) * (size_t)P), "alloc staged pairs");
    CK(ensure(ctx->st_src, sizeof(int32_t) * (size_t)P), "alloc staged pairs");
    int64_t* cnt = as<int64_t>(ctx->counters);
    k_reset_counters<<<1, 64, 0, s>>>(cnt);
    CK(hipGetLastError(), "clear counters");
    if (P > 0) {
        CK(launch_stage_classify(pairs->tuples, P, V, mesh->x, xr, pm, as<uint8_t>(ctx->cand_ft),
                                 as<int4>(ctx->cand_vid), as<int32_t>(ctx->bcount), cnt, s),
           "stage classify");
        CK((exclusive_scan<int32_t, int64_t>(as<int32_t>(ctx->bcount), 8 * nb, as<int64_t>(ctx->boff), ctx, s,
                                             cnt + C_ACTIVE)),
           "stage scan");
        CK(launch_stage_scatter(as<uint8_t>(ctx->cand_ft), as<int4>(ctx->cand_vid), P, as<int64_t>(ctx->boff),
                                as<int4>(ctx->st_vid), as<int32_t>(ctx->st_src), s),
           "stage scatter");
        CK(launch_stage_offsets(as<int64_t>(ctx->boff), nb, cnt + C_OFF, s), "stage offsets");
    }
    int64_t hc[C_NSLOTS] = {0};
    if ((st = read_counters(ctx, hc, 0, C_NSLOTS, s)) != GIPC_OK) return st;
    if (hc[C_NBAD] > 0)
        return fail(ctx, GIPC_ERR_INDEX, "%lld malformed tuple(s) or vertex id(s) out of [0, %d); first at %lld",
                    (long long)hc[C_NBAD], V, (long long)hc[C_FIRST_BAD]);
    if (hc[C_NSPAN] > 0)
        return fail(ctx, GIPC_ERR_INDEX, "%lld tuple(s) with vertices in two scenes; first at %lld",
                    (long long)hc[C_NSPAN], (long long)hc[C_FIRST_SPAN]);
    TypeRanges tr;
    for (int t = 0; t < 9; ++t) tr.off[t] = P > 0 ? hc[C_OFF + t] : 0;
    tr.off[0] = 0;
    const TypeRanges raw = tr;
    if (raw.off[8] >= (int64_t(1) << 28))
        return fail(ctx, GIPC_ERR_WORKSPACE, "more than 2^28 active pairs (%lld)", (long long)raw.off[8]);
    ctx->merged = false;
    if (tr.off[8] > 0 && !(params->flags & GIPC_FLAG_NO_MERGE)) {
        ctx->ranges = tr;
        CK(merge_duplicates(ctx, V, s, cnt + C_MOFF), "merge duplicates");
        if ((st = read_counters(ctx, hc, C_MOFF, 9, s)) != GIPC_OK) return st;
        for (int t = 0; t < 9; ++t) tr.off[t] = hc[C_MOFF + t];
        ctx->merged = true;
    }
    const int64_t Ps = tr.off[8];
    if (Ps >= (int64_t(1) << 28)) return fail(ctx, GIPC_ERR_WORKSPACE, "more than 2^28 staged pairs (%lld)", (long long)Ps);

    // ---- symbolic
    const size_t Vs = (size_t)(V > 0 ? V : 1);
    CK(ensure(ctx->deg, sizeof(int32_t) * Vs), "alloc pattern");
    CK(ensure(ctx->kcount, sizeof(int32_t) * Vs), "alloc pattern");
    CK(ensure(ctx->fill, sizeof(int32_t) * Vs), "alloc pattern");
    CK(ensure(ctx->inc_ptr, sizeof(int64_t) * (Vs + 1)), "alloc pattern");
    CK(ensure(ctx->kptr, sizeof(int64_t) * (Vs + 1)), "alloc pattern");
    CK(ensure(ctx->ncols, sizeof(int32_t) * Vs), "alloc pattern");
    CK(ensure(ctx->row_ptr, sizeof(int32_t) * (Vs + 1)), "alloc pattern");
    CK(ensure(ctx->diag_slot, sizeof(int32_t) * Vs), "alloc pattern");
    CK(zero_i32(as<int32_t>(ctx->deg), as<int32_t>(ctx->kcount), as<int32_t>(ctx->fill), (int64_t)Vs, s),
       "clear pattern");
    CK(launch_sym_count(as<int4>(ctx->st_vid), tr, as<int32_t>(ctx->deg), as<int32_t>(ctx->kcount), s), "count");
    CK(reduce_max_i32(as<int32_t>(ctx->deg), V, reinterpret_cast<int32_t*>(cnt + C_MAXDEG), s), "max degree");
    CK((exclusive_scan<int32_t, int64_t>(as<int32_t>(ctx->deg), V, as<int64_t>(ctx->inc_ptr), ctx, s, cnt + C_INC)),
       "incidence scan");
    CK((exclusive_scan<int32_t, int64_t>(as<int32_t>(ctx->kcount), V, as<int64_t>(ctx->kptr), ctx, s, cnt + C_K)),
       "contribution scan");
    if ((st = read_counters(ctx, hc, C_INC, 4, s)) != GIPC_OK) return st;
    const int32_t max_deg = (int32_t)(hc[C_MAXDEG] & 0xffffffff);
    if (max_deg > kMaxRowPairs)
        return fail(ctx, GIPC_ERR_WORKSPACE, "a vertex is touched by %d active pairs (limit %d)", max_deg,
                    kMaxRowPairs);
    const int64_t ninc = hc[C_INC], K = hc[C_K];
    CK(ensure(ctx->incr, sizeof(int4) * (size_t)(ninc > 0 ? ninc : 1)), "alloc incidences");
    CK(ensure(ctx->contrib, sizeof(uint32_t) * (size_t)K), "alloc contributions");
    CK(ensure(ctx->kcol, sizeof(int32_t) * (size_t)K), "alloc contributions");
    CK(ensure(ctx->kbeg, sizeof(int32_t) * (size_t)K), "alloc contributions");
    CK(launch_sym_scatter(as<int4>(ctx->st_vid), tr, as<int64_t>(ctx->inc_ptr), as<int32_t>(ctx->fill),
                          as<int4>(ctx->incr), s),
       "incidence scatter");
    CK(ensure(ctx->bigrows, sizeof(int32_t) * Vs), "alloc pattern");
    CK(launch_sym_rowsort(V, max_deg, as<int64_t>(ctx->inc_ptr), as<int4>(ctx->incr), tr,
                          as<int64_t>(ctx->kptr), as<uint32_t>(ctx->contrib), as<int32_t>(ctx->kcol),
                          as<int32_t>(ctx->kbeg), as<int32_t>(ctx->ncols), as<int32_t>(ctx->bigrows), cnt + C_NBIG,
                          s),
       "row sort");
    CK((exclusive_scan<int32_t, int32_t>(as<int32_t>(ctx->ncols), V, as<int32_t>(ctx->row_ptr), ctx, s,
                                         cnt + C_NNZB)),
       "row scan");
    if ((st = read_counters(ctx, hc, C_NNZB, 1, s)) != GIPC_OK) return st;
    const int64_t nnzb = hc[C_NNZB];
    if (nnzb >= (int64_t(1) << 31)) return fail(ctx, GIPC_ERR_WORKSPACE, "more than 2^31 blocks");
    CK(ensure(ctx->col_idx, sizeof(int32_t) * (size_t)nnzb), "alloc pattern");
    CK(ensure(ctx->slot_row, sizeof(int32_t) * (size_t)nnzb), "alloc pattern");
    CK(ensure(ctx->cptr, sizeof(int64_t) * (size_t)(nnzb + 1)), "alloc pattern");
    const int64_t nwave = (nnzb + 63) / 64 > 0 ? (nnzb + 63) / 64 : 1;
    CK(ensure(ctx->whead, sizeof(uint64_t) * (size_t)nwave), "alloc pattern");
    CK(ensure(ctx->wrow, sizeof(int32_t) * (size_t)nwave), "alloc pattern");
    CK(launch_sym_fill(V, as<int64_t>(ctx->kptr), as<int32_t>(ctx->kcol), as<int32_t>(ctx->kbeg),
                       as<int32_t>(ctx->row_ptr),
                       as<int32_t>(ctx->col_idx), as<int64_t>(ctx->cptr), as<int32_t>(ctx->slot_row),
                       as<int32_t>(ctx->diag_slot), as<unsigned long long>(ctx->whead), as<int32_t>(ctx->wrow),
                       nnzb, s),
       "pattern fill");
    CK(ensure(ctx->tslot, sizeof(int32_t) * (size_t)(nnzb > 0 ? nnzb : 1)), "alloc pattern");
    CK(launch_sym_transpose(nnzb, as<int32_t>(ctx->slot_row), as<int32_t>(ctx->col_idx), as<int32_t>(ctx->row_ptr),
                            as<int32_t>(ctx->tslot), s),
       "pattern transpose");
    CK(build_row_order(ctx, mesh->x, V, batch ? batch->vert_off : nullptr, Sc, s), "row order");

    ctx->ranges = tr;
    ctx->Ps = Ps;
    ctx->V = V;
    ctx->nnzb = nnzb;
    ctx->K = K;
    ctx->ninc = ninc;
    ctx->max_deg = max_deg;
    gipc_info& in = ctx->info;
    memset(&in, 0, sizeof(in));
    in.n_candidates = P;
    in.n_active = raw.off[8];
    for (int t = 1; t < 8; ++t) in.n_by_type[t] = raw.off[t + 1] - raw.off[t];
    in.n_staged = Ps;
    for (int t = 1; t < 8; ++t) in.n_staged_by_type[t] = tr.off[t + 1] - tr.off[t];
    in.n_degenerate = hc[C_NDEG];
    in.first_degenerate = hc[C_NDEG] > 0 ? hc[C_FIRST_DEG] : -1;
    in.nnzb = nnzb;
    in.n_contrib = K;
    in.max_row_pairs = max_deg;
    in.n_degenerate_prims = hc[C_NDPRIM];
    in.first_degenerate_prim = hc[C_NDPRIM] > 0 ? hc[C_FIRST_DPRIM] : -1;
    if (info) *info = in;
    ctx->built = true;
    return GIPC_OK;
}

gipc_status gipc_pairs_check(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_pairs* pairs,
                             const gipc_params* params, gipc_check* out, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    if (!pairs || (pairs->P > 0 && !pairs->tuples)) return fail(ctx, GIPC_ERR_INVALID_ARG, "pairs is NULL");
    DevParams pm;
    if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "gipc_pairs_build has not succeeded");
    if (mesh->V != ctx->V) return fail(ctx, GIPC_ERR_STATE, "V = %d differs from the build (%d)", mesh->V, ctx->V);
    if (pairs->P != ctx->info.n_candidates)
        return fail(ctx, GIPC_ERR_STATE, "P = %lld differs from the build (%lld)", (long long)pairs->P,
                    (long long)ctx->info.n_candidates);
    if ((st = bind_batch(ctx, params, pm)) != GIPC_OK) return st;
    hipStream_t s = S(stream);
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    CK(ensure(ctx->chk, sizeof(int64_t) * 6), "alloc check counters");
    const int64_t init[6] = {0, 0, 0, 0, 0, INT64_MAX};
    CK(hipMemcpyAsync(ctx->chk.p, init, sizeof(init), hipMemcpyHostToDevice, s), "clear check counters");
    CK(launch_stage_check(pairs->tuples, pairs->P, mesh->V, mesh->x, xr, pm, as<uint8_t>(ctx->cand_ft),
                          as<int4>(ctx->cand_vid), as<int64_t>(ctx->chk), s),
       "check");
    int64_t h[6];
    CK(hipMemcpyAsync(h, ctx->chk.p, sizeof(h), hipMemcpyDeviceToHost, s), "copy check counters");
    CK(hipStreamSynchronize(s), "stream synchronize");
    if (h[4] > 0) return fail(ctx, GIPC_ERR_INDEX, "%lld malformed tuple(s)", (long long)h[4]);
    gipc_check c{h[0], h[1], h[2], h[3], (h[0] + h[2] > 0) ? h[5] : -1};
    if (out) *out = c;
    return (c.n_entered + c.n_changed > 0) ? GIPC_WARN_STALE : GIPC_OK;
}

gipc_status gipc_get_info(const gipc_ctx* ctx, gipc_info* info) {
    if (!ctx || !info) return GIPC_ERR_INVALID_ARG;
    if (!ctx->built) return GIPC_ERR_STATE;
    *info = ctx->info;
    return GIPC_OK;
}

gipc_status gipc_bsr_pattern(const gipc_ctx* ctx, gipc_bsr* A) {
    if (!ctx || !A) return GIPC_ERR_INVALID_ARG;
    if (!ctx->built) return GIPC_ERR_STATE;
    A->nbrows = ctx->V;
    A->nnzb = ctx->nnzb;
    A->row_ptr = static_cast<const int32_t*>(ctx->row_ptr.p);
    A->col_idx = static_cast<const int32_t*>(ctx->col_idx.p);
    A->wave_head = static_cast<const uint64_t*>(ctx->whead.p);
    A->wave_row = static_cast<const int32_t*>(ctx->wrow.p);
    return GIPC_OK;
}

// ---------------------------------------------------------------- eval

namespace {

// rows of the gradient / diagonal pass and of the off-diagonal blocks: the
// spatial cells of the build's positions, or storage order (null) when
// row_order = 1; the results are the same bits either way
const int32_t* visit_order(gipc_ctx* ctx, int32_t row_order) {
    return row_order ? nullptr : as<int32_t>(ctx->order);
}

// argument checks shared by the eval entry points; fills pm
gipc_status eval_check(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                       double* grad, const gipc_bsr* A, bool assemble, DevParams& pm) {
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;
    if (!energy || (!grad && mesh->V > 0)) return fail(ctx, GIPC_ERR_INVALID_ARG, "energy or grad is NULL");
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "gipc_pairs_build has not succeeded");
    if (mesh->V != ctx->V) return fail(ctx, GIPC_ERR_STATE, "V = %d differs from the build (%d)", mesh->V, ctx->V);
    if ((st = bind_batch(ctx, params, pm)) != GIPC_OK) return st;
    if (assemble) {
        if (!A || !A->val) return fail(ctx, GIPC_ERR_INVALID_ARG, "A or A->val is NULL");
        if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad dtype");
        if (!same_pattern(ctx, A)) return fail(ctx, GIPC_ERR_STATE, "A is not the pattern of the last build");
    }
    return GIPC_OK;
}

// size the factor and energy buffers for the current build
gipc_status eval_prepare(gipc_ctx* ctx) {
    const TypeRanges& tr = ctx->ranges;
    const int64_t Ps = ctx->Ps, Pm = tr.off[8] - tr.off[FT_EEM];
    CK(ensure(ctx->rec_main, sizeof(double) * 8 * (size_t)Ps), "alloc factors");
    CK(ensure(ctx->rec_extra, sizeof(double) * 8 * (size_t)Pm), "alloc factors");
    CK(ensure(ctx->rec_a1, sizeof(double) * (size_t)Pm), "alloc factors");
    CK(ensure(ctx->ev, sizeof(double) * (size_t)(ctx->V > 0 ? ctx->V : 1)), "alloc energy shares");
    CK(ensure(ctx->epart, sizeof(double) * (size_t)(ctx->npieces > 0 ? ctx->npieces : 1)), "alloc energy pieces");
    return GIPC_OK;
}

// the launch sequence: no allocation, memset or synchronisation (graph-safe)
hipError_t eval_enqueue(gipc_ctx* ctx, const DevParams& pm, const gipc_mesh* mesh, double* energy, double* grad,
                        const double* diag, const gipc_bsr* A, bool assemble, const gipc_tune& t, hipStream_t s) {
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    const TypeRanges& tr = ctx->ranges;
    const int64_t m0 = tr.off[FT_EEM], e0 = tr.off[FT_EE];
    const int32_t* mult = ctx->merged ? as<int32_t>(ctx->mult) : nullptr;
    hipError_t e = launch_eval(as<int4>(ctx->st_vid), mult, tr, mesh->x, xr, pm, as<double>(ctx->rec_main),
                               as<double>(ctx->rec_extra), as<double>(ctx->rec_a1), t.eval_waves, s);
    if (e != hipSuccess) return e;
    e = launch_rows_diag(assemble ? 3 : 1, ctx->V, visit_order(ctx, t.row_order), as<int32_t>(ctx->diag_slot), as<int64_t>(ctx->cptr),
                         as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main), as<double>(ctx->rec_extra), as<double>(ctx->rec_a1), e0, m0,
                         diag, grad, as<double>(ctx->ev), assemble ? A->val : nullptr, assemble ? A->dtype : 0,
                         ctx->nnzb, t.row_lanes, s);
    if (e != hipSuccess) return e;
    if (assemble) {
        e = launch_offdiag(ctx->V, visit_order(ctx, t.row_order), as<int32_t>(ctx->row_ptr), as<int32_t>(ctx->diag_slot),
                           ctx->nnzb, as<int32_t>(ctx->col_idx), as<int32_t>(ctx->tslot), as<int64_t>(ctx->cptr),
                           as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main), as<double>(ctx->rec_extra), e0, m0,
                           A->val, A->dtype, t.offdiag_waves, s);
        if (e != hipSuccess) return e;
    }
    return launch_energy(as<double>(ctx->ev), as<int2>(ctx->pieces), ctx->npieces, as<int32_t>(ctx->poff), ctx->S,
                         as<double>(ctx->epart), energy, s);
}

bool tune_ok(const gipc_tune& t) {
    auto w = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
    return w(t.eval_waves) && w(t.offdiag_waves) &&
           (t.row_lanes == 4 || t.row_lanes == 8 || t.row_lanes == 16 || t.row_lanes == 32) &&
           (t.row_order == 0 || t.row_order == 1);
}

}  // namespace

static gipc_status eval_impl(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                             double* grad, const double* diag, const gipc_bsr* A, bool assemble, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    DevParams pm;
    if ((st = eval_check(ctx, mesh, params, energy, grad, A, assemble, pm)) != GIPC_OK) return st;
    if ((st = eval_prepare(ctx)) != GIPC_OK) return st;
    CK(eval_enqueue(ctx, pm, mesh, energy, grad, diag, A, assemble, ctx->tune, S(stream)), "eval");
    ctx->evaluated = true;
    ++ctx->eval_gen;
    return GIPC_OK;
}

gipc_status gipc_barrier_eval(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                              double* grad, void* stream) {
    return eval_impl(ctx, mesh, params, energy, grad, nullptr, nullptr, false, stream);
}

gipc_status gipc_eval_assemble(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                               double* grad, const double* diag, const gipc_bsr* A, void* stream) {
    return eval_impl(ctx, mesh, params, energy, grad, diag, A, true, stream);
}

gipc_status gipc_assemble_bsr(gipc_ctx* ctx, const double* diag, const gipc_bsr* A, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!A || !A->val) return fail(ctx, GIPC_ERR_INVALID_ARG, "A or A->val is NULL");
    if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad dtype");
    if (!ctx->built || !ctx->evaluated) return fail(ctx, GIPC_ERR_STATE, "build and eval must precede assembly");
    if (!same_pattern(ctx, A)) return fail(ctx, GIPC_ERR_STATE, "A is not the pattern of the last build");
    hipStream_t s = S(stream);
    const int64_t m0 = ctx->ranges.off[FT_EEM], e0 = ctx->ranges.off[FT_EE];
    CK(launch_rows_diag(2, ctx->V, visit_order(ctx, ctx->tune.row_order), as<int32_t>(ctx->diag_slot), as<int64_t>(ctx->cptr), as<uint32_t>(ctx->contrib),
                        as<double>(ctx->rec_main), as<double>(ctx->rec_extra), as<double>(ctx->rec_a1), e0, m0, diag, nullptr, nullptr, A->val,
                        A->dtype, ctx->nnzb, ctx->tune.row_lanes, s),
       "diagonal blocks");
    CK(launch_offdiag(ctx->V, visit_order(ctx, ctx->tune.row_order), as<int32_t>(ctx->row_ptr), as<int32_t>(ctx->diag_slot),
                           ctx->nnzb, as<int32_t>(ctx->col_idx), as<int32_t>(ctx->tslot), as<int64_t>(ctx->cptr),
                      as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main), as<double>(ctx->rec_extra), e0, m0,
                      A->val, A->dtype, ctx->tune.offdiag_waves, s),
       "off-diagonal blocks");
    return GIPC_OK;
}

gipc_status gipc_bsr_spmv(const gipc_bsr* A, const void* x, void* y, void* stream) {
    if (!A || A->nbrows < 0 || A->nnzb < 0) return GIPC_ERR_INVALID_ARG;
    if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return GIPC_ERR_INVALID_ARG;
    if (A->nbrows > 0 && (!A->row_ptr || !x || !y)) return GIPC_ERR_INVALID_ARG;
    if (A->nnzb > 0 && (!A->col_idx || !A->val)) return GIPC_ERR_INVALID_ARG;
    if (launch_spmv(*A, x, y, S(stream)) != hipSuccess) return GIPC_ERR_HIP;
    return GIPC_OK;
}

gipc_status gipc_accd(gipc_ctx* ctx, const gipc_mesh* mesh, const double* disp, const gipc_pairs* pairs, double s,
                      double tc, int32_t max_iter, double* toi, gipc_accd_info* info, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    if (!pairs || pairs->P < 0 || (pairs->P > 0 && !pairs->tuples))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "bad pair list");
    if (pairs->P > 0 && (!disp || mesh->V <= 0)) return fail(ctx, GIPC_ERR_INVALID_ARG, "displacement is NULL");
    if (!(s > 0.0 && s < 1.0)) return fail(ctx, GIPC_ERR_INVALID_ARG, "s must lie in (0, 1)");
    if (!(tc >= 0.0) || !std::isfinite(tc)) return fail(ctx, GIPC_ERR_INVALID_ARG, "tc must be >= 0 and finite");
    if (max_iter < 1) return fail(ctx, GIPC_ERR_INVALID_ARG, "max_iter must be >= 1");
    hipStream_t hs = S(stream);
    CK(ensure(ctx->accd_cnt, sizeof(unsigned long long) * 8), "alloc ccd counters");
    auto* cnt = as<unsigned long long>(ctx->accd_cnt);
    CK(launch_accd(pairs->tuples, pairs->P, mesh->V, mesh->x, disp, s, tc, max_iter, toi, cnt, hs), "ccd");
    unsigned long long h[6];
    CK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, hs), "copy");
    CK(hipStreamSynchronize(hs), "stream synchronize");
    if (h[0] > 0)
        return fail(ctx, GIPC_ERR_INDEX, "%llu malformed tuples (first: %llu)", h[0], h[1]);
    if (info) {
        double step;
        std::memcpy(&step, &h[4], sizeof(step));
        info->step = step;
        info->n_capped = (int64_t)h[2];
        info->n_touching = (int64_t)h[3];
        info->max_steps = (int32_t)h[5];
    }
    return GIPC_OK;
}

gipc_status gipc_pcg(gipc_ctx* ctx, const gipc_bsr* A, const double* b, double* x, double rtol, int32_t maxit,
                     int32_t* iters, double* relres, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!A || A->nbrows < 0 || A->nnzb < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad matrix");
    if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad dtype");
    if (A->nbrows > 0 && (!A->row_ptr || !A->col_idx || !A->val || !b || !x))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "NULL matrix or vector");
    if (!(rtol >= 0.0) || maxit < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "rtol must be >= 0 and maxit >= 0");
    int32_t it = 0;
    double rr = 0.0;
    int brk = 0;
    if (A->nbrows > 0) CK(pcg_run(ctx, *A, b, x, rtol, maxit, &it, &rr, &brk, S(stream)), "pcg");
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (brk) return fail(ctx, GIPC_ERR_BREAKDOWN, "p^T A p <= 0 at iteration %d", it);
    if (rtol > 0.0 && rr > rtol) return GIPC_WARN_NOT_CONVERGED;
    return GIPC_OK;
}

gipc_status gipc_pcg_delta(gipc_ctx* ctx, const gipc_bsr* A, const double* b, double* x, double eps,
                           int32_t maxit, int32_t* iters, double* relres, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!A || A->nbrows < 0 || A->nnzb < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad matrix");
    if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad dtype");
    if (A->nbrows > 0 && (!A->row_ptr || !A->col_idx || !A->val || !b || !x))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "NULL matrix or vector");
    if (!(eps >= 0.0) || maxit < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "eps must be >= 0 and maxit >= 0");
    int32_t it = 0;
    double rr = 0.0;
    int brk = 0, conv = 1;
    if (A->nbrows > 0)
        CK(pcg_run(ctx, *A, b, x, eps, maxit, &it, &rr, &brk, S(stream), nullptr, 1, &conv), "pcg");
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (brk) return fail(ctx, GIPC_ERR_BREAKDOWN, "p^T A p <= 0 at iteration %d", it);
    if (eps > 0.0 && !conv) return GIPC_WARN_NOT_CONVERGED;
    return GIPC_OK;
}

}  // extern "C"

namespace {

// the matrix-free operator over the factors of the last eval
gipc_status mf_view(gipc_ctx* ctx, const double* diag, MfView& m, hipStream_t stream) {
    if (!ctx->built || !ctx->evaluated) return fail(ctx, GIPC_ERR_STATE, "build and eval must precede the operator");
    const int64_t Ps = ctx->ranges.off[8];
    const int64_t ninc = ctx->ninc;
    CK(ensure(ctx->mfg, sizeof(double) * 3 * (size_t)(ninc > 0 ? ninc : 1)), "alloc operator vectors");
    CK(ensure(ctx->mfab, sizeof(double2) * (size_t)(Ps > 0 ? Ps : 1)), "alloc operator scratch");
    m.V = ctx->V;
    m.tr = ctx->ranges;
    m.st_vid = as<int4>(ctx->st_vid);
    m.order = as<int32_t>(ctx->order);
    m.diag_slot = as<int32_t>(ctx->diag_slot);
    m.cptr = as<int64_t>(ctx->cptr);
    m.contrib = as<uint32_t>(ctx->contrib);
    m.rec_main = as<double>(ctx->rec_main);
    m.rec_extra = as<double>(ctx->rec_extra);
    m.diag = diag;
    m.inc_ptr = as<int64_t>(ctx->inc_ptr);
    m.g = as<double>(ctx->mfg);
    m.ab = as<double2>(ctx->mfab);
    if (ctx->mfg_gen != ctx->eval_gen) {
        CK(launch_mf_coef(m, as<double>(ctx->mfg), stream), "operator vectors");
        ctx->mfg_gen = ctx->eval_gen;
    }
    return GIPC_OK;
}

// the dense operator over hess [Ps][12][12] of the current build
gipc_status dense_view(gipc_ctx* ctx, const double* hess, int32_t scheme, const double* diag, MfView& m) {
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "no build");
    if (scheme != GIPC_DENSE_THREAD && scheme != GIPC_DENSE_ENTRY)
        return fail(ctx, GIPC_ERR_INVALID_ARG, "scheme must be GIPC_DENSE_THREAD or GIPC_DENSE_ENTRY");
    if (!hess && ctx->ranges.off[8] > 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "hess is NULL");
    m.V = ctx->V;
    m.tr = ctx->ranges;
    m.st_vid = as<int4>(ctx->st_vid);
    m.order = as<int32_t>(ctx->order);
    m.diag_slot = as<int32_t>(ctx->diag_slot);
    m.cptr = as<int64_t>(ctx->cptr);
    m.contrib = as<uint32_t>(ctx->contrib);
    m.diag = diag;
    m.inc_ptr = as<int64_t>(ctx->inc_ptr);
    m.dense = hess;
    m.dense_scheme = scheme;
    return GIPC_OK;
}

}  // namespace

extern "C" {

gipc_status gipc_dense_apply(gipc_ctx* ctx, const double* hess, int32_t scheme, const double* diag, const double* x,
                             double* y, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    MfView m{};
    if ((st = dense_view(ctx, hess, scheme, diag, m)) != GIPC_OK) return st;
    if (m.V > 0 && (!x || !y)) return fail(ctx, GIPC_ERR_INVALID_ARG, "x or y is NULL");
    if (x == y && m.V > 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "x and y must not alias");
    CK(launch_mf_apply(m, x, y, nullptr, nullptr, S(stream)), "dense operator");
    return GIPC_OK;
}

gipc_status gipc_pcg_dense(gipc_ctx* ctx, const double* hess, int32_t scheme, const double* diag, const double* b,
                           double* x, double rtol, int32_t maxit, int32_t* iters, double* relres, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    MfView m{};
    if ((st = dense_view(ctx, hess, scheme, diag, m)) != GIPC_OK) return st;
    if (m.V > 0 && (!b || !x)) return fail(ctx, GIPC_ERR_INVALID_ARG, "b or x is NULL");
    if (!(rtol >= 0.0) || maxit < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "rtol must be >= 0 and maxit >= 0");
    int32_t it = 0;
    double rr = 0.0;
    int brk = 0;
    gipc_bsr none{};
    if (m.V > 0) CK(pcg_run(ctx, none, b, x, rtol, maxit, &it, &rr, &brk, S(stream), &m), "pcg");
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (brk) return fail(ctx, GIPC_ERR_BREAKDOWN, "p^T A p <= 0 at iteration %d", it);
    if (rtol > 0.0 && rr > rtol) return GIPC_WARN_NOT_CONVERGED;
    return GIPC_OK;
}

gipc_status gipc_mf_apply(gipc_ctx* ctx, const double* diag, const double* x, double* y, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    MfView m{};
    if ((st = mf_view(ctx, diag, m, S(stream))) != GIPC_OK) return st;
    if (m.V > 0 && (!x || !y)) return fail(ctx, GIPC_ERR_INVALID_ARG, "x or y is NULL");
    if (x == y && m.V > 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "x and y must not alias");
    CK(launch_mf_apply(m, x, y, nullptr, nullptr, S(stream)), "operator");
    return GIPC_OK;
}

gipc_status gipc_pcg_mf(gipc_ctx* ctx, const double* diag, const double* b, double* x, double rtol, int32_t maxit,
                        int32_t* iters, double* relres, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    MfView m{};
    if ((st = mf_view(ctx, diag, m, S(stream))) != GIPC_OK) return st;
    if (m.V > 0 && (!b || !x)) return fail(ctx, GIPC_ERR_INVALID_ARG, "b or x is NULL");
    if (!(rtol >= 0.0) || maxit < 0) return fail(ctx, GIPC_ERR_INVALID_ARG, "rtol must be >= 0 and maxit >= 0");
    int32_t it = 0;
    double rr = 0.0;
    int brk = 0;
    gipc_bsr none{};
    if (m.V > 0) CK(pcg_run(ctx, none, b, x, rtol, maxit, &it, &rr, &brk, S(stream), &m), "pcg");
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (brk) return fail(ctx, GIPC_ERR_BREAKDOWN, "p^T A p <= 0 at iteration %d", it);
    if (rtol > 0.0 && rr > rtol) return GIPC_WARN_NOT_CONVERGED;
    return GIPC_OK;
}

gipc_status gipc_pair_inspect(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, int32_t* src,
                              int32_t* type, int32_t* vid, int32_t* mult, double* energy, double* grad,
                              double* hess, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "no build");
    if ((grad || hess) && !ctx->evaluated) return fail(ctx, GIPC_ERR_STATE, "grad / hess need an eval");
    DevParams pm{};
    const double *x = nullptr, *xr = nullptr;
    if (energy) {
        if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
        if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;
        if (mesh->V != ctx->V) return fail(ctx, GIPC_ERR_STATE, "V differs from the build");
        if ((st = bind_batch(ctx, params, pm)) != GIPC_OK) return st;
        x = mesh->x;
        xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    }
    CK(launch_pair_inspect(as<int4>(ctx->st_vid), as<int32_t>(ctx->st_src),
                           ctx->merged ? as<int32_t>(ctx->mult) : nullptr, ctx->ranges, as<double>(ctx->rec_main),
                           as<double>(ctx->rec_extra), as<double>(ctx->rec_a1), x, xr, pm, src, type, vid, mult, energy, grad, hess,
                           S(stream)),
       "pair inspect");
    return GIPC_OK;
}

gipc_status gipc_candidates(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_topology* topo, double dhat,
                            int32_t* tuples, int64_t cap, int64_t* count, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    if (!topo || !count) return fail(ctx, GIPC_ERR_INVALID_ARG, "topology or count is NULL");
    if (topo->F < 0 || topo->E < 0 || topo->F >= (int64_t(1) << 31) || topo->E >= (int64_t(1) << 31))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "F and E must be in [0, 2^31)");
    if ((topo->F > 0 && !topo->tris) || (topo->E > 0 && !topo->edges) || (mesh->V > 0 && !topo->vobj))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "topology array is NULL");
    if (!(dhat >= 0.0) || !std::isfinite(dhat)) return fail(ctx, GIPC_ERR_INVALID_ARG, "dhat must be >= 0, finite");
    *count = 0;
    const int32_t V = mesh->V;
    const int64_t F = topo->F, E = topo->E;
    if (V == 0) return GIPC_OK;
    hipStream_t s = S(stream);
    const double* x = mesh->x;

    // topology ids
    CK(ensure(ctx->ccnt, sizeof(int64_t) * 2), "alloc candidates");
    const int64_t init[2] = {0, INT64_MAX};
    CK(hipMemcpyAsync(ctx->ccnt.p, init, sizeof(init), hipMemcpyHostToDevice, s), "copy");
    CK(launch_cand_check(V, topo->vobj, topo->tris, F, topo->edges, E, as<int64_t>(ctx->ccnt), s), "topology check");
    int64_t bad[2];
    CK(hipMemcpyAsync(bad, ctx->ccnt.p, sizeof(bad), hipMemcpyDeviceToHost, s), "copy");
    CK(hipStreamSynchronize(s), "stream synchronize");
    if (bad[0] > 0)
        return fail(ctx, GIPC_ERR_INDEX, "%lld primitives have vertex ids out of range or repeated (first: %lld)",
                    (long long)bad[0], (long long)bad[1]);

    // bounds and grid
    const int32_t nb = cand_bound_blocks(V, F + E);
    CK(ensure(ctx->cpart, sizeof(double) * 9 * (size_t)nb), "alloc candidates");
    CK(launch_cand_bounds(x, V, topo->tris, F, topo->edges, E, as<double>(ctx->cpart), nb, s), "bounds");
    std::vector<double> part(9 * (size_t)nb);
    CK(hipMemcpyAsync(part.data(), ctx->cpart.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s), "copy");
    CK(hipStreamSynchronize(s), "stream synchronize");
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, ext[3] = {0, 0, 0};
    for (int32_t b = 0; b < nb; ++b) {
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], part[9 * b + d]);
            hi[d] = std::max(hi[d], part[9 * b + 3 + d]);
            ext[d] = std::max(ext[d], part[9 * b + 6 + d]);
        }
    }
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d])) return fail(ctx, GIPC_ERR_INVALID_ARG, "non-finite positions");
    // per axis: the largest extent plus dhat (at least a thousandth of the
    // largest one, so flat meshes do not make empty slivers of cells)
    CandGrid g;
    const double hmax = std::max(ext[0], std::max(ext[1], ext[2])) + dhat;
    double ncell_d = 1.0;
    for (int d = 0; d < 3; ++d) {
        g.h[d] = std::max(ext[d] + dhat, 1e-3 * hmax);
        if (!(g.h[d] > 0.0)) g.h[d] = 1.0;
        g.org[d] = lo[d] - 4.0 * dhat;
        const double nd = std::floor((hi[d] + dhat - g.org[d]) / g.h[d]) + 1.0;
        if (!(nd < 2147483647.0)) return fail(ctx, GIPC_ERR_WORKSPACE, "grid too large");
        g.n[d] = (int32_t)std::max(1.0, nd);
        ncell_d *= g.n[d];
    }
    if (ncell_d > (double)(int64_t(1) << 28))
        return fail(ctx, GIPC_ERR_WORKSPACE,
                    "grid of %.0f cells exceeds 2^28 (extent too large for the largest primitive plus dhat)", ncell_d);
    const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];

    // four cell tables: triangles, edges (each primitive in the cells its box
    // covers, lists sorted by id), and the point and edge queries (each in
    // the cells its box inflated by dhat covers); counters and fills per table
    const int64_t Q[2] = {V, E};
    CK(ensure(ctx->ccount, sizeof(int32_t) * 4 * (size_t)ncell), "alloc candidates");
    CK(ensure(ctx->cfill, sizeof(int32_t) * 4 * (size_t)ncell), "alloc candidates");
    int32_t* cnt4 = as<int32_t>(ctx->ccount);
    int32_t* fill4 = as<int32_t>(ctx->cfill);
    DevBuf* toff[2] = {&ctx->coff_t, &ctx->coff_e};
    DevBuf* tent[2] = {&ctx->cent_t, &ctx->cent_e};
    DevBuf* trec[2] = {&ctx->crec_t, &ctx->crec_e};
    DevBuf* qtoff[2] = {&ctx->qtoff_p, &ctx->qtoff_e};
    DevBuf* qent[2] = {&ctx->qent_p, &ctx->qent_e};
    DevBuf* qeoff[2] = {&ctx->qoff_p, &ctx->qoff_e};
    DevBuf* ecnt[2] = {&ctx->ecnt_p, &ctx->ecnt_e};
    DevBuf* eoff[2] = {&ctx->eoff_p, &ctx->eoff_e};
    for (int k = 0; k < 2; ++k) {
        CK(ensure(*toff[k], sizeof(int64_t) * (size_t)(ncell + 1)), "alloc candidates");
        CK(ensure(*qtoff[k], sizeof(int64_t) * (size_t)(ncell + 1)), "alloc candidates");
        CK(ensure(*qeoff[k], sizeof(int64_t) * (size_t)(Q[k] + 1)), "alloc candidates");
    }
    CK(ensure(ctx->qcnt, sizeof(int32_t) * (size_t)std::max<int64_t>(std::max<int64_t>(V, E), 1)), "alloc candidates");
    CK(ensure(ctx->crec_t, (size_t)kPrimRecBytes * (size_t)(F > 0 ? F : 1)), "alloc candidates");
    CK(ensure(ctx->crec_e, (size_t)kPrimRecBytes * (size_t)(E > 0 ? E : 1)), "alloc candidates");
    CK(launch_prim_records(x, topo->tris, 3, F, topo->vobj, ctx->crec_t.p, s), "triangle records");
    CK(launch_prim_records(x, topo->edges, 2, E, topo->vobj, ctx->crec_e.p, s), "edge records");
    CK(launch_cell_count(ctx, x, topo->tris, 3, F, g, cnt4, fill4, as<int64_t>(ctx->coff_t), s), "triangle cells");
    CK(launch_cell_count(ctx, x, topo->edges, 2, E, g, cnt4 + ncell, fill4 + ncell, as<int64_t>(ctx->coff_e), s),
       "edge cells");
    CK(hipMemsetAsync(cnt4 + 2 * ncell, 0, sizeof(int32_t) * 2 * (size_t)ncell, s), "clear");
    CK(hipMemsetAsync(fill4 + 2 * ncell, 0, sizeof(int32_t) * 2 * (size_t)ncell, s), "clear");
    for (int k = 0; k < 2; ++k) {
        int32_t* span = as<int32_t>(ctx->qcnt);
        CK(launch_qcells_count(k, x, Q[k], k ? ctx->crec_e.p : nullptr, g, dhat, span, cnt4 + (2 + k) * ncell, s),
           "query cells");
        CK((exclusive_scan<int32_t, int64_t>(cnt4 + (2 + k) * ncell, ncell, as<int64_t>(*qtoff[k]), ctx, s)), "scan");
        CK((exclusive_scan<int32_t, int64_t>(span, Q[k], as<int64_t>(*qeoff[k]), ctx, s)), "scan");
    }
    // hit-mask slots of each kind's pairs pass, per cell
    DevBuf* boff[2] = {&ctx->boff_p, &ctx->boff_e};
    DevBuf* bal[2] = {&ctx->bal_p, &ctx->bal_e};
    DevBuf* evis[2] = {&ctx->evis_p, &ctx->evis_e};
    CK(ensure(ctx->bslot, sizeof(int64_t) * (size_t)ncell), "alloc candidates");
    for (int k = 0; k < 2; ++k) {
        CK(ensure(*boff[k], sizeof(int64_t) * (size_t)(ncell + 1)), "alloc candidates");
        CK(launch_cell_slots(k, g, as<int64_t>(*qtoff[k]), as<int64_t>(*toff[k]), as<int64_t>(ctx->bslot), s),
           "mask slots");
        CK((exclusive_scan<int64_t, int64_t>(as<int64_t>(ctx->bslot), ncell, as<int64_t>(*boff[k]), ctx, s)), "scan");
    }
    int64_t tot[6];  // triangle entries, edge entries, point visits, edge visits, mask slots (2)
    CK(hipMemcpyAsync(&tot[0], as<int64_t>(ctx->coff_t) + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&tot[1], as<int64_t>(ctx->coff_e) + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&tot[2], as<int64_t>(ctx->qoff_p) + V, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&tot[3], as<int64_t>(ctx->qoff_e) + E, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&tot[4], as<int64_t>(ctx->boff_p) + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&tot[5], as<int64_t>(ctx->boff_e) + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipStreamSynchronize(s), "stream synchronize");

    // fills, then per query and cell visited: candidate counts, offsets
    const int32_t* tp[2] = {topo->tris, topo->edges};
    CK(ensure(ctx->craw, sizeof(int32_t) * (size_t)(std::max(tot[0], tot[1]) + 1)), "alloc candidates");
    for (int k = 0; k < 2; ++k) {
        CK(ensure(*tent[k], sizeof(int32_t) * (size_t)(tot[k] + 1)), "alloc candidates");
        CK(ensure(*qent[k], sizeof(int32_t) * (size_t)(tot[2 + k] + 1)), "alloc candidates");
        CK(ensure(*ecnt[k], sizeof(int32_t) * (size_t)(tot[2 + k] + 1)), "alloc candidates");
        CK(ensure(*eoff[k], sizeof(int64_t) * (size_t)(tot[2 + k] + 1)), "alloc candidates");
        CK(ensure(*bal[k], sizeof(uint64_t) * (size_t)(tot[4 + k] + 1)), "alloc candidates");
        CK(ensure(*evis[k], sizeof(int64_t) * (size_t)(tot[2 + k] + 1)), "alloc candidates");
        CK(launch_cell_fill(x, tp[k], 3 - k, k ? E : F, g, fill4 + k * ncell, as<int64_t>(*toff[k]),
                            as<int32_t>(ctx->craw), as<int32_t>(*tent[k]), s),
           "primitive cells");
        CK(launch_qcells_fill(k, x, Q[k], k ? ctx->crec_e.p : nullptr, g, dhat, as<int64_t>(*qtoff[k]),
                              fill4 + (2 + k) * ncell, as<int32_t>(*qent[k]), s),
           "query cells");
    }
    for (int k = 0; k < 2; ++k) {
        CK(launch_cell_pairs(k, false, x, topo->vobj, k ? ctx->crec_e.p : nullptr, trec[k]->p, g, dhat,
                             as<int64_t>(*qtoff[k]), as<int32_t>(*qent[k]), as<int64_t>(*qeoff[k]),
                             as<int64_t>(*toff[k]), as<int32_t>(*tent[k]), as<int32_t>(*ecnt[k]), nullptr,
                             as<int64_t>(*boff[k]), as<uint64_t>(*bal[k]), as<int64_t>(*evis[k]), nullptr, s),
           k ? "edge-edge count" : "point-triangle count");
        CK((exclusive_scan<int32_t, int64_t>(as<int32_t>(*ecnt[k]), tot[2 + k], as<int64_t>(*eoff[k]), ctx, s)),
           "scan");
    }
    int64_t npt = 0, nee = 0;
    CK(hipMemcpyAsync(&npt, as<int64_t>(ctx->eoff_p) + tot[2], sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipMemcpyAsync(&nee, as<int64_t>(ctx->eoff_e) + tot[3], sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
    CK(hipStreamSynchronize(s), "stream synchronize");
    *count = npt + nee;
    if (!tuples) return GIPC_OK;
    if (cap < *count)
        return fail(ctx, GIPC_ERR_WORKSPACE, "cap = %lld is below the %lld candidates", (long long)cap,
                    (long long)*count);
    for (int k = 0; k < 2; ++k) {
        CK(launch_cell_pairs(k, true, x, topo->vobj, k ? ctx->crec_e.p : nullptr, trec[k]->p, g, dhat,
                             as<int64_t>(*qtoff[k]), as<int32_t>(*qent[k]), as<int64_t>(*qeoff[k]),
                             as<int64_t>(*toff[k]), as<int32_t>(*tent[k]), nullptr, as<int64_t>(*eoff[k]),
                             as<int64_t>(*boff[k]), as<uint64_t>(*bal[k]), as<int64_t>(*evis[k]),
                             tuples + (k ? 4 * npt : 0), s),
           k ? "edge-edge emit" : "point-triangle emit");
    }
    CK(hipStreamSynchronize(s), "stream synchronize");
    return GIPC_OK;
}

gipc_status gipc_friction_lag(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params,
                              const gipc_friction* fr, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!fr) return fail(ctx, GIPC_ERR_INVALID_ARG, "friction parameters are NULL");
    if (!(fr->mu >= 0.0) || !std::isfinite(fr->mu) || !(fr->eps_v > 0.0) || !std::isfinite(fr->eps_v) ||
        !(fr->dt > 0.0) || !std::isfinite(fr->dt))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "need mu >= 0, eps_v > 0 and dt > 0, finite");
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    DevParams pm;
    if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "gipc_pairs_build has not succeeded");
    if (mesh->V != ctx->V) return fail(ctx, GIPC_ERR_STATE, "V = %d differs from the build (%d)", mesh->V, ctx->V);
    if ((st = bind_batch(ctx, params, pm)) != GIPC_OK) return st;
    const int64_t Ps = ctx->Ps;
    CK(ensure(ctx->flag, sizeof(double) * 9 * (size_t)(Ps > 0 ? Ps : 1)), "alloc friction");
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    CK(launch_fric_lag(as<int4>(ctx->st_vid), ctx->merged ? as<int32_t>(ctx->mult) : nullptr, ctx->ranges, mesh->x,
                       xr, pm, fr->mu, as<double>(ctx->flag), S(stream)),
       "friction lag");
    ctx->fric_gen = ctx->build_gen;
    ctx->fric_sv = fr->eps_v * fr->dt;
    return GIPC_OK;
}

gipc_status gipc_friction_eval(gipc_ctx* ctx, const double* x, double* energy, double* grad, const gipc_bsr* A,
                               void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (!ctx->built || ctx->fric_gen != ctx->build_gen)
        return fail(ctx, GIPC_ERR_STATE, "gipc_friction_lag must follow the last gipc_pairs_build");
    if (!energy || (ctx->V > 0 && (!x || !grad))) return fail(ctx, GIPC_ERR_INVALID_ARG, "x, energy or grad is NULL");
    if (A) {
        if (!A->val) return fail(ctx, GIPC_ERR_INVALID_ARG, "A->val is NULL");
        if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return fail(ctx, GIPC_ERR_INVALID_ARG, "bad dtype");
        if (!same_pattern(ctx, A)) return fail(ctx, GIPC_ERR_STATE, "A is not the pattern of the last build");
    }
    const int64_t Ps = ctx->Ps;
    CK(ensure(ctx->ffr, sizeof(double) * 16 * (size_t)(Ps > 0 ? Ps : 1)), "alloc friction");
    CK(ensure(ctx->fev, sizeof(double) * (size_t)(ctx->V > 0 ? ctx->V : 1)), "alloc friction");
    CK(ensure(ctx->fpart, sizeof(double) * (size_t)(ctx->npieces > 0 ? ctx->npieces : 1)), "alloc friction");
    hipStream_t s = S(stream);
    CK(launch_fric_eval(ctx->V, as<int4>(ctx->st_vid), ctx->ranges, as<double>(ctx->flag), x, ctx->fric_sv,
                        as<double>(ctx->ffr), as<int32_t>(ctx->row_ptr), as<int32_t>(ctx->diag_slot),
                        as<int64_t>(ctx->cptr), as<uint32_t>(ctx->contrib), grad, as<double>(ctx->fev),
                        A ? A->val : nullptr, A ? A->dtype : 0, ctx->nnzb, s),
       "friction eval");
    CK(launch_energy(as<double>(ctx->fev), as<int2>(ctx->pieces), ctx->npieces, as<int32_t>(ctx->poff), ctx->S,
                     as<double>(ctx->fpart), energy, s),
       "friction energy");
    return GIPC_OK;
}

gipc_status gipc_proxy_dense(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, int32_t method,
                             double* hess, void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (method != GIPC_PROJ_ANALYTIC && method != GIPC_PROJ_NUMERIC && method != GIPC_PROJ_EXACT)
        return fail(ctx, GIPC_ERR_INVALID_ARG, "method must be GIPC_PROJ_ANALYTIC, _NUMERIC or _EXACT");
    if ((st = check_mesh(ctx, mesh)) != GIPC_OK) return st;
    DevParams pm;
    if ((st = to_dev_params(ctx, params, pm)) != GIPC_OK) return st;
    if (!ctx->built) return fail(ctx, GIPC_ERR_STATE, "gipc_pairs_build has not succeeded");
    if (mesh->V != ctx->V) return fail(ctx, GIPC_ERR_STATE, "V = %d differs from the build (%d)", mesh->V, ctx->V);
    if ((st = bind_batch(ctx, params, pm)) != GIPC_OK) return st;
    if (ctx->Ps > 0 && !hess) return fail(ctx, GIPC_ERR_INVALID_ARG, "hess is NULL");
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    CK(launch_proxy_dense(method, as<int4>(ctx->st_vid), ctx->merged ? as<int32_t>(ctx->mult) : nullptr,
                          ctx->ranges, mesh->x, xr, pm, hess, S(stream)),
       "dense proxy Hessians");
    return GIPC_OK;
}

gipc_status gipc_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    if (bytes < 0 || (bytes > 0 && (!src || !dst))) return GIPC_ERR_INVALID_ARG;
    if (launch_copy(src, dst, bytes, S(stream)) != hipSuccess) return GIPC_ERR_HIP;
    return GIPC_OK;
}

gipc_status gipc_read(const void* src, int64_t bytes, void* sink, void* stream) {
    if (bytes < 0 || (bytes >= 16 && (!src || !sink)) || (reinterpret_cast<uintptr_t>(src) & 15))
        return GIPC_ERR_INVALID_ARG;
    if (launch_read(src, bytes, static_cast<uint32_t*>(sink), S(stream)) != hipSuccess) return GIPC_ERR_HIP;
    return GIPC_OK;
}

// ---------------------------------------------------------------- tuning

gipc_status gipc_get_tune(const gipc_ctx* ctx, gipc_tune* tune) {
    if (!ctx || !tune) return GIPC_ERR_INVALID_ARG;
    *tune = ctx->tune;
    return GIPC_OK;
}

gipc_status gipc_set_tune(gipc_ctx* ctx, const gipc_tune* tune) {
    if (!ctx || !tune) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!tune_ok(*tune))
        return fail(ctx, GIPC_ERR_INVALID_ARG, "unsupported launch shape {%d, %d, %d, %d}", tune->eval_waves,
                    tune->row_lanes, tune->offdiag_waves, tune->row_order);
    ctx->tune = *tune;
    return GIPC_OK;
}

gipc_status gipc_autotune(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                          double* grad, const double* diag, const gipc_bsr* A, int32_t reps, gipc_tune* best,
                          void* stream) {
    if (!ctx) return GIPC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (reps < 1) return fail(ctx, GIPC_ERR_INVALID_ARG, "reps must be >= 1");
    gipc_status st;
    DevParams pm;
    if ((st = eval_check(ctx, mesh, params, energy, grad, A, true, pm)) != GIPC_OK) return st;
    if ((st = eval_prepare(ctx)) != GIPC_OK) return st;
    hipStream_t s = S(stream);
    const double* xr = mesh->x_rest ? mesh->x_rest : mesh->x;
    const TypeRanges& tr = ctx->ranges;
    const int64_t m0 = tr.off[FT_EEM], e0 = tr.off[FT_EE];
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    CK(hipEventCreate(&ev0), "event");
    if (hipEventCreate(&ev1) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return fail(ctx, GIPC_ERR_HIP, "event");
    }
    hipError_t err = hipSuccess;
    // one warm-up launch, then `reps` timed launches of the same kernel
    auto time_it = [&](auto launch) -> float {
        float ms = INFINITY;
        if (err != hipSuccess) return ms;
        if ((err = launch()) != hipSuccess) return ms;
        if ((err = hipEventRecord(ev0, s)) != hipSuccess) return ms;
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(ev1, s);
        if (err == hipSuccess) err = hipEventSynchronize(ev1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev0, ev1);
        return ms;
    };
    gipc_tune t = ctx->tune;
    const int waves[4] = {1, 2, 4, 8}, lanes[4] = {4, 8, 16, 32};
    float bt = INFINITY;
    for (int w : waves) {
        float ms = time_it([&] {
            return launch_eval(as<int4>(ctx->st_vid), ctx->merged ? as<int32_t>(ctx->mult) : nullptr, tr, mesh->x,
                               xr, pm, as<double>(ctx->rec_main), as<double>(ctx->rec_extra),
                               as<double>(ctx->rec_a1), w, s);
        });
        if (ms < bt) { bt = ms; t.eval_waves = w; }
    }
    bt = INFINITY;
    for (int l : lanes) {
        float ms = time_it([&] {
            return launch_rows_diag(3, ctx->V, visit_order(ctx, t.row_order), as<int32_t>(ctx->diag_slot), as<int64_t>(ctx->cptr),
                                    as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main), as<double>(ctx->rec_extra), as<double>(ctx->rec_a1),
                                    e0, m0, diag, grad, as<double>(ctx->ev), A->val, A->dtype, ctx->nnzb, l, s);
        });
        if (ms < bt) { bt = ms; t.row_lanes = l; }
    }
    bt = INFINITY;
    for (int w : waves) {
        float ms = time_it([&] {
            return launch_offdiag(ctx->V, visit_order(ctx, t.row_order), as<int32_t>(ctx->row_ptr), as<int32_t>(ctx->diag_slot),
                           ctx->nnzb, as<int32_t>(ctx->col_idx), as<int32_t>(ctx->tslot),
                                  as<int64_t>(ctx->cptr), as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main),
                                  as<double>(ctx->rec_extra), e0, m0, A->val, A->dtype, w, s);
        });
        if (ms < bt) { bt = ms; t.offdiag_waves = w; }
    }
    // the row order, both passes together with the chosen shapes
    bt = INFINITY;
    for (int o = 0; o < 2; ++o) {
        float ms = time_it([&] {
            hipError_t e2 = launch_rows_diag(3, ctx->V, visit_order(ctx, o), as<int32_t>(ctx->diag_slot),
                                             as<int64_t>(ctx->cptr), as<uint32_t>(ctx->contrib),
                                             as<double>(ctx->rec_main), as<double>(ctx->rec_extra),
                                             as<double>(ctx->rec_a1), e0, m0, diag, grad, as<double>(ctx->ev),
                                             A->val, A->dtype, ctx->nnzb, t.row_lanes, s);
            if (e2 != hipSuccess) return e2;
            return launch_offdiag(ctx->V, visit_order(ctx, o), as<int32_t>(ctx->row_ptr), as<int32_t>(ctx->diag_slot),
                                  ctx->nnzb, as<int32_t>(ctx->col_idx), as<int32_t>(ctx->tslot),
                                  as<int64_t>(ctx->cptr), as<uint32_t>(ctx->contrib), as<double>(ctx->rec_main),
                                  as<double>(ctx->rec_extra), e0, m0, A->val, A->dtype, t.offdiag_waves, s);
        });
        if (ms < bt) { bt = ms; t.row_order = o; }
    }
    if (err == hipSuccess)
        err = launch_energy(as<double>(ctx->ev), as<int2>(ctx->pieces), ctx->npieces, as<int32_t>(ctx->poff),
                            ctx->S, as<double>(ctx->epart), energy, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (err != hipSuccess) return hip_fail(ctx, err, "autotune");
    ctx->tune = t;
    ctx->evaluated = true;
    ++ctx->eval_gen;
    if (best) *best = t;
    return GIPC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- graphs

struct gipc_graph {
    gipc_ctx* ctx = nullptr;
    uint64_t gen = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

gipc_status gipc_graph_create(gipc_ctx* ctx, const gipc_mesh* mesh, const gipc_params* params, double* energy,
                              double* grad, const double* diag, const gipc_bsr* A, gipc_graph** out) {
    if (!ctx || !out) return GIPC_ERR_INVALID_ARG;
    *out = nullptr;
    ctx->err.clear();
    gipc_status st;
    DevParams pm;
    if ((st = eval_check(ctx, mesh, params, energy, grad, A, true, pm)) != GIPC_OK) return st;
    if ((st = eval_prepare(ctx)) != GIPC_OK) return st;
    gipc_graph* g = new (std::nothrow) gipc_graph();
    if (!g) return fail(ctx, GIPC_ERR_WORKSPACE, "graph handle");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = eval_enqueue(ctx, pm, mesh, energy, grad, diag, A, true, ctx->tune, cs);
            e = hipStreamEndCapture(cs, &g->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
    }
    if (e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(ctx, e, "graph capture");
    }
    g->ctx = ctx;
    g->gen = ctx->build_gen;
    *out = g;
    return GIPC_OK;
}

gipc_status gipc_graph_launch(gipc_graph* g, void* stream) {
    if (!g || !g->ctx) return GIPC_ERR_INVALID_ARG;
    gipc_ctx* ctx = g->ctx;
    ctx->err.clear();
    gipc_status st;
    if ((st = check_device(ctx)) != GIPC_OK) return st;
    if (g->gen != ctx->build_gen || !ctx->built)
        return fail(ctx, GIPC_ERR_STATE, "the graph was captured before the last gipc_pairs_build");
    CK(hipGraphLaunch(g->exec, S(stream)), "graph launch");
    ctx->evaluated = true;
    ++ctx->eval_gen;
    return GIPC_OK;
}

void gipc_graph_destroy(gipc_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
