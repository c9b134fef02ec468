// gipc_pcg_static: the block-Jacobi PCG of gipc_pcg on a work area that is
// part of the library's code object, for callers that cannot allocate
// device memory.  The kernels and the launch sequence are gipc_pcg's own
// (pcg_run_in); only the buffers differ.
#include <mutex>

#include "internal.hpp"

namespace {

// One per device: HIP places a copy of every __device__ variable on each
// GPU the code object is loaded on, at that GPU's own address.
static __device__ __align__(256) char scratch[GIPC_PCG_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// The device address of this GPU's copy of `scratch`, looked up once per
// device with that device current (the array's name is only a host-side
// stand-in in host code).
hipError_t scratch_ptr(int dev, void** out) {
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" gipc_status gipc_pcg_static(const gipc_bsr* A, const double* b, double* x, double rtol, int32_t maxit,
                                       int32_t* iters, double* relres, void* stream) {
    using namespace gipc;
    if (!A || A->nbrows < 0 || A->nnzb < 0) return GIPC_ERR_INVALID_ARG;
    if (A->dtype != GIPC_F64 && A->dtype != GIPC_F32) return GIPC_ERR_INVALID_ARG;
    if (A->nbrows > 0 && (!A->row_ptr || !A->col_idx || !A->val || !b || !x)) return GIPC_ERR_INVALID_ARG;
    if (!(rtol >= 0.0) || maxit < 0) return GIPC_ERR_INVALID_ARG;
    if (pcg_workspace_bytes(*A, nullptr) > (size_t)GIPC_PCG_STATIC_SCRATCH_BYTES) return GIPC_ERR_WORKSPACE;
    int32_t it = 0;
    double rr = 0.0;
    int brk = 0;
    // rtol = 0 with no counts asked for: enqueue only (nothing read back)
    const bool enqueue_only = rtol == 0.0 && !iters && !relres;
    if (A->nbrows > 0) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GIPC_ERR_HIP;
        void* ws = nullptr;
        if (scratch_ptr(dev, &ws) != hipSuccess) return GIPC_ERR_HIP;
        if (pcg_run_in(ws, *A, b, x, rtol, maxit, enqueue_only ? nullptr : &it, enqueue_only ? nullptr : &rr,
                       enqueue_only ? nullptr : &brk, static_cast<hipStream_t>(stream)) != hipSuccess) {
            (void)hipGetLastError();
            return GIPC_ERR_HIP;
        }
    }
    if (iters) *iters = it;
    if (relres) *relres = rr;
    if (brk) return GIPC_ERR_BREAKDOWN;
    if (rtol > 0.0 && rr > rtol) return GIPC_WARN_NOT_CONVERGED;
    return GIPC_OK;
}
