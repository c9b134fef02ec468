/*
 * The library's C ABI driven from plain C: no Python binding, no torch.
 * Test infrastructure (tests/test_gpu_abi_c.py writes the input, runs this
 * program and checks the output against the oracle).
 *
 * usage: abi_check <input> <output>
 *   input  (little endian): int32 V, int64 P, double dhat, double kappa,
 *          int32 maxit, double x[V][3], double x_rest[V][3], double diag[V],
 *          int32 tuples[P][4]
 *   output: int32 status of every call in order (6), double energy,
 *          int64 nnzb, int32 iters, double relres, double grad[V][3],
 *          int32 row_ptr[V+1], int32 col_idx[nnzb], double val[9][nnzb],
 *          double y[V][3] (A grad), double sol[V][3] (PCG on A s = -grad,
 *          s0 = 0, rtol 0, maxit iterations)
 * Exit status 0 when every call ran (the statuses are in the output), 1 for
 * a bad input file, 2 for a HIP runtime error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "gipc.h"

#define HIPCHK(x)                                                              \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            return 2;                                                          \
        }                                                                      \
    } while (0)

static int rd(FILE* f, void* p, size_t n) { return fread(p, 1, n, f) == n; }
static int wr(FILE* f, const void* p, size_t n) { return fwrite(p, 1, n, f) == n; }

/* device copy of a host array, NULL for n = 0 */
static hipError_t up(void** d, const void* h, size_t n) {
    *d = NULL;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc(d, n);
    if (e == hipSuccess) e = hipMemcpy(*d, h, n, hipMemcpyHostToDevice);
    return e;
}

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s <input> <output>\n", argv[0]);
        return 1;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t V = 0, maxit = 0;
    int64_t P = 0;
    double dhat = 0.0, kappa = 0.0;
    if (!rd(f, &V, 4) || !rd(f, &P, 8) || !rd(f, &dhat, 8) || !rd(f, &kappa, 8) || !rd(f, &maxit, 4) || V <= 0 ||
        P < 0) {
        fclose(f);
        return 1;
    }
    double* hx = malloc(sizeof(double) * 3 * (size_t)V);
    double* hxr = malloc(sizeof(double) * 3 * (size_t)V);
    double* hdiag = malloc(sizeof(double) * (size_t)V);
    int32_t* ht = malloc(sizeof(int32_t) * 4 * (size_t)(P > 0 ? P : 1));
    int ok = hx && hxr && hdiag && ht && rd(f, hx, sizeof(double) * 3 * (size_t)V) &&
             rd(f, hxr, sizeof(double) * 3 * (size_t)V) &&
             rd(f, hdiag, sizeof(double) * (size_t)V) && rd(f, ht, sizeof(int32_t) * 4 * (size_t)P);
    fclose(f);
    if (!ok) return 1;

    void *dx, *dxr, *ddiag, *dt, *dE, *dg, *dy, *db, *ds;
    HIPCHK(up(&dx, hx, sizeof(double) * 3 * (size_t)V));
    HIPCHK(up(&dxr, hxr, sizeof(double) * 3 * (size_t)V));
    HIPCHK(up(&ddiag, hdiag, sizeof(double) * (size_t)V));
    HIPCHK(up(&dt, ht, sizeof(int32_t) * 4 * (size_t)P));
    HIPCHK(hipMalloc(&dE, sizeof(double)));
    HIPCHK(hipMalloc(&dg, sizeof(double) * 3 * (size_t)V));
    HIPCHK(hipMalloc(&dy, sizeof(double) * 3 * (size_t)V));
    HIPCHK(hipMalloc(&db, sizeof(double) * 3 * (size_t)V));
    HIPCHK(hipMalloc(&ds, sizeof(double) * 3 * (size_t)V));
    HIPCHK(hipMemset(ds, 0, sizeof(double) * 3 * (size_t)V));

    int32_t st[6] = {-100, -100, -100, -100, -100, -100};
    gipc_ctx* ctx = NULL;
    st[0] = gipc_ctx_create(&ctx);
    gipc_mesh mesh = {V, (const double*)dx, (const double*)dxr};
    gipc_pairs pairs = {P, (const int32_t*)dt};
    gipc_params prm = {dhat, kappa, 0.1, 1e-3, GIPC_FLAG_FILTER | GIPC_FLAG_MOLLIFY, NULL};
    gipc_info info;
    memset(&info, 0, sizeof(info));
    gipc_bsr A;
    memset(&A, 0, sizeof(A));
    double* val = NULL;
    int32_t iters = 0;
    double relres = 0.0;
    if (st[0] == GIPC_OK) st[1] = gipc_pairs_build(ctx, &mesh, &pairs, &prm, NULL, &info);
    if (st[1] == GIPC_OK) st[2] = gipc_bsr_pattern(ctx, &A);
    if (st[2] == GIPC_OK) {
        HIPCHK(hipMalloc((void**)&val, sizeof(double) * 9 * (size_t)(A.nnzb > 0 ? A.nnzb : 1)));
        A.val = val;
        A.dtype = GIPC_F64;
        st[3] = gipc_eval_assemble(ctx, &mesh, &prm, (double*)dE, (double*)dg, (const double*)ddiag, &A, NULL);
    }
    if (st[3] == GIPC_OK) st[4] = gipc_bsr_spmv(&A, dg, dy, NULL);
    if (st[4] == GIPC_OK) {
        /* b = -grad, on the host (the library has no vector kernels to offer) */
        double* hg = malloc(sizeof(double) * 3 * (size_t)V);
        if (!hg) return 1;
        HIPCHK(hipMemcpy(hg, dg, sizeof(double) * 3 * (size_t)V, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < 3 * (int64_t)V; ++i) hg[i] = -hg[i];
        HIPCHK(hipMemcpy(db, hg, sizeof(double) * 3 * (size_t)V, hipMemcpyHostToDevice));
        free(hg);
        st[5] = gipc_pcg(ctx, &A, (const double*)db, (double*)ds, 0.0, maxit, &iters, &relres, NULL);
    }
    HIPCHK(hipDeviceSynchronize());

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 1;
    double E = 0.0;
    const int64_t nnzb = st[2] == GIPC_OK ? A.nnzb : 0;
    const size_t n3 = sizeof(double) * 3 * (size_t)V;
    void* buf = malloc(n3 > sizeof(double) * 9 * (size_t)nnzb ? n3 + 64 : sizeof(double) * 9 * (size_t)nnzb + 64);
    if (!buf) return 1;
    if (st[3] == GIPC_OK) HIPCHK(hipMemcpy(&E, dE, sizeof(double), hipMemcpyDeviceToHost));
    ok = wr(o, st, sizeof(st)) && wr(o, &E, 8) && wr(o, &nnzb, 8) && wr(o, &iters, 4) && wr(o, &relres, 8);
    if (ok && st[5] == GIPC_OK) {
        HIPCHK(hipMemcpy(buf, dg, n3, hipMemcpyDeviceToHost));
        ok = wr(o, buf, n3);
        HIPCHK(hipMemcpy(buf, A.row_ptr, sizeof(int32_t) * ((size_t)V + 1), hipMemcpyDeviceToHost));
        ok = ok && wr(o, buf, sizeof(int32_t) * ((size_t)V + 1));
        HIPCHK(hipMemcpy(buf, A.col_idx, sizeof(int32_t) * (size_t)nnzb, hipMemcpyDeviceToHost));
        ok = ok && wr(o, buf, sizeof(int32_t) * (size_t)nnzb);
        HIPCHK(hipMemcpy(buf, val, sizeof(double) * 9 * (size_t)nnzb, hipMemcpyDeviceToHost));
        ok = ok && wr(o, buf, sizeof(double) * 9 * (size_t)nnzb);
        HIPCHK(hipMemcpy(buf, dy, n3, hipMemcpyDeviceToHost));
        ok = ok && wr(o, buf, n3);
        HIPCHK(hipMemcpy(buf, ds, n3, hipMemcpyDeviceToHost));
        ok = ok && wr(o, buf, n3);
    }
    fclose(o);
    free(buf);
    gipc_ctx_destroy(ctx);
    hipFree(val);
    hipFree(dx);
    hipFree(dxr);
    hipFree(ddiag);
    hipFree(dt);
    hipFree(dE);
    hipFree(dg);
    hipFree(dy);
    hipFree(db);
    hipFree(ds);
    free(hx);
    free(hxr);
    free(hdiag);
    free(ht);
    return ok ? 0 : 1;
}
