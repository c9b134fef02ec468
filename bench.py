"""Benchmark of the GIPC barrier hot path on one MI355X.

Headline workload: 10 stacked cloth sheets of 256 x 256 vertices over the
unit square, sheet k at z = 0.6 k dhat with +-0.3 dhat per-vertex jitter, one
sheet sheared by 1 degree, dhat = 1e-3, kappa = 1e4, mass 1e-3 and dt = 1e-2
(diagonal term m / dt^2 = 10); contact candidates from an AABB broad phase
within dhat (host, untimed, seeded).

One step = the whole hot path on the resident candidate list:
  stage + pattern build (classification, type sort, BSR symbolic)
  + fused energy / gradient / proxy Hessian / BSR assembly
  + one BSR SpMV + 100 block-Jacobi PCG iterations on (M/dt^2 + H) d = -grad.
`value` is contact pairs per second -- the candidates that classification
finds closer than dhat, each one a term of the barrier sum -- through stage
+ build + eval/assembly (the metric's scope); candidate and staged-pair rates
are reported beside it, and the SpMV and PCG are timed in the same step.
Prints one JSON line.

After the headline steps the default run also measures the two targets of
the extensions on their own workloads (`targets` in the JSON; skip with
--no-targets), with contact candidates generated on the GPU:
  batch64: 64 two-sheet scenes of 32..256 vertices per side with per-scene
    dhat log-uniform in [1e-4, 1e-2] in one batch; a step is the batched
    stage + build and the eval + assembly replayed from a HIP graph (FP32
    blocks); against it the plain path: one context per scene, no merging
    of duplicate constraints, evaluation and assembly as separate calls,
    FP64 blocks, and the HBM fraction of the graph step;
  sheets40: 40 sheets (seed 5), FP32 Hessian blocks and FP32 SpMV, PCG to
    ||r|| / ||b|| <= 1e-6; the FP32 product and PCG iteration against the
    HBM roofline, and the FP64 path once on the same pattern for the
    comparison (block error, iterations, PCG time, solution difference).
--workload batch64 / sheets40 run one of them alone as the headline line.

After the timed steps the headline workload also runs the matrix-free
operator once against the FP64 BSR matrix of the same eval (one product
each; the PCG of the step both ways), reported under `matrix_free`, times
the dense projected proxy Hessians of all staged pairs from the analytic
eigensystems against the numeric baseline under `numeric_eigen_baseline`,
the lagged friction on the same pairs under `friction`, and the GPU contact
candidates of the scene's surfaces under `candidates`.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak

# HBM bytes per launch of the roofline kernel on the headline workload from
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled by what the
# same counters read for the library's copy kernel on a 2 GiB buffer.  The
# figure holds only for the kernel source it was measured on: it is reported
# only while the SHA-256 of that source file still matches, else null.
MEASURED_TRAFFIC = {
    "kernel": "k_spmv_ent",
    "bytes": 1.801e9,
    "source": "profiles/sheets10_path.md (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 per dispatch, "
              "calibrated on the library's 2 GiB copy in the same run)",
    "file": "paper_2308_09400_amd/csrc/solve.hip",
    "sha256": "c6291caeb05ad8fcec59206c3ce7ac75e8bd7a46e7f4f484bed6b3e3c729ff19",
}


def _traffic_if_current():
    m = MEASURED_TRAFFIC
    try:
        with open(os.path.join(ROOT, m["file"]), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None, None
    if m["sha256"] is None or h != m["sha256"]:
        return None, f"null: {m['file']} changed since the counters were taken"
    return m["bytes"], m["source"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["sheets10", "sheets40", "batch64", "sheets2"], default="sheets10")
    ap.add_argument("--pcg-iters", type=int, default=100)
    ap.add_argument("--cpu-sample", type=int, default=5_000_000, help="candidates in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-targets", action="store_true", help="skip the batch64 / sheets40 target legs")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the matrix-free, numeric-eigen, friction and candidate legs")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch64: time only the batched step (no eager, per-scene or plain comparisons)")
    return ap.parse_args()


def gpu_candidates(gp, x, s):
    """Contact candidates of a scene's surfaces on the GPU (the same set as
    the host grid generator; device int32 [P][4])."""
    import torch
    dev = x.device
    ctx = gp.Context()
    vobj = torch.tensor(s.vobj, dtype=torch.int32, device=dev)
    tris = torch.tensor(s.tris, dtype=torch.int32, device=dev)
    edges = torch.tensor(s.edges, dtype=torch.int32, device=dev)
    t = gp.candidates(ctx, x, vobj, tris, edges, s.dhat)
    ctx.close()
    return t


def make_scene(name, with_pairs=True):
    import scenes
    if name == "sheets10":
        s = scenes.stacked_sheets(n_sheets=10, n=256, seed=2, with_pairs=with_pairs)
        desc = ("10 stacked 256x256 sheets, spacing 0.6 dhat, jitter +-0.3 dhat, 1 sheared sheet, dhat=1e-3, "
                "kappa=1e4, m/dt^2=10, AABB candidates within dhat")
    elif name == "sheets40":
        s = scenes.stacked_sheets(n_sheets=40, n=256, seed=5, with_pairs=with_pairs)
        desc = ("40 stacked 256x256 sheets, spacing 0.6 dhat, jitter +-0.3 dhat, 1 sheared sheet, dhat=1e-3, "
                "kappa=1e4, m/dt^2=10, AABB candidates within dhat; FP32 blocks and SpMV, PCG to 1e-6")
    else:
        s = scenes.two_sheets(n=16, seed=1, with_pairs=with_pairs)
        s.diag = np.full(s.V, 10.0)
        desc = "two 16x16 sheets, offset 0.5 dhat, jitter +-0.2 dhat, dhat=1e-3, kappa=1e4"
    return s, desc


def cpu_baseline(s, n_sample, nthreads=0):
    """The oracle as it stands (eval with per-pair Hessians + assembly) on a
    seeded sample, each stage timed, then its SpMV and ten PCG iterations on
    the sample's matrix."""
    import oracle
    import scenes
    sub = scenes.subsample(s, n_sample, seed=7)
    prm = oracle.params(dhat=s.dhat, kappa=s.kappa)
    t0 = time.perf_counter()
    r = oracle.eval_scene(s.x, sub, prm, x_rest=s.x_rest, nthreads=nthreads, per_pair=True)
    t1 = time.perf_counter()
    rows, cols, vals = oracle.assemble(s.V, sub, r["pairH"], s.diag)
    t2 = time.perf_counter()
    xv = np.random.default_rng(0).normal(size=3 * s.V)
    oracle.spmv(s.V, rows, cols, vals, xv)
    t3 = time.perf_counter()
    oracle.pcg(s.V, rows, cols, vals, -r["grad"].reshape(-1), rtol=0.0, maxit=10)
    t4 = time.perf_counter()
    dt = t2 - t0
    cores = nthreads if nthreads > 0 else oracle.num_threads()
    return {"value": len(sub) / dt, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sub)} candidates drawn (seed 7) from the same list; oracle eval with per-pair "
                      f"Hessians ({cores} thread(s), {t1 - t0:.1f} s) + assembly (serial sort, {t2 - t1:.1f} s); "
                      f"{dt:.1f} s",
            "eval_pairs_per_s": len(sub) / (t1 - t0), "assembly_s": t2 - t1,
            "sample_nnzb": int(len(rows)), "spmv_ms": (t3 - t2) * 1e3, "pcg_ms_per_iter": (t4 - t3) * 1e3 / 10}


def precision_compare(gp, ctx, x, xr, prm, diag, last, stream):
    """The FP64 path once on the same pattern: block error of the FP32
    matrix, PCG iterations and time at the same tolerance, solution gap."""
    import torch
    _, _, A32, d32, b = last
    A64 = gp.BsrMatrix(ctx, dtype=gp.F64)
    gp.eval_assemble(ctx, x, prm, A64, diag=diag, x_rest=xr)
    n = A64.nnzb
    fro = float(torch.linalg.norm(A32.val[:, :n].double() - A64.val[:, :n]) / torch.linalg.norm(A64.val[:, :n]))
    out = {"block_rel_fro": fro}
    for name, A in (("f64", A64), ("f32", A32)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d, it, rr, st = gp.pcg(ctx, A, b, rtol=1e-6, maxit=20000)
        e1.record(stream)
        torch.cuda.synchronize()
        out[f"pcg_{name}"] = {"iters": it, "relres": rr, "ms": e0.elapsed_time(e1), "status": st}
        out[f"x_{name}"] = d
    x64, x32 = out.pop("x_f64"), out.pop("x_f32")
    out["x_rel_diff"] = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    out["fp32_true_relres"] = float(torch.linalg.norm(b - gp.bsr_spmv(A64, x32)) / torch.linalg.norm(b))
    del A64
    return out


INC_PER_TYPE = {"PT": 4, "PE": 3, "PP": 2, "EE": 4, "EE_moll": 4, "PE_moll": 4, "PP_moll": 4}


def matrix_free_compare(gp, ctx, x, xr, prm, diag, info, rtol, maxit, stream):
    """The matrix-free operator against the FP64 BSR matrix of the same eval:
    one product each, and the linear solve of a Newton step both ways
    (eval + assembly + PCG against eval + matrix-free PCG)."""
    import torch
    A = gp.BsrMatrix(ctx, dtype=gp.F64)
    gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
    V = x.shape[0]
    v = torch.tensor(np.random.default_rng(0).normal(size=(V, 3)), device=x.device)
    yb, ym = torch.empty_like(v), torch.empty_like(v)
    t_spmv = _median_ms(lambda: gp.bsr_spmv(A, v, yb), 20, stream)
    t_mf = _median_ms(lambda: gp.mf_apply(ctx, v, ym, diag=diag), 20, stream)
    gap = float((ym - yb).abs().max() / yb.abs().max())
    st = info["n_staged_by_type"]
    Ps = sum(st.values())
    Pm = st["EE_moll"] + st["PE_moll"] + st["PP_moll"]
    inc = sum(INC_PER_TYPE[k] * n for k, n in st.items())
    # algorithmic bytes of one matrix-free product (two passes), each datum
    # counted once: stencils 16 B and the operator fields of the records
    # (c1 c2 w~ P22: 48 B; u v P11 P12: 64 B); (alpha, beta) 16 B written
    # and read; per incidence its 24 B vector c_i w~ and 4 B list code; x and
    # diag read and y written; 16 B of row metadata
    mf_bytes = Ps * (16 + 48 + 32) + Pm * 64 + inc * (24 + 4) + V * (24 + 8 + 24 + 16)
    nnzb = A.nnzb
    spmv_bytes = nnzb * (9 * 8 + 4) + 4 * (V + 1) + 48 * V
    t_eval = _median_ms(lambda: gp.barrier_eval(ctx, x, prm, x_rest=xr), 5, stream)
    E, g = gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
    t_evas = _median_ms(lambda: gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr), 5, stream)
    b = -g
    res = {}
    for name, fn in (("bsr", lambda: gp.pcg(ctx, A, b, rtol=rtol, maxit=maxit)),
                     ("mf", lambda: gp.pcg_mf(ctx, b, diag=diag, rtol=rtol, maxit=maxit))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d, it, rr, stt = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = {"iters": it, "relres": rr, "ms": e0.elapsed_time(e1), "d": d}
    dgap = float(torch.linalg.norm(res["mf"]["d"] - res["bsr"]["d"]) / torch.linalg.norm(res["bsr"]["d"]))
    for r in res.values():
        r.pop("d")
        r["ms_per_iter"] = r["ms"] / max(r["iters"], 1)
    del A
    return {
        "apply_ms": t_mf,
        "apply_gbs": mf_bytes / (t_mf * 1e-3) / 1e9,
        "apply_bytes": int(mf_bytes),
        "bsr_spmv_f64_ms": t_spmv,
        "bsr_spmv_f64_gbs": spmv_bytes / (t_spmv * 1e-3) / 1e9,
        "bsr_spmv_f64_bytes": int(spmv_bytes),
        "apply_vs_spmv_max_rel_gap": gap,
        "eval_only_ms": t_eval,
        "eval_assemble_f64_ms": t_evas,
        "pcg_bsr_f64": res["bsr"],
        "pcg_mf": res["mf"],
        "solution_rel_gap": dgap,
        "newton_solve_ms": {"bsr": t_evas + res["bsr"]["ms"], "mf": t_eval + res["mf"]["ms"]},
    }


def numeric_compare(gp, ctx, x, xr, prm, info, stream):
    """Table 1's comparison on this GPU: every staged pair's dense projected
    proxy Hessian from the analytic eigensystems against the numeric route
    (x-space matrix projected by cyclic Jacobi rotations), same output."""
    import torch
    n = int(info["n_staged"])
    st = info["n_staged_by_type"]
    hess = torch.empty((n, 12, 12), dtype=torch.float64, device=x.device)
    t_a = _median_ms(lambda: gp.proxy_dense(ctx, x, prm, gp.PROJ_ANALYTIC, x_rest=xr, hess=hess), 3, stream)
    t_n = _median_ms(lambda: gp.proxy_dense(ctx, x, prm, gp.PROJ_NUMERIC, x_rest=xr, hess=hess), 3, stream)
    del hess
    return {
        "pairs": n,
        "pairs_12x12": st["PT"] + st["EE"] + st["EE_moll"] + st["PE_moll"] + st["PP_moll"],
        "pairs_9x9": st["PE"], "pairs_6x6": st["PP"],
        "analytic_ms": t_a, "numeric_jacobi_ms": t_n, "speedup": t_n / t_a,
        "output_gb": n * 1152 / 1e9,
        "paper_table1": "10^7 12x12 Hessians: Eigen (CPU) 2.42e3 ms vs analytic 4.95e2 ms on the CPU (4.9x); "
                        "analytic on the GPU 9.01e1 ms; 16-core Intel Core i9 12900K and RTX 4090 (Sec. 8)",
    }


def dense_compare(gp, ctx, x, xr, prm, diag, info, stream, maxit=100):
    """Table 2's comparison on wave64: the matrix-free product from dense
    local Hessians, one lane per local mat-vec against one lane per matrix
    entry with a wavefront segmented reduction (both adding to y with FP64
    atomics), one product and a fixed-length PCG each, next to the
    factor-form operator and the BSR matrix of the same eval."""
    import torch
    st = info["n_staged_by_type"]
    n = int(info["n_staged"])
    n12 = st["PT"] + st["EE"] + st["EE_moll"] + st["PE_moll"] + st["PP_moll"]
    H = gp.proxy_dense(ctx, x, prm, gp.PROJ_ANALYTIC, x_rest=xr)
    E, g = gp.barrier_eval(ctx, x, prm, x_rest=xr)
    V = x.shape[0]
    v = torch.tensor(np.random.default_rng(0).normal(size=(V, 3)), device=x.device)
    y = torch.empty_like(v)
    entries = 144 * n12 + 81 * st["PE"] + 36 * st["PP"]
    # algorithmic bytes of one product: the dense entries, the stencils, x
    # and diag read, y written
    dbytes = 8 * entries + 16 * n + 24 * V + 8 * V + 24 * V
    ym = gp.mf_apply(ctx, v, diag=diag)
    res = {"pairs": n, "entries": int(entries), "apply_bytes": int(dbytes)}
    for name, scheme in (("thread_per_matvec", gp.DENSE_THREAD), ("entry_segmented", gp.DENSE_ENTRY)):
        t = _median_ms(lambda: gp.dense_apply(ctx, H, v, y=y, diag=diag, scheme=scheme), 5, stream)
        gap = float((y - ym).abs().max() / ym.abs().max())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d, it, rr, stt = gp.pcg_dense(ctx, H, -g, diag=diag, scheme=scheme, rtol=0.0, maxit=maxit)
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = {"apply_ms": t, "apply_gbs": dbytes / (t * 1e-3) / 1e9, "vs_factor_operator_max_rel_gap": gap,
                     "pcg_iters": it, "pcg_ms": e0.elapsed_time(e1), "pcg_ms_per_iter": e0.elapsed_time(e1) / it}
    res["entry_vs_thread_apply"] = res["thread_per_matvec"]["apply_ms"] / res["entry_segmented"]["apply_ms"]
    res["entry_vs_thread_pcg"] = res["thread_per_matvec"]["pcg_ms"] / res["entry_segmented"]["pcg_ms"]
    res["paper_table2"] = ("PCG time, warp reduction vs thread per local mat-vec: 3.82x-4.11x (avg 3.97x), "
                           "RTX 4090, FP64 (Table 2)")
    del H
    return res


def _table1_tuples(kind, n, dhat, seed, dev):
    """n active tuples of one kind, each on its own vertices (seeded, on the
    device): a point over a triangle's interior (12 x 12), beside a segment's
    interior (9 x 9) or near a point (6 x 6), at distance (0.1 .. 0.9) dhat."""
    import torch
    g = torch.Generator(device=dev).manual_seed(seed)
    L = 20.0 * dhat
    u = lambda *sh: torch.rand(*sh, generator=g, device=dev, dtype=torch.float64)  # noqa: E731
    h = (0.1 + 0.8 * u(n)) * dhat
    i64 = torch.arange(n, device=dev, dtype=torch.int64)
    base = 3.0 * L * torch.stack([i64 % 256, (i64 // 256) % 256, i64 // 65536], 1).to(torch.float64)
    if kind == 12:
        t0 = base
        t1 = base + torch.stack([L * (0.9 + 0.2 * u(n)), L * 0.1 * (u(n) - 0.5), torch.zeros_like(h)], 1)
        t2 = base + torch.stack([L * 0.1 * (u(n) - 0.5), L * (0.9 + 0.2 * u(n)), torch.zeros_like(h)], 1)
        p = base + torch.stack([L * (0.15 + 0.2 * u(n)), L * (0.15 + 0.2 * u(n)), h], 1)
        x = torch.stack([p, t0, t1, t2], 1).reshape(-1, 3)
        i = torch.arange(n, device=dev, dtype=torch.int32) * 4
        tup = torch.stack([-(i + 1), i + 1, i + 2, i + 3], 1)
    elif kind == 9:
        th = 2.0 * np.pi * u(n)
        e1 = base + torch.stack([L * (0.9 + 0.2 * u(n)), torch.zeros_like(h), torch.zeros_like(h)], 1)
        p = base + torch.stack([L * (0.2 + 0.6 * u(n)) * 0.9, h * torch.cos(th), h * torch.sin(th)], 1)
        x = torch.stack([p, base, e1], 1).reshape(-1, 3)
        i = torch.arange(n, device=dev, dtype=torch.int32) * 3
        tup = torch.stack([-(i + 1), i + 1, i + 2, torch.full_like(i, -1)], 1)
    else:
        dirs = torch.randn(n, 3, generator=g, device=dev, dtype=torch.float64)
        dirs = dirs / dirs.norm(dim=1, keepdim=True)
        x = torch.stack([base + h[:, None] * dirs, base], 1).reshape(-1, 3)
        i = torch.arange(n, device=dev, dtype=torch.int32) * 2
        tup = torch.stack([-(i + 1), i + 1, torch.full_like(i, -1), torch.full_like(i, -1)], 1)
    return x.contiguous(), tup.contiguous()


def table1_compare(gp, counts=(10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7)):
    """Table 1 on this GPU: time to construct and PSD-project n barrier
    Hessians of one size (12 x 12 point-triangle, 9 x 9 point-edge, 6 x 6
    point-point), by the analytic eigensystems against the traditional route
    (the exact Hessian, Eq. 15 with the second derivative of J, projected by
    cyclic Jacobi rotations) and the Gauss-Newton matrix projected in x-space."""
    import torch
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    dhat = 1e-3
    prm = gp.params(dhat=dhat, kappa=1e4)
    rows = []
    for dim in (12, 9, 6):
        for n in counts:
            x, tup = _table1_tuples(dim, n, dhat, 1000 + dim, dev)
            ctx = gp.Context()
            info = gp.pairs_build(ctx, x, tup, prm)
            assert int(info["n_staged"]) == n, (dim, n, info["n_staged"])
            hess = torch.empty((n, 12, 12), dtype=torch.float64, device=dev)
            reps = 5 if n <= 10 ** 6 else 3
            t = {name: _median_ms(lambda: gp.proxy_dense(ctx, x, prm, m, hess=hess), reps, stream)
                 for name, m in (("analytic", gp.PROJ_ANALYTIC), ("exact_jacobi", gp.PROJ_EXACT),
                                 ("gauss_newton_jacobi", gp.PROJ_NUMERIC))}
            rows.append({"dims": dim, "count": n, **{f"{k}_ms": v for k, v in t.items()},
                         "speedup_vs_exact": t["exact_jacobi"] / t["analytic"]})
            ctx.close()
            del x, tup, hess
            torch.cuda.empty_cache()
    print(f"[bench] table1 done", file=sys.stderr, flush=True)
    return {"rows": rows,
            "paper_table1": "RTX 4090 FP64, GPU analytic: 10^7 12x12 90.1 ms, 9x9 41.0 ms, 6x6 13.2 ms; CPU "
                            "(i9 12900K) Eigen numeric 2.42e3 / 1.45e3 / 4.79e2 ms vs analytic 4.95e2 / 2.29e2 / "
                            "96.8 ms"}


def accd_compare(gp, ctx, x, tup, d, stream):
    """The line search's step bound (additive CCD) over every candidate of
    the scene along the step's PCG direction d."""
    P = int(tup.shape[0])
    toi, info = gp.accd(ctx, x, d, tup, s=0.1, tc=1.0)
    t = _median_ms(lambda: gp.accd(ctx, x, d, tup, s=0.1, tc=1.0, toi=toi), 5, stream)
    return {"tuples": P, "ms": t, "tuples_per_s": P / (t * 1e-3), "step": info["step"],
            "max_trial_steps": info["max_steps"], "capped": info["n_capped"], "touching": info["n_touching"],
            "direction": "the PCG solution of the step (Newton direction), tc = 1, s = 0.1"}


def friction_compare(gp, ctx, x, xr, prm, diag, info, stream):
    """Lagged friction on the same staged pairs: lag at x, then energy,
    gradient and Hessian blocks added to the FP64 matrix at a moved x, next
    to the barrier's own eval (mu 0.2, eps_v 1e-3, dt 1e-2)."""
    import torch
    A = gp.BsrMatrix(ctx, dtype=gp.F64)
    gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
    g = torch.Generator(device=x.device).manual_seed(7)
    x1 = x + 1e-5 * torch.randn(x.shape, dtype=x.dtype, device=x.device, generator=g)
    t_lag = _median_ms(lambda: gp.friction_lag(ctx, x, prm, 0.2, 1e-3, 1e-2, x_rest=xr), 5, stream)
    t_eval = _median_ms(lambda: gp.friction_eval(ctx, x1, prm), 5, stream)
    t_asm = _median_ms(lambda: gp.friction_eval(ctx, x1, prm, A), 5, stream)
    t_bar = _median_ms(lambda: gp.barrier_eval(ctx, x, prm, x_rest=xr), 5, stream)
    t_bar_asm = _median_ms(lambda: gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr), 5, stream)
    del A
    return {"pairs": int(info["n_staged"]), "lag_ms": t_lag, "eval_ms": t_eval, "eval_add_blocks_ms": t_asm,
            "barrier_eval_ms": t_bar, "barrier_eval_assemble_ms": t_bar_asm}


def candidates_compare(gp, ctx, s, x, stream):
    """Contact candidates of the scene's surfaces on the GPU (count + emit in
    one call, capacity known), next to the host grid generator that made the
    bench's input list (same set; its time on the host's threads)."""
    import torch
    import scenes
    dev = x.device
    vobj = torch.tensor(s.vobj, dtype=torch.int32, device=dev)
    tris = torch.tensor(s.tris, dtype=torch.int32, device=dev)
    edges = torch.tensor(s.edges, dtype=torch.int32, device=dev)
    out = gp.candidates(ctx, x, vobj, tris, edges, s.dhat)
    n = int(out.shape[0])
    mesh = gp.Context._mesh(x, None)
    topo = gp.Topology(vobj.data_ptr(), tris.data_ptr(), int(tris.shape[0]), edges.data_ptr(), int(edges.shape[0]))
    cnt = ctypes.c_int64()

    def run():
        gp.lib().gipc_candidates(ctx.h, ctypes.byref(mesh), ctypes.byref(topo),
                                 float(s.dhat), ctypes.c_void_p(out.data_ptr()), n,
                                 ctypes.byref(cnt), gp._stream(None))
    t_gpu = _median_ms(run, 3, stream)
    t0 = time.perf_counter()
    host = scenes.broadphase(s.x, s.vobj, s.tris, s.edges, s.dhat)
    t_host = (time.perf_counter() - t0) * 1e3
    del out
    return {"candidates": n, "same_count_as_host": int(len(host)) == n, "gpu_ms": t_gpu,
            "gpu_candidates_per_s": n / (t_gpu * 1e-3), "host_grid_ms": t_host, "host_threads": os.cpu_count(),
            "triangles": int(s.tris.shape[0]), "edges": int(s.edges.shape[0])}


def _median_ms(fn, reps, stream):
    import torch
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _batch_scene_gpu(gp, dev):
    """The 64-scene batch with each scene's candidates found on the GPU at
    its own dhat (the host generator's set), concatenated with offsets."""
    import torch
    import scenes
    rng_scenes = []
    for s in range(64):
        rng = np.random.default_rng(1000 + s)
        r = int(rng.integers(32, 257))
        dhat = float(10.0 ** rng.uniform(-4.0, -2.0))
        rng_scenes.append(scenes.two_sheets(n=r, dhat=dhat, kappa=1e4, seed=1000 + s, with_pairs=False))
    b = scenes.concat_scenes(rng_scenes, name="batch_two_sheets_64")
    xs = torch.tensor(b.x, device=dev)
    tups, pair_off = [], [0]
    for s, sc in enumerate(b.scenes):
        v0, v1 = int(b.vert_off[s]), int(b.vert_off[s + 1])
        t = gpu_candidates(gp, xs[v0:v1], sc)
        sc.tuples = t.cpu().numpy()
        tups.append(torch.tensor(scenes.offset_tuples(sc.tuples, v0), device=dev))
        pair_off.append(pair_off[-1] + sc.tuples.shape[0])
    b.tuples = np.zeros((0, 4), np.int32)
    b.pair_off = np.array(pair_off, np.int64)
    return b, xs, torch.cat(tups)


def batch_leg(gp, steps, warmup, compare=True):
    """The batching target: batched build + eval/assembly replayed from a HIP
    graph (FP32 blocks) against the plain per-scene FP64 path."""
    import torch
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    b, x, tup = _batch_scene_gpu(gp, dev)
    P = int(tup.shape[0])
    print(f"[bench] batch64: S={b.S} V={b.V} candidates={P} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    xr = torch.tensor(b.x_rest, device=dev)
    diag = torch.full((b.V,), 10.0, dtype=torch.float64, device=dev)
    bt = gp.Batch(b.vert_off, b.dhat, b.kappa)
    prm = gp.params(batch=bt)
    ctx = gp.Context()
    info = gp.pairs_build(ctx, x, tup, prm, x_rest=xr)
    A32 = gp.BsrMatrix(ctx, dtype=gp.F32)
    tune = gp.autotune(ctx, x, prm, A32, diag=diag, x_rest=xr, reps=3)
    graph = gp.Graph(ctx, x, prm, A32, diag=diag, x_rest=xr)

    # a rebuild invalidates a graph: each step times the build, captures the
    # graph again outside the timed events, then times its replay
    for _ in range(warmup):
        gp.pairs_build(ctx, x, tup, prm, x_rest=xr)
        graph.close()
        graph = gp.Graph(ctx, x, prm, A32, diag=diag, x_rest=xr)
        graph.launch()
    torch.cuda.synchronize()
    build_ms, replay_ms = [], []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        gp.pairs_build(ctx, x, tup, prm, x_rest=xr)
        e[1].record(stream)
        torch.cuda.synchronize()
        build_ms.append(e[0].elapsed_time(e[1]))
        graph.close()
        graph = gp.Graph(ctx, x, prm, A32, diag=diag, x_rest=xr)
        replay_ms.append(_median_ms(graph.launch, 3, stream))
    build = float(np.median(build_ms))
    replay = float(np.median(replay_ms))
    path_ms = build + replay
    nnzb = A32.nnzb
    V = b.V
    n_active = int(info["n_active"])
    # algorithmic bytes of the numeric eval + assembly with a cached pattern:
    # staged pairs 16 B, positions and rest positions, gradient, BSR (FP32
    # values + column), row pointers, diagonal term, per-scene energies
    num_bytes = 16 * info["n_staged"] + 48 * V + 24 * V + nnzb * (36 + 4) + 4 * (V + 1) + 8 * V + 8 * b.S
    num_gbs = num_bytes / (replay * 1e-3) / 1e9
    # the whole step from a fresh candidate list: candidates 16 B read once
    # on top of the numeric bytes
    path_bytes = num_bytes + 16 * P
    path_gbs = path_bytes / (path_ms * 1e-3) / 1e9

    common = {
        "workload": "64 two-sheet scenes, 32..256 vertices per side, dhat log-uniform in [1e-4, 1e-2], "
                    "kappa=1e4, seeds 1000+s, AABB candidates within each scene's dhat (found on the GPU)",
        "scenes": b.S, "vertices": V, "candidates": P, "active_pairs": n_active,
        "staged_pairs": int(info["n_staged"]), "active_by_type": info["n_by_type"], "nnzb": int(nnzb),
        "tune": tune,
        "active_pairs_per_s": n_active / (path_ms * 1e-3),
        "ms_per_step": path_ms,
        "graph_step_gbs": num_gbs, "graph_step_hbm_frac": num_gbs / HBM_PEAK_GBS,
        "graph_step_bytes": int(num_bytes),
        "path_gbs": path_gbs, "path_hbm_frac": path_gbs / HBM_PEAK_GBS,
    }
    if not compare:
        graph.close()
        ctx.close()
        common["breakdown_ms"] = {"stage_build": build, "eval_assemble_graph_f32": replay}
        return common

    # the same pairs, FP64 blocks, eager eval_assemble (no graph) and the
    # unfused barrier_eval + assemble_bsr
    A64 = gp.BsrMatrix(ctx, dtype=gp.F64)
    fused64 = _median_ms(lambda: gp.eval_assemble(ctx, x, prm, A64, diag=diag, x_rest=xr), 3, stream)
    unfused64 = _median_ms(lambda: (gp.barrier_eval(ctx, x, prm, x_rest=xr), gp.assemble_bsr(ctx, A64, diag=diag)),
                           3, stream)
    graph.close()
    del A64
    ctx.close()

    # one context per scene, built and evaluated one after the other (FP64)
    per_ms = []
    ctxs = []
    for s, sc in enumerate(b.scenes):
        v0, v1 = int(b.vert_off[s]), int(b.vert_off[s + 1])
        c = gp.Context()
        ps = gp.params(dhat=sc.dhat, kappa=sc.kappa)
        ctxs.append((c, ps, x[v0:v1], xr[v0:v1], torch.tensor(sc.tuples, device=dev), diag[v0:v1]))
    for rep in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for c, ps, xs, xrs, ts, ds in ctxs:
            gp.pairs_build(c, xs, ts, ps, x_rest=xrs)
            As = gp.BsrMatrix(c)
            gp.eval_assemble(c, xs, ps, As, diag=ds, x_rest=xrs)
        e1.record(stream)
        torch.cuda.synchronize()
        per_ms.append(e0.elapsed_time(e1))
    # the plain path: one context per scene, every tuple its own staged pair
    # (no merging of duplicate constraints), evaluation and assembly as two
    # calls, FP64 blocks
    plain_ms = []
    flags_plain = gp.FLAGS_DEFAULT | gp.FLAG_NO_MERGE
    for rep in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for (c, ps, xs, xrs, ts, ds), sc in zip(ctxs, b.scenes):
            pp = gp.params(dhat=sc.dhat, kappa=sc.kappa, flags=flags_plain)
            gp.pairs_build(c, xs, ts, pp, x_rest=xrs)
            As = gp.BsrMatrix(c)
            gp.barrier_eval(c, xs, pp, x_rest=xrs)
            gp.assemble_bsr(c, As, diag=ds)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms.append(e0.elapsed_time(e1))
    for c, *_ in ctxs:
        c.close()
    per_scene = float(np.median(per_ms))
    plain = float(np.median(plain_ms))
    return {
        **common,
        "breakdown_ms": {"stage_build": build, "eval_assemble_graph_f32": replay,
                         "eval_assemble_eager_f64": fused64, "eval_then_assemble_f64": unfused64,
                         "per_scene_contexts_build_eval_assemble_f64": per_scene,
                         "plain_per_scene_unmerged_unfused_f64": plain},
        "speedup_vs_per_scene_contexts": per_scene / path_ms,
        "speedup_vs_plain": plain / path_ms,
        "target_speedup_vs_plain": 3.0,
        "target_hbm_frac": 0.60,
    }


def single_run(gp, args, workload, steps, warmup, cands_on_gpu):
    """One single-scene workload: timed steps of build + eval/assembly + SpMV
    + PCG; returns the result dict and what the comparison legs need."""
    import torch
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    s, desc = make_scene(workload, with_pairs=not cands_on_gpu)
    x = torch.tensor(s.x, device=dev)
    tup = gpu_candidates(gp, x, s) if cands_on_gpu else torch.tensor(s.tuples, device=dev)
    P = int(tup.shape[0])
    print(f"[bench] scene {workload}: V={s.V} candidates={P} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    xr = torch.tensor(s.x_rest, device=dev)
    diag = torch.tensor(s.diag, device=dev)
    ctx = gp.Context()
    stream = torch.cuda.current_stream()
    mixed = workload == "sheets40"
    dt = gp.F32 if mixed else gp.F64
    rtol, maxit = (1e-6, 20000) if mixed else (0.0, args.pcg_iters)

    def step(rec):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ev[0].record(stream)
        info = gp.pairs_build(ctx, x, tup, prm, x_rest=xr)
        ev[1].record(stream)
        A = gp.BsrMatrix(ctx, dtype=dt)
        E, g = gp.eval_assemble(ctx, x, prm, A, diag=diag, x_rest=xr)
        gv = g.float() if mixed else g
        ev[2].record(stream)
        y = gp.bsr_spmv(A, gv)
        ev[3].record(stream)
        b = -g
        ev[4].record(stream)
        d, it, rr, st = gp.pcg(ctx, A, b, rtol=rtol, maxit=maxit)
        ev[5].record(stream)
        if rec is not None:
            rec.append((ev, info, it, A.nnzb, rr))
        return E, y, A, d, b

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        last = step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] {workload}: {steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    build_ms = np.array([r[0][0].elapsed_time(r[0][1]) for r in recs])
    evas_ms = np.array([r[0][1].elapsed_time(r[0][2]) for r in recs])
    spmv_ms = np.array([r[0][2].elapsed_time(r[0][3]) for r in recs])
    pcg_ms = np.array([r[0][4].elapsed_time(r[0][5]) for r in recs])
    step_ms = np.array([r[0][0].elapsed_time(r[0][5]) for r in recs])
    info, iters, nnzb = recs[-1][1], recs[-1][2], recs[-1][3]
    V = s.V
    path_ms = float(np.median(build_ms + evas_ms))
    n_active = int(info["n_active"])
    # algorithmic bytes of one BSR SpMV: blocks (9 values + 4 B column), row
    # pointers, x read once, y written once
    sv = 4 if mixed else 8
    spmv_bytes = nnzb * (9 * sv + 4) + 4 * (V + 1) + 3 * sv * V + 3 * sv * V
    spmv_gbs = spmv_bytes / (np.mean(spmv_ms) * 1e-3) / 1e9
    # one PCG iteration: the product, plus the vector passes (x, r, z, p, q
    # read or written, 13 passes of 3V FP64) and the inverse diagonal blocks
    pcg_iter_ms = float(np.median(pcg_ms) / max(iters, 1))
    pcg_iter_bytes = spmv_bytes + 13 * 24 * V + 72 * V
    # algorithmic bytes of stage + build + eval/assembly (metric scope):
    # candidates 16 B, positions + rest read once, gradient written, BSR
    # written, diagonal term
    path_bytes = 16 * P + 48 * V + 24 * V + nnzb * (9 * sv + 4) + 4 * (V + 1) + 8 * V
    out = {
        "metric": "contact pairs/s (energy+grad+proxy Hessian+BSR assembly); BSR SpMV GB/s vs roofline",
        "value": float(n_active / (path_ms * 1e-3)),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry, f32 blocks and SpMV" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "vertices": V,
            "candidates": P,
            "contact_pairs": n_active,
            "active_by_type": info["n_by_type"],
            "staged_pairs": int(info["n_staged"]),
            "nnzb": int(nnzb),
            "pcg_iters": int(iters),
            "pcg_rtol": rtol,
        },
        "value_counts": "contact pairs = candidates closer than dhat after classification (one term of the "
                        "barrier sum each); candidates and staged pairs (after merging duplicate point-edge / "
                        "point-point constraints) are reported as rates beside it",
        "candidates_per_s": float(P / (path_ms * 1e-3)),
        "staged_pairs_per_s": float(info["n_staged"] / (path_ms * 1e-3)),
        "breakdown_ms": {
            "stage_build": float(np.median(build_ms)),
            "eval_assemble": float(np.median(evas_ms)),
            "spmv": float(np.median(spmv_ms)),
            "pcg": float(np.median(pcg_ms)),
            "pcg_per_iter": pcg_iter_ms,
        },
        "path_gbs": float(path_bytes / (path_ms * 1e-3) / 1e9),
        "path_hbm_frac": float(path_bytes / (path_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
        "spmv_gbs": float(spmv_gbs),
        "pcg_iter_gbs": float(pcg_iter_bytes / (pcg_iter_ms * 1e-3) / 1e9),
        "pcg_iter_vs_spmv": float(pcg_iter_ms / np.mean(spmv_ms)),
    }
    traffic, tsrc = (None, None) if mixed else _traffic_if_current()
    out["roofline"] = {
        "kernel": "k_spmv<float> (FP32 BSR SpMV by rows)" if mixed
        else "k_spmv_ent (FP64 BSR SpMV, one lane per block)",
        "bound": "hbm",
        "achieved": float(spmv_gbs),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": float(spmv_gbs / HBM_PEAK_GBS),
        "traffic": traffic,
        "traffic_source": tsrc,
        "bytes_per_launch": int(spmv_bytes),
    }
    return out, (ctx, s, x, xr, prm, diag, info, rtol, maxit, stream, last, tup)


def bandwidth_reference(gp, stream):
    """Achievable HBM bandwidth with the library's own streaming kernels on a
    2 GiB buffer: a copy (read + write) and a plain read."""
    import torch
    dev = torch.device("cuda", 0)
    nbytes = 2 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {}
    for name, fn, moved in (("copy_gbs", lambda: gp.copy(src, dst), 2 * nbytes),
                            ("read_gbs", lambda: gp.read(src, sink=sink), nbytes)):
        fn()
        ce = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        for i in range(5):
            ce[i].record(stream)
            fn()
        ce[5].record(stream)
        torch.cuda.synchronize()
        ms = np.median([ce[i].elapsed_time(ce[i + 1]) for i in range(5)])
        out[name] = float(moved / (ms * 1e-3) / 1e9)
    del src, dst
    return out


def sheets40_leg(gp, args):
    """The precision target: FP32 blocks and SpMV on forty sheets, PCG to 1e-6,
    against the HBM roofline; the FP64 path once for the comparison."""
    out, (ctx, s, x, xr, prm, diag, info, rtol, maxit, stream, last, _) = single_run(gp, args, "sheets40", 2, 1,
                                                                                     True)
    leg = {k: out[k] for k in ("config", "breakdown_ms", "spmv_gbs", "pcg_iter_gbs", "pcg_iter_vs_spmv", "roofline")}
    leg["value_contact_pairs_per_s"] = out["value"]
    leg["spmv_hbm_frac"] = out["spmv_gbs"] / HBM_PEAK_GBS
    leg["pcg_iter_hbm_frac"] = out["pcg_iter_gbs"] / HBM_PEAK_GBS
    leg["precision"] = precision_compare(gp, ctx, x, xr, prm, diag, last, stream)
    ctx.close()
    return leg


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (sharding is described, "
                                   "not implemented)"}))
        sys.exit(2)
    import torch
    import paper_2308_09400_amd as gp

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "batch64":
        leg = batch_leg(gp, args.steps, args.warmup, compare=not args.no_compare)
        line = {"metric": "contact pairs/s (energy+grad+proxy Hessian+BSR assembly), batched scenes",
                "value": leg["active_pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f64 geometry, f32 blocks", "data": "synthetic",
                "config": {"workload": leg["workload"]}, "batch64": leg}
        print(json.dumps(line))
        return
    workload = args.workload
    out, (ctx, s, x, xr, prm, diag, info, rtol, maxit, stream, last, tup) = single_run(
        gp, args, workload, args.steps, args.warmup, workload == "sheets40")
    bw = bandwidth_reference(gp, stream)
    out["bandwidth_reference"] = bw
    out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / bw["copy_gbs"]
    out["roofline"]["frac_of_read"] = out["roofline"]["achieved"] / bw["read_gbs"]
    if workload == "sheets40":
        out["precision"] = precision_compare(gp, ctx, x, xr, prm, diag, last, stream)
    if not args.no_extras:
        out["matrix_free"] = matrix_free_compare(gp, ctx, x, xr, prm, diag, info, rtol, maxit, stream)
        if workload == "sheets10":
            out["numeric_eigen_baseline"] = numeric_compare(gp, ctx, x, xr, prm, info, stream)
            out["dense_local_hessians_table2"] = dense_compare(gp, ctx, x, xr, prm, diag, info, stream)
            out["accd"] = accd_compare(gp, ctx, x, tup, last[3], stream)
            out["friction"] = friction_compare(gp, ctx, x, xr, prm, diag, info, stream)
            out["candidates"] = candidates_compare(gp, ctx, s, x, stream)
            print(f"[bench] extras done", file=sys.stderr, flush=True)
    ctx.close()
    del x, xr, diag
    if workload == "sheets10" and not args.no_extras:
        torch.cuda.empty_cache()
        out["table1"] = table1_compare(gp)
    if workload == "sheets10" and not args.no_targets:
        torch.cuda.empty_cache()
        out["targets"] = {"batch64": batch_leg(gp, 3, 1)}
        torch.cuda.empty_cache()
        out["targets"]["sheets40"] = sheets40_leg(gp, args)
        torch.cuda.empty_cache()
    if not args.no_cpu and workload == "sheets10":
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_sample)
        out["cpu_baseline_1thread"] = cpu_baseline(s, max(args.cpu_sample // 20, 1000), nthreads=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
