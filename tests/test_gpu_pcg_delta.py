"""gipc_pcg_delta: block-Jacobi PCG stopped by the paper's termination
(r.z <= eps r0.z0, its PCG in the implementation section), on the two-sheet
scene's assembled matrix:

* FP64 and FP32 blocks: status OK; r.z recomputed with numpy from the
  returned solution (and the matrix read back from the device) meets the
  test, and the solution of a run one iteration shorter does not;
* the iteration count is the oracle's (orc_pcg_delta on the oracle's
  assembly) within one (the ratio may sit at the threshold up to rounding),
  and equal counts give solutions within 1e-8 of the oracle's;
* maxit reached first: WARN_NOT_CONVERGED after maxit iterations; eps < 0:
  INVALID_ARG.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
scipy_sparse = pytest.importorskip("scipy.sparse")

import oracle  # noqa: E402
import scenes  # noqa: E402


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _delta(G, b, x):
    """r.z at x with z = (3x3 block diagonal of G)^-1 r (numpy, FP64)"""
    r = b - G @ x
    V = r.shape[0] // 3
    D = G.tobsr(blocksize=(3, 3))
    z = np.zeros_like(r)
    for v in range(V):
        blk = None
        for k in range(D.indptr[v], D.indptr[v + 1]):
            if D.indices[k] == v:
                blk = D.data[k]
        z[3 * v:3 * v + 3] = np.linalg.solve(blk, r[3 * v:3 * v + 3])
    return float(r @ z)


def test_pcg_delta(gp):
    dev = torch.device("cuda", 0)
    s = scenes.two_sheets(n=16, seed=1)
    diag_np = np.linspace(1.0, 2.0, s.V)
    x = torch.tensor(s.x, device=dev)
    xr = torch.tensor(s.x_rest, device=dev)
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    ctx = gp.Context()
    gp.pairs_build(ctx, x, torch.tensor(s.tuples, device=dev), prm, x_rest=xr)
    ref = oracle.eval_scene(s.x, s.tuples, oracle.params(dhat=s.dhat, kappa=s.kappa), x_rest=s.x_rest, per_pair=True)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, ref["pairH"], diag_np)
    bo = -ref["grad"].reshape(-1)
    for dtype in (gp.F64, gp.F32):
        # FP32 products make the recursive residual drift from b - A x
        tol = 1e-6 if dtype == gp.F64 else 2e-2
        A = gp.BsrMatrix(ctx, dtype=dtype)
        _, g = gp.eval_assemble(ctx, x, prm, A, diag=torch.tensor(diag_np, device=dev), x_rest=xr)
        b = -g
        G = A.to_scipy().tocsr().astype(np.float64)
        bn = b.cpu().numpy().reshape(-1)
        d0 = _delta(G, bn, np.zeros_like(bn))
        for eps in (1e-2, 1e-4):
            xs, it, rr, st = gp.pcg(ctx, A, b, rtol=eps, maxit=500, stop="delta")
            assert st == gp.OK and 0 < it < 500, (dtype, eps, st, it)
            xn = xs.cpu().numpy().reshape(-1)
            assert _delta(G, bn, xn) <= eps * d0 * (1 + tol), (dtype, eps)
            assert rr == pytest.approx(np.linalg.norm(bn - G @ xn) / np.linalg.norm(bn), rel=tol)
            xm, itm, _, stm = gp.pcg(ctx, A, b, rtol=eps, maxit=it - 1, stop="delta")
            assert itm == it - 1 and stm == gp.WARN_NOT_CONVERGED
            assert _delta(G, bn, xm.cpu().numpy().reshape(-1)) > eps * d0 * (1 - tol), (dtype, eps)
            if dtype == gp.F64:
                xo, ito, _ = oracle.pcg(s.V, rows, cols, vals, bo, rtol=eps, maxit=500, delta=True)
                assert abs(ito - it) <= 1, (eps, it, ito)
                if ito == it:
                    assert np.abs(xn - xo).max() <= 1e-8 * np.abs(xo).max()
    A = gp.BsrMatrix(ctx, dtype=gp.F64)
    _, g = gp.eval_assemble(ctx, x, prm, A, diag=torch.tensor(diag_np, device=dev), x_rest=xr)
    xs, it, rr, st = gp.pcg(ctx, A, -g, rtol=1e-14, maxit=3, stop="delta")
    assert it == 3 and st == gp.WARN_NOT_CONVERGED
    with pytest.raises(gp.GipcError) as e:
        gp.pcg(ctx, A, -g, rtol=-1.0, maxit=3, stop="delta")
    assert e.value.status == gp.ERR_INVALID_ARG
    ctx.close()
