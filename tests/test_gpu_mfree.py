"""The matrix-free operator (gipc_mf_apply) and the PCG on it (gipc_pcg_mf).

* against the oracle's sum of dense local products (no global matrix) on the
  same seeded scenes: within 1e-9 of the largest entry of y (the factors
  themselves are within 1e-9 of the oracle's local Hessians);
* against gipc_bsr_spmv on the FP64 matrix of the same eval: within 1e-12
  of the largest entry (same products, summed in another order);
* at the 10-sheet, 256 x 256 size: 40 sampled rows against the oracle's
  local products over the pairs that touch them;
* a batch of scenes, the empty pair list, no diagonal term, determinism and
  the argument / state errors;
* PCG: a fixed number of iterations follows the oracle's PCG on the
  assembled matrix to 1e-8; to a tolerance it converges in the same number
  of iterations as gipc_pcg to within one.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402

TOL = 1e-9


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _prm(gp, s):
    return gp.params(dhat=s.dhat, kappa=s.kappa), oracle.params(dhat=s.dhat, kappa=s.kappa)


def _setup(gp, s, diag, dtype=0):
    dev = torch.device("cuda", 0)
    pg, po = _prm(gp, s)
    X = torch.tensor(s.x, device=dev)
    XR = torch.tensor(s.x_rest, device=dev)
    T = torch.tensor(np.asarray(s.tuples, np.int32).reshape(-1, 4), device=dev)
    D = torch.tensor(diag, device=dev) if diag is not None else None
    ctx = gp.Context()
    gp.pairs_build(ctx, X, T, pg, x_rest=XR)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    E, g = gp.eval_assemble(ctx, X, pg, A, diag=D, x_rest=XR)
    return dict(ctx=ctx, A=A, D=D, g=g, pg=pg, po=po, X=X, XR=XR)


@pytest.mark.parametrize("which", ["tiny", "sheets16"])
@pytest.mark.parametrize("with_diag", [True, False])
def test_apply_matches_oracle_and_bsr(gp, which, with_diag):
    if which == "tiny":
        s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    else:
        s = scenes.two_sheets(n=16, seed=1)
    diag = np.linspace(1.0, 3.0, s.V) if with_diag else None
    r = _setup(gp, s, diag)
    ref = oracle.eval_scene(s.x, s.tuples, r["po"], x_rest=s.x_rest, per_pair=True)
    rng = np.random.default_rng(7)
    for _ in range(2):
        xv = rng.normal(size=(s.V, 3))
        xt = torch.tensor(xv, device="cuda")
        y = gp.mf_apply(r["ctx"], xt, diag=r["D"]).cpu().numpy().reshape(-1)
        yo = oracle.matfree(s.V, s.tuples, ref["pairH"], xv, diag)
        assert np.abs(y - yo).max() <= TOL * np.abs(yo).max()
        yb = gp.bsr_spmv(r["A"], xt).cpu().numpy().reshape(-1)
        assert np.abs(y - yb).max() <= 1e-12 * np.abs(yb).max()
    r["ctx"].close()


def test_apply_on_a_batch(gp):
    b = scenes.batch_two_sheets(S=5, r_lo=6, r_hi=20, dhat_lo=1e-3, dhat_hi=2e-1, seed_base=700)
    dev = torch.device("cuda", 0)
    X = torch.tensor(b.x, device=dev)
    XR = torch.tensor(b.x_rest, device=dev)
    T = torch.tensor(b.tuples, device=dev)
    prm = gp.params(batch=gp.Batch(b.vert_off, b.dhat, b.kappa))
    ctx = gp.Context()
    gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx)
    diag = torch.full((b.V,), 10.0, dtype=torch.float64, device=dev)
    gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
    xt = torch.tensor(np.random.default_rng(2).normal(size=(b.V, 3)), device=dev)
    y = gp.mf_apply(ctx, xt, diag=diag).cpu().numpy()
    yb = gp.bsr_spmv(A, xt).cpu().numpy()
    assert np.abs(y - yb).max() <= 1e-12 * np.abs(yb).max()
    # scene 0 (vertices from 0) against the oracle on its own
    v0, v1 = int(b.vert_off[0]), int(b.vert_off[1])
    assert v0 == 0
    kind, st = scenes.decode_tuples(b.tuples)
    sel = (st < v1).all(1)
    po = oracle.params(dhat=float(b.dhat[0]), kappa=float(b.kappa[0]))
    ref = oracle.eval_scene(b.x[v0:v1], b.tuples[sel], po, x_rest=b.x_rest[v0:v1], per_pair=True)
    yo = oracle.matfree(v1 - v0, b.tuples[sel], ref["pairH"], xt[v0:v1].cpu().numpy(), np.full(v1 - v0, 10.0))
    assert np.abs(y[v0:v1].reshape(-1) - yo).max() <= TOL * np.abs(yo).max()
    ctx.close()


def test_empty_list_deterministic_and_errors(gp):
    s = scenes.two_sheets(n=16, seed=1)
    diag = np.full(s.V, 4.0)
    r = _setup(gp, s, diag)
    xt = torch.tensor(np.random.default_rng(3).normal(size=(s.V, 3)), device="cuda")
    y1 = gp.mf_apply(r["ctx"], xt, diag=r["D"])
    y2 = gp.mf_apply(r["ctx"], xt, diag=r["D"])
    assert torch.equal(y1, y2)
    with pytest.raises(gp.GipcError) as ei:  # x and y alias
        gp.mf_apply(r["ctx"], xt, y=xt)
    assert ei.value.status == gp.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        gp.mf_apply(r["ctx"], xt[:-1].contiguous())
    r["ctx"].close()
    # build without eval: state error
    pg, _ = _prm(gp, s)
    ctx = gp.Context()
    gp.pairs_build(ctx, r["X"], torch.tensor(s.tuples, device="cuda"), pg, x_rest=r["XR"])
    with pytest.raises(gp.GipcError) as ei:
        gp.mf_apply(ctx, xt)
    assert ei.value.status == gp.ERR_STATE
    ctx.close()
    # an empty pair list leaves the diagonal term only
    ctx = gp.Context()
    empty = torch.zeros((0, 4), dtype=torch.int32, device="cuda")
    gp.pairs_build(ctx, r["X"], empty, pg, x_rest=r["XR"])
    gp.barrier_eval(ctx, r["X"], pg, x_rest=r["XR"])
    y = gp.mf_apply(ctx, xt, diag=r["D"])
    assert torch.equal(y, 4.0 * xt)
    assert torch.equal(gp.mf_apply(ctx, xt), torch.zeros_like(xt))
    ctx.close()


def test_full_scale_sampled_rows(gp):
    s = scenes.stacked_sheets(n_sheets=10, n=256, seed=2)
    r = _setup(gp, s, s.diag)
    xv = np.random.default_rng(11).normal(size=(s.V, 3))
    xt = torch.tensor(xv, device="cuda")
    y = gp.mf_apply(r["ctx"], xt, diag=r["D"]).cpu().numpy()
    yb = gp.bsr_spmv(r["A"], xt).cpu().numpy()
    assert np.abs(y - yb).max() <= 1e-12 * np.abs(yb).max()
    rows = np.random.default_rng(5).choice(s.V, 40, replace=False)
    kind, st = scenes.decode_tuples(s.tuples)
    sub = s.tuples[np.isin(st, rows).any(1)]
    ref = oracle.eval_scene(s.x, sub, r["po"], x_rest=s.x_rest, per_pair=True)
    yo = oracle.matfree(s.V, sub, ref["pairH"], xv, s.diag).reshape(-1, 3)
    scale = np.abs(yo[rows]).max()
    assert np.abs(y[rows] - yo[rows]).max() <= TOL * scale
    r["ctx"].close()


def test_pcg_mf_matches_oracle_and_bsr_pcg(gp):
    s = scenes.two_sheets(n=16, seed=1)
    diag = np.full(s.V, 10.0)
    r = _setup(gp, s, diag)
    ref = oracle.eval_scene(s.x, s.tuples, r["po"], x_rest=s.x_rest, per_pair=True)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, ref["pairH"], diag)
    b = -ref["grad"].reshape(-1)
    bt = -r["g"]
    x10, it, rr, st = gp.pcg_mf(r["ctx"], bt, diag=r["D"], rtol=0.0, maxit=10)
    xo, ito, _ = oracle.pcg(s.V, rows, cols, vals, b, rtol=0.0, maxit=10)
    assert it == ito == 10 and st == gp.OK
    assert np.linalg.norm(x10.cpu().numpy().reshape(-1) - xo) <= 1e-8 * np.linalg.norm(xo)
    xm, itm, rrm, stm = gp.pcg_mf(r["ctx"], bt, diag=r["D"], rtol=1e-6, maxit=500)
    xb, itb, rrb, stb = gp.pcg(r["ctx"], r["A"], bt, rtol=1e-6, maxit=500)
    assert stm == gp.OK and rrm <= 1e-6 and abs(itm - itb) <= 1
    assert torch.linalg.norm(xm - xb) <= 1e-5 * torch.linalg.norm(xb)
    # warm start at the solution: no iteration; a cap: warning status
    _, it0, _, _ = gp.pcg_mf(r["ctx"], bt, x=xm.clone(), diag=r["D"], rtol=1e-3, maxit=10)
    assert it0 == 0
    _, it1, _, st1 = gp.pcg_mf(r["ctx"], bt, diag=r["D"], rtol=1e-14, maxit=3)
    assert it1 == 3 and st1 == gp.WARN_NOT_CONVERGED
    r["ctx"].close()


def test_pcg_mf_reports_breakdown(gp):
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    r = _setup(gp, s, np.full(s.V, -5.0))
    bt = torch.ones(s.V, 3, dtype=torch.float64, device="cuda")
    with pytest.raises(gp.GipcError) as ei:
        gp.pcg_mf(r["ctx"], bt, diag=r["D"], rtol=1e-8, maxit=50)
    assert ei.value.status == gp.ERR_BREAKDOWN
    r["ctx"].close()


def test_apply_follows_the_last_eval(gp):
    # the operator's per-eval vectors are rebuilt after every eval: eager,
    # and replayed from a graph
    s = scenes.two_sheets(n=16, seed=1)
    diag = np.full(s.V, 10.0)
    r = _setup(gp, s, diag)
    ctx, A, D = r["ctx"], r["A"], r["D"]
    xt = torch.tensor(np.random.default_rng(4).normal(size=(s.V, 3)), device="cuda")
    gp.mf_apply(ctx, xt, diag=D)
    x2 = r["X"] + 0.05 * s.dhat * torch.tensor(np.random.default_rng(6).uniform(-1, 1, size=(s.V, 3)), device="cuda")
    gp.eval_assemble(ctx, x2, r["pg"], A, diag=D, x_rest=r["XR"])
    y = gp.mf_apply(ctx, xt, diag=D)
    yb = gp.bsr_spmv(A, xt)
    assert float((y - yb).abs().max()) <= 1e-12 * float(yb.abs().max())
    graph = gp.Graph(ctx, r["X"], r["pg"], A, diag=D, x_rest=r["XR"])
    graph.launch()
    y = gp.mf_apply(ctx, xt, diag=D)
    yb = gp.bsr_spmv(A, xt)
    assert float((y - yb).abs().max()) <= 1e-12 * float(yb.abs().max())
    graph.close()
    ctx.close()
