"""The entry-parallel FP64 BSR product (one lane per block, rows cut by the
pattern's row-start map) against the CPU oracle and the row-by-row product.

* the row-start map (head bits per 64 blocks, first row per 64 blocks) is
  compared exactly with the one derived from row_ptr on the host;
* products: within 1e-12 of the largest entry of the oracle's product, and
  within 1e-13 of the row-by-row product (the two differ only in rounding
  order); two calls agree bit for bit;
* a fan scene (one point over a fine patch, about 1600 blocks in the point's
  row) puts a row across many wavefronts and over a whole workgroup of 512
  blocks (a workgroup with no row start),
  with the long row first, last and in the middle of the pattern;
* the PCG follows the same iterates with either product;
* FP32 blocks ignore the map (both descriptors give the same bits);
* at the ten-sheet size of the benchmark (17.4M blocks, the launch the
  benchmark times), sampled rows are recomputed on the host in FP64.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _map_from_row_ptr(rp):
    nnzb = int(rp[-1])
    W = (nnzb + 63) // 64
    head = np.zeros(W, dtype=np.uint64)
    starts = rp[:-1].astype(np.int64)
    np.bitwise_or.at(head, starts >> 6, np.left_shift(np.uint64(1), (starts & 63).astype(np.uint64)))
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return head.view(np.int64), rows[::64].astype(np.int32)


def _fan_scene(n=30, where="last", dhat=1e-3):
    """One point 0.3 dhat above an n x n patch of side 0.5 dhat: every
    triangle of the patch is within dhat of the point."""
    g = np.linspace(0.0, 0.5 * dhat, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    grid = np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], 1)
    pt = np.array([[0.25 * dhat, 0.25 * dhat, 0.3 * dhat]])
    if where == "first":
        x, P, off = np.vstack([pt, grid]), 0, 1
    elif where == "middle":
        h = (n * n) // 2
        x, P, off = np.vstack([grid[:h], pt, grid[h:]]), h, 0
    else:
        x, P, off = np.vstack([grid, pt]), n * n, 0

    def vid(i, j):
        k = i * n + j
        if where == "middle":
            return k if k < P else k + 1
        return k + off

    tup = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i, j + 1), vid(i + 1, j + 1)
            tup += [[-(P + 1), a, b, c], [-(P + 1), b, d, c]]
    return x, np.asarray(tup, np.int32), dhat


def _build(gp, x, tuples, dhat, kappa=1e4, diag=None, dtype=0):
    dev = torch.device("cuda", 0)
    X = torch.tensor(x, device=dev)
    T = torch.tensor(np.asarray(tuples, np.int32).reshape(-1, 4), device=dev)
    prm = gp.params(dhat=dhat, kappa=kappa)
    ctx = gp.Context()
    gp.pairs_build(ctx, X, T, prm)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    D = torch.tensor(diag, device=dev) if diag is not None else None
    gp.eval_assemble(ctx, X, prm, A, diag=D)
    return ctx, A


def _check_product(gp, A, V, seed=0):
    rp = A.row_ptr().cpu().numpy()
    ci = A.col_idx().cpu().numpy()
    vals = A.val[:, :A.nnzb].cpu().numpy().T.reshape(-1, 3, 3)
    rows = np.repeat(np.arange(V), np.diff(rp))
    xv = np.random.default_rng(seed).normal(size=(V, 3))
    xt = torch.tensor(xv, device="cuda")
    y = gp.bsr_spmv(A, xt)
    y2 = gp.bsr_spmv(A, xt)
    yr = gp.bsr_spmv(A, xt, by_rows=True)
    assert torch.equal(y, y2)
    yo = oracle.spmv(V, rows, ci, vals, xv).reshape(V, 3)
    scale = np.abs(yo).max()
    yc = y.cpu().numpy()
    assert np.abs(yc - yo).max() <= 1e-12 * scale
    assert np.abs(yc - yr.cpu().numpy()).max() <= 1e-13 * scale
    return rp


@pytest.mark.parametrize("n", [4, 16, 40])
def test_map_and_product_two_sheets(gp, n):
    s = scenes.two_sheets(n=n, seed=3)
    ctx, A = _build(gp, s.x, s.tuples, s.dhat, s.kappa, diag=np.full(s.V, 10.0))
    rp = _check_product(gp, A, s.V)
    head, wrow = A.wave_map()
    h_ref, w_ref = _map_from_row_ptr(rp)
    assert np.array_equal(head.cpu().numpy(), h_ref)
    assert np.array_equal(wrow.cpu().numpy(), w_ref)
    ctx.close()


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_long_row_crosses_workgroups(gp, where):
    x, tup, dhat = _fan_scene(40, where)
    V = x.shape[0]
    ctx, A = _build(gp, x, tup, dhat, diag=np.linspace(1.0, 2.0, V))
    rp = _check_product(gp, A, V, seed=1)
    assert np.diff(rp).max() > 2 * 512  # one row over more than two workgroups of blocks
    head, wrow = A.wave_map()
    h_ref, w_ref = _map_from_row_ptr(rp)
    assert np.array_equal(head.cpu().numpy(), h_ref) and np.array_equal(wrow.cpu().numpy(), w_ref)
    ctx.close()


def test_single_row_and_tiny_patterns(gp):
    # one vertex pair: a 2-row pattern far below one wavefront
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 5e-4]])
    ctx, A = _build(gp, x, [[-1, 1, -1, -1]], 1e-3, diag=np.array([1.0, 2.0]))
    assert A.nnzb == 4
    _check_product(gp, A, 2)
    ctx.close()


def test_pcg_same_iterates_either_product(gp):
    s = scenes.two_sheets(n=24, seed=5)
    ctx, A = _build(gp, s.x, s.tuples, s.dhat, s.kappa, diag=np.full(s.V, 10.0))
    b = torch.tensor(np.random.default_rng(2).normal(size=(s.V, 3)), device="cuda")
    x1, it1, rr1, st1 = gp.pcg(ctx, A, b, rtol=0.0, maxit=25)
    x2, it2, rr2, st2 = gp.pcg(ctx, A, b, rtol=0.0, maxit=25, by_rows=True)
    assert it1 == it2 == 25 and st1 == st2 == gp.OK
    assert torch.linalg.norm(x1 - x2) <= 1e-11 * torch.linalg.norm(x2)
    x1, it1, rr1, _ = gp.pcg(ctx, A, b, rtol=1e-8, maxit=500)
    x2, it2, rr2, _ = gp.pcg(ctx, A, b, rtol=1e-8, maxit=500, by_rows=True)
    assert abs(it1 - it2) <= 1 and rr1 <= 1e-8 and rr2 <= 1e-8
    ctx.close()


def test_fp32_blocks_ignore_the_map(gp):
    s = scenes.two_sheets(n=16, seed=7)
    ctx, A = _build(gp, s.x, s.tuples, s.dhat, s.kappa, diag=np.full(s.V, 10.0), dtype=gp.F32)
    xt = torch.tensor(np.random.default_rng(3).normal(size=(s.V, 3)), device="cuda", dtype=torch.float32)
    assert torch.equal(gp.bsr_spmv(A, xt), gp.bsr_spmv(A, xt, by_rows=True))
    ctx.close()


def test_full_size_sampled_rows(gp):
    from bench import make_scene
    s, _ = make_scene("sheets10")
    ctx, A = _build(gp, s.x, s.tuples, s.dhat, s.kappa, diag=np.full(s.V, 10.0))
    xt = torch.tensor(np.random.default_rng(4).normal(size=(s.V, 3)), device="cuda")
    y = gp.bsr_spmv(A, xt)
    yr = gp.bsr_spmv(A, xt, by_rows=True)
    scale = float(y.abs().max())
    assert float((y - yr).abs().max()) <= 1e-13 * scale
    rp = A.row_ptr().cpu().numpy()
    rows = np.sort(np.random.default_rng(5).choice(s.V, 3000, replace=False))
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    it = torch.tensor(idx, device="cuda")
    # the sampled rows' blocks, gathered on the device and multiplied on the host in FP64
    cols = A.col_idx()[it].long()
    blk = A.val[:, it].T.reshape(-1, 3, 3).cpu().numpy()
    xs = xt[cols].cpu().numpy()
    seg = np.repeat(np.arange(len(rows)), np.diff(rp)[rows])
    yo = oracle.spmv(len(rows), seg, np.arange(len(idx)), blk, xs)
    yo = yo.reshape(-1, 3)
    rows = torch.tensor(rows, device="cuda")
    assert np.abs(y[rows].cpu().numpy() - yo).max() <= 1e-12 * scale
    ctx.close()
