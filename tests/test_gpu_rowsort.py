"""The symbolic row sort over all of its paths, against patterns and matrices
built on the host.

A row with n incidences (staged pairs touching the vertex) holds n own-column
contributions (slot j = i) and T = sum over its pairs of (nv - 1) others.
The wavefront sort takes rows with n <= 128: the own-column codes one or two
per lane (n <= 64 or not) and the others 1, 2, 4 or 8 per lane (T <= 64,
128, 256 or more); rows with more incidences go to the workgroup sort.  The
scenes (two sheets with growing dhat, a coarse sheet over fine ones, one
point over a fine patch) put rows in every one of these regimes, which the
test checks from the staged pairs, and for each scene:

* the pattern (row_ptr, col_idx) equals, exactly, the one derived on the host
  from the staged stencils (every pair of stencil vertices, plus the
  diagonal), which fixes the sorted distinct columns of every row;
* the FP64 matrix equals the oracle's assembly within 1e-9 of its largest
  entry, which needs every contribution under its block;
* two builds give the same bits.
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


def _fan(n=40, dhat=1e-3):
    g = np.linspace(0.0, 0.5 * dhat, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.vstack([np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], 1), [[0.25 * dhat, 0.25 * dhat, 0.3 * dhat]]])
    P = n * n
    tup = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = i * n + j, (i + 1) * n + j, i * n + j + 1, (i + 1) * n + j + 1
            tup += [[-(P + 1), a, b, c], [-(P + 1), b, d, c]]
    return x, None, np.asarray(tup, np.int32), dhat, 1e4


def _coarse_over_fine(n_lo, n_up, dhat, seed=0):
    """An n_up x n_up sheet 0.5 dhat over an n_lo x n_lo one: a coarse vertex
    meets the fine points under its triangles and the fine edges its edges
    cross, pairs of four vertices each (three other slots per incidence)."""
    rng = np.random.default_rng(seed)
    t_lo, e_lo = scenes.sheet_topology(n_lo)
    t_up, e_up = scenes.sheet_topology(n_up)
    xl, yl = scenes._sheet_xy(n_lo)
    xu, yu = scenes._sheet_xy(n_up)
    lo = np.stack([xl, yl, np.zeros(n_lo * n_lo)], 1)
    up = np.stack([xu, yu, 0.5 * dhat + rng.uniform(-0.1, 0.1, n_up * n_up) * dhat], 1)
    x = np.vstack([lo, up])
    off = n_lo * n_lo
    tris = np.vstack([t_lo, t_up + off]).astype(np.int32)
    edges = np.vstack([e_lo, e_up + off]).astype(np.int32)
    vobj = np.concatenate([np.zeros(off, np.int32), np.ones(n_up * n_up, np.int32)])
    return x, None, scenes.broadphase(x, vobj, tris, edges, dhat), dhat, 1e4


def _scenes():
    out = []
    for n, dhat, seed in ((12, 0.05, 2), (16, 1e-3, 3), (10, 0.12, 4), (10, 0.15, 5), (10, 0.17, 6), (10, 0.19, 7)):
        s = scenes.two_sheets(n=n, dhat=dhat, seed=seed)
        out.append((f"two_sheets_{n}_{dhat}", s.x, s.x_rest, s.tuples, s.dhat, s.kappa))
    for n_lo, n_up, dhat in ((13, 5, 0.06), (11, 4, 0.06), (15, 5, 0.05)):
        x, xr, t, dh, k = _coarse_over_fine(n_lo, n_up, dhat)
        out.append((f"coarse_{n_up}_over_{n_lo}", x, xr, t, dh, k))
    x, xr, t, dh, k = _fan()
    out.append(("fan_40", x, xr, t, dh, k))
    return out


def _run(gp, x, xr, tuples, dhat, kappa, diag):
    dev = torch.device("cuda", 0)
    X = torch.tensor(x, device=dev)
    XR = torch.tensor(xr, device=dev) if xr is not None else None
    T = torch.tensor(np.asarray(tuples, np.int32).reshape(-1, 4), device=dev)
    prm = gp.params(dhat=dhat, kappa=kappa)
    ctx = gp.Context()
    gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx, dtype=gp.F64)
    gp.eval_assemble(ctx, X, prm, A, diag=torch.tensor(diag, device=dev), x_rest=XR)
    vid = gp.pair_inspect(ctx, want=("vid",))["vid"].cpu().numpy()
    return ctx, A, vid


def test_row_sort_paths(gp):
    seen = set()
    for name, x, xr, tuples, dhat, kappa in _scenes():
        V = x.shape[0]
        diag = np.linspace(1.0, 2.0, V)
        ctx, A, vid = _run(gp, x, xr, tuples, dhat, kappa, diag)
        rp = A.row_ptr().cpu().numpy()
        ci = A.col_idx().cpu().numpy()
        # the pattern from the staged stencils
        cols = [{r} for r in range(V)]
        ninc = np.zeros(V, int)
        tsum = np.zeros(V, int)
        for st in vid:
            vs = [int(v) for v in st if v >= 0]
            for a in vs:
                ninc[a] += 1
                tsum[a] += len(vs) - 1
                cols[a].update(vs)
        ref_rp = np.concatenate([[0], np.cumsum([len(c) for c in cols])])
        ref_ci = np.concatenate([np.array(sorted(c), np.int32) for c in cols])
        assert np.array_equal(rp, ref_rp), name
        assert np.array_equal(ci, ref_ci), name
        # values against the oracle's assembly
        r = oracle.eval_scene(x, tuples, oracle.params(dhat=dhat, kappa=kappa), x_rest=xr, per_pair=True)
        rows, ocols, vals = oracle.assemble(V, tuples, r["pairH"], diag)
        G = np.zeros((3 * V, 3 * V))
        for rr, cc, b in zip(rows, ocols, vals.reshape(-1, 3, 3)):
            G[3 * rr:3 * rr + 3, 3 * cc:3 * cc + 3] += b
        D = A.to_scipy().toarray()
        assert np.abs(D - G).max() <= 1e-9 * np.abs(G).max(), name
        # a second build gives the same bits
        ctx2, A2, _ = _run(gp, x, xr, tuples, dhat, kappa, diag)
        assert torch.equal(A.val, A2.val), name
        ctx2.close()
        ctx.close()
        for n_, t_ in zip(ninc, tsum):
            if n_ == 0:
                seen.add("empty")
            elif n_ > 128:
                seen.add("workgroup")
            else:
                seen.add("own2" if n_ > 64 else "own1")
                seen.add("M1" if t_ <= 64 else "M2" if t_ <= 128 else "M4" if t_ <= 256 else "M8")
        print(name, "incidences per row: max", ninc.max(), "median", int(np.median(ninc)),
              "other slots: max", tsum.max(), flush=True)
    print("row-sort paths seen:", sorted(seen), flush=True)
    for need in ("own1", "own2", "M1", "M2", "M4", "M8", "workgroup"):
        assert need in seen, need
