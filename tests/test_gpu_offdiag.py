"""The off-diagonal assembly over its regimes, against the oracle's assembly.

The off-diagonal pass takes a row's blocks above the diagonal 32 at a time (a
window) and deals the window's contribution lists, which are contiguous, to
its 32 lanes 64 contributions at a time (a step); each block's owner lane
adds its terms in list order.  The scenes put rows in every regime, checked
from the staged pairs:

* a point numbered first over a fine 40 x 40 patch: its row holds over a
  thousand blocks above the diagonal (many windows);
* the same over a 30 x 30 patch with merging off and 100 copies of one typed
  point-point tuple: windows whose lists span several steps, and one block
  list longer than a step;
* two sheets: rows within one window and one step.

For each scene: the FP64 matrix equals the oracle's assembly within 1e-9 of
its largest entry, A is exactly symmetric, and every launch shape of the
off-diagonal pass and both row orders give the same bits.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
scipy_sparse = pytest.importorskip("scipy.sparse")

import oracle  # noqa: E402
import scenes  # noqa: E402

WINDOW = 32   # blocks per window
STEP = 64     # contributions per step


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _fan_first(n=40, dhat=1e-3, copies=0):
    """A point (vertex 0) 0.3 dhat over an n x n patch of side 0.5 dhat, one
    point-triangle candidate per patch triangle, and `copies` typed
    point-point tuples (0, 5)."""
    g = np.linspace(0.0, 0.5 * dhat, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.vstack([[[0.25 * dhat, 0.25 * dhat, 0.3 * dhat]], np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], 1)])
    tup = []
    for i in range(n - 1):
        for j in range(n - 1):
            a, b, c, d = (1 + i * n + j, 1 + (i + 1) * n + j, 1 + i * n + j + 1, 1 + (i + 1) * n + j + 1)
            tup += [[-1, a, b, c], [-1, b, d, c]]
    tup += [[-1, 5, -1, -1]] * copies
    return x, np.asarray(tup, np.int32), dhat, 1e4


def _scenes():
    s = scenes.two_sheets(n=16, seed=3)
    out = [("two_sheets_16", s.x, s.x_rest, s.tuples, s.dhat, s.kappa, False)]
    x, t, dh, k = _fan_first()
    out.append(("fan_first", x, None, t, dh, k, False))
    x, t, dh, k = _fan_first(n=30, copies=100)  # the point row stays under 2048 pairs
    out.append(("fan_first_unmerged_copies", x, None, t, dh, k, True))
    return out


def _regimes(vid, V):
    """Windows per row, contributions per window and per block, from the
    staged stencils (one contribution per pair per stencil vertex pair)."""
    cnt = {}
    for st in vid:
        vs = [int(v) for v in st if v >= 0]
        for a in range(len(vs)):
            for b in range(a + 1, len(vs)):
                key = (min(vs[a], vs[b]), max(vs[a], vs[b]))
                cnt[key] = cnt.get(key, 0) + 1
    rows = {}
    for (r, c), n in cnt.items():
        rows.setdefault(r, []).append((c, n))
    max_blocks = max(len(v) for v in rows.values())
    max_window = 0
    for v in rows.values():
        v.sort()
        for w in range(0, len(v), WINDOW):
            max_window = max(max_window, sum(n for _, n in v[w:w + WINDOW]))
    return max_blocks, max_window, max(cnt.values())


def _oracle_matrix(x, xr, tuples, dhat, kappa, diag):
    V = x.shape[0]
    r = oracle.eval_scene(x, tuples, oracle.params(dhat=dhat, kappa=kappa), x_rest=xr, per_pair=True)
    rows, cols, vals = oracle.assemble(V, tuples, r["pairH"], diag)
    b = vals.reshape(-1, 3, 3)
    ii = (3 * np.asarray(rows)[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2)
    jj = (3 * np.asarray(cols)[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1)
    return scipy_sparse.coo_matrix((b.ravel(), (ii.ravel(), jj.ravel())), shape=(3 * V, 3 * V)).tocsr()


def test_offdiag_regimes_shapes_and_orders(gp):
    dev = torch.device("cuda", 0)
    seen = set()
    for name, x, xr, tuples, dhat, kappa, no_merge in _scenes():
        V = x.shape[0]
        diag = torch.tensor(np.linspace(1.0, 2.0, V), device=dev)
        X = torch.tensor(x, device=dev)
        XR = torch.tensor(xr, device=dev) if xr is not None else None
        T = torch.tensor(np.asarray(tuples, np.int32).reshape(-1, 4), device=dev)
        flags = gp.FLAGS_DEFAULT | (gp.FLAG_NO_MERGE if no_merge else 0)
        prm = gp.params(dhat=dhat, kappa=kappa, flags=flags)
        ctx = gp.Context()
        gp.pairs_build(ctx, X, T, prm, x_rest=XR)
        vid = gp.pair_inspect(ctx, want=("vid",))["vid"].cpu().numpy()
        mb, mw, mc = _regimes(vid, V)
        print(name, "blocks above the diagonal per row: max", mb, "contributions per window: max", mw,
              "per block: max", mc, flush=True)
        if mb > WINDOW:
            seen.add("windows")
        if mw > STEP:
            seen.add("window_steps")
        if mc > STEP:
            seen.add("block_steps")
        A = gp.BsrMatrix(ctx, dtype=gp.F64)
        ref = None
        for waves in (1, 2, 4, 8):
            for order in (0, 1):
                gp.set_tune(ctx, offdiag_waves=waves, row_order=order)
                gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
                torch.cuda.synchronize()
                if ref is None:
                    ref = A.val.clone()
                else:
                    assert torch.equal(A.val, ref), (name, waves, order)
        D = A.to_scipy().tocsr()
        G = _oracle_matrix(x, xr, tuples, dhat, kappa, diag.cpu().numpy())
        assert abs(D - G).max() <= 1e-9 * abs(G).max(), name
        assert abs(D - D.T).max() == 0.0, name
        ctx.close()
    for need in ("windows", "window_steps", "block_steps"):
        assert need in seen, need
