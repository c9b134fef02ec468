"""The C-ABI boundary on the GPU: the paper's tuple encodings, degenerate
input, the filter and cut-off edges of the barrier, and the check that tells
a caller when the staged pairs no longer describe the tuples at new
positions.

* close-to-parallel point-edge / point-point encodings (Sec. 7.2) against the
  oracle: energy, gradient and every BSR block to 1e-9;
* a zero-length edge, a zero-area triangle and a non-finite position, forced
  from the host among regular pairs: counted (degenerate primitives, or
  degenerate distances for the non-finite one), no NaN anywhere in energy,
  gradient or blocks, and the rest against the oracle;
* pairs at g = eps_g (1 -+ 1e-6) (Eq. 23's filter switch) and g -> 1 (the
  barrier's cut-off at dhat), point-point, point-triangle and edge-edge,
  against the oracle per pair: 1e-9 relative, loosened only at g = 1 - 1e-6
  by the conditioning of (1 - g) there (64 eps / (1 - g));
* gipc_pairs_check: OK at the build's positions and after moves that keep
  every active set; GIPC_WARN_STALE when a point slides off its triangle
  (point-triangle -> point-edge) and when a pair comes within dhat; after the
  rebuild, parity with the oracle at the new positions; a pair that leaves
  dhat over the same sub-type counts as harmless.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

TOL = 1e-9
DH = 1e-3


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _neg(i):
    return -(i + 1)


def _run(gp, x, tuples, dhat=DH, kappa=1e4, diag=10.0, xr=None):
    dev = torch.device("cuda", 0)
    X = torch.tensor(x, device=dev)
    XR = torch.tensor(xr if xr is not None else x, device=dev)
    T = torch.tensor(np.asarray(tuples, np.int32).reshape(-1, 4), device=dev)
    prm = gp.params(dhat=dhat, kappa=kappa)
    ctx = gp.Context()
    info = gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx)
    D = torch.full((x.shape[0],), diag, dtype=torch.float64, device=dev)
    E, g = gp.eval_assemble(ctx, X, prm, A, diag=D, x_rest=XR)
    return dict(ctx=ctx, info=info, A=A, E=E.item(), grad=g.cpu().numpy(), X=X, XR=XR, T=T, prm=prm, D=D)


def _blocks(A):
    rp = A.row_ptr().cpu().numpy()
    ci = A.col_idx().cpu().numpy()
    v = A.val[:, :A.nnzb].double().cpu().numpy().T.reshape(-1, 3, 3)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return {(int(r), int(c)): B for r, c, B in zip(rows, ci, v)}


def _oracle(x, tuples, dhat=DH, kappa=1e4, diag=10.0, xr=None):
    po = oracle.params(dhat=dhat, kappa=kappa)
    r = oracle.eval_scene(x, np.asarray(tuples, np.int32).reshape(-1, 4), po,
                          x_rest=xr if xr is not None else x, per_pair=True)
    rows, cols, vals = oracle.assemble(x.shape[0], np.asarray(tuples, np.int32).reshape(-1, 4), r["pairH"],
                                       np.full(x.shape[0], diag))
    r["blocks"] = {(int(a), int(b)): B for a, b, B in zip(rows, cols, vals)}
    return r


def _compare(gpu, ref, tol=TOL):
    assert gpu["E"] == pytest.approx(ref["E"], rel=tol, abs=1e-300)
    gs = np.abs(ref["grad"]).max()
    assert np.abs(gpu["grad"] - ref["grad"]).max() <= tol * max(gs, 1e-300)
    gb, ob = _blocks(gpu["A"]), ref["blocks"]
    hs = max(np.abs(B).max() for B in ob.values())
    for k in set(gb) | set(ob):
        assert np.abs(gb.get(k, 0.0) - ob.get(k, 0.0)).max() <= tol * hs, k


# ------------------------------------------------------------ encodings


def _parallel_scene():
    """Three groups of two nearly parallel edges, each group 10 units apart:
    point p of (p, o) over the interior of (e0, e1) (point-edge), p beyond
    e0's end (point-point), and the same with a larger tilt (no mollifier)."""
    xs, tup = [], []

    def add(p, o, e0, e1, enc):
        b = len(xs)
        xs.extend([p, o, e0, e1])
        if enc == "pe":
            tup.append([_neg(b), _neg(b + 1), b + 2, _neg(b + 3)])
        elif enc == "pp":
            tup.append([_neg(b), _neg(b + 1), _neg(b + 2), _neg(b + 3)])
        tup.append([b, _neg(b + 1), b + 2, b + 3])      # the edge-edge pair, parallel-flagged

    for k, tilt in enumerate((2e-2 * DH, 0.2)):
        off = np.array([10.0 * k, 0.0, 0.0])
        add(off + [0.0, 0.0, 0.5 * DH], off + [-1.0, 0.0, 0.5 * DH + tilt], off + [-0.5, 0.0, 0.0],
            off + [0.5, 0.0, 0.0], "pe")
        off = off + [0.0, 5.0, 0.0]
        add(off + [-0.3 * DH, 0.0, 0.4 * DH], off + [-1.0, 0.0, 0.4 * DH + tilt], off + [0.0, 0.0, 0.0],
            off + [1.0, 0.0, 0.0], "pp")
    return np.array(xs, float), np.array(tup, np.int32)


def test_parallel_encodings_against_oracle(gp):
    x, t = _parallel_scene()
    gpu = _run(gp, x, t)
    ref = _oracle(x, t)
    print(f"[boundary] parallel encodings: active {gpu['info']['n_active']} by type {gpu['info']['n_by_type']}",
          flush=True)
    assert gpu["info"]["n_active"] == len(t)
    by = gpu["info"]["n_by_type"]
    assert by["PE_moll"] >= 2 and by["PP_moll"] >= 2 and by["PE"] + by["PP"] >= 4
    _compare(gpu, ref)
    gpu["ctx"].close()


# ------------------------------------------------------------ degenerate input


def test_degenerate_inputs_counted_without_nan(gp):
    rng = np.random.default_rng(8)
    x = []
    # 0-3: a regular point-triangle pair
    x += [[0.2, 0.2, 0.4 * DH], [0, 0, 0], [1, 0, 0], [0, 1, 0]]
    # 4-7: point over a zero-area triangle (collinear vertices)
    x += [[10.3, 0.0, 0.3 * DH], [10, 0, 0], [11, 0, 0], [10.5, 0, 0]]
    # 8-11: an edge of zero length against an edge
    x += [[20.2, 0.0, 0.5 * DH], [20.2, 0.0, 0.5 * DH], [20, 0, 0], [21, 0, 0]]
    # 12-15: a pair touching a non-finite position
    x += [[30.2, 0.2, 0.4 * DH], [30, 0, 0], [31, 0, 0], [30, 1, 0]]
    # 16-19: a regular edge-edge pair
    x += [[40.5, -0.5, 0.6 * DH], [40.5, 0.5, 0.6 * DH], [40, 0, 0], [41, 0, 0]]
    x = np.array(x, float)
    x[[1, 2, 3, 17]] += rng.uniform(-1e-5, 1e-5, (4, 3))
    t = np.array([[_neg(0), 1, 2, 3], [_neg(4), 5, 6, 7], [8, 9, 10, 11], [_neg(12), 13, 14, 15],
                  [16, 17, 18, 19]], np.int32)
    xn = x.copy()
    xn[12, 2] = np.nan
    gpu = _run(gp, xn, t)
    info = gpu["info"]
    print(f"[boundary] degenerate: {info['n_degenerate']} distance, {info['n_degenerate_prims']} primitive", flush=True)
    assert info["n_degenerate"] == 1 and info["first_degenerate"] == 3
    assert info["n_degenerate_prims"] == 2 and info["first_degenerate_prim"] == 1
    assert info["n_active"] == 4
    assert np.isfinite(gpu["E"]) and np.isfinite(gpu["grad"]).all()
    assert torch.isfinite(gpu["A"].val[:, :gpu["A"].nnzb]).all()
    # the non-finite tuple contributes nothing; the rest equals the oracle on
    # the same list with that tuple dropped (the vertex keeps its diagonal)
    ref = _oracle(x, np.delete(t, 3, axis=0))
    _compare(gpu, ref)
    gpu["ctx"].close()


# ------------------------------------------------------------ filter and cut-off


def _pair_at(kind, d):
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    if kind == "pp":
        x = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3] + d * u])
        return x, np.array([[_neg(0), 1, -1, -1]], np.int32)
    if kind == "pt":
        x = np.array([[0.25, 0.25, d], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
        return x, np.array([[_neg(0), 1, 2, 3]], np.int32)
    x = np.array([[0.5, -0.5, d], [0.5, 0.5, d], [0, 0, 0], [1, 0, 0]], float)     # crossing edges
    return x, np.array([[0, 1, 2, 3]], np.int32)


@pytest.mark.parametrize("kind", ["pp", "pt", "ee"])
@pytest.mark.parametrize("g", [0.01 * (1 - 1e-6), 0.01 * (1 + 1e-6), 1 - 1e-2, 1 - 1e-4, 1 - 1e-6, 1 + 1e-9])
def test_filter_switch_and_cutoff_against_oracle(gp, kind, g):
    d = DH * np.sqrt(g)
    x, t = _pair_at(kind, d)
    gpu = _run(gp, x, t, diag=0.0)
    ref = _oracle(x, t, diag=0.0)
    if g > 1:
        assert gpu["info"]["n_active"] == 0 and gpu["E"] == 0.0 and ref["E"] == 0.0
        assert not np.any(gpu["grad"]) and not np.any(ref["grad"])
    else:
        assert gpu["info"]["n_active"] == 1
        tol = max(TOL, 64 * np.finfo(float).eps / (1 - g))
        assert gpu["E"] > 0.0
        _compare(gpu, ref, tol)
    gpu["ctx"].close()


# ------------------------------------------------------------ staleness check


def _check_scene():
    # 0-3: point 0.5 dhat over triangle (0,0,0) (1,0,0) (0,1,0), near its
    # long edge; 4-7: two crossing edges 2 dhat apart (inactive)
    x = np.array([[0.45, 0.45, 0.5 * DH], [0, 0, 0], [1, 0, 0], [0, 1, 0],
                  [10.5, -0.5, 2 * DH], [10.5, 0.5, 2 * DH], [10, 0, 0], [11, 0, 0]], float)
    t = np.array([[_neg(0), 1, 2, 3], [4, 5, 6, 7]], np.int32)
    return x, t


def test_pairs_check_reports_stale_builds(gp):
    x0, t = _check_scene()
    gpu = _run(gp, x0, t)
    ctx, prm, T = gpu["ctx"], gpu["prm"], gpu["T"]
    dev = gpu["X"].device
    assert gpu["info"]["n_active"] == 1
    stale, c = gp.pairs_check(ctx, gpu["X"], T, prm, x_rest=gpu["XR"])
    assert not stale and c == {"n_entered": 0, "n_left": 0, "n_changed": 0, "n_degenerate": 0, "first": -1}
    # a small move that keeps both active sets
    x1 = x0.copy()
    x1[0] += [0.01, -0.02, 0.1 * DH]
    stale, c = gp.pairs_check(ctx, torch.tensor(x1, device=dev), T, prm, x_rest=gpu["XR"])
    assert not stale and c["n_changed"] == 0 and c["n_entered"] == 0
    # the point slides off the triangle across its long edge (point-triangle
    # -> point-edge) and the edges come within dhat
    x2 = x0.copy()
    x2[0] = [0.5 + 0.3 * DH, 0.5 + 0.3 * DH, 0.5 * DH]
    x2[4:6, 2] = 0.5 * DH
    X2 = torch.tensor(x2, device=dev)
    stale, c = gp.pairs_check(ctx, X2, T, prm, x_rest=gpu["XR"])
    print(f"[boundary] check after the move: {c}", flush=True)
    assert stale and c["n_changed"] == 1 and c["n_entered"] == 1 and c["first"] == 0
    # evaluating the old build there uses the plane distance of the point-
    # triangle sub-type: not the oracle's energy at x2
    E_old, _ = gp.barrier_eval(ctx, X2, prm, x_rest=gpu["XR"])
    ref = _oracle(x2, t)
    assert abs(E_old.item() - ref["E"]) > 1e-3 * abs(ref["E"])
    ctx.close()
    # rebuilt at x2: parity again, and the check is clean
    gpu2 = _run(gp, x2, t)
    assert gpu2["info"]["n_active"] == 2 and gpu2["info"]["n_by_type"]["PE"] == 1
    _compare(gpu2, ref)
    stale, c = gp.pairs_check(gpu2["ctx"], gpu2["X"], T, prm, x_rest=gpu2["XR"])
    assert not stale and c["n_changed"] == 0
    # leaving dhat over the triangle's interior: harmless (the staged
    # point-triangle formula also puts it beyond dhat)
    x3 = x2.copy()
    x3[0] = [0.3, 0.3, 2 * DH]        # far from the staged edge's line as well
    stale, c = gp.pairs_check(gpu2["ctx"], torch.tensor(x3, device=dev), T, prm, x_rest=gpu2["XR"])
    assert not stale and c["n_left"] == 1 and c["n_changed"] == 0
    gpu2["ctx"].close()
    gpu3 = _run(gp, x0, t)
    x4 = x0.copy()
    x4[0, 2] = 2 * DH                 # straight up: the staged plane distance is 2 dhat too
    stale, c = gp.pairs_check(gpu3["ctx"], torch.tensor(x4, device=dev), T, prm, x_rest=gpu3["XR"])
    assert not stale and c["n_left"] == 1 and c["n_changed"] == 0
    # far off the triangle but still near its plane: inactive, while the
    # staged point-triangle formula (the plane distance) would count it
    x5 = x0.copy()
    x5[0] = [2.0, 2.0, 0.5 * DH]
    stale, c = gp.pairs_check(gpu3["ctx"], torch.tensor(x5, device=dev), T, prm, x_rest=gpu3["XR"])
    assert stale and c["n_left"] == 0 and c["n_changed"] == 1 and c["first"] == 0
    # wrong list size: a state error
    with pytest.raises(gp.GipcError) as ei:
        gp.pairs_check(gpu3["ctx"], gpu3["X"], T[:1].contiguous(), prm, x_rest=gpu3["XR"])
    assert ei.value.status == gp.ERR_STATE
    gpu3["ctx"].close()
