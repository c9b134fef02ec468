"""GPU contact candidates (gipc_candidates) against the oracle's brute force.

* small seeded two-sheet scenes (several sizes and dhat): the candidate set
  equals the brute-force set exactly (integer work: bit-exact), in the
  documented order (point-triangle by point, then edge-edge by first edge);
  two calls give the same array; the largest puts hundreds of primitives
  and queries in a cell (several 64-wide chunks per cell);
* a context's capacity hint: calls whose count grows past it, then falls
  back under it, each give the brute-force set;
* the two-sheet 16 x 16 and ten-sheet 256 x 256 scenes: the set equals the
  scenes' own grid generator's (pinned against brute force on the CPU);
* the list fed to the hot path gives the same active pairs and energy as
  the host list;
* edge cases and errors: no vertices, no primitives, a bad vertex id, a
  negative dhat, a too small capacity.
"""
import ctypes

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


def _dev(s):
    d = torch.device("cuda", 0)
    return (torch.tensor(s.x, device=d), torch.tensor(s.vobj, dtype=torch.int32, device=d),
            torch.tensor(s.tris, dtype=torch.int32, device=d), torch.tensor(s.edges, dtype=torch.int32, device=d))


def _set(t):
    return set(map(tuple, np.asarray(t).reshape(-1, 4).tolist()))


@pytest.mark.parametrize("n,dhat,seed", [(6, 0.15, 3), (9, 0.3, 7), (12, 0.05, 1), (8, 0.0, 2), (24, 0.3, 5)])
def test_small_scenes_against_brute_force(gp, n, dhat, seed):
    s = scenes.two_sheets(n=n, dhat=max(dhat, 1e-3), kappa=10.0, seed=seed, offset=0.5, jitter=0.3)
    x, vobj, tris, edges = _dev(s)
    ctx = gp.Context()
    c = gp.candidates(ctx, x, vobj, tris, edges, dhat).cpu().numpy()
    ref = oracle.candidates(s.x, s.vobj, s.tris, s.edges, dhat)
    assert len(c) == len(ref) and _set(c) == _set(ref)
    # order: PT grouped by increasing point, then EE grouped by increasing first edge
    pt = c[:, 0] < 0
    npt = int(pt.sum())
    assert pt[:npt].all() and not pt[npt:].any()
    p = -c[:npt, 0] - 1
    assert (np.diff(p) >= 0).all()
    eid = {tuple(e): i for i, e in enumerate(s.edges.tolist())}
    first = np.array([eid[(a, b)] for a, b in c[npt:, :2].tolist()])
    assert (np.diff(first) >= 0).all()
    c2 = gp.candidates(ctx, x, vobj, tris, edges, dhat).cpu().numpy()
    assert np.array_equal(c, c2)
    ctx.close()


def test_capacity_hint_across_calls(gp):
    s = scenes.two_sheets(n=9, dhat=0.3, kappa=10.0, seed=7, offset=0.5, jitter=0.3)
    x, vobj, tris, edges = _dev(s)
    ctx = gp.Context()
    got = []
    for dhat in (0.02, 0.3, 0.02, 0.02):
        c = gp.candidates(ctx, x, vobj, tris, edges, dhat).cpu().numpy()
        ref = oracle.candidates(s.x, s.vobj, s.tris, s.edges, dhat)
        assert len(c) == len(ref) and _set(c) == _set(ref), dhat
        assert ctx._cand_cap >= len(c)
        got.append(c)
    assert len(got[1]) > 2 * len(got[0])  # the second call outgrew the hint
    assert np.array_equal(got[0], got[2]) and np.array_equal(got[2], got[3])
    ctx.close()


@pytest.mark.parametrize("which", ["sheets16", "sheets10x256"])
def test_matches_the_grid_generator(gp, which):
    s = scenes.two_sheets(n=16, seed=1) if which == "sheets16" else scenes.stacked_sheets(n_sheets=10, n=256, seed=2)
    x, vobj, tris, edges = _dev(s)
    ctx = gp.Context()
    c = gp.candidates(ctx, x, vobj, tris, edges, s.dhat)
    h = torch.tensor(s.tuples, device="cuda")
    assert c.shape == h.shape
    assert torch.equal(_lexsorted(c), _lexsorted(h))
    ctx.close()


def _lexsorted(t):
    """rows in lexicographic order (stable sorts from the last column)"""
    idx = torch.arange(t.shape[0], device=t.device)
    for col in range(t.shape[1] - 1, -1, -1):
        idx = idx[torch.sort(t[idx, col], stable=True).indices]
    return t[idx]


def test_feeds_the_hot_path(gp):
    s = scenes.two_sheets(n=16, seed=1)
    x, vobj, tris, edges = _dev(s)
    xr = torch.tensor(s.x_rest, device="cuda")
    prm = gp.params(dhat=s.dhat, kappa=s.kappa)
    ctx = gp.Context()
    c = gp.candidates(ctx, x, vobj, tris, edges, s.dhat)
    info_g = gp.pairs_build(ctx, x, c, prm, x_rest=xr)
    Eg, _ = gp.barrier_eval(ctx, x, prm, x_rest=xr)
    ctx2 = gp.Context()
    info_h = gp.pairs_build(ctx2, x, torch.tensor(s.tuples, device="cuda"), prm, x_rest=xr)
    Eh, _ = gp.barrier_eval(ctx2, x, prm, x_rest=xr)
    assert info_g["n_active"] == info_h["n_active"] and info_g["n_staged"] == info_h["n_staged"]
    assert Eg.item() == pytest.approx(Eh.item(), rel=1e-12)
    ctx.close(); ctx2.close()


def test_edge_cases_and_errors(gp):
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    x, vobj, tris, edges = _dev(s)
    ctx = gp.Context()
    none3 = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
    none2 = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    assert gp.candidates(ctx, x, vobj, none3, none2, 0.1).shape == (0, 4)
    only_pt = gp.candidates(ctx, x, vobj, tris, none2, 0.15).cpu().numpy()
    assert (only_pt[:, 0] < 0).all() and len(only_pt) > 0
    only_ee = gp.candidates(ctx, x, vobj, none3, edges, 0.15).cpu().numpy()
    ref_ee = oracle.candidates(s.x, s.vobj, np.zeros((0, 3), np.int32), s.edges, 0.15)
    assert (only_ee[:, 0] >= 0).all() and len(only_ee) > 0 and _set(only_ee) == _set(ref_ee)
    x0 = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    assert gp.candidates(ctx, x0, vobj[:0], none3, none2, 0.1).shape == (0, 4)
    bad = tris.clone()
    bad[3, 1] = s.V + 7
    with pytest.raises(gp.GipcError) as ei:
        gp.candidates(ctx, x, vobj, bad, edges, 0.1)
    assert ei.value.status == gp.ERR_INDEX
    rep = edges.clone()
    rep[0, 1] = rep[0, 0]
    with pytest.raises(gp.GipcError) as ei:
        gp.candidates(ctx, x, vobj, tris, rep, 0.1)
    assert ei.value.status == gp.ERR_INDEX
    with pytest.raises(gp.GipcError) as ei:
        gp.candidates(ctx, x, vobj, tris, edges, -1.0)
    assert ei.value.status == gp.ERR_INVALID_ARG
    # capacity below the count: WORKSPACE and the count reported
    mesh = gp.Context._mesh(x, None)
    topo = gp.Topology(vobj.data_ptr(), tris.data_ptr(), tris.shape[0], edges.data_ptr(),
                       edges.shape[0])
    out = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    st = gp.lib().gipc_candidates(ctx.h, ctypes.byref(mesh), ctypes.byref(topo), 0.15, ctypes.c_void_p(out.data_ptr()),
                                  1, ctypes.byref(n), None)
    assert st == gp.ERR_WORKSPACE and n.value == len(oracle.candidates(s.x, s.vobj, s.tris, s.edges, 0.15))
    ctx.close()
