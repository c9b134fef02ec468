"""Batches of independent scenes (per-scene dhat and kappa in one launch
sequence), the HIP-graph replay of eval + assembly, and the autotuner.

* a small batch of two-sheet scenes against the oracle run scene by scene:
  per-scene energies and the gradient to 1e-9 relative, every BSR block to
  1e-9 of the largest entry;
* the batch against the same scenes built and evaluated one at a time:
  bitwise equal (a scene's pairs keep their relative order, so every sum
  runs in the same order);
* errors: a tuple spanning two scenes, malformed scene offsets, a call
  without the build's batch;
* graph replays with positions changed in place between them, and with
  eager work in between, equal eager gipc_eval_assemble bitwise;
* the autotuner returns supported shapes; the results with them match the
  default shapes to 1e-12 (only summation order changes);
* the 64-scene workload (resolution 32..256 per side, dhat log-uniform in
  [1e-4, 1e-2], seeds 1000 + s): per-scene energies of four scenes vs the
  oracle; BSR blocks on sampled rows of six scenes vs the oracle, FP64
  (1e-9) and the FP32 graph replay (1e-5); three scenes vs their own
  single-scene runs, bitwise.
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


def small_batch(S=6, seed_base=500):
    return scenes.batch_two_sheets(S=S, r_lo=6, r_hi=20, dhat_lo=1e-3, dhat_hi=2e-1, seed_base=seed_base)


def run_batch(gp, b, dtype=0):
    dev = torch.device("cuda", 0)
    X = torch.tensor(b.x, device=dev)
    XR = torch.tensor(b.x_rest, device=dev)
    T = torch.tensor(b.tuples, device=dev)
    bt = gp.Batch(b.vert_off, b.dhat, b.kappa)
    prm = gp.params(batch=bt)
    ctx = gp.Context()
    info = gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    diag = torch.full((b.V,), 10.0, dtype=torch.float64, device=dev)
    E, g = gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
    return dict(ctx=ctx, info=info, A=A, E=E, g=g, X=X, XR=XR, prm=prm, diag=diag, batch=bt)


def run_single(gp, sc):
    dev = torch.device("cuda", 0)
    X = torch.tensor(sc.x, device=dev)
    XR = torch.tensor(sc.x_rest, device=dev)
    T = torch.tensor(sc.tuples, device=dev)
    prm = gp.params(dhat=sc.dhat, kappa=sc.kappa)
    ctx = gp.Context()
    gp.pairs_build(ctx, X, T, prm, x_rest=XR)
    A = gp.BsrMatrix(ctx)
    diag = torch.full((sc.V,), 10.0, dtype=torch.float64, device=dev)
    E, g = gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
    return dict(ctx=ctx, A=A, E=E, g=g)


def blocks(A, r0=0, r1=None):
    rp = A.row_ptr().cpu().numpy()
    ci = A.col_idx().cpu().numpy()
    v = A.val[:, :A.nnzb].double().cpu().numpy().T.reshape(-1, 3, 3)
    r1 = len(rp) - 1 if r1 is None else r1
    out = {}
    for r in range(r0, r1):
        for s in range(rp[r], rp[r + 1]):
            out[(r - r0, int(ci[s]) - r0)] = v[s]
    return out


def test_small_batch_against_oracle(gp):
    b = small_batch()
    res = run_batch(gp, b)
    E = res["E"].cpu().numpy()
    g = res["g"].cpu().numpy()
    assert E.shape == (b.S,)
    for s, sc in enumerate(b.scenes):
        v0, v1 = b.vert_off[s], b.vert_off[s + 1]
        po = oracle.params(dhat=sc.dhat, kappa=sc.kappa)
        r = oracle.eval_scene(sc.x, sc.tuples, po, x_rest=sc.x_rest, per_pair=True)
        assert E[s] == pytest.approx(r["E"], rel=TOL, abs=1e-300), s
        gs = g[v0:v1]
        assert np.abs(gs - r["grad"]).max() <= TOL * max(np.abs(r["grad"]).max(), 1e-300), s
        rows, cols, vals = oracle.assemble(sc.V, sc.tuples, r["pairH"], np.full(sc.V, 10.0))
        o = {}
        for rr, cc, B in zip(rows, cols, vals):
            o[(int(rr), int(cc))] = o.get((int(rr), int(cc)), 0.0) + B
        gb = blocks(res["A"], v0, v1)
        hs = max(np.abs(B).max() for B in o.values())
        for key in set(o) | set(gb):
            assert np.abs(gb.get(key, 0.0) - o.get(key, 0.0)).max() <= TOL * hs, (s, key)
    res["ctx"].close()


def test_batch_equals_scenes_run_one_at_a_time(gp):
    b = small_batch(S=5, seed_base=700)
    res = run_batch(gp, b)
    for s, sc in enumerate(b.scenes):
        v0, v1 = b.vert_off[s], b.vert_off[s + 1]
        one = run_single(gp, sc)
        assert res["E"][s].item() == one["E"].item(), s
        assert torch.equal(res["g"][v0:v1], one["g"]), s
        gb, ob = blocks(res["A"], v0, v1), blocks(one["A"])
        assert gb.keys() == ob.keys()
        assert all(np.array_equal(gb[k], ob[k]) for k in gb), s
        one["ctx"].close()
    res["ctx"].close()


def test_batch_errors(gp):
    b = small_batch(S=3, seed_base=900)
    dev = torch.device("cuda", 0)
    X = torch.tensor(b.x, device=dev)
    ctx = gp.Context()
    # a tuple joining the first vertex of scene 0 and of scene 1 (at index 5,
    # which the message names)
    bad = b.tuples.copy()
    bad[5] = [-(0 + 1), int(b.vert_off[1]), -1, -1]
    bt = gp.Batch(b.vert_off, b.dhat, b.kappa)
    with pytest.raises(gp.GipcError, match="two scenes") as ei:
        gp.pairs_build(ctx, X, torch.tensor(bad, device=dev), gp.params(batch=bt))
    assert ei.value.status == gp.ERR_INDEX and "first at 5" in str(ei.value)
    # scene offsets that do not end at V, or decrease
    for vo in ([0, 5, 3, b.V], [0, 10, 20, b.V - 1]):
        with pytest.raises(gp.GipcError) as ei:
            gp.pairs_build(ctx, X, torch.tensor(b.tuples, device=dev),
                           gp.params(batch=gp.Batch(vo, b.dhat, b.kappa)))
        assert ei.value.status == gp.ERR_INVALID_ARG
    with pytest.raises(gp.GipcError) as ei:
        gp.pairs_build(ctx, X, torch.tensor(b.tuples, device=dev),
                       gp.params(batch=gp.Batch(b.vert_off, [1e-3, -1.0, 1e-3], b.kappa)))
    assert ei.value.status == gp.ERR_INVALID_ARG
    # built with the batch, evaluated without it
    gp.pairs_build(ctx, X, torch.tensor(b.tuples, device=dev), gp.params(batch=bt))
    with pytest.raises(gp.GipcError) as ei:
        gp.barrier_eval(ctx, X, gp.params())
    assert ei.value.status == gp.ERR_STATE
    ctx.close()


def test_graph_replays_equal_eager(gp):
    b = small_batch(S=4, seed_base=1100)
    res = run_batch(gp, b)
    ctx, X, XR, prm, A, diag = res["ctx"], res["X"], res["XR"], res["prm"], res["A"], res["diag"]
    graph = gp.Graph(ctx, X, prm, A, diag=diag, x_rest=XR)
    A2 = gp.BsrMatrix(ctx)
    X0 = X.clone()
    rng = np.random.default_rng(3)
    for rep in range(4):
        # positions moved in place (small enough to keep every staged pair's type)
        X.copy_(X0 + torch.tensor(rng.uniform(-1e-9, 1e-9, size=b.x.shape), device=X.device))
        E, g = graph.launch()
        Eg, gg, Vg = E.clone(), g.clone(), A.val.clone()
        # eager work between replays, on the same context
        Ee, ge = gp.eval_assemble(ctx, X, prm, A2, diag=diag, x_rest=XR)
        torch.cuda.synchronize()
        assert torch.equal(Eg, Ee) and torch.equal(gg, ge) and torch.equal(Vg, A2.val), rep
    graph.close()
    # a rebuild invalidates the graph
    graph2 = gp.Graph(ctx, X, prm, A, diag=diag, x_rest=XR)
    gp.pairs_build(ctx, X, torch.tensor(b.tuples, device=X.device), prm, x_rest=XR)
    with pytest.raises(gp.GipcError) as ei:
        graph2.launch()
    assert ei.value.status == gp.ERR_STATE
    graph2.close()
    ctx.close()


def test_autotune(gp, tmp_path):
    b = small_batch(S=6, seed_base=1300)
    res = run_batch(gp, b)
    ctx, X, XR, prm, A, diag = res["ctx"], res["X"], res["XR"], res["prm"], res["A"], res["diag"]
    E0, g0, V0 = res["E"].clone(), res["g"].clone(), A.val.clone()
    cache = tmp_path / "tune.json"
    best = gp.autotune(ctx, X, prm, A, diag=diag, x_rest=XR, reps=3, cache=str(cache), key="small")
    assert best["eval_waves"] in (1, 2, 4, 8) and best["offdiag_waves"] in (1, 2, 4, 8)
    assert best["row_lanes"] in (4, 8, 16, 32) and best["row_order"] in (0, 1)
    assert gp.get_tune(ctx) == best
    E1, g1 = gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
    assert torch.allclose(E1, E0, rtol=1e-12, atol=0)
    assert float((g1 - g0).abs().max()) <= 1e-12 * float(g0.abs().max())
    assert float((A.val - V0).abs().max()) <= 1e-12 * float(V0.abs().max())
    # the cache answers without timing
    gp.set_tune(ctx, 4, 16, 4)
    again = gp.autotune(ctx, X, prm, A, diag=diag, x_rest=XR, cache=str(cache), key="small")
    assert again == best and gp.get_tune(ctx) == best
    # an entry written before a tune field existed is timed again, not applied
    import json
    table = json.loads(cache.read_text())
    (k,) = [k for k in table if k.endswith("|small")]
    assert "gfx" in k.split("|")[0] and k.split("|")[2] == gp._lib_digest()
    # an entry stored by another build of the library is not applied: the
    # choice is timed again and stored under the loaded library's key
    other = k.replace(gp._lib_digest(), "0" * 16)
    cache.write_text(json.dumps({other: table[k]}))
    gp.set_tune(ctx, 4, 16, 4)
    gp.autotune(ctx, X, prm, A, diag=diag, x_rest=XR, reps=1, cache=str(cache), key="small")
    assert set(json.loads(cache.read_text())) == {other, k}
    cache.write_text(json.dumps(table))
    stale = dict(table[k])
    del stale["row_order"]
    table[k] = stale
    cache.write_text(json.dumps(table))
    gp.set_tune(ctx, 4, 16, 4)
    fresh = gp.autotune(ctx, X, prm, A, diag=diag, x_rest=XR, reps=1, cache=str(cache), key="small")
    assert set(fresh) == {"eval_waves", "row_lanes", "offdiag_waves", "row_order"}
    assert "row_order" in json.loads(cache.read_text())[k]
    gp.set_tune(ctx, **best)
    with pytest.raises(gp.GipcError):
        gp.set_tune(ctx, 3, 16, 4)
    with pytest.raises(gp.GipcError):
        gp.set_tune(ctx, 4, 16, 4, 2)
    # the row order changes only the schedule: the same bits
    out = []
    for order in (0, 1):
        gp.set_tune(ctx, 4, 16, 4, order)
        E, g = gp.eval_assemble(ctx, X, prm, A, diag=diag, x_rest=XR)
        out.append((E.clone(), g.clone(), A.val.clone()))
    assert all(torch.equal(a, b) for a, b in zip(out[0], out[1]))
    ctx.close()


@pytest.fixture(scope="module")
def c4(gp):
    b = scenes.batch_two_sheets(S=64, seed_base=1000)
    res = run_batch(gp, b)
    yield b, res
    res["ctx"].close()


def test_64_scene_batch_energies_against_oracle(c4):
    b, res = c4
    E = res["E"].cpu().numpy()
    sizes = np.diff(b.pair_off)
    for s in np.argsort(sizes)[:4]:
        sc = b.scenes[s]
        r = oracle.eval_scene(sc.x, sc.tuples, oracle.params(dhat=sc.dhat, kappa=sc.kappa), x_rest=sc.x_rest)
        assert E[s] == pytest.approx(r["E"], rel=TOL), s
        g = res["g"][b.vert_off[s]:b.vert_off[s + 1]].cpu().numpy()
        assert np.abs(g - r["grad"]).max() <= TOL * np.abs(r["grad"]).max(), s


def _row_blocks(A, r):
    rp = A.row_ptr()
    lo, hi = int(rp[r]), int(rp[r + 1])
    ci = A.col_idx()[lo:hi].cpu().numpy()
    vals = A.val[:, lo:hi].double().cpu().numpy().T.reshape(-1, 3, 3)
    return {int(c): B for c, B in zip(ci, vals)}


def test_64_scene_batch_blocks_against_oracle_on_sampled_rows(gp, c4):
    # FP64 blocks of the eager call and FP32 blocks replayed from the graph,
    # both on sampled rows of the largest, the smallest and four more scenes
    b, res = c4
    ctx, A64 = res["ctx"], res["A"]
    A32 = gp.BsrMatrix(ctx, dtype=gp.F32)
    graph = gp.Graph(ctx, res["X"], res["prm"], A32, diag=res["diag"], x_rest=res["XR"])
    E32, g32 = graph.launch()
    torch.cuda.synchronize()
    assert torch.equal(E32, res["E"]) and torch.equal(g32, res["g"])   # FP32 changes only the blocks
    sizes = np.diff(b.pair_off)
    rng = np.random.default_rng(31)
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes))] + [int(v) for v in rng.choice(b.S, 4, replace=False)]
    for s in pick:
        sc = b.scenes[s]
        v0 = int(b.vert_off[s])
        rows = rng.choice(sc.V, 4, replace=False)
        kind, st = scenes.decode_tuples(sc.tuples)
        sub = sc.tuples[np.isin(st, rows).any(1)]
        po = oracle.params(dhat=sc.dhat, kappa=sc.kappa)
        r = oracle.eval_scene(sc.x, sub, po, x_rest=sc.x_rest, per_pair=True)
        orows, ocols, ovals = oracle.assemble(sc.V, sub, r["pairH"], np.full(sc.V, 10.0))
        for row in rows:
            sel = orows == row
            o = {int(c): B for c, B in zip(ocols[sel], ovals[sel])}
            hs = max(np.abs(B).max() for B in o.values())
            for A, tol in ((A64, TOL), (A32, 1e-5)):
                g = {c - v0: B for c, B in _row_blocks(A, v0 + int(row)).items()}
                assert all(0 <= c < sc.V for c in g), s
                for c in set(g) | set(o):
                    assert np.abs(g.get(c, 0.0) - o.get(c, 0.0)).max() <= tol * hs, (s, int(row), c, tol)
    graph.close()


def test_64_scene_batch_equals_single_runs(gp, c4):
    b, res = c4
    for s in (0, 17, 63):
        v0, v1 = b.vert_off[s], b.vert_off[s + 1]
        one = run_single(gp, b.scenes[s])
        assert res["E"][s].item() == one["E"].item(), s
        assert torch.equal(res["g"][v0:v1], one["g"]), s
        one["ctx"].close()


def test_autograd_with_per_scene_energies(gp):
    b = small_batch(S=4, seed_base=1500)
    res = run_batch(gp, b)
    ctx, X, XR, prm = res["ctx"], res["X"], res["XR"], res["prm"]
    x = X.clone().requires_grad_(True)
    E = gp.barrier_energy(x, ctx, prm, x_rest=XR)
    assert E.shape == (b.S,)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device=X.device)
    (E * w).sum().backward()
    scene = torch.repeat_interleave(torch.arange(b.S, device=X.device),
                                    torch.tensor(np.diff(b.vert_off), device=X.device).long())
    assert torch.equal(x.grad, w[scene].unsqueeze(1) * res["g"])
    assert torch.equal(E.detach(), res["E"])
    ctx.close()
