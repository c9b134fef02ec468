"""Lagged friction on the GPU (gipc_friction_lag / gipc_friction_eval)
against the oracle's friction (supplement Sec. 5, the sliding basis and
2x2 projection written literally), on the same seeded scenes.

* build and lag at x^n, evaluate at x = x^n + a seeded motion, in the
  static (|u| < eps_v dt) and sliding regimes: energy and gradient within
  1e-9 relative, and the BSR blocks of barrier (at x^n) + friction (at x)
  within 1e-9 of the largest entry against the oracle's assembly of both
  local Hessians;
* FP32 blocks: friction added to the FP32 matrix within 1e-5 relative
  Frobenius of the FP64 sum;
* a batch (per-scene dhat, kappa): per-scene friction energies;
* ten sheets, 256 x 256: energy, gradient and 40 sampled rows;
* no motion: D = mu lambda eps_v dt / 3 per pair and zero gradient;
* errors: eval without lag, lag after a rebuild, bad parameters.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402

TOL = 1e-9
MU, EPS_V, DT = 0.3, 1e-2, 1e-2


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


def _blocks(A):
    rp = A.row_ptr().cpu().numpy()
    ci = A.col_idx().cpu().numpy()
    v = A.val[:, :A.nnzb].double().cpu().numpy().T.reshape(-1, 3, 3)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return {(int(r), int(c)): B for r, c, B in zip(rows, ci, v)}


def _run(gp, s, x, diag, dtype=0):
    dev = torch.device("cuda", 0)
    pg = gp.params(dhat=s.dhat, kappa=s.kappa)
    Xn = torch.tensor(s.x, device=dev)
    XR = torch.tensor(s.x_rest, device=dev)
    X = torch.tensor(x, device=dev)
    T = torch.tensor(np.asarray(s.tuples, np.int32).reshape(-1, 4), device=dev)
    D = torch.tensor(diag, device=dev)
    ctx = gp.Context()
    gp.pairs_build(ctx, Xn, T, pg, x_rest=XR)
    gp.friction_lag(ctx, Xn, pg, MU, EPS_V, DT, x_rest=XR)
    A = gp.BsrMatrix(ctx, dtype=dtype)
    # the barrier part at the build positions (its pair types were decided
    # there), the friction part at the moved positions
    gp.eval_assemble(ctx, Xn, pg, A, diag=D, x_rest=XR)
    E, g = gp.friction_eval(ctx, X, pg, A)
    return dict(ctx=ctx, A=A, E=E.item(), grad=g.cpu().numpy(), pg=pg, X=X, Xn=Xn, XR=XR)


def _oracle(s, x, diag):
    po = oracle.params(dhat=s.dhat, kappa=s.kappa)
    fo = oracle.fparams(MU, EPS_V, DT)
    fr = oracle.friction_scene(s.x, x, s.tuples, po, fo, x_rest=s.x_rest, per_pair=True)
    bar = oracle.eval_scene(s.x, s.tuples, po, x_rest=s.x_rest, per_pair=True)
    rows, cols, vals = oracle.assemble(s.x.shape[0], s.tuples, bar["pairH"] + fr["pairH"], diag)
    return fr, {(int(r), int(c)): B for r, c, B in zip(rows, cols, vals)}


def _motion(s, regime, seed):
    amp = 0.3 * EPS_V * DT if regime == "static" else 30 * EPS_V * DT
    amp = min(amp, 0.05 * s.dhat)
    return s.x + np.random.default_rng(seed).normal(scale=amp, size=s.x.shape)


@pytest.mark.parametrize("which", ["tiny", "sheets16"])
@pytest.mark.parametrize("regime", ["static", "sliding"])
def test_friction_against_the_oracle(gp, which, regime):
    if which == "tiny":
        s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    else:
        s = scenes.two_sheets(n=16, seed=1)
    x = _motion(s, regime, 11)
    diag = np.full(s.V, 10.0)
    g = _run(gp, s, x, diag)
    fr, ob = _oracle(s, x, diag)
    assert g["E"] == pytest.approx(fr["E"], rel=TOL)
    assert np.abs(g["grad"] - fr["grad"]).max() <= TOL * np.abs(fr["grad"]).max()
    gb = _blocks(g["A"])
    hs = max(np.abs(B).max() for B in ob.values())
    worst = max(np.abs(gb.get(k, 0.0) - ob.get(k, 0.0)).max() for k in set(gb) | set(ob))
    assert worst <= TOL * hs, worst / hs
    g["ctx"].close()


def test_fp32_blocks(gp):
    s = scenes.two_sheets(n=16, seed=1)
    x = _motion(s, "sliding", 12)
    diag = np.full(s.V, 10.0)
    g64 = _run(gp, s, x, diag, dtype=0)
    g32 = _run(gp, s, x, diag, dtype=1)
    n = g64["A"].nnzb
    a64 = g64["A"].val[:, :n].T.reshape(-1, 9)
    a32 = g32["A"].val[:, :n].double().T.reshape(-1, 9)
    fro = torch.linalg.norm(a32 - a64, dim=1) / torch.linalg.norm(a64, dim=1).clamp_min(1e-300)
    assert float(fro.max()) <= 1e-5
    g64["ctx"].close(); g32["ctx"].close()


def test_no_motion(gp):
    s = scenes.two_sheets(n=16, seed=1)
    g = _run(gp, s, s.x, np.full(s.V, 10.0))
    fr, _ = _oracle(s, s.x, np.full(s.V, 10.0))
    assert np.abs(g["grad"]).max() <= 1e-12 * max(np.abs(fr["grad"]).max(), 1.0)
    assert g["E"] == pytest.approx(fr["E"], rel=TOL)
    g["ctx"].close()


def test_batch_per_scene_energies(gp):
    b = scenes.batch_two_sheets(S=4, r_lo=6, r_hi=16, dhat_lo=1e-3, dhat_hi=2e-1, seed_base=950)
    dev = torch.device("cuda", 0)
    x = b.x + np.random.default_rng(3).normal(scale=1e-5, size=b.x.shape)
    Xn, XR, T, X = (torch.tensor(a, device=dev) for a in (b.x, b.x_rest, b.tuples, x))
    prm = gp.params(batch=gp.Batch(b.vert_off, b.dhat, b.kappa))
    ctx = gp.Context()
    gp.pairs_build(ctx, Xn, T, prm, x_rest=XR)
    gp.friction_lag(ctx, Xn, prm, MU, EPS_V, DT, x_rest=XR)
    E, g = gp.friction_eval(ctx, X, prm)
    E = E.cpu().numpy()
    fo = oracle.fparams(MU, EPS_V, DT)
    for si, sc in enumerate(b.scenes):
        v0, v1 = int(b.vert_off[si]), int(b.vert_off[si + 1])
        po = oracle.params(dhat=sc.dhat, kappa=sc.kappa)
        ref = oracle.friction_scene(b.x[v0:v1], x[v0:v1], sc.tuples, po, fo, x_rest=b.x_rest[v0:v1])
        assert E[si] == pytest.approx(ref["E"], rel=TOL)
        gs = g[v0:v1].cpu().numpy()
        assert np.abs(gs - ref["grad"]).max() <= TOL * max(np.abs(ref["grad"]).max(), 1e-300)
    ctx.close()


def test_full_scale(gp):
    s = scenes.stacked_sheets(n_sheets=10, n=256, seed=2)
    x = _motion(s, "sliding", 13)
    g = _run(gp, s, x, s.diag)
    po = oracle.params(dhat=s.dhat, kappa=s.kappa)
    fo = oracle.fparams(MU, EPS_V, DT)
    fr = oracle.friction_scene(s.x, x, s.tuples, po, fo, x_rest=s.x_rest)
    assert g["E"] == pytest.approx(fr["E"], rel=TOL)
    assert np.abs(g["grad"] - fr["grad"]).max() <= TOL * np.abs(fr["grad"]).max()
    rows = np.random.default_rng(5).choice(s.V, 40, replace=False)
    kind, st = scenes.decode_tuples(s.tuples)
    sub = s.tuples[np.isin(st, rows).any(1)]
    frs = oracle.friction_scene(s.x, x, sub, po, fo, x_rest=s.x_rest, per_pair=True)
    bar = oracle.eval_scene(s.x, sub, po, x_rest=s.x_rest, per_pair=True)
    r_, c_, v_ = oracle.assemble(s.V, sub, bar["pairH"] + frs["pairH"], s.diag)
    A = g["A"]
    rp = A.row_ptr().cpu().numpy()
    ci_all = A.col_idx()
    for r in rows:
        lo, hi = int(rp[r]), int(rp[r + 1])
        ci = ci_all[lo:hi].cpu().numpy()
        vals = A.val[:, lo:hi].cpu().numpy().T.reshape(-1, 3, 3)
        gb = {int(c): B for c, B in zip(ci, vals)}
        sel = r_ == r
        ob = {int(c): B for c, B in zip(c_[sel], v_[sel])}
        hs = max(np.abs(B).max() for B in ob.values())
        for c in set(gb) | set(ob):
            assert np.abs(gb.get(c, 0.0) - ob.get(c, 0.0)).max() <= TOL * hs, (r, c)
    g["ctx"].close()


def test_errors(gp):
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    dev = torch.device("cuda", 0)
    pg = gp.params(dhat=s.dhat, kappa=s.kappa)
    Xn = torch.tensor(s.x, device=dev)
    T = torch.tensor(s.tuples, device=dev)
    ctx = gp.Context()
    gp.pairs_build(ctx, Xn, T, pg)
    with pytest.raises(gp.GipcError) as ei:
        gp.friction_eval(ctx, Xn, pg)
    assert ei.value.status == gp.ERR_STATE
    for bad in ((-1.0, EPS_V, DT), (MU, 0.0, DT), (MU, EPS_V, -1.0), (MU, float("nan"), DT)):
        with pytest.raises(gp.GipcError) as ei:
            gp.friction_lag(ctx, Xn, pg, *bad)
        assert ei.value.status == gp.ERR_INVALID_ARG
    gp.friction_lag(ctx, Xn, pg, MU, EPS_V, DT)
    gp.friction_eval(ctx, Xn, pg)
    gp.pairs_build(ctx, Xn, T, pg)          # a rebuild drops the lag
    with pytest.raises(gp.GipcError) as ei:
        gp.friction_eval(ctx, Xn, pg)
    assert ei.value.status == gp.ERR_STATE
    ctx.close()
