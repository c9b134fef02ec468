"""Additive CCD on the GPU (gipc_accd) against the oracle's orc_accd.

* straight approach along the contact normal (point-triangle, point-edge,
  point-point, crossing edges and the close-to-parallel encodings): the
  closed form (1 - s) h / v, the oracle's value, in two trial steps;
* a dense tiny scene (large dhat: every tuple kind) moved by a seeded
  random displacement with an approach of the upper sheet, and the same
  with the close-to-parallel encodings: every tuple's time against the
  oracle to 1e-9 relative, the step (smallest time) and the counts;
* no relative motion (a common translation) gives tc; a pair at distance 0
  gives 0 and is counted; max_iter caps a search and is counted, with the
  time accumulated so far (as the oracle);
* the ten-sheet candidate list (51M tuples) moved toward contact: sampled
  tuples against the oracle, the step against the smallest sampled time
  and the whole-list minimum;
* without the per-tuple output the same step;
* malformed tuples and bad arguments are errors.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import scenes  # noqa: E402

S = 0.1
REL = 1e-9


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09400_amd as gp
    torch.cuda.set_device(0)
    return gp


@pytest.fixture(scope="module")
def ctx(gp):
    c = gp.Context()
    yield c
    c.close()


def _dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _neg(i):
    return -(i + 1)


def _run(gp, ctx, x, d, t, tc=1.0, max_iter=1_000_000):
    toi, info = gp.accd(ctx, _dev(x), _dev(d), _dev(np.asarray(t, np.int32).reshape(-1, 4), torch.int32), s=S,
                        tc=tc, max_iter=max_iter)
    return toi.cpu().numpy(), info


def _check(gpu, ref):
    den = np.maximum(np.abs(ref), 1e-300)
    err = np.abs(gpu - ref) / den
    bad = np.flatnonzero(err > REL)
    assert bad.size == 0, f"{bad.size} of {ref.size} tuples differ; first {bad[:5]}: {gpu[bad[:5]]} vs {ref[bad[:5]]}"


@pytest.mark.parametrize("kind", ["pt", "pe", "pp", "ee", "pe_par", "pp_par"])
def test_normal_approach(gp, ctx, kind):
    h, v = 0.3, 2.5
    if kind == "pt":
        X = [[0.2, 0.3, h], [0, 0, 0], [1, 0, 0], [0, 1, 0]]
        P = [[0, 0, -v], [0, 0, 0], [0, 0, 0], [0, 0, 0]]
        t = [_neg(0), 1, 2, 3]
    elif kind == "pe":
        X = [[0.4, 0.0, h], [0, 0, 0], [1, 0, 0], [5, 5, 5]]
        P = [[0, 0, -v], [0, 0, 0], [0, 0, 0], [0, 0, 0]]
        t = [_neg(0), 1, 2, -1]
    elif kind == "pp":
        X = [[0.0, 0.0, h], [0, 0, 0], [5, 5, 5], [6, 6, 6]]
        P = [[0, 0, -v / 2], [0, 0, v / 2], [0, 0, 0], [0, 0, 0]]
        t = [_neg(0), 1, -1, -1]
    elif kind == "ee":
        X = [[0.5, -0.5, h], [0.5, 0.5, h], [0, 0, 0], [1, 0, 0]]
        P = [[0, 0, -v], [0, 0, -v], [0, 0, 0], [0, 0, 0]]
        t = [0, 1, 2, 3]
    elif kind == "pe_par":  # point 0 of edge (0, 1) against edge (2, 3)
        X = [[0.4, 0.0, h], [1.4, 0.0, h], [0, 0, 0], [1, 0, 0]]
        P = [[0, 0, -v], [0, 0, -v], [0, 0, 0], [0, 0, 0]]
        t = [_neg(0), _neg(1), 2, _neg(3)]
    else:  # point 0 of edge (0, 1) against point 2 of edge (2, 3)
        X = [[0.0, 0.0, h], [-1.0, 0.0, h], [0, 0, 0], [1, 0, 0]]
        P = [[0, 0, -v], [0, 0, -v], [0, 0, 0], [0, 0, 0]]
        t = [_neg(0), _neg(1), _neg(2), _neg(3)]
    X, P = np.array(X, float), np.array(P, float)
    ref, it = oracle.accd(t, X, P, s=S, tc=1e9)
    assert ref == pytest.approx((1 - S) * h / v, rel=1e-12)
    toi, info = _run(gp, ctx, X, P, t, tc=1e9)
    assert toi[0] == pytest.approx(ref, rel=1e-12)
    assert info["step"] == toi[0]
    assert info["max_steps"] == it == 2
    assert info["n_capped"] == 0 and info["n_touching"] == 0


def _moving_scene(seed):
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=seed, offset=0.5, jitter=0.3)
    rng = np.random.default_rng(100 + seed)
    d = rng.normal(size=s.x.shape) * 0.05
    upper = s.x[:, 2] > 1e-12
    d[upper, 2] -= 0.12  # the upper sheet approaches
    return s, d, s.tuples


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_dense_scene_against_oracle(gp, ctx, seed):
    s, d, t = _moving_scene(seed)
    ref, capped = oracle.accd_scene(s.x, d, t, s=S, tc=1.0)
    toi, info = _run(gp, ctx, s.x, d, t)
    print(f"accd seed={seed} P={len(t)} step={info['step']:.6e} below tc: {(ref < 1.0).sum()} "
          f"max_steps={info['max_steps']}", flush=True)
    assert len(t) > 100 and (ref < 1.0).sum() > 10
    _check(toi, ref)
    assert info["step"] == pytest.approx(ref.min(), rel=REL)
    assert info["n_capped"] == capped == 0
    assert info["n_touching"] == 0
    # without the per-tuple output: the same step
    none, info2 = gp.accd(ctx, _dev(s.x), _dev(d), _dev(t, torch.int32), s=S, tc=1.0, per_tuple=False)
    assert none is None and info2["step"] == info["step"]


def test_encoded_tuples_against_oracle(gp, ctx):
    """Point-edge / point-point tuples in both encodings (plain and cut from
    close-to-parallel edge pairs) on random positions and displacements."""
    rng = np.random.default_rng(11)
    V = 400
    x = rng.normal(size=(V, 3))
    d = rng.normal(size=(V, 3))
    tup = []
    for _ in range(2000):
        a, b, c, e = (int(i) for i in rng.choice(V, 4, replace=False))
        k = rng.integers(0, 6)
        if k == 0:
            tup.append([a, b, c, e])
        elif k == 1:
            tup.append([_neg(a), b, c, e])
        elif k == 2:
            tup.append([_neg(a), b, c, -1])
        elif k == 3:
            tup.append([_neg(a), b, -1, -1])
        elif k == 4:
            tup.append([_neg(a), _neg(b), c, _neg(e)])
        else:
            tup.append([_neg(a), _neg(b), _neg(c), _neg(e)])
    tup = np.array(tup, np.int32)
    ref, capped = oracle.accd_scene(x, d, tup, s=S, tc=1.0)
    toi, info = _run(gp, ctx, x, d, tup)
    _check(toi, ref)
    assert info["step"] == pytest.approx(ref.min(), rel=REL)
    assert info["n_capped"] == capped


def test_translation_touching_and_cap(gp, ctx):
    x = np.array([[0.2, 0.3, 0.5], [0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.3, 0.0]], float)
    d = np.tile([0.3, -0.2, 0.7], (5, 1))
    # a common translation: no relative motion, tc
    toi, info = _run(gp, ctx, x, d, [[_neg(0), 1, 2, 3]], tc=0.75)
    assert toi[0] == 0.75 and info["step"] == 0.75 and info["max_steps"] == 0
    # vertex 4 lies in the triangle: distance 0 gives 0 and is counted
    d2 = np.zeros_like(x)
    d2[0, 2] = -1.0
    toi, info = _run(gp, ctx, x, d2, [[_neg(0), 1, 2, 3], [_neg(4), 1, 2, 3]])
    assert toi[1] == 0.0 and info["n_touching"] == 1 and info["step"] == 0.0
    assert toi[0] == pytest.approx(0.9 * 0.5, rel=1e-12)
    # a cap of one trial step: the time accumulated so far, as the oracle
    d3 = np.zeros_like(x)
    d3[0, 2] = -0.4
    ref, it = oracle.accd([_neg(0), 1, 2, 3], x[:4], d3[:4], s=S, tc=10.0, max_iter=1)
    toi, info = _run(gp, ctx, x, d3, [[_neg(0), 1, 2, 3]], tc=10.0, max_iter=1)
    assert it == -1 and info["n_capped"] == 1 and info["max_steps"] == 1
    assert toi[0] == pytest.approx(ref, rel=1e-12)


def test_empty_list(gp, ctx):
    toi, info = _run(gp, ctx, np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((0, 4), np.int32), tc=0.5)
    assert toi.size == 0 and info["step"] == 0.5


@pytest.mark.parametrize("bad", [[0, 1, 2, 10 ** 6], [-1, 1, -1, 3], [5, 5, 1, 2]])
def test_malformed_tuple_is_an_index_error(gp, ctx, bad):
    x = np.random.default_rng(0).normal(size=(8, 3))
    with pytest.raises(gp.GipcError) as e:
        _run(gp, ctx, x, x, [[_neg(0), 1, 2, 3], bad])
    assert e.value.status == gp.ERR_INDEX


def test_argument_errors(gp, ctx):
    x = _dev(np.zeros((4, 3)))
    t = _dev(np.array([[_neg(0), 1, 2, 3]], np.int32), torch.int32)
    for kw in (dict(s=0.0), dict(s=1.0), dict(tc=-1.0), dict(tc=float("inf")), dict(max_iter=0)):
        with pytest.raises(gp.GipcError) as e:
            gp.accd(ctx, x, x, t, **kw)
        assert e.value.status == gp.ERR_INVALID_ARG


def test_ten_sheets_sampled(gp, ctx):
    s = scenes.stacked_sheets(n_sheets=10, n=256, seed=2, with_pairs=False)
    x = _dev(s.x)
    vobj = _dev(s.vobj, torch.int32)
    tris = _dev(s.tris, torch.int32)
    edges = _dev(s.edges, torch.int32)
    c2 = gp.Context()
    tup = gp.candidates(c2, x, vobj, tris, edges, s.dhat)
    c2.close()
    rng = np.random.default_rng(21)
    disp = rng.normal(size=s.x.shape) * 0.3 * s.dhat
    disp[:, 2] -= 0.4 * s.dhat * (s.x[:, 2] / max(s.x[:, 2].max(), 1e-30))  # the stack settles
    toi, info = gp.accd(ctx, x, _dev(disp), tup, s=S, tc=1.0)
    P = int(tup.shape[0])
    print(f"accd ten sheets: P={P} step={info['step']:.6e} max_steps={info['max_steps']} "
          f"capped={info['n_capped']}", flush=True)
    assert P > 50_000_000
    sel = np.sort(rng.choice(P, 200_000, replace=False))
    t_h = tup[torch.tensor(sel, device="cuda")].cpu().numpy()
    ref, capped = oracle.accd_scene(s.x, disp, t_h, s=S, tc=1.0)
    g = toi.cpu().numpy()
    _check(g[sel], ref)
    assert info["step"] == g.min()
    assert info["step"] <= ref.min()
    assert info["n_capped"] == 0 and capped == 0
    _, info2 = gp.accd(ctx, x, _dev(disp), tup, s=S, tc=1.0, per_tuple=False)
    assert info2["step"] == info["step"] and info2["max_steps"] == info["max_steps"]
