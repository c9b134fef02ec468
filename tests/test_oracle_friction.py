"""Pins of the oracle's lagged friction (supplement Sec. 5).

* f0, f1, f1': f0' = f1 and f1' by sympy on both branches, f0(eps h) = eps h,
  f1(0) = 0, continuity at eps h.
* gradient against central differences of D, in both regimes of |u|;
* Hessian against central differences of the gradient (the 2x2 block is
  PSD analytically, so the projection is inactive), away from |u| = eps h;
* the normal force lambda against the barrier gradient at the lagged
  positions (non-mollified pairs: |grad_0 . n| = lambda |c_0|);
* no sliding (x = x^n): D = mu lambda eps h / 3, zero gradient, Hessian
  mu lambda (2 / (eps h)) (c c^T) (x) (I - n n^T) built here from n and c;
* |u| = |(I - n n^T) sum_i c_i (x_i - x_i^n)| for any motion (the sliding
  does not depend on the basis chosen in the tangent plane), a rigid
  translation does not slide, a normal motion of the point does not slide;
* pairs inactive at x^n give nothing; the scene sum equals the pair calls.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
import scenes
from test_oracle_pair import CASES, prm

FP = dict(mu=0.3, eps_v=1e-2, dt=1e-2)
S = FP["eps_v"] * FP["dt"]


def fpr():
    return oracle.fparams(**FP)


def test_transition_functions():
    y, s = sp.symbols("y s", positive=True)
    f1 = -y ** 2 / s ** 2 + 2 * y / s
    f0 = -y ** 3 / (3 * s ** 2) + y ** 2 / s + s / 3
    assert sp.simplify(sp.diff(f0, y) - f1) == 0
    for yy in (0.0, 0.3 * S, 0.999 * S, S, 2 * S):
        a0, a1, a2 = oracle.friction_f(yy, FP["eps_v"], FP["dt"])
        if yy < S:
            assert a0 == pytest.approx(float(f0.subs({y: yy, s: S})), rel=1e-14, abs=1e-300)
            assert a1 == pytest.approx(float(f1.subs({y: yy, s: S})), rel=1e-14, abs=1e-300)
            assert a2 == pytest.approx(float(sp.diff(f1, y).subs({y: yy, s: S})), rel=1e-14, abs=1e-11 * 2 / S)
        else:
            assert (a0, a1, a2) == (yy, 1.0, 0.0)
    assert oracle.friction_f(0.0, FP["eps_v"], FP["dt"])[1] == 0.0
    lo = oracle.friction_f(S * (1 - 1e-12), FP["eps_v"], FP["dt"])
    hi = oracle.friction_f(S, FP["eps_v"], FP["dt"])
    assert lo[0] == pytest.approx(hi[0], rel=1e-10) and lo[1] == pytest.approx(hi[1], rel=1e-10)


def _slide(rng, X, scale):
    return X + rng.normal(scale=scale, size=X.shape)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("regime", ["static", "sliding"])
@pytest.mark.parametrize("seed", range(3))
def test_derivatives(name, regime, seed):
    rng = np.random.default_rng(300 + seed)
    t, Xn, Xr = CASES[name](rng)
    P = prm()
    amp = 0.2 * S if regime == "static" else 20 * S
    X = _slide(rng, Xn, amp)
    out = oracle.friction_pair(t, Xn, X, Xr, P, fpr())
    assert out["lam"] > 0
    y = np.linalg.norm(out["u"])
    if abs(y - S) < 1e-3 * S:
        pytest.skip("at the kink")
    g, H = out["grad"], out["hess"]
    h = 1e-4 * amp
    for _ in range(6):
        d = rng.normal(size=12)
        d /= np.linalg.norm(d)
        Dp = oracle.friction_pair(t, Xn, X + h * d.reshape(4, 3), Xr, P, fpr())
        Dm = oracle.friction_pair(t, Xn, X - h * d.reshape(4, 3), Xr, P, fpr())
        fd = (Dp["D"] - Dm["D"]) / (2 * h)
        assert g @ d == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.linalg.norm(g) + 1e-300)
        hd = (Dp["grad"] - Dm["grad"]) / (2 * h)
        assert np.abs(H @ d - hd).max() <= 1e-5 * np.abs(H).max() + 1e-300


@pytest.mark.parametrize("name", ["pt_interior", "pt_edge", "pt_vertex", "ee_cross", "ee_endpoint"])
def test_normal_force_is_the_barrier_force(name):
    rng = np.random.default_rng(5)
    t, Xn, Xr = CASES[name](rng)
    P = prm()
    bar = oracle.pair_local(t, Xn, Xr, P)
    assert not bar["mollified"]
    fr = oracle.friction_pair(t, Xn, Xn, Xr, P, fpr())
    g0 = bar["grad"][0:3]
    assert abs(g0 @ fr["normal"]) == pytest.approx(fr["lam"] * abs(fr["coef"][0]), rel=1e-10)


@pytest.mark.parametrize("name", list(CASES))
def test_no_sliding_and_invariances(name):
    rng = np.random.default_rng(9)
    t, Xn, Xr = CASES[name](rng)
    P = prm()
    out = oracle.friction_pair(t, Xn, Xn, Xr, P, fpr())
    lam, n, c = out["lam"], out["normal"], out["coef"]
    ml = FP["mu"] * lam
    assert out["D"] == pytest.approx(ml * S / 3, rel=1e-14)
    assert not out["grad"].any()
    Pi = np.eye(3) - np.outer(n, n)
    ref = ml * (2.0 / S) * np.kron(np.outer(c, c), Pi)
    assert np.abs(out["hess"] - ref).max() <= 1e-12 * np.abs(ref).max()
    # sliding magnitude from the tangent projector, for any motion
    for _ in range(4):
        X = _slide(rng, Xn, 5 * S)
        o2 = oracle.friction_pair(t, Xn, X, Xr, P, fpr())
        tvec = Pi @ np.einsum("i,ij->j", c, X - Xn)
        assert np.linalg.norm(o2["u"]) == pytest.approx(np.linalg.norm(tvec), rel=1e-12)
    # a rigid translation does not slide
    o3 = oracle.friction_pair(t, Xn, Xn + rng.normal(size=3), Xr, P, fpr())
    assert np.linalg.norm(o3["u"]) <= 1e-12 and o3["D"] == pytest.approx(out["D"], rel=1e-12)
    # moving the slot-0 vertex along the normal does not slide
    X4 = Xn.copy()
    X4[0] += 0.37 * S * n
    assert np.linalg.norm(oracle.friction_pair(t, Xn, X4, Xr, P, fpr())["u"]) <= 1e-12 * S


def test_inactive_pair_and_scene_sum():
    rng = np.random.default_rng(1)
    t, Xn, Xr = CASES["pt_interior"](rng)
    far = Xn.copy()
    far[0] += 10.0 * np.array([0, 0, 1.0])
    o = oracle.friction_pair(t, far, far, Xr, prm(), fpr())
    assert o["D"] == 0 and not o["grad"].any() and not o["hess"].any() and o["lam"] == 0
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    P = oracle.params(dhat=s.dhat, kappa=s.kappa)
    x = s.x + np.random.default_rng(2).normal(scale=1e-3, size=s.x.shape)
    sc = oracle.friction_scene(s.x, x, s.tuples, P, fpr(), x_rest=s.x_rest, per_pair=True)
    tot = 0.0
    for p in range(0, len(s.tuples), max(1, len(s.tuples) // 20)):
        nv, vid = oracle.stencil(s.tuples[p])
        xn = np.zeros((4, 3)); xc = np.zeros((4, 3)); xr = np.zeros((4, 3))
        xn[:nv] = s.x[vid[:nv]]; xc[:nv] = x[vid[:nv]]; xr[:nv] = s.x_rest[vid[:nv]]
        o = oracle.friction_pair(s.tuples[p], xn, xc, xr, P, fpr())
        assert o["D"] == sc["pairE"][p]
        assert np.array_equal(o["grad"], sc["pairG"][p])
    assert sc["E"] == pytest.approx(sc["pairE"].sum(), rel=1e-12)
    with pytest.raises(ValueError):
        oracle.friction_scene(s.x, x, np.array([[0, 1, 2, 10 ** 6]], np.int32), P, fpr())
    del tot
