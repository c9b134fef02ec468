"""Pins of the oracle's additive CCD (the line search's step bound).

* straight approach along the contact normal at constant relative speed v
  from distance h (point toward a triangle's interior, point toward an
  edge, point toward a point, crossing edges): the distance falls at exactly
  l_p, so the first sub-step lands at s h and the second would cross g: the
  method returns (1 - s) h / v, a closed form;
* receding or tangential motion, and no relative motion: no impact before
  t_c, t_c returned;
* a common translation of the whole pair changes nothing;
* random trajectories (all tuple kinds): the result is conservative -- the
  distance stays positive on [0, toi] (dense sampling) and is still at
  least s d0 at toi -- and never exceeds the exact time of impact found by
  bisection on the sampled distance;
* a starting distance of 0 gives 0.
"""
import numpy as np
import pytest

import oracle

S = 0.1


def _neg(i):
    return -(i + 1)


def _d(tuple4, X):
    return np.sqrt(oracle.pair_local(tuple4, X, X, oracle.params(dhat=1e9))["d2"])


@pytest.mark.parametrize("kind", ["pt", "pe", "pp", "ee"])
@pytest.mark.parametrize("h,v", [(1.0, 1.0), (0.3, 2.5), (1e-3, 0.05)])
def test_normal_approach_closed_form(kind, h, v):
    if kind == "pt":
        X = np.array([[0.2, 0.3, h], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
        P = np.array([[0, 0, -v], [0, 0, 0], [0, 0, 0], [0, 0, 0]], float)
        t = [_neg(0), 1, 2, 3]
    elif kind == "pe":
        X = np.array([[0.4, 0.0, h], [0, 0, 0], [1, 0, 0], [0, 0, 0]], float)
        P = np.array([[0, 0, -v], [0, 0, 0], [0, 0, 0], [0, 0, 0]], float)
        t = [_neg(0), 1, 2, -1]
    elif kind == "pp":
        X = np.array([[0.0, 0.0, h], [0, 0, 0], [0, 0, 0], [0, 0, 0]], float)
        P = np.array([[0, 0, -v / 2], [0, 0, v / 2], [0, 0, 0], [0, 0, 0]], float)
        t = [_neg(0), 1, -1, -1]
    else:
        X = np.array([[0.5, -0.5, h], [0.5, 0.5, h], [0, 0, 0], [1, 0, 0]], float)
        P = np.array([[0, 0, -v], [0, 0, -v], [0, 0, 0], [0, 0, 0]], float)
        t = [0, 1, 2, 3]
    toi, it = oracle.accd(t, X, P, s=S, tc=1e9)
    assert toi == pytest.approx((1 - S) * h / v, rel=1e-12)
    assert it == 2


@pytest.mark.parametrize("motion", ["recede", "tangent", "still"])
def test_no_impact_returns_tc(motion):
    X = np.array([[0.2, 0.3, 0.5], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    P = np.zeros((4, 3))
    if motion == "recede":
        P[0] = [0, 0, 0.7]
    elif motion == "tangent":
        P[0] = [0.01, 0.01, 0.0]
    toi, _ = oracle.accd([_neg(0), 1, 2, 3], X, P, s=S, tc=1.0)
    assert toi == 1.0


def test_common_translation_changes_nothing():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(4, 3))
    P = rng.normal(size=(4, 3))
    a, _ = oracle.accd([0, 1, 2, 3], X, P, s=S, tc=1.0)
    b, _ = oracle.accd([0, 1, 2, 3], X, P + rng.normal(size=3), s=S, tc=1.0)
    assert a == pytest.approx(b, rel=1e-12)


def _random_case(rng, kind):
    X = rng.normal(size=(4, 3)) * 0.5
    P = rng.normal(size=(4, 3)) * rng.uniform(0.5, 3.0)
    if rng.uniform() < 0.5:
        # head the first vertex at the last one, through or past it
        P[0] = (X[3 if kind in ("pt", "ee", "pe-par") else 1] - X[0]) * rng.uniform(0.8, 1.5) + rng.normal(size=3) * 0.05
        P[1:] *= 0.1
    if kind == "pt":
        return [_neg(0), 1, 2, 3], X, P
    if kind == "ee":
        return [0, 1, 2, 3], X, P
    if kind == "pe":
        return [_neg(0), 1, 2, -1], X, P
    if kind == "pe-par":
        return [_neg(0), _neg(1), 2, _neg(3)], X, P
    return [_neg(0), 1, -1, -1], X, P


@pytest.mark.parametrize("kind", ["pt", "ee", "pe", "pe-par", "pp"])
def test_conservative_on_random_trajectories(kind):
    rng = np.random.default_rng({"pt": 1, "ee": 2, "pe": 3, "pe-par": 4, "pp": 5}[kind])
    stopped = 0
    for _ in range(60):
        t, X, P = _random_case(rng, kind)
        toi, it = oracle.accd(t, X, P, s=S, tc=1.0)
        d0 = _d(t, X)
        ts = np.linspace(0.0, 1.0, 2001)
        ds = np.array([_d(t, X + tt * P) for tt in ts])
        assert 0.0 <= toi <= 1.0
        assert (ds[ts <= toi] > 0).all()
        assert _d(t, X + toi * P) >= S * d0 * (1 - 1e-12) or toi == 1.0
        # not beyond the first time the sampled distance comes within 1e-9 of 0
        close = np.nonzero(ds < 1e-6 * d0)[0]
        if close.size:
            assert toi <= ts[close[0]]
        stopped += toi < 1.0
    assert stopped >= 1


@pytest.mark.parametrize("th", [0.3, 0.8])
def test_trajectories_through_contact_stop_before_it(th):
    # The point is steered onto a moving triangle's interior at time th (a
    # true collision): the step must end strictly before th, at a
    # configuration no closer than s times the start distance.
    rng = np.random.default_rng(9)
    for _ in range(40):
        X = rng.normal(size=(4, 3)) * 0.5
        P = rng.normal(size=(4, 3))
        bary = rng.dirichlet([2.0, 2.0, 2.0])
        hit = bary @ (X[1:] + th * P[1:])
        P[0] = (hit - X[0]) / th
        t = [_neg(0), 1, 2, 3]
        assert _d(t, X + th * P) < 1e-12
        toi, _ = oracle.accd(t, X, P, s=S, tc=1.0)
        assert 0.0 < toi < th
        d0 = _d(t, X)
        assert _d(t, X + toi * P) >= S * d0 * (1 - 1e-12)


def test_zero_distance_gives_zero():
    X = np.array([[0.2, 0.3, 0.0], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    P = np.array([[0, 0, 1.0], [0, 0, 0], [0, 0, 0], [0, 0, 0]], float)
    toi, _ = oracle.accd([_neg(0), 1, 2, 3], X, P, s=S, tc=1.0)
    assert toi == 0.0
