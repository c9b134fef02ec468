"""Pins of the oracle's tuple encodings and degenerate primitives.

* The paper's close-to-parallel point-edge and point-point encodings
  (Sec. 7.2, "Data structures": second entry negative) name one boundary
  sub-problem of Eq. 5 on two edges.  Where the edge-edge candidate on the
  same two edges reduces to that sub-problem (its constrained minimum is that
  point against that segment, or that pair of endpoints), the encoded tuple
  must give the candidate's energy, gradient and proxy Hessian exactly, with
  the mollifier (Eq. 25) decided from the two edges in both: a special case
  reducing to the already pinned edge-edge evaluation.
* Malformed sign patterns are rejected.
* Degenerate primitives: a triangle of zero area and an edge of zero length
  still have a constrained distance (Eq. 4 / Eq. 5), the smallest over the
  remaining boundary sub-problems, checked by dense sampling of the
  primitive; the result is finite and matches it.
"""
import numpy as np
import pytest

import oracle

DH = 1e-3


def _p(**kw):
    base = dict(dhat=DH, kappa=1e4)
    base.update(kw)
    return oracle.params(**base)


def _neg(i):
    return -(i + 1)


def _same(a, b):
    assert a["subtype"] == b["subtype"] and a["mollified"] == b["mollified"]
    assert a["E"] == b["E"]
    assert np.array_equal(a["grad"], b["grad"])
    assert np.array_equal(a["hess"], b["hess"])


def _edges_pe(h, tilt):
    # edge A = (p, o) leaving p upward; edge B = (e0, e1) below p: the
    # closest points are p and its foot on B's interior
    p = np.array([0.0, 0.0, h])
    o = np.array([-1.0, 0.0, h + tilt])
    e0 = np.array([-0.5, 0.0, 0.0])
    e1 = np.array([0.5, 0.0, 0.0])
    return np.stack([p, o, e0, e1])


def _edges_pp(h, tilt):
    # p beyond e0's end of B: the closest points are p and e0
    p = np.array([-0.3 * DH, 0.0, h])
    o = np.array([-1.0, 0.0, h + tilt])
    e0 = np.array([0.0, 0.0, 0.0])
    e1 = np.array([1.0, 0.0, 0.0])
    return np.stack([p, o, e0, e1])


@pytest.mark.parametrize("tilt", [1e-2 * DH, 0.2])   # mollified, not mollified
def test_parallel_point_edge_encoding_is_the_edge_edge_subproblem(tilt):
    X = _edges_pe(0.5 * DH, tilt)
    ee = oracle.pair_local([0, 1, 2, 3], X, X, _p())
    pe = oracle.pair_local([_neg(0), _neg(1), 2, _neg(3)], X, X, _p())
    assert ee["subtype"] == oracle.PE
    assert ee["mollified"] == (tilt < 0.1)
    _same(ee, pe)
    assert ee["E"] > 0.0


@pytest.mark.parametrize("tilt", [1e-2 * DH, 0.2])
def test_parallel_point_point_encoding_is_the_edge_edge_subproblem(tilt):
    X = _edges_pp(0.5 * DH, tilt)
    ee = oracle.pair_local([0, 1, 2, 3], X, X, _p())
    pp = oracle.pair_local([_neg(0), _neg(1), _neg(2), _neg(3)], X, X, _p())
    assert ee["subtype"] == oracle.PP
    assert ee["mollified"] == (tilt < 0.1)
    _same(ee, pp)
    # the encoded point-edge tuple on the same edges clamps to the same endpoint
    pe = oracle.pair_local([_neg(0), _neg(1), 2, _neg(3)], X, X, _p())
    _same(ee, pe)


def test_parallel_encodings_stencil_and_rejection():
    nv, vid = oracle.stencil([_neg(5), _neg(6), 7, _neg(8)])
    assert nv == 4 and list(vid) == [5, 6, 7, 8]
    nv, vid = oracle.stencil([_neg(5), _neg(6), _neg(7), _neg(0)])
    assert nv == 4 and list(vid) == [5, 6, 7, 0]
    for bad in ([_neg(1), _neg(2), 3, 4], [_neg(1), _neg(2), _neg(3), 4], [-2 ** 31, 1, 2, 3]):
        nv, _ = oracle.stencil(bad)
        assert nv == -1, bad


def _seg_d2(p, a, b, n=4001):
    t = np.linspace(0.0, 1.0, n)[:, None]
    q = a + t * (b - a)
    return float(((q - p) ** 2).sum(1).min())


def test_zero_area_triangle_distance_is_the_edges_minimum():
    rng = np.random.default_rng(4)
    for _ in range(20):
        t0, t1 = rng.normal(size=3) * DH, rng.normal(size=3) * DH
        t2 = t0 + rng.uniform(0.2, 0.8) * (t1 - t0)          # collinear: zero area
        p = 0.5 * (t0 + t1) + rng.normal(size=3) * 0.3 * DH
        X = np.stack([p, t0, t1, t2])
        r = oracle.pair_local([_neg(0), 1, 2, 3], X, X, _p(dhat=10 * DH))
        ref = min(_seg_d2(p, t0, t1), _seg_d2(p, t1, t2), _seg_d2(p, t2, t0))
        assert np.isfinite(r["d2"]) and r["d2"] == pytest.approx(ref, rel=1e-5)
        assert np.isfinite(r["E"]) and np.isfinite(r["grad"]).all() and np.isfinite(r["hess"]).all()


def test_zero_length_edge_distance_is_point_against_segment():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a0 = rng.normal(size=3) * DH
        b0, b1 = rng.normal(size=3) * DH, rng.normal(size=3) * DH
        X = np.stack([a0, a0.copy(), b0, b1])                 # edge a has zero length
        r = oracle.pair_local([0, 1, 2, 3], X, X, _p(dhat=10 * DH))
        assert np.isfinite(r["d2"]) and r["d2"] == pytest.approx(_seg_d2(a0, b0, b1), rel=1e-5)
        assert not r["mollified"]                              # eps_x = 0 at rest: c < eps_x never holds
        assert np.isfinite(r["E"]) and np.isfinite(r["grad"]).all() and np.isfinite(r["hess"]).all()
