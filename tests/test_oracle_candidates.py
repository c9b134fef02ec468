"""Pins of the oracle's brute-force contact candidates.

* hand-built cases: a point over a triangle of another object just inside
  and just outside dhat (box test, inclusive), same-object and shared-vertex
  exclusions, an edge pair once with i < j;
* the scene generator's uniform-grid broad phase (an independent grid
  implementation) produces the same set on small seeded scenes.
"""
import numpy as np

import oracle
import scenes


def _set(t):
    return set(map(tuple, np.asarray(t).reshape(-1, 4).tolist()))


def test_hand_built():
    # triangle (0,1,2) in z = 0 of object 0; point 3 of object 1 above it
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 0.1], [0.2, 0.2, 0.1]], float)
    tris = np.array([[0, 1, 2]], np.int32)
    edges = np.zeros((0, 2), np.int32)
    vobj = np.array([0, 0, 0, 1, 0], np.int32)
    c = oracle.candidates(x, vobj, tris, edges, 0.1)        # box gap 0.1 == dhat: inclusive
    assert _set(c) == {(-4, 0, 1, 2)}                        # vertex 4 is of the same object
    assert len(oracle.candidates(x, vobj, tris, edges, 0.0999)) == 0
    # edges: (0,1) object 0 and (3,4) object 1 crossing above it; (1,2) shares nothing with (3,4)
    x = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0.5, -0.5, 0.05], [0.5, 0.5, 0.05]], float)
    edges = np.array([[0, 1], [1, 2], [3, 4], [0, 3]], np.int32)
    vobj = np.array([0, 0, 0, 1, 1], np.int32)
    c = oracle.candidates(x, vobj, np.zeros((0, 3), np.int32), edges, 0.1)
    # (0,1)-(3,4) overlap; (1,2)-(3,4): x-range [1,1] vs [0.5,0.5] is 0.5 apart -> no;
    # (0,3) is of mixed objects: its object is that of vertex 0; it shares vertex 3 with (3,4)
    assert _set(c) == {(0, 1, 3, 4)}


def test_matches_the_grid_generator():
    for seed, n, dhat in ((3, 6, 0.15), (1, 12, 0.05), (7, 9, 0.3)):
        s = scenes.two_sheets(n=n, dhat=dhat, kappa=10.0, seed=seed, offset=0.5, jitter=0.3)
        ref = oracle.candidates(s.x, s.vobj, s.tris, s.edges, s.dhat)
        assert len(ref) > 0
        assert _set(ref) == _set(s.tuples)
        assert len(ref) == len(s.tuples)
