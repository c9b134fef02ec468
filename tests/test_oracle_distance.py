"""Pins of the oracle's constrained distances (Eq. 4 point-triangle, Eq. 5
edge-edge) against brute force on tiny inputs, and of its eigen-solver
against LAPACK.

* Edge-edge: Eq. 5 is a least-squares problem with box bounds, solved
  exactly by scipy's bounded-variable least squares.
* Point-triangle: Eq. 4 over the simplex, by dense barycentric sampling
  refined with SLSQP, and by non-negative least squares in barycentric form.
* Hand-built cases with a known answer (point over the interior, over an
  edge region, over a vertex region; crossing, parallel and endpoint-closest
  edges) also check the reported sub-type.
"""
import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize, nnls

import oracle

PRM = oracle.params(dhat=10.0, kappa=1.0)   # dhat large: every tiny case is active


def _pt_bruteforce(p, t0, t1, t2):
    e1, e2 = t1 - t0, t2 - t0
    f = lambda b: float(np.sum((t0 + b[0] * e1 + b[1] * e2 - p) ** 2))
    u = np.linspace(0, 1, 121)
    best = None
    for b1 in u:
        for b2 in u[u <= 1 - b1 + 1e-15]:
            v = f((b1, b2))
            if best is None or v < best[0]:
                best = (v, (b1, b2))
    r = minimize(f, best[1], method="SLSQP", bounds=[(0, 1), (0, 1)],
                 constraints=[{"type": "ineq", "fun": lambda b: 1 - b[0] - b[1]}],
                 options={"ftol": 1e-16, "maxiter": 500})
    # exact active-set solve of the same problem in barycentric form:
    # min |sum_i l_i t_i - p|^2, l >= 0, sum l = 1 (equality by heavy weight)
    W = 1e6
    A = np.vstack([np.stack([t0, t1, t2], 1), W * np.ones((1, 3))])
    lam, _ = nnls(A, np.concatenate([p, [W]]))
    lam = lam / lam.sum()
    q = np.stack([t0, t1, t2], 1) @ lam
    return min(best[0], r.fun if r.success else np.inf, float(np.sum((q - p) ** 2)))


def _ee_bruteforce(a0, a1, b0, b1):
    A = np.stack([a1 - a0, -(b1 - b0)], 1)
    r = lsq_linear(A, b0 - a0, bounds=(0, 1), method="bvls", tol=1e-15)
    g1, g2 = r.x
    w = (a0 + g1 * (a1 - a0)) - (b0 + g2 * (b1 - b0))
    return float(w @ w)


def _pair(tuple4, X):
    return oracle.pair_local(np.array(tuple4, np.int32), np.asarray(X, float), prm=PRM)


@pytest.mark.parametrize("seed", range(40))
def test_pt_distance_random(seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(4, 3))
    out = _pair([-1, 1, 2, 3], X)
    bf = _pt_bruteforce(*X)
    assert out["d2"] <= bf * (1 + 1e-12) + 1e-15
    assert out["d2"] == pytest.approx(bf, rel=1e-9, abs=1e-13)


@pytest.mark.parametrize("seed", range(40))
def test_ee_distance_random(seed):
    rng = np.random.default_rng(100 + seed)
    X = rng.normal(size=(4, 3))
    out = _pair([0, 1, 2, 3], X)
    bf = _ee_bruteforce(*X)
    assert out["d2"] == pytest.approx(bf, rel=1e-11, abs=1e-14)


def test_pt_known_cases():
    T = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    # interior: straight above (0.2, 0.3) at height 0.4
    o = _pair([-1, 1, 2, 3], np.vstack([[0.2, 0.3, 0.4], T]))
    assert o["subtype"] == oracle.PT and o["d2"] == pytest.approx(0.16, rel=1e-14)
    # edge region of the hypotenuse: closest point (0.5, 0.5, 0)
    o = _pair([-1, 1, 2, 3], np.vstack([[0.8, 0.8, 0.1], T]))
    assert o["subtype"] == oracle.PE and o["d2"] == pytest.approx(2 * 0.3 ** 2 + 0.01, rel=1e-13)
    # vertex region of t0
    o = _pair([-1, 1, 2, 3], np.vstack([[-0.3, -0.4, 0.0], T]))
    assert o["subtype"] == oracle.PP and o["d2"] == pytest.approx(0.25, rel=1e-14)


def test_ee_known_cases():
    # crossing edges, 0.3 apart in z
    X = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0.3], [0, 1, 0.3]], float)
    o = _pair([0, 1, 2, 3], X)
    assert o["subtype"] == oracle.EE and o["d2"] == pytest.approx(0.09, rel=1e-14)
    # exactly parallel, overlapping: the interior system is singular, the
    # boundary sub-problems give the separation
    X = np.array([[0, 0, 0], [1, 0, 0], [0.25, 0, 0.2], [1.5, 0, 0.2]], float)
    o = _pair([0, 1, 2, 3], X)
    assert o["subtype"] in (oracle.PE, oracle.PP) and o["d2"] == pytest.approx(0.04, rel=1e-14)
    # skew edges whose closest points are two endpoints
    X = np.array([[0, 0, 0], [1, 0, 0], [2, 0.5, 0.0], [3, 1, 0.0]], float)
    o = _pair([0, 1, 2, 3], X)
    assert o["subtype"] == oracle.PP and o["d2"] == pytest.approx(1.0 + 0.25, rel=1e-14)


def test_pe_pp_typed():
    X = np.array([[0.5, 0.2, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0]], float)
    o = _pair([-1, 1, 2, -1], X)
    assert o["subtype"] == oracle.PE and o["d2"] == pytest.approx(0.04, rel=1e-14)
    o = _pair([-1, 1, -1, -1], X)
    assert o["subtype"] == oracle.PP and o["d2"] == pytest.approx(0.29, rel=1e-14)


def test_malformed_tuples_rejected():
    X = np.zeros((4, 3))
    for t in ([-1, -2, 3, 4], [0, 1, -1, 3], [-1, 2, -1, 3], [0, 1, 2, -5]):
        with pytest.raises(ValueError):
            _pair(t, X)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 12])
def test_jacobi_matches_lapack(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        A = rng.normal(size=(n, n))
        A = A + A.T
        lam, vec = oracle.jacobi_eig(A)
        ref = np.linalg.eigvalsh(A)
        assert np.sort(lam) == pytest.approx(ref, rel=1e-12, abs=1e-12 * np.abs(ref).max())
        assert vec @ np.diag(lam) @ vec.T == pytest.approx(A, abs=1e-12 * np.abs(A).max())
        assert vec.T @ vec == pytest.approx(np.eye(n), abs=1e-13)
