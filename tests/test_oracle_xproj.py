"""Pins of the oracle's x-space route (the traditional projection of the
3n x 3n proxy Hessian by Jacobi rotations, the baseline the analytic
eigensystems replace).

* The matrix before projection, kappa D^T H D, equals the proxy Hessian
  whenever the projection of the inner Hessian is inactive (inner Hessian
  already PSD), on every case kind: this pins its construction.
* Non-mollified pairs: the proxy Hessian is rank one, lambda g g^T, whose
  projection is max(lambda, 0) g g^T in any basis, so the x-space projection
  equals the analytic one.
* Every pair: the projection P of K is characterised (Moreau decomposition
  on the PSD cone) by P >= 0, P - K >= 0 and P (P - K) = 0, and agrees with
  numpy's eigh-based projection.
"""
import numpy as np
import pytest

import oracle
import scenes
from test_oracle_pair import CASES, prm


def _psd_min(A):
    return np.linalg.eigvalsh(0.5 * (A + A.T)).min()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("filt", [True, False])
@pytest.mark.parametrize("seed", range(3))
def test_xspace_route(name, filt, seed):
    rng = np.random.default_rng(100 + seed)
    t, X, Xr = CASES[name](rng)
    P = prm(filter=filt)
    out = oracle.pair_local(t, X, Xr, P, debug=True)
    K, Px = oracle.pair_xproj(t, X, Xr, P)
    H = out["hess"]
    scale = max(np.abs(K).max(), np.abs(H).max(), 1e-300)
    # construction: no clamping in the inner space -> K is the proxy Hessian
    if np.allclose(out["innerH"], out["innerHp"], rtol=0, atol=1e-13 * np.abs(out["innerH"]).max()):
        assert np.abs(K - H).max() <= 1e-12 * scale
    # Moreau characterisation of the projection
    assert _psd_min(Px) >= -1e-12 * scale
    assert _psd_min(Px - K) >= -1e-12 * scale
    assert np.abs(Px @ (Px - K)).max() <= 1e-11 * scale ** 2
    lam, Q = np.linalg.eigh(0.5 * (K + K.T))
    ref = (Q * np.maximum(lam, 0)) @ Q.T
    assert np.abs(Px - ref).max() <= 1e-11 * scale
    if not out["mollified"]:
        assert np.abs(Px - H).max() <= 1e-12 * scale


def test_mollified_routes_differ_only_when_the_inner_block_is_indefinite():
    # over many nearly parallel configurations both situations occur, and the
    # two routes agree exactly when the inner projection is inactive
    rng = np.random.default_rng(7)
    n_same = n_diff = 0
    for seed in range(40):
        t, X, Xr = CASES["ee_parallel"](np.random.default_rng(seed))
        P = prm(filter=bool(seed % 2))
        out = oracle.pair_local(t, X, Xr, P, debug=True)
        if not out["mollified"]:
            continue
        K, Px = oracle.pair_xproj(t, X, Xr, P)
        H = out["hess"]
        scale = np.abs(H).max()
        inactive = np.allclose(out["innerH"], out["innerHp"], rtol=0, atol=1e-13 * np.abs(out["innerH"]).max())
        if inactive:
            assert np.abs(Px - H).max() <= 1e-12 * scale
            n_same += 1
        elif np.abs(Px - H).max() > 1e-8 * scale:
            n_diff += 1
    del rng
    assert n_diff > 0


def test_scene_list_matches_pair_calls():
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    P = oracle.params(dhat=s.dhat, kappa=s.kappa)
    Pxs = oracle.eval_xproj(s.x, s.tuples, P, x_rest=s.x_rest)
    for p in range(0, len(s.tuples), max(1, len(s.tuples) // 25)):
        nv, vid = oracle.stencil(s.tuples[p])
        xs = np.zeros((4, 3)); xr = np.zeros((4, 3))
        xs[:nv] = s.x[vid[:nv]]; xr[:nv] = s.x_rest[vid[:nv]]
        _, Px = oracle.pair_xproj(s.tuples[p], xs, xr, P)
        assert np.array_equal(Px, Pxs[p])
    with pytest.raises(ValueError):
        oracle.eval_xproj(s.x, np.array([[0, 1, 2, 10 ** 6]], np.int32), P)
