"""Pins of the oracle's assembly, SpMV and PCG, and of scene-level sums.

* Assembly: the supplement's matrix decomposition (Sec. 6, the three-node,
  two-spring example rebuilt with 3x3 blocks): the global matrix is the sum
  of the local matrices placed by the local-to-global map, so the product
  with any vector equals the sum of the local products.  Checked against a
  dense numpy build and against scipy.sparse.
* SpMV against scipy's BSR product.
* Matrix-free mat-vec (sum of local products, no global matrix) against the
  hand-built two-spring product and the dense matrix of a small scene.
* PCG against numpy.linalg.solve; the paper's termination (r.z <= eps
  r0.z0) pinned by r.z recomputed with numpy from the returned solutions:
  met after the reported iterations, not one iteration earlier; a block
  diagonal system (the preconditioner is its inverse) stops after one.
* Scene level: energy and gradient of a list equal the sums of the per-pair
  values; a duplicated tuple counts twice (contact multiplicity); the
  gradient of the whole scene is translation invariant.
"""
import numpy as np
import pytest
import scipy.sparse as sps

import oracle
import scenes


def _dense(V, rows, cols, vals):
    A = np.zeros((3 * V, 3 * V))
    for r, c, B in zip(rows, cols, vals):
        A[3 * r:3 * r + 3, 3 * c:3 * c + 3] += B
    return A


def test_two_spring_decomposition():
    # two point-point "springs" sharing vertex 1: local 6x6 matrices A, B
    rng = np.random.default_rng(0)
    A6 = rng.normal(size=(6, 6)); A6 = A6 + A6.T
    B6 = rng.normal(size=(6, 6)); B6 = B6 + B6.T
    H = np.zeros((2, 12, 12))
    H[0, :6, :6] = A6
    H[1, :6, :6] = B6
    tuples = np.array([[-1, 1, -1, -1], [-2, 2, -1, -1]], np.int32)   # (0,1) and (1,2)
    rows, cols, vals = oracle.assemble(3, tuples, H)
    G = _dense(3, rows, cols, vals)
    ref = np.zeros((9, 9))
    ref[:6, :6] += A6
    ref[3:, 3:] += B6                     # the shared vertex's block is A22 + B11
    assert G == pytest.approx(ref, abs=1e-15)
    c = rng.normal(size=9)
    local = np.zeros(9)
    local[:6] += A6 @ c[:6]
    local[3:] += B6 @ c[3:]
    assert oracle.spmv(3, rows, cols, vals, c) == pytest.approx(local, rel=1e-13)
    # the same product without a global matrix, with a diagonal term
    d = np.array([1.0, 2.0, 3.0])
    assert oracle.matfree(3, tuples, H, c, d) == pytest.approx(local + np.repeat(d, 3) * c, rel=1e-13)


def _tiny_scene():
    s = scenes.two_sheets(n=6, dhat=0.15, kappa=10.0, seed=3, offset=0.5, jitter=0.3)
    prm = oracle.params(dhat=s.dhat, kappa=s.kappa)
    return s, prm


def test_assembly_equals_sum_of_local_matrices():
    s, prm = _tiny_scene()
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest, per_pair=True)
    diag = np.linspace(1.0, 2.0, s.V)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, out["pairH"], diag)
    G = _dense(s.V, rows, cols, vals)
    ref = np.kron(np.diag(diag), np.eye(3))
    for t, H in zip(s.tuples, out["pairH"]):
        nv, vid = oracle.stencil(t)
        for k in range(nv):
            for l in range(nv):
                ref[3 * vid[k]:3 * vid[k] + 3, 3 * vid[l]:3 * vid[l] + 3] += H[3 * k:3 * k + 3, 3 * l:3 * l + 3]
    assert G == pytest.approx(ref, abs=1e-12 * np.abs(ref).max())
    # sorted and duplicate-free
    key = rows.astype(np.int64) * s.V + cols
    assert (np.diff(key) > 0).all()
    # SpMV against scipy
    x = np.random.default_rng(1).normal(size=3 * s.V)
    M = sps.csr_matrix((vals.reshape(-1), (np.repeat(3 * rows, 9) + np.tile(np.repeat(np.arange(3), 3), len(rows)),
                                           np.repeat(3 * cols, 9) + np.tile(np.tile(np.arange(3), 3), len(rows)))),
                       shape=(3 * s.V, 3 * s.V))
    assert oracle.spmv(s.V, rows, cols, vals, x) == pytest.approx(M @ x, rel=1e-12, abs=1e-12 * np.abs(M @ x).max())
    # the assembled proxy Hessian is symmetric PSD, so with diag > 0 it is SPD
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
    assert np.linalg.eigvalsh(G).min() > 0


def test_matfree_equals_dense_product():
    s, prm = _tiny_scene()
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest, per_pair=True)
    diag = np.linspace(1.0, 2.0, s.V)
    ref = np.kron(np.diag(diag), np.eye(3))
    for t, H in zip(s.tuples, out["pairH"]):
        nv, vid = oracle.stencil(t)
        S = np.zeros((3 * nv, 3 * s.V))   # selection matrix of the stencil
        for k in range(nv):
            S[3 * k:3 * k + 3, 3 * vid[k]:3 * vid[k] + 3] = np.eye(3)
        ref += S.T @ H[:3 * nv, :3 * nv] @ S
    rng = np.random.default_rng(5)
    for _ in range(3):
        x = rng.normal(size=3 * s.V)
        y = oracle.matfree(s.V, s.tuples, out["pairH"], x, diag)
        assert np.abs(y - ref @ x).max() <= 1e-12 * np.abs(ref @ x).max()
    # no diagonal term: a zero vector maps to zero, and the map is linear
    x1, x2 = rng.normal(size=(2, 3 * s.V))
    y12 = oracle.matfree(s.V, s.tuples, out["pairH"], 2.0 * x1 - x2)
    y1 = oracle.matfree(s.V, s.tuples, out["pairH"], x1)
    y2 = oracle.matfree(s.V, s.tuples, out["pairH"], x2)
    assert np.abs(y12 - (2.0 * y1 - y2)).max() <= 1e-12 * np.abs(y12).max()
    with pytest.raises(ValueError):
        oracle.matfree(s.V, np.array([[0, 1, 2, 10 ** 6]], np.int32), np.zeros((1, 12, 12)), np.zeros(3 * s.V))


def test_pcg_matches_direct_solve():
    s, prm = _tiny_scene()
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest, per_pair=True)
    diag = np.full(s.V, 10.0)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, out["pairH"], diag)
    b = -out["grad"].reshape(-1)
    x, it, rr = oracle.pcg(s.V, rows, cols, vals, b, rtol=1e-12, maxit=2000)
    ref = np.linalg.solve(_dense(s.V, rows, cols, vals), b)
    assert rr <= 1e-12
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    # x0 = exact solution: zero iterations
    x2, it2, _ = oracle.pcg(s.V, rows, cols, vals, b, x0=ref, rtol=1e-6, maxit=10)
    assert it2 == 0


def _delta(V, A, rows, cols, vals, b, x):
    """r.z at x, z = (block diagonal of A)^-1 r, with numpy"""
    r = b - A @ x
    z = np.zeros_like(r)
    for v in range(V):
        D = A[3 * v:3 * v + 3, 3 * v:3 * v + 3]
        z[3 * v:3 * v + 3] = np.linalg.solve(D, r[3 * v:3 * v + 3])
    return float(r @ z)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_pcg_delta_termination(eps):
    s, prm = _tiny_scene()
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest, per_pair=True)
    diag = np.full(s.V, 10.0)
    rows, cols, vals = oracle.assemble(s.V, s.tuples, out["pairH"], diag)
    A = _dense(s.V, rows, cols, vals)
    b = -out["grad"].reshape(-1)
    d0 = _delta(s.V, A, rows, cols, vals, b, np.zeros_like(b))
    x, it, rr = oracle.pcg(s.V, rows, cols, vals, b, rtol=eps, maxit=500, delta=True)
    assert 0 < it < 500
    assert _delta(s.V, A, rows, cols, vals, b, x) <= eps * d0 * (1 + 1e-9)
    xm, itm, _ = oracle.pcg(s.V, rows, cols, vals, b, rtol=eps, maxit=it - 1, delta=True)
    assert itm == it - 1 and _delta(s.V, A, rows, cols, vals, b, xm) > eps * d0 * (1 - 1e-9)
    assert rr == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b), rel=1e-9)
    # block diagonal system: one iteration to the exact solution
    keep = rows == cols
    xd, itd, rrd = oracle.pcg(s.V, rows[keep], cols[keep], vals[keep], b, rtol=eps, maxit=50, delta=True)
    assert itd == 1 and rrd <= 1e-14


def test_scene_sums_and_multiplicity():
    s, prm = _tiny_scene()
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest, per_pair=True)
    assert out["E"] == pytest.approx(out["pairE"].sum(), rel=1e-14)
    assert np.abs(out["grad"].sum(0)).max() <= 1e-12 * np.abs(out["grad"]).max()
    active = out["subtype"] > 0
    assert active.sum() > 10
    dup = np.concatenate([s.tuples, s.tuples[active][:7]])
    out2 = oracle.eval_scene(s.x, dup, prm, x_rest=s.x_rest, per_pair=True)
    assert out2["E"] == pytest.approx(out["E"] + out["pairE"][active][:7].sum(), rel=1e-13)


def test_out_of_range_index_rejected():
    s, prm = _tiny_scene()
    bad = s.tuples.copy()
    bad[0, 1] = s.V + 5
    with pytest.raises(ValueError):
        oracle.eval_scene(s.x, bad, prm)


def test_c1_scene_sanity():
    s = scenes.two_sheets()
    prm = oracle.params(dhat=s.dhat, kappa=s.kappa)
    out = oracle.eval_scene(s.x, s.tuples, prm, x_rest=s.x_rest)
    assert np.isfinite(out["E"]) and out["E"] > 0
    assert out["n_degenerate"] == 0
    counts = np.bincount(out["subtype"], minlength=8)
    # every sub-type of the method occurs in this scene
    for st in (oracle.PT, oracle.PE, oracle.PP, oracle.EE):
        assert counts[st] > 0
    assert out["mollified"].sum() > 0
    assert np.abs(out["grad"].sum(0)).max() <= 1e-9 * np.abs(out["grad"]).max()
