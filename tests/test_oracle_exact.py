"""Pins of the oracle's exact-Hessian route (the traditional "construct the
exact local Hessian, then project it numerically" of Table 1).

* the exact Hessian against central finite differences of the oracle's
  gradient (itself pinned against finite differences of the energy), for
  every sub-type and for mollified edge pairs, to 1e-6 relative;
* point-point pairs: exact minus the unfiltered proxy equals the dropped
  term kappa b_d grad^2 d of Eq. 22, with the textbook Hessian of a distance,
  grad^2 d = (I - n n^T) / d on the 3x3 block pattern [[1, -1], [-1, 1]];
* the projection against numpy's eigh (clamping the negative eigenvalues),
  PSD, symmetric, and equal to the input where the input is already PSD;
* the exact Hessian is indefinite on most pairs (b' < 0 times the curvature
  of the distance), so the projection has work to do.
"""
import numpy as np
import pytest

import oracle

DH = 1.0
KAPPA = 3.0


def prm(**kw):
    base = dict(dhat=DH, kappa=KAPPA)
    base.update(kw)
    return oracle.params(**base)


def _neg(i):
    return -(i + 1)


def _configs():
    rng = np.random.default_rng(17)
    out = []
    for _ in range(6):
        # point over a triangle's interior
        t = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float) + rng.normal(size=(3, 3)) * 0.05
        p = np.array([0.3, 0.3, rng.uniform(0.25, 0.85)]) + rng.normal(size=3) * 0.02
        out.append(("pt", [_neg(0), 1, 2, 3], np.vstack([p, t])))
        # point near a triangle edge (point-edge sub-problem) and corner (point-point)
        out.append(("pt-pe", [_neg(0), 1, 2, 3], np.vstack([[0.5, -0.3, rng.uniform(0.2, 0.5)], t])))
        out.append(("pt-pp", [_neg(0), 1, 2, 3], np.vstack([[-0.3, -0.3, rng.uniform(0.1, 0.4)], t])))
        # crossing edges
        a0, a1 = np.array([0.5, -0.5, 0.0]), np.array([0.5, 0.5, 0.0])
        h = rng.uniform(0.25, 0.85)
        X = np.array([a0 + [0, 0, h], a1 + [0, 0, h], [0, 0, 0], [1, 0, 0]]) + rng.normal(size=(4, 3)) * 0.02
        out.append(("ee", [0, 1, 2, 3], X))
        # nearly parallel edges (mollified), interior and endpoint sub-problems
        tilt = rng.uniform(0.005, 0.02)
        X = np.array([[0.1, 0.0, h], [0.9, tilt, h + 0.1 * tilt], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
        out.append(("ee-moll", [0, 1, 2, 3], X))
        Xp = np.array([[0.0, 0.0, 0.4], [-0.8, tilt, 0.4 + tilt], [-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
        out.append(("pe-par", [_neg(0), _neg(1), 2, _neg(3)], Xp))
        # typed point-point
        out.append(("pp", [_neg(0), 1, -1, -1], np.vstack([[0, 0, 0], rng.normal(size=3) / np.sqrt(3) * h])))
    return out


@pytest.mark.parametrize("case", range(42))
def test_exact_hessian_against_finite_differences_of_the_gradient(case):
    name, t, X = _configs()[case]
    pr = prm(epsx_ratio=1.0 if "moll" in name or "par" in name else 1e-3)
    base = oracle.pair_local(t, X, X, pr)
    assert base["subtype"] > 0, name
    H, Hp = oracle.pair_exact(t, X, X, pr)
    assert np.array_equal(H, H.T)
    nv, _ = oracle.stencil(t)
    n = 3 * nv
    h = 1e-6
    F = np.zeros((n, n))
    for j in range(n):
        Xp, Xm = X.copy(), X.copy()
        Xp.reshape(-1)[j] += h
        Xm.reshape(-1)[j] -= h
        gp_ = oracle.pair_local(t, Xp, X, pr)["grad"][:n]
        gm_ = oracle.pair_local(t, Xm, X, pr)["grad"][:n]
        F[:, j] = (gp_ - gm_) / (2 * h)
    scale = np.abs(H[:n, :n]).max()
    assert np.abs(F - H[:n, :n]).max() <= 1e-6 * scale, (name, np.abs(F - H[:n, :n]).max() / scale)
    if "moll" in name or "par" in name:
        assert base["mollified"], name


def test_point_point_exact_minus_proxy_is_the_dropped_term():
    rng = np.random.default_rng(3)
    for _ in range(20):
        d = rng.uniform(0.05, 0.95) * DH
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        X = np.vstack([[0.1, 0.2, 0.3], np.array([0.1, 0.2, 0.3]) - d * n])
        t = [_neg(0), 1, -1, -1]
        H, _ = oracle.pair_exact(t, X, X, prm())
        proxy = oracle.pair_local(t, X, X, prm(filter=False))["hess"]
        # b as a function of d: b_d = b'(g) 2 d / dhat^2
        b, db, _ = oracle.barrier(d * d / DH ** 2, DH)
        b_d = db * 2 * d / DH ** 2
        hd = (np.eye(3) - np.outer(n, n)) / d
        ref = KAPPA * b_d * np.block([[hd, -hd], [-hd, hd]])
        diff = H[:6, :6] - proxy[:6, :6]
        assert np.abs(diff - ref).max() <= 1e-9 * np.abs(H[:6, :6]).max()


@pytest.mark.parametrize("case", range(42))
def test_projection_against_eigh(case):
    name, t, X = _configs()[case]
    pr = prm(epsx_ratio=1.0 if "moll" in name or "par" in name else 1e-3)
    H, Hp = oracle.pair_exact(t, X, X, pr)
    nv, _ = oracle.stencil(t)
    n = 3 * nv
    lam, V = np.linalg.eigh(H[:n, :n])
    ref = (V * np.maximum(lam, 0.0)) @ V.T
    scale = np.abs(lam).max()
    assert np.abs(Hp[:n, :n] - ref).max() <= 1e-10 * scale, name
    assert np.abs(Hp - Hp.T).max() <= 1e-14 * scale
    assert np.linalg.eigvalsh(Hp[:n, :n]).min() >= -1e-12 * scale
    assert not np.any(Hp[n:, :]) and not np.any(Hp[:, n:])


def test_exact_hessians_are_indefinite_and_psd_ones_are_kept():
    neg = 0
    for name, t, X in _configs():
        H, Hp = oracle.pair_exact(t, X, X, prm(epsx_ratio=1.0 if "moll" in name or "par" in name else 1e-3))
        lam = np.linalg.eigvalsh(H)
        if lam.min() < -1e-9 * np.abs(lam).max():
            neg += 1
        else:
            assert np.allclose(Hp, H, rtol=0, atol=1e-10 * np.abs(H).max())
    assert neg >= 30
    # a PSD input (the projected matrix itself) is returned as it is
    name, t, X = _configs()[0]
    _, Hp = oracle.pair_exact(t, X, X, prm())
    lam, V = np.linalg.eigh(Hp[:12, :12])
    assert lam.min() >= -1e-12 * np.abs(lam).max()


def test_inactive_pair_gives_zeros():
    X = np.array([[0.3, 0.3, 1.5], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    H, Hp = oracle.pair_exact([_neg(0), 1, 2, 3], X, X, prm())
    assert not H.any() and not Hp.any()
