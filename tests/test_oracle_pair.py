"""Pins of the oracle's per-pair energy, gradient and proxy Hessian.

Each pin comes from outside the oracle:

* gradient: central finite differences of the oracle's own energy along
  random directions (the energy itself is pinned by the scalar and distance
  tests);
* non-mollified proxy Hessian: Eq. 18 with f = d / dhat makes
  lambda_1 / dhat^2 = d^2 b / dd^2, so the projected Gauss-Newton Hessian
  must equal kappa * b_dd(max(d, d_thr)) grad d grad d^T (the IPC
  Gauss-Newton term of Eq. 22 applied to the Eq. 24 barrier), with b_dd from
  sympy and grad d by finite differences;
* inner Hessian eigenvalues against the paper's analytic eigensystems
  (Eq. 18-19 non-mollified; Eq. 32-35 mollified) and the eigenvector Q'_8;
* App. B norms; symmetry, PSD-ness, rank and translation invariance;
* the dropped term: for a point-point pair the exact Hessian (finite
  differences of the gradient) minus the proxy equals
  kappa [2 f b'(g) Hess(f) + (lambda_1(g) - lambda_1(g_f)) grad f grad f^T],
  with the textbook Hess(f) of a point-point distance.
"""
import numpy as np
import pytest
import sympy as sp

import oracle

DH = 1.0          # unit scale keeps finite differences well conditioned
KAPPA = 3.0

d_s, g_s, c_s, eps_s = sp.symbols("d g c eps", positive=True)
_bd = (DH ** 2 - d_s ** 2) ** 2 * sp.log(d_s ** 2 / DH ** 2) ** 2          # Eq. 24 as a function of d
_bdd = sp.lambdify(d_s, sp.diff(_bd, d_s, 2), "mpmath")
_bg = (DH ** 2 - DH ** 2 * g_s) ** 2 * sp.log(g_s) ** 2
_bg_f = [sp.lambdify(g_s, sp.diff(_bg, g_s, k), "mpmath") for k in range(3)]
_e = -c_s ** 2 / eps_s ** 2 + 2 * c_s / eps_s
_e_f = [sp.lambdify((c_s, eps_s), sp.diff(_e, c_s, k), "mpmath") for k in range(3)]


def prm(**kw):
    base = dict(dhat=DH, kappa=KAPPA)
    base.update(kw)
    return oracle.params(**base)


def rand_rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


# ---------------------------------------------------------------- cases


def case_pt(rng, region):
    T = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    h = rng.uniform(0.05, 0.9)
    if region == "interior":
        p = np.array([0.2, 0.25, h])
    elif region == "edge":
        p = np.array([0.5 + 0.2 * h, 0.5 + 0.2 * h, 0.3 * h])
    else:
        p = np.array([-0.3 * h, -0.4 * h, 0.2 * h])
    R = rand_rot(rng)
    X = (np.vstack([p, T]) + rng.normal(scale=0.01, size=(4, 3))) @ R.T
    return np.array([-1, 1, 2, 3], np.int32), X, X


def case_ee(rng, parallel=False):
    gap = rng.uniform(0.1, 0.8)
    th = rng.uniform(0.005, 0.02) if parallel else rng.uniform(0.5, 1.5)
    a0, a1 = np.array([-0.6, 0, 0]), np.array([0.7, 0, 0])
    b0 = np.array([-0.5 * np.cos(th), -0.5 * np.sin(th), gap])
    b1 = np.array([0.8 * np.cos(th), 0.8 * np.sin(th), gap])
    X = np.vstack([a0, a1, b0, b1])
    R = rand_rot(rng)
    X = X @ R.T
    Xr = X + rng.normal(scale=0.02, size=(4, 3))
    return np.array([0, 1, 2, 3], np.int32), X, Xr


def case_ee_endpoint(rng, parallel=False):
    # edges whose closest points involve an endpoint (PE / PP sub-types)
    th = rng.uniform(0.005, 0.02) if parallel else 0.9
    a0, a1 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0])
    b0 = np.array([1.2, 0.1, 0.3])
    b1 = b0 + 1.0 * np.array([np.cos(th), np.sin(th), 0])
    X = np.vstack([a0, a1, b0, b1]) @ rand_rot(rng).T
    return np.array([0, 1, 2, 3], np.int32), X, X


CASES = {
    "pt_interior": lambda r: case_pt(r, "interior"),
    "pt_edge": lambda r: case_pt(r, "edge"),
    "pt_vertex": lambda r: case_pt(r, "vertex"),
    "ee_cross": lambda r: case_ee(r, False),
    "ee_parallel": lambda r: case_ee(r, True),
    "ee_endpoint": lambda r: case_ee_endpoint(r, False),
    "ee_endpoint_parallel": lambda r: case_ee_endpoint(r, True),
}


def energy(t, X, Xr, P):
    return oracle.pair_local(t, X, Xr, P)["E"]


# ---------------------------------------------------------------- tests


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("seed", range(4))
def test_gradient_vs_central_fd(name, seed):
    rng = np.random.default_rng(seed)
    t, X, Xr = CASES[name](rng)
    P = prm()
    out = oracle.pair_local(t, X, Xr, P)
    assert out["subtype"] != oracle.INACTIVE
    g = out["grad"]
    for _ in range(6):
        u = rng.normal(size=12)
        u /= np.linalg.norm(u)
        h = 1e-6
        fd = (energy(t, X + h * u.reshape(4, 3), Xr, P) - energy(t, X - h * u.reshape(4, 3), Xr, P)) / (2 * h)
        assert g @ u == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.linalg.norm(g))


@pytest.mark.parametrize("name", ["pt_interior", "pt_edge", "pt_vertex", "ee_cross", "ee_endpoint"])
@pytest.mark.parametrize("filt", [True, False])
@pytest.mark.parametrize("seed", range(3))
def test_nonmollified_hessian_is_ipc_gauss_newton(name, filt, seed):
    rng = np.random.default_rng(10 + seed)
    t, X, Xr = CASES[name](rng)
    P = prm(filter=filt)
    out = oracle.pair_local(t, X, Xr, P)
    assert not out["mollified"]
    d = np.sqrt(out["d2"])
    # grad d by central differences of the (brute-force pinned) distance
    gd = np.zeros(12)
    h = 1e-6
    for i in range(12):
        e = np.zeros(12); e[i] = h
        dp = np.sqrt(oracle.pair_local(t, X + e.reshape(4, 3), Xr, P)["d2"])
        dm = np.sqrt(oracle.pair_local(t, X - e.reshape(4, 3), Xr, P)["d2"])
        gd[i] = (dp - dm) / (2 * h)
    df = max(d, 0.1 * DH) if filt else d
    ref = KAPPA * float(_bdd(df)) * np.outer(gd, gd)
    assert np.linalg.norm(out["hess"] - ref) <= 1e-6 * np.linalg.norm(ref)


def _analytic_mollified_eigs(c, epsx, g, filt):
    f = np.sqrt(g)
    ff = max(f, 0.1) if filt else f
    gf = ff * ff
    b, db, d2b = (float(F(gf)) for F in _bg_f)
    e, de, d2e = (float(F(c, epsx)) for F in _e_f)
    bg, bgg = de * b, d2e * b          # d b~/d gamma, d2 b~/d gamma2
    bq, bqq = e * db, e * d2b          # d b~/d g,     d2 b~/d g2
    bgq = de * db                      # d2 b~/d gamma dg
    lg1 = 2 * (bg + 2 * c * bgg)
    lg23 = 2 * bg
    lq1 = 2 * (bq + 2 * gf * bqq)
    lq23 = 2 * bq
    t = bgq * np.sqrt(c) * ff                                   # Eq. 33
    p = np.sqrt(lg1 ** 2 - 2 * lg1 * lq1 + lq1 ** 2 + 64 * t ** 2) / 2
    l7 = (lg1 + lq1) / 2 - p                                    # Eq. 34
    l8 = (lg1 + lq1) / 2 + p                                    # Eq. 35
    k2 = (lg1 - lq1 + 2 * p) / (8 * t) if t != 0 else None
    return np.sort([lg23, lg23, lq23, lq23, l7, l8, 0, 0, 0]), dict(lg1=lg1, lg23=lg23, lq1=lq1, lq23=lq23, l7=l7,
                                                                      l8=l8, k2=k2)


@pytest.mark.parametrize("name", ["ee_parallel", "ee_endpoint_parallel"])
@pytest.mark.parametrize("filt", [True, False])
@pytest.mark.parametrize("seed", range(4))
def test_mollified_inner_eigensystem(name, filt, seed):
    rng = np.random.default_rng(20 + seed)
    t, X, Xr = CASES[name](rng)
    P = prm(filter=filt)
    out = oracle.pair_local(t, X, Xr, P, debug=True)
    assert out["mollified"] and out["m"] == 3
    a, b = X[1] - X[0], X[3] - X[2]
    c = float(np.sum(np.cross(a, b) ** 2))
    epsx = 1e-3 * np.sum((Xr[1] - Xr[0]) ** 2) * np.sum((Xr[3] - Xr[2]) ** 2)
    ref, parts = _analytic_mollified_eigs(c, epsx, out["d2"] / DH ** 2, filt)
    lam, vec = np.linalg.eigh(out["innerH"])
    scale = np.abs(ref).max()
    assert np.sort(lam) == pytest.approx(ref, abs=1e-10 * scale)
    # sign facts (Sec. 5.2): lambda_gamma2,3 >= 0, lambda_g1 >= 0, lambda_g2,3 <= 0
    assert parts["lg23"] >= 0 and parts["lq1"] >= 0 and parts["lq23"] <= 0
    if filt:
        assert parts["l7"] <= 1e-12 * scale       # lambda'_7 <= 0 holds under the filter
    # Q'_8: (k2 at J22, 1 at J33), normalised, is an eigenvector for lambda'_8
    if parts["k2"] is not None:
        q = np.zeros(9); q[4] = parts["k2"]; q[8] = 1.0
        q /= np.linalg.norm(q)
        assert np.linalg.norm(out["innerH"] @ q - parts["l8"] * q) <= 1e-9 * scale
    # lambda_gamma1 > 0 exactly when c < eps_x / 3
    assert (parts["lg1"] > 0) == (c < epsx / 3)


@pytest.mark.parametrize("name", ["pt_interior", "pt_edge", "pt_vertex", "ee_cross", "ee_endpoint"])
@pytest.mark.parametrize("filt", [True, False])
def test_nonmollified_inner_eigs_and_app_b_norms(name, filt):
    rng = np.random.default_rng(7)
    t, X, Xr = CASES[name](rng)
    out = oracle.pair_local(t, X, Xr, prm(filter=filt), debug=True)
    g = out["d2"] / DH ** 2
    gf = max(g, 0.01) if filt else g
    b, db, d2b = (float(F(gf)) for F in _bg_f)
    lam1 = 4 * gf * d2b + 2 * db                                  # Eq. 18
    m = out["m"]
    ref = np.sort([lam1] + [2 * db] * (m - 1) + [0.0] * (m * m - m))   # Eq. 19
    lam = np.linalg.eigvalsh(out["innerH"])
    assert np.sort(lam) == pytest.approx(ref, abs=1e-10 * abs(lam1))
    # App. B: |db/dJ|_F = -2 sqrt(g) b'(g) at the actual g; |projected|_F = lambda_1
    _, db_a, _ = (float(F(g)) for F in _bg_f)
    assert np.linalg.norm(out["dbdJ"]) == pytest.approx(-2 * np.sqrt(g) * db_a, rel=1e-10)
    assert np.linalg.norm(out["innerHp"]) == pytest.approx(lam1, rel=1e-10)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("seed", range(3))
def test_hessian_invariants(name, seed):
    rng = np.random.default_rng(30 + seed)
    t, X, Xr = CASES[name](rng)
    P = prm()
    out = oracle.pair_local(t, X, Xr, P)
    H, g = out["hess"], out["grad"]
    assert np.array_equal(H, H.T) or np.abs(H - H.T).max() <= 1e-14 * np.abs(H).max()
    lam = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert lam.min() >= -1e-12 * lam.max()
    rank = int(np.sum(lam > 1e-10 * lam.max()))
    assert rank <= (2 if out["mollified"] else 1)
    T = np.tile(np.eye(3), (4, 1))               # rigid translations of all 4 slots
    assert np.abs(H @ T).max() <= 1e-10 * np.abs(H).max()
    assert np.abs(g.reshape(4, 3).sum(0)).max() <= 1e-10 * np.abs(g).max()
    # rotation invariance of the energy (rest shape rotated alike)
    R = rand_rot(rng)
    E2 = oracle.pair_local(t, X @ R.T, Xr @ R.T, P)["E"]
    assert E2 == pytest.approx(out["E"], rel=1e-12)


@pytest.mark.parametrize("filt", [True, False])
@pytest.mark.parametrize("d", [0.05, 0.3, 0.8])
def test_dropped_term_point_point(filt, d):
    """Exact Hessian - proxy = kappa [2 f b'(g) Hess f + (l1(g) - l1(g_f)) grad f grad f^T] (Eq. 15, 22)."""
    rng = np.random.default_rng(int(d * 100))
    n = rng.normal(size=3); n /= np.linalg.norm(n)
    p0 = rng.normal(size=3)
    X = np.zeros((4, 3)); X[0] = p0 + d * n; X[1] = p0
    t = np.array([-1, 1, -1, -1], np.int32)
    P = prm(filter=filt)
    out = oracle.pair_local(t, X, X, P)
    # exact Hessian by central differences of the (FD-pinned) gradient
    h = 1e-6
    Hx = np.zeros((6, 6))
    for i in range(6):
        e = np.zeros(12); e[i] = h
        gp = oracle.pair_local(t, X + e.reshape(4, 3), X, P)["grad"][:6]
        gm = oracle.pair_local(t, X - e.reshape(4, 3), X, P)["grad"][:6]
        Hx[:, i] = (gp - gm) / (2 * h)
    f, g = d / DH, (d / DH) ** 2
    gf = max(g, 0.01) if filt else g
    gradf = np.concatenate([n, -n]) / DH
    Pn = (np.eye(3) - np.outer(n, n)) / (DH * d)          # Hess of |p - q| / dhat
    Hf = np.block([[Pn, -Pn], [-Pn, Pn]])
    _, db, _ = (float(F(g)) for F in _bg_f)
    l1 = lambda gg: float(4 * gg * _bg_f[2](gg) + 2 * _bg_f[1](gg))
    ref = KAPPA * (2 * f * db * Hf + (l1(g) - l1(gf)) * np.outer(gradf, gradf))
    diff = Hx - out["hess"][:6, :6]
    assert np.abs(diff - ref).max() <= 1e-6 * max(np.abs(Hx).max(), 1e-12)


def test_inactive_and_degenerate():
    X = np.zeros((4, 3)); X[0] = [0, 0, 1.5 * DH]
    out = oracle.pair_local(np.array([-1, 1, -1, -1], np.int32), X, X, prm())
    assert out["subtype"] == oracle.INACTIVE and out["E"] == 0 and not out["grad"].any() and not out["hess"].any()
    X[0] = [0, 0, 0]
    out = oracle.pair_local(np.array([-1, 1, -1, -1], np.int32), X, X, prm())
    assert out["subtype"] == oracle.DEGENERATE and out["E"] == 0 and not out["grad"].any()


def test_exactly_parallel_edges_contribute_nothing():
    # c = 0: the mollifier is 0, grad c is 0; sqrt(c) has no gradient, its
    # row of dJ/dx is taken as zero, so the proxy Hessian vanishes too
    X = np.array([[0, 0, 0], [1, 0, 0], [0.2, 0, 0.4], [1.3, 0, 0.4]], float)
    out = oracle.pair_local(np.array([0, 1, 2, 3], np.int32), X, X, prm())
    assert out["mollified"] and out["E"] == 0 and not out["grad"].any() and not out["hess"].any()


def test_rounding_level_parallel_edges_follow_exact_cross_product():
    # Two facing diagonals of a cube lattice (m = 2, n = 10, seed 3): parallel
    # in exact arithmetic before the vertex coordinates were rounded.  The
    # rounded input is not quite parallel: |a x b| is 4.9e-32, while the
    # plain product formula returns exactly 0 here.  The parallelness c of
    # Eq. 25 is a function of the input coordinates, so c > 0, and the proxy
    # Hessian is the rank-1 mollifier term along grad c (the distance term is
    # scaled by e(c) ~ 1e-57).  grad c is taken exactly: sympy's derivative of
    # |(x1 - x0) x (x3 - x2)|^2 evaluated in rationals.
    from fractions import Fraction
    X = np.array([[1.7779462971114925, 1.0, 1.1118521306832763],
                  [1.8890574082226037, 1.0, 1.2229632417943872],
                  [1.8890574082226037, 1.000289448405277, 1.2229632417943872],
                  [2.000168519333715, 1.000289448405277, 1.3340743529054984]])
    xs = sp.Matrix(4, 3, lambda i, j: sp.Symbol(f"x{i}{j}"))
    a = xs[1, :] - xs[0, :]
    b = xs[3, :] - xs[2, :]
    n = a.cross(b)
    c = n.dot(n)
    subs = {xs[i, j]: sp.Rational(Fraction(float(X[i, j]))) for i in range(4) for j in range(3)}
    c_exact = c.subs(subs)
    assert c_exact > 0
    grad = [sp.diff(c, xs[i, j]).subs(subs) for i in range(4) for j in range(3)]
    top = max(abs(gk) for gk in grad)
    gdir = np.array([float(gk / top) for gk in grad])
    gdir /= np.linalg.norm(gdir)
    out = oracle.pair_local(np.array([0, 1, 2, 3], np.int32), X, X, oracle.params(dhat=1e-3, kappa=1.0))
    assert out["mollified"] and out["subtype"] == oracle.PP
    lam, Q = np.linalg.eigh(out["hess"])
    assert lam[-1] > 0 and np.abs(lam[:-1]).max() <= 1e-12 * lam[-1]
    assert abs(abs(Q[:, -1] @ gdir) - 1.0) <= 1e-12
