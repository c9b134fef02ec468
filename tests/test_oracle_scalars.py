"""Pins of the oracle's scalar functions against sympy and the paper's printed
closed forms.

* b(g) of Eq. 24 (and Eq. 12) and its first two derivatives: symbolic
  differentiation by sympy, independent of the oracle's hand-written product
  rule.
* The mollifier e(c) of Eq. 25 and its derivatives: sympy.
* Eq. 18-19 for Eq. 12: the expanded lambda_1 printed in the supplement
  (Sec. 3) must equal 4 g b'' + 2 b' built from the oracle's derivatives;
  lambda_{2,3} matches 2 b' only with the denominator read as g (the printed
  g^2 is a typo, documented reading).
* Sign facts the paper states (Sec. 5.3, supplement Sec. 3; Sec. 5.2).
"""
import os

import numpy as np
import pytest
import sympy as sp

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "supplement_eq12_eigenvalues.txt")
G_SAMPLES = [1e-6, 1e-4, 1e-3, 0.01, 0.05, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99, 0.999999]

g_s, dh_s, c_s, eps_s = sp.symbols("g dh c eps", positive=True)
B24 = (dh_s ** 2 - dh_s ** 2 * g_s) ** 2 * sp.log(g_s) ** 2          # Eq. 24
B12 = -(dh_s ** 2 - dh_s ** 2 * g_s) ** 2 * sp.log(g_s)              # Eq. 12


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split("=", 1)
        out[k.strip()] = sp.sympify(v.strip(), locals={"g": g_s, "dh": dh_s, "log": sp.log})
    return out


@pytest.mark.parametrize("eq12,expr", [(False, B24), (True, B12)])
@pytest.mark.parametrize("dhat", [1e-3, 1.0])
def test_barrier_derivatives_vs_sympy(eq12, expr, dhat):
    d1 = sp.diff(expr, g_s)
    d2 = sp.diff(expr, g_s, 2)
    for g in G_SAMPLES:
        sub = {g_s: sp.Float(g, 40), dh_s: sp.Float(dhat, 40)}
        ref = [float(expr.subs(sub).evalf(30)), float(d1.subs(sub).evalf(30)), float(d2.subs(sub).evalf(30))]
        got = oracle.barrier(g, dhat, eq12)
        for r, v in zip(ref, got):
            scale = max(abs(r), 1e-300)
            # the derivatives are sums of large cancelling terms near g -> 1
            assert abs(v - r) <= 1e-11 * max(scale, 1e-9 * dhat ** 4), (g, eq12, r, v)


def test_barrier_reference_constants():
    # b(0.01), b'(0.01) and lambda_1(0.01) in units of dhat^4, evaluated by
    # sympy from Eq. 24 and Eq. 18 (the filter threshold g = (0.1)^2)
    for dhat in (1e-3, 1.0):
        sub = {g_s: sp.Rational(1, 100), dh_s: 1}
        b = float(B24.subs(sub).evalf(30))
        db = float(sp.diff(B24, g_s).subs(sub).evalf(30))
        lam = float((4 * g_s * sp.diff(B24, g_s, 2) + 2 * sp.diff(B24, g_s)).subs(sub).evalf(30))
        ob, odb, od2b = oracle.barrier(0.01, dhat)
        s = dhat ** 4
        assert ob / s == pytest.approx(b, rel=1e-13)
        assert odb / s == pytest.approx(db, rel=1e-13)
        assert (4 * 0.01 * od2b + 2 * odb) / s == pytest.approx(lam, rel=1e-12)


def test_mollifier_vs_sympy():
    e = -c_s ** 2 / eps_s ** 2 + 2 * c_s / eps_s      # Eq. 25, c < eps
    for eps in (1e-3, 2.5e-7):
        for r in (0.0, 1e-6, 0.1, 1.0 / 3.0, 0.5, 0.9, 0.999):
            c = r * eps
            sub = {c_s: sp.Float(c, 40), eps_s: sp.Float(eps, 40)}
            ref = [float(e.subs(sub)), float(sp.diff(e, c_s).subs(sub)), float(sp.diff(e, c_s, 2).subs(sub))]
            got = oracle.mollifier(c, eps)
            for rr, v in zip(ref, got):
                assert v == pytest.approx(rr, rel=1e-13, abs=1e-300)
        assert oracle.mollifier(eps, eps) == (1.0, 0.0, 0.0)
        assert oracle.mollifier(2 * eps, eps) == (1.0, 0.0, 0.0)
        # C1 continuity at c = eps
        e0, de0, _ = oracle.mollifier(eps * (1 - 1e-12), eps)
        assert e0 == pytest.approx(1.0, abs=1e-11) and abs(de0) * eps < 1e-10


def test_eq12_lambda1_matches_supplement():
    gold = _golden()
    for dhat in (1e-3, 1.0):
        for g in G_SAMPLES[:-1]:
            b, db, d2b = oracle.barrier(g, dhat, eq12=True)
            lam1 = 4 * g * d2b + 2 * db                                  # Eq. 18
            ref = float(gold["lambda1"].subs({g_s: g, dh_s: dhat}))
            assert lam1 == pytest.approx(ref, rel=1e-9, abs=1e-12 * dhat ** 4), g


def test_eq12_lambda23_denominator_reading():
    gold = _golden()
    for g in (0.01, 0.3, 0.7):
        _, db, _ = oracle.barrier(g, 1.0, eq12=True)
        lam23 = 2 * db                                                  # Eq. 19
        corr = float(gold["lambda23_corrected"].subs({g_s: g, dh_s: 1}))
        printed = float(gold["lambda23_printed"].subs({g_s: g, dh_s: 1}))
        assert lam23 == pytest.approx(corr, rel=1e-12)
        assert abs(lam23 - printed) > 1e-3 * abs(corr)   # the printed g^2 differs


def test_eq12_printed_derivative_of_lambda1():
    # the printed d lambda_1 / dg is the derivative of the printed lambda_1
    gold = _golden()
    assert sp.simplify(sp.diff(gold["lambda1"], g_s) - gold["dlambda1"]) == 0


@pytest.mark.parametrize("eq12", [False, True])
def test_lambda1_positive_and_decreasing(eq12):
    gs = np.unique(np.concatenate([np.logspace(-8, -1, 200), np.linspace(0.1, 0.9999, 400)]))
    lam = []
    for g in gs:
        b, db, d2b = oracle.barrier(g, 1.0, eq12)
        lam.append(4 * g * d2b + 2 * db)
        assert 2 * db <= 0.0                        # lambda_{2,3} <= 0 (supplement Sec. 3)
    lam = np.array(lam)
    assert (lam > 0).all()
    assert (np.diff(lam) < 0).all()                # so Eq. 23 caps lambda_1 at lambda_1(eps_g)
