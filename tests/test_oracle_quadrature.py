"""Pins of the oracle's Gauss rules against closed forms.

The paper fixes a symmetric rule of order 4 with six weights (Section
3.2.1).  Closed form: int_ref xi^a eta^b = a! b! / (a+b+2)!.  A rule of
degree d integrates every monomial with a+b <= d exactly and some monomial
of degree d+1 inexactly.
"""
import math

import numpy as np
import pytest

import oracle as O


def monomial_error(xi, eta, w, a, b):
    exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
    return abs(float(np.sum(w * xi ** a * eta ** b)) - exact)


@pytest.mark.parametrize("npts,degree", [(6, 4), (4, 3)])
def test_rule_degree(npts, degree):
    xi, eta, w = O.rule(npts)
    assert xi.size == npts
    assert abs(w.sum() - 0.5) < 1e-15
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            assert monomial_error(xi, eta, w, a, b) < 1e-15, (a, b)
    worst = max(monomial_error(xi, eta, w, a, degree + 1 - a) for a in range(degree + 2))
    assert worst > 1e-5


@pytest.mark.parametrize("npts", [6, 4])
def test_rule_symmetric_and_inside(npts):
    xi, eta, w = O.rule(npts)
    l0 = 1.0 - xi - eta
    assert (xi > 0).all() and (eta > 0).all() and (l0 > 0).all()
    pts = {(round(a, 12), round(b, 12), round(c, 12), round(ww, 12)) for a, b, c, ww in zip(l0, xi, eta, w)}
    # invariant under every permutation of the barycentric coordinates
    for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0)]:
        permuted = {tuple(np.array(p[:3])[list(perm)]) + (p[3],) for p in pts}
        assert permuted == pts


def test_six_point_positive_weights():
    # positivity makes single-layer entries sums of positive terms
    _, _, w = O.rule(6)
    assert (w > 0).all()


def test_subdivided_rule_converges_to_closed_form():
    # int_ref exp(xi + 2 eta) = (e - 1)^2 / 2
    exact = (math.e - 1.0) ** 2 / 2.0
    errs = []
    for level in range(4):
        xi, eta, w = O.subdivided_rule(level)
        assert abs(w.sum() - 0.5) < 1e-14
        errs.append(abs(float(np.sum(w * np.exp(xi + 2 * eta))) - exact))
    # degree-4 rule on h/2 sub-triangles: error falls by ~2^5..2^6 per level
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 20.0
    assert errs[-1] < 1e-9
