"""Pins of the oracle's Green's function and its normal derivatives.

g(x,y) = exp(i k r)/(4 pi r) (Section 2, Green's function of the Helmholtz
equation, Laplace at k = 0); the double layer uses dg/dn_y (Eq. dlp), the
adjoint double layer dg/dn_x (Eq. adlp).
"""
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.Generator(np.random.PCG64(3))


def unit(v):
    return v / np.linalg.norm(v)


def test_laplace_slp_value():
    x = np.array([0.0, 0.0, 0.0])
    y = np.array([3.0, 4.0, 0.0])
    assert abs(O.kernel(O.LAPLACE_SLP, 0.0, x, y, [0, 0, 1]).real - 1.0 / (4 * math.pi * 5.0)) < 1e-17


def test_unit_sphere_double_layer_is_minus_half_single_layer():
    # on the unit sphere with n_y = y: (x - y).y = -|x - y|^2 / 2
    for _ in range(20):
        x = unit(RNG.normal(size=3))
        y = unit(RNG.normal(size=3))
        s = O.kernel(O.LAPLACE_SLP, 0.0, x, y, y).real
        d = O.kernel(O.LAPLACE_DLP, 0.0, x, y, y).real
        assert abs(d + 0.5 * s) <= 1e-14 * abs(s)


@pytest.mark.parametrize("pair", [(O.HELMHOLTZ_SLP, O.LAPLACE_SLP), (O.HELMHOLTZ_DLP, O.LAPLACE_DLP)])
def test_helmholtz_at_zero_wavenumber_is_laplace(pair):
    h, l = pair
    for _ in range(10):
        x, y, n = RNG.normal(size=3), RNG.normal(size=3), unit(RNG.normal(size=3))
        gh = O.kernel(h, 0.0, x, y, n)
        gl = O.kernel(l, 0.0, x, y, n)
        assert abs(gh - gl) <= 1e-15 * abs(gl)


@pytest.mark.parametrize("op,k", [(O.LAPLACE_DLP, 0.0), (O.HELMHOLTZ_DLP, 2.7), (O.HELMHOLTZ_DLP, 11.0)])
def test_double_layer_is_normal_derivative_in_y(op, k):
    slp = O.LAPLACE_SLP if op == O.LAPLACE_DLP else O.HELMHOLTZ_SLP
    eps = 1e-5
    for _ in range(10):
        x, y, n = RNG.normal(size=3), RNG.normal(size=3), unit(RNG.normal(size=3))
        fd = (O.kernel(slp, k, x, y + eps * n, n) - O.kernel(slp, k, x, y - eps * n, n)) / (2 * eps)
        d = O.kernel(op, k, x, y, n)
        assert abs(fd - d) <= 1e-7 * abs(d) + 1e-12


@pytest.mark.parametrize("k", [0.0, 1.5, 6.0])
def test_single_layer_solves_helmholtz_equation(k):
    # Delta_x g + k^2 g = 0 away from y (7-point finite differences)
    eps = 1e-3
    op = O.LAPLACE_SLP if k == 0.0 else O.HELMHOLTZ_SLP
    for _ in range(5):
        y = RNG.normal(size=3)
        x = y + unit(RNG.normal(size=3)) * 1.3
        g0 = O.kernel(op, k, x, y, [0, 0, 1])
        lap = -6.0 * g0
        for d in range(3):
            e = np.zeros(3)
            e[d] = eps
            lap += O.kernel(op, k, x + e, y, [0, 0, 1]) + O.kernel(op, k, x - e, y, [0, 0, 1])
        lap /= eps * eps
        assert abs(lap + k * k * g0) <= 2e-5 * max(1.0, k * k) * abs(g0)


def test_helmholtz_phase_convention_outgoing():
    # exp(+i k r): the phase grows with r at rate k, modulus is 1/(4 pi r)
    k = 4.0
    x = np.zeros(3)
    prev = None
    for r in np.linspace(1.0, 2.0, 11):
        g = O.kernel(O.HELMHOLTZ_SLP, k, x, [r, 0.0, 0.0], [0, 0, 1])
        assert abs(abs(g) - 1.0 / (4 * math.pi * r)) < 1e-16
        if prev is not None:
            dphi = np.angle(g / prev[0])
            assert abs(dphi - k * (r - prev[1])) < 1e-12
        prev = (g, r)


@pytest.mark.parametrize("op,k", [(O.LAPLACE_ADLP, 0.0), (O.HELMHOLTZ_ADLP, 2.7), (O.HELMHOLTZ_ADLP, 11.0)])
def test_adjoint_double_layer_is_normal_derivative_in_x(op, k):
    slp = O.LAPLACE_SLP if op == O.LAPLACE_ADLP else O.HELMHOLTZ_SLP
    eps = 1e-5
    for _ in range(10):
        x, y, n = RNG.normal(size=3), RNG.normal(size=3), unit(RNG.normal(size=3))
        fd = (O.kernel(slp, k, x + eps * n, y, n) - O.kernel(slp, k, x - eps * n, y, n)) / (2 * eps)
        d = O.kernel(op, k, x, y, n)
        assert abs(fd - d) <= 1e-7 * abs(d) + 1e-12


@pytest.mark.parametrize("pair,k", [((O.LAPLACE_ADLP, O.LAPLACE_DLP), 0.0), ((O.HELMHOLTZ_ADLP, O.HELMHOLTZ_DLP), 4.2)])
def test_adjoint_kernel_is_double_layer_with_points_exchanged(pair, k):
    """g is symmetric in (x, y), so dg/dn_x at (x, y) is dg/dn_y at (y, x)
    with the same normal."""
    adj, dl = pair
    for _ in range(10):
        x, y, n = RNG.normal(size=3), RNG.normal(size=3), unit(RNG.normal(size=3))
        a = O.kernel(adj, k, x, y, n)
        d = O.kernel(dl, k, y, x, n)
        assert abs(a - d) <= 1e-15 * abs(d)
