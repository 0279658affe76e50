"""The Helmholtz singular pairs' radial series and the range the library
accepts it in (host only).

The device integrates the radial factor of a vertex-sharing pair as the
power series sum_n (i omega)^n mu_n / n! of the moments mu_n of the radial
polynomial, 48 terms in Horner form (omega = k |c| with x - y = rho c).  For
the identical-pair polynomial (1 - rho)^2 the integral has a closed form;
the same series evaluated in FP64 here matches it to ~1e-9 relative at
omega = 12 and loses all accuracy by omega = 20, which is why requests whose
pairs reach k |c| > 12 are refused (the constant in mesh_expand.cpp).
"""
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def series(om, terms=48):
    # coefficients of the device's table: mu_n = 2 / ((n+1)(n+2)(n+3)), i^n / n!
    re_c, im_c = [], []
    fact = 1.0
    for n in range(terms):
        if n:
            fact *= n
        a = 2.0 / ((n + 1) * (n + 2) * (n + 3)) / fact
        sgn = -1.0 if (n // 2) % 2 else 1.0
        (re_c if n % 2 == 0 else im_c).append(sgn * a)
    w2 = om * om
    r, i = re_c[-1], im_c[-1]
    for m in range(len(re_c) - 2, -1, -1):
        r = r * w2 + re_c[m]
        i = i * w2 + im_c[m]
    return complex(r, om * i)


def closed_form(om):
    # int_0^1 (1 - rho)^2 e^{i om rho} d rho = 2 / (i om)^3 (e^{i om} - 1) - 2 / (i om)^2 - 1 / (i om)
    z = 1j * om
    return 2.0 * (np.exp(z) - 1.0) / z ** 3 - 2.0 / z ** 2 - 1.0 / z


def test_closed_form_against_quadrature():
    x, w = np.polynomial.legendre.leggauss(200)
    rho, wt = 0.5 * (x + 1.0), 0.5 * w
    for om in (0.5, 6.0, 12.0, 20.0):
        q = np.sum(wt * (1.0 - rho) ** 2 * np.exp(1j * om * rho))
        assert abs(q - closed_form(om)) <= 1e-14 * max(1.0, abs(q))


def test_series_accuracy_decides_the_bound():
    src = open(os.path.join(ROOT, "paper_1711_01897_amd", "csrc", "mesh_expand.cpp")).read()
    bound = float(re.search(r"constexpr double kOmegaMax = ([0-9.]+);", src).group(1))
    assert bound == 12.0
    for om in np.linspace(0.1, bound, 60):
        ref = closed_form(om)
        assert abs(series(om) - ref) <= 1e-8 * abs(ref), om
    errs = {om: abs(series(om) - closed_form(om)) / abs(closed_form(om)) for om in (16.0, 20.0, 24.0)}
    assert errs[20.0] > 1e-6 and errs[24.0] > 1e-2, errs
    assert math.isfinite(errs[16.0])
