"""Pins of the oracle's B-spline basis against Table 1, closed forms and scipy."""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_exact():
    rows = np.loadtxt(os.path.join(GOLD, "table1_w.txt"), dtype=int)
    for d, k, num, den in rows:
        assert bspline.w_exact(int(k), int(d)) == Fraction(int(num), int(den))


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_w_binomial_and_moments(d):
    from math import comb, factorial
    for k in range(d + 2):
        assert bspline.w_exact(k, d) == Fraction((-1) ** k * comb(d + 1, k), factorial(d))
    # a (d+1)-th difference annihilates polynomials of degree <= d
    for m in range(d + 1):
        assert sum(bspline.w_exact(k, d) * k ** m for k in range(d + 2)) == 0


@pytest.mark.parametrize("d", [1, 2, 3])
def test_against_scipy_bspline(d):
    t = np.linspace(-1.0, d + 3.0, 997)
    ref = BSpline.basis_element(np.arange(d + 2, dtype=float), extrapolate=False)(t)
    ref = np.nan_to_num(ref)
    assert np.max(np.abs(bspline.basis(0, d, t) - ref)) < 1e-12


@pytest.mark.parametrize("d", [1, 2, 3])
def test_partition_of_unity_support_and_collocation(d):
    t = np.linspace(d, 12.0, 500)
    tot = sum(bspline.basis(b, d, t) for b in range(0, 14))
    assert np.max(np.abs(tot - 1.0)) < 1e-12
    # support [t_beta, t_{beta+d+1}] (Remark support)
    tt = np.linspace(-3, 12, 1501)
    v = bspline.basis(3, d, tt)
    assert np.all(np.abs(v[(tt <= 3) | (tt >= 3 + d + 1)]) < 1e-12)
    # N^{alpha-1,d}(t_alpha) = w^{0,d}
    for a in range(1, 8):
        assert abs(bspline.basis(a - 1, d, np.array([float(a)]))[0] - bspline.weights(d)[0]) < 1e-14
