"""Pins of the oracle's Eq.(4) operators: the printed coefficients, polynomial
exactness, the Fourier symbol and D- = -(D+)^T under the zero-halo rules."""
import json
import os

import numpy as np
import pytest

import oracle
from helpers import modified_wavenumber

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_impulse_response_is_eq4():
    """A unit impulse through D+ returns the Eq.(4) weights at the right offsets."""
    c1 = GOLD["eq4_stencil"]["coeff_half"]
    c2 = GOLD["eq4_stencil"]["coeff_three_halves"]
    n, m, h = 16, 7, 1.0
    f = np.zeros(n)
    f[m] = 1.0
    out = oracle.deriv1d(f, h, plus=True)
    # D+ f at slot i (position i+1/2): c1 (f[i+1]-f[i]) + c2 (f[i+2]-f[i-1])
    want = np.zeros(n)
    want[m - 1] = c1
    want[m] = -c1
    want[m - 2] = c2
    want[m + 1] = -c2
    assert np.array_equal(out, want)
    # D- on half samples: c1 (g[i]-g[i-1]) + c2 (g[i+1]-g[i-2])
    out = oracle.deriv1d(f, h, plus=False)
    want = np.zeros(n)
    want[m] = c1
    want[m + 1] = -c1
    want[m - 1] = c2
    want[m + 2] = -c2
    assert np.array_equal(out, want)


@pytest.mark.parametrize("h", [1.0, 10.0, 0.37])
def test_cubic_exact(h):
    """Away from the edges both operators differentiate cubics exactly."""
    rng = np.random.default_rng(1)
    a = rng.standard_normal(4)
    n = 24
    p = lambda x: a[0] + a[1] * x + a[2] * x ** 2 + a[3] * x ** 3
    dp = lambda x: a[1] + 2 * a[2] * x + 3 * a[3] * x ** 2
    xi = np.arange(n) * h
    out = oracle.deriv1d(p(xi), h, plus=True)
    sl = slice(2, n - 3)
    np.testing.assert_allclose(out[sl], dp(xi[sl] + h / 2), rtol=1e-12, atol=1e-12)
    xh = (np.arange(n) + 0.5) * h
    out = oracle.deriv1d(p(xh), h, plus=False)
    sl = slice(2, n - 2)
    np.testing.assert_allclose(out[sl], dp(xi[sl]), rtol=1e-12, atol=1e-12)


def test_quartic_not_exact_and_order():
    """Fourth order: the error on sin(kx) falls ~16x when h halves."""
    errs = []
    for n in (40, 80):
        h = 1.0 / n
        x = np.arange(n) * h
        f = np.sin(2 * np.pi * 3 * x)
        out = oracle.deriv1d(f, h, plus=True)
        sl = slice(3, n - 4)
        exact = 2 * np.pi * 3 * np.cos(2 * np.pi * 3 * (x[sl] + h / 2))
        errs.append(np.max(np.abs(out[sl] - exact)))
    assert 13.0 < errs[0] / errs[1] < 19.0


@pytest.mark.parametrize("kh", [0.3, 1.1, 2.5, np.pi])
def test_fourier_symbol(kh):
    h = 2.0
    k = kh / h
    n = 64
    x = np.arange(n) * h
    out = oracle.deriv1d(np.sin(k * x), h, plus=True)
    sl = slice(2, n - 3)
    want = modified_wavenumber(k, h) * np.cos(k * (x[sl] + h / 2))
    np.testing.assert_allclose(out[sl], want, rtol=0, atol=1e-13 * (1 + abs(modified_wavenumber(k, h))))


def test_adjointness_zero_halo():
    """<D+ f, g> = -<f, D- g>, with g's last (pinned) slot excluded."""
    rng = np.random.default_rng(3)
    for n in (5, 6, 17):
        f = rng.standard_normal(n)
        g = rng.standard_normal(n)
        g[n - 1] = 0.0
        lhs = np.dot(oracle.deriv1d(f, 0.7, plus=True)[: n - 1], g[: n - 1])
        rhs = -np.dot(f, oracle.deriv1d(g, 0.7, plus=False))
        assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + 1.0)


def test_pinned_slot_ignored():
    """The last half slot is pinned: its input value never reaches D-."""
    rng = np.random.default_rng(4)
    g = rng.standard_normal(12)
    g2 = g.copy()
    g2[-1] = 1e9
    assert np.array_equal(oracle.deriv1d(g, 1.0, plus=False), oracle.deriv1d(g2, 1.0, plus=False))
