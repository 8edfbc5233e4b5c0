"""Pins of the oracle's elementary functions against the paper and independent mathematics."""
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y
from sympy.physics.wigner import wigner_3j

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_ftrans_printed_values(oracle):
    """Eq. (S1): exact dyadic values and the two plateaus (golden fixture)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "ftrans_values.txt"))
    for x, lo, hi, want in rows:
        got = oracle.ftrans(x, lo, hi)
        if want in (0.896484375, 0.5, 0.103515625, 1.0, 0.0):
            assert got == want
        else:
            assert abs(got - want) < 1e-15


def test_ftrans_smoothness(oracle):
    """Eq. (S1): monotone, f'(mid) = -1.875/(hi-lo), f' and f'' vanish at both ends."""
    lo, hi = 1.3, 2.9
    xs = np.linspace(lo, hi, 201)
    f = np.array([oracle.ftrans(x, lo, hi) for x in xs])
    assert np.all(np.diff(f) <= 0)
    assert oracle.ftrans_d(0.5 * (lo + hi), lo, hi) == pytest.approx(-1.875 / (hi - lo), rel=1e-14)
    for x0, s in ((lo, 1.0), (hi, -1.0)):
        e = 1e-3
        # one-sided: f(x0 + s e) - f(x0) = O(e^3) since f' = f'' = 0 at the ends
        assert abs(oracle.ftrans(x0 + s * e, lo, hi) - oracle.ftrans(x0, lo, hi)) < 5 * e ** 3 * 1.875 * 8 / (hi - lo) ** 3
    h = 1e-6
    for x in np.linspace(lo + 0.01, hi - 0.01, 17):
        fd = (oracle.ftrans(x + h, lo, hi) - oracle.ftrans(x - h, lo, hi)) / (2 * h)
        assert oracle.ftrans_d(x, lo, hi) == pytest.approx(fd, abs=1e-8)


def _w000_closed(l1, l2, l3):
    """(l1 l2 l3; 0 0 0) for even J = l1 + l2 + l3 (textbook closed form, no Racah sum)."""
    J = l1 + l2 + l3
    if J % 2:
        return 0.0
    g = J // 2
    f = math.factorial
    return (-1) ** g * math.sqrt(f(J - 2 * l1) * f(J - 2 * l2) * f(J - 2 * l3) / f(J + 1)) * f(g) / (
        f(g - l1) * f(g - l2) * f(g - l3))


def test_wigner3j_against_sympy(oracle):
    rng = np.random.default_rng(7)
    for _ in range(300):
        l1, l2 = rng.integers(0, 7, 2)
        l3 = int(rng.integers(abs(l1 - l2), min(l1 + l2, 6) + 1))
        m1 = int(rng.integers(-l1, l1 + 1))
        m2 = int(rng.integers(-l2, l2 + 1))
        m3 = -m1 - m2
        want = float(wigner_3j(int(l1), int(l2), l3, m1, m2, m3)) if abs(m3) <= l3 else 0.0
        assert oracle.wigner3j(int(l1), int(l2), l3, m1, m2, m3) == pytest.approx(want, abs=1e-14)


def test_wigner3j_special_values_and_orthogonality(oracle):
    for l in range(7):
        for m in range(-l, l + 1):
            assert oracle.wigner3j(l, l, 0, m, -m, 0) == pytest.approx((-1) ** (l - m) / math.sqrt(2 * l + 1), abs=1e-15)
    for l1 in range(5):
        for l2 in range(5):
            for l3 in range(abs(l1 - l2), l1 + l2 + 1):
                assert oracle.wigner3j(l1, l2, l3, 0, 0, 0) == pytest.approx(_w000_closed(l1, l2, l3), abs=1e-15)
                for m3 in range(-l3, l3 + 1):
                    s = sum(oracle.wigner3j(l1, l2, l3, m1, -m1 - m3, m3) ** 2
                            for m1 in range(-l1, l1 + 1) if abs(m1 + m3) <= l2)
                    assert (2 * l3 + 1) * s == pytest.approx(1.0, abs=1e-13)


def test_ylm_against_scipy_and_addition_theorem(oracle):
    rng = np.random.default_rng(3)
    for _ in range(20):
        u = rng.normal(size=3) * rng.uniform(0.5, 5)
        r = np.linalg.norm(u)
        th, ph = math.acos(u[2] / r), math.atan2(u[1], u[0])
        Y, dY = oracle.ylm(6, u)
        for l in range(7):
            for m in range(-l, l + 1):
                assert Y[l * l + l + m] == pytest.approx(complex(sph_harm_y(l, m, th, ph)), abs=1e-13)
            s = sum(abs(Y[l * l + l + m]) ** 2 for m in range(-l, l + 1))
            assert s == pytest.approx((2 * l + 1) / (4 * math.pi), rel=1e-13)
    u = np.array([0.3, -1.2, 0.7])
    Y, _ = oracle.ylm(2, u)
    r = np.linalg.norm(u)
    assert Y[0] == pytest.approx(1 / math.sqrt(4 * math.pi))
    assert Y[2] == pytest.approx(math.sqrt(3 / (4 * math.pi)) * u[2] / r)
    assert Y[3] == pytest.approx(-math.sqrt(3 / (8 * math.pi)) * (u[0] + 1j * u[1]) / r)


def test_ylm_gradient_fd(oracle):
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(5):
        u = rng.normal(size=3) * 2
        _, dY = oracle.ylm(6, u)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (oracle.ylm(6, u + e)[0] - oracle.ylm(6, u - e)[0]) / (2 * h)
            assert np.allclose(dY[:, a], fd, atol=1e-8)


def test_ylm_orthonormal_quadrature(oracle):
    x, w = np.polynomial.legendre.leggauss(16)
    nphi = 32
    phis = 2 * np.pi * np.arange(nphi) / nphi
    nlm = 49
    G = np.zeros((nlm, nlm), complex)
    for xi, wi in zip(x, w):
        st = math.sqrt(1 - xi * xi)
        for p in phis:
            Y, _ = oracle.ylm(6, np.array([st * math.cos(p), st * math.sin(p), xi]))
            G += wi * (2 * np.pi / nphi) * np.outer(Y, Y.conj())
    assert np.allclose(G, np.eye(nlm), atol=1e-12)


def test_radial_chebyshev(oracle):
    rc = 5.5
    for r in np.linspace(0.3, 5.49, 23):
        g, dg = oracle.radial(12, rc, r)
        x = 2 * r / rc - 1
        fc = 0.5 * (1 + math.cos(math.pi * r / rc))
        for n in range(12):
            T = np.polynomial.chebyshev.chebval(x, [0] * n + [1])
            assert g[n] == pytest.approx(T * fc, abs=1e-14)
        h = 1e-6
        fd = (oracle.radial(12, rc, r + h)[0] - oracle.radial(12, rc, r - h)[0]) / (2 * h)
        assert np.allclose(dg, fd, atol=1e-7)
    g, dg = oracle.radial(8, rc, rc)
    assert np.all(g == 0) and np.all(dg == 0)
