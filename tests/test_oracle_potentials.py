"""Pins of the oracle's EAM (B1)-(B2) and ACE site energy against closed forms and invariances."""
import math

import numpy as np
import pytest

import synth
from tests.helpers import EAM, rotation, small_ace
from tests.test_oracle_math import _w000_closed

SHELLS_BCC = [(1.0, 8), (2 / math.sqrt(3), 6), (math.sqrt(8 / 3), 12), (math.sqrt(11 / 3), 24), (2.0, 8)]


def _fs(r, p):
    x, y = r - p["r_rho"], r - p["r_phi"]
    z = x * x + p["beta"] * x ** 3 / p["r_rho"] if r < p["r_rho"] else 0.0
    ph = y * y * (p["c0"] + p["c1"] * r + p["c2"] * r * r) if r < p["r_phi"] else 0.0
    return z, ph


def _sys(pos, box, ace=None, lam_sw=None):
    return dict(pos=pos, box=box, eam=dict(EAM), ace=ace or small_ace(),
                sw=lam_sw or dict(d_lo=1e9, d_hi=2e9, r_w=5.5, d0=0.0, n_csp=8))


def test_eam_perfect_lattice_shell_sum(oracle):
    """(B1) on a perfect bcc lattice: E = xi(sum_s n_s zeta(r_s)) + 1/2 sum_s n_s Phi(r_s), F = 0."""
    a = 3.16
    pos, box = synth.bcc(a, 5)
    r = oracle.evaluate(_sys(pos, box), lam_mode=1)
    nn = a * math.sqrt(3) / 2
    z = sum(k * _fs(f * nn, EAM)[0] for f, k in SHELLS_BCC)
    ph = sum(k * _fs(f * nn, EAM)[1] for f, k in SHELLS_BCC)
    want = -EAM["A"] * math.sqrt(z) + 0.5 * ph
    assert np.allclose(r["E_atom"], want, rtol=1e-13)
    assert np.abs(r["F"]).max() < 1e-11


def test_eam_dimer(oracle):
    """Two atoms in a large box: E = 2 xi(zeta(r)) + Phi(r)."""
    box = np.array([20.0, 20.0, 20.0])
    for d in (2.3, 3.7, 5.2):
        pos = np.array([[1.0, 2.0, 3.0], [1.0 + d * 0.6, 2.0 + d * 0.8, 3.0]])
        r = oracle.evaluate(_sys(pos, box), lam_mode=1)
        z, ph = _fs(d, EAM)
        assert r["E"] == pytest.approx(2 * (-EAM["A"] * math.sqrt(z)) + ph, rel=1e-14)


def test_ace_single_neighbour_closed_forms(oracle):
    """One neighbour at u: B1 = g_n/sqrt(4 pi); B2 = g_n1 g_n2 (2l+1)/(4 pi);
    B3 = g g g sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi)^3) (l1 l2 l3; 0 0 0)."""
    ace = small_ace(8, 4, seed=2)
    u = np.array([[1.1, -2.0, 1.7]])
    out = oracle.ace_env(u, ace)
    g, _ = oracle.radial(8, 5.5, np.linalg.norm(u))
    for f, row in enumerate(ace["func"]):
        n1, l1, n2, l2, n3, l3 = row
        if n2 < 0:
            want = g[n1] / math.sqrt(4 * math.pi)
        elif n3 < 0:
            want = g[n1] * g[n2] * (2 * l1 + 1) / (4 * math.pi)
        else:
            want = g[n1] * g[n2] * g[n3] * math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / (4 * math.pi) ** 3) \
                * _w000_closed(l1, l2, l3)
        assert out["B"][f] == pytest.approx(want, abs=1e-14)


def test_ace_lmax0_radial_products(oracle):
    """With l_max = 0 the product basis reduces to products of radial sums s_n = sum_j g_n(r_j):
    order 2 -> s1 s2 / (4 pi), order 3 (l = 0,0,0) -> s1 s2 s3 / (4 pi)^(3/2)."""
    func = synth.ace_basis(4, 0)
    ace = dict(small_ace(4, 0), func=func, c=np.zeros(len(func)))
    u = np.random.default_rng(1).normal(size=(9, 3)) * 1.6
    out = oracle.ace_env(u, ace)
    s = sum(oracle.radial(4, 5.5, np.linalg.norm(v))[0] for v in u)
    for f, (n1, _, n2, _, n3, _) in enumerate(func):
        want = s[n1] / math.sqrt(4 * math.pi) if n2 < 0 else (
            s[n1] * s[n2] / (4 * math.pi) if n3 < 0 else s[n1] * s[n2] * s[n3] / (4 * math.pi) ** 1.5)
        assert out["B"][f] == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_ace_rotation_permutation_invariance_and_fd(oracle):
    ace = small_ace(8, 4, seed=4, scale=0.003)
    rng = np.random.default_rng(11)
    u = rng.normal(size=(14, 3))
    u *= rng.uniform(2.2, 5.3, (14, 1)) / np.linalg.norm(u, axis=1, keepdims=True)
    base = oracle.ace_env(u, ace)
    rot = oracle.ace_env(u @ rotation(3).T, ace)
    perm = oracle.ace_env(u[rng.permutation(14)], ace)
    assert np.allclose(rot["B"], base["B"], rtol=1e-10, atol=1e-12)
    assert rot["E"] == pytest.approx(base["E"], rel=1e-13)
    assert perm["E"] == pytest.approx(base["E"], rel=1e-13)
    h = 1e-6
    for j in (0, 5, 13):
        for a in range(3):
            up, um = u.copy(), u.copy()
            up[j, a] += h
            um[j, a] -= h
            fd = (oracle.ace_env(up, ace)["E"] - oracle.ace_env(um, ace)["E"]) / (2 * h)
            assert base["dEdu"][j, a] == pytest.approx(fd, abs=2e-8)
    # translation of the whole cluster is not a variable here; the sum of the gradients is the
    # centre's force: it equals minus the sum over neighbours
    assert np.isfinite(base["dEdu"]).all()


def test_ace_imaginary_parts_vanish(oracle):
    """B is real (invariant polynomials): rebuild B2 from the complex A returned by the oracle."""
    ace = small_ace(4, 2, seed=6)
    u = np.random.default_rng(2).normal(size=(7, 3)) * 1.8
    out = oracle.ace_env(u, ace)
    A = out["A"]
    for f, (n1, l, n2, l2, n3, _) in enumerate(ace["func"]):
        if n2 >= 0 and n3 < 0:
            b = sum((-1) ** m * A[n1, l * l + l + m] * A[n2, l * l + l - m] for m in range(-l, l + 1))
            assert abs(b.imag) < 1e-13 and b.real == pytest.approx(out["B"][f], abs=1e-13)
