"""Pins of the oracle's learned indicator: the sixteen features (closed forms, invariances), the
network's input gradient and training gradient (central differences), and the AP forces with the
network as g in Eq. (6) (central differences of the energy, zero net force per family, virial)."""
import numpy as np
import pytest

import synth
from synth.learned import OFF, mlp_init
from tests.helpers import rotation, small_system


def _cluster(seed, n=20):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    u *= rng.uniform(2.0, 5.4, n)[:, None] / np.linalg.norm(u, axis=1)[:, None]
    return u


def _features_of(oracle, u):
    """features of an isolated environment: centre at the middle of a big box, neighbours at u"""
    box = np.array([40.0, 40.0, 40.0])
    pos = np.concatenate([[[20.0, 20.0, 20.0]], 20.0 + u])
    return oracle.mlp_features(pos, box)[0]


def test_single_neighbour_closed_forms(oracle):
    """One neighbour at r: q_n = g_n(r), and sum_m |A_nlm|^2 = g_n(r)^2 (2l+1)/(4 pi) (addition theorem)."""
    for r, d in ((2.7, [1, 0, 0]), (4.1, [0.3, -0.5, 0.8]), (5.3, [0, 0, -1])):
        d = np.array(d, float) / np.linalg.norm(d)
        q = _features_of(oracle, (r * d)[None])
        g, _ = oracle.radial(8, 5.5, r)
        assert np.allclose(q[:8], g, rtol=1e-13, atol=1e-15)
        for n in range(2):
            for l in range(1, 5):
                assert q[8 + 4 * n + l - 1] == pytest.approx(g[n] ** 2 * (2 * l + 1) / (4 * np.pi), rel=1e-12)


def test_two_neighbours_closed_form(oracle):
    """Two neighbours at angle theta: sum_m |A_nlm|^2 = (2l+1)/(4 pi) [g1^2 + g2^2 + 2 g1 g2 P_l(cos theta)]."""
    from numpy.polynomial import legendre
    u1 = np.array([3.1, 0.0, 0.0])
    th = 1.1
    u2 = 4.2 * np.array([np.cos(th), np.sin(th), 0.0])
    q = _features_of(oracle, np.array([u1, u2]))
    g1, _ = oracle.radial(8, 5.5, 3.1)
    g2, _ = oracle.radial(8, 5.5, 4.2)
    for n in range(2):
        for l in range(1, 5):
            P = legendre.legval(np.cos(th), [0] * l + [1])
            want = (2 * l + 1) / (4 * np.pi) * (g1[n] ** 2 + g2[n] ** 2 + 2 * g1[n] * g2[n] * P)
            assert q[8 + 4 * n + l - 1] == pytest.approx(want, rel=1e-12)


def test_features_rotation_permutation_invariant(oracle):
    u = _cluster(3)
    q = _features_of(oracle, u)
    R = rotation(5)
    assert np.allclose(_features_of(oracle, u @ R.T), q, rtol=1e-12, atol=1e-14)
    assert np.allclose(_features_of(oracle, u[::-1].copy()), q, rtol=1e-12, atol=1e-14)


def _params(seed=1, q=None):
    p = mlp_init(seed, b3=0.3)
    if q is not None:
        p[OFF["mu"]:OFF["mu"] + 16] = q.mean(0)
        p[OFF["sig"]:OFF["sig"] + 16] = q.std(0) + 1e-3
    return p


def test_network_input_gradient_fd(oracle):
    rng = np.random.default_rng(2)
    q = rng.normal(size=(5, 16))
    p = _params(4)
    o, g, dg = oracle.mlp_forward(q, p)
    assert np.allclose(g, np.log1p(np.exp(o)), rtol=1e-14)
    h = 1e-6
    for s in range(5):
        for f in (0, 7, 12, 15):
            q1, q2 = q.copy(), q.copy()
            q1[s, f] += h
            q2[s, f] -= h
            fd = (oracle.mlp_forward(q1, p, False)[1][s] - oracle.mlp_forward(q2, p, False)[1][s]) / (2 * h)
            assert dg[s, f] == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_training_gradient_fd(oracle):
    """Central differences of the loss mean((o - t)^2) in every kind of parameter."""
    rng = np.random.default_rng(3)
    q = rng.normal(size=(7, 16))
    t = rng.normal(-4.0, 1.0, 7)
    p = _params(6)
    loss, grad = oracle.mlp_loss_grad(q, t, p)
    o, _, _ = oracle.mlp_forward(q, p, False)
    assert loss == pytest.approx(np.mean((o - t) ** 2), rel=1e-14)
    assert np.all(grad[:32] == 0.0)
    h = 1e-6
    picks = [OFF["W1"] + 5, OFF["W1"] + 1000, OFF["b1"] + 3, OFF["W2"] + 77, OFF["W2"] + 4000,
             OFF["b2"] + 60, OFF["w3"] + 9, OFF["b3"]]
    for k in picks:
        p1, p2 = p.copy(), p.copy()
        p1[k] += h
        p2[k] -= h
        fd = (oracle.mlp_loss_grad(q, t, p1)[0] - oracle.mlp_loss_grad(q, t, p2)[0]) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-6, abs=1e-10)


@pytest.fixture(scope="module")
def mlp_sys(oracle):
    s = small_system(nc=4, sigma=0.12)
    q = oracle.mlp_features(s["pos"], s["box"])
    p = _params(7, q)
    # thresholds inside the range of the descriptor so that the transition region is populated
    probe = oracle.evaluate(dict(s, sw=dict(s["sw"], d_lo=1e9, d_hi=2e9)), skip=2, mlp=(p, 5.5))
    d = probe["aux"]["d"]
    s["sw"] = dict(s["sw"], d_lo=float(np.quantile(d, 0.3)), d_hi=float(np.quantile(d, 0.9)))
    return s, p


def test_mlp_indicator_transition_populated(oracle, mlp_sys):
    s, p = mlp_sys
    r = oracle.evaluate(s, mlp=(p, 5.5))
    lam = r["aux"]["lam"]
    assert ((lam > 0) & (lam < 1)).sum() >= 20
    q = oracle.mlp_features(s["pos"], s["box"])
    assert np.allclose(r["aux"]["g"], oracle.mlp_forward(q, p, False)[1], rtol=1e-14)


def test_mlp_indicator_forces_are_minus_energy_gradient(oracle, mlp_sys):
    s, p = mlp_sys
    r = oracle.evaluate(s, skip=0, mlp=(p, 5.5))
    assert np.abs(r["fam"][3]).max() > 1e-3 * np.abs(r["F"]).max()
    h = 1e-5
    for i in (0, 9, 40, 101):
        for a in range(3):
            p1, p2 = s["pos"].copy(), s["pos"].copy()
            p1[i, a] += h
            p2[i, a] -= h
            fd = -(oracle.evaluate(s, pos=p1, mlp=(p, 5.5))["E"] - oracle.evaluate(s, pos=p2, mlp=(p, 5.5))["E"]) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, abs=3e-7 * max(1.0, abs(fd)))


def test_mlp_indicator_families_sum_to_zero_and_virial(oracle, mlp_sys):
    s, p = mlp_sys
    r = oracle.evaluate(s, mlp=(p, 5.5))
    for f in r["fam"]:
        assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(r["fam"]).max() * len(f)
    # virial = -dE/d(strain) by central differences of an affine diagonal strain
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        sp = dict(s, pos=s["pos"] * (1 + e), box=s["box"] * (1 + e))
        sm = dict(s, pos=s["pos"] * (1 - e), box=s["box"] * (1 - e))
        fd = -(oracle.evaluate(sp, mlp=(p, 5.5))["E"] - oracle.evaluate(sm, mlp=(p, 5.5))["E"]) / (2 * h)
        assert r["virial"][a, a] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_training_cells_recipe():
    cells = synth.learned.training_cells(n_cells=12, seed=11)
    sizes = [len(p) for p, _ in cells]
    assert min(sizes) >= 1024 - 6 and max(sizes) <= 1024 + 6
    for p, b in cells:
        assert np.all(p >= 0) and np.all(p < b)
        assert np.all(np.abs(b / (8 * 3.16) - 1) <= 0.05 + 1e-12)
