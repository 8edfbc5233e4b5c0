"""Closed-form pins of the oracle's descriptor (Eq. (6)) and of its network forward pass.

Each check takes the oracle module and an optional bound library (`_lib`), so that the same checks
run on the oracle as built and on copies built with a deliberate mistake (tests/test_oracle_pin_strength.py):
a pin that a plausible mistake does not break pins nothing.

Eq. (6): d_i = sum_k g_k w(r_ik) / wbar_i - d0, wbar_i = sum_k w(r_ik), both sums over the atoms within
r_w including k = i (w(0) = 1), w(r) = f_trans(r, r_w - 1, r_w) (App. B). The values below follow from that
definition by hand, not from the oracle's code.
"""
import numpy as np

import synth


def _ftrans(x, lo, hi):
    # Eq. (S1), written out again here only to give the value of w at one shell radius
    if x <= lo:
        return 1.0
    if x >= hi:
        return 0.0
    y = (hi + lo - 2.0 * x) / (hi - lo)
    return 0.5 + 0.9375 * y - 0.625 * y ** 3 + 0.1875 * y ** 5


def uniform_indicator(O, _lib=None):
    """g = c on every atom of a noisy bcc cell: every d_i = c - d0, whatever the weights. The cell has atoms
    inside the weight's transition band, so a sum normalised by anything but sum_k w fails."""
    rng = np.random.default_rng(11)
    ref, box = synth.bcc(3.16, 5)
    pos = synth.gaussian_displace(ref, 0.12, rng)
    c, d0, r_w = 0.37, 0.11, 6.5
    wbar, d = O.descriptor(pos, box, np.full(len(pos), c), r_w, d0, _lib=_lib)
    # the band 5.5 < r < 6.5 is populated: wbar is not an integer
    assert np.abs(wbar - np.rint(wbar)).max() > 0.05
    assert np.abs(d - (c - d0)).max() < 1e-14, np.abs(d - (c - d0)).max()


def perfect_bcc_normalisation(O, _lib=None):
    """Perfect bcc (a = 3.16 A) at r_w = 6.5 A: the shells inside 5.5 A hold 8 + 6 + 12 + 24 + 8 = 58 atoms
    (weight 1), the shell at 2a = 6.32 A holds 6 in the band, the next shell (6.89 A) lies outside; with the
    atom itself wbar = 1 + 58 + 6 w(6.32)."""
    ref, box = synth.bcc(3.16, 5)
    want = 1.0 + 58.0 + 6.0 * _ftrans(6.32, 5.5, 6.5)
    wbar, _ = O.descriptor(ref, box, np.zeros(len(ref)), 6.5, 0.0, _lib=_lib)
    assert np.abs(wbar - want).max() < 1e-12, (wbar[:3], want)


def isolated_atoms(O, _lib=None):
    """Atoms further apart than r_w: wbar = 1 (the atom itself) and d = g - d0."""
    g = np.array([0.0, 0.25, 1.5, 3.0])
    pos = np.array([[1.0, 1.0, 1.0], [11.0, 1.0, 1.0], [1.0, 11.0, 1.0], [11.0, 11.0, 11.0]])
    wbar, d = O.descriptor(pos, [20.0, 20.0, 20.0], g, 4.0, 0.2, _lib=_lib)
    assert np.array_equal(wbar, np.ones(4)), wbar
    assert np.abs(d - (g - 0.2)).max() < 1e-15, d


def two_shells_by_hand(O, _lib=None):
    """Atom 0 at the origin (g = 0.3) with two neighbours at 3 A (g = 1 and 2, weight 1) and three at 6 A
    (g = 4, weight w(6) = f_trans(6; 5.5, 6.5) = 1/2), r_w = 6.5, d0 = 0.25:
    wbar_0 = 1 + 2 + 3/2 = 4.5, d_0 = (0.3 + 1 + 2 + 3 * 4 / 2) / 4.5 - 0.25 = 9.3 / 4.5 - 0.25."""
    c = 20.0
    pos = np.array([[0, 0, 0], [3, 0, 0], [-3, 0, 0], [0, 6, 0], [0, -6, 0], [0, 0, 6]], float) + c
    g = np.array([0.3, 1.0, 2.0, 4.0, 4.0, 4.0])
    wbar, d = O.descriptor(pos, [40.0, 40.0, 40.0], g, 6.5, 0.25, _lib=_lib)
    assert abs(wbar[0] - 4.5) < 1e-15, wbar[0]
    assert abs(d[0] - (9.3 / 4.5 - 0.25)) < 1e-14, d[0]


DESCRIPTOR_PINS = (uniform_indicator, perfect_bcc_normalisation, isolated_atoms, two_shells_by_hand)


def _silu(a):
    return a / (1.0 + np.exp(-a))


def _dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def one_path_network(O, _lib=None):
    """A 16-64-64-1 network whose weights are zero except one path, feature 3 -> hidden unit 0 of layer 1 ->
    unit 5 of layer 2 -> output, with a normalisation of feature 3. Its output, g = softplus(o) and dg/dq
    follow by hand:
      z3 = (q3 - mu3) / sig3, a1 = W1[0][3] z3 + b1[0], a2 = W2[5][0] silu(a1) + b2[5],
      o = w3[5] silu(a2) + b3, g = log(1 + e^o),
      dg/dq3 = sigmoid(o) w3[5] silu'(a2) W2[5][0] silu'(a1) W1[0][3] / sig3, the other dg/dq_f = 0.
    The path's units are placed so that a transposed W1 or W2 reads a zero instead, and a1 > 0 > a2 so that
    another activation than SiLU changes the value."""
    NQ, NH = 16, 64
    MU, SIG, W1 = 0, 16, 32
    B1 = W1 + NH * NQ
    W2 = B1 + NH
    B2 = W2 + NH * NH
    W3 = B2 + NH
    B3 = W3 + NH
    P = np.zeros(B3 + 1)
    P[SIG:SIG + NQ] = 1.0
    P[MU + 3], P[SIG + 3] = 0.5, 2.0
    P[W1 + 0 * NQ + 3] = 1.5
    P[B1 + 0] = -0.2
    P[W2 + 5 * NH + 0] = -0.8
    P[B2 + 5] = 0.1
    P[W3 + 5] = 2.0
    P[B3] = -0.3
    q = np.linspace(0.7, 2.2, NQ)
    q[3] = 1.1
    z3 = (q[3] - 0.5) / 2.0
    a1 = 1.5 * z3 - 0.2
    a2 = -0.8 * _silu(a1) + 0.1
    o = 2.0 * _silu(a2) - 0.3
    g = np.log1p(np.exp(o))
    dg3 = 1.0 / (1.0 + np.exp(-o)) * 2.0 * _dsilu(a2) * -0.8 * _dsilu(a1) * 1.5 / 2.0
    assert a1 > 0 > a2
    oo, gg, dg = O.mlp_forward(q[None], P, _lib=_lib)
    assert abs(oo[0] - o) < 1e-14, (oo[0], o)
    assert abs(gg[0] - g) < 1e-14, (gg[0], g)
    want = np.zeros(NQ)
    want[3] = dg3
    assert np.abs(dg[0] - want).max() < 1e-14, (dg[0], want)


MLP_PINS = (one_path_network,)
