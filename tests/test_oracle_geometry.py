"""Pins of the oracle's neighbour sets and CSP^list (B3)."""
import numpy as np
import pytest

import synth


def _brute_numpy(pos, box, r):
    pos = pos - box * np.floor(pos / box)
    d = pos[None, :, :] - pos[:, None, :]
    d -= box * np.rint(d / box)
    d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
    np.fill_diagonal(d2, np.inf)
    return [np.nonzero(row < r * r)[0] for row in d2]


@pytest.mark.parametrize("nc,r", [(4, 5.5), (8, 7.0), (9, 6.5)])
def test_nblist_matches_numpy_bruteforce(oracle, nc, r):
    pos, box = synth.bcc(3.16, nc)
    pos = synth.gaussian_displace(pos, 0.1, np.random.default_rng(nc)) + 30.0  # unwrapped input
    got = oracle.nblist(pos, box, r)
    want = _brute_numpy(pos, box, r)
    assert all(np.array_equal(g, w) for g, w in zip(got, want))


def test_nblist_shell_counts(oracle):
    """Static lattice shell sums: bcc a=3.16 has 58 neighbours within 5.5 and 6.0 A, 64 within 6.5,
    88 within 7.0; fcc a=3.61 has 54 within 5.5 and 78 within 6.0."""
    pos, box = synth.bcc(3.16, 8)
    for r, k in ((5.5, 58), (6.0, 58), (6.5, 64), (7.0, 88)):
        assert {len(v) for v in oracle.nblist(pos, box, r)} == {k}
    pos, box = synth.fcc(3.61, 6)
    for r, k in ((5.5, 54), (6.0, 78)):
        assert {len(v) for v in oracle.nblist(pos, box, r)} == {k}


def test_nblist_box_error(oracle):
    pos, box = synth.bcc(3.16, 3)
    with pytest.raises(oracle.OracleError):
        oracle.nblist(pos, box, 5.0)


def _csp_g(pos, box, lst):
    """g_i of (B3) from a pair list, in numpy."""
    u = lambda i, j: (pos[j] - pos[i]) - box * np.rint((pos[j] - pos[i]) / box)
    g = np.zeros(len(pos))
    for i in range(len(pos)):
        for t in range(lst.shape[1]):
            v = u(i, lst[i, t]) + u(i, lst[i, t ^ 1])
            g[i] += 0.5 * v @ v
    return g


@pytest.mark.parametrize("lattice,nc,n_csp,a,factor", [("bcc", 4, 8, 3.16, 16.0), ("fcc", 4, 12, 3.61, 24.0)])
def test_csp_list_lattice_facts(oracle, lattice, nc, n_csp, a, factor):
    pos, box = (synth.bcc if lattice == "bcc" else synth.fcc)(a, nc)
    lst = oracle.csp_pairs(pos, box, n_csp)
    n = len(pos)
    # opposite partners: u_a + u_b = 0 in the perfect lattice; the list is an involution
    g = _csp_g(pos, box, lst)
    assert np.abs(g).max() < 1e-24
    assert all(len(set(row)) == n_csp for row in lst)
    # displacing the centre by delta: every pair gives |2 delta|^2 -> (n_csp/2) * 4 |delta|^2
    delta = np.array([0.031, -0.017, 0.022])
    p2 = pos.copy()
    p2[5] += delta
    g2 = _csp_g(p2, box, lst)
    assert g2[5] == pytest.approx(factor * delta @ delta, rel=1e-10)
    # a displaced listed neighbour shows up once in the centre's CSP: |delta|^2
    j = lst[7, 0]
    p3 = pos.copy()
    p3[j] += delta
    assert _csp_g(p3, box, lst)[7] == pytest.approx(delta @ delta, rel=1e-10)
    # the oracle's own g inside the full evaluation agrees with the numpy (B3) sum
    from tests.helpers import EAM, small_ace
    sysd = dict(pos=p2, box=box, eam=EAM, ace=small_ace(), sw=dict(d_lo=1e9, d_hi=2e9, r_w=5.5, d0=0.0,
                                                                    n_csp=n_csp))
    aux = oracle.evaluate(sysd, csp=lst, skip=2)["aux"]
    assert np.allclose(aux["g"], g2, rtol=1e-12, atol=1e-15)
    assert n == len(lst)


def test_csp_list_translation_invariant(oracle):
    pos, box = synth.bcc(3.16, 5)
    pos = synth.gaussian_displace(pos, 0.04, np.random.default_rng(1))
    a = oracle.csp_pairs(pos, box, 8)
    b = oracle.csp_pairs(pos + np.array([0.37, -1.9, 2.25]), box, 8)
    # translation changes rounding only: the selected pairs (as sets) are the same
    assert all({frozenset(r[2 * p:2 * p + 2]) for p in range(4)} == {frozenset(s[2 * p:2 * p + 2]) for p in range(4)}
               for r, s in zip(a, b))
