"""Seeded inputs of the learned indicator: initial network parameters and the training cells.

Random draws only: the network's arithmetic, its features and its training live in the library
(and, for checking, in the oracle).
"""
import numpy as np

from . import structures as st

NQ, NH = 16, 64
# parameter block: mu[16] sig[16] W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3
OFF = dict(mu=0, sig=16, W1=32, b1=32 + NH * NQ, W2=32 + NH * NQ + NH, b2=32 + NH * NQ + NH + NH * NH,
           w3=32 + NH * NQ + 2 * NH + NH * NH, b3=32 + NH * NQ + 3 * NH + NH * NH)
NPARAMS = OFF["b3"] + 1


def mlp_init(seed, b3=-5.0):
    """Glorot-uniform weights, zero hidden biases, output bias b3, mu = 0, sig = 1 (to be replaced
    by the training set's feature statistics)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS)
    p[OFF["sig"]:OFF["sig"] + NQ] = 1.0
    p[OFF["W1"]:OFF["b1"]] = rng.uniform(-1, 1, NH * NQ) * np.sqrt(6.0 / (NQ + NH))
    p[OFF["W2"]:OFF["b2"]] = rng.uniform(-1, 1, NH * NH) * np.sqrt(6.0 / (2 * NH))
    p[OFF["w3"]:OFF["b3"]] = rng.uniform(-1, 1, NH) * np.sqrt(6.0 / (NH + 1))
    p[OFF["b3"]] = b3
    return p


def training_cells(n_cells=200, nc=8, a=3.16, seed=6004):
    """Seeded strained and defected bcc cells: per-axis strain U(-5 %, 5 %), Gaussian noise
    sigma U(0.03, 0.15) A, and 0-6 point defects, each a vacancy or a tetrahedral-site
    interstitial with equal odds. Returns a list of (pos (n, 3), box (3,))."""
    rng = np.random.default_rng(seed)
    cells = []
    for _ in range(n_cells):
        ref, box = st.bcc(a, nc)
        n_def = int(rng.integers(0, 7))
        keep = np.ones(len(ref), dtype=bool)
        extra = []
        for _ in range(n_def):
            site = int(rng.integers(0, len(ref)))
            if rng.uniform() < 0.5:
                keep[site] = False
            else:
                # tetrahedral site (a/2, a/4, 0) of the cube at this lattice site
                extra.append((ref[site] + np.array([0.5, 0.25, 0.0]) * a) % box)
        pos = ref[keep]
        if extra:
            pos = np.concatenate([pos, np.array(extra)])
        pos = st.gaussian_displace(pos, float(rng.uniform(0.03, 0.15)), rng)
        pos, box = st.strain_cell(pos, box, np.diag(rng.uniform(-0.05, 0.05, 3)))
        cells.append((pos % box, box))
    return cells
