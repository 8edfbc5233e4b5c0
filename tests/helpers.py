"""Small seeded systems for the tests (built from synth/, the shared input generators)."""
import numpy as np

import synth


def small_ace(n_max=4, l_max=2, seed=0, scale=0.01):
    func = synth.ace_basis(n_max, l_max)
    rng = np.random.default_rng(seed)
    c = rng.normal(0, scale, len(func))
    n1 = int((func[:, 2] < 0).sum())
    c[:n1] = rng.normal(0, 0.3, n1)
    b = np.zeros(n_max)
    b[0], b[1] = 1.0, 0.5
    return dict(n_max=n_max, l_max=l_max, rc=5.5, func=func, c=c, b_dens=b, emb_A=2.0, E0=0.1, precision="fp64")


EAM = dict(A=1.896373, beta=0.01, c0=47.1346499, c1=-33.7665655, c2=6.2541999, r_rho=4.400224, r_phi=3.25)


def small_system(nc=4, sigma=0.12, seed=0, d_lo=0.7, d_hi=1.6, r_w=6.0, lattice="bcc", n_max=4, l_max=2):
    """Periodic bcc (a=3.16) or fcc (a=3.61) cell with Gaussian noise; thresholds that put many atoms in
    the transition region 0 < lambda < 1; CSP pairs to be detected on the perfect lattice."""
    rng = np.random.default_rng(seed)
    if lattice == "bcc":
        ref, box = synth.bcc(3.16, nc)
        n_csp = 8
    else:
        ref, box = synth.fcc(3.61, nc)
        n_csp = 12
    pos = synth.gaussian_displace(ref, sigma, rng)
    return dict(pos=pos, box=box, pos_ref=ref, eam=dict(EAM), ace=small_ace(n_max, l_max, seed),
                sw=dict(d_lo=d_lo, d_hi=d_hi, r_w=r_w, d0=0.0, n_csp=n_csp), mass=183.84,
                run=dict(dt=1e-3), vel=synth.maxwell_velocities(len(pos), 183.84, 300.0, rng))


def rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
