"""Seeded atomic structures in metal units (Angstrom, atomic mass units, ps).

Positions are returned as float64 arrays of shape (n, 3), atom index order =
((ix * nc + iy) * nc + iz) * n_basis + b, and are NOT wrapped into the box:
wrapping is part of the method and done by the consumers.
"""
import numpy as np

KB_EV = 8.617333262e-5          # Boltzmann constant, eV/K
EV_PER_U_A2_PS2 = 9648.533212   # 1 eV / (u * A^2/ps^2): converts eV/(A u) to A/ps^2

_BCC = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
_FCC = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])


def _cubic(basis, a, nc):
    g = np.array([(i, j, k) for i in range(nc) for j in range(nc) for k in range(nc)], dtype=np.float64)
    pos = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return pos, np.array([a * nc] * 3, dtype=np.float64)


def bcc(a, nc):
    """Perfect body-centred cubic lattice of nc^3 conventional cells."""
    return _cubic(_BCC, a, nc)


def fcc(a, nc):
    """Perfect face-centred cubic lattice of nc^3 conventional cells."""
    return _cubic(_FCC, a, nc)


def gaussian_displace(pos, sigma, rng):
    """i.i.d. Gaussian displacement of every Cartesian component."""
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def screw_dipole_z(pos, box, b, x1, x2, yc):
    """Displacement u_z = b/(2 pi) [atan2(y-yc, x-x1) - atan2(y-yc, x-x2)].

    Two line cores parallel to z at (x1, yc) and (x2, yc) with opposite sign; the
    field jumps by b across the strip yc, x1 < x < x2 between the cores.
    """
    out = pos.copy()
    th1 = np.arctan2(pos[:, 1] - yc, pos[:, 0] - x1)
    th2 = np.arctan2(pos[:, 1] - yc, pos[:, 0] - x2)
    out[:, 2] += b / (2.0 * np.pi) * (th1 - th2)
    return out


def local_noise(pos, box, centre, radius, sigma, rng):
    """Extra Gaussian noise on atoms within `radius` (minimum image) of `centre`."""
    d = pos - centre
    d -= box * np.rint(d / box)
    sel = np.einsum("ij,ij->i", d, d) < radius * radius
    out = pos.copy()
    out[sel] += rng.normal(0.0, sigma, size=(int(sel.sum()), 3))
    return out


def remove_atoms(pos, mask):
    """Drop atoms where mask is True (the remaining atoms keep their order)."""
    return pos[~mask].copy()


def vacancy_clusters(pos, box, n_clusters, rng, min_size=1, max_size=4):
    """Remove n_clusters seeded clusters of 1-4 nearest atoms around random centres."""
    remove = np.zeros(len(pos), dtype=bool)
    for _ in range(n_clusters):
        c = rng.uniform(0.0, 1.0, 3) * box
        k = int(rng.integers(min_size, max_size + 1))
        d = pos - c
        d -= box * np.rint(d / box)
        order = np.argsort(np.einsum("ij,ij->i", d, d), kind="stable")
        remove[order[:k]] = True
    return remove_atoms(pos, remove)


def penny_crack(pos, box, radius, half_width, centre):
    """Remove atoms within a slab |z - zc| < half_width and in-plane distance < radius."""
    d = pos - centre
    d -= box * np.rint(d / box)
    rho2 = d[:, 0] ** 2 + d[:, 1] ** 2
    return remove_atoms(pos, (np.abs(d[:, 2]) < half_width) & (rho2 < radius * radius))


def frenkel_pairs(a, nc, n_pairs, rng):
    """Perfect bcc of nc^3 cells with n_pairs vacancy-interstitial pairs: 2 n_pairs distinct conventional
    cells are drawn; the first n_pairs lose their corner atom, the other n_pairs gain an atom at the
    tetrahedral site (a/2, a/4, 0) from their corner. The atom count stays 2 nc^3; every vacancy is
    removed from its interstitial by the random draw of the cells."""
    pos, box = bcc(a, nc)
    cells = rng.choice(nc ** 3, size=2 * n_pairs, replace=False)
    vac, itl = cells[:n_pairs], cells[n_pairs:]
    keep = np.ones(len(pos), dtype=bool)
    keep[2 * vac] = False  # the corner atom of conventional cell c is atom 2 c
    extra = pos[2 * itl] + np.array([0.5, 0.25, 0.0]) * a
    return np.concatenate([pos[keep], extra]), box


def strain_cell(pos, box, eps):
    """Apply a symmetric strain (3x3, small) to an orthorhombic cell: only the
    diagonal is applied to the box (the cell stays orthorhombic); shear components
    are ignored so the periodic box remains rectangular."""
    f = 1.0 + np.diag(eps)
    return pos * f, box * f


def maxwell_velocities(n, mass, temperature, rng):
    """Maxwell velocities in A/ps; centre-of-mass motion removed and rescaled to
    exactly `temperature` with 3n-3 degrees of freedom."""
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    sig = np.sqrt(KB_EV * temperature / m * EV_PER_U_A2_PS2)
    v = rng.normal(0.0, 1.0, size=(n, 3)) * sig[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ekin = 0.5 * (m[:, None] * v * v).sum() / EV_PER_U_A2_PS2
    t_now = 2.0 * ekin / ((3 * n - 3) * KB_EV)
    return v * np.sqrt(temperature / t_now)


def dilatation_inclusion(pos, box, centre, radius, eps):
    """Spherical inclusion with a uniform dilatation eps inside radius R (u = eps d) and the
    continuous far field u = eps R^3 d / r^3 outside; d is the minimum-image vector from centre."""
    d = pos - centre
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(1))
    f = np.where(r < radius, eps, eps * radius ** 3 / np.maximum(r, 1e-12) ** 3)
    return (pos + f[:, None] * d) % box
