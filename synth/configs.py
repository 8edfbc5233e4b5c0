"""Seeded recipes for the five workloads.

A recipe fixes the structure (lattice, size, noise, planted defect), the random
draws of the potentials and the switching thresholds. Scalars that have to be
derived from the potentials themselves (zero-pressure c0, the two-body fit of
the ACE radial channels, the many-body coefficient scale, d_lo / d_hi, the size
of the planted defect) are not computed here: they are read from
synth/data/cfg<k>.json, which is written by oracle/calibrate.py.

Seeds per workload k: structure 1000+k, EAM 2000+k, ACE 3000+k, velocities 4000+k,
defects 5000+k.
"""
import json
import os

import numpy as np

from . import structures as st
from .basis import ace_basis

CONFIG_NAMES = {
    1: "bcc8_fp64_n8l4",
    2: "bcc40_screwdipole_fp32_n12l6",
    3: "batch64_ragged_fp32_n8l4caps",
    4: "bcc80_vacancy_clusters_learned",
    5: "fcc80_penny_crack_fp32_n12l6",
}

_DATA = os.path.join(os.path.dirname(__file__), "data")

# EAM draw ranges (analytic Finnis-Sinclair form); c0 is solved for zero pressure.
# EAM draws: the Finnis-Sinclair form with tungsten-like nominal values (density cutoff 4.400224 A,
# pair cutoff 3.25 A; bcc ground state at a = 3.165 A, cohesive energy 8.90 eV); A is drawn +-2 %
# and beta in [0, 0.02], c0 is then solved for zero pressure at the workload's lattice constant.
# fcc: a copper-like set of the same form (density cutoff between the 2nd and 3rd fcc shells, pair cutoff
# between the 1st and 2nd), fitted by lattice sums at a = 3.61 A to E_coh 3.54 eV and positive C', C44 with
# bcc 75 meV/atom above fcc.
_EAM_NOMINAL = {
    "bcc": dict(A=1.896373, c1=-33.7665655, c2=6.2541999, r_rho=4.400224, r_phi=3.25),
    "fcc": dict(A=1.27726, c1=-11.7176, c2=2.37883, r_rho=4.0, r_phi=3.4),
}
_EAM_RANGES = {"bcc": dict(A=(0.98, 1.02), beta=(0.0, 0.02)), "fcc": dict(A=(0.98, 1.02), beta=(0.0, 0.02))}

_RECIPES = {
    1: dict(lattice="bcc", a=3.16, nc=8, sigma=0.05, mass=183.84, n_max=8, l_max=4, caps={},
            precision="fp64", r_w=6.5, skin=0.5, dt=1e-3, steps=10, T=300.0,
            defect=dict(kind="local_noise", radius=3.0, sigma=0.30)),
    2: dict(lattice="bcc", a=3.16, nc=40, sigma=0.08, mass=183.84, n_max=12, l_max=6, caps={},
            precision="fp32", r_w=6.5, skin=0.5, dt=1e-3, steps=1000, T=300.0,
            defect=dict(kind="screw_dipole", d_sep=12.0)),
    3: dict(lattice="batch", a=3.16, nc=None, sigma=0.10, mass=183.84, n_max=8, l_max=4,
            caps=dict(n1_cap=8, n2_cap=8, l2_cap=4, n3_cap=6, l3_cap=4),
            precision="fp32", r_w=6.5, skin=0.5, dt=1e-3, steps=0, T=300.0, defect=None),
    4: dict(lattice="bcc", a=3.16, nc=80, sigma=0.05, mass=183.84, n_max=12, l_max=6, caps={},
            precision="fp32", r_w=6.5, skin=0.5, dt=1e-3, steps=1000, T=300.0,
            defect=dict(kind="vacancy_clusters", n=20)),
    5: dict(lattice="fcc", a=3.61, nc=80, sigma=0.05, mass=63.546, n_max=12, l_max=6, caps={},
            precision="fp32", r_w=6.5, skin=0.5, dt=1e-3, steps=1000, T=300.0,
            defect=dict(kind="penny_crack", radius=40.0, half_width=1.0)),
}


def load_config(k):
    """Calibrated scalars of workload k (empty dict when not calibrated yet)."""
    path = os.path.join(_DATA, "cfg%d.json" % k)
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def recipe(k):
    return dict(_RECIPES[k])


def eam_draw(k, lattice):
    """Seeded Finnis-Sinclair EAM parameters of workload k (c0 still to be solved)."""
    if lattice not in _EAM_NOMINAL:
        raise NotImplementedError("no EAM parameter set for the %s lattice" % lattice)
    rng = np.random.default_rng(2000 + k)
    p = dict(_EAM_NOMINAL[lattice])
    p["A"] *= float(rng.uniform(*_EAM_RANGES[lattice]["A"]))
    p["beta"] = float(rng.uniform(*_EAM_RANGES[lattice]["beta"]))
    return p


def ace_unit_draw(k, n_funcs):
    """Seeded N(0,1) vector that, times the calibrated scale, gives the order-2/3 coefficients."""
    return np.random.default_rng(3000 + k).normal(0.0, 1.0, n_funcs)


def _structure(rc, k, cal, nc_override=None, defect_override=None):
    """(pos, box, pos_ref): pos_ref is the lattice with the planted defect, before the seeded
    Gaussian noise; pos = pos_ref + noise. The CSP opposite-neighbour pairs are detected on
    pos_ref (the initial structure)."""
    rng = np.random.default_rng(1000 + k)
    nc = nc_override or rc["nc"]
    maker = st.bcc if rc["lattice"] == "bcc" else st.fcc
    pos, box = maker(rc["a"], nc)
    d = rc["defect"]
    drng = np.random.default_rng(5000 + k)
    if d is not None:
        d = dict(d)
        d.update(cal.get("defect", {}))
        d.update(defect_override or {})
        if d["kind"] == "screw_dipole":
            b = rc["a"] * np.sqrt(3.0) / 2.0
            off = drng.uniform(-0.25, 0.25, 2) * rc["a"]
            xc, yc = 0.5 * box[0] + off[0], 0.5 * box[1] + 0.25 * rc["a"] + off[1]
            pos = st.screw_dipole_z(pos, box, b, xc - 0.5 * d["d_sep"], xc + 0.5 * d["d_sep"], yc)
        elif d["kind"] == "vacancy_clusters":
            pos = st.vacancy_clusters(pos, box, d["n"], drng)
        elif d["kind"] == "penny_crack":
            centre = 0.5 * box + drng.uniform(-0.5, 0.5, 3)
            pos = st.penny_crack(pos, box, d["radius"], d["half_width"], centre)
    pos_ref = pos.copy()
    pos = st.gaussian_displace(pos, rc["sigma"], rng)
    if d is not None and d["kind"] == "local_noise":
        # a hot spot: extra noise on top of the reference, after the pairs are fixed
        centre = drng.uniform(0.25, 0.75, 3) * box
        pos = st.local_noise(pos, box, centre, d["radius"], d["sigma"], drng)
    return pos, box, pos_ref


def build_system(k, nc=None, with_velocities=True, defect=None):
    """Everything workload k feeds the method, as float64/int32 numpy arrays.

    nc overrides the number of cells (smaller test variants of the same recipe); defect overrides entries of
    the planted defect (e.g. the penny crack's radius, to set the precise fraction x by the defect's size).
    """
    rc = recipe(k)
    cal = load_config(k)
    lattice = "bcc" if rc["lattice"] in ("bcc", "batch") else "fcc"
    eam = dict(eam_draw(k, lattice))
    eam.update(cal.get("eam", {}))
    eam.setdefault("c0", 47.1346499)
    func = ace_basis(rc["n_max"], rc["l_max"], **rc["caps"])
    n1 = int((func[:, 2] < 0).sum())
    ace_cal = cal.get("ace", {})
    c = ace_unit_draw(k, len(func)) * float(ace_cal.get("c_scale", 0.0))
    c[:n1] = np.asarray(ace_cal.get("c_order1", np.zeros(n1)), dtype=np.float64)[:n1]
    ace = dict(n_max=rc["n_max"], l_max=rc["l_max"], rc=5.5, func=func, c=c,
               b_dens=np.asarray(ace_cal.get("b_dens", np.zeros(rc["n_max"])), dtype=np.float64),
               emb_A=float(eam["A"]), E0=float(ace_cal.get("E0", 0.0)), precision=rc["precision"])
    sw_cal = cal.get("sw", {})
    sw = dict(d_lo=float(sw_cal.get("d_lo", 0.6)), d_hi=float(sw_cal.get("d_hi", 1.6)),
              r_w=rc["r_w"], d0=0.0, n_csp=8 if lattice == "bcc" else 12)
    out = dict(name=CONFIG_NAMES[k], k=k, eam=eam, ace=ace, sw=sw, mass=rc["mass"],
               run=dict(dt=rc["dt"], steps=rc["steps"], T=rc["T"], skin=rc["skin"]))
    if rc["lattice"] == "batch":
        return out
    pos, box, pos_ref = _structure(rc, k, cal, nc, defect)
    out.update(pos=pos, box=box, pos_ref=pos_ref)
    if with_velocities:
        out["vel"] = st.maxwell_velocities(len(pos), rc["mass"], rc["T"], np.random.default_rng(4000 + k))
    return out


def batch_cells(k=3, n_cells=64):
    """Ragged batch of periodic bcc / fcc-like cells for the differentiation workload:
    bcc n^3 (n = 5..10) and fcc n^3 (n = 4..7), seeded diagonal strain +-3 % and
    sigma = 0.1 A noise. Returns a list of (pos, box)."""
    rng = np.random.default_rng(1000 + k)
    cells = []
    for s in range(n_cells):
        if s % 2 == 0:
            n = int(rng.integers(5, 11))
            pos, box = st.bcc(3.16, n)
        else:
            n = int(rng.integers(4, 8))
            pos, box = st.fcc(3.61 * 3.16 / 3.16, n)
        eps = np.diag(rng.uniform(-0.03, 0.03, 3))
        pos, box = st.strain_cell(pos, box, eps)
        pos = st.gaussian_displace(pos, 0.10, rng)
        cells.append((pos, box))
    return cells
