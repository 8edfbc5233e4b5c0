"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bars: neighbour sets and CSP pair lists bit-exact; FP64 forces max|dF|/max|F| <= 1e-11; FP32 ACE
forces rms|dF|/rms|F| <= 2e-5; energies |dE|/N <= 1e-6 eV/atom.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import (TOL_ENERGY, TOL_F32_FORCE, TOL_F64_FORCE, force_err_max, force_err_rms, make_ctx,
                            soa_to_aos, to_dev)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _lt(name, value, tol):
    _say("  %-10s %.3e (bar %.1e)" % (name, value, tol))
    assert value < tol, "%s = %.3e exceeds %.1e" % (name, value, tol)


def _rel(gpu, ref):
    g = gpu.detach().cpu().numpy() if hasattr(gpu, "detach") else np.asarray(gpu)
    ref = np.asarray(ref)
    return float(np.abs(g - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def cfg1():
    return synth.build_system(1)


@pytest.fixture(scope="module")
def cfg1_oracle(oracle, cfg1):
    csp = oracle.csp_pairs(cfg1["pos_ref"], cfg1["box"], 8)
    return csp, oracle.evaluate(cfg1, csp=csp)


def test_nblist_bit_exact(oracle, cfg1):
    import torch
    from paper_2512_07693_amd import ap
    rng = np.random.default_rng(0)
    for r, pos in ((7.0, cfg1["pos"]), (5.5, cfg1["pos"] + rng.uniform(-40, 40, 3)),
                   (6.0, cfg1["pos"] + rng.normal(0, 0.3, cfg1["pos"].shape))):
        _say("nblist r=%.1f n=%d" % (r, len(pos)))
        ctx = ap.Context(len(pos), max_nbr=160)
        cnt, idx = ctx.nblist_build(to_dev(pos), cfg1["box"], r)
        torch.cuda.synchronize()
        cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
        want = oracle.nblist(pos, cfg1["box"], r)
        for i in range(len(pos)):
            assert np.array_equal(np.sort(idx[:cnt[i], i]), want[i]), i
        ctx.close()


@pytest.mark.parametrize("r,cap", [(9.0, 256), (9.0, 320), (7.0, 320)],
                         ids=["staged_one_cell", "unstaged_one_cell", "unstaged_3cells"])
def test_nblist_bit_exact_other_paths(oracle, cfg1, r, cap):
    """The list build's other instantiations on the 1,024-atom cell (box 25.3 A): with more than 256 slots
    per atom the lists go straight to memory instead of through LDS; at r = 9 A a box holds only two cells
    per dimension, so one cell spans it and every candidate takes its own minimum image. Bit-exact sets."""
    import torch
    from paper_2512_07693_amd import ap
    pos = cfg1["pos"]
    _say("nblist r=%.1f max_nbr=%d n=%d" % (r, cap, len(pos)))
    ctx = ap.Context(len(pos), max_nbr=cap)
    cnt, idx = ctx.nblist_build(to_dev(pos), cfg1["box"], r)
    torch.cuda.synchronize()
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    want = oracle.nblist(pos, cfg1["box"], r)
    assert max(len(w) for w in want) > (150 if r > 8 else 80)  # long lists
    for i in range(len(pos)):
        assert np.array_equal(np.sort(idx[:cnt[i], i]), want[i]), i
    ctx.close()


def _oracle_lists(oracle, pos, box, r, cap):
    """The oracle's neighbour sets as an (n, cap) array, ascending, padded with INT32_MAX."""
    n = len(pos)
    cnt = np.zeros(n, np.int32)
    idx = np.zeros(n * cap, np.int32)
    rc = oracle.lib().ora_nblist(n, np.ascontiguousarray(pos), np.ascontiguousarray(box, dtype=np.float64),
                                 float(r), cap, cnt, idx)
    assert rc == 0
    idx = idx.reshape(n, cap)
    idx[np.arange(cap)[None, :] >= cnt[:, None]] = np.iinfo(np.int32).max
    return cnt, idx


@pytest.mark.parametrize("cfg,r_list,max_nbr", [(2, 7.0, 128), (5, 7.0, 160)], ids=["bcc128k", "fcc2M"])
def test_nblist_bit_exact_full_size(oracle, cfg, r_list, max_nbr):
    """Every atom's neighbour set at the evaluation's list radius (max(rc, r_w) + skin) of the 128,000-atom
    and 2,047,229-atom workloads, against the oracle's binned build: the same sets, bit for bit (a pair
    dropped between the cutoff and the skin would only show once atoms move)."""
    import torch
    from paper_2512_07693_amd import ap
    s = synth.build_system(cfg, with_velocities=False)
    n = len(s["pos"])
    _say("nblist full size n=%d r=%.1f" % (n, r_list))
    ctx = ap.Context(n, max_nbr=max_nbr, skin=s["run"]["skin"])
    ctx.set_potential(s["eam"], s["ace"], s["sw"])
    cnt, idx = ctx.nblist_build(to_dev(s["pos"]), s["box"], r_list)
    big = torch.iinfo(torch.int32).max
    slot = torch.arange(max_nbr, device="cuda")[None, :]
    got = torch.where(slot < cnt[:, None].long(), idx.t().long(), big).sort(dim=1).values.int().cpu().numpy()
    cnt = cnt.cpu().numpy()
    ctx.close()
    want_cnt, want = _oracle_lists(oracle, s["pos"], s["box"], r_list, max_nbr)
    _say("  mean count %.2f, max %d" % (want_cnt.mean(), want_cnt.max()))
    assert np.array_equal(cnt, want_cnt)
    assert np.array_equal(got, want)


def test_nblist_parts_in_index_order():
    """The list build's slot order on the 128,000-atom workload: every atom's list holds first the neighbours
    inside max(r_rho, r_phi) + skin, then the rest, and each of the two parts is in ascending atom index (lists of
    up to 256 slots). Distances from the positions in FP64 (atoms with a pair within 1e-9 A^2 of the
    part boundary are left out)."""
    import torch
    from paper_2512_07693_amd import ap
    s = synth.build_system(2, with_velocities=False)
    n, r_list, cap = len(s["pos"]), 7.0, 128
    _say("nblist order n=%d" % n)
    ctx = ap.Context(n, max_nbr=cap, skin=s["run"]["skin"])
    ctx.set_potential(s["eam"], s["ace"], s["sw"])
    cnt, idx = ctx.nblist_build(to_dev(s["pos"]), s["box"], r_list)
    torch.cuda.synchronize()
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    ctx.close()
    rs2 = (max(s["eam"]["r_rho"], s["eam"]["r_phi"]) + s["run"]["skin"]) ** 2
    box = np.asarray(s["box"], float)
    pos = np.asarray(s["pos"], float)
    valid = np.arange(cap)[:, None] < cnt[None, :]
    inner = np.zeros((cap, n), bool)
    border = np.zeros(n, bool)
    for q in range(cap):
        u = pos[np.where(valid[q], idx[q], 0)] - pos
        u -= box * np.rint(u / box)
        d2 = (u * u).sum(axis=1)
        inner[q] = valid[q] & (d2 < rs2)
        border |= valid[q] & (np.abs(d2 - rs2) < 1e-9)
    ks = inner.sum(axis=0)
    # the inner part is a prefix of every list
    assert np.array_equal(inner[:, ~border], (np.arange(cap)[:, None] < ks[None, :])[:, ~border])
    # within each part the indices rise from slot to slot
    pair = valid[1:] & (np.arange(1, cap)[:, None] != ks[None, :])
    rise = idx[1:].astype(np.int64) > idx[:-1].astype(np.int64)
    assert np.all(rise | ~pair)
    assert int(border.sum()) < n // 100 and ks.min() > 0 and (cnt - ks).min() > 0


def _near_errors(s, want, F):
    """FP32 error measures over the atoms that carry FP32 ACE terms: the precise atoms and every atom within
    the ACE cutoff of one (the rest of the cell is FP64 throughout)."""
    from scipy.spatial import cKDTree
    box = np.asarray(s["box"], float)
    p = np.mod(s["pos"], box)
    p[p >= box] = 0.0
    prec = np.nonzero(want["aux"]["lam"] < 1)[0]
    tree = cKDTree(p, boxsize=box)
    near = np.zeros(len(p), bool)
    near[prec] = True
    for lst in tree.query_ball_point(p[prec], s["ace"]["rc"]):
        near[lst] = True
    dF, Fr = F[near] - want["F"][near], want["F"][near]
    rms = float(np.sqrt((dF ** 2).mean()) / np.sqrt((Fr ** 2).mean()))
    mx = float(np.abs(dF).max() / np.abs(Fr).max())
    return int(near.sum()), rms, mx


def test_csp_pairs_bit_exact(oracle, cfg1, cfg1_oracle):
    _say("csp pairs cfg1")
    ctx, csp = make_ctx(cfg1)
    assert np.array_equal(csp.cpu().numpy(), cfg1_oracle[0])
    ctx.close()


def test_switching_matches_oracle(cfg1, cfg1_oracle):
    _say("switch_eval cfg1")
    ctx, _ = make_ctx(cfg1)
    out = ctx.switch_eval(to_dev(cfg1["pos"]), cfg1["box"])
    aux = cfg1_oracle[1]["aux"]
    for k in ("g", "d", "wbar", "lam", "dlam"):
        assert np.allclose(out[k].cpu().numpy(), aux[k], rtol=1e-12, atol=1e-13), k
    assert int(out["n_precise"].item()) == int((aux["lam"] < 1).sum())
    ctx.close()


@pytest.mark.parametrize("lattice", ["bcc", "fcc"])
def test_csp_value_closed_forms(cfg1, lattice):
    """The CSP value kernel, (B3), against its closed forms on a perfect lattice (bcc a = 3.16 A, 8^3 cells, or
    fcc a = 3.61 A, 6^3 cells; pairs detected on it): g = 0 everywhere; the centre atom moved by delta gives
    4 (n_csp / 2) |delta|^2 (each opposite pair |-2 delta|^2: 16 |delta|^2 with 8 entries, 24 with 12); one
    listed neighbour moved by delta gives |delta|^2 at the centre."""
    import synth.structures as st
    _say("csp value closed forms, %s" % lattice)
    lat, box = st.bcc(3.16, 8) if lattice == "bcc" else st.fcc(3.61, 6)
    n_csp = 8 if lattice == "bcc" else 12
    s = dict(cfg1, pos=lat, pos_ref=lat, box=box, sw=dict(cfg1["sw"], n_csp=n_csp))
    ctx, csp = make_ctx(s, max_nbr=160)  # (fcc: 134 neighbours at the 7 A list radius)
    assert csp.shape[1] == n_csp
    g = ctx.switch_eval(to_dev(lat), box)["g"].cpu().numpy()
    _lt("g perfect", float(np.abs(g).max()), 1e-24)
    delta = np.array([0.031, -0.017, 0.023])
    dd = float(delta @ delta)
    i = 300
    p = lat.copy()
    p[i] += delta
    g = ctx.switch_eval(to_dev(p), box)["g"].cpu().numpy()
    want = 2.0 * n_csp * dd
    _lt("g centre", abs(g[i] - want) / want, 1e-12)
    j = int(csp.cpu().numpy()[i, 3])
    p = lat.copy()
    p[j] += delta
    g = ctx.switch_eval(to_dev(p), box)["g"].cpu().numpy()
    _lt("g partner", abs(g[i] - dd) / dd, 1e-12)
    ctx.close()


def test_eam_matches_oracle(oracle, cfg1):
    _say("eam_eval cfg1")
    ctx, _ = make_ctx(cfg1, lambda_mode=1)
    out = ctx.eam_eval(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, lam_mode=1)
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["F"]), TOL_F64_FORCE)
    _lt("E_atom", _rel(out["E_atom"], want["E_atom"]), 1e-13)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(cfg1["pos"]), TOL_ENERGY)
    _lt("virial", _rel(out["virial"], want["virial"]), 1e-11)
    ctx.close()


def test_eam_per_atom_lambda_matches_oracle(cfg1, cfg1_oracle):
    # ap_eam_eval with a per-atom lambda: E = sum_i lambda_i E^f_i and F = -grad E, which is the
    # oracle's EAM-weighted force family (S12) of the mixed evaluation at the same lambda
    _say("eam_eval cfg1 with per-atom lambda")
    want = cfg1_oracle[1]
    lam = want["aux"]["lam"]
    assert ((lam > 0) & (lam < 1)).sum() > 0 and (lam == 1).sum() > 0
    ctx, _ = make_ctx(cfg1, lambda_mode=1)
    out = ctx.eam_eval(to_dev(cfg1["pos"]), cfg1["box"], lam=to_dev(lam))
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["fam"][0]), TOL_F64_FORCE)
    _lt("E/N", abs(out["E"].item() - float((lam * want["aux"]["Ef"]).sum())) / len(lam), TOL_ENERGY)
    ctx.close()


def test_ace_fp64_matches_oracle(oracle, cfg1):
    _say("ace_eval cfg1 fp64 all atoms")
    ctx, _ = make_ctx(cfg1, lambda_mode=0)
    out = ctx.ace_eval(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, lam_mode=0)
    _lt("E_atom", _rel(out["E_atom"], want["E_atom"]), 1e-12)
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["F"]), TOL_F64_FORCE)
    _lt("virial", _rel(out["virial"], want["virial"]), 1e-10)
    ctx.close()


def test_mixed_fp64_matches_oracle(cfg1, cfg1_oracle):
    _say("mixed cfg1 fp64")
    ctx, _ = make_ctx(cfg1)
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = cfg1_oracle[1]
    assert ((want["aux"]["lam"] > 0) & (want["aux"]["lam"] < 1)).sum() > 10
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["F"]), TOL_F64_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(cfg1["pos"]), TOL_ENERGY)
    _lt("E_atom", _rel(out["E_atom"], want["E_atom"]), 1e-12)
    _lt("virial", _rel(out["virial"], want["virial"]), 1e-10)
    assert np.array_equal(out["lam"].cpu().numpy() < 1, want["aux"]["lam"] < 1)
    ctx.close()


def test_mixed_limits_are_bitwise(cfg1):
    """Eq. (4) with exact weights: the mixed evaluation with lambda forced to 1 is the EAM evaluation, and with
    lambda forced to 0 the ACE evaluation, bit for bit (energies, per-atom energies and forces)."""
    _say("mixed limits cfg1")
    pos = to_dev(cfg1["pos"])
    for mode, single in ((1, "eam_eval"), (0, "ace_eval")):
        ctx, _ = make_ctx(cfg1, lambda_mode=mode)
        mixed = ctx.mixed_energy_forces(pos, cfg1["box"])
        alone = getattr(ctx, single)(pos, cfg1["box"])
        for k in ("E", "E_atom", "F"):
            a, b = mixed[k].cpu().numpy(), alone[k].cpu().numpy()
            _say("  lambda = %d, %s: max |diff| %.3e" % (mode, k, float(np.abs(a - b).max())))
            assert np.array_equal(a, b)
        ctx.close()


def test_ace_rotation_invariance_isolated_cluster(cfg1):
    """The ACE site energies are rotation invariants of the neighbourhood and the forces rotate with it: an
    isolated cluster cut from the 1,024-atom cell (every atom within 8 A of the cell centre, in a 40 A box) and
    the same cluster under a random rotation about its centre, pure ACE in FP64. A pin of the real harmonics and
    their coupling tables that does not go through the oracle."""
    from tests.helpers import rotation
    _say("ace rotation invariance, isolated cluster")
    L = np.asarray(cfg1["box"], dtype=np.float64)
    p = np.asarray(cfg1["pos"], dtype=np.float64) - 0.5 * L
    p -= L * np.rint(p / L)
    u = p[np.einsum("ij,ij->i", p, p) < 64.0]
    R = rotation(11)
    box = np.array([40.0, 40.0, 40.0])
    out = []
    for q in (u, u @ R.T):
        s = dict(cfg1, pos=q + 20.0, pos_ref=q + 20.0, box=box)
        ctx, _ = make_ctx(s, lambda_mode=0)
        r = ctx.ace_eval(to_dev(s["pos"]), box)
        out.append({k: r[k].cpu().numpy() for k in ("E", "E_atom")} | {"F": soa_to_aos(r["F"])})
        ctx.close()
    _say("  %d atoms" % len(u))
    _lt("E_atom", _rel(out[1]["E_atom"], out[0]["E_atom"]), 1e-12)
    _lt("F", force_err_max(out[1]["F"], out[0]["F"] @ R.T), TOL_F64_FORCE)
    assert np.abs(out[0]["F"]).max() > 0.1  # the surface atoms carry real forces


def test_mixed_cubic_rotation(cfg1):
    """The periodic cell turned by 90 degrees about z, (x, y, z) -> (L - y, x, z), with the same CSP pair list
    (by atom index): the mixed energies, lambda and per-atom energies are unchanged and the forces turn with
    the cell."""
    _say("mixed, cell turned by 90 degrees")
    L = float(cfg1["box"][0])
    assert np.allclose(cfg1["box"], L)

    def turn(p):
        p = np.asarray(p, dtype=np.float64)
        return np.stack([L - p[:, 1], p[:, 0], p[:, 2]], axis=1)

    ctx, csp = make_ctx(cfg1)
    a = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    a = {k: a[k].cpu().numpy() for k in ("E", "E_atom", "lam")} | {"F": soa_to_aos(a["F"])}
    ctx.close()
    s = dict(cfg1, pos=turn(cfg1["pos"]), pos_ref=turn(cfg1["pos_ref"]))
    ctx, _ = make_ctx(s, build_csp=False)
    ctx.set_csp_list(csp)
    b = ctx.mixed_energy_forces(to_dev(s["pos"]), s["box"])
    b = {k: b[k].cpu().numpy() for k in ("E", "E_atom", "lam")} | {"F": soa_to_aos(b["F"])}
    ctx.close()
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    _say("  precise atoms %d" % int((a["lam"] < 1).sum()))
    assert (a["lam"] < 1).sum() > 10
    _lt("lambda", float(np.abs(b["lam"] - a["lam"]).max()), 1e-10)
    _lt("E_atom", _rel(b["E_atom"], a["E_atom"]), 1e-12)
    _lt("E/N", abs(float(b["E"].item()) - float(a["E"].item())) / len(a["lam"]), 1e-12)
    _lt("F", force_err_max(b["F"], a["F"] @ Rz.T), TOL_F64_FORCE)


def test_mixed_forces_are_minus_energy_gradient(cfg1):
    """Eq. (5) on the HIP path alone: central differences (h = 1e-4 A) of the mixed energy against the forces,
    FP64. The switching window is set at the 85th and 97th percentiles of d, so that lambda spans the whole band:
    atoms at lambda = 0, across 0 < lambda < 1 (where the gradient of lambda acts) and fast atoms next to it."""
    import torch
    _say("mixed forces vs central differences of the energy, cfg1")
    ctx, _ = make_ctx(cfg1)
    pos = to_dev(cfg1["pos"])
    d = ctx.switch_eval(pos, cfg1["box"])["d"].cpu().numpy()
    ctx.close()
    s = dict(cfg1, sw=dict(cfg1["sw"], d_lo=float(np.quantile(d, 0.85)), d_hi=float(np.quantile(d, 0.97))))
    ctx, _ = make_ctx(s)
    out = ctx.mixed_energy_forces(pos, s["box"])
    lam, F = out["lam"].cpu().numpy(), out["F"].cpu().numpy()
    band = np.nonzero((lam > 0) & (lam < 1))[0]
    band = band[np.argsort(lam[band])]
    inner = np.nonzero(lam == 0)[0]
    outer = np.nonzero(lam == 1)[0]
    # the fast atoms nearest to the band, where only the gradient of lambda reaches
    L = np.asarray(s["box"], float)
    p = np.asarray(s["pos"], float)
    dmin = np.full(len(outer), np.inf)
    for b in band:
        u = p[outer] - p[b]
        u -= L * np.rint(u / L)
        dmin = np.minimum(dmin, np.einsum("ij,ij->i", u, u))
    assert len(band) >= 6 and len(inner) >= 2
    picks = (list(inner[:2]) + list(band[[0, len(band) // 4, len(band) // 2, 3 * len(band) // 4, len(band) - 1]])
             + list(outer[np.argsort(dmin)[:3]]))
    h, worst = 1e-4, 0.0
    for i in picks:
        for c in range(3):
            e = []
            for sgn in (1.0, -1.0):
                q = pos.clone()
                q[c, i] += sgn * h
                e.append(ctx.mixed_energy_forces(q, s["box"])["E"].item())
            fd = -(e[0] - e[1]) / (2 * h)
            worst = max(worst, abs(fd - F[c, i]) / max(1.0, abs(F[c, i])))
    torch.cuda.synchronize()
    ctx.close()
    _say("  %d atoms (lambda %s)" % (len(picks), " ".join("%.2f" % lam[i] for i in picks)))
    _lt("|fd - F|", worst, 1e-6)


def test_mixed_virial_is_minus_strain_derivative(cfg1):
    """The virial of the HIP path against central differences of its own energy under a diagonal affine strain
    of box and positions (eps = 1e-6), FP64, with the switching window of the gradient test above (lambda
    spanning the band). The strained cells keep the same CSP pair list by atom index."""
    _say("mixed virial vs strain derivative, cfg1")
    ctx, csp = make_ctx(cfg1)
    pos0 = np.asarray(cfg1["pos"], float)
    d = ctx.switch_eval(to_dev(pos0), cfg1["box"])["d"].cpu().numpy()
    ctx.close()
    s = dict(cfg1, sw=dict(cfg1["sw"], d_lo=float(np.quantile(d, 0.85)), d_hi=float(np.quantile(d, 0.97))))
    ctx, _ = make_ctx(s, build_csp=False)
    ctx.set_csp_list(csp)
    box0 = np.asarray(s["box"], float)
    W = ctx.mixed_energy_forces(to_dev(pos0), box0)["virial"].cpu().numpy()
    eps, worst = 1e-6, 0.0
    for a in range(3):
        e = []
        for sgn in (1.0, -1.0):
            f = np.ones(3)
            f[a] += sgn * eps
            e.append(ctx.mixed_energy_forces(to_dev(pos0 * f), box0 * f)["E"].item())
        fd = -(e[0] - e[1]) / (2 * eps)
        _say("  W[%d][%d] = %.6f, -dE/deps = %.6f eV" % (a, a, W[a, a], fd))
        worst = max(worst, abs(fd - W[a, a]) / max(1.0, abs(W[a, a])))
    ctx.close()
    _lt("|fd - W|", worst, 1e-5)


def test_mixed_is_deterministic(cfg1):
    _say("determinism cfg1")
    ctx, _ = make_ctx(cfg1)
    a = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    b = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    assert np.array_equal(a["F"].cpu().numpy(), b["F"].cpu().numpy())
    assert a["E"].item() == b["E"].item()
    ctx.close()


def test_vv_is_bit_reproducible_full_size():
    """Two fresh contexts run 30 velocity-Verlet steps of the 128,000-atom workload (FP32 ACE, x = 1 %: more
    precise atoms than resident energy workgroups, so some atoms run split into parts taken from the device
    work queue in whatever order the workgroups arrive). Every sum runs in a fixed order, so positions,
    velocities, forces and the thermo rows agree bit for bit."""
    import torch
    s = synth.build_system(2)
    _say("bit reproducibility, n=%d, 30 steps" % len(s["pos"]))
    runs = []
    for _ in range(2):
        ctx, _ = make_ctx(s)
        pos, vel = to_dev(s["pos"]), to_dev(s["vel"])
        F = ctx.mixed_energy_forces(pos, s["box"])["F"]
        th = ctx.vv_step(pos, vel, F, s["mass"], s["run"]["dt"], 30, s["box"])
        torch.cuda.synchronize()
        runs.append([t.cpu().numpy() for t in (pos, vel, F, th)])
        ctx.close()
    _say("  precise atoms per step: %d-%d" % (int(runs[0][3][:, 6].min()), int(runs[0][3][:, 6].max())))
    assert runs[0][3][:, 6].max() > 1024  # the split into parts is exercised
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


def test_velocity_verlet_10_steps(oracle, cfg1, cfg1_oracle):
    _say("vv 10 steps cfg1")
    ctx, _ = make_ctx(cfg1)
    pos, vel = to_dev(cfg1["pos"]), to_dev(cfg1["vel"])
    F = ctx.mixed_energy_forces(pos, cfg1["box"])["F"]
    th = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 10, cfg1["box"]).cpu().numpy()
    p_ref, v_ref, F_ref, th_ref = oracle.velocity_verlet(cfg1, 10, csp=cfg1_oracle[0])
    d = soa_to_aos(pos) - p_ref
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    _lt("pos", float(np.abs(d).max()), 1e-10)
    _lt("vel", float(np.abs(soa_to_aos(vel) - v_ref).max()), 1e-8)
    _lt("thermo", float(np.abs(th[:, :6] - th_ref).max()), 1e-7)
    ctx.close()


def test_velocity_verlet_across_rebuilds(oracle, cfg1, cfg1_oracle):
    """200 steps at 300 K: the list is rebuilt on the way (skin check), and every cache keyed on the list
    (the ACE pair kernel's reverse slots) must follow; positions, velocities and thermo rows against the
    oracle's velocity Verlet, which builds exact neighbour sets every step."""
    _say("vv 200 steps cfg1")
    ctx, _ = make_ctx(cfg1)
    pos, vel = to_dev(cfg1["pos"]), to_dev(cfg1["vel"])
    F = ctx.mixed_energy_forces(pos, cfg1["box"])["F"]
    th = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 200, cfg1["box"]).cpu().numpy()
    rebuilds = int(th[1:, 7].sum())
    _say("  rebuilds after the first step: %d" % rebuilds)
    assert rebuilds >= 1
    p_ref, v_ref, F_ref, th_ref = oracle.velocity_verlet(cfg1, 200, csp=cfg1_oracle[0])
    d = soa_to_aos(pos) - p_ref
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    _lt("pos", float(np.abs(d).max()), 1e-9)
    _lt("vel", float(np.abs(soa_to_aos(vel) - v_ref).max()), 1e-7)
    _lt("thermo", float(np.abs(th[:, :6] - th_ref).max()), 1e-6)
    ctx.close()


def test_velocity_verlet_time_reversible(cfg1):
    """Velocity Verlet is time reversible: 100 FP64 steps of the mixed potential (with list rebuilds and atoms
    entering and leaving S on the way), then the velocities negated and 100 steps more, return every atom to
    its start and its velocity to minus its start. A pin independent of the oracle."""
    _say("vv time reversal cfg1")
    ctx, _ = make_ctx(cfg1)
    pos, vel = to_dev(cfg1["pos"]), to_dev(cfg1["vel"])
    p0, v0 = soa_to_aos(pos).copy(), soa_to_aos(vel).copy()
    F = ctx.mixed_energy_forces(pos, cfg1["box"])["F"]
    th_f = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 100, cfg1["box"]).cpu().numpy()
    d = soa_to_aos(pos) - p0
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    moved = float(np.abs(d).max())
    vel.neg_()
    th_b = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 100, cfg1["box"]).cpu().numpy()
    _say("  rebuilds forward %d, back %d; largest excursion %.3f A" % (int(th_f[:, 7].sum()), int(th_b[:, 7].sum()),
                                                                        moved))
    assert moved > 0.05
    d = soa_to_aos(pos) - p0
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    _lt("pos", float(np.abs(d).max()), 1e-10)
    _lt("vel", float(np.abs(soa_to_aos(vel) + v0).max()), 1e-8)
    # the backward run's total energy retraces the forward run's (thermo rows in reverse order)
    _lt("E_tot", float(np.abs(th_b[::-1, 2][1:] - th_f[:-1, 2]).max()) / len(p0), 1e-12)
    ctx.close()


def test_ace_fp32_large_basis(oracle):
    """Pure ACE with the n_max 12 / l_max 6 basis (32,686 functions) in FP32 on a 250-atom cell."""
    s = synth.build_system(2, nc=5)
    _say("ace fp32 n12l6 250 atoms")
    ctx, _ = make_ctx(s, lambda_mode=0, precision="fp32")
    out = ctx.ace_eval(to_dev(s["pos"]), s["box"])
    want = oracle.evaluate(s, lam_mode=0)
    _lt("F rms", force_err_rms(soa_to_aos(out["F"]), want["F"]), TOL_F32_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(s["pos"]), TOL_ENERGY)
    _lt("E_atom max", float(np.abs(out["E_atom"].cpu().numpy() - want["E_atom"]).max()), 1e-5)
    ctx.close()


def test_mixed_fp32_full_screw_dipole(oracle):
    """The 128,000-atom bcc workload with the screw dipole (x ~ 1 %), FP32 ACE: every atom's force
    against the oracle (S-skip mode)."""
    s = synth.build_system(2, with_velocities=False)
    n = len(s["pos"])
    _say("mixed fp32 cfg2 n=%d" % n)
    ctx, csp = make_ctx(s)
    out = ctx.mixed_energy_forces(to_dev(s["pos"]), s["box"])
    csp_ref = oracle.csp_pairs(s["pos_ref"], s["box"], 8)
    assert np.array_equal(csp.cpu().numpy(), csp_ref)
    _say("  oracle ...")
    want = oracle.evaluate(s, csp=csp_ref)
    x = float((want["aux"]["lam"] < 1).mean())
    _say("  x = %.4f" % x)
    F = soa_to_aos(out["F"])
    _lt("F rms", force_err_rms(F, want["F"]), TOL_F32_FORCE)
    m, rms, mx = _near_errors(s, want, F)
    _say("  %d atoms near S" % m)
    _lt("F rms near", rms, TOL_F32_FORCE)
    _lt("F max near", mx, TOL_F32_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / n, TOL_ENERGY)
    _lt("sum F", float(np.abs(F.sum(0)).max()), 1e-9 * n)
    ctx.close()


def test_error_codes(cfg1):
    from paper_2512_07693_amd import ap
    _say("error codes")
    ctx, _ = make_ctx(cfg1)
    with pytest.raises(ap.APError) as e:
        ctx.nblist_build(to_dev(cfg1["pos"]), cfg1["box"], 13.0)
    assert e.value.code == -2
    with pytest.raises(ap.APError) as e:
        ctx.nblist_build(to_dev(cfg1["pos"]), cfg1["box"], 7.0, max_nbr=20)
    assert e.value.code == -3
    ctx.close()
    small = ap.Context(len(cfg1["pos"]), max_nbr=40)
    small.set_potential(cfg1["eam"], cfg1["ace"], cfg1["sw"])
    small.csp_pairs_build(to_dev(cfg1["pos_ref"]), cfg1["box"], 8)
    with pytest.raises(ap.APError) as e:
        small.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    assert e.value.code == -3
    small.close()


def test_mixed_fp32_full_vacancy_clusters(oracle):
    """The 1,023,947-atom bcc workload with 20 vacancy clusters (x ~ 0.34 %), FP32 ACE, CSP indicator: the CSP list
    bit-exact and every atom's force against the oracle (S-skip mode)."""
    import time
    s = synth.build_system(4, with_velocities=False)
    n = len(s["pos"])
    _say("mixed fp32 vacancy clusters n=%d" % n)
    ctx, csp = make_ctx(s)
    out = ctx.mixed_energy_forces(to_dev(s["pos"]), s["box"])
    csp_ref = oracle.csp_pairs(s["pos_ref"], s["box"], 8)
    assert np.array_equal(csp.cpu().numpy(), csp_ref)
    t = time.time()
    want = oracle.evaluate(s, csp=csp_ref)
    x = float((want["aux"]["lam"] < 1).mean())
    _say("  oracle %.1f s, x = %.4f" % (time.time() - t, x))
    F = soa_to_aos(out["F"])
    _lt("F rms", force_err_rms(F, want["F"]), TOL_F32_FORCE)
    m, rms, mx = _near_errors(s, want, F)
    _say("  %d atoms near S" % m)
    _lt("F rms near", rms, TOL_F32_FORCE)
    _lt("F max near", mx, TOL_F32_FORCE)
    _lt("E/N", abs(float(out["E"]) - want["E"]) / n, TOL_ENERGY)
    _lt("sum F", float(np.abs(F.sum(0)).max() / np.abs(F).max()), 1e-5)
    ctx.close()


def test_mixed_fp32_full_fcc_penny_crack(oracle):
    """The 2,047,229-atom fcc workload with a 4 nm penny crack (x ~ 0.39 %), FP32 ACE, 12-neighbour CSP: the CSP
    list bit-exact and every atom's force against the oracle (S-skip mode)."""
    import time
    s = synth.build_system(5, with_velocities=False)
    n = len(s["pos"])
    _say("mixed fp32 fcc penny crack n=%d" % n)
    ctx, csp = make_ctx(s, max_nbr=160)
    out = ctx.mixed_energy_forces(to_dev(s["pos"]), s["box"])
    csp_ref = oracle.csp_pairs(s["pos_ref"], s["box"], 12)
    assert np.array_equal(csp.cpu().numpy(), csp_ref)
    t = time.time()
    want = oracle.evaluate(s, csp=csp_ref)
    x = float((want["aux"]["lam"] < 1).mean())
    _say("  oracle %.1f s, x = %.4f" % (time.time() - t, x))
    F = soa_to_aos(out["F"])
    _lt("F rms", force_err_rms(F, want["F"]), TOL_F32_FORCE)
    m, rms, mx = _near_errors(s, want, F)
    _say("  %d atoms near S" % m)
    _lt("F rms near", rms, TOL_F32_FORCE)
    _lt("F max near", mx, TOL_F32_FORCE)
    _lt("E/N", abs(float(out["E"]) - want["E"]) / n, TOL_ENERGY)
    _lt("sum F", float(np.abs(F.sum(0)).max() / np.abs(F).max()), 1e-5)
    ctx.close()


def test_nve_drift_bounded_128k():
    """1,000 velocity-Verlet steps (1 ps) of the 128,000-atom workload after 200 of equilibration: the
    least-squares slope of E_tot / N stays below 1e-6 eV/atom/ps and the total momentum below 1e-8 u A/ps per
    atom. (A window much shorter than 1 ps measures the energy's oscillation, not its drift.)"""
    import torch
    s = synth.build_system(2)
    n = len(s["pos"])
    _say("nve drift n=%d" % n)
    ctx, _ = make_ctx(s)
    pos, vel = to_dev(s["pos"]), to_dev(s["vel"])
    F = ctx.mixed_energy_forces(pos, s["box"])["F"]
    ctx.vv_step(pos, vel, F, s["mass"], s["run"]["dt"], 200, s["box"])
    th = ctx.vv_step(pos, vel, F, s["mass"], s["run"]["dt"], 1000, s["box"]).cpu().numpy()
    e = th[:, 2] / n
    t = (np.arange(len(e)) + 1) * s["run"]["dt"]
    slope = float(np.polyfit(t, e, 1)[0])
    _lt("|drift|", abs(slope), 1e-6)
    _lt("|P|/N", float(np.abs(th[:, 3:6]).max()) / n, 1e-8)
    torch.cuda.synchronize()
    ctx.close()


def test_ace_work_split_consistent():
    """The energy kernel takes an atom whole or splits it into two to four parts of its coupling blocks,
    by the size of S against the resident workgroups. The same atoms must get the same site energies
    whatever the split, and the forces of disjoint subsets must add up (FP32 ACE, 1,024-atom cell)."""
    import torch
    s = synth.build_system(2, nc=8)
    n = len(s["pos"])
    _say("ace work split n=%d" % n)
    ctx, _ = make_ctx(s, lambda_mode=0, precision="fp32")
    pos = to_dev(s["pos"])
    perm = np.random.default_rng(7).permutation(n).astype(np.int32)
    A, BC = perm[:96], perm[96:608]

    def run(idx):
        out = ctx.ace_eval(pos, s["box"], subset=torch.tensor(np.sort(idx), device="cuda"))
        return out["E_atom"].cpu().numpy(), soa_to_aos(out["F"])

    E_a, F_a = run(A)                      # 96 atoms: four parts each
    E_ab, _ = run(perm[:416])              # 416 atoms: halves
    E_bc, F_bc = run(BC)                   # 512 atoms: halves
    E_all, F_all = run(perm[:608])         # 608 atoms: whole, or one round of more than half the slots
    for name, E in (("E_atom 416", E_ab), ("E_atom 608", E_all)):
        _lt(name, float(np.abs(E[A] - E_a[A]).max() / np.abs(E_a[A]).max()), 1e-12)
    _lt("E_atom BC", float(np.abs(E_all[BC] - E_bc[BC]).max() / np.abs(E_bc[BC]).max()), 1e-12)
    _lt("F additive", force_err_rms(F_a + F_bc, F_all), 2e-6)
    ctx.close()
