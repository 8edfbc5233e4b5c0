"""Pins of the oracle's adaptive-precision energy and forces: Eq. (4), Eq. (5), (A1)-(A2), (S5)-(S29)."""
import numpy as np
import pytest

from tests.helpers import small_system


@pytest.fixture(scope="module")
def sysd(oracle):
    s = small_system(nc=4, sigma=0.12)
    s["csp"] = oracle.csp_pairs(s["pos_ref"], s["box"], 8)
    return s


def test_transition_region_is_populated(oracle, sysd):
    lam = oracle.evaluate(sysd)["aux"]["lam"]
    assert ((lam > 0) & (lam < 1)).sum() >= 20


def test_forces_are_minus_energy_gradient(oracle, sysd):
    """Central differences of E_AP (h = 1e-5 A) against the pair-form force of (S5)-(S29)."""
    r = oracle.evaluate(sysd, skip=0)
    h = 1e-5
    for i in (0, 9, 40, 101):
        for a in range(3):
            p1, p2 = sysd["pos"].copy(), sysd["pos"].copy()
            p1[i, a] += h
            p2[i, a] -= h
            fd = -(oracle.evaluate(sysd, pos=p1)["E"] - oracle.evaluate(sysd, pos=p2)["E"]) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, abs=3e-7 * max(1.0, abs(fd)))


def test_each_force_family_sums_to_zero(oracle, sysd):
    """Antisymmetry of the pair form (A1): the EAM-weighted, ACE-weighted, grad-w and grad-CSP families
    each have zero net force, so total momentum is conserved."""
    fam = oracle.evaluate(sysd)["fam"]
    scale = np.abs(fam).max()
    assert scale > 0
    for f in fam:
        assert np.abs(f.sum(0)).max() < 1e-12 * scale * len(f)


def test_limits_reproduce_pure_models_bitwise(oracle, sysd):
    """Eq. (4) with lambda == 1 is the EAM, with lambda == 0 the ACE, bit for bit."""
    eam = oracle.evaluate(sysd, lam_mode=1)
    ace = oracle.evaluate(sysd, lam_mode=0)
    full = oracle.evaluate(sysd, skip=0)
    assert np.array_equal(eam["E_atom"], full["aux"]["Ef"])
    assert np.array_equal(ace["E_atom"], full["aux"]["Ep"])
    assert np.abs(eam["fam"][1:]).max() == 0 and np.abs(ace["fam"][0]).max() == 0


def test_skip_mode_is_bit_identical(oracle, sysd):
    s = dict(sysd, sw=dict(sysd["sw"], d_lo=1.0, d_hi=1.4))  # some atoms at lambda == 1
    a, b = oracle.evaluate(s, skip=0), oracle.evaluate(s, skip=1)
    assert (a["aux"]["lam"] == 1.0).sum() > 5
    assert np.array_equal(a["F"], b["F"]) and a["E"] == b["E"] and np.array_equal(a["virial"], b["virial"])


def test_without_grad_lambda_is_force_minus_grad_lambda_part(oracle, sysd):
    r = oracle.evaluate(sysd)
    w = oracle.evaluate(sysd, no_gradlam=1)
    assert np.allclose(w["F"], r["F"] - r["fam"][2] - r["fam"][3], rtol=0, atol=1e-12)
    assert np.abs(r["fam"][2]).max() > 0 and np.abs(r["fam"][3]).max() > 0


def test_translation_and_cubic_symmetry(oracle, sysd):
    r = oracle.evaluate(sysd)
    t = oracle.evaluate(sysd, pos=sysd["pos"] + np.array([1.3, -0.7, 2.9]))
    assert t["E"] == pytest.approx(r["E"], rel=1e-12)
    assert np.allclose(t["F"], r["F"], atol=1e-9)
    # axis permutation x->y->z (box is cubic): energies permute with the atoms, forces rotate
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)
    s2 = dict(sysd, pos=sysd["pos"] @ P.T, pos_ref=sysd["pos_ref"] @ P.T)
    q = oracle.evaluate(s2, csp=oracle.csp_pairs(s2["pos_ref"], s2["box"], 8))
    assert q["E"] == pytest.approx(r["E"], rel=1e-12)
    assert np.allclose(q["F"], r["F"] @ P.T, atol=1e-9)


def test_virial_is_minus_strain_derivative(oracle, sysd):
    r = oracle.evaluate(sysd)
    eps = 1e-6
    for a in range(3):
        f1, f2 = np.ones(3), np.ones(3)
        f1[a] += eps
        f2[a] -= eps
        e1 = oracle.evaluate(dict(sysd, pos=sysd["pos"] * f1, box=sysd["box"] * f1))["E"]
        e2 = oracle.evaluate(dict(sysd, pos=sysd["pos"] * f2, box=sysd["box"] * f2))["E"]
        assert r["virial"][a, a] == pytest.approx(-(e1 - e2) / (2 * eps), rel=1e-6)


def test_velocity_verlet_conserves_and_reverses(oracle):
    """NVE on the calibrated 1024-atom bcc workload (x ~ 5 %): total momentum stays at its initial
    value, the total energy fluctuates at the O(dt^2) level of velocity Verlet without drifting away,
    and integrating back with negated velocities returns to the start (time reversibility)."""
    import synth
    s = synth.build_system(1)
    n_steps = 30
    pos, vel, F, th = oracle.velocity_verlet(s, n_steps)
    P0 = (s["mass"] * s["vel"]).sum(0)
    assert np.abs(th[:, 3:6] - P0).max() < 1e-9
    assert np.ptp(th[:, 2]) / len(pos) < 2e-4
    back_pos, back_vel, _, _ = oracle.velocity_verlet(dict(s, pos=pos, vel=-vel), n_steps)
    d = back_pos - s["pos"]
    d -= s["box"] * np.rint(d / s["box"])
    assert np.abs(d).max() < 1e-9


def test_coefficient_gradient_closed_form_and_fd(oracle, sysd):
    """dE/dc_nu = sum_i (1 - lambda_i) B_i,nu; checked against finite differences of E_AP in c."""
    r = oracle.evaluate(sysd)
    w = 1.0 - r["aux"]["lam"]
    dEdc, dEdb, _ = oracle.ace_coeff_grad(sysd["pos"], sysd["box"], sysd["ace"], weight=w)
    rng = np.random.default_rng(0)
    for f in rng.choice(len(dEdc), 6, replace=False):
        h = 1e-4
        c1, c2 = sysd["ace"]["c"].copy(), sysd["ace"]["c"].copy()
        c1[f] += h
        c2[f] -= h
        e1 = oracle.evaluate(dict(sysd, ace=dict(sysd["ace"], c=c1)))["E"]
        e2 = oracle.evaluate(dict(sysd, ace=dict(sysd["ace"], c=c2)))["E"]
        assert dEdc[f] == pytest.approx((e1 - e2) / (2 * h), rel=1e-6, abs=5e-8)
    n = 1
    h = 1e-5
    b1, b2 = sysd["ace"]["b_dens"].copy(), sysd["ace"]["b_dens"].copy()
    b1[n] += h
    b2[n] -= h
    e1 = oracle.evaluate(dict(sysd, ace=dict(sysd["ace"], b_dens=b1)))["E"]
    e2 = oracle.evaluate(dict(sysd, ace=dict(sysd["ace"], b_dens=b2)))["E"]
    assert dEdb[n] == pytest.approx((e1 - e2) / (2 * h), rel=1e-6)


# ---------------------------------------------------------------------------------------------------
# Force mixing, Eq. (3): the non-conservative comparison force
# ---------------------------------------------------------------------------------------------------
def test_force_mixing_is_lambda_weighted_pure_forces(oracle, sysd):
    """F_i = lambda_i F^f_i + (1 - lambda_i) F^p_i with the complete EAM and ACE forces, each pinned on its
    own by finite differences (the lambda == 1 / 0 limits of the AP evaluation)."""
    mix = oracle.evaluate(sysd, force_mix=1)
    lam = mix["aux"]["lam"][:, None]
    want = lam * oracle.evaluate(sysd, lam_mode=1)["F"] + (1 - lam) * oracle.evaluate(sysd, lam_mode=0)["F"]
    assert np.abs(mix["F"] - want).max() < 1e-12 * np.abs(want).max()
    ap = oracle.evaluate(sysd)
    assert mix["E"] == ap["E"] and np.array_equal(mix["E_atom"], ap["E_atom"])  # Eq. (4) energies


def test_force_mixing_breaks_newtons_third_law(oracle, sysd):
    """With lambda varying between atoms the mixed forces do not sum to zero (the paper's momentum
    violation); the conservative AP forces do."""
    mix = oracle.evaluate(sysd, force_mix=1)
    ap = oracle.evaluate(sysd)
    scale = np.abs(ap["F"]).max()
    assert np.abs(mix["F"].sum(0)).max() > 1e-3 * scale
    assert np.abs(ap["F"].sum(0)).max() < 1e-12 * scale * len(ap["F"])


def test_force_mixing_skip_mode_is_bit_identical(oracle, sysd):
    """ACE only on the atoms with lambda < 1 and the atoms within the ACE cutoff of one gives the same bits
    as ACE on every atom."""
    s = dict(sysd, sw=dict(sysd["sw"], d_lo=1.0, d_hi=1.4))
    a, b = oracle.evaluate(s, skip=0, force_mix=1), oracle.evaluate(s, skip=1, force_mix=1)
    assert (a["aux"]["lam"] == 1.0).sum() > 5
    assert np.array_equal(a["F"], b["F"]) and a["E"] == b["E"]


def test_force_mixing_momentum_drifts_in_nve(oracle):
    """Velocity Verlet with force mixing changes the total momentum; with the AP force it stays."""
    import synth
    s = synth.build_system(1)
    P0 = (s["mass"] * s["vel"]).sum(0)
    _, _, _, th_mix = oracle.velocity_verlet(s, 10, force_mix=1)
    _, _, _, th_ap = oracle.velocity_verlet(s, 10)
    assert np.abs(th_mix[-1, 3:6] - P0).max() > 1e-4
    assert np.abs(th_ap[:, 3:6] - P0).max() < 1e-9


# ---------------------------------------------------------------------------------------------------
# Constant switching parameters on chosen atoms (App. B, after (B4))
# ---------------------------------------------------------------------------------------------------
def _mask(lam, seed=3):
    """Some atoms of the transition region fixed to 0, some to 1, the rest computed."""
    rng = np.random.default_rng(seed)
    fix = np.full(len(lam), -1, np.int32)
    mid = np.nonzero((lam > 0) & (lam < 1))[0]
    pick = rng.choice(mid, 12, replace=False)
    fix[pick[:6]] = 0
    fix[pick[6:]] = 1
    return fix


def test_constant_lambda_forces_are_minus_energy_gradient(oracle, sysd):
    """With lambda fixed on a subset (dlambda/dd = 0 there) the energy stays conservative: (B4) with the
    fixed atoms' terms removed is still -grad E (central differences)."""
    fix = _mask(oracle.evaluate(sysd)["aux"]["lam"])
    r = oracle.evaluate(sysd, skip=0, lam_fix=fix)
    assert np.array_equal(r["aux"]["lam"][fix >= 0], fix[fix >= 0].astype(float))
    assert np.all(r["aux"]["dlam"][fix >= 0] == 0.0)
    h = 1e-5
    near = np.nonzero(fix >= 0)[0][:2].tolist() + [9]
    for i in near:
        for a in range(3):
            p1, p2 = sysd["pos"].copy(), sysd["pos"].copy()
            p1[i, a] += h
            p2[i, a] -= h
            fd = -(oracle.evaluate(sysd, pos=p1, lam_fix=fix)["E"] -
                   oracle.evaluate(sysd, pos=p2, lam_fix=fix)["E"]) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, abs=3e-7 * max(1.0, abs(fd)))


def test_constant_lambda_conserves_momentum_per_family(oracle, sysd):
    fix = _mask(oracle.evaluate(sysd)["aux"]["lam"])
    fam = oracle.evaluate(sysd, lam_fix=fix)["fam"]
    scale = np.abs(fam).max()
    for f in fam:
        assert np.abs(f.sum(0)).max() < 1e-12 * scale * len(f)


def test_constant_lambda_on_saturated_atoms_changes_nothing(oracle, sysd):
    """Fixing lambda on atoms whose computed lambda is already 0 or 1 (with dlambda/dd = 0) gives the same
    bits as no mask."""
    s = dict(sysd, sw=dict(sysd["sw"], d_lo=1.0, d_hi=1.15))
    r = oracle.evaluate(s)
    lam, dlam = r["aux"]["lam"], r["aux"]["dlam"]
    fix = np.full(len(lam), -1, np.int32)
    fix[(lam == 1.0) & (dlam == 0.0)] = 1
    fix[(lam == 0.0) & (dlam == 0.0)] = 0
    assert (fix == 1).sum() > 5 and (fix == 0).sum() > 5
    q = oracle.evaluate(s, lam_fix=fix)
    assert np.array_equal(q["F"], r["F"]) and q["E"] == r["E"] and np.array_equal(q["virial"], r["virial"])


def test_constant_lambda_everywhere_is_a_pure_model(oracle, sysd):
    n = len(sysd["pos"])
    eam = oracle.evaluate(sysd, lam_fix=np.ones(n, np.int32))
    ace = oracle.evaluate(sysd, lam_fix=np.zeros(n, np.int32))
    assert np.array_equal(eam["F"], oracle.evaluate(sysd, lam_mode=1)["F"])
    assert np.array_equal(ace["F"], oracle.evaluate(sysd, lam_mode=0)["F"])
    assert np.abs(eam["fam"][2:]).max() == 0 and np.abs(ace["fam"][2:]).max() == 0


# ---------------------------------------------------------------------------------------------------
# Vector-Jacobian product of the ACE forces with respect to the coefficients
# ---------------------------------------------------------------------------------------------------
def _vjp_case(oracle):
    from tests.helpers import small_ace
    s = small_system(nc=4, sigma=0.12, seed=2)
    s["ace"] = small_ace(4, 2, seed=5, scale=0.05)
    G = np.random.default_rng(9).normal(size=s["pos"].shape)
    return s, G


def test_force_vjp_is_directional_derivative_of_dEdc(oracle):
    """dL/dc = -D_G (sum_i B_i): central differences of the oracle's dE/dc along the displacement G."""
    s, G = _vjp_case(oracle)
    dLdc, _ = oracle.ace_force_vjp(s["pos"], s["box"], s["ace"], G)
    h = 1e-5
    c1, _, _ = oracle.ace_coeff_grad(s["pos"] + h * G, s["box"], s["ace"])
    c2, _, _ = oracle.ace_coeff_grad(s["pos"] - h * G, s["box"], s["ace"])
    fd = -(c1 - c2) / (2 * h)
    assert np.abs(dLdc - fd).max() < 1e-6 * np.abs(fd).max()


def test_force_vjp_equals_forces_of_unit_coefficients(oracle):
    """F is linear in c: dL/dc_nu = sum_k G_k . F_k with c = e_nu and no embedding, from the oracle's
    pinned pure-ACE forces."""
    s, G = _vjp_case(oracle)
    dLdc, _ = oracle.ace_force_vjp(s["pos"], s["box"], s["ace"], G)
    nf = len(s["ace"]["c"])
    for nu in [0, 2, nf // 3, nf // 2, nf - 1]:
        c = np.zeros(nf)
        c[nu] = 1.0
        ace = dict(s["ace"], c=c, b_dens=np.zeros(s["ace"]["n_max"]), emb_A=0.0, E0=0.0)
        F = oracle.evaluate(dict(s, ace=ace), lam_mode=0)["F"]
        assert dLdc[nu] == pytest.approx(float((G * F).sum()), rel=1e-10, abs=1e-12)


def test_force_vjp_density_coefficients_by_finite_differences(oracle):
    s, G = _vjp_case(oracle)
    w = np.random.default_rng(4).uniform(0.2, 1.0, len(s["pos"]))
    _, dLdb = oracle.ace_force_vjp(s["pos"], s["box"], s["ace"], G)
    _, dLdb_w = oracle.ace_force_vjp(s["pos"], s["box"], s["ace"], G, weight=w)
    h = 1e-6
    for n in range(s["ace"]["n_max"]):
        b1, b2 = s["ace"]["b_dens"].copy(), s["ace"]["b_dens"].copy()
        b1[n] += h
        b2[n] -= h
        L1 = (G * oracle.evaluate(dict(s, ace=dict(s["ace"], b_dens=b1)), lam_mode=0)["F"]).sum()
        L2 = (G * oracle.evaluate(dict(s, ace=dict(s["ace"], b_dens=b2)), lam_mode=0)["F"]).sum()
        assert dLdb[n] == pytest.approx((L1 - L2) / (2 * h), rel=1e-6, abs=1e-8)
    # constant weights: every atom's share scales by its weight, so the weighted sum differs
    assert np.abs(dLdb_w - dLdb).max() > 1e-6 * np.abs(dLdb).max()
