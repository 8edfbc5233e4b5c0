"""GPU parity of the comparison forces and of constant switching parameters, through the C ABI, against the
FP64 oracle on the 1,024-atom bcc workload (FP64 ACE, x ~ 5 %):

* force mixing, Eq. (3): F_i = lambda_i F^f_i + (1 - lambda_i) F^p_i (non-conservative);
* AP without grad lambda with the CSP indicator (the flagged force of the Fig. 3 discussion);
* atoms with a constant lambda of 0 or 1 (App. B, after (B4)), conservative.

Bars as in test_gpu_parity: FP64 forces max|dF|/max|F| <= 1e-11, energies |dE|/N <= 1e-6, 10 velocity-Verlet
steps within 1e-10 A."""
import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_ENERGY, TOL_F64_FORCE, force_err_max, make_ctx, soa_to_aos, to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _lt(name, value, tol):
    _say("  %-10s %.3e (bar %.1e)" % (name, value, tol))
    assert value < tol, "%s = %.3e exceeds %.1e" % (name, value, tol)


@pytest.fixture(scope="module")
def cfg1():
    return synth.build_system(1)


@pytest.fixture(scope="module")
def csp1(oracle, cfg1):
    return oracle.csp_pairs(cfg1["pos_ref"], cfg1["box"], 8)


def _mixing_ctx(s):
    from paper_2512_07693_amd import ap
    import torch
    ctx = ap.Context(len(s["pos"]), max_nbr=128, skin=s["run"]["skin"])
    ctx.set_potential(s["eam"], s["ace"], s["sw"], mixing=ap.AP_MIX_FORCE)
    ctx.csp_pairs_build(to_dev(s["pos_ref"]), s["box"], s["sw"]["n_csp"])
    torch.cuda.synchronize()
    return ctx


def test_force_mixing_matches_oracle(oracle, cfg1, csp1):
    _say("force mixing cfg1 fp64")
    ctx = _mixing_ctx(cfg1)
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, csp=csp1, force_mix=1)
    F = soa_to_aos(out["F"])
    _lt("F", force_err_max(F, want["F"]), TOL_F64_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(F), TOL_ENERGY)
    # the paper's point: force mixing does not conserve momentum
    _say("  |sum F| = %.3e eV/A" % float(np.abs(F.sum(0)).max()))
    assert np.abs(F.sum(0)).max() > 1e-3
    assert np.abs(out["virial"].cpu().numpy()).max() == 0.0
    ctx.close()


def test_force_mixing_velocity_verlet_10_steps(oracle, cfg1, csp1):
    _say("force mixing vv 10 steps cfg1")
    ctx = _mixing_ctx(cfg1)
    pos, vel = to_dev(cfg1["pos"]), to_dev(cfg1["vel"])
    F = ctx.mixed_energy_forces(pos, cfg1["box"])["F"]
    th = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 10, cfg1["box"]).cpu().numpy()
    p_ref, v_ref, _, th_ref = oracle.velocity_verlet(cfg1, 10, csp=csp1, force_mix=1)
    d = soa_to_aos(pos) - p_ref
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    _lt("pos", float(np.abs(d).max()), 1e-10)
    _lt("vel", float(np.abs(soa_to_aos(vel) - v_ref).max()), 1e-8)
    _lt("thermo", float(np.abs(th[:, :6] - th_ref).max()), 1e-7)
    ctx.close()


def test_without_grad_lambda_csp_matches_oracle(oracle, cfg1, csp1):
    """grad_lambda = 0 with the CSP indicator: the conservative force minus its grad-lambda families."""
    _say("AP without grad lambda cfg1 fp64")
    ctx, _ = make_ctx(cfg1, grad_lambda=False)
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, csp=csp1, no_gradlam=1)
    full = oracle.evaluate(cfg1, csp=csp1)
    assert np.abs(full["fam"][2:]).max() > 1e-3  # the dropped families are not empty
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["F"]), TOL_F64_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(cfg1["pos"]), TOL_ENERGY)
    ctx.close()


def _mask(cfg1, lam):
    """A boundary layer (z < 3 A) fixed to the fast model, and six atoms of the transition region fixed to
    0, six to 1."""
    rng = np.random.default_rng(3)
    fix = np.full(len(lam), -1, np.int32)
    z = np.mod(cfg1["pos"][:, 2], cfg1["box"][2])
    fix[z < 3.0] = 1
    mid = np.nonzero((lam > 0) & (lam < 1) & (fix < 0))[0]
    pick = rng.choice(mid, 12, replace=False)
    fix[pick[:6]] = 0
    fix[pick[6:]] = 1
    return fix


def test_constant_lambda_matches_oracle(oracle, cfg1, csp1):
    import torch
    _say("constant lambda cfg1 fp64")
    lam0 = oracle.evaluate(cfg1, csp=csp1)["aux"]["lam"]
    fix = _mask(cfg1, lam0)
    ctx, _ = make_ctx(cfg1)
    ctx.set_lambda_fixed(torch.tensor(fix, device="cuda"))
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, csp=csp1, lam_fix=fix)
    assert np.array_equal(out["lam"].cpu().numpy()[fix >= 0], fix[fix >= 0].astype(float))
    _lt("F", force_err_max(soa_to_aos(out["F"]), want["F"]), TOL_F64_FORCE)
    _lt("E/N", abs(out["E"].item() - want["E"]) / len(cfg1["pos"]), TOL_ENERGY)
    _lt("virial", float(np.abs(out["virial"].cpu().numpy() - want["virial"]).max() /
                        np.abs(want["virial"]).max()), 1e-10)
    sw = ctx.switch_eval(to_dev(cfg1["pos"]), cfg1["box"])
    assert np.allclose(sw["lam"].cpu().numpy(), want["aux"]["lam"], rtol=1e-12, atol=1e-13)
    assert np.all(sw["dlam"].cpu().numpy()[fix >= 0] == 0.0)
    # removing the mask restores the computed lambda
    ctx.set_lambda_fixed(None)
    plain = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    _lt("F plain", force_err_max(soa_to_aos(plain["F"]), oracle.evaluate(cfg1, csp=csp1)["F"]), TOL_F64_FORCE)
    ctx.close()


def test_constant_lambda_velocity_verlet_10_steps(oracle, cfg1, csp1):
    import torch
    _say("constant lambda vv 10 steps cfg1")
    lam0 = oracle.evaluate(cfg1, csp=csp1)["aux"]["lam"]
    fix = _mask(cfg1, lam0)
    ctx, _ = make_ctx(cfg1)
    ctx.set_lambda_fixed(torch.tensor(fix, device="cuda"))
    pos, vel = to_dev(cfg1["pos"]), to_dev(cfg1["vel"])
    F = ctx.mixed_energy_forces(pos, cfg1["box"])["F"]
    th = ctx.vv_step(pos, vel, F, cfg1["mass"], 1e-3, 10, cfg1["box"]).cpu().numpy()
    p_ref, v_ref, _, th_ref = oracle.velocity_verlet(cfg1, 10, csp=csp1, lam_fix=fix)
    d = soa_to_aos(pos) - p_ref
    d -= cfg1["box"] * np.rint(d / cfg1["box"])
    _lt("pos", float(np.abs(d).max()), 1e-10)
    _lt("thermo", float(np.abs(th[:, :6] - th_ref).max()), 1e-7)
    ctx.close()


def test_constant_lambda_rejects_bad_values(cfg1):
    import torch
    from paper_2512_07693_amd import ap
    ctx, _ = make_ctx(cfg1)
    bad = torch.full((len(cfg1["pos"]),), -1, dtype=torch.int32, device="cuda")
    bad[5] = 2
    with pytest.raises(ap.APError) as e:
        ctx.set_lambda_fixed(bad)
    assert e.value.code == -1
    ctx.close()
