"""The boundary's error codes that the other GPU tests do not reach, on the 1,024-atom bcc workload:
AP_E_STATE (call order), AP_E_CSP (a CSP list of the wrong width, an entry out of range or the atom itself)
and AP_E_NONFINITE (a non-finite coordinate). Each error comes back as a return code with its text, and the
context evaluates normally afterwards. Out-of-range list entries are replaced on the device before any use,
and a NaN coordinate only meets clamped cell indices, so no kernel reads outside its buffers."""
import numpy as np
import pytest

import synth
from tests.gpu_util import TOL_F64_FORCE, force_err_max, make_ctx, soa_to_aos, to_dev

pytestmark = pytest.mark.gpu

E_NONFINITE, E_CSP, E_STATE = -4, -6, -7  # AP_E_NONFINITE, AP_E_CSP, AP_E_STATE of ap.h


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cfg1():
    return synth.build_system(1)


def _expect(code, fn, *args):
    from paper_2512_07693_amd import ap
    with pytest.raises(ap.APError) as e:
        fn(*args)
    _say("  code %d: %s" % (e.value.code, e.value))
    assert e.value.code == code
    return e.value


def test_state_errors(cfg1):
    from paper_2512_07693_amd import ap
    _say("call-order errors")
    ctx = ap.Context(len(cfg1["pos"]), max_nbr=128)
    _expect(E_STATE, ctx.mixed_energy_forces, to_dev(cfg1["pos"]), cfg1["box"])  # no potential
    ctx.set_potential(cfg1["eam"], cfg1["ace"], cfg1["sw"])
    _expect(E_STATE, ctx.mixed_energy_forces, to_dev(cfg1["pos"]), cfg1["box"])  # no CSP list
    ctx.close()


def test_csp_list_errors_and_recovery(oracle, cfg1):
    import torch
    _say("CSP list errors")
    ctx, csp = make_ctx(cfg1)
    n = len(cfg1["pos"])
    good = csp.clone()
    _expect(E_CSP, ctx.set_csp_list, torch.zeros((n, 10), dtype=torch.int32, device="cuda"))
    bad = good.clone()
    bad[17, 3] = n + 5
    _expect(E_CSP, ctx.set_csp_list, bad)
    bad = good.clone()
    bad[100, 0] = 100
    _expect(E_CSP, ctx.set_csp_list, bad)
    bad = good.clone()
    bad[5, 7] = -2
    _expect(E_CSP, ctx.set_csp_list, bad)
    # a valid list again: the evaluation matches the oracle
    ctx.set_csp_list(good)
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, csp=oracle.csp_pairs(cfg1["pos_ref"], cfg1["box"], 8))
    err = force_err_max(soa_to_aos(out["F"]), want["F"])
    _say("  after recovery: max|dF|/max|F| = %.2e" % err)
    assert err < TOL_F64_FORCE
    ctx.close()


def test_nonfinite_position(oracle, cfg1):
    _say("non-finite coordinate")
    ctx, _ = make_ctx(cfg1)
    pos = np.array(cfg1["pos"], dtype=np.float64)
    pos[321, 1] = np.nan
    e = _expect(E_NONFINITE, ctx.mixed_energy_forces, to_dev(pos), cfg1["box"])
    assert "non-finite" in str(e)
    out = ctx.mixed_energy_forces(to_dev(cfg1["pos"]), cfg1["box"])
    want = oracle.evaluate(cfg1, csp=oracle.csp_pairs(cfg1["pos_ref"], cfg1["box"], 8))
    err = force_err_max(soa_to_aos(out["F"]), want["F"])
    _say("  after recovery: max|dF|/max|F| = %.2e" % err)
    assert err < TOL_F64_FORCE
    ctx.close()
