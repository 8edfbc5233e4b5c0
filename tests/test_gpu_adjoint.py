"""The ACE coefficient adjoint on a ragged batch of 64 periodic cells in one launch, through the C ABI
and the torch.autograd binding: energies, forces, dE/dc and dE/db against the FP64 oracle (FP32
arithmetic: forces rms 2e-5, energies 1e-6 eV/atom), and central finite differences (h = 1e-4 A
for positions) of the same kernels run in FP64."""
import numpy as np
import pytest

import synth
from synth import configs as cf
from tests.gpu_util import TOL_ENERGY, TOL_F32_FORCE, force_err_rms, to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _lt(name, value, tol):
    _say("  %-12s %.3e (bar %.1e)" % (name, value, tol))
    assert value < tol, "%s = %.3e exceeds %.1e" % (name, value, tol)


@pytest.fixture(scope="module")
def batch():
    s = synth.build_system(3)
    cells = cf.batch_cells(3)
    pos = np.concatenate([p for p, _ in cells])
    off = np.concatenate([[0], np.cumsum([len(p) for p, _ in cells])]).astype(np.int32)
    boxes = np.array([b for _, b in cells])
    return s, cells, pos, off, boxes


def test_batch_matches_oracle(oracle, batch):
    import torch
    from paper_2512_07693_amd.autograd import ACEBatch
    s, cells, pos, off, boxes = batch
    _say("batch of %d cells, %d atoms, %d functions, fp32" % (len(cells), len(pos), len(s["ace"]["func"])))
    b = ACEBatch(s["ace"], off, boxes)
    b._load(torch.tensor(s["ace"]["c"]))
    out = b.ctx.ace_batch_eval(to_dev(pos), off, boxes)
    E, F = out["E"].cpu().numpy(), out["F"].cpu().numpy().T
    dc, db = out["dEdc"].cpu().numpy(), out["dEdb"].cpu().numpy()
    worst = dict(E=0.0, F=0.0, c=0.0, b=0.0)
    for k in range(0, len(cells), 4):  # every fourth cell against the oracle
        p, bx = cells[k]
        sysd = dict(pos=p, box=bx, eam=s["eam"], ace=s["ace"], sw=s["sw"])
        want = oracle.evaluate(sysd, lam_mode=0)
        wdc, wdb, _ = oracle.ace_coeff_grad(p, bx, s["ace"])
        sl = slice(off[k], off[k + 1])
        worst["E"] = max(worst["E"], abs(E[k] - want["E"]) / len(p))
        worst["F"] = max(worst["F"], force_err_rms(F[sl], want["F"]))
        worst["c"] = max(worst["c"], float(np.abs(dc[k] - wdc).max() / np.abs(wdc).max()))
        worst["b"] = max(worst["b"], float(np.abs(db[k] - wdb).max() / np.abs(wdb).max()))
    _lt("E/N", worst["E"], TOL_ENERGY)
    _lt("F rms", worst["F"], TOL_F32_FORCE)
    _lt("dE/dc", worst["c"], 2e-5)
    _lt("dE/db", worst["b"], 2e-5)
    b.ctx.close()


def test_autograd_finite_differences_fp64(batch):
    """Central differences of the batch energy in positions (h = 1e-4 A) and in coefficients, with the
    kernels in FP64, against the autograd gradients (the hand-written adjoint)."""
    import torch
    from paper_2512_07693_amd.autograd import ACEBatch
    s, cells, _, _, _ = batch
    sub = [cells[0], cells[1], cells[6]]
    pos = np.concatenate([p for p, _ in sub])
    off = np.concatenate([[0], np.cumsum([len(p) for p, _ in sub])]).astype(np.int32)
    boxes = np.array([b for _, b in sub])
    ace = dict(s["ace"], precision="fp64")
    b = ACEBatch(ace, off, boxes)
    dev = b.ctx.device
    P = to_dev(pos).requires_grad_(True)
    c = torch.tensor(ace["c"], device=dev, requires_grad=True)
    g = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device=dev)
    L = (b(P, c) * g).sum()
    L.backward()
    gp, gc = P.grad.cpu().numpy(), c.grad.cpu().numpy()

    def loss(pp, cc):
        with torch.no_grad():
            return float((b(pp, cc) * g).sum())

    h = 1e-4
    worst = 0.0
    rng = np.random.default_rng(0)
    for i in rng.choice(len(pos), 6, replace=False):
        for a in range(3):
            p1, p2 = P.detach().clone(), P.detach().clone()
            p1[a, i] += h
            p2[a, i] -= h
            fd = (loss(p1, c.detach()) - loss(p2, c.detach())) / (2 * h)
            worst = max(worst, abs(fd - gp[a, i]) / max(1.0, abs(fd)))
    _lt("dL/dpos", worst, 1e-6)
    worst = 0.0
    for f in list(rng.choice(len(ace["c"]), 8, replace=False)) + [0, 3]:
        hc = 1e-4 * max(1.0, abs(float(ace["c"][f])))
        c1, c2 = c.detach().clone(), c.detach().clone()
        c1[f] += hc
        c2[f] -= hc
        fd = (loss(P.detach(), c1) - loss(P.detach(), c2)) / (2 * hc)
        worst = max(worst, abs(fd - gc[f]) / max(1.0, abs(fd)))
    _lt("dL/dc", worst, 1e-6)
    b.ctx.close()


def test_force_vjp_matches_oracle(oracle, batch):
    """dL/dc and dL/db of L = sum_k G_k . F_k on the 64-cell batch (FP32 arithmetic), per structure against the
    oracle (every fourth cell); the same on three cells in FP64."""
    import torch
    from paper_2512_07693_amd.autograd import ACEBatch
    s, cells, pos, off, boxes = batch
    G = np.random.default_rng(12).normal(size=pos.shape)
    for prec, stride, bar_c, bar_b in (("fp32", 4, 2e-5, 2e-5), ("fp64", 21, 1e-11, 1e-11)):
        _say("force vjp, %s" % prec)
        ace = dict(s["ace"], precision=prec)
        b = ACEBatch(ace, off, boxes)
        b._load(torch.tensor(ace["c"]))
        dc, db = b.ctx.ace_batch_force_vjp(to_dev(pos), off, boxes, to_dev(G))
        dc, db = dc.cpu().numpy(), db.cpu().numpy()
        wc = wb = 0.0
        for k in range(0, len(cells), stride):
            p, bx = cells[k]
            sl = slice(off[k], off[k + 1])
            want_c, want_b = oracle.ace_force_vjp(p, bx, ace, G[sl])
            wc = max(wc, float(np.abs(dc[k] - want_c).max() / np.abs(want_c).max()))
            wb = max(wb, float(np.abs(db[k] - want_b).max() / np.abs(want_b).max()))
        _lt("dL/dc " + prec, wc, bar_c)
        _lt("dL/db " + prec, wb, bar_b)
        b.ctx.close()


def test_force_vjp_autograd_finite_differences_fp64(batch):
    """ACEBatch.forces and its backward pass: the gradient of L = sum G . F with respect to c against central
    differences of the forward kernels (FP64; F is linear in c)."""
    import torch
    from paper_2512_07693_amd.autograd import ACEBatch
    s, cells, _, _, _ = batch
    sub = [cells[2], cells[5]]
    pos = np.concatenate([p for p, _ in sub])
    off = np.concatenate([[0], np.cumsum([len(p) for p, _ in sub])]).astype(np.int32)
    boxes = np.array([b for _, b in sub])
    ace = dict(s["ace"], precision="fp64")
    b = ACEBatch(ace, off, boxes)
    P = to_dev(pos)
    G = torch.tensor(np.random.default_rng(3).normal(size=(3, len(pos))), device=P.device)
    c = torch.tensor(ace["c"], device=P.device, requires_grad=True)
    (b.forces(P, c) * G).sum().backward()
    gc = c.grad.cpu().numpy()

    def loss(cc):
        with torch.no_grad():
            return float((b.forces(P, cc) * G).sum())

    worst = 0.0
    rng = np.random.default_rng(1)
    for f in list(rng.choice(len(ace["c"]), 8, replace=False)) + [0, 5]:
        hc = 1e-3
        c1, c2 = c.detach().clone(), c.detach().clone()
        c1[f] += hc
        c2[f] -= hc
        fd = (loss(c1) - loss(c2)) / (2 * hc)
        worst = max(worst, abs(fd - gc[f]) / max(1.0, abs(fd)))
    _lt("dL/dc", worst, 1e-8)
    b.ctx.close()


@pytest.mark.parametrize("cfg,prec", [(1, "fp64"), (2, "fp32")], ids=["n8l4_fp64", "n12l6_fp32"])
def test_device_coefficient_update_equals_set_potential(cfg, prec):
    """ap_set_ace_coefficients (new c and b straight into the installed tables on the device) gives the same
    bits as ap_set_potential with those coefficients."""
    import torch
    from paper_2512_07693_amd import ap
    s = synth.build_system(cfg, nc=5 if cfg == 2 else None)
    ace = dict(s["ace"], precision=prec)
    rng = np.random.default_rng(8)
    c2 = ace["c"] * (1.0 + 0.1 * rng.normal(size=len(ace["c"])))
    b2 = ace["b_dens"] * 1.05
    _say("coefficient update n_funcs=%d %s" % (len(c2), prec))
    P = to_dev(s["pos"])
    outs = []
    for mode in ("table", "device"):
        ctx = ap.Context(len(s["pos"]), max_nbr=128)
        if mode == "table":
            ctx.set_potential(s["eam"], dict(ace, c=c2, b_dens=b2), s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
        else:
            ctx.set_potential(s["eam"], ace, s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
            ctx.set_ace_coefficients(torch.tensor(c2, device="cuda"), torch.tensor(b2, device="cuda"))
        o = ctx.ace_eval(P, s["box"])
        outs.append((o["E_atom"].cpu().numpy(), o["F"].cpu().numpy()))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
