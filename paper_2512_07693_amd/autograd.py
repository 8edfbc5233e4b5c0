"""torch.autograd binding of the library's ACE batch evaluation and its coefficient adjoint.

ACEBatch(potential, offsets, boxes) describes a ragged batch of periodic cells; calling it with
positions (3, n) and the linear ACE coefficients c (n_funcs,) returns the per-structure energies
E_s = sum_{i in s} E^p_i. The backward pass uses the library's hand-written adjoint:
  dL/dpos_i = g_{s(i)} * dE_{s(i)}/dpos_i = -g_{s(i)} F_i   (cells are independent)
  dL/dc     = sum_s g_s dE_s/dc,   dE_s/dc_nu = sum_{i in s} B_i,nu
ACEBatch.forces(positions, c) returns the forces (3, n); its backward pass is the vector-Jacobian product
of the forces with respect to c (ap_ace_batch_force_vjp), for fitting coefficients to forces.
Everything runs in the HIP kernels; torch only holds the tensors.
"""
import numpy as np
import torch

from . import ap


class _ACEEnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pos, coeffs, batch):
        batch._load(coeffs)
        need_c = coeffs.requires_grad
        out = batch.ctx.ace_batch_eval(pos.detach().contiguous(), batch.offsets, batch.boxes, forces=True,
                                       coeff_grad=need_c)
        fctx.save_for_backward(out["F"], out["dEdc"] if need_c else torch.empty(0, device=pos.device))
        fctx.sid = batch.sid_t
        fctx.need_c = need_c
        return out["E"]

    @staticmethod
    def backward(fctx, gE):
        F, dEdc = fctx.saved_tensors
        gpos = -F * gE[fctx.sid].unsqueeze(0)
        gc = None
        if fctx.need_c:
            gc = (gE.unsqueeze(1) * dEdc).sum(0)
        return gpos, gc, None


class _ACEForceFn(torch.autograd.Function):
    """Forces of the batch as a function of the coefficients, for fitting to forces: the backward pass is the
    library's vector-Jacobian product dL/dc = sum_k G_k . dF_k/dc (positions are data here: no gradient)."""

    @staticmethod
    def forward(fctx, pos, coeffs, batch):
        batch._load(coeffs)
        out = batch.ctx.ace_batch_eval(pos.detach().contiguous(), batch.offsets, batch.boxes, forces=True,
                                       coeff_grad=False)
        fctx.pos = pos.detach().contiguous()
        fctx.batch = batch
        return out["F"]

    @staticmethod
    def backward(fctx, gF):
        dc, _ = fctx.batch.ctx.ace_batch_force_vjp(fctx.pos, fctx.batch.offsets, fctx.batch.boxes,
                                                   gF.contiguous().double())
        return None, dc.sum(0), None


class ACEBatch:
    """A ragged batch of periodic cells bound to one library context with an ACE potential."""

    def __init__(self, ace, offsets, boxes, eam=None, device=None, max_nbr=160):
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        self.boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        n = int(self.offsets[-1])
        self.ace = dict(ace)
        # EAM parameters are unused by a pure-ACE batch but the context holds a full potential
        self.eam = eam or dict(A=1.0, beta=0.0, c0=0.0, c1=0.0, c2=0.0, r_rho=1.0, r_phi=1.0)
        self.sw = dict(d_lo=0.0, d_hi=1.0, r_w=2.0, d0=0.0, n_csp=8)
        self.ctx = ap.Context(n, max_nbr=max_nbr, skin=0.0, device=device)
        sid = np.repeat(np.arange(len(self.offsets) - 1), np.diff(self.offsets))
        self.sid_t = torch.tensor(sid, dtype=torch.long, device=self.ctx.device)
        self._loaded = None

    def _load(self, coeffs):
        if self._loaded is None:
            # the tables (couplings, block layout) once; later coefficients go straight into them on the device
            c = coeffs.detach().double().cpu().numpy()
            self.ctx.set_potential(self.eam, dict(self.ace, c=c), self.sw, lambda_mode=ap.AP_LAMBDA_PRECISE)
            self._loaded = True
        else:
            self.ctx.set_ace_coefficients(coeffs.detach().to(self.ctx.device, torch.float64).contiguous())

    def __call__(self, pos, coeffs):
        return _ACEEnergyFn.apply(pos, coeffs, self)

    def forces(self, pos, coeffs):
        """Forces (3, n) of the batch, differentiable with respect to the coefficients."""
        return _ACEForceFn.apply(pos, coeffs, self)
