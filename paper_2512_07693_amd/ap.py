"""ctypes binding of libap.so (include/ap.h): argument marshalling only.

Every computation runs in the library's HIP kernels; PyTorch only provides device memory and the
stream. Positions, velocities and forces are float64 CUDA tensors of shape (3, n) (structure of
arrays); per-atom outputs are (n,). There is no CPU fallback: a missing library raises.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libap.so")

AP_FP64, AP_FP32 = 0, 1
AP_LAMBDA_COMPUTED, AP_LAMBDA_PRECISE, AP_LAMBDA_FAST = -1, 0, 1
AP_IND_CSP, AP_IND_MLP = 0, 1
AP_MIX_ENERGY, AP_MIX_FORCE = 0, 1
ERRORS = {-1: "AP_E_ARG", -2: "AP_E_BOX", -3: "AP_E_NBR_OVERFLOW", -4: "AP_E_NONFINITE", -5: "AP_E_HIP",
          -6: "AP_E_CSP", -7: "AP_E_STATE"}
SYMBOLS = ["ap_ctx_create", "ap_ctx_destroy", "ap_last_error", "ap_set_potential", "ap_csp_pairs_build",
           "ap_set_csp_list", "ap_nblist_build", "ap_eam_eval", "ap_switch_eval", "ap_ace_eval",
           "ap_mixed_energy_forces", "ap_vv_step", "ap_set_profiling", "ap_get_profile", "ap_ace_cost",
           "ap_ace_batch_eval", "ap_set_mlp", "ap_mlp_features", "ap_mlp_eval", "ap_mlp_loss_grad",
           "ap_mlp_train", "ap_nblist_build_noalloc", "ap_set_lambda_fixed", "ap_ace_batch_force_vjp",
           "ap_set_ace_coefficients"]
MLP_NQ, MLP_NPARAMS = 16, 5345


class APError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class Box(C.Structure):
    _fields_ = [("L", C.c_double * 3)]


EAM_KEYS = ("A", "beta", "c0", "c1", "c2", "r_rho", "r_phi")


class EamParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in EAM_KEYS]


class AceParams(C.Structure):
    _fields_ = [("n_max", C.c_int), ("l_max", C.c_int), ("n_funcs", C.c_int), ("rc", C.c_double),
                ("func", C.POINTER(C.c_int32)), ("c", C.POINTER(C.c_double)), ("b_dens", C.POINTER(C.c_double)),
                ("emb_A", C.c_double), ("E0", C.c_double), ("precision", C.c_int)]


class SwitchParams(C.Structure):
    _fields_ = [("d_lo", C.c_double), ("d_hi", C.c_double), ("r_w", C.c_double), ("d0", C.c_double),
                ("n_csp", C.c_int), ("lambda_mode", C.c_int), ("indicator", C.c_int), ("grad_lambda", C.c_int),
                ("mixing", C.c_int)]


_lib = None


def lib():
    """Load libap.so (built in-tree by __graft_entry__.build()); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libap.so not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.ap_ctx_create.argtypes = [C.POINTER(vp), i, i, d, vp]
        L.ap_ctx_destroy.argtypes = [vp]
        L.ap_ctx_destroy.restype = None
        L.ap_last_error.argtypes = [vp]
        L.ap_last_error.restype = C.c_char_p
        L.ap_set_potential.argtypes = [vp, C.POINTER(EamParams), C.POINTER(AceParams), C.POINTER(SwitchParams)]
        L.ap_csp_pairs_build.argtypes = [vp, i, vp, C.POINTER(Box), i, vp]
        L.ap_set_csp_list.argtypes = [vp, i, i, vp]
        L.ap_nblist_build.argtypes = [vp, i, vp, C.POINTER(Box), d, i, vp, vp]
        L.ap_eam_eval.argtypes = [vp, i, vp, vp, C.POINTER(Box), vp, vp, vp, vp, vp]
        L.ap_switch_eval.argtypes = [vp, i, vp, C.POINTER(Box), vp, vp, vp, vp, vp, vp]
        L.ap_ace_eval.argtypes = [vp, i, vp, vp, C.POINTER(Box), vp, i, vp, vp, vp, vp]
        L.ap_mixed_energy_forces.argtypes = [vp, i, vp, vp, C.POINTER(Box), vp, vp, vp, vp, vp]
        L.ap_vv_step.argtypes = [vp, i, vp, vp, vp, d, d, i, C.POINTER(Box), vp]
        L.ap_set_profiling.argtypes = [vp, i]
        L.ap_get_profile.argtypes = [vp, i, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.ap_ace_cost.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ap_ace_batch_eval.argtypes = [vp, i, C.POINTER(C.c_int32), C.POINTER(C.c_double), vp, vp, vp, vp, vp, vp]
        L.ap_set_mlp.argtypes = [vp, vp, d]
        L.ap_mlp_features.argtypes = [vp, i, vp, C.POINTER(Box), d, vp]
        L.ap_mlp_eval.argtypes = [vp, i, vp, vp, vp, vp]
        L.ap_mlp_loss_grad.argtypes = [vp, i, vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.ap_mlp_train.argtypes = [vp, i, vp, vp, i, i, d, i, vp, C.POINTER(C.c_double)]
        L.ap_nblist_build_noalloc.argtypes = [i, vp, C.POINTER(Box), d, i, vp, vp, vp]
        L.ap_set_lambda_fixed.argtypes = [vp, i, vp]
        L.ap_set_ace_coefficients.argtypes = [vp, vp, vp]
        L.ap_ace_batch_force_vjp.argtypes = [vp, i, C.POINTER(C.c_int32), C.POINTER(C.c_double), vp, vp, vp, vp,
                                             vp]
        for s in SYMBOLS:
            if s not in ("ap_ctx_destroy", "ap_last_error"):
                getattr(L, s).restype = i
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _box(box):
    b = Box()
    for a in range(3):
        b.L[a] = float(box[a])
    return b


def _dev(t, dtype, shape=None):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous %s CUDA tensor" % dtype)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
    return t


def nblist_build_noalloc(pos, box, r_list, nbr_count, nbr_idx, stream=None):
    """ap_nblist_build_noalloc: neighbour sets without a context; the outputs nbr_count (int32, (n,)) and
    nbr_idx (int32, (max_nbr, n)) are the caller's CUDA tensors, written in place."""
    n = pos.shape[1]
    _dev(pos, torch.float64, (3, n))
    _dev(nbr_count, torch.int32, (n,))
    _dev(nbr_idx, torch.int32)
    if nbr_idx.dim() != 2 or nbr_idx.shape[1] != n:
        raise ValueError("nbr_idx must be (max_nbr, n)")
    s = torch.cuda.current_stream(pos.device) if stream is None else stream
    rc = lib().ap_nblist_build_noalloc(n, _ptr(pos), C.byref(_box(box)), float(r_list), int(nbr_idx.shape[0]),
                                       _ptr(nbr_count), _ptr(nbr_idx), C.c_void_p(s.cuda_stream))
    if rc != 0:
        raise APError(rc, lib().ap_last_error(None).decode())


class Context:
    """One library context (scratch buffers for up to n_max_atoms atoms) bound to a HIP stream."""

    def __init__(self, n_max_atoms, max_nbr=128, skin=0.5, stream=None, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        self.stream = s
        h = C.c_void_p()
        rc = lib().ap_ctx_create(C.byref(h), int(n_max_atoms), int(max_nbr), float(skin), C.c_void_p(s.cuda_stream))
        if rc != 0:
            raise APError(rc, lib().ap_last_error(None).decode())
        self.h = h
        self.max_nbr = int(max_nbr)
        self._keep = None

    def close(self):
        if getattr(self, "h", None):
            lib().ap_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != 0:
            raise APError(rc, lib().ap_last_error(self.h).decode())

    def _zeros(self, *shape, dtype=torch.float64):
        return torch.zeros(*shape, dtype=dtype, device=self.device)

    def set_potential(self, eam, ace, sw, lambda_mode=AP_LAMBDA_COMPUTED, grad_lambda=True, precision=None,
                      indicator=AP_IND_CSP, mixing=AP_MIX_ENERGY):
        e = EamParams(*[float(eam[k]) for k in EAM_KEYS])
        func = np.ascontiguousarray(ace["func"], dtype=np.int32)
        c = np.ascontiguousarray(ace["c"], dtype=np.float64)
        b = np.ascontiguousarray(ace["b_dens"], dtype=np.float64)
        prec = ace.get("precision", "fp64") if precision is None else precision
        a = AceParams(int(ace["n_max"]), int(ace["l_max"]), len(func), float(ace["rc"]),
                      func.ctypes.data_as(C.POINTER(C.c_int32)), c.ctypes.data_as(C.POINTER(C.c_double)),
                      b.ctypes.data_as(C.POINTER(C.c_double)), float(ace["emb_A"]), float(ace["E0"]),
                      AP_FP32 if prec in ("fp32", AP_FP32) else AP_FP64)
        s = SwitchParams(float(sw["d_lo"]), float(sw["d_hi"]), float(sw["r_w"]), float(sw.get("d0", 0.0)),
                         int(sw["n_csp"]), int(lambda_mode), int(indicator), 1 if grad_lambda else 0, int(mixing))
        self._chk(lib().ap_set_potential(self.h, C.byref(e), C.byref(a), C.byref(s)))
        self._nf, self._nm = len(func), int(ace["n_max"])

    def set_ace_coefficients(self, coeffs=None, b_dens=None):
        """New linear / density coefficients (float64 CUDA tensors) into the installed ACE tables."""
        if coeffs is not None:
            _dev(coeffs, torch.float64, (self._nf,))
        if b_dens is not None:
            _dev(b_dens, torch.float64, (self._nm,))
        self._chk(lib().ap_set_ace_coefficients(self.h, _ptr(coeffs), _ptr(b_dens)))

    def set_lambda_fixed(self, lam_fix):
        """Constant switching parameters: int32 CUDA tensor (n,) of -1 (computed), 0 or 1; None removes."""
        if lam_fix is None:
            self._chk(lib().ap_set_lambda_fixed(self.h, 0, None))
            return
        _dev(lam_fix, torch.int32)
        self._chk(lib().ap_set_lambda_fixed(self.h, int(lam_fix.numel()), _ptr(lam_fix)))

    def csp_pairs_build(self, pos_ref, box, n_csp):
        n = pos_ref.shape[1]
        _dev(pos_ref, torch.float64, (3, n))
        out = self._zeros(n, n_csp, dtype=torch.int32)
        self._chk(lib().ap_csp_pairs_build(self.h, n, _ptr(pos_ref), C.byref(_box(box)), int(n_csp), _ptr(out)))
        return out

    def set_csp_list(self, csp):
        _dev(csp, torch.int32)
        self._keep = csp
        self._chk(lib().ap_set_csp_list(self.h, csp.shape[0], csp.shape[1], _ptr(csp)))

    def nblist_build(self, pos, box, r_list, max_nbr=None):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        m = int(max_nbr or self.max_nbr)
        cnt = self._zeros(n, dtype=torch.int32)
        idx = torch.full((m, n), -1, dtype=torch.int32, device=self.device)
        self._chk(lib().ap_nblist_build(self.h, n, _ptr(pos), C.byref(_box(box)), float(r_list), m, _ptr(cnt),
                                        _ptr(idx)))
        return cnt, idx

    def eam_eval(self, pos, box, lam=None):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        E, Ea, F, V = self._zeros(1), self._zeros(n), self._zeros(3, n), self._zeros(9)
        self._chk(lib().ap_eam_eval(self.h, n, _ptr(pos), None, C.byref(_box(box)), _ptr(lam), _ptr(E), _ptr(Ea),
                                    _ptr(F), _ptr(V)))
        return dict(E=E, E_atom=Ea, F=F, virial=V.view(3, 3))

    def switch_eval(self, pos, box):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        g, d, w, l, dl = (self._zeros(n) for _ in range(5))
        npr = self._zeros(1, dtype=torch.int32)
        self._chk(lib().ap_switch_eval(self.h, n, _ptr(pos), C.byref(_box(box)), _ptr(g), _ptr(d), _ptr(w), _ptr(l),
                                       _ptr(dl), _ptr(npr)))
        return dict(g=g, d=d, wbar=w, lam=l, dlam=dl, n_precise=npr)

    def ace_eval(self, pos, box, subset=None):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        E, Ea, F, V = self._zeros(1), self._zeros(n), self._zeros(3, n), self._zeros(9)
        ns = 0 if subset is None else int(subset.numel())
        self._chk(lib().ap_ace_eval(self.h, n, _ptr(pos), None, C.byref(_box(box)), _ptr(subset), ns, _ptr(E),
                                    _ptr(Ea), _ptr(F), _ptr(V)))
        return dict(E=E, E_atom=Ea, F=F, virial=V.view(3, 3))

    def mixed_energy_forces(self, pos, box):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        E, Ea, F, V, lam = self._zeros(1), self._zeros(n), self._zeros(3, n), self._zeros(9), self._zeros(n)
        self._chk(lib().ap_mixed_energy_forces(self.h, n, _ptr(pos), None, C.byref(_box(box)), _ptr(E), _ptr(Ea),
                                               _ptr(F), _ptr(V), _ptr(lam)))
        return dict(E=E, E_atom=Ea, F=F, virial=V.view(3, 3), lam=lam)

    def ace_batch_eval(self, pos, offsets, boxes, weight=None, forces=True, coeff_grad=True):
        """ACE over a ragged batch of periodic cells (one launch): per-structure energies, forces and
        dE/dc, dE/db per structure. offsets: int sequence [n_struct + 1]; boxes: (n_struct, 3)."""
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        ns, n = len(off) - 1, int(off[-1])
        _dev(pos, torch.float64, (3, n))
        if weight is not None:
            _dev(weight, torch.float64, (n,))
        E = self._zeros(ns)
        F = self._zeros(3, n) if forces else None
        nf, nm = self._nf, self._nm
        dc = self._zeros(ns, nf) if coeff_grad else None
        db = self._zeros(ns, nm) if coeff_grad else None
        self._chk(lib().ap_ace_batch_eval(self.h, ns, off.ctypes.data_as(C.POINTER(C.c_int32)),
                                          bx.ctypes.data_as(C.POINTER(C.c_double)), _ptr(pos), _ptr(weight),
                                          _ptr(E), _ptr(F), _ptr(dc), _ptr(db)))
        return dict(E=E, F=F, dEdc=dc, dEdb=db)

    def ace_batch_force_vjp(self, pos, offsets, boxes, G, weight=None):
        """dL/dc (n_struct, n_funcs) and dL/db (n_struct, n_max) of L = sum_k G_k . F_k over the batch of
        ace_batch_eval; G: float64 CUDA tensor (3, n)."""
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        ns, n = len(off) - 1, int(off[-1])
        _dev(pos, torch.float64, (3, n))
        _dev(G, torch.float64, (3, n))
        if weight is not None:
            _dev(weight, torch.float64, (n,))
        dc = self._zeros(ns, self._nf)
        db = self._zeros(ns, self._nm)
        self._chk(lib().ap_ace_batch_force_vjp(self.h, ns, off.ctypes.data_as(C.POINTER(C.c_int32)),
                                               bx.ctypes.data_as(C.POINTER(C.c_double)), _ptr(pos), _ptr(weight),
                                               _ptr(G), _ptr(dc), _ptr(db)))
        return dc, db

    # ---- learned indicator ----
    def set_mlp(self, params, rc=5.5):
        """Install the network (float32 CUDA tensor of MLP_NPARAMS) used when the indicator is AP_IND_MLP."""
        _dev(params, torch.float32, (MLP_NPARAMS,))
        self._chk(lib().ap_set_mlp(self.h, _ptr(params), float(rc)))

    def mlp_features(self, pos, box, rc=5.5):
        n = pos.shape[1]
        _dev(pos, torch.float64, (3, n))
        q = self._zeros(n, MLP_NQ, dtype=torch.float32)
        self._chk(lib().ap_mlp_features(self.h, n, _ptr(pos), C.byref(_box(box)), float(rc), _ptr(q)))
        return q

    def mlp_eval(self, q, params, grad=True):
        m = q.shape[0]
        _dev(q, torch.float32, (m, MLP_NQ))
        _dev(params, torch.float32, (MLP_NPARAMS,))
        g = self._zeros(m, dtype=torch.float32)
        dg = self._zeros(m, MLP_NQ, dtype=torch.float32) if grad else None
        self._chk(lib().ap_mlp_eval(self.h, m, _ptr(q), _ptr(params), _ptr(g), _ptr(dg) if grad else None))
        return g, dg

    def mlp_loss_grad(self, q, target, params):
        m = q.shape[0]
        _dev(q, torch.float32, (m, MLP_NQ))
        _dev(target, torch.float32, (m,))
        _dev(params, torch.float32, (MLP_NPARAMS,))
        grad = self._zeros(MLP_NPARAMS, dtype=torch.float32)
        loss = C.c_double()
        self._chk(lib().ap_mlp_loss_grad(self.h, m, _ptr(q), _ptr(target), _ptr(params), _ptr(grad),
                                         C.byref(loss)))
        return loss.value, grad

    def mlp_train(self, q, target, params, batch=4096, epochs=20, lr=1e-3, fit_norm=True):
        """Adam on the library's forward/backward kernels; params (float32 CUDA) is updated in place.
        Returns the mean batch loss of every epoch."""
        m = q.shape[0]
        _dev(q, torch.float32, (m, MLP_NQ))
        _dev(target, torch.float32, (m,))
        _dev(params, torch.float32, (MLP_NPARAMS,))
        hist = (C.c_double * max(1, epochs))()
        self._chk(lib().ap_mlp_train(self.h, m, _ptr(q), _ptr(target), int(batch), int(epochs), float(lr),
                                     1 if fit_norm else 0, _ptr(params), hist))
        return np.array(hist[:epochs])

    def set_profiling(self, on=True, every=1):
        """Times every kernel group (every > 1: in vv_step, only the launches of every every-th step)."""
        self._chk(lib().ap_set_profiling(self.h, (max(1, int(every)) if on else 0)))

    def get_profile(self):
        """{kernel group: (average ms, launches)} from the HIP events recorded while profiling."""
        m = 64
        names = C.create_string_buffer(32 * m)
        avg = (C.c_double * m)()
        cnt = (C.c_int64 * m)()
        k = lib().ap_get_profile(self.h, m, names, avg, cnt)
        if k < 0:
            self._chk(k)
        raw = names.raw
        return {raw[32 * q:32 * q + 32].split(b"\0")[0].decode(): (avg[q], cnt[q]) for q in range(min(k, m))}

    def ace_cost(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._chk(lib().ap_ace_cost(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(fixed_per_atom=a.value, per_neighbor_energy=b.value, per_neighbor_force=c.value)

    def vv_step(self, pos, vel, F, mass, dt, n_steps, box, thermo=None):
        n = pos.shape[1]
        for t in (pos, vel, F):
            _dev(t, torch.float64, (3, n))
        th = self._zeros(max(1, n_steps), 8) if thermo is None else thermo
        self._chk(lib().ap_vv_step(self.h, n, _ptr(pos), _ptr(vel), _ptr(F), float(mass), float(dt), int(n_steps),
                                   C.byref(_box(box)), _ptr(th)))
        return th
