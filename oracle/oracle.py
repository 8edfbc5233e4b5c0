"""Python access to the FP64 CPU oracle (oracle/ap_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the benchmark's
CPU-baseline leg. The product path never imports this module.

Arrays are numpy float64 / int32; positions are AoS (n, 3).
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ap_oracle.c")
_LIB = os.path.join(_HERE, "libap_oracle.so")
AUX_COLS = ["g", "d", "wbar", "lam", "dlam", "Ef", "Ep", "Et", "W", "xip", "phi2", "nnb"]

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force=False):
    """Compile the oracle with gcc (-O2 -fopenmp -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = bind(_LIB)
    return _lib


def bind(path):
    """Load an oracle shared library and declare its entry points (the tests also bind copies of the
    oracle built with a deliberate mistake, to show that the pins catch it)."""
    L = C.CDLL(path)
    d, i = C.c_double, C.c_int
    L.ora_set_threads.argtypes = [i]
    L.ora_set_threads.restype = i
    L.ora_ftrans.argtypes = [d, d, d]
    L.ora_ftrans.restype = d
    L.ora_ftrans_d.argtypes = [d, d, d]
    L.ora_ftrans_d.restype = d
    L.ora_wigner3j.argtypes = [i] * 6
    L.ora_wigner3j.restype = d
    L.ora_radial.argtypes = [i, d, d, _dp, _dp]
    L.ora_radial.restype = None
    L.ora_ylm.argtypes = [i, _dp, _dp, _dp, _dp, _dp]
    L.ora_ylm.restype = None
    L.ora_nblist.argtypes = [i, _dp, _dp, d, i, _ip, _ip]
    L.ora_nblist.restype = i
    L.ora_csp_pairs.argtypes = [i, _dp, _dp, d, i, _ip]
    L.ora_csp_pairs.restype = i
    L.ora_ace_env.argtypes = [i, _dp, i, i, d, i, _ip, _dp, _dp, d, d, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_ace_env.restype = i
    L.ora_eval.argtypes = [i, _dp, _dp, _dp, i, i, d, i, _ip, _dp, _dp, d, d, _dp, i, _ip, i, i, i,
                           _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_eval.restype = i
    L.ora_eval_ind.argtypes = L.ora_eval.argtypes + [i, C.c_void_p, d]
    L.ora_eval_ind.restype = i
    L.ora_eval_full.argtypes = L.ora_eval_ind.argtypes + [i, C.c_void_p]
    L.ora_eval_full.restype = i
    L.ora_descriptor.argtypes = [i, _dp, _dp, _dp, d, d, _dp, _dp]
    L.ora_descriptor.restype = i
    L.ora_mlp_nparams.restype = i
    L.ora_mlp_features.argtypes = [i, _dp, _dp, d, _dp]
    L.ora_mlp_features.restype = i
    L.ora_mlp_forward.argtypes = [i, _dp, _dp, _dp, _dp, C.c_void_p]
    L.ora_mlp_forward.restype = None
    L.ora_mlp_loss_grad.argtypes = [i, _dp, _dp, _dp, _dp]
    L.ora_mlp_loss_grad.restype = d
    L.ora_ace_coeff_grad.argtypes = [i, _dp, _dp, i, i, d, i, _ip, _dp, _dp, d, C.c_void_p, _dp, _dp, _dp]
    L.ora_ace_coeff_grad.restype = i
    L.ora_vv.argtypes = [i, _dp, _dp, _dp, d, d, i, _dp, _dp, i, i, d, i, _ip, _dp, _dp, d, d, _dp, i, _ip,
                         i, _dp]
    L.ora_vv.restype = i
    L.ora_vv_full.argtypes = L.ora_vv.argtypes + [i, C.c_void_p]
    L.ora_ace_force_vjp.argtypes = [i, _dp, _dp, i, i, d, i, _ip, _dp, _dp, d, C.c_void_p, _dp, _dp, _dp]
    L.ora_ace_force_vjp.restype = i
    L.ora_vv_full.restype = i
    return L


def set_threads(t=0):
    return lib().ora_set_threads(int(t))


class OracleError(RuntimeError):
    pass


def _chk(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def ftrans(x, lo, hi):
    return lib().ora_ftrans(float(x), float(lo), float(hi))


def ftrans_d(x, lo, hi):
    return lib().ora_ftrans_d(float(x), float(lo), float(hi))


def wigner3j(j1, j2, j3, m1, m2, m3):
    return lib().ora_wigner3j(j1, j2, j3, m1, m2, m3)


def radial(n_max, rc, r):
    g = np.zeros(n_max)
    dg = np.zeros(n_max)
    lib().ora_radial(n_max, float(rc), float(r), g, dg)
    return g, dg


def ylm(l_max, u):
    """Complex Y_l^m(u/|u|) at index l*l+l+m and gradient (nlm, 3) with respect to u."""
    nlm = (l_max + 1) ** 2
    yr, yi = np.zeros(nlm), np.zeros(nlm)
    dr, di = np.zeros(3 * nlm), np.zeros(3 * nlm)
    lib().ora_ylm(l_max, _f64(u), yr, yi, dr, di)
    return yr + 1j * yi, (dr + 1j * di).reshape(nlm, 3)


def nblist(pos, box, r, cap=512):
    """Per-atom neighbour index arrays (ascending) at radius r (strict)."""
    n = len(pos)
    cnt = np.zeros(n, np.int32)
    idx = np.zeros(n * cap, np.int32)
    _chk(lib().ora_nblist(n, _f64(pos), _f64(box), float(r), cap, cnt, idx), "ora_nblist")
    idx = idx.reshape(n, cap)
    return [idx[i, :cnt[i]].copy() for i in range(n)]


def csp_pairs(pos, box, n_csp, r_search=5.5):
    n = len(pos)
    out = np.zeros(n * n_csp, np.int32)
    _chk(lib().ora_csp_pairs(n, _f64(pos), _f64(box), float(r_search), n_csp, out), "ora_csp_pairs")
    return out.reshape(n, n_csp)


def _ace_args(ace):
    return (int(ace["n_max"]), int(ace["l_max"]), float(ace["rc"]), int(len(ace["func"])), _i32(ace["func"]),
            _f64(ace["c"]), _f64(ace["b_dens"]), float(ace["emb_A"]), float(ace["E0"]))


def ace_env(u, ace):
    """Site energy of one environment (neighbour vectors u (nn, 3)); returns dict E, dEdu, B, A, phi2."""
    u = _f64(np.asarray(u).reshape(-1, 3))
    n_max, l_max = int(ace["n_max"]), int(ace["l_max"])
    nlm = (l_max + 1) ** 2
    E = np.zeros(1)
    dEdu = np.zeros(max(1, len(u)) * 3)
    B = np.zeros(len(ace["func"]))
    Ar, Ai = np.zeros(n_max * nlm), np.zeros(n_max * nlm)
    phi2 = np.zeros(1)
    _chk(lib().ora_ace_env(len(u), u if len(u) else np.zeros(3), *_ace_args(ace), E, dEdu, B, Ar, Ai, phi2),
         "ora_ace_env")
    return dict(E=E[0], dEdu=dEdu[:3 * len(u)].reshape(-1, 3), B=B, A=(Ar + 1j * Ai).reshape(n_max, nlm),
                phi2=phi2[0])


def _eam_vec(eam):
    return _f64([eam["A"], eam["beta"], eam["c0"], eam["c1"], eam["c2"], eam["r_rho"], eam["r_phi"]])


def _sw_vec(sw):
    return _f64([sw["d_lo"], sw["d_hi"], sw["r_w"], sw.get("d0", 0.0)])


def descriptor(pos, box, g, r_w, d0=0.0, _lib=None):
    """Eq. (6) for a given per-atom g: returns (wbar, d)."""
    pos = _f64(pos)
    n = len(pos)
    wbar, d = np.zeros(n), np.zeros(n)
    _chk((_lib or lib()).ora_descriptor(n, pos, _f64(box), _f64(g), float(r_w), float(d0), wbar, d),
         "ora_descriptor")
    return wbar, d


def _fix_ptr(lam_fix, n):
    if lam_fix is None:
        return None, None
    a = _i32(lam_fix)
    assert a.shape == (n,)
    return a, a.ctypes.data


def evaluate(sys, pos=None, csp=None, lam_mode=-1, skip=1, no_gradlam=0, mlp=None, force_mix=0, lam_fix=None):
    """Full AP evaluation of a system dict (synth.build_system). Returns a dict with E, E_atom,
    F (n,3), virial (3,3), aux (dict of per-atom arrays) and fam (4, n, 3): EAM-weighted,
    ACE-weighted, grad-w and grad-indicator force families. mlp = (params, rc) selects the
    learned indicator instead of CSP. force_mix = 1: the force of Eq. (3) instead of Eq. (5).
    lam_fix: per-atom -1 (lambda from Eq. (2)) or a constant 0 / 1 (App. B)."""
    pos = _f64(sys["pos"] if pos is None else pos)
    n = len(pos)
    box = _f64(sys["box"])
    sw = sys["sw"]
    if csp is None:
        csp = sys.get("csp")
    if csp is None:
        ref = _f64(sys.get("pos_ref", pos))
        csp = np.zeros((n, sw["n_csp"]), np.int32) if (lam_mode >= 0 or mlp is not None) else \
            csp_pairs(ref, box, sw["n_csp"])
    E = np.zeros(1)
    Ea = np.zeros(n)
    F = np.zeros(3 * n)
    vir = np.zeros(9)
    aux = np.zeros(n * len(AUX_COLS))
    fam = np.zeros(12 * n)
    P = None if mlp is None else _f64(mlp[0])
    fix, fix_p = _fix_ptr(lam_fix, n)
    rc = lib().ora_eval_full(n, pos, box, _eam_vec(sys["eam"]), *_ace_args(sys["ace"]), _sw_vec(sw),
                             int(sw["n_csp"]), _i32(csp), int(lam_mode), int(skip), int(no_gradlam), E, Ea, F, vir,
                             aux, fam, 0 if mlp is None else 1, None if P is None else P.ctypes.data,
                             0.0 if mlp is None else float(mlp[1]), int(force_mix), fix_p)
    _chk(rc, "ora_eval")
    aux = aux.reshape(n, len(AUX_COLS))
    return dict(E=E[0], E_atom=Ea, F=F.reshape(n, 3), virial=vir.reshape(3, 3),
                aux={k: aux[:, q].copy() for q, k in enumerate(AUX_COLS)}, fam=fam.reshape(4, n, 3))


def ace_coeff_grad(pos, box, ace, weight=None):
    """dE/dc [n_funcs], dE/db [n_max] and per-atom site energies (without E0) of one cell."""
    n = len(pos)
    dEdc = np.zeros(len(ace["func"]))
    dEdb = np.zeros(int(ace["n_max"]))
    Ea = np.zeros(n)
    a = _ace_args(ace)
    w = None if weight is None else _f64(weight)
    _chk(lib().ora_ace_coeff_grad(n, _f64(pos), _f64(box), *a[:8], w.ctypes.data if w is not None else None,
                                  dEdc, dEdb, Ea), "ora_ace_coeff_grad")
    return dEdc, dEdb, Ea


def ace_force_vjp(pos, box, ace, G, weight=None):
    """dL/dc [n_funcs] and dL/db [n_max] of L = sum_k G_k . F_k, F = -grad sum_i w_i E^ACE_i (G (n, 3))."""
    n = len(pos)
    dLdc = np.zeros(len(ace["func"]))
    dLdb = np.zeros(int(ace["n_max"]))
    a = _ace_args(ace)
    w = None if weight is None else _f64(weight)
    _chk(lib().ora_ace_force_vjp(n, _f64(pos), _f64(box), *a[:8], w.ctypes.data if w is not None else None,
                                 _f64(G).reshape(-1), dLdc, dLdb), "ora_ace_force_vjp")
    return dLdc, dLdb


def velocity_verlet(sys, n_steps, pos=None, vel=None, csp=None, lam_mode=-1, dt=None, force_mix=0, lam_fix=None):
    """n_steps of FP64 velocity Verlet; returns (pos, vel, F, thermo[n_steps][6])."""
    pos = _f64(sys["pos"] if pos is None else pos).copy()
    vel = _f64(sys["vel"] if vel is None else vel).copy()
    box = _f64(sys["box"])
    sw = sys["sw"]
    if csp is None:
        csp = sys.get("csp")
    if csp is None:
        csp = csp_pairs(_f64(sys.get("pos_ref", pos)), box, sw["n_csp"])
    r0 = evaluate(sys, pos=pos, csp=csp, lam_mode=lam_mode, force_mix=force_mix, lam_fix=lam_fix)
    F = _f64(r0["F"]).reshape(-1).copy()
    th = np.zeros(6 * n_steps)
    dt = float(sys["run"]["dt"] if dt is None else dt)
    flat_pos = pos.reshape(-1).copy()
    flat_vel = vel.reshape(-1).copy()
    fix, fix_p = _fix_ptr(lam_fix, len(pos))
    rc = lib().ora_vv_full(len(pos), flat_pos, flat_vel, F, float(sys["mass"]), dt, int(n_steps), box,
                           _eam_vec(sys["eam"]), *_ace_args(sys["ace"]), _sw_vec(sw), int(sw["n_csp"]), _i32(csp),
                           int(lam_mode), th, int(force_mix), fix_p)
    _chk(rc, "ora_vv")
    n = len(pos)
    return flat_pos.reshape(n, 3), flat_vel.reshape(n, 3), F.reshape(n, 3), th.reshape(n_steps, 6)


MLP_NQ, MLP_NH = 16, 64


def mlp_nparams():
    return int(lib().ora_mlp_nparams())


def mlp_features(pos, box, rc=5.5):
    """The sixteen invariant features q (n, 16) of every atom."""
    pos = _f64(pos)
    q = np.zeros(len(pos) * MLP_NQ)
    _chk(lib().ora_mlp_features(len(pos), pos, _f64(box), float(rc), q), "ora_mlp_features")
    return q.reshape(-1, MLP_NQ)


def mlp_forward(q, params, grad=True, _lib=None):
    """Network output o, indicator g = softplus(o) and dg/dq (m, 16) for features q (m, 16)."""
    q = _f64(np.asarray(q).reshape(-1, MLP_NQ))
    m = len(q)
    o, g = np.zeros(m), np.zeros(m)
    dg = np.zeros(m * MLP_NQ) if grad else None
    (_lib or lib()).ora_mlp_forward(m, q, _f64(params), o, g, dg.ctypes.data if grad else None)
    return o, g, (dg.reshape(m, MLP_NQ) if grad else None)


def mlp_loss_grad(q, target, params):
    """Training loss mean((o - t)^2) and its gradient over the parameter block."""
    q = _f64(np.asarray(q).reshape(-1, MLP_NQ))
    grad = np.zeros(mlp_nparams())
    loss = lib().ora_mlp_loss_grad(len(q), q, _f64(target), _f64(params), grad)
    return float(loss), grad
