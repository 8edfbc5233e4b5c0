"""Helpers of the GPU tests: device tensors in the library's layout and tolerance checks."""
import numpy as np

TOL_F64_FORCE = 1e-11   # max |dF| / max |F| in FP64
TOL_F32_FORCE = 2e-5    # rms |dF| / rms |F| with FP32 ACE arithmetic
TOL_ENERGY = 1e-6       # |dE| / N in eV/atom


def to_dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device="cuda")


def soa_to_aos(t):
    return t.detach().cpu().numpy().T.copy()


def make_ctx(s, lambda_mode=-1, max_nbr=128, grad_lambda=True, precision=None, n_cap=None, build_csp=True):
    """Context with the potential of system s; CSP pairs detected on the GPU from pos_ref."""
    import torch
    from paper_2512_07693_amd import ap
    n = len(s["pos"])
    ctx = ap.Context(n_cap or n, max_nbr=max_nbr, skin=s.get("run", {}).get("skin", 0.5))
    ctx.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=lambda_mode, grad_lambda=grad_lambda,
                      precision=precision)
    csp = None
    if build_csp and lambda_mode == -1:
        csp = ctx.csp_pairs_build(to_dev(s["pos_ref"]), s["box"], s["sw"]["n_csp"])
        torch.cuda.synchronize()
    return ctx, csp


def force_err_max(F_gpu, F_ref):
    return float(np.abs(F_gpu - F_ref).max() / max(np.abs(F_ref).max(), 1e-300))


def force_err_rms(F_gpu, F_ref):
    return float(np.sqrt(np.mean((F_gpu - F_ref) ** 2)) / np.sqrt(np.mean(F_ref ** 2)))
