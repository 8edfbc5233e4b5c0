"""Benchmark: adaptive-precision EAM/ACE NVE steps on one MI355X.

Workload: bcc a = 3.16 A, 40^3 cells = 128,000 atoms with a planted screw dipole (Burgers vector
a*sqrt(3)/2 along z) and sigma = 0.08 A noise; Finnis-Sinclair EAM on every atom; ACE n_max 12,
l_max 6 (32,686 functions, FP32 arithmetic) on the precise atoms (x ~ 1 %); r_w = 6.5 A; 300 K
Maxwell velocities; velocity Verlet at dt = 1 fs in FP64. One step = one velocity-Verlet step over the
whole hot path (neighbour-list check/rebuild, CSP, descriptor, lambda, EAM, ACE on S, grad-lambda
forces, assembly, reductions, integration), inputs resident in HBM.

Printed: one JSON line with the mixed atom-steps/s (value), the pure-ACE rate on the same GPU and
potential, the NVE drift over a fixed 1-ps leg, the roofline of the dominant kernel (timed with HIP events
on the library's stream) and the CPU oracle baseline on a bounded sample; and, as extra keys, the
conservation contrast of the paper's comparison forces (force mixing, AP without grad lambda, the pure
models), the time-step study of the per-step energy change, the 2M-atom fcc run and the learned indicator.

`--speedup-map` runs instead the sweep of the speedup over the precise fraction x and the averaging radius
r_w on a 2M-atom bcc cell with vacancy-interstitial pairs, fitted to Eq. (1).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mixed EAM/ACE atom-steps/s vs pure-ACE at x=1%, 1 GPU; NVE drift eV/atom/ps"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# kernel durations are taken from HIP events around the launches of every PROF_EVERY-th timed step
# (the event records cost a few microseconds each; the other steps run without them)
PROF_EVERY = 10
FP64_PEAK_TFLOPS = 78.6


# HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counter passes on this workload, scaled by what the
# same counters read for a 1 GiB device copy (fetch x2.0, write x1.0), with a digest of the kernel's source
# file, the list build (its slot order decides how the gathers fall on cache lines) and the shared header at
# the time: a kernel whose sources have changed reports null until re-measured.
MEASURED_TRAFFIC = {
    "ace_energy": (11.72e6, "ace.hip", "392b02967584bc7e"),
    "ace_basis": (10.14e6, "ace.hip", "392b02967584bc7e"),
    "ace_pairforce": (20.49e6, "ace.hip", "392b02967584bc7e"),
    "force": (71.70e6, "forces.hip", "f4a1ce24f00696a4"),
    "dens_desc": (83.92e6, "forces.hip", "f4a1ce24f00696a4"),
    "W": (7.55e6, "forces.hip", "f4a1ce24f00696a4"),
}


def measured_traffic(kernel):
    import hashlib
    if kernel not in MEASURED_TRAFFIC:
        return None
    b, src, digest = MEASURED_TRAFFIC[kernel]
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2512_07693_amd", "csrc")
    h = hashlib.sha256()
    for f in (src, "geometry.hip", "ap_internal.h"):
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return b if h.hexdigest()[:16] == digest else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def drift_fit(thermo, n, dt_ps):
    e = thermo[:, 2] / n
    t = (np.arange(len(e)) + 1) * dt_ps
    slope = float(np.polyfit(t, e, 1)[0]) if len(e) > 2 else 0.0
    return dict(drift_eV_per_atom_per_ps=slope, max_abs_dE_per_atom=float(np.abs(e - e[0]).max()),
                max_abs_dP=float(np.abs(thermo[:, 3:6] - thermo[0, 3:6]).max()),
                steps=int(len(e)), rebuilds=int(thermo[:, 7].sum()),
                x_mean=float(thermo[:, 6].mean() / n), x_max=float(thermo[:, 6].max() / n))


def algorithmic_bytes(kernel, n, nnb, n_s, nnb_rc, n_csp, n_near=None, nnb_short=None):
    """Minimal HBM bytes per launch of the HBM-bound kernels: the slot-major lists are read once (4 B
    per entry), every per-atom array once, outputs written once. n_near atoms (the precise ones and
    their list neighbours) need the full lists in the W and force passes; the others need only their
    flag (W) or their nnb_short EAM-range slots (force). Without those counts every atom is charged the
    full list."""
    if n_near is None:
        n_near, nnb_short = n, nnb
    full = {
        "dens_desc": 4 * nnb + 4 + 24 + 8 + 8 * 8,        # list + count, position, g; 8 outputs
        "force": 4 * nnb + 4 + 24 + 8 * 8 + 4 + 32 + 48,  # list + count, position, 8 own scalars, sidx, F, E_i,
                                                          # the half-kick's velocity in and out
        "W": 4 * nnb + 4 + 4 + 24 + 8 + 8 + 12,          # list + count, flag, position, E~, lambda; W, act
        "csp_value": 4 * n_csp + 24 + 8,
        "vv_first": 6 * 8 + 3 * 8 + 6 * 8,
    }.get(kernel)
    if full is None:
        return None
    # the atoms away from every precise atom
    far = {"W": 4 + 12,                                                   # flag; W, act
           "force": 4 * nnb_short + 4 + 4 + 24 + 4 * 8 + 32 + 48}.get(kernel)  # short list, flag, 4 scalars,
                                                                                   # F, E_i, velocity
    if far is None:
        b = full * n
    else:
        b = full * n_near + far * (n - n_near)
    if kernel == "force":
        b += n_s * nnb_rc * 3 * 4 * 2  # FP32 pair gradients of S read from both sides
    return float(b)


def near_counts(ctx, pos, box, r_list, r_short, max_nbr):
    """Atoms that are precise or in a precise atom's list at these positions, and the mean count of
    neighbours inside the EAM range plus skin (the lists' short part)."""
    lam = ctx.switch_eval(pos, box)["lam"]
    cnt, idx = ctx.nblist_build(pos, box, r_list, max_nbr)
    near = lam < 1.0
    prec = near.nonzero().flatten()
    if prec.numel():
        nb = idx[:, prec].flatten()
        near[nb[nb >= 0].long()] = True
    cnt_s, _ = ctx.nblist_build(pos, box, r_short, max_nbr)
    return int(near.sum().item()), float(cnt_s.double().mean().item())


def run_md(ctx, s, pos0, vel0, steps, warmup, profile_steps, dt=None, final=None):
    """warmup untimed velocity-Verlet steps, then steps timed between HIP events on the library's stream
    (kernel groups timed on every PROF_EVERY-th step). final: a dict that receives the end state."""
    import torch
    box = s["box"]
    dt = s["run"]["dt"] if dt is None else dt
    pos = pos0.clone()
    vel = vel0.clone()
    F = ctx.mixed_energy_forces(pos, box)["F"]
    th_w = None
    if warmup:
        th_w = ctx.vv_step(pos, vel, F, s["mass"], dt, warmup, box).cpu().numpy()
    stream = ctx.stream
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    ctx.set_profiling(True, every=PROF_EVERY)
    t0.record(stream)
    thermo = ctx.vv_step(pos, vel, F, s["mass"], dt, steps, box)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    if final is not None:
        final.update(pos=pos, vel=vel)
    return ms, thermo.cpu().numpy(), prof, th_w


def naive_ace_flops(func):
    """Floating-point operations per precise atom of the product basis by its plain definition (the count
    the scope table gives the energy kernel): order 3 costs 4 flop per (m1, m2) term of every function for
    the value and about three times that for the adjoint, order 2 costs 2 flop per m."""
    func = np.asarray(func)
    t3 = 0
    for n1, l1, n2, l2, n3, l3 in func[func[:, 4] >= 0]:
        m1 = np.arange(-l1, l1 + 1)[:, None]
        m2 = np.arange(-l2, l2 + 1)[None, :]
        t3 += int((np.abs(m1 + m2) <= l3).sum())
    o2 = func[(func[:, 2] >= 0) & (func[:, 4] < 0)]
    t2 = int((2 * o2[:, 1] + 1).sum())
    return float(16 * t3 + 2 * t2), t3, t2


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(s, steps, x):
    """The FP64 oracle as it stands, on the host: velocity-Verlet steps of the full workload on every core
    (the reported value), one force evaluation on one core, and the per-atom times of Eq. (1): t^(f) from a
    pure-EAM evaluation of the workload, t^(p) from pure ACE on a 250-atom cell of the same potential and
    density, t^(d) as what the mixed evaluation costs beyond x t^(p) + t^(f)."""
    import synth
    from oracle import oracle as O
    n = len(s["pos"])
    cores = O.set_threads(0)
    csp = O.csp_pairs(s["pos_ref"], s["box"], s["sw"]["n_csp"])
    t = time.time()
    O.velocity_verlet(s, steps, csp=csp)
    t_vv = time.time() - t
    t = time.time()
    O.evaluate(s, csp=csp)
    t_mix = time.time() - t
    t = time.time()
    O.evaluate(s, csp=csp, lam_mode=1)
    t_eam = time.time() - t
    small = synth.build_system(2, nc=5, with_velocities=False)
    t = time.time()
    O.evaluate(small, lam_mode=0, skip=0)
    t_ace = (time.time() - t) / len(small["pos"])
    t_f = t_eam / n
    t_d = max(0.0, t_mix / n - x * t_ace - t_f)
    O.set_threads(1)
    t = time.time()
    O.evaluate(s, csp=csp)
    t_one = time.time() - t
    O.set_threads(0)
    # the velocity_verlet call also evaluates the initial forces once (steps + 1 evaluations): that
    # evaluation, timed on its own above, is taken out
    t_steps = max(t_vv - t_mix, 1e-9)
    return dict(value=n * steps / t_steps, unit="atom-steps/s", cores=int(cores), kind="oracle",
                sample="%d velocity-Verlet steps of the full %d-atom workload, FP64 oracle in S-skip mode, "
                       "%.1f s (%.1f s with the initial force evaluation)" % (steps, n, t_steps, t_vv),
                cpu_model=cpu_model(),
                single_core=dict(value=n / t_one, unit="atom-steps/s", cores=1,
                                 sample="one force evaluation (S-skip) of the full workload, %.1f s" % t_one),
                per_atom_us=dict(t_precise=t_ace * 1e6, t_fast=t_f * 1e6, t_switch=t_d * 1e6,
                                 t_mixed=t_mix / n * 1e6,
                                 note="t_precise from pure ACE on a 250-atom cell of the same potential; "
                                      "t_switch = t_mixed - x t_precise - t_fast"),
                speedup_eq1=dict(x=x, s_eq1_paper=t_ace / (x * t_ace + (1 - x) * t_f + t_d),
                                 s_eq1_all_eam=t_ace / (x * t_ace + t_f + t_d)))


def thermo_summary(th, n, dt_ps, every=50):
    """Drift, energy and momentum change, temperature change, and traces every `every` steps."""
    kB = 8.617333262e-5
    e = th[:, 2] / n
    T = 2.0 * th[:, 1] / ((3 * n - 3) * kB)
    t = (np.arange(len(e)) + 1) * dt_ps
    P = th[:, 3:6]
    dP = np.abs(P - P[0]).max(1)
    q = max(1, min(100, len(e) // 10))
    return dict(drift_eV_per_atom_per_ps=float(np.polyfit(t, e, 1)[0]) if len(e) > 2 else 0.0,
                max_abs_dE_per_atom=float(np.abs(e - e[0]).max()), max_abs_dP=float(dP.max()),
                dT_K=float(T[-q:].mean() - T[:q].mean()), T_start_K=float(T[:q].mean()),
                x_mean=float(th[:, 6].mean() / n),
                trace=dict(step=list(range(0, len(e), every)), dE_per_atom=[float(v) for v in (e - e[0])[::every]],
                           dP=[float(v) for v in dP[::every]], T_K=[float(v) for v in T[::every]]))


def conservation_contrast(s, pos0, vel0, steps):
    """The paper's NVE contrast (Fig. 5, Fig. S2): the same start integrated with the conservative AP force,
    the AP force without its grad-lambda terms, force mixing (Eq. (3)), pure EAM and pure ACE."""
    from paper_2512_07693_amd import ap
    n = len(s["pos"])
    variants = (("ap", dict()), ("ap_without_grad_lambda", dict(grad_lambda=False)),
                ("force_mixing", dict(mixing=ap.AP_MIX_FORCE)), ("eam", dict(lambda_mode=ap.AP_LAMBDA_FAST)),
                ("ace", dict(lambda_mode=ap.AP_LAMBDA_PRECISE)))
    out = dict(steps=steps, dt_fs=s["run"]["dt"] * 1e3, workload=s["name"])
    for name, kw in variants:
        ctx = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
        ctx.set_potential(s["eam"], s["ace"], s["sw"], **kw)
        if kw.get("lambda_mode", ap.AP_LAMBDA_COMPUTED) == ap.AP_LAMBDA_COMPUTED:
            ctx.csp_pairs_build(torch_dev(s["pos_ref"]), s["box"], s["sw"]["n_csp"])
        log("contrast: %s, %d steps ..." % (name, steps))
        ms, th, _, _ = run_md(ctx, s, pos0, vel0, steps, 0, 0)
        out[name] = dict(ms_per_step=ms / steps, **thermo_summary(th, n, s["run"]["dt"]))
        ctx.close()
    return out


def dt_study(s, pos0, vel0, steps, dts_fs=(0.25, 0.5, 1.0, 2.0)):
    """Per-step energy change against the time step (SM Fig. S3): from one equilibrated state, the mean
    |E_tot(t + dt) - E_tot(t)| / N over `steps` velocity-Verlet steps at each dt, for AP, EAM and ACE, the
    slope of its log against log dt over all four and over each interval (velocity Verlet with smooth
    forces: 3). ACE runs in FP64 here: its FP32 site energies round at about 1e-9 eV/atom per step, which
    would set a floor under the small time steps."""
    from paper_2512_07693_amd import ap
    n = len(s["pos"])
    out = dict(steps=steps, dt_fs=list(dts_fs), ace_precision="fp64")
    for name, mode in (("ap", ap.AP_LAMBDA_COMPUTED), ("eam", ap.AP_LAMBDA_FAST), ("ace", ap.AP_LAMBDA_PRECISE)):
        ctx = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
        ctx.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=mode, precision="fp64")
        if mode == ap.AP_LAMBDA_COMPUTED:
            ctx.csp_pairs_build(torch_dev(s["pos_ref"]), s["box"], s["sw"]["n_csp"])
        de = []
        for dt_fs in dts_fs:
            log("dt study: %s dt = %.2f fs ..." % (name, dt_fs))
            _, th, _, _ = run_md(ctx, s, pos0, vel0, steps, 0, 0, dt=dt_fs * 1e-3)
            de.append(float(np.abs(np.diff(th[:, 2])).mean() / n))
        ctx.close()
        slope = float(np.polyfit(np.log(dts_fs), np.log(de), 1)[0])
        pair = [float(np.log(de[q + 1] / de[q]) / np.log(dts_fs[q + 1] / dts_fs[q])) for q in range(len(de) - 1)]
        out[name] = dict(mean_abs_dE_per_step_per_atom=de, loglog_slope=slope, interval_slopes=pair)
    return out


def nbr_build_roofline(ctx, pos, box, r_list, max_nbr, reps=5):
    """A forced neighbour-list build (cell binning, sort, lists), timed with HIP events: minimal bytes are
    the positions read once and the list written once (24 + 4 + 4 nnb per atom)."""
    ctx.set_profiling(True)
    for _ in range(reps):
        cnt, _ = ctx.nblist_build(pos, box, r_list, max_nbr)
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    n = pos.shape[1]
    nnb = float(cnt.double().mean().item())
    ms = prof["nbr_build"][0]
    b = n * (24.0 + 4.0 + 4.0 * nnb)
    return dict(avg_ms=ms, algorithmic_bytes=b, nnb=nnb, GBs=b / (ms * 1e-3) / 1e9,
                frac=b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, launches=int(prof["nbr_build"][1]))


def torch_dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device="cuda")


def train_indicator(eam, ace, sw, n_cells=200, epochs=150):
    """The learned indicator, trained by the library's kernels on per-atom |E^ACE - E^EAM| that the
    library computes on seeded strained and defected bcc cells."""
    import torch
    from paper_2512_07693_amd import ap
    from synth.learned import mlp_init, training_cells
    cells = training_cells(n_cells)
    nmax = max(len(p) for p, _ in cells)
    c_ace = ap.Context(nmax, max_nbr=128, skin=0.0)
    c_ace.set_potential(eam, ace, sw, lambda_mode=ap.AP_LAMBDA_PRECISE)
    c_eam = ap.Context(nmax, max_nbr=128, skin=0.0)
    c_eam.set_potential(eam, ace, sw, lambda_mode=ap.AP_LAMBDA_FAST)
    Q, Y = [], []
    for p, b in cells:
        P = torch.tensor(np.ascontiguousarray(p.T), device="cuda")
        Y.append((c_ace.ace_eval(P, b)["E_atom"] - c_eam.eam_eval(P, b)["E_atom"]).abs())
        Q.append(c_ace.mlp_features(P, b))
    perm = torch.tensor(np.random.default_rng(0).permutation(sum(len(q) for q in Q)), device="cuda")
    Q = torch.cat(Q)[perm].contiguous()
    T = torch.log(torch.cat(Y)[perm] + 1e-4).float().contiguous()
    params = torch.tensor(mlp_init(1, b3=float(T.mean())), dtype=torch.float32, device="cuda")
    t = time.time()
    hist = c_ace.mlp_train(Q, T, params, batch=4096, epochs=epochs, lr=2e-3)
    torch.cuda.synchronize()
    return params, dict(samples=int(len(Q)), epochs=epochs, train_s=time.time() - t, loss_first=float(hist[0]),
                        loss_last=float(hist[-1]), target_var=float(T.var()))


def learned_comparison(steps, warmup, cal_iters=6):
    """Vacancy-cluster workload (1M atoms): CSP against the trained network at the same precise
    fraction x, on drift, force error near the clusters (against pure ACE) and atom-steps/s."""
    import torch
    import synth
    from synth import structures as st
    from paper_2512_07693_amd import ap
    s = synth.build_system(4)
    n, box = len(s["pos"]), s["box"]
    log("learned indicator: training ...")
    params, train = train_indicator(s["eam"], s["ace"], s["sw"])
    pos0 = torch.tensor(np.ascontiguousarray(s["pos"].T), device="cuda")
    vel0 = torch.tensor(np.ascontiguousarray(s["vel"].T), device="cuda")
    # atoms within 8 A of a removed lattice site
    full, _ = st.bcc(3.16, 80)
    key = lambda a: set(map(tuple, np.round(a / 0.79).astype(np.int64).tolist()))
    removed = np.array(sorted(key(full) - key(s["pos_ref"]))) * 0.79
    near = np.zeros(n, dtype=bool)
    for r in removed:
        d = s["pos"] - r
        d -= box * np.rint(d / box)
        near |= (d * d).sum(1) < 64.0
    c_ref = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
    c_ref.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
    Fref = c_ref.mixed_energy_forces(pos0, box)["F"].cpu().numpy().T
    c_ref.close()
    del c_ref

    def ctx_for(indicator, sw):
        c = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
        c.set_potential(s["eam"], s["ace"], sw, indicator=indicator)
        if indicator == ap.AP_IND_MLP:
            c.set_mlp(params, 5.5)
        else:
            c.csp_pairs_build(torch.tensor(np.ascontiguousarray(s["pos_ref"].T), device="cuda"), box, 8)
        return c

    out = dict(workload=s["name"], n_atoms=n, removed_sites=int(len(removed)), atoms_near=int(near.sum()),
               training=train)

    def leg(name, ctx, final=None):
        F = ctx.mixed_energy_forces(pos0, box)["F"].cpu().numpy().T
        log("learned indicator: %s run, %d + %d steps ..." % (name, warmup, steps))
        ms, thermo, prof, th_w = run_md(ctx, s, pos0, vel0, steps, warmup, 0, final=final)
        nve = drift_fit(thermo, n, s["run"]["dt"])
        return dict(x0=float((ctx.switch_eval(pos0, box)["lam"] < 1).double().mean()),
                    value=n * steps / (ms / 1e3), ms_per_step=ms / steps,
                    force_rmse_near=float(np.sqrt(((F - Fref)[near] ** 2).sum(1).mean())),
                    force_rmse_all=float(np.sqrt(((F - Fref) ** 2).sum(1).mean())),
                    drift_eV_per_atom_per_ps=nve["drift_eV_per_atom_per_ps"],
                    max_abs_dE_per_atom=nve["max_abs_dE_per_atom"], x_mean=nve["x_mean"],
                    kernels={k: round(v[0], 5) for k, v in prof.items()})

    # The network's thresholds (d_lo, d_hi = 2 d_lo) are set on the ensemble its own dynamics produce: where
    # ACE acts the structure relaxes toward ACE's minimum and |E^ACE - E^EAM|, which the network predicts,
    # grows there (x rises along a run), so a threshold matched to CSP's x on the starting frame gives twice
    # CSP's mean x over the run, and one matched on CSP's own thermalised frame almost none. A geometric
    # bisection between those two brackets on the mean x of learned runs of the measured length (warmup +
    # steps from the same start) matches CSP's mean x over its run.
    c = ctx_for(ap.AP_IND_CSP, s["sw"])
    fin = {}
    out["csp"] = leg("csp", c, final=fin)
    pos_t = fin["pos"]
    x_csp0 = float((c.switch_eval(pos0, box)["lam"] < 1).double().mean())
    x_csp_t = float((c.switch_eval(pos_t, box)["lam"] < 1).double().mean())
    c.close()
    cm = ctx_for(ap.AP_IND_MLP, dict(s["sw"], d_lo=1.0, d_hi=2.0))

    def set_thr(d):
        cm.set_potential(s["eam"], s["ace"], dict(s["sw"], d_lo=d, d_hi=2 * d), indicator=ap.AP_IND_MLP)

    def match_frame(P, x_target):
        lo, hi = 1e-4, 10.0
        for _ in range(40):
            mid = np.sqrt(lo * hi)
            set_thr(mid)
            x = float((cm.switch_eval(P, box)["lam"] < 1).double().mean())
            lo, hi = (mid, hi) if x > x_target else (lo, mid)
        return hi

    d_a, d_b = match_frame(pos0, x_csp0), match_frame(pos_t, x_csp_t)
    lo, hi = min(d_a, d_b), max(d_a, d_b)
    x_target = out["csp"]["x_mean"]
    cal = []
    for _ in range(cal_iters):
        mid = np.sqrt(lo * hi)
        set_thr(mid)
        _, th, _, _ = run_md(cm, s, pos0, vel0, steps, warmup, 0)
        xm = float(th[:, 6].mean() / n)
        cal.append(dict(d_lo=float(mid), x_mean=xm))
        lo, hi = (mid, hi) if xm > x_target else (lo, mid)
    d_lo = min(cal, key=lambda e: abs(np.log(max(e["x_mean"], 1e-12) / x_target)))["d_lo"]
    set_thr(d_lo)
    out["learned"] = leg("learned", cm)
    out["learned"]["d_lo"] = float(d_lo)
    cm.close()
    out["threshold_calibration"] = dict(bracket=[float(d_a), float(d_b)], steps=steps, warmup=warmup,
                                        x_target=x_target, iterations=cal)
    out["x_mean_ratio"] = out["learned"]["x_mean"] / max(out["csp"]["x_mean"], 1e-30)
    out["step_ratio"] = out["learned"]["ms_per_step"] / out["csp"]["ms_per_step"]
    return out


def speedup_map(r_ws=(6.5, 9.0, 12.0, 16.0), pairs=(4, 16, 64, 256, 1024, 2048), nc=100, steps=10, warmup=5):
    """Speedup of the mixed loop over pure ACE against the precise fraction x and the averaging radius r_w
    (Fig. 4 with Eq. (1)): bcc 100^3 = 2,000,000 atoms (sigma = 0.08 A, 300 K) with a growing number of
    vacancy-interstitial pairs, the potentials of the 128,000-atom workload, and per r_w the thresholds
    d_lo = mean + 1.25 (max - mean) of d on the defect-free cell, d_hi = d_lo + 1 A^2. Per-atom times:
    t^(p) from pure ACE, t^(f) from pure EAM on the same cell, t^(d) per r_w from the intercept of the mixed
    step time against x; Eq. (1) in the form of this build (EAM on every atom) then predicts each point."""
    import torch
    import synth
    from synth import structures as st
    from paper_2512_07693_amd import ap
    base = synth.build_system(2, nc=4, with_velocities=False)  # the potentials and run parameters only
    eam, ace, sw0, mass, skin = base["eam"], base["ace"], base["sw"], base["mass"], base["run"]["skin"]
    a = 3.16
    slots = {6.5: 128, 9.0: 320, 12.0: 640, 16.0: 1408}
    sysd = dict(eam=eam, ace=ace, mass=mass, run=dict(base["run"]))

    def cell(n_pairs, seed):
        rng = np.random.default_rng(6000 + seed)
        if n_pairs:
            ref, box = st.frenkel_pairs(a, nc, n_pairs, rng)
        else:
            ref, box = st.bcc(a, nc)
        pos = st.gaussian_displace(ref, 0.08, rng)
        vel = st.maxwell_velocities(len(pos), mass, 300.0, rng)
        return ref, pos, vel, box

    out = dict(n_atoms=2 * nc ** 3, steps=steps, warmup=warmup, r_w=list(r_ws), pairs=list(pairs))
    # pure models on the defect-free cell
    ref, pos, vel, box = cell(0, 0)
    d = dict(sysd, box=box)
    P, V = torch_dev(pos), torch_dev(vel)
    times = {}
    for name, mode, k in (("ace", ap.AP_LAMBDA_PRECISE, 3), ("eam", ap.AP_LAMBDA_FAST, 20)):
        c = ap.Context(len(pos), max_nbr=128, skin=skin)
        c.set_potential(eam, ace, sw0, lambda_mode=mode)
        log("speedup map: pure %s ..." % name)
        ms, _, _, _ = run_md(c, d, P, V, k, 1, 0)
        times[name] = ms / k / len(pos)
        c.close()
    t_p, t_f = times["ace"], times["eam"]
    out["t_precise_ns"], out["t_fast_ns"] = t_p * 1e6, t_f * 1e6
    for r_w in r_ws:
        m = slots[r_w]
        # thresholds from the defect-free cell at this radius
        c = ap.Context(len(pos), max_nbr=m, skin=skin)
        c.set_potential(eam, ace, dict(sw0, r_w=r_w, d_lo=1.0, d_hi=2.0))
        c.csp_pairs_build(torch_dev(ref), box, 8)
        dd = c.switch_eval(P, box)["d"]
        dmean, dmax = float(dd.mean()), float(dd.max())
        c.close()
        d_lo = dmean + 1.25 * (dmax - dmean)
        sw = dict(sw0, r_w=r_w, d_lo=d_lo, d_hi=d_lo + 1.0)
        rows = []
        for k_p in pairs:
            ref_k, pos_k, vel_k, box_k = cell(k_p, k_p)
            Pk, Vk = torch_dev(pos_k), torch_dev(vel_k)
            c = ap.Context(len(pos_k), max_nbr=m, skin=skin)
            c.set_potential(eam, ace, sw)
            c.csp_pairs_build(torch_dev(ref_k), box_k, 8)
            log("speedup map: r_w = %.1f, %d pairs ..." % (r_w, k_p))
            ms, th, prof, _ = run_md(c, dict(sysd, box=box_k), Pk, Vk, steps, warmup, 0)
            c.close()
            n = len(pos_k)
            x = float(th[:, 6].mean() / n)
            t_m = ms / steps / n
            rows.append(dict(pairs=k_p, x=x, ms_per_step=ms / steps, t_mixed_ns=t_m * 1e6, s_measured=t_p / t_m,
                             kernels={q: round(v[0], 4) for q, v in prof.items()}))
            del Pk, Vk
            torch.cuda.empty_cache()
        xs = np.array([r["x"] for r in rows])
        tm = np.array([r["t_mixed_ns"] for r in rows]) * 1e-6
        slope, icpt = np.polyfit(xs, tm, 1)
        t_d = max(0.0, icpt - t_f)
        for r in rows:
            r["s_eq1"] = t_p / (r["x"] * t_p + t_f + t_d)
            r["rel_err"] = r["s_eq1"] / r["s_measured"] - 1.0
        out["r_w=%g" % r_w] = dict(d_lo=d_lo, d_hi=d_lo + 1.0, d_mean_bulk=dmean, d_max_bulk=dmax,
                                   t_switch_ns=t_d * 1e6, t_precise_in_mixed_ns=slope * 1e6, points=rows,
                                   max_abs_rel_err=float(max(abs(r["rel_err"]) for r in rows)))
    return out


def large_run(steps, warmup, pure_steps):
    """The 2M-atom fcc penny-crack workload: the mixed loop against pure ACE on the same GPU, with the
    per-kernel times and the memory-bound kernels' achieved bandwidth at a working set far above the
    Infinity Cache."""
    import torch
    import synth
    from paper_2512_07693_amd import ap
    s = synth.build_system(5)
    n, box = len(s["pos"]), s["box"]
    pos0 = torch.tensor(np.ascontiguousarray(s["pos"].T), device="cuda")
    vel0 = torch.tensor(np.ascontiguousarray(s["vel"].T), device="cuda")
    ctx = ap.Context(n, max_nbr=160, skin=s["run"]["skin"])
    ctx.set_potential(s["eam"], s["ace"], s["sw"])
    ctx.csp_pairs_build(torch.tensor(np.ascontiguousarray(s["pos_ref"].T), device="cuda"), box, s["sw"]["n_csp"])
    log("fcc penny crack: mixed %d + %d steps ..." % (warmup, steps))
    ms, thermo, prof, _ = run_md(ctx, s, pos0, vel0, steps, warmup, 0)
    nve = drift_fit(thermo, n, s["run"]["dt"])
    r_list = max(s["ace"]["rc"], s["sw"]["r_w"]) + s["run"]["skin"]
    cnt, _ = ctx.nblist_build(pos0, box, r_list, 160)
    nnb = float(cnt.double().mean().item())
    n_near, nnb_short = near_counts(ctx, pos0, box, r_list, max(s["eam"]["r_rho"], s["eam"]["r_phi"]) + s["run"]["skin"],
                                    160)
    ctx.close()
    del ctx
    hbm = {}
    for k in ("dens_desc", "force", "W"):
        if k in prof:
            b = algorithmic_bytes(k, n, nnb, nve["x_mean"] * n, 54.0, s["sw"]["n_csp"], n_near, nnb_short)
            hbm[k] = dict(avg_ms=prof[k][0], GBs=b / (prof[k][0] * 1e-3) / 1e9,
                          frac=b / (prof[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS)
    out = dict(workload=s["name"], n_atoms=n, value=n * steps / (ms / 1e3), ms_per_step=ms / steps, nve=nve,
               kernels={k: round(v[0], 5) for k, v in prof.items()}, hbm_kernels=hbm)
    if pure_steps > 0:
        cp = ap.Context(n, max_nbr=160, skin=s["run"]["skin"])
        cp.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
        log("fcc penny crack: pure ACE %d steps ..." % pure_steps)
        ms_p, _, _, _ = run_md(cp, s, pos0, vel0, pure_steps, 1, 0)
        out["pure_ace"] = dict(value=n * pure_steps / (ms_p / 1e3), ms_per_step=ms_p / pure_steps)
        out["speedup_vs_pure_ace"] = (ms_p / pure_steps) / (ms / steps)
        cp.close()
    # the same recipe at x = 0.1 % and 1 %: the precise fraction set by the crack's size (radius 18 and 67 A
    # instead of 40 A), the switching thresholds unchanged
    out["x_variants"] = []
    for radius in (18.0, 67.0):
        sv = synth.build_system(5, defect=dict(radius=radius))
        nv = len(sv["pos"])
        pv = torch.tensor(np.ascontiguousarray(sv["pos"].T), device="cuda")
        vv = torch.tensor(np.ascontiguousarray(sv["vel"].T), device="cuda")
        cv = ap.Context(nv, max_nbr=160, skin=sv["run"]["skin"])
        cv.set_potential(sv["eam"], sv["ace"], sv["sw"])
        cv.csp_pairs_build(torch.tensor(np.ascontiguousarray(sv["pos_ref"].T), device="cuda"), sv["box"],
                           sv["sw"]["n_csp"])
        log("fcc penny crack, radius %.0f A: mixed %d + %d steps ..." % (radius, warmup, steps))
        msv, thv, _, _ = run_md(cv, sv, pv, vv, steps, warmup, 0)
        cv.close()
        nvev = drift_fit(thv, nv, sv["run"]["dt"])
        e = dict(crack_radius_A=radius, n_atoms=nv, x_mean=nvev["x_mean"], value=nv * steps / (msv / 1e3),
                 ms_per_step=msv / steps, drift_eV_per_atom_per_ps=nvev["drift_eV_per_atom_per_ps"])
        if "pure_ace" in out:
            e["speedup_vs_pure_ace"] = out["pure_ace"]["ms_per_step"] / (msv / steps)
        out["x_variants"].append(e)
    return out


def main():
    ap_ = argparse.ArgumentParser()
    ap_.add_argument("--gpus", type=int, default=1)
    ap_.add_argument("--steps", type=int, default=1000)
    ap_.add_argument("--warmup", type=int, default=200)
    ap_.add_argument("--pure-steps", type=int, default=20)
    ap_.add_argument("--cpu-steps", type=int, default=16)
    ap_.add_argument("--no-cpu", action="store_true")
    ap_.add_argument("--drift-steps", type=int, default=1000,
                     help="the NVE drift leg: steps fitted after --equil steps of equilibration (independent of "
                          "--steps)")
    ap_.add_argument("--equil", type=int, default=200)
    ap_.add_argument("--contrast-steps", type=int, default=1000,
                     help="NVE steps of each run of the conservation contrast (0: skip)")
    ap_.add_argument("--dt-steps", type=int, default=100,
                     help="steps per time step of the time-step study (0: skip)")
    ap_.add_argument("--speedup-map", action="store_true",
                     help="run only the sweep of the speedup over x and r_w (2M-atom bcc, Eq. (1) fit)")
    ap_.add_argument("--large-steps", type=int, default=1000,
                     help="NVE steps of the 2M-atom fcc penny-crack run (0: skip)")
    ap_.add_argument("--learned-steps", type=int, default=1000,
                     help="NVE steps of the learned-indicator comparison on the 1M-atom workload (0: skip)")
    ap_.add_argument("--profile-run", action="store_true",
                     help="only the timed mixed loop and (with --pure-steps > 0) the pure-ACE loop, for profiler "
                          "and counter runs; prints one line of timings")
    ap_.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                     help="only copy a MIB-sized buffer 5 times (calibrates the HBM byte counters)")
    args = ap_.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes 5 times" % (src.numel() * 4))
        return

    import synth
    from paper_2512_07693_amd import ap

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.speedup_map:
        print(json.dumps(dict(metric="speedup over pure ACE against x and r_w", speedup_map=speedup_map())),
              flush=True)
        return
    log("building workload ...")
    s = synth.build_system(2)
    n = len(s["pos"])
    box = s["box"]
    pos0 = torch.tensor(np.ascontiguousarray(s["pos"].T), device=dev)
    vel0 = torch.tensor(np.ascontiguousarray(s["vel"].T), device=dev)
    ref = torch.tensor(np.ascontiguousarray(s["pos_ref"].T), device=dev)

    ctx = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
    ctx.set_potential(s["eam"], s["ace"], s["sw"])
    ctx.csp_pairs_build(ref, box, s["sw"]["n_csp"])
    log("mixed: %d warmup + %d timed steps ..." % (args.warmup, args.steps))
    ms, thermo, prof, th_w = run_md(ctx, s, pos0, vel0, args.steps, args.warmup, 0)
    value = n * args.steps / (ms / 1e3)
    window = drift_fit(thermo, n, s["run"]["dt"])
    log("mixed: %.3f ms/step, %.3e atom-steps/s, x=%.4f" % (ms / args.steps, value, window["x_mean"]))
    if args.profile_run:
        out = dict(mixed_ms_per_step=ms / args.steps, x=window["x_mean"],
                   kernels_ms={k: round(v[0], 5) for k, v in prof.items()})
        if args.pure_steps > 0:
            ctx_p = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
            ctx_p.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
            ms_p, _, _, _ = run_md(ctx_p, s, pos0, vel0, args.pure_steps, 1, 0)
            out["pure_ace_ms_per_step"] = ms_p / args.pure_steps
            ctx_p.close()
        print(json.dumps(out), flush=True)
        return
    # the drift on a fixed 1-ps leg after a stated equilibration, whatever --steps is (a short window
    # measures the energy's oscillation, not its drift); also fitted with the transient included
    log("drift leg: %d + %d steps ..." % (args.equil, args.drift_steps))
    eq_state = {}
    _, th_d, _, th_e = run_md(ctx, s, pos0, vel0, args.drift_steps, args.equil, 0, final=eq_state)
    nve = drift_fit(th_d, n, s["run"]["dt"])
    nve["equilibration_steps"] = args.equil
    if th_e is not None:
        nve["from_step_0"] = {k: v for k, v in drift_fit(np.concatenate([th_e, th_d]), n, s["run"]["dt"]).items()
                              if k in ("drift_eV_per_atom_per_ps", "max_abs_dE_per_atom", "steps", "x_max")}
    nve["bar_eV_per_atom_per_ps"] = 1e-6
    nve["margin"] = 1e-6 / max(abs(nve["drift_eV_per_atom_per_ps"]), 1e-30)
    nve["timed_window"] = {k: window[k] for k in ("drift_eV_per_atom_per_ps", "max_abs_dE_per_atom", "steps")}
    log("drift: %.3e eV/atom/ps over %d steps (%.3e with the transient)" %
        (nve["drift_eV_per_atom_per_ps"], nve["steps"], nve.get("from_step_0", {}).get("drift_eV_per_atom_per_ps",
                                                                                          float("nan"))))

    # pure ACE: the same potential with lambda == 0 everywhere
    ms_p, value_p, prof_p = None, None, {}
    if args.pure_steps > 0:
        ctx_p = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
        ctx_p.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=ap.AP_LAMBDA_PRECISE)
        log("pure ACE: %d timed steps ..." % args.pure_steps)
        ms_p, thermo_p, prof_p, _ = run_md(ctx_p, s, pos0, vel0, args.pure_steps, 2, 0)
        value_p = n * args.pure_steps / (ms_p / 1e3)
        log("pure ACE: %.3f ms/step, %.3e atom-steps/s" % (ms_p / args.pure_steps, value_p))

    # Eq. (1): per-atom times of the fast model, the precise model and the switching overhead, measured
    # separately, predict the speedup of the mixed loop over pure ACE
    eq1 = None
    if ms_p:
        ctx_f = ap.Context(n, max_nbr=128, skin=s["run"]["skin"])
        ctx_f.set_potential(s["eam"], s["ace"], s["sw"], lambda_mode=ap.AP_LAMBDA_FAST)
        log("pure EAM: 100 timed steps ...")
        ms_f, _, prof_f, _ = run_md(ctx_f, s, pos0, vel0, 100, 5, 0)
        ctx_f.close()
        x = window["x_mean"]
        t_p, t_f, t_m = ms_p / args.pure_steps / n, ms_f / 100 / n, ms / args.steps / n
        sw_ms = sum(prof[k][0] for k in ("csp_value", "compact", "W") if k in prof)
        sw_ms += sum(max(0.0, prof[k][0] - prof_f.get(k, (0.0,))[0]) for k in ("dens_desc",))
        t_d = sw_ms / n
        # the force kernel of the mixed step also gathers the ACE pair terms and the grad-lambda terms:
        # what it costs above the EAM-only force kernel counts with the overhead too
        t_d += max(0.0, prof["force"][0] - prof_f["force"][0]) / n if "force" in prof and "force" in prof_f else 0.0
        eq1 = dict(t_precise_ns=t_p * 1e6, t_fast_ns=t_f * 1e6, t_switch_ns=t_d * 1e6, x=x,
                   s_measured=t_p / t_m,
                   s_eq1_paper=t_p / (x * t_p + (1 - x) * t_f + t_d),
                   s_eq1_all_eam=t_p / (x * t_p + t_f + t_d))
        eq1["rel_err_all_eam"] = eq1["s_eq1_all_eam"] / eq1["s_measured"] - 1.0
        # the precise model's cost per atom inside the mixed step (a few thousand atoms fill the GPU
        # less well than the pure run's 128k): with it, Eq. (1) predicts the mixed step itself
        t_pm = sum(prof[k][0] for k in ("ace_basis", "ace_energy", "ace_pairforce") if k in prof) / max(1.0, x * n)
        eq1["t_precise_in_mixed_ns"] = t_pm * 1e6
        eq1["s_eq1_mixed_tp"] = t_p / (x * t_pm + t_f + t_d)
        log("Eq. (1): measured %.2f, predicted %.2f (EAM on all atoms), %.2f (paper form)" %
            (eq1["s_measured"], eq1["s_eq1_all_eam"], eq1["s_eq1_paper"]))

    # roofline of the dominant kernel of the mixed step
    cost = ctx.ace_cost()
    cnt_rc, _ = ctx.nblist_build(pos0, box, s["ace"]["rc"], 128)
    cnt_w, _ = ctx.nblist_build(pos0, box, max(s["ace"]["rc"], s["sw"]["r_w"]) + s["run"]["skin"], 128)
    nnb_rc = float(cnt_rc.double().mean().item())
    nnb = float(cnt_w.double().mean().item())
    n_s = window["x_mean"] * n
    n_near, nnb_short = near_counts(ctx, pos0, box, max(s["ace"]["rc"], s["sw"]["r_w"]) + s["run"]["skin"],
                                    max(s["eam"]["r_rho"], s["eam"]["r_phi"]) + s["run"]["skin"], 128)
    tot = {k: v[0] * v[1] for k, v in prof.items()}
    dom = max(tot, key=tot.get)
    avg_ms, launches = prof[dom]
    ace_per = {"ace_energy": cost["fixed_per_atom"], "ace_basis": nnb_rc * cost["per_neighbor_energy"],
               "ace_pairforce": nnb_rc * cost["per_neighbor_force"]}
    naive, t3, t2 = naive_ace_flops(s["ace"]["func"])
    if dom in ace_per:
        # achieved: the product basis by its plain definition (B2 + B3 + the adjoint, about 20 Mflop per atom
        # at n_max 12 / l_max 6) over the kernel's time; executed: the flops the coupling-block form performs
        per = naive if dom == "ace_energy" else ace_per[dom]
        flops = per * n_s
        achieved = flops / (avg_ms * 1e-3) / 1e12
        ex = ace_per[dom] * n_s / (avg_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / FP32_PEAK_TFLOPS, traffic=measured_traffic(dom), kernel=dom, avg_ms=avg_ms,
                    work_per_launch="%.4g flop (%.0f precise atoms x %.4g flop)" % (flops, n_s, per),
                    count="algorithmic: 16 x %d order-3 (m1, m2) terms + 2 x %d order-2 terms per atom" % (t3, t2)
                    if dom == "ace_energy" else "executed",
                    executed=dict(achieved=ex, frac=ex / FP32_PEAK_TFLOPS, flop_per_atom=ace_per[dom],
                                  note="flops the coupling-block kernels perform (ap_ace_cost)"))
    else:
        b = algorithmic_bytes(dom, n, nnb, n_s, nnb_rc, s["sw"]["n_csp"], n_near, nnb_short)
        achieved = b / (avg_ms * 1e-3) / 1e9 if b else None
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=(achieved / HBM_PEAK_GBS) if achieved else None, traffic=measured_traffic(dom), kernel=dom,
                    avg_ms=avg_ms, work_per_launch="%.4g B" % (b or 0))
    kernels = {k: dict(avg_ms=round(v[0], 5), launches=int(v[1]), share=round(tot[k] / sum(tot.values()), 4))
               for k, v in sorted(prof.items(), key=lambda kv: -tot[kv[0]])}
    r_list = max(s["ace"]["rc"], s["sw"]["r_w"]) + s["run"]["skin"]
    nbr_roof = nbr_build_roofline(ctx, pos0, box, r_list, 128)
    log("nbr build: %.1f us, %.0f GB/s" % (nbr_roof["avg_ms"] * 1e3, nbr_roof["GBs"]))
    hbm = {}
    for k in ("dens_desc", "force", "W"):
        if k in prof:
            b = algorithmic_bytes(k, n, nnb, n_s, nnb_rc, s["sw"]["n_csp"], n_near, nnb_short)
            hbm[k] = dict(GBs=b / (prof[k][0] * 1e-3) / 1e9, frac=b / (prof[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          algorithmic_bytes=b, traffic=measured_traffic(k))
    ace_roof = {}
    for tag, pf, ns in (("mixed", prof, n_s), ("pure_ace", prof_p, float(n))):
        for k in ("ace_basis", "ace_energy", "ace_pairforce"):
            if k in pf:
                tf = ace_per[k] * ns / (pf[k][0] * 1e-3) / 1e12
                ace_roof.setdefault(tag, {})[k] = dict(TFLOPs=tf, frac=tf / FP32_PEAK_TFLOPS, avg_ms=pf[k][0])

    contrast = None
    if args.contrast_steps > 0:
        # from the state the drift leg ends in (equilibrated), like the paper's runs at room temperature
        contrast = conservation_contrast(s, eq_state["pos"], eq_state["vel"], args.contrast_steps)
    dts = None
    if args.dt_steps > 0:
        dts = dt_study(s, eq_state["pos"], eq_state["vel"], args.dt_steps)

    large = None
    if args.large_steps > 0:
        try:
            large = large_run(args.large_steps, 50, 3)
        except Exception as e:  # reported, not fatal to the headline line
            large = dict(error=repr(e))

    learned = None
    if args.learned_steps > 0:
        try:
            learned = learned_comparison(args.learned_steps, 50)
        except Exception as e:  # reported, not fatal to the headline line
            learned = dict(error=repr(e))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, %d steps) ..." % args.cpu_steps)
        cpu = cpu_baseline(s, args.cpu_steps, window["x_mean"])
        log("cpu: %.3e atom-steps/s on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (ACE) + f64 (EAM, switching, forces, integration)",
        "data": "synthetic (seeded; see synth/configs.py)",
        "config": {"workload": s["name"], "n_atoms": n, "lattice": "bcc a=3.16 40^3, screw dipole",
                   "ace_basis": int(len(s["ace"]["func"])), "n_max": 12, "l_max": 6, "r_w": s["sw"]["r_w"],
                   "dt_fs": 1.0, "x": window["x_mean"]},
        "pure_ace": {"value": value_p, "unit": "atom-steps/s", "steps": args.pure_steps,
                     "ms_per_step": ms_p / args.pure_steps if ms_p else None},
        "speedup_vs_pure_ace": value / value_p if value_p else None,
        "speedup_eq1": eq1,
        "nve": nve,
        "roofline": roof,
        "ace_roofline": ace_roof,
        "hbm_kernels": hbm,
        "nbr_build": nbr_roof,
        "conservation_contrast": contrast,
        "dt_study": dts,
        "path_counts": {"n_near_precise": n_near, "nnb_list": nnb, "nnb_eam_short": nnb_short, "nnb_ace": nnb_rc},
        "kernels": kernels,
        "kernels_timed_every_nth_step": PROF_EVERY,
        "cpu_baseline": cpu,
        "learned_indicator": learned,
        "large_fcc_penny_crack": large,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
