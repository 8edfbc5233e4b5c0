/*
 * ap.h - C ABI of the MI355X (gfx950) library for the conservative adaptive-precision EAM/ACE
 * energy and force evaluation of Immel, Drautz and Sutmann, "Conservative adaptive-precision
 * interatomic potentials" (arXiv 2512.07693).
 *
 * What one evaluation computes (paper's notation):
 *   E_i   = lambda_i E^f_i + (1 - lambda_i) E^p_i                               Eq. (4)
 *   lambda_i = f_trans(d_i, d_lo, d_hi)                                          Eq. (2), (S1)
 *   d_i   = sum_k g_k w(r_ik) / wbar_i - d0,  wbar_i = sum_k w(r_ik)              Eq. (6)
 *   g_i   = CSP_i^list (pairs fixed at set-up)                                   (B3)
 *           or the learned indicator of ap_set_mlp (a network on invariant features)
 *   E^f   = EAM (B1) on every atom; E^p = ACE on the atoms with lambda_i < 1
 *   F_i   = -grad_i sum_k E_k, assembled in the pair form (A1)-(A2) with the EAM,
 *           ACE and grad-lambda contributions (S12), (S14), (S21), (S27)-(S29).
 *
 * Conventions (all entry points):
 *   - Metal units: Angstrom, eV, ps, atomic mass units.
 *   - Per-step arrays (positions, velocities, forces, per-atom outputs) are DEVICE pointers
 *     owned by the caller. Positions, velocities and forces are FP64 structure-of-arrays
 *     [3][n]: the x block, then the y block, then the z block. Per-atom arrays are [n].
 *   - Atom order is the caller's; atom index = the unique identifier the CSP list refers to.
 *   - Potential parameters (ap_*_params) are HOST structures with HOST arrays; they are copied
 *     into library-owned device tables by ap_set_potential.
 *   - Outputs are overwritten, never accumulated. Output pointers documented "optional" may be
 *     NULL.
 *   - Each call enqueues its kernels on the context's HIP stream and synchronises that stream
 *     before returning, so that device-side error flags (neighbour overflow, non-finite values)
 *     are reported in the return code. The library never allocates memory visible to the caller;
 *     it owns only scratch (cell lists, neighbour lists, per-atom intermediates, ACE buffers).
 *   - Return codes: AP_OK (0) or a negative AP_E_* code; ap_last_error() then gives the text.
 *     No C++ exception crosses the ABI.
 *   - A context is not thread safe: calls on one context must not overlap.
 */
#ifndef AP_H
#define AP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AP_OK 0
#define AP_E_ARG -1          /* null pointer, size out of range, unsupported option          */
#define AP_E_BOX -2          /* a cutoff (+ skin) >= half the box                             */
#define AP_E_NBR_OVERFLOW -3 /* an atom has more neighbours than max_nbr                      */
#define AP_E_NONFINITE -4    /* non-finite energy or force, or non-positive embedding density */
#define AP_E_HIP -5          /* a HIP runtime call failed                                     */
#define AP_E_CSP -6          /* n_csp not 8 or 12, list entry out of range, too few neighbours */
#define AP_E_STATE -7        /* call order: potential or CSP list not set                     */

#define AP_FP64 0
#define AP_FP32 1

#define AP_LAMBDA_COMPUTED -1 /* lambda from the descriptor, Eq. (2)                    */
#define AP_LAMBDA_PRECISE 0   /* lambda == 0 everywhere: pure ACE (paper orientation)    */
#define AP_LAMBDA_FAST 1      /* lambda == 1 everywhere: pure EAM                         */

#define AP_MIX_ENERGY 0 /* the conservative adaptive-precision force of Eq. (4)-(5)                */
#define AP_MIX_FORCE 1  /* force mixing, Eq. (3): F_i = lambda_i F^f_i + (1 - lambda_i) F^p_i (the
                           paper's non-conservative comparison; no energy behind it, no virial)     */

#define AP_IND_CSP 0 /* g = CSP^list of (B3)                                                  */
#define AP_IND_MLP 1 /* g = learned indicator: the network set by ap_set_mlp (no CSP list needed) */

/* Orthorhombic periodic box with its origin at 0. */
typedef struct {
    double L[3];
} ap_box;

/* Finnis-Sinclair EAM, (B1): density zeta(r) = (r-r_rho)^2 + beta (r-r_rho)^3 / r_rho for r < r_rho,
 * pair Phi(r) = (r-r_phi)^2 (c0 + c1 r + c2 r^2) for r < r_phi (both zero beyond), embedding
 * xi(z) = -A sqrt(z). */
typedef struct {
    double A, beta, c0, c1, c2, r_rho, r_phi;
} ap_eam_params;

/* ACE (the paper cites the definition; the concrete form is):
 *   radial channels g_n(r) = T_n(2r/rc - 1) (1 + cos(pi r / rc)) / 2, n < n_max
 *   atomic basis A_{n l m} = sum_{j: r_ij < rc} g_n(r_ij) Y_l^m(rhat_ij), l <= l_max
 *   product basis: order 1 A_{n00}; order 2 sum_m (-1)^m A_{n1 l m} A_{n2 l -m};
 *                  order 3 sum (l1 l2 l3; m1 m2 m3) A_{n1 l1 m1} A_{n2 l2 m2} A_{n3 l3 m3}
 *   site energy E^p_i = E0 + sum_nu c_nu B_i,nu - emb_A sqrt(phi2_i),
 *               phi2_i = sum_n b_dens[n] sqrt(4 pi) A_{i,n00}   (no embedding if phi2 <= 0)
 * func: [n_funcs][6] int32 rows (n1,l1,n2,l2,n3,l3), -1 in unused slots; order-2 rows have
 * l1 == l2, order-3 rows satisfy the triangle rule with an even l1+l2+l3.
 * Supported (n_max, l_max): (4,2), (8,4), (12,6). precision: AP_FP64 or AP_FP32 (basis and
 * product arithmetic in FP32; geometry, energy sums and forces in FP64). */
typedef struct {
    int n_max, l_max, n_funcs;
    double rc;
    const int32_t *func;
    const double *c;
    const double *b_dens;
    double emb_A, E0;
    int precision;
} ap_ace_params;

/* Switching, Eq. (2), (6) and the weighting function of App. B:
 * w(r) = f_trans(r, r_w - 1 A, r_w); the sums of Eq. (6) include k = i (w(0) = 1).
 * lambda_mode: AP_LAMBDA_COMPUTED / _PRECISE / _FAST. grad_lambda: 1 conservative forces;
 * 0 drops the grad-lambda contributions (the non-conservative "AP without grad lambda" force).
 * mixing: AP_MIX_ENERGY (Eq. (4)-(5)) or AP_MIX_FORCE (Eq. (3): the complete EAM and ACE forces of
 * each atom weighted by its own lambda_i; ACE then runs on the atoms with lambda < 1 and on every atom
 * within the ACE cutoff of one; energies are still those of Eq. (4), the virial output is zero). */
typedef struct {
    double d_lo, d_hi, r_w, d0;
    int n_csp;
    int lambda_mode;
    int indicator;
    int grad_lambda;
    int mixing;
} ap_switch_params;

typedef struct ap_ctx ap_ctx;

/* Create a context for up to n_max_atoms atoms and max_nbr neighbours per atom within the list
 * radius max(rc_eam, rc_ace, r_w) + skin. hip_stream: a hipStream_t (NULL = default stream).
 * Returns AP_OK and *out, or an error (then *out = NULL). */
int ap_ctx_create(ap_ctx **out, int n_max_atoms, int max_nbr, double skin, void *hip_stream);
void ap_ctx_destroy(ap_ctx *ctx);
/* Text of the last error on ctx (or of the last failed ap_ctx_create when ctx is NULL). */
const char *ap_last_error(const ap_ctx *ctx);

/* Copy the potentials and switching parameters into device tables (the coupling tables of the
 * real-harmonic ACE form are derived here). Must precede every evaluation. */
int ap_set_potential(ap_ctx *ctx, const ap_eam_params *eam, const ap_ace_params *ace, const ap_switch_params *sw);

/* New ACE coefficients without rebuilding the tables: coeffs (device [n_funcs], the rows of the installed
 * ap_ace_params.func) and b_dens (device [n_max]), each optional (NULL keeps the installed values). The
 * result equals ap_set_potential with the same basis and the new values (for fitting loops: no host round
 * trip). AP_E_ARG when the installed basis repeats a row; AP_E_STATE before ap_set_potential. */
int ap_set_ace_coefficients(ap_ctx *ctx, const double *coeffs, const double *b_dens);

/* One-time detection of the CSP opposite-neighbour pairs, (B3): for every atom the n_csp
 * nearest neighbours by (|u|^2, index) are paired greedily by the smallest |u_a + u_b|^2 (ties:
 * smaller lower index, then smaller higher index); pairs are written in choice order with the
 * lower index first, so entries 2p and 2p+1 are opposite partners.
 * pos_ref: device [3][n], the initial structure. csp_list: device [n][n_csp] int32 output.
 * The list is also installed in ctx (as by ap_set_csp_list). */
int ap_csp_pairs_build(ap_ctx *ctx, int n, const double *pos_ref, const ap_box *box, int n_csp, int32_t *csp_list);

/* Install a CSP pair list (device [n][n_csp], same layout) and build its reverse list. */
int ap_set_csp_list(ap_ctx *ctx, int n, int n_csp, const int32_t *csp_list);

/* Atoms with a constant switching parameter (App. B, the paragraph after (B4)): lam_fix device [n]
 * int32, -1 = lambda from Eq. (2), 0 or 1 = lambda fixed at that value with dlambda/dd = 0 (the
 * grad-lambda terms of that atom vanish and (B4) stays the exact force). The mask is copied into the
 * context and applies to every later evaluation with a computed lambda; NULL removes it. Any other
 * value returns AP_E_ARG (and the mask is not installed). */
int ap_set_lambda_fixed(ap_ctx *ctx, int n, const int32_t *lam_fix);

/* Neighbour sets at radius r_list (strict |u|^2 < r_list^2, minimum image, positions wrapped
 * into the box first): nbr_count device [n]; nbr_idx device [max_nbr][n] (slot-major: the k-th
 * neighbour of atom i is nbr_idx[k * n + i]). Slot order, with max_nbr <= 256: the neighbours inside
 * max(r_rho, r_phi) + skin of the context's EAM come first, then the rest, each part in ascending atom
 * index; with more slots, the order of a scan of the 27 cells. */
int ap_nblist_build(ap_ctx *ctx, int n, const double *pos, const ap_box *box, double r_list, int max_nbr,
                    int32_t *nbr_count, int32_t *nbr_idx);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the neighbour sets of ap_nblist_build without a context. The
 * library's scratch for it (wrapped positions, cell arrays and records, flags; 11.0 MiB) is one static
 * device array per GPU, held until the process ends; the call allocates nothing. Limits: n <= 131072
 * atoms and at most 131072 cells (cells of edge >= r_list, floor(L / r_list) per axis); larger inputs
 * return AP_E_ARG before anything is launched. Same arguments and output layout as ap_nblist_build
 * (pos, nbr_count, nbr_idx device; box host; strict |u|^2 < r_list^2 after wrapping); the slots of an
 * atom hold its neighbours in ascending atom index when max_nbr <= 256, else in the order of a scan of
 * the 27 cells. hip_stream: a hipStream_t (NULL =
 * default stream); the call synchronises it to report overflow (AP_E_NBR_OVERFLOW). Calls that overlap
 * on one GPU (other threads or streams) share the scratch and race: serialise them. Errors are read
 * with ap_last_error(NULL). */
int ap_nblist_build_noalloc(int n, const double *pos, const ap_box *box, double r_list, int max_nbr,
                            int32_t *nbr_count, int32_t *nbr_idx, void *hip_stream);

/* EAM, (B1) and (S12): E_atom[i] = E^EAM_i, F = sum_k (lambda_i f_ki - lambda_k f_ik) with
 * lambda = the device array lambda [n] (NULL: lambda == 1, i.e. the plain EAM force (S13)).
 * E_tot: device [1]; virial9: device [9] row-major W_ab = -sum_e (dE/du_e)_a (u_e)_b over the
 * relative vectors u_e the energy depends on. All outputs optional. */
int ap_eam_eval(ap_ctx *ctx, int n, const double *pos, const int32_t *species, const ap_box *box,
                const double *lambda, double *E_tot, double *E_atom, double *F, double *virial9);

/* Switching quantities, (B3), Eq. (6), Eq. (2): g, d, wbar, lambda, dlambda/dd (device [n],
 * each optional) and n_precise = |{i : lambda_i < 1}| (device [1], optional). */
int ap_switch_eval(ap_ctx *ctx, int n, const double *pos, const ap_box *box, double *g, double *d, double *wbar,
                   double *lambda, double *dlambda, int32_t *n_precise);

/* ACE site energies E^p_i and the pure-ACE force F = sum_k (f_ki - f_ik) (S13 with ACE pair
 * contributions) on the atoms listed in subset (device [n_subset], NULL = all atoms); atoms not
 * in the subset contribute no energy. E_atom [n], F [3][n], virial9 [9], E_tot [1]: optional. */
int ap_ace_eval(ap_ctx *ctx, int n, const double *pos, const int32_t *species, const ap_box *box,
                const int32_t *subset, int n_subset, double *E_tot, double *E_atom, double *F, double *virial9);

/* ACE on a ragged batch of periodic cells in one launch, with the adjoint with respect to the ACE
 * coefficients: structure s holds atoms offsets[s] .. offsets[s+1]-1 of pos (device [3][n],
 * n = offsets[n_struct]) in the orthorhombic box boxes[3s..3s+2] (host arrays offsets [n_struct+1],
 * boxes [n_struct][3]). With w_i = weight[i] (device [n], NULL = 1), i.e. the ACE weight 1 - lambda_i
 * of Eq. (4):
 *   E_struct[s]      = sum_{i in s} w_i E^p_i                        device [n_struct]
 *   F                = -grad of sum_s E_struct[s]                    device [3][n]          (optional)
 *   dEdc[s][nu]      = sum_{i in s} w_i B_i,nu = dE_struct/dc_nu     device [n_struct][n_funcs] (opt.)
 *   dEdb[s][n]       = sum_{i in s} w_i xi'(phi2_i) sqrt(4 pi) A_i,n00  device [n_struct][n_max] (opt.)
 * where nu indexes the rows of ap_ace_params.func. The coefficients are those of ap_set_potential. */
int ap_ace_batch_eval(ap_ctx *ctx, int n_struct, const int32_t *offsets, const double *boxes, const double *pos,
                      const double *weight, double *E_struct, double *F, double *dEdc, double *dEdb);

/* Vector-Jacobian product of the batch forces with respect to the ACE coefficients (fitting to forces).
 * With the batch, weights and F of ap_ace_batch_eval and an upstream gradient G (device [3][n], one
 * vector per atom), L = sum_k G_k . F_k and, per structure s (its own atoms; the cells are independent):
 *   dLdc[s][nu] = dL/dc_nu = -sum_{i in s} w_i Bdot_i,nu                   device [n_struct][n_funcs] (opt.)
 *   dLdb[s][n]  = dL/db_n  = -sum_{i in s} w_i d/dt [xi'(phi2_i) sqrt(4 pi) A_i,n00]  device [n_struct][n_max]
 * where d/dt, written Bdot, is the derivative along the motion r_k -> r_k + t G_k of the atoms (each
 * neighbour vector u_ij moves with G_j - G_i): F is linear in c, and d/dc of F = -grad E is minus the
 * gradient of dE/dc = sum_i w_i B_i. The coefficients are those of ap_set_potential. */
int ap_ace_batch_force_vjp(ap_ctx *ctx, int n_struct, const int32_t *offsets, const double *boxes, const double *pos,
                           const double *weight, const double *G, double *dLdc, double *dLdb);

/* The adaptive-precision evaluation: Eq. (4) energies and the conservative force Eq. (5).
 * E_tot [1], E_atom [n], F [3][n], virial9 [9], lambda_out [n]: device, each optional. */
int ap_mixed_energy_forces(ap_ctx *ctx, int n, const double *pos, const int32_t *species, const ap_box *box,
                           double *E_tot, double *E_atom, double *F, double *virial9, double *lambda_out);

/* n_steps of velocity Verlet (NVE, FP64) with the adaptive-precision forces:
 * v += dt/2 F/m; x += dt v (wrapped); F = F(x); v += dt/2 F/m.  F must hold F(x) on entry (from
 * ap_mixed_energy_forces) and holds F(x) on exit. mass: atomic mass (u) of the single species.
 * thermo: device [n_steps][8] rows {E_pot, E_kin, E_tot, P_x, P_y, P_z, n_precise, rebuilt}.
 * The neighbour list is rebuilt only when an atom moved more than skin/2 since the last build. */
int ap_vv_step(ap_ctx *ctx, int n, double *pos, double *vel, double *F, double mass, double dt, int n_steps,
               const ap_box *box, double *thermo);

/* Measurement support (not part of the method).
 * ap_set_profiling: on != 0 records HIP events on the context stream around every kernel group
 * (neighbour list, CSP value or learned indicator, density/descriptor, compaction, ACE basis, ACE
 * energy, ACE pair gradients, W, learned-indicator gradients, force assembly, reductions,
 * velocity-Verlet kernels) and clears the accumulated times. With on = k > 1, ap_vv_step times only
 * the launches of every k-th step (steps 0, k, 2k, ...), so that the event records, which cost a few
 * microseconds each, stay out of the other steps; the other entry points time every launch.
 * ap_get_profile: returns the number of kernel groups m (or an error) and fills, for the first
 * max_entries of them, names [m][32] (NUL-terminated), the average duration in ms and the count of
 * timed launches (host arrays, each optional). */
int ap_set_profiling(ap_ctx *ctx, int on);
int ap_get_profile(ap_ctx *ctx, int max_entries, char *names, double *avg_ms, int64_t *count);

/* Floating-point operations the ACE kernels perform with the installed basis (host doubles):
 * per precise atom independent of its neighbours (orders 2-3 values and adjoints), per neighbour
 * inside the ACE cutoff in the energy kernel, and per neighbour in the pair-gradient kernel. */
int ap_ace_cost(ap_ctx *ctx, double *fixed_per_atom, double *per_neighbor_energy, double *per_neighbor_force);

/* ---------------------------------------------------------------------------------------------
 * Learned switching indicator. Eq. (6) accepts any per-atom g; here g_i = softplus(o_i) of a
 * 16-64-64-1 network (SiLU, FP32) on sixteen rotation invariants of the neighbours inside rc:
 *   q[n] = sum_j g_n(r_ij) (n = 0..7, the Chebyshev channels of the ACE basis, cutoff rc);
 *   q[8 + 4n + l - 1] = sum_m A_nlm^2 with A_nlm = sum_j g_n(r_ij) Y_lm(rhat_ij), n = 0, 1, l = 1..4.
 * Its force is the general grad-g term of (S16): F_i += sum_j W_j grad_i g_j, W_j of (S25).
 * Parameter block (AP_MLP_NPARAMS floats, device memory):
 *   mu[16] sig[16] W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3;  z = (q - mu) / sig,
 *   h1 = silu(W1 z + b1), h2 = silu(W2 h1 + b2), o = w3 . h2 + b3, g = softplus(o).
 * The network is trained on o against log(|E^ACE_i - E^EAM_i| + eps) (the caller builds targets).
 * ------------------------------------------------------------------------------------------- */
#define AP_MLP_NQ 16
#define AP_MLP_NPARAMS 5345

/* Copies the parameter block (device pointer) into the context and sets the feature cutoff rc;
 * used by every evaluation whose switching parameters select AP_IND_MLP. */
int ap_set_mlp(ap_ctx *ctx, const float *params, double rc);
/* Features q[n][16] (device, FP32) of every atom of one periodic cell (pos device SoA [3][n]). */
int ap_mlp_features(ap_ctx *ctx, int n, const double *pos, const ap_box *box, double rc, float *q);
/* g[m] and, if dgdq != NULL, dg/dq [m][16] of m feature rows q[m][16] (all device, FP32). */
int ap_mlp_eval(ap_ctx *ctx, int m, const float *q, const float *params, float *g, float *dgdq);
/* Loss L = (1/m) sum_s (o_s - t_s)^2 over m samples (device q[m][16], t[m]) and its gradient with
 * respect to every parameter (device grad[AP_MLP_NPARAMS]; 0 for mu and sig); *loss on the host.
 * m is limited only by device memory (274 floats of scratch per sample). */
int ap_mlp_loss_grad(ap_ctx *ctx, int m, const float *q, const float *target, const float *params, float *grad,
                     double *loss);
/* Adam training (beta 0.9 / 0.999, eps 1e-8, learning rate lr) over epochs x floor(m / batch)
 * mini-batches in the given sample order (the ragged tail of each epoch is left out). fit_norm != 0
 * first sets mu and sig to the mean and standard deviation of the features. params (device) are
 * updated in place; loss_hist (host, may be NULL) receives the mean batch loss of each epoch. */
int ap_mlp_train(ap_ctx *ctx, int m, const float *q, const float *target, int batch, int epochs, double lr,
                 int fit_norm, float *params, double *loss_hist);

#ifdef __cplusplus
}
#endif
#endif
