// C ABI entry points (include/ap.h): argument checks, the evaluation pipeline and velocity Verlet.
#include <algorithm>
#include <cstring>

#include "ap_internal.h"

// text of the last error of a call without a context (a fixed buffer: setting it allocates nothing)
static thread_local char g_create_error[256];

namespace ap {

int set_error_text(int code, const char *msg) {
    std::strncpy(g_create_error, msg, sizeof(g_create_error) - 1);
    g_create_error[sizeof(g_create_error) - 1] = 0;
    return code;
}

int set_error(ap_ctx *c, int code, const std::string &msg) {
    if (c)
        c->err = msg;
    else
        set_error_text(code, msg.c_str());
    return code;
}

int hip_check(ap_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return AP_OK;
    return set_error(c, AP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static hipEvent_t take_event(ap_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(ap_ctx *ctx, const char *name) : c(ctx) {
    if (!c->prof_on || c->prof_skip) return;
    for (size_t q = 0; q < c->prof_names.size(); q++)
        if (c->prof_names[q] == name) label = (int)q;
    if (label < 0) {
        label = (int)c->prof_names.size();
        c->prof_names.push_back(name);
        c->prof_ms.push_back(0.0);
        c->prof_cnt.push_back(0);
    }
    a = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
}

ProfScope::~ProfScope() {
    if (!c->prof_on || !a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({label, a, b});
}

void prof_resolve(ap_ctx *c) {
    for (const auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof_ms[p.label] += ms;
            c->prof_cnt[p.label] += 1;
        }
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
}

int sync_and_check(ap_ctx *c) {
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (rc) return rc;
    prof_resolve(c);
    int flags[4];
    rc = hip_check(c, hipMemcpy(flags, c->d_flags, sizeof(flags), hipMemcpyDeviceToHost), "flags");
    if (rc) return rc;
    const int e = flags[1];
    // a list built from non-finite positions, or truncated, is not kept: the next call rebuilds it
    if (e & (kErrOverflow | kErrAceNbr | kErrAsym | kErrNonFinite)) c->list_r = -1;
    if (e & kErrOverflow) return set_error(c, AP_E_NBR_OVERFLOW, "neighbour count above max_nbr, or index out of range");
    if (e & kErrAceNbr) return set_error(c, AP_E_NBR_OVERFLOW, "more than 128 neighbours inside the ACE cutoff");
    if (e & kErrCsp) return set_error(c, AP_E_CSP, "CSP list invalid or too few neighbours for the CSP pairs");
    if (e & kErrAsym) return set_error(c, AP_E_NBR_OVERFLOW, "neighbour lists not symmetric (truncated list)");
    if (e & kErrNonFinite) return set_error(c, AP_E_NONFINITE, "non-finite energy or force");
    if (e & kErrLamFix) return set_error(c, AP_E_ARG, "constant switching parameters must be -1, 0 or 1");
    return AP_OK;
}

static double list_radius(const ap_ctx *c, bool switching) {
    double r = std::max(std::max(c->eam.r_rho, c->eam.r_phi), c->ace.rc);
    if (switching) r = std::max(r, c->sw.r_w);
    if (switching && c->sw.indicator == AP_IND_MLP) r = std::max(r, c->mlp_rc);
    return r + c->skin;
}

static int nblocks(int n) { return (n + kBlock - 1) / kBlock; }

// The force evaluation on the positions already in c->pos.
static int evaluate(ap_ctx *c, int n, const double *box, const EvalFlags &f, const double *lam_in,
                    const int32_t *subset, int n_subset, bool run_ace, double *E_tot, double *E_atom, double *F,
                    double *virial, bool force_list, bool skin_checked = false, bool reduce = true) {
    int rc;
    {
        ProfScope p(c, "nbr_list");
        // the rebuild flag is committed by the density pass below
        rc = ensure_list(c, n, box, list_radius(c, f.switching), force_list, skin_checked, false);
    }
    if (rc) return rc;
    if (f.switching && c->sw.indicator == AP_IND_MLP) {
        ProfScope p(c, "mlp_indicator");
        launch_mlp_indicator(c, n, box);
    } else if (f.switching) {
        ProfScope p(c, "csp_value");
        launch_csp_value(c, n, box);
    }
    const bool counted = run_ace && !subset && !f.force_mix && n <= kCountedCompactMax;
    {
        ProfScope p(c, "dens_desc");
        launch_dens_desc(c, n, box, f, lam_in, counted);
    }
    // the precise atoms stamp themselves and their list neighbours (ACE pair kernel) for the W pass
    c->stamp_gen = c->stamp_gen == 0x7fffffff ? 1 : c->stamp_gen + 1;
    if (run_ace && f.force_mix) {
        // Eq. (3): ACE on the atoms with lambda < 1 and on every atom within the ACE cutoff of one
        {
            ProfScope p(c, "compact");
            launch_mix_mark(c, n, box);
            launch_compact_marked(c, n);
        }
        rc = launch_ace(c, n, box, std::min(n, 8192));
        if (rc) return rc;
    } else if (run_ace) {
        {
            ProfScope p(c, "compact");
            launch_compact(c, n, subset, n_subset, counted);
        }
        rc = launch_ace(c, n, box, std::min(n, 8192));
        if (rc) return rc;
    } else {
        launch_fill_int(c, c->sidx, -1, n);
        launch_fill_int(c, c->d_flags + 2, 0, 1);
    }
    // with the stamps, W != 0 only near S: the W pass marks the atoms with reverse CSP terms
    const bool stamped = run_ace && !subset;
    // (with the learned indicator, the list neighbours of each atom with W != 0, which receive its
    // grad-g terms)
    const bool csp_marks = stamped && (c->sw.indicator == AP_IND_MLP || c->n_csp > 0);
    if (f.switching && f.grad_lambda && !f.force_mix) {
        ProfScope p(c, "W");
        launch_W(c, n, box, stamped, csp_marks);
    }
    if (f.switching && f.grad_lambda && !f.force_mix && c->sw.indicator == AP_IND_MLP) {
        ProfScope p(c, "mlp_gradg");
        launch_mlp_gradg(c, n, box);
    }
    {
        ProfScope p(c, "force");
        launch_force(c, n, box, f, E_atom, F, nullptr, lam_in == nullptr,
                     csp_marks && f.switching && f.grad_lambda && !f.force_mix);
    }
    if (reduce) {
        ProfScope p(c, "reduce");
        launch_reduce(c, force_blocks(n), E_tot, virial);
    }
    return hip_check(c, hipGetLastError(), "evaluate");
}

static int check_common(ap_ctx *c, int n, const double *pos, const ap_box *box, bool need_pot) {
    if (!c) return AP_E_ARG;
    if (n <= 0 || n > c->n_cap) return set_error(c, AP_E_ARG, "n out of range (1..n_max_atoms)");
    if (!pos || !box) return set_error(c, AP_E_ARG, "null positions or box");
    for (int a = 0; a < 3; a++)
        if (!(box->L[a] > 0) || !std::isfinite(box->L[a])) return set_error(c, AP_E_ARG, "box lengths must be > 0");
    if (need_pot && !c->have_pot) return set_error(c, AP_E_STATE, "ap_set_potential has not been called");
    return AP_OK;
}

static int check_csp(ap_ctx *c, int n) {
    if (c->sw.indicator == AP_IND_MLP) {
        if (!c->have_mlp) return set_error(c, AP_E_STATE, "the learned indicator needs ap_set_mlp");
        return AP_OK;
    }
    if (!c->csp_t || c->csp_n != n) return set_error(c, AP_E_STATE, "no CSP pair list for this atom count");
    return AP_OK;
}

static EvalFlags mixed_flags(const ap_ctx *c) {
    EvalFlags f;
    f.switching = c->sw.lambda_mode == AP_LAMBDA_COMPUTED;
    f.grad_lambda = c->sw.grad_lambda != 0;
    f.lam_const = c->sw.lambda_mode == AP_LAMBDA_FAST ? 1.0 : 0.0;
    f.eam_forces = true;
    f.ace_forces = true;
    f.force_mix = f.switching && c->sw.mixing == AP_MIX_FORCE;
    return f;
}

// ------------------------------------------------------------------------------------------
// Velocity Verlet kernels
// ------------------------------------------------------------------------------------------
// First half kick and drift. Also the neighbour-list work of the step's start: the skin check of the
// new positions (flags[0] |= 1 when an atom moved more than skin/2 since the last build) and zeroed
// cell counts for a rebuild (the geometry is that of the last build; a new one is cleared anew).
// First half-kick, drift and wrap, the skin check against the list's build positions, and the clearing
// of the cell counters for a possible rebuild.
__global__ __launch_bounds__(kBlock) void k_vv_first(double *pos, double *vel, const double *F, double *ipos, int n,
                                                     double hdtm, double dt, double Lx, double Ly, double Lz,
                                                     const double *__restrict__ pos_build, double half_skin2,
                                                     int *flags, int *cell_cnt, int *cell_fill, int ncell) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int q = i; q < ncell; q += gridDim.x * blockDim.x) {
        cell_cnt[q] = 0;
        cell_fill[q] = 0;
    }
    if (i >= n) return;
    const double L[3] = {Lx, Ly, Lz};
    double u[3];
    for (int a = 0; a < 3; a++) {
        const size_t o = (size_t)a * n + i;
        const double v = vel[o] + hdtm * F[o];
        vel[o] = v;
        const double x = wrap_coord(pos[o] + dt * v, L[a]);
        pos[o] = x;
        ipos[o] = x;
        u[a] = min_image_w(x - pos_build[o], L[a]);
    }
    // (a non-finite displacement also asks for a rebuild)
    if (!(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] <= half_skin2)) atomicOr(&flags[0], 1);
}

// The thermo row of the last step of a velocity-Verlet call (the earlier ones are taken by the density
// pass of the step after them).
__global__ __launch_bounds__(kBlock) void k_thermo(const double *partials, int nbf, int pstride, int *flags,
                                                   double *row) {
    thermo_row_block(partials, nbf, pstride, flags[2], flags[3], flags, row);
}

}  // namespace ap

using namespace ap;

extern "C" {

const char *ap_last_error(const ap_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error; }

void ap_ctx_destroy(ap_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    prof_resolve(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    ace_free(c);
    mlp_free(c);
    void *bufs[] = {c->csp_t, c->rev_start, c->rev_code, c->pos, c->pos_build, c->d_flags, c->cell_of, c->cell_cnt,
                    c->cell_start, c->cell_fill, c->cell_atoms, c->cell_rec, c->nbr_cnt, c->nbr_idx, c->g, c->d,
                    c->wbar, c->lam, c->dlam, c->Ef, c->Ep, c->Et, c->W, c->xip, c->sidx, c->slist, c->blk_cnt,
                    c->chunk_cnt, c->mark, c->fpair, c->frev, c->xg, c->xl, c->eb, c->xe, c->nbr_short, c->act, c->stamp, c->cmark, c->rslot, c->rstamp, c->list_gen, c->gbuf, c->partials, c->scalars, c->sid, c->b_off, c->b_box, c->bval,
                    c->lam_fix};
    for (void *p : bufs) (void)hipFree(p);
    delete c;
}

int ap_ctx_create(ap_ctx **out, int n_max_atoms, int max_nbr, double skin, void *hip_stream) {
    if (!out) return set_error(nullptr, AP_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_max_atoms <= 0 || max_nbr <= 0 || max_nbr > 1536 || !(skin >= 0.0))
        return set_error(nullptr, AP_E_ARG, "n_max_atoms > 0, 0 < max_nbr <= 1536, skin >= 0 required");
    ap_ctx *c = new ap_ctx();
    c->stream = (hipStream_t)hip_stream;
    c->n_cap = n_max_atoms;
    c->max_nbr = max_nbr;
    c->skin = skin;
    (void)hipGetDevice(&c->device);
    const size_t n = (size_t)n_max_atoms, nb = (size_t)nblocks(n_max_atoms);
    int rc = AP_OK;
    auto alloc = [&](auto **p, size_t count, size_t elem) {
        if (rc) return;
        rc = hip_check(c, hipMalloc((void **)p, std::max<size_t>(1, count * elem)), "context allocation");
    };
    alloc(&c->pos, 3 * n, 8);
    alloc(&c->pos_build, 3 * n, 8);
    alloc(&c->d_flags, 8, 4);
    alloc(&c->cell_of, n + 1, 4);
    alloc(&c->cell_atoms, n, 4);
    alloc(&c->cell_rec, n, sizeof(ap::CandRec));
    alloc(&c->nbr_cnt, n, 4);
    alloc(&c->nbr_idx, n * max_nbr, 4);
    alloc(&c->rslot, n * max_nbr, 4);
    alloc(&c->rstamp, n, 4);
    alloc(&c->list_gen, 1, 4);
    alloc(&c->nbr_short, n, 4);
    alloc(&c->act, n, 4);
    alloc(&c->stamp, n, 4);
    alloc(&c->cmark, n, 4);
    alloc(&c->lam_fix, n, 4);
    double **per_atom[] = {&c->g, &c->d, &c->wbar, &c->lam, &c->dlam, &c->Ef, &c->Ep, &c->Et, &c->W, &c->xip};
    for (double **p : per_atom) alloc(p, n, 8);
    alloc(&c->xg, n, sizeof(ap::Rec4));
    alloc(&c->xl, n, sizeof(ap::Rec4));
    alloc(&c->eb, n, sizeof(ap::Rec4));
    alloc(&c->xe, n, sizeof(ap::Rec4));
    alloc(&c->sidx, n, 4);
    alloc(&c->slist, n, 4);
    alloc(&c->mark, n, 4);
    alloc(&c->sid, n, 4);
    alloc(&c->blk_cnt, 2 * nb + 2, 4);
    alloc(&c->chunk_cnt, (n * kDensLanes + kBlock - 1) / kBlock, 4);
    c->pstride = (int)std::max<long long>((long long)nb, force_blocks((int)n));
    alloc(&c->partials, (size_t)c->pstride * 16, 8);
    alloc(&c->scalars, 16, 8);
    if (rc) {
        set_error_text(rc, c->err.c_str());
        ap_ctx_destroy(c);
        return rc;
    }
    launch_fill_int(c, c->d_flags, 0, 8);
    launch_fill_int(c, c->stamp, 0, (int)n);
    launch_fill_int(c, c->cmark, 0, (int)n);
    launch_fill_int(c, c->rstamp, -1, (int)n);
    launch_fill_int(c, c->list_gen, 0, 1);
    launch_fill_double(c, c->g, 0.0, (int)n);
    launch_fill_double(c, c->W, 0.0, (int)n);
    launch_fill_double(c, c->d, 0.0, (int)n);
    rc = hip_check(c, hipStreamSynchronize(c->stream), "context init");
    if (rc) {
        set_error_text(rc, c->err.c_str());
        ap_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return AP_OK;
}

int ap_set_potential(ap_ctx *c, const ap_eam_params *eam, const ap_ace_params *ace, const ap_switch_params *sw) {
    if (!c) return AP_E_ARG;
    if (!eam || !ace || !sw) return set_error(c, AP_E_ARG, "null parameter struct");
    if (!(eam->r_rho > 0) || !(eam->r_phi > 0) || !(ace->rc > 0)) return set_error(c, AP_E_ARG, "cutoffs must be > 0");
    if (sw->lambda_mode != AP_LAMBDA_COMPUTED && sw->lambda_mode != AP_LAMBDA_PRECISE &&
        sw->lambda_mode != AP_LAMBDA_FAST)
        return set_error(c, AP_E_ARG, "lambda_mode");
    if (sw->indicator != AP_IND_CSP && sw->indicator != AP_IND_MLP) return set_error(c, AP_E_ARG, "indicator");
    if (sw->mixing != AP_MIX_ENERGY && sw->mixing != AP_MIX_FORCE) return set_error(c, AP_E_ARG, "mixing");
    if (sw->lambda_mode == AP_LAMBDA_COMPUTED && (!(sw->d_hi > sw->d_lo) || !(sw->r_w > 1.0)))
        return set_error(c, AP_E_ARG, "switching parameters need d_hi > d_lo and r_w > 1 A");
    int rc = ace_setup(c, ace);
    if (rc) return rc;
    const int NA = ace->n_max * (ace->l_max + 1) * (ace->l_max + 1);
    const size_t es = ace->precision == AP_FP32 ? 4 : 8;
    // ACE scratch per S atom: A, the FP64 radial sums, two rows of dE/dA parts and four site-energy parts
    const size_t fb = (size_t)c->n_cap * c->max_nbr * 3 * es,
                 gb = (size_t)c->n_cap * (3 * NA * es + ace->n_max * sizeof(double) + 4 * sizeof(double));
    if (fb != c->fpair_bytes) {
        (void)hipFree(c->fpair);
        c->fpair = nullptr;
        (void)hipFree(c->frev);
        c->frev = nullptr;
        rc = hip_check(c, hipMalloc(&c->fpair, fb), "ACE pair buffer");
        if (!rc) rc = hip_check(c, hipMalloc(&c->frev, fb), "ACE reverse pair buffer");
        if (rc) return rc;
        c->fpair_bytes = fb;
    }
    if (gb != c->gbuf_bytes) {
        (void)hipFree(c->gbuf);
        c->gbuf = nullptr;
        rc = hip_check(c, hipMalloc(&c->gbuf, gb), "ACE adjoint buffer");
        if (rc) return rc;
        c->gbuf_bytes = gb;
    }
    c->eam = *eam;
    c->sw = *sw;
    c->have_pot = true;
    c->list_r = -1;
    return AP_OK;
}

int ap_set_ace_coefficients(ap_ctx *c, const double *coeffs, const double *b_dens) {
    if (!c) return AP_E_ARG;
    if (!c->have_pot) return set_error(c, AP_E_STATE, "ap_set_potential has not been called");
    int rc = ace_set_coefficients(c, coeffs, b_dens);
    if (!rc) rc = sync_and_check(c);
    return rc;
}

int ap_csp_pairs_build(ap_ctx *c, int n, const double *pos_ref, const ap_box *box, int n_csp, int32_t *csp_list) {
    int rc = check_common(c, n, pos_ref, box, false);
    if (rc) return rc;
    if (!csp_list) return set_error(c, AP_E_ARG, "csp_list is NULL");
    if (n_csp != 8 && n_csp != 12) return set_error(c, AP_E_CSP, "n_csp must be 8 or 12");
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos_ref, box->L);
    if (!rc) rc = build_csp_pairs(c, n, box->L, n_csp, csp_list);
    if (!rc) rc = sync_and_check(c);
    if (!rc) rc = install_csp(c, n, n_csp, csp_list);
    return rc;
}

int ap_set_csp_list(ap_ctx *c, int n, int n_csp, const int32_t *csp_list) {
    if (!c) return AP_E_ARG;
    if (n <= 0 || n > c->n_cap || !csp_list) return set_error(c, AP_E_ARG, "n or csp_list");
    int rc = install_csp(c, n, n_csp, csp_list);
    return rc;
}

__global__ void k_copy_fix(const int32_t *src, int n, int *dst, int *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int v = src[i];
    if (v < -1 || v > 1) {
        atomicOr(&flags[1], kErrLamFix);
        v = -1;
    }
    dst[i] = v;
}

int ap_set_lambda_fixed(ap_ctx *c, int n, const int32_t *lam_fix) {
    if (!c) return AP_E_ARG;
    if (!lam_fix) {
        c->have_fix = false;
        return AP_OK;
    }
    if (n <= 0 || n > c->n_cap) return set_error(c, AP_E_ARG, "n out of range (1..n_max_atoms)");
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    k_copy_fix<<<nblocks(n), kBlock, 0, c->stream>>>(lam_fix, n, c->lam_fix, c->d_flags);
    int rc = hip_check(c, hipGetLastError(), "lambda mask");
    if (!rc) rc = sync_and_check(c);
    c->have_fix = rc == AP_OK;
    return rc;
}

__global__ void k_copy_list(const int32_t *cnt, const int32_t *idx, int n, int max_out, int32_t *ocnt, int32_t *oidx,
                            int *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int k = cnt[i];
    if (k > max_out) {
        atomicOr(&flags[1], kErrOverflow);
        k = max_out;
    }
    ocnt[i] = cnt[i];
    for (int q = 0; q < k; q++) oidx[(size_t)q * n + i] = idx[(size_t)q * n + i];
}

int ap_nblist_build(ap_ctx *c, int n, const double *pos, const ap_box *box, double r_list, int max_nbr,
                    int32_t *nbr_count, int32_t *nbr_idx) {
    int rc = check_common(c, n, pos, box, false);
    if (rc) return rc;
    if (!(r_list > 0) || max_nbr <= 0 || !nbr_count || !nbr_idx) return set_error(c, AP_E_ARG, "list arguments");
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos, box->L);
    if (!rc) {
        ProfScope p(c, "nbr_build");  // one forced build: cells, sort, lists
        rc = ensure_list(c, n, box->L, r_list, true);
    }
    if (!rc) {
        k_copy_list<<<nblocks(n), kBlock, 0, c->stream>>>(c->nbr_cnt, c->nbr_idx, n, max_nbr, nbr_count, nbr_idx,
                                                          c->d_flags);
        rc = hip_check(c, hipGetLastError(), "copy list");
    }
    if (!rc) rc = sync_and_check(c);
    c->list_r = -1;  // the evaluation list uses its own radius
    return rc;
}

int ap_eam_eval(ap_ctx *c, int n, const double *pos, const int32_t *species, const ap_box *box,
                const double *lambda, double *E_tot, double *E_atom, double *F, double *virial9) {
    int rc = check_common(c, n, pos, box, true);
    if (rc) return rc;
    if (species) return set_error(c, AP_E_ARG, "single-species potentials: species must be NULL");
    EvalFlags f{false, false, 1.0, true, false};
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos, box->L);
    if (!rc) rc = evaluate(c, n, box->L, f, lambda, nullptr, 0, false, E_tot, E_atom, F, virial9, false);
    if (!rc) rc = sync_and_check(c);
    return rc;
}

__global__ void k_copy_d(const double *src, double *dst, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

int ap_switch_eval(ap_ctx *c, int n, const double *pos, const ap_box *box, double *g, double *d, double *wbar,
                   double *lambda, double *dlambda, int32_t *n_precise) {
    int rc = check_common(c, n, pos, box, true);
    if (rc) return rc;
    rc = check_csp(c, n);
    if (rc) return rc;
    EvalFlags f{true, false, 1.0, true, false};
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos, box->L);
    if (!rc) rc = ensure_list(c, n, box->L, list_radius(c, true), true);
    if (rc) return rc;
    if (c->sw.indicator == AP_IND_MLP)
        launch_mlp_indicator(c, n, box->L);
    else
        launch_csp_value(c, n, box->L);
    launch_dens_desc(c, n, box->L, f, nullptr, false);
    launch_compact(c, n, nullptr, 0, false);
    const int nb = nblocks(n);
    if (g) k_copy_d<<<nb, kBlock, 0, c->stream>>>(c->g, g, n);
    if (d) k_copy_d<<<nb, kBlock, 0, c->stream>>>(c->d, d, n);
    if (wbar) k_copy_d<<<nb, kBlock, 0, c->stream>>>(c->wbar, wbar, n);
    if (lambda) k_copy_d<<<nb, kBlock, 0, c->stream>>>(c->lam, lambda, n);
    if (dlambda) k_copy_d<<<nb, kBlock, 0, c->stream>>>(c->dlam, dlambda, n);
    if (n_precise) (void)hipMemcpyAsync(n_precise, c->d_flags + 2, sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream);
    rc = hip_check(c, hipGetLastError(), "switch");
    if (!rc) rc = sync_and_check(c);
    return rc;
}

int ap_ace_eval(ap_ctx *c, int n, const double *pos, const int32_t *species, const ap_box *box,
                const int32_t *subset, int n_subset, double *E_tot, double *E_atom, double *F, double *virial9) {
    int rc = check_common(c, n, pos, box, true);
    if (rc) return rc;
    if (species) return set_error(c, AP_E_ARG, "single-species potentials: species must be NULL");
    if (subset && (n_subset < 0 || n_subset > n)) return set_error(c, AP_E_ARG, "n_subset");
    EvalFlags f{false, false, 0.0, false, true};
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos, box->L);
    if (!rc) rc = evaluate(c, n, box->L, f, nullptr, subset, n_subset, true, E_tot, E_atom, F, virial9, false);
    if (!rc) rc = sync_and_check(c);
    return rc;
}

int ap_mixed_energy_forces(ap_ctx *c, int n, const double *pos, const int32_t *species, const ap_box *box,
                           double *E_tot, double *E_atom, double *F, double *virial9, double *lambda_out) {
    int rc = check_common(c, n, pos, box, true);
    if (rc) return rc;
    if (species) return set_error(c, AP_E_ARG, "single-species potentials: species must be NULL");
    const EvalFlags f = mixed_flags(c);
    if (f.switching) {
        rc = check_csp(c, n);
        if (rc) return rc;
    }
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    rc = prepare_positions(c, n, pos, box->L);
    const bool run_ace = !(c->sw.lambda_mode == AP_LAMBDA_FAST);
    if (!rc) rc = evaluate(c, n, box->L, f, nullptr, nullptr, 0, run_ace, E_tot, E_atom, F, virial9, false);
    if (!rc && lambda_out) k_copy_d<<<nblocks(n), kBlock, 0, c->stream>>>(c->lam, lambda_out, n);
    if (!rc) rc = sync_and_check(c);
    return rc;
}

__global__ void k_batch_fill(int n, const double *weight, const double *pos, double *lam, double *dlam, double *wbar,
                             double *Ef, double *xip, double *Et, Rec4 *xl, Rec4 *eb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = weight ? 1.0 - weight[i] : 0.0;  // the ACE weight of Eq. (4) is 1 - lambda
    lam[i] = l;
    xl[i] = Rec4{pos[i], pos[n + i], pos[2 * n + i], l};
    eb[i] = Rec4{0.0, 0.0, 0.0, 0.0};
    dlam[i] = 0.0;
    wbar[i] = 1.0;
    Ef[i] = 0.0;
    xip[i] = 0.0;
    Et[i] = 0.0;
}

// Checks and uploads of a batch of cells, the per-cell lists, the per-atom weights and S = every atom; the
// per-atom coefficient buffer is sized when want_b. *n_out: the atom count.
static int batch_prepare(ap_ctx *c, int n_struct, const int32_t *offsets, const double *boxes, const double *pos,
                         const double *weight, bool want_b, int *n_out) {
    if (!c) return AP_E_ARG;
    if (!c->have_pot) return set_error(c, AP_E_STATE, "ap_set_potential has not been called");
    if (n_struct <= 0 || !offsets || !boxes || !pos) return set_error(c, AP_E_ARG, "batch arguments");
    if (offsets[0] != 0) return set_error(c, AP_E_ARG, "offsets[0] must be 0");
    for (int s = 0; s < n_struct; s++) {
        if (offsets[s + 1] < offsets[s]) return set_error(c, AP_E_ARG, "offsets must not decrease");
        for (int a = 0; a < 3; a++)
            if (!(c->ace.rc < 0.5 * boxes[3 * s + a])) return set_error(c, AP_E_BOX, "ACE cutoff >= half a cell");
    }
    const int n = offsets[n_struct];
    if (n <= 0 || n > c->n_cap) return set_error(c, AP_E_ARG, "total atom count out of range (1..n_max_atoms)");
    int rc = AP_OK;
    if (n_struct > c->b_cap) {
        (void)hipFree(c->b_off);
        (void)hipFree(c->b_box);
        c->b_off = nullptr;
        c->b_box = nullptr;
        rc = hip_check(c, hipMalloc(&c->b_off, sizeof(int) * (n_struct + 1)), "batch");
        if (!rc) rc = hip_check(c, hipMalloc(&c->b_box, sizeof(double) * 3 * n_struct), "batch");
        if (rc) return rc;
        c->b_cap = n_struct;
    }
    const size_t es = c->ace.precision == AP_FP32 ? 4 : 8;
    const size_t bb = (size_t)c->n_cap * (c->ace.n_funcs + c->ace.n_max) * es;
    if (want_b && bb != c->bval_bytes) {
        (void)hipFree(c->bval);
        c->bval = nullptr;
        rc = hip_check(c, hipMalloc(&c->bval, bb), "coefficient-gradient buffer");
        if (rc) return rc;
        c->bval_bytes = bb;
    }
    rc = hip_check(c, hipMemcpyAsync(c->b_off, offsets, sizeof(int) * (n_struct + 1), hipMemcpyHostToDevice, c->stream),
                   "batch");
    if (!rc)
        rc = hip_check(c, hipMemcpyAsync(c->b_box, boxes, sizeof(double) * 3 * n_struct, hipMemcpyHostToDevice, c->stream),
                       "batch");
    if (rc) return rc;
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    {
        ProfScope p(c, "batch_list");
        rc = batch_lists(c, n, n_struct, c->b_off, c->b_box, pos, c->ace.rc);
    }
    if (rc) return rc;
    k_batch_fill<<<nblocks(n), kBlock, 0, c->stream>>>(n, weight, c->pos, c->lam, c->dlam, c->wbar, c->Ef, c->xip,
                                                       c->Et, c->xl, c->eb);
    {
        ProfScope p(c, "compact");
        launch_compact(c, n, nullptr, 0, false);
    }
    *n_out = n;
    return AP_OK;
}

int ap_ace_batch_eval(ap_ctx *c, int n_struct, const int32_t *offsets, const double *boxes, const double *pos,
                      const double *weight, double *E_struct, double *F, double *dEdc, double *dEdb) {
    const bool want_b = dEdc || dEdb;
    int n = 0;
    int rc = batch_prepare(c, n_struct, offsets, boxes, pos, weight, want_b, &n);
    if (rc) return rc;
    rc = launch_ace(c, n, boxes, std::min(n, 8192), c->b_box, want_b);
    if (rc) return rc;
    if (F) {
        const EvalFlags f{false, false, 0.0, false, true};
        ProfScope p(c, "force");
        launch_force(c, n, boxes, f, nullptr, F, c->b_box);
    }
    {
        ProfScope p(c, "struct_reduce");
        launch_struct_reduce(c, n, n_struct, c->b_off, weight, E_struct, dEdc, dEdb);
    }
    rc = hip_check(c, hipGetLastError(), "batch");
    if (!rc) rc = sync_and_check(c);
    return rc;
}

int ap_ace_batch_force_vjp(ap_ctx *c, int n_struct, const int32_t *offsets, const double *boxes, const double *pos,
                           const double *weight, const double *G, double *dLdc, double *dLdb) {
    if (!c) return AP_E_ARG;
    if (!G || (!dLdc && !dLdb)) return set_error(c, AP_E_ARG, "G and at least one output needed");
    int n = 0;
    int rc = batch_prepare(c, n_struct, offsets, boxes, pos, weight, true, &n);
    if (rc) return rc;
    rc = launch_ace_vjp(c, n, boxes, std::min(n, 8192), c->b_box, G);
    if (rc) return rc;
    {
        ProfScope p(c, "struct_reduce");
        launch_struct_reduce(c, n, n_struct, c->b_off, weight, nullptr, dLdc, dLdb, -1.0);
    }
    rc = hip_check(c, hipGetLastError(), "batch vjp");
    if (!rc) rc = sync_and_check(c);
    return rc;
}

int ap_set_profiling(ap_ctx *c, int on) {
    if (!c) return AP_E_ARG;
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    prof_resolve(c);
    c->prof_on = on != 0;
    c->prof_every = on > 1 ? on : 1;
    c->prof_skip = false;
    c->prof_names.clear();
    c->prof_ms.clear();
    c->prof_cnt.clear();
    return rc;
}

int ap_get_profile(ap_ctx *c, int max_entries, char *names, double *avg_ms, int64_t *count) {
    if (!c) return AP_E_ARG;
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (rc) return rc;
    prof_resolve(c);
    const int m = (int)c->prof_names.size();
    for (int q = 0; q < m && q < max_entries; q++) {
        if (names) {
            std::memset(names + 32 * q, 0, 32);
            std::strncpy(names + 32 * q, c->prof_names[q].c_str(), 31);
        }
        if (avg_ms) avg_ms[q] = c->prof_cnt[q] ? c->prof_ms[q] / c->prof_cnt[q] : 0.0;
        if (count) count[q] = c->prof_cnt[q];
    }
    return m;
}

int ap_ace_cost(ap_ctx *c, double *fixed_per_atom, double *per_neighbor_energy, double *per_neighbor_force) {
    if (!c) return AP_E_ARG;
    if (!c->have_pot) return set_error(c, AP_E_STATE, "ap_set_potential has not been called");
    double a, b, d;
    ace_cost(c, &a, &b, &d);
    if (fixed_per_atom) *fixed_per_atom = a;
    if (per_neighbor_energy) *per_neighbor_energy = b;
    if (per_neighbor_force) *per_neighbor_force = d;
    return AP_OK;
}

int ap_vv_step(ap_ctx *c, int n, double *pos, double *vel, double *F, double mass, double dt, int n_steps,
               const ap_box *box, double *thermo) {
    int rc = check_common(c, n, pos, box, true);
    if (rc) return rc;
    if (!vel || !F || !thermo || n_steps < 0 || !(mass > 0) || !(dt > 0))
        return set_error(c, AP_E_ARG, "vel, F, thermo, n_steps >= 0, mass > 0, dt > 0 required");
    const EvalFlags f = mixed_flags(c);
    if (f.switching) {
        rc = check_csp(c, n);
        if (rc) return rc;
    }
    const bool run_ace = !(c->sw.lambda_mode == AP_LAMBDA_FAST);
    const double hdtm = 0.5 * dt / mass * kConv;
    const int nb = nblocks(n), nbf = force_blocks(n);
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    // the list of the previous call stays valid while every atom is within skin / 2 of its build position
    // (the first step's skin check, in k_vv_first, decides); a new n, box or radius rebuilds it anyway
    bool force = false;
    for (int s = 0; s < n_steps; s++) {
        c->prof_skip = c->prof_every > 1 && s % c->prof_every != 0;
        if (s == 0) {
            ProfScope p(c, "vv_first");
            // the skin check of the drifted positions against the last build, and the cells of that build's
            // geometry cleared for a possible rebuild (a new geometry is cleared by the list code itself)
            k_vv_first<<<nb, kBlock, 0, c->stream>>>(pos, vel, F, c->pos, n, hdtm, dt, box->L[0], box->L[1],
                                                     box->L[2], c->pos_build, 0.25 * c->skin * c->skin, c->d_flags,
                                                     c->cell_cnt, c->cell_fill, c->ncell_cur);
        }
        // the force pass applies the second half-kick and sums E_kin and P with the energy, then (but on
        // the last step) the next step's first half-kick, drift and skin check; the density pass of this
        // step takes the thermo row of the previous one from the partials it left
        c->thermo_prev = s > 0 ? thermo + (size_t)8 * (s - 1) : nullptr;
        c->kick_vel = vel;
        c->kick_hdtm = hdtm;
        c->kick_mass = mass;
        c->drift_pos = s + 1 < n_steps ? pos : nullptr;
        c->drift_dt = dt;
        rc = evaluate(c, n, box->L, f, nullptr, nullptr, 0, run_ace, nullptr, nullptr, F, nullptr, force, !force,
                      false);
        c->kick_vel = nullptr;
        c->drift_pos = nullptr;
        if (rc) {
            c->prof_skip = false;
            c->thermo_prev = nullptr;
            return rc;
        }
        force = false;
    }
    c->prof_skip = false;
    c->thermo_prev = nullptr;
    if (n_steps > 0) {
        ProfScope p(c, "thermo");
        k_thermo<<<1, kBlock, 0, c->stream>>>(c->partials, nbf, c->pstride, c->d_flags,
                                              thermo + (size_t)8 * (n_steps - 1));
    }
    rc = hip_check(c, hipGetLastError(), "vv");
    if (!rc) rc = sync_and_check(c);
    return rc;
}

}  // extern "C"
