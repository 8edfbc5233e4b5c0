// Switching parameter, EAM and the conservative force assembly.
//
//   k_dens_desc : one pass over the neighbour list per atom gives the EAM density and pair energy
//                 (B1) and, when switching, the descriptor Eq. (6) and lambda Eq. (2).
//   k_compact   : ordered compaction of S = {i : lambda_i < 1} (device-side count).
//   k_W         : W_j = sum_k E~_k w(r_kj) of (S25), E~ of (S17) written by the ACE kernel.
//   k_force     : gather-only assembly of F_i = sum_k (f_ki - f_ik), (A1)-(A2), with the EAM (S12),
//                 ACE (S14), weight (S21) and CSP (S27) families; E_i of Eq. (4); per-block partial
//                 sums of the energy and of the virial.
// Every sum runs in a fixed order, so results are bit-reproducible run to run.
#include "ap_internal.h"

namespace ap {

struct EamP {
    double A, beta, c0, c1, c2, r_rho, r_phi, rc2, inv_rr;  // rc2 = max(r_rho, r_phi)^2, inv_rr = 1 / r_rho
};
static EamP eamp(const ap_eam_params &e) {
    const double m = e.r_rho > e.r_phi ? e.r_rho : e.r_phi;
    return {e.A, e.beta, e.c0, e.c1, e.c2, e.r_rho, e.r_phi, m * m, 1.0 / e.r_rho};
}

// zeta, zeta', Phi, Phi' of the Finnis-Sinclair form at r (each zero beyond its own cutoff)
__device__ __forceinline__ void eam_pair(const EamP &p, double r, double &z, double &dz, double &ph, double &dph) {
    z = dz = ph = dph = 0.0;
    if (r < p.r_rho) {
        const double x = r - p.r_rho;
        z = x * x * (1.0 + p.beta * x * p.inv_rr);
        dz = x * (2.0 + 3.0 * p.beta * x * p.inv_rr);
    }
    if (r < p.r_phi) {
        const double y = r - p.r_phi;
        const double q = p.c0 + r * (p.c1 + p.c2 * r);
        ph = y * y * q;
        dph = y * (2.0 * q + y * (p.c1 + 2.0 * p.c2 * r));
    }
}

struct SwP {
    // inv_ww = 1 / (r_w - (r_w - 1)), the weight window; below lo2 (the largest double under (r_w - 1)^2)
    // the weight is 1
    double d_lo, d_hi, r_w, r_w2, d0, inv_ww, lo2;
};
static SwP swp(const ap_ctx *c) {
    const double lo = c->sw.r_w - 1.0;
    return {c->sw.d_lo, c->sw.d_hi, c->sw.r_w, c->sw.r_w * c->sw.r_w, c->sw.d0, 1.0 / (c->sw.r_w - lo),
            std::nextafter(lo * lo, 0.0)};
}

// SUB lanes per atom: lane `sub` takes slots sub, sub + SUB, ...; the lane partials are combined by
// a fixed xor butterfly inside the group (the same pairs on every lane, so the sums are identical
// and the result does not depend on scheduling).
template <int SUB>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = 1; m < SUB; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int SUB>
__global__ __launch_bounds__(kBlock) void k_dens_desc(const double *__restrict__ pos, int n, double Lx, double Ly,
                                                      double Lz, EamP ep, SwP sp, int switching, double lam_const,
                                                      const double *__restrict__ lam_in,
                                                      const int32_t *__restrict__ ncount,
                                                      const int32_t *__restrict__ nidx, const double *__restrict__ g,
                                                      const Rec4 *__restrict__ xg, Rec4 *__restrict__ xl,
                                                      Rec4 *__restrict__ eb, Rec4 *__restrict__ xe,
                                                      double *__restrict__ Ef,
                                                      double *__restrict__ xip,
                                                      double *__restrict__ wbar, double *__restrict__ dd,
                                                      double *__restrict__ lam, double *__restrict__ dlam,
                                                      double *__restrict__ Ep, double *__restrict__ Et, int *flags,
                                                      int *__restrict__ chunk_cnt, int *list_gen,
                                                      const double *__restrict__ partials, int nbf, int pstride,
                                                      double *row_prev, const int *__restrict__ lam_fix) {
    // commit of the neighbour-list rebuild flag, after every list kernel of this evaluation (workgroup 0
    // keeps the previous value for the thermo row below)
    __shared__ int s_prev_rebuild, s_prev_S;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s_prev_rebuild = flags[3];
        s_prev_S = flags[2];
        if (flags[0]) list_gen[0]++;
        flags[3] = flags[0];
        flags[0] = 0;
    }
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int i = t / SUB, sub = t - i * SUB;
    double z = 0.0, pair = 0.0, ws = 0.0, gs = 0.0;
    if (i < n) {
        const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
        const int cnt = ncount[i];
        // two-deep software pipeline: the record of slot k + SUB and the index of slot k + 2 SUB are in
        // flight while slot k is evaluated (the gathers are latency bound, not bandwidth bound)
        // ({x, y, z, g} in one record when switching)
        int jn = sub < cnt ? nidx[(size_t)sub * n + i] : 0;
        Rec4 rc{0.0, 0.0, 0.0, 0.0};
        if (sub < cnt) {
            if (switching)
                rc = xg[jn];
            else
                rc = Rec4{pos[jn], pos[n + jn], pos[2 * n + jn], 0.0};
        }
        jn = sub + SUB < cnt ? nidx[(size_t)(sub + SUB) * n + i] : 0;
        for (int k = sub; k < cnt; k += SUB) {
            Rec4 rn = rc;
            if (k + SUB < cnt) {
                if (switching)
                    rn = xg[jn];
                else
                    rn = Rec4{pos[jn], pos[n + jn], pos[2 * n + jn], 0.0};
            }
            if (k + 2 * SUB < cnt) jn = nidx[(size_t)(k + 2 * SUB) * n + i];
            const double ux = min_image_w(rc.x - xi, Lx), uy = min_image_w(rc.y - yi, Ly), uz = min_image_w(rc.z - zi, Lz);
            const double r2 = ux * ux + uy * uy + uz * uz;
            // one square root, taken only inside the EAM range or the weight's transition band
            const bool in_eam = r2 < ep.rc2;
            const bool in_band = switching && r2 > sp.lo2 && r2 < sp.r_w2;
            double r = 0.0;
            if (in_eam || in_band) r = sqrt(r2);
            if (in_eam) {
                double zz, dz, ph, dph;
                eam_pair(ep, r, zz, dz, ph, dph);
                z += zz;
                pair += ph;
            }
            if (switching && r2 < sp.r_w2) {
                const double w = in_band ? ftrans_i(r, sp.r_w - 1.0, sp.r_w, sp.inv_ww) : 1.0;
                ws += w;
                gs += rc.w * w;
            }
            rc = rn;
        }
    }
    z = group_sum<SUB>(z);
    pair = group_sum<SUB>(pair);
    ws = group_sum<SUB>(ws);
    gs = group_sum<SUB>(gs);
    bool prec = false;  // lambda_i < 1
    if (i < n && sub == 0) {
        ws += 1.0;  // self term of Eq. (6): w(0) = 1
        if (switching) gs += g[i];
        double emb = 0.0, demb = 0.0;
        if (z > 0.0) {
            const double s = sqrt(z);
            emb = -ep.A * s;
            demb = -0.5 * ep.A / s;
        }
        Ef[i] = emb + 0.5 * pair;
        xip[i] = demb;
        double l, dl = 0.0, d = 0.0;
        if (switching) {
            d = gs / ws - sp.d0;
            const int fx = lam_fix ? lam_fix[i] : -1;
            if (fx >= 0) {
                // a constant switching parameter (App. B, after (B4)): not a function of d, dlambda/dd = 0
                l = (double)fx;
            } else {
                l = ftrans(d, sp.d_lo, sp.d_hi);
                dl = ftrans_d(d, sp.d_lo, sp.d_hi);
            }
        } else {
            l = lam_in ? lam_in[i] : lam_const;
            ws = 1.0;
        }
        wbar[i] = ws;
        dd[i] = d;
        lam[i] = l;
        dlam[i] = dl;
        Ep[i] = 0.0;
        Et[i] = 0.0;
        xl[i] = Rec4{pos[i], pos[n + i], pos[2 * n + i], l};
        eb[i] = Rec4{demb, switching ? g[i] : 0.0, d + sp.d0, 0.0};
        xe[i] = Rec4{pos[i], pos[n + i], pos[2 * n + i], demb};
        prec = l < 1.0;
    }
    if (chunk_cnt) {
        // the count of precise atoms among this workgroup's kBlock / SUB atoms, for the compaction
        __shared__ int sc[kBlock / 64];
        const unsigned long long m = __ballot(prec);
        if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = __popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < kBlock / 64; w++) s += sc[w];
            chunk_cnt[t / (int)blockDim.x] = s;
        }
    }
    // inside velocity Verlet: the previous step's thermo row, from the partials its force pass left
    // (|S| and the rebuild flag as they were before this evaluation)
    if (row_prev && blockIdx.x == 0) {
        __syncthreads();
        thermo_row_block(partials, nbf, pstride, s_prev_S, s_prev_rebuild, flags, row_prev);
    }
}

void launch_dens_desc(ap_ctx *c, int n, const double *box, const EvalFlags &f, const double *lam_in, bool count) {
    const SwP sp = swp(c);
    // kDensLanes lanes per atom up to the sizes whose compaction uses the per-workgroup counts; above, where
    // the count-scan-scatter compaction runs, eight lanes hide the gathers' latency better (2M atoms: 1.25
    // against 1.38 ms)
    auto go = [&](auto lanes) {
        constexpr int SUB = decltype(lanes)::value;
        k_dens_desc<SUB><<<((size_t)n * SUB + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
            c->pos, n, box[0], box[1], box[2], eamp(c->eam), sp, f.switching ? 1 : 0, f.lam_const, lam_in,
            c->nbr_cnt, c->nbr_idx, c->g, c->xg, c->xl, c->eb, c->xe, c->Ef, c->xip, c->wbar, c->d, c->lam, c->dlam,
            c->Ep, c->Et, c->d_flags, count ? c->chunk_cnt : nullptr, c->list_gen, c->partials, force_blocks(n),
            c->pstride, c->thermo_prev, c->have_fix && f.switching ? c->lam_fix : nullptr);
    };
    if (n <= kCountedCompactMax)
        go(std::integral_constant<int, kDensLanes>());
    else
        go(std::integral_constant<int, kLanesPerAtom>());
}

// ------------------------------------------------------------------------------------------
// Ordered compaction of S = {i : lambda_i < 1}, or of an explicit subset.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ bool in_s(const double *lam, const int *mark, int i) {
    return mark ? mark[i] != 0 : lam[i] < 1.0;
}

__global__ __launch_bounds__(kBlock) void k_compact_count(int n, const double *__restrict__ lam,
                                                          const int *__restrict__ mark, int *__restrict__ bcnt) {
    __shared__ int sh[kBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = i < n && in_s(lam, mark, i);
    const unsigned long long m = __ballot(f);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kBlock / 64; w++) s += sh[w];
        bcnt[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(int n, const double *__restrict__ lam,
                                                            const int *__restrict__ mark, const int *__restrict__ boff,
                                                            int *__restrict__ sidx, int *__restrict__ slist) {
    __shared__ int sh[kBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = i < n && in_s(lam, mark, i);
    const unsigned long long m = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = __popcll(m);
    __syncthreads();
    int off = boff[blockIdx.x];
    for (int q = 0; q < w; q++) off += sh[q];
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (i < n) {
        if (f) {
            slist[off + rank] = i;
            sidx[i] = off + rank;
        } else {
            sidx[i] = -1;
        }
    }
}

__global__ void k_mark_subset(const int32_t *__restrict__ subset, int m, int n, int *mark, int *flags) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    int i = subset[q];
    if (i < 0 || i >= n) {
        atomicOr(&flags[1], kErrOverflow);
        return;
    }
    mark[i] = 1;
}

// Ordered compaction from the density pass's counts of lambda < 1 per kBlock / kDensLanes atoms: each
// workgroup of kBlock atoms sums the counts before it (integers: exact in any order) and ranks its own
// atoms by ballot; the last one writes |S|.
__global__ __launch_bounds__(kBlock) void k_compact_chunks(int n, const double *__restrict__ lam,
                                                           const int *__restrict__ chunk_cnt, int per_block,
                                                           int *__restrict__ sidx, int *__restrict__ slist,
                                                           int *__restrict__ S_out) {
    __shared__ int sh[kBlock / 64], sb[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int part = 0;
    for (int q = threadIdx.x; q < (int)blockIdx.x * per_block; q += blockDim.x) part += chunk_cnt[q];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = i < n && lam[i] < 1.0;
    const unsigned long long m = __ballot(f);
    if (lane == 0) {
        sb[w] = part;
        sh[w] = __popcll(m);
    }
    __syncthreads();
    int off = 0;
    for (int q = 0; q < kBlock / 64; q++) off += sb[q];
    for (int q = 0; q < w; q++) off += sh[q];
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (i < n) {
        if (f) {
            slist[off + rank] = i;
            sidx[i] = off + rank;
        } else {
            sidx[i] = -1;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        int tot = 0;
        for (int q = 0; q < kBlock / 64; q++) tot += sb[q] + sh[q];
        *S_out = tot;
    }
}

void launch_compact_marked(ap_ctx *c, int n) {
    const int nb = (n + kBlock - 1) / kBlock;
    k_compact_count<<<nb, kBlock, 0, c->stream>>>(n, c->lam, c->mark, c->blk_cnt);
    launch_scan(c, c->blk_cnt, c->blk_cnt + nb, nb, c->d_flags + 2, nullptr);
    k_compact_scatter<<<nb, kBlock, 0, c->stream>>>(n, c->lam, c->mark, c->blk_cnt + nb, c->sidx, c->slist);
}

void launch_compact(ap_ctx *c, int n, const int32_t *subset, int n_subset, bool counted) {
    const int nb = (n + kBlock - 1) / kBlock;
    if (counted && !subset) {
        k_compact_chunks<<<nb, kBlock, 0, c->stream>>>(n, c->lam, c->chunk_cnt, kDensLanes, c->sidx, c->slist,
                                                       c->d_flags + 2);
        return;
    }
    int *mark = nullptr;
    if (subset) {
        mark = c->mark;
        launch_fill_int(c, mark, 0, n);
        if (n_subset > 0)
            k_mark_subset<<<(n_subset + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(subset, n_subset, n, mark,
                                                                                       c->d_flags);
    }
    k_compact_count<<<nb, kBlock, 0, c->stream>>>(n, c->lam, mark, c->blk_cnt);
    launch_scan(c, c->blk_cnt, c->blk_cnt + nb, nb, c->d_flags + 2, nullptr);
    k_compact_scatter<<<nb, kBlock, 0, c->stream>>>(n, c->lam, mark, c->blk_cnt + nb, c->sidx, c->slist);
}

// ------------------------------------------------------------------------------------------
// Force mixing, Eq. (3): F^p_i of an atom with lambda_i < 1 needs E^p_k of every atom k within the ACE
// cutoff of i. mark = 1 selects those atoms and the atoms with lambda < 1 for the ACE kernels; act = 1
// the atoms whose force has an ACE part (lambda_i < 1), the others take F^f_i alone. The cutoff test
// has a margin, so the marked set contains every atom the ACE kernels find inside rc (an extra atom
// only adds zero pair terms).
// ------------------------------------------------------------------------------------------
template <int SUB>
__global__ __launch_bounds__(kBlock) void k_mix_mark(int n, double Lx, double Ly, double Lz, double rc2m,
                                                     const int32_t *__restrict__ ncount,
                                                     const int32_t *__restrict__ nidx, const Rec4 *__restrict__ xl,
                                                     int *__restrict__ mark, int *__restrict__ act) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / SUB, sub = t - i * SUB;
    int near = 0, own = 0;
    if (i < n) {
        const Rec4 pi = xl[i];
        own = pi.w < 1.0;
        const int cnt = ncount[i];
        for (int k = sub; k < cnt && !near; k += SUB) {
            const Rec4 pj = xl[nidx[(size_t)k * n + i]];
            if (!(pj.w < 1.0)) continue;
            const double ux = min_image_w(pj.x - pi.x, Lx), uy = min_image_w(pj.y - pi.y, Ly),
                         uz = min_image_w(pj.z - pi.z, Lz);
            near = ux * ux + uy * uy + uz * uz < rc2m;
        }
    }
#pragma unroll
    for (int m = 1; m < SUB; m <<= 1) near |= __shfl_xor(near, m, 64);
    if (i < n && sub == 0) {
        mark[i] = own | near;
        act[i] = own;
    }
}

void launch_mix_mark(ap_ctx *c, int n, const double *box) {
    constexpr int SUB = kLanesPerAtom;
    const double rcm = c->ace.rc * (1.0 + 1e-9);
    k_mix_mark<SUB><<<((size_t)n * SUB + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        n, box[0], box[1], box[2], rcm * rcm, c->nbr_cnt, c->nbr_idx, c->xl, c->mark, c->act);
}

// ------------------------------------------------------------------------------------------
// W_j = sum_k E~_k w(r_kj), including k = j (w(0) = 1).
// ------------------------------------------------------------------------------------------
template <int SUB>
__global__ __launch_bounds__(kBlock) void k_W(const double *__restrict__ pos, int n, double Lx, double Ly, double Lz,
                                              double r_w, const int32_t *__restrict__ ncount,
                                              const int32_t *__restrict__ nidx, const double *__restrict__ Et,
                                              const Rec4 *__restrict__ xl, const double *__restrict__ lam,
                                              double *__restrict__ W, int *__restrict__ act,
                                              const int *__restrict__ stamp, int gen, int use_stamp,
                                              const int32_t *__restrict__ csp_t, int n_csp, int *__restrict__ cmark,
                                              int mark_list) {
    // plain block order: the stamped atoms are a few contiguous index ranges, and an XCD-contiguous
    // mapping would put them all on one or two XCDs
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = t / SUB, sub = t - j * SUB;
    double s = 0.0;
    int near_s = 0;  // a neighbour with lambda < 1
    // an atom that no precise atom stamped (not precise, none in its symmetric list) has W = 0 and no
    // lambda < 1 in reach: only the stamped ones gather
    if (j < n && (!use_stamp || stamp[j] == gen)) {
        const double xj = pos[j], yj = pos[n + j], zj = pos[2 * n + j];
        const double r_w2 = r_w * r_w;
        const int cnt = ncount[j];
        // {x, y, z, lambda} and E~ of slot q + SUB and the index of slot q + 2 SUB in flight during slot q
        int kn = sub + SUB < cnt ? nidx[(size_t)(sub + SUB) * n + j] : 0;
        Rec4 pc{0.0, 0.0, 0.0, 1.0};
        double ec = 0.0;
        if (sub < cnt) {
            const int k0 = nidx[(size_t)sub * n + j];
            pc = xl[k0];
            ec = Et[k0];
        }
        for (int q = sub; q < cnt; q += SUB) {
            const Rec4 pk = pc;
            const double e = ec;
            if (q + SUB < cnt) {
                pc = xl[kn];
                ec = Et[kn];
            }
            if (q + 2 * SUB < cnt) kn = nidx[(size_t)(q + 2 * SUB) * n + j];
            near_s |= pk.w < 1.0;
            if (e == 0.0) continue;
            const double ux = min_image_w(pk.x - xj, Lx), uy = min_image_w(pk.y - yj, Ly), uz = min_image_w(pk.z - zj, Lz);
            const double r2 = ux * ux + uy * uy + uz * uz;
            if (r2 < r_w2) s += e * ftrans_i(sqrt(r2), r_w - 1.0, r_w, 1.0 / (r_w - (r_w - 1.0)));
        }
    }
    s = group_sum<SUB>(s);
#pragma unroll
    for (int m = 1; m < SUB; m <<= 1) near_s |= __shfl_xor(near_s, m, 64);
    if (j < n) {
        const bool stamped = !use_stamp || stamp[j] == gen;
        const double Wj = stamped ? Et[j] + s : 0.0;
        if (sub == 0) {
            W[j] = Wj;
            act[j] = stamped ? (near_s | (lam[j] < 1.0)) : 0;
        }
        // the atoms in j's CSP list receive a reverse term of (S27) from W_j; with the learned indicator,
        // the atoms of j's neighbour list receive its grad-g term (S16) (all writers store gen)
        if (cmark && Wj != 0.0) {
            if (mark_list) {
                const int cnt = ncount[j];
                for (int q = sub; q < cnt; q += SUB) cmark[nidx[(size_t)q * n + j]] = gen;
            } else {
                for (int t = sub; t < n_csp; t += SUB) cmark[csp_t[(size_t)t * n + j]] = gen;
            }
        }
    }
}

// stamped: the ACE pair kernel of this evaluation stamped the precise atoms' neighbourhoods
void launch_W(ap_ctx *c, int n, const double *box, bool stamped, bool csp_marks) {
    constexpr int SUB = kLanesPerAtom;
    k_W<SUB><<<((size_t)n * SUB + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
        c->pos, n, box[0], box[1], box[2], c->sw.r_w, c->nbr_cnt, c->nbr_idx, c->Et, c->xl, c->lam, c->W, c->act,
        c->stamp, c->stamp_gen, stamped ? 1 : 0, c->csp_t, c->n_csp, csp_marks ? c->cmark : nullptr,
        c->sw.indicator == AP_IND_MLP ? 1 : 0);
}

// ------------------------------------------------------------------------------------------
// Force assembly
// ------------------------------------------------------------------------------------------
struct ForceArgs {
    const double *pos;
    int n;
    double L[3];
    EamP ep;
    SwP sp;
    int switching, grad_lambda, eam_on, ace_on;
    const int32_t *ncount, *nidx;
    const double *lam, *xip, *Ef, *Ep, *Et, *W, *g, *d;
    const int *sidx;
    const void *fpair, *frev;
    int fp32, max_nbr, n_csp;
    double ace_rc2;  // reverse ACE terms exist only inside the ACE cutoff
    double mlp_rc2;  // and reverse grad-g terms only inside the feature cutoff
    const int32_t *csp_t, *rev_start, *rev_code;
    double *E_atom, *F, *partials;  // partials: [16][pstride] per-tile sums, column-major
    int ntiles;                     // tiles of kBlock / SUB atoms (force_blocks(n))
    int split_grid, half_grid;      // two grid halves (tiles with full-list atoms first), each half_grid blocks
    int pstride;
    int *flags;
    const double *sbox;  // per-structure boxes of a batch (null: L)
    const int *sid;
    int ind_mlp;                      // learned indicator: grad-g terms from hpair / hrev
    const float *hpair, *hrev;
    const int *widx;
    const Rec4 *xl, *eb;  // neighbour records {x, y, z, lambda}, {xi', g, d + d0, E~}
    const Rec4 *xe;       // {x, y, z, xi'} for the EAM-only gather
    // 0: every slot; 1: atoms with act == 0 take the EAM-only gather over their nshort EAM-range
    // slots; 2: all atoms do; 3: all atoms stop after nshort slots (per-atom lambda)
    int short_mode;
    const int *act;
    const int32_t *nshort;
    const int *cmark;  // null: every atom scans its reverse CSP entries; else only those with cmark == cgen
    int cgen;
    // velocity Verlet's second half-kick v += hdtm F on the new forces, with the block sums of the
    // kinetic energy and momentum in partial columns 10-13 (null: no kick)
    double *vel;
    double hdtm, mass;
    // and, when drift_pos is set (not the last step), the next step's first half-kick and drift: the
    // wrapped positions go to drift_pos (the caller's) and ipos (the context's copy), the skin check
    // against pos_build to flags[0], and the cell counts are cleared for a possible rebuild
    double *drift_pos, *ipos;
    const double *pos_build;
    double dt, half_skin2;
    int *cell_cnt, *cell_fill;
    int ncell;
};

template <typename TF>
__device__ __forceinline__ void load_f(const TF *fp, size_t o, double &a, double &b, double &c) {
    a = (double)fp[o];
    b = (double)fp[o + 1];
    c = (double)fp[o + 2];
}

// Deterministic workgroup sums of NV values at once (a fixed shuffle tree per wavefront, then the
// wavefronts in order); thread q < NV of the workgroup writes sum q to out[q * stride].
template <int NV>
__device__ __forceinline__ void block_sums(const double *v, double *sh, double *out, int stride) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[w * NV + q] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int k = 0; k < kBlock / 64; k++) s += sh[k * NV + threadIdx.x];
        out[(size_t)threadIdx.x * stride] = s;
    }
}

// FULL = false: only the EAM-only gather (every atom in that mode), compiled without the full-list loop
// and the CSP part so that it keeps its own, lower register count. With FP32 pair terms the full kernel
// is bounded to four workgroups per CU (128 VGPRs, no spills).
// MIX: force mixing, Eq. (3) (an instantiation of its own, so that the conservative kernel keeps its registers).
constexpr int kForceChunk = 16;
template <typename TF, int SUB, bool FULL, bool MIX = false>
__global__ __launch_bounds__(kBlock, (FULL && sizeof(TF) == 4) ? 4 : 1) void k_force(ForceArgs a) {
    __shared__ double sh[kBlock / 64 * 14];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < a.ncell; q += gridDim.x * blockDim.x) {
        a.cell_cnt[q] = 0;  // (with the fused drift)
        a.cell_fill[q] = 0;
    }
    // Block b runs on XCD b % 8. Each XCD takes chunks of kForceChunk consecutive tiles (kBlock / SUB
    // atoms each), the chunks dealt round-robin over the XCDs: a chunk's atoms share their neighbours in
    // that XCD's L2, while the few contiguous index ranges of atoms near S still spread over every XCD.
    // A grid half is a multiple of 8 kForceChunk; blocks past the last tile only clear cells.
    // With the EAM-only gather (short_mode 1, up to 2^18 atoms) the grid has two halves over the same tiles:
    // a tile with an atom on the full-list path is taken by the first half, which is dispatched first, so
    // that those few long tiles run alongside the many short ones instead of after them; the others by the
    // second half.
    const int half = a.split_grid && (int)blockIdx.x >= a.half_grid ? 1 : 0;
    const int bb = (int)blockIdx.x - half * a.half_grid;
    const int xcd = bb & 7, kth = bb >> 3;
    const int blk = ((kth / kForceChunk) * 8 + xcd) * kForceChunk + kth % kForceChunk;
    if (blk >= a.ntiles) return;
    const int t = blk * blockDim.x + threadIdx.x;
    const int i = t / SUB, sub = t - i * SUB;  // SUB lanes per atom, slots sub, sub + SUB, ...
    const int n = a.n;
    if (a.split_grid) {
        // (the negation of the EAM-only test below)
        const bool full = i < n && (a.act[i] || (a.ind_mlp && a.cmark[i] == a.cgen));
        if ((__syncthreads_or(full) != 0) != (half == 0)) return;  // (the same answer on every thread)
    }
    double F0 = 0, F1 = 0, F2 = 0, Ei = 0;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const bool gl = a.switching && a.grad_lambda;
    if (i < n) {
        const double xi = a.pos[i], yi = a.pos[n + i], zi = a.pos[2 * n + i];
        const double li = a.lam[i], xpi = a.xip[i];
        const double Eti = a.Et[i], gi = a.g[i], di = a.d[i];
        const int si = a.sidx[i];
        const TF *fp = reinterpret_cast<const TF *>(a.fpair);
        // without a precise atom in reach only the EAM pairs contribute: those are the first nshort
        // slots, and every lambda in reach equals lambda_i (no switching, or lambda = 1 all around)
        // (with the learned indicator an atom that a W != 0 neighbour marked gathers its grad-g terms)
        const bool eam_only = a.short_mode == 2 ||
                              (a.short_mode == 1 && !a.act[i] && !(a.ind_mlp && a.cmark[i] == a.cgen));
        const int cnt = (!FULL || eam_only) ? 0 : (a.short_mode == 3 ? a.nshort[i] : a.ncount[i]);
        const int wi = (gl && a.ind_mlp) ? a.widx[i] : -1;
        const double *Lb = a.sbox ? a.sbox + 3 * a.sid[i] : a.L;  // own cell in a batch of cells
        const double Lx = Lb[0], Ly = Lb[1], Lz = Lb[2];
        if (eam_only && a.eam_on) {
            // (S12) with lambda_k = lambda_i, from one {x, y, z, xi'} record per neighbour
            // (two-deep pipeline of the gathers, as in the density pass)
            const int cs = a.nshort[i];
            int jn = sub + SUB < cs ? a.nidx[(size_t)(sub + SUB) * n + i] : 0;
            Rec4 pc = sub < cs ? a.xe[a.nidx[(size_t)sub * n + i]] : Rec4{0.0, 0.0, 0.0, 0.0};
            for (int k = sub; k < cs; k += SUB) {
                Rec4 pn = pc;
                if (k + SUB < cs) pn = a.xe[jn];
                if (k + 2 * SUB < cs) jn = a.nidx[(size_t)(k + 2 * SUB) * n + i];
                const Rec4 pj = pc;
                pc = pn;
                const double ux = min_image_w(pj.x - xi, Lx), uy = min_image_w(pj.y - yi, Ly),
                             uz = min_image_w(pj.z - zi, Lz);
                const double r2 = ux * ux + uy * uy + uz * uz;
                if (r2 < a.ep.rc2) {
                    const double r = sqrt(r2), ir = 1.0 / r;
                    double zz, dz, ph, dph;
                    eam_pair(a.ep, r, zz, dz, ph, dph);
                    const double own = li * (xpi * dz + 0.5 * dph);
                    const double s = (own + li * (pj.w * dz + 0.5 * dph)) * ir;
                    F0 += s * ux;
                    F1 += s * uy;
                    F2 += s * uz;
                    const double t = MIX ? 0.0 : -own * ir;
                    v[0] += t * ux * ux; v[1] += t * ux * uy; v[2] += t * ux * uz;
                    v[3] += t * uy * ux; v[4] += t * uy * uy; v[5] += t * uy * uz;
                    v[6] += t * uz * ux; v[7] += t * uz * uy; v[8] += t * uz * uz;
                }
            }
        }
        if (cnt > 0) {  // the full-list loop; its gathers run one slot ahead (indices two)
            const bool need_q = a.eam_on || gl;
            int jc = sub < cnt ? a.nidx[(size_t)sub * n + i] : 0;
            Rec4 pc{0.0, 0.0, 0.0, 0.0}, qc{0.0, 0.0, 0.0, 0.0};
            int sc = -1;
            if (sub < cnt) {
                pc = a.xl[jc];
                if (need_q) qc = a.eb[jc];
                sc = a.sidx[jc];
            }
            int jn = sub + SUB < cnt ? a.nidx[(size_t)(sub + SUB) * n + i] : 0;
            for (int k = sub; k < cnt; k += SUB) {
                const int j = jc;
                const Rec4 pj = pc, qj = qc;
                const int sj = sc;
                if (k + SUB < cnt) {
                    jc = jn;
                    pc = a.xl[jn];
                    if (need_q) qc = a.eb[jn];
                    sc = a.sidx[jn];
                }
                if (k + 2 * SUB < cnt) jn = a.nidx[(size_t)(k + 2 * SUB) * n + i];
                const double ux = min_image_w(pj.x - xi, Lx), uy = min_image_w(pj.y - yi, Ly), uz = min_image_w(pj.z - zi, Lz);
                const double r2 = ux * ux + uy * uy + uz * uz;
                const double r = sqrt(r2), ir = 1.0 / r;
                const double ex = ux * ir, ey = uy * ir, ez = uz * ir;
                const double lj = pj.w;
                if (a.eam_on && r2 < a.ep.rc2) {
                    double zz, dz, ph, dph;
                    eam_pair(a.ep, r, zz, dz, ph, dph);
                    // lambda_i f_ki - lambda_k f_ik, (S12), along rhat_ki = u / r (force mixing, Eq. (3):
                    // lambda_i (f_ki - f_ik), the complete EAM force of i weighted by its own lambda)
                    const double own = li * (xpi * dz + 0.5 * dph);
                    const double s = own + (MIX ? li : lj) * (qj.x * dz + 0.5 * dph);
                    F0 += s * ex;
                    F1 += s * ey;
                    F2 += s * ez;
                    // virial of the edge owned by i: -(d(lambda_i E_i)/du)_a u_b
                    const double t = MIX ? 0.0 : -own * ir;
                    v[0] += t * ux * ux; v[1] += t * ux * uy; v[2] += t * ux * uz;
                    v[3] += t * uy * ux; v[4] += t * uy * uy; v[5] += t * uy * uz;
                    v[6] += t * uz * ux; v[7] += t * uz * uy; v[8] += t * uz * uz;
                }
                if (gl && r2 < a.sp.r_w2) {
                    // weight part (S19)-(S21): F_i -= (s_i + s_k) u / r
                    const double dw = ftrans_d_i(r, a.sp.r_w - 1.0, a.sp.r_w, a.sp.inv_ww);
                    const double s_i = Eti * (qj.y - di - a.sp.d0) * dw;
                    const double s_k = qj.w * (gi - qj.z) * dw;
                    const double s = -(s_i + s_k);
                    F0 += s * ex;
                    F1 += s * ey;
                    F2 += s * ez;
                    const double t = s_i * ir;
                    v[0] += t * ux * ux; v[1] += t * ux * uy; v[2] += t * ux * uz;
                    v[3] += t * uy * ux; v[4] += t * uy * uy; v[5] += t * uy * uz;
                    v[6] += t * uz * ux; v[7] += t * uz * uy; v[8] += t * uz * uz;
                }
                if (gl && a.ind_mlp) {
                    // learned indicator, (S16): F_i -= W_i dg_i/du_ik (own), F_i += W_j dg_j/du_ji (j's)
                    if (wi >= 0) {
                        const float *h = a.hpair + ((size_t)wi * a.max_nbr + k) * 3;
                        const double hx = (double)h[0], hy = (double)h[1], hz = (double)h[2];
                        F0 -= hx;
                        F1 -= hy;
                        F2 -= hz;
                        v[0] += hx * ux; v[1] += hx * uy; v[2] += hx * uz;
                        v[3] += hy * ux; v[4] += hy * uy; v[5] += hy * uz;
                        v[6] += hz * ux; v[7] += hz * uy; v[8] += hz * uz;
                    }
                    if (a.widx[j] >= 0 && r2 < a.mlp_rc2) {
                        const size_t st = (size_t)a.max_nbr * n, o = (size_t)k * n + i;
                        F0 += (double)a.hrev[o];
                        F1 += (double)a.hrev[st + o];
                        F2 += (double)a.hrev[2 * st + o];
                    }
                }
                if (a.ace_on) {
                    // (S14): (1 - lambda_i) f_ki from i's own site, minus (1 - lambda_k) f_ik from k's site
                    if (si >= 0) {
                        double fx, fy, fz;
                        load_f(fp, ((size_t)si * a.max_nbr + k) * 3, fx, fy, fz);
                        const double wgt = 1.0 - li;
                        F0 += wgt * fx;
                        F1 += wgt * fy;
                        F2 += wgt * fz;
                        const double vw = MIX ? 0.0 : wgt;
                        v[0] -= vw * fx * ux; v[1] -= vw * fx * uy; v[2] -= vw * fx * uz;
                        v[3] -= vw * fy * ux; v[4] -= vw * fy * uy; v[5] -= vw * fy * uz;
                        v[6] -= vw * fz * ux; v[7] -= vw * fz * uy; v[8] -= vw * fz * uz;
                    }
                    if (sj >= 0 && r2 < a.ace_rc2) {  // precise j: its term for this pair, stored at (k, i)
                        const TF *fr = reinterpret_cast<const TF *>(a.frev);
                        const size_t st = (size_t)a.max_nbr * n, o = (size_t)k * n + i;
                        const double fx = (double)fr[o], fy = (double)fr[st + o], fz = (double)fr[2 * st + o];
                        const double wgt = 1.0 - (MIX ? li : lj);
                        F0 -= wgt * fx;
                        F1 -= wgt * fy;
                        F2 -= wgt * fz;
                    }
                }
            }
        }
        if (FULL && gl && !a.ind_mlp) {
            // CSP part (S24)-(S27), its terms spread over the atom's SUB lanes: own list 2 W_i sum_l (r_il +
            // r_i,opp(l)); reverse entries -2 W_j (r_ji + r_j,opp(i)), looked for only where the W pass marked
            // a CSP neighbour with W_j != 0
            const double Wi = a.W[i];
            if (Wi != 0.0) {
                for (int t = sub; t < a.n_csp; t += SUB) {
                    const int l = a.csp_t[(size_t)t * n + i], o = a.csp_t[(size_t)(t ^ 1) * n + i];
                    // (other atoms' positions from their records: with the fused drift an atom's own
                    // entry of pos changes during this pass)
                    const Rec4 pl = a.xl[l], po = a.xl[o];
                    const double lx = min_image_w(pl.x - xi, a.L[0]), ly = min_image_w(pl.y - yi, a.L[1]),
                                 lz = min_image_w(pl.z - zi, a.L[2]);
                    const double ox = min_image_w(po.x - xi, a.L[0]), oy = min_image_w(po.y - yi, a.L[1]),
                                 oz = min_image_w(po.z - zi, a.L[2]);
                    const double sx = lx + ox, sy = ly + oy, sz = lz + oz;
                    F0 -= 2.0 * Wi * sx;
                    F1 -= 2.0 * Wi * sy;
                    F2 -= 2.0 * Wi * sz;
                    const double t2 = 2.0 * Wi;
                    v[0] += t2 * sx * lx; v[1] += t2 * sx * ly; v[2] += t2 * sx * lz;
                    v[3] += t2 * sy * lx; v[4] += t2 * sy * ly; v[5] += t2 * sy * lz;
                    v[6] += t2 * sz * lx; v[7] += t2 * sz * ly; v[8] += t2 * sz * lz;
                }
            }
            if (!a.cmark || a.cmark[i] == a.cgen) {
                const int rb = a.rev_start[i], re = a.rev_start[i + 1];
                for (int q = rb + sub; q < re; q += SUB) {
                    const int code = a.rev_code[q];
                    const int jj = code >> 4, t = code & 15;
                    const double Wj = a.W[jj];
                    if (Wj == 0.0) continue;
                    const int o = a.csp_t[(size_t)(t ^ 1) * n + jj];
                    const Rec4 pj = a.xl[jj], po = a.xl[o];
                    const double xj = pj.x, yj = pj.y, zj = pj.z;
                    const double sx = min_image_w(xi - xj, a.L[0]) + min_image_w(po.x - xj, a.L[0]);
                    const double sy = min_image_w(yi - yj, a.L[1]) + min_image_w(po.y - yj, a.L[1]);
                    const double sz = min_image_w(zi - zj, a.L[2]) + min_image_w(po.z - zj, a.L[2]);
                    F0 += 2.0 * Wj * sx;
                    F1 += 2.0 * Wj * sy;
                    F2 += 2.0 * Wj * sz;
                }
            }
        }
    }
    F0 = group_sum<SUB>(F0);
    F1 = group_sum<SUB>(F1);
    F2 = group_sum<SUB>(F2);
    double kin[4] = {0.0, 0.0, 0.0, 0.0};  // kinetic energy and momentum after the half-kick
    if (i < n && sub == 0) {
        const double li = a.lam[i];
        Ei = li * a.Ef[i] + (1.0 - li) * a.Ep[i];
        if (a.vel) {
            const double Fa[3] = {F0, F1, F2};
            double u2 = 0.0;
            for (int q = 0; q < 3; q++) {
                const size_t o = (size_t)q * n + i;
                double vq = a.vel[o] + a.hdtm * Fa[q];
                kin[0] += 0.5 * a.mass * vq * vq / kConv;
                kin[1 + q] = a.mass * vq;
                if (a.drift_pos) {
                    // the next step's first half-kick and drift, and the skin check of its list
                    vq = vq + a.hdtm * Fa[q];
                    const double x = wrap_coord(a.drift_pos[o] + a.dt * vq, a.L[q]);
                    a.drift_pos[o] = x;
                    a.ipos[o] = x;
                    const double u = min_image_w(x - a.pos_build[o], a.L[q]);
                    u2 += u * u;
                }
                a.vel[o] = vq;
            }
            if (a.drift_pos && u2 > a.half_skin2) atomicOr(&a.flags[0], 1);
        }
        if (a.E_atom) a.E_atom[i] = Ei;
        if (a.F) {
            a.F[i] = F0;
            a.F[n + i] = F1;
            a.F[2 * n + i] = F2;
        }
        if (!(isfinite(F0) && isfinite(F1) && isfinite(F2) && isfinite(Ei))) atomicOr(&a.flags[1], kErrNonFinite);
    }
    // this block's partials, column-major (column q at q * pstride): E, the virial (9) and, with the
    // half-kick, E_kin and P (4)
    const double vals[14] = {Ei, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8],
                             kin[0], kin[1], kin[2], kin[3]};
    if (a.vel)
        block_sums<14>(vals, sh, a.partials + blk, a.pstride);
    else
        block_sums<10>(vals, sh, a.partials + blk, a.pstride);
}

void launch_force(ap_ctx *c, int n, const double *box, const EvalFlags &f, double *E_atom, double *F,
                  const double *sbox, bool uniform_lambda, bool csp_marked) {
    ForceArgs a;
    a.cmark = csp_marked ? c->cmark : nullptr;
    a.cgen = c->stamp_gen;
    a.vel = sbox ? nullptr : c->kick_vel;
    a.hdtm = c->kick_hdtm;
    a.mass = c->kick_mass;
    a.drift_pos = a.vel ? c->drift_pos : nullptr;
    a.ipos = c->pos;
    a.pos_build = c->pos_build;
    a.dt = c->drift_dt;
    a.half_skin2 = 0.25 * c->skin * c->skin;
    a.cell_cnt = c->cell_cnt;
    a.cell_fill = c->cell_fill;
    a.ncell = a.drift_pos ? c->ncell_cur : 0;
    a.sbox = sbox;
    a.sid = c->sid;
    a.pos = c->pos;
    a.n = n;
    for (int q = 0; q < 3; q++) a.L[q] = box[q];
    a.ep = eamp(c->eam);
    a.sp = swp(c);
    a.switching = f.switching;
    a.grad_lambda = f.grad_lambda && !f.force_mix;
    a.eam_on = f.eam_forces;
    a.ace_on = f.ace_forces;
    a.ncount = c->nbr_cnt;
    a.nidx = c->nbr_idx;
    a.lam = c->lam;
    a.xip = c->xip;
    a.Ef = c->Ef;
    a.Ep = c->Ep;
    a.Et = c->Et;
    a.W = c->W;
    a.g = c->g;
    a.d = c->d;
    a.sidx = c->sidx;
    a.fpair = c->fpair;
    a.frev = c->frev;
    a.fp32 = c->ace.precision == AP_FP32;
    a.ace_rc2 = c->ace.rc * c->ace.rc;
    a.mlp_rc2 = c->mlp_rc * c->mlp_rc;
    a.max_nbr = c->max_nbr;
    a.n_csp = c->n_csp;
    a.csp_t = c->csp_t;
    a.rev_start = c->rev_start;
    a.rev_code = c->rev_code;
    a.E_atom = E_atom;
    a.F = F;
    a.partials = c->partials;
    a.pstride = c->pstride;
    a.flags = c->d_flags;
    a.ind_mlp = f.switching && !f.force_mix && c->sw.indicator == AP_IND_MLP;
    a.hpair = c->hpair;
    a.hrev = c->hrev;
    a.widx = c->widx;
    a.xl = c->xl;
    a.eb = c->eb;
    a.xe = c->xe;
    a.act = c->act;
    a.nshort = c->nbr_short;
    // 0: full lists; 1: EAM-only gather for the atoms with no lambda < 1 in reach; 2: EAM-only gather
    // for every atom; 3: EAM pairs only (short lists) with a per-atom lambda
    a.short_mode = 0;
    if (!sbox && f.switching && f.grad_lambda && c->sw.indicator == AP_IND_CSP) a.short_mode = 1;
    // force mixing: act (from the mixing marks) is lambda_i < 1; every other atom takes F^f_i alone, which
    // the EAM-only gather computes with lambda_i = 1 at both ends of each pair
    if (!sbox && f.force_mix) a.short_mode = 1;
    // the learned indicator needs the marks of the W pass to know who receives grad-g terms
    if (!sbox && f.switching && f.grad_lambda && c->sw.indicator == AP_IND_MLP && csp_marked) a.short_mode = 1;
    if (!sbox && !f.switching && (!f.ace_forces || f.lam_const == 1.0)) a.short_mode = uniform_lambda ? 2 : 3;
    a.ntiles = force_blocks(n);
    a.half_grid = (a.ntiles + 8 * kForceChunk - 1) / (8 * kForceChunk) * (8 * kForceChunk);
    // (above 2^18 atoms the first half's tens of thousands of empty blocks cost more than the overlap gains:
    // force pass 0.70 -> 0.76 ms at 2M atoms, 0.36 -> 0.37 ms at 1M)
    a.split_grid = a.short_mode == 1 && n <= kCountedCompactMax ? 1 : 0;
    const int nb = a.split_grid ? 2 * a.half_grid : a.half_grid;
    if (a.short_mode == 2)
        k_force<double, kForceLanes, false><<<nb, kBlock, 0, c->stream>>>(a);
    else if (f.force_mix && a.fp32)
        k_force<float, kForceLanes, true, true><<<nb, kBlock, 0, c->stream>>>(a);
    else if (f.force_mix)
        k_force<double, kForceLanes, true, true><<<nb, kBlock, 0, c->stream>>>(a);
    else if (a.fp32)
        k_force<float, kForceLanes, true><<<nb, kBlock, 0, c->stream>>>(a);
    else
        k_force<double, kForceLanes, true><<<nb, kBlock, 0, c->stream>>>(a);
}

// Sums the per-block partials (energy, virial; column-major [16][pstride]) in a fixed order, one workgroup
// per column.
__global__ __launch_bounds__(1024) void k_reduce_partials(const double *__restrict__ part, int nb, int pstride,
                                                          double *__restrict__ out, int *flags) {
    __shared__ double sh[1024 / 64];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(size_t)col * pstride + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); q++) t += sh[q];
        out[col] = t;
        if (!isfinite(t)) atomicOr(&flags[1], kErrNonFinite);
    }
}

void launch_reduce(ap_ctx *c, int nblocks, double *E_tot, double *virial9) {
    k_reduce_partials<<<10, 1024, 0, c->stream>>>(c->partials, nblocks, c->pstride, c->scalars, c->d_flags);
    if (E_tot) (void)hipMemcpyAsync(E_tot, c->scalars, sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (virial9) (void)hipMemcpyAsync(virial9, c->scalars + 1, 9 * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
}

// One thread per (structure, column): column 0 sums E^p_i, the next n_funcs columns dE_i/dc and the
// last n_max columns dE_i/db, each weighted by weight_i (1 when null), over the structure's atoms
// in index order.
template <typename TB>
__global__ void k_struct_reduce(int n_struct, int ncol, int n_funcs, const int *__restrict__ off,
                                const int *__restrict__ sidx, const double *__restrict__ weight,
                                const double *__restrict__ Ep, const TB *__restrict__ bval, int bstride,
                                double *E_struct, double *dEdc, double *dEdb, double sign) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n_struct * ncol) return;
    const int s = (int)(t / ncol), col = (int)(t % ncol);
    double acc = 0.0;
    for (int i = off[s]; i < off[s + 1]; i++) {
        const int si = sidx[i];
        if (si < 0) continue;
        const double w = weight ? weight[i] : 1.0;
        acc += w * (col == 0 ? Ep[i] : (double)bval[(size_t)si * bstride + col - 1]);
    }
    acc *= sign;
    if (col == 0) {
        if (E_struct) E_struct[s] = acc;
    } else if (col - 1 < n_funcs) {
        if (dEdc) dEdc[(size_t)s * n_funcs + col - 1] = acc;
    } else if (dEdb) {
        dEdb[(size_t)s * (ncol - 1 - n_funcs) + col - 1 - n_funcs] = acc;
    }
}

void launch_struct_reduce(ap_ctx *c, int n, int n_struct, const int *d_off, const double *weight, double *E_struct,
                          double *dEdc, double *dEdb, double sign) {
    (void)n;
    const int nf = c->ace.n_funcs, nm = c->ace.n_max;
    const int ncol = (dEdc || dEdb) ? 1 + nf + nm : 1;
    const long long tot = (long long)n_struct * ncol;
    const int nb = (int)((tot + kBlock - 1) / kBlock);
    if (c->ace.precision == AP_FP32)
        k_struct_reduce<float><<<nb, kBlock, 0, c->stream>>>(n_struct, ncol, nf, d_off, c->sidx, weight, c->Ep,
                                                            (const float *)c->bval, nf + nm, E_struct, dEdc, dEdb,
                                                            sign);
    else
        k_struct_reduce<double><<<nb, kBlock, 0, c->stream>>>(n_struct, ncol, nf, d_off, c->sidx, weight, c->Ep,
                                                             (const double *)c->bval, nf + nm, E_struct, dEdc, dEdb,
                                                             sign);
}

}  // namespace ap
