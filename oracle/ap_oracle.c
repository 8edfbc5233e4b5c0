/*
 * FP64 CPU oracle of the conservative adaptive-precision (AP) EAM/ACE energy and forces.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this file;
 * only the tests, the smoke check and the benchmark's CPU baseline use it. It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * It is written to be checked by eye against the paper:
 *   transition function f_trans ............ Eq. (2) and Eq. (S1)
 *   descriptor d_i, weight w, normalisation  Eq. (6) / (S2), weighting function of App. B
 *   switching parameter lambda_i ........... Eq. (2) / (S3)
 *   constant lambda on chosen atoms ........ App. B, the paragraph after (B4)
 *   AP energy E_i = l E^f + (1-l) E^p ...... Eq. (4)
 *   AP force (pair form) ................... Eq. (5), (A1)-(A2), (S5)-(S6)
 *   force mixing (non-conservative) ........ Eq. (3)
 *   EAM energy and pair force .............. (B1), (B2), (S7)-(S13)
 *   ACE pair force weighting ............... (S14)
 *   grad-lambda forces ..................... (S15)-(S21) (weight part), (S22)-(S27) (CSP part),
 *                                            (S28)-(S29)
 *   differentiable CSP with a fixed list ... (B3) / (S22)
 *   learned indicator g (network) .......... Eq. (6) with a general g, force term (S16)
 *   ACE coefficient gradient and the vector-Jacobian product of the forces with respect to the
 *   coefficients (derivatives of the ACE site energy; the paper cites ACE)
 *   velocity Verlet NVE .................... main text, time integration paragraph
 * The paper defines ACE only by reference; the concrete form used here (Chebyshev radial
 * channels, complex spherical harmonics with the Condon-Shortley phase, product basis of
 * body order <= 4 coupled with Wigner 3j symbols, site energy E0 + sum_nu c_nu B_nu minus
 * A*sqrt(density)) is the reading stated with each function below.
 *
 * Conventions: positions are AoS [n][3]; u_ij = r_j - r_i is the minimum-image vector from i
 * to j; f_ki = grad_k E_i (so that F_i = sum_k (f_ki - f_ik)). Units: Angstrom, eV, ps, u.
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fused multiply-add anywhere, so that the
 * neighbour distance test is the plain left-to-right sum of squares).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_E_ARG -1
#define ORA_E_BOX -2
#define ORA_E_NBR -3
#define ORA_E_CSP -6
#define ORA_E_MEM -7

#define AUX_W 12 /* per-atom diagnostic columns, see ora_eval */

static const double PI = 3.14159265358979323846;
static const double CONV = 9648.533212; /* eV/(A u) -> A/ps^2 */

int ora_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Transition function, Eq. (S1): 1 below lo, quintic in y = (hi+lo-2x)/(hi-lo), 0 above hi.  */
/* ------------------------------------------------------------------------------------------ */
double ora_ftrans(double x, double lo, double hi) {
    if (x <= lo) return 1.0;
    if (x >= hi) return 0.0;
    double y = (hi + lo - 2.0 * x) / (hi - lo);
    return 0.5 + 0.9375 * y - 0.625 * y * y * y + 0.1875 * y * y * y * y * y;
}

/* d f_trans / dx: df/dy = 0.9375 - 1.875 y^2 + 0.9375 y^4 and dy/dx = -2/(hi-lo). */
double ora_ftrans_d(double x, double lo, double hi) {
    if (x <= lo || x >= hi) return 0.0;
    double y = (hi + lo - 2.0 * x) / (hi - lo);
    double dfdy = 0.9375 - 1.875 * y * y + 0.9375 * y * y * y * y;
    return dfdy * (-2.0 / (hi - lo));
}

/* ------------------------------------------------------------------------------------------ */
/* Periodic geometry                                                                           */
/* ------------------------------------------------------------------------------------------ */
static double wrap1(double x, double L) {
    double y = x - L * floor(x / L);
    if (y >= L) y = 0.0;
    return y;
}

void ora_wrap(int n, double *pos, const double *L) {
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) pos[3 * i + a] = wrap1(pos[3 * i + a], L[a]);
}

/* u = r_j - r_i, minimum image with round-half-even. */
static void mic(const double *pos, const double *L, int i, int j, double u[3]) {
    for (int a = 0; a < 3; a++) {
        double d = pos[3 * j + a] - pos[3 * i + a];
        u[a] = d - L[a] * nearbyint(d / L[a]);
    }
}

static double sq3(const double u[3]) { return u[0] * u[0] + u[1] * u[1] + u[2] * u[2]; }

/* CSR neighbour list: for every i all j != i with |u_ij|^2 < r^2, ascending j. */
typedef struct {
    int n;
    int *start; /* [n+1] */
    int *idx;
} csr_t;

static void csr_free(csr_t *c) {
    free(c->start);
    free(c->idx);
    c->start = NULL;
    c->idx = NULL;
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Brute force O(n^2) when fewer than 3 cells per dimension fit, else a plain cell list. */
static int build_csr(int n, const double *pos, const double *L, double r, csr_t *out) {
    double r2 = r * r;
    out->n = n;
    out->start = (int *)calloc((size_t)n + 1, sizeof(int));
    if (!out->start) return ORA_E_MEM;
    int nc[3], use_cells = 1;
    for (int a = 0; a < 3; a++) {
        nc[a] = (int)floor(L[a] / r);
        if (nc[a] < 3) use_cells = 0;
    }
    int *cnt = (int *)calloc((size_t)n, sizeof(int));
    int *cell_of = NULL, *cstart = NULL, *catoms = NULL;
    if (use_cells) {
        int ncell = nc[0] * nc[1] * nc[2];
        cell_of = (int *)malloc(sizeof(int) * (size_t)n);
        cstart = (int *)calloc((size_t)ncell + 1, sizeof(int));
        catoms = (int *)malloc(sizeof(int) * (size_t)n);
        for (int i = 0; i < n; i++) {
            int c[3];
            for (int a = 0; a < 3; a++) {
                c[a] = (int)floor(pos[3 * i + a] / L[a] * nc[a]);
                if (c[a] >= nc[a]) c[a] = nc[a] - 1;
                if (c[a] < 0) c[a] = 0;
            }
            cell_of[i] = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
            cstart[cell_of[i] + 1]++;
        }
        for (int c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
        int *fill = (int *)calloc((size_t)ncell, sizeof(int));
        for (int i = 0; i < n; i++) catoms[cstart[cell_of[i]] + fill[cell_of[i]]++] = i;
        free(fill);
    }
    for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; i++) {
            int k = 0;
            int *dst = pass ? out->idx + out->start[i] : NULL;
            if (!use_cells) {
                for (int j = 0; j < n; j++) {
                    if (j == i) continue;
                    double u[3];
                    mic(pos, L, i, j, u);
                    if (sq3(u) < r2) {
                        if (pass) dst[k] = j;
                        k++;
                    }
                }
            } else {
                int ci = cell_of[i];
                int c0 = ci / (nc[1] * nc[2]), c1 = (ci / nc[2]) % nc[1], c2 = ci % nc[2];
                for (int dx = -1; dx <= 1; dx++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dz = -1; dz <= 1; dz++) {
                            int x = (c0 + dx + nc[0]) % nc[0], y = (c1 + dy + nc[1]) % nc[1],
                                z = (c2 + dz + nc[2]) % nc[2];
                            int c = (x * nc[1] + y) * nc[2] + z;
                            for (int p = cstart[c]; p < cstart[c + 1]; p++) {
                                int j = catoms[p];
                                if (j == i) continue;
                                double u[3];
                                mic(pos, L, i, j, u);
                                if (sq3(u) < r2) {
                                    if (pass) dst[k] = j;
                                    k++;
                                }
                            }
                        }
                if (pass) qsort(dst, (size_t)k, sizeof(int), cmp_int);
            }
            if (!pass) cnt[i] = k;
        }
        if (!pass) {
            for (int i = 0; i < n; i++) out->start[i + 1] = out->start[i] + cnt[i];
            out->idx = (int *)malloc(sizeof(int) * ((size_t)out->start[n] + 1));
            if (!out->idx) return ORA_E_MEM;
        }
    }
    free(cnt);
    free(cell_of);
    free(cstart);
    free(catoms);
    return ORA_OK;
}

static int check_box(const double *L, double r) {
    for (int a = 0; a < 3; a++)
        if (!(r < 0.5 * L[a])) return ORA_E_BOX;
    return ORA_OK;
}

/* Neighbour sets at radius r (strict), written as [n][cap] ascending with counts. The positions
 * are wrapped into the box first. Returns ORA_E_NBR if any atom has more than cap neighbours. */
int ora_nblist(int n, const double *pos_in, const double *L, double r, int cap, int *count, int *idx) {
    if (n < 0 || !pos_in || !L || cap < 0) return ORA_E_ARG;
    int rc = check_box(L, r);
    if (rc) return rc;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t c;
    rc = build_csr(n, pos, L, r, &c);
    if (!rc) {
        for (int i = 0; i < n; i++) {
            int k = c.start[i + 1] - c.start[i];
            count[i] = k;
            if (k > cap) {
                rc = ORA_E_NBR;
                continue;
            }
            for (int q = 0; q < k; q++) idx[(size_t)i * cap + q] = c.idx[c.start[i] + q];
        }
    }
    csr_free(&c);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* CSP pair list, (B3): the opposite-neighbour pairs are detected once and then kept.          */
/* Reading: the n_csp nearest neighbours ordered by (|u|^2, index); all pairs (a,b) scored by   */
/* |u_ia + u_ib|^2; greedy choice of the smallest score (ties: smaller lower index, then        */
/* smaller higher index) over unused atoms until n_csp/2 pairs. Stored pair by pair in choice   */
/* order, lower index first, so entry 2p and 2p+1 are each other's opposite partner.            */
/* ------------------------------------------------------------------------------------------ */
int ora_csp_pairs(int n, const double *pos_in, const double *L, double r_search, int n_csp, int *list) {
    if (n_csp != 8 && n_csp != 12) return ORA_E_CSP;
    int rc = check_box(L, r_search);
    if (rc) return rc;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t c;
    rc = build_csr(n, pos, L, r_search, &c);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int i = 0; i < n; i++) {
        int k = c.start[i + 1] - c.start[i];
        if (k < n_csp) {
            bad = 1;
            continue;
        }
        int sel[12];
        double seld[12];
        int used_n = 0;
        /* selection of the n_csp smallest (d2, j) by repeated minimum search */
        char *taken = (char *)calloc((size_t)k, 1);
        for (int s = 0; s < n_csp; s++) {
            int best = -1;
            double bd = 0;
            for (int q = 0; q < k; q++) {
                if (taken[q]) continue;
                int j = c.idx[c.start[i] + q];
                double u[3];
                mic(pos, L, i, j, u);
                double d2 = sq3(u);
                if (best < 0 || d2 < bd || (d2 == bd && j < c.idx[c.start[i] + best])) {
                    best = q;
                    bd = d2;
                }
            }
            taken[best] = 1;
            sel[used_n] = c.idx[c.start[i] + best];
            seld[used_n] = bd;
            used_n++;
        }
        free(taken);
        (void)seld;
        int used[12] = {0};
        for (int p = 0; p < n_csp / 2; p++) {
            int ba = -1, bb = -1;
            double bs = 0;
            for (int a = 0; a < n_csp; a++) {
                if (used[a]) continue;
                for (int b = a + 1; b < n_csp; b++) {
                    if (used[b]) continue;
                    double ua[3], ub[3];
                    mic(pos, L, i, sel[a], ua);
                    mic(pos, L, i, sel[b], ub);
                    double sx = ua[0] + ub[0], sy = ua[1] + ub[1], sz = ua[2] + ub[2];
                    double s = sx * sx + sy * sy + sz * sz;
                    int lo = sel[a] < sel[b] ? sel[a] : sel[b];
                    int hi = sel[a] < sel[b] ? sel[b] : sel[a];
                    int blo = 0, bhi = 0;
                    if (ba >= 0) {
                        blo = sel[ba] < sel[bb] ? sel[ba] : sel[bb];
                        bhi = sel[ba] < sel[bb] ? sel[bb] : sel[ba];
                    }
                    if (ba < 0 || s < bs || (s == bs && (lo < blo || (lo == blo && hi < bhi)))) {
                        ba = a;
                        bb = b;
                        bs = s;
                    }
                }
            }
            used[ba] = used[bb] = 1;
            int lo = sel[ba] < sel[bb] ? sel[ba] : sel[bb];
            int hi = sel[ba] < sel[bb] ? sel[bb] : sel[ba];
            list[(size_t)i * n_csp + 2 * p] = lo;
            list[(size_t)i * n_csp + 2 * p + 1] = hi;
        }
    }
    csr_free(&c);
    free(pos);
    if (rc) return rc;
    return bad ? ORA_E_CSP : ORA_OK;
}

/* g_i = CSP_i^list of (B3): sum over the n_csp listed j of (1/2)|r_ij + r_i,opp(j)|^2, i.e. the
 * sum over the n_csp/2 stored pairs of |u_ia + u_ib|^2. */
static double csp_value(const double *pos, const double *L, int i, int n_csp, const int *list) {
    double g = 0.0;
    for (int p = 0; p < n_csp / 2; p++) {
        double ua[3], ub[3];
        mic(pos, L, i, list[(size_t)i * n_csp + 2 * p], ua);
        mic(pos, L, i, list[(size_t)i * n_csp + 2 * p + 1], ub);
        double s[3] = {ua[0] + ub[0], ua[1] + ub[1], ua[2] + ub[2]};
        g += sq3(s);
    }
    return g;
}

/* ------------------------------------------------------------------------------------------ */
/* EAM, Finnis-Sinclair form of (B1): zeta(r) = (r-r_rho)^2 + beta (r-r_rho)^3/r_rho for r < r_rho, */
/* Phi(r) = (r-r_phi)^2 (c0 + c1 r + c2 r^2) for r < r_phi, xi(z) = -A sqrt(z).                   */
/* eam_p = {A, beta, c0, c1, c2, r_rho, r_phi}.                                                   */
/* ------------------------------------------------------------------------------------------ */
static void eam_pair(const double *p, double r, double *z, double *dz, double *ph, double *dph) {
    double rr = p[5], rp = p[6];
    *z = *dz = *ph = *dph = 0.0;
    if (r < rr) {
        double x = r - rr;
        *z = x * x + p[1] * x * x * x / rr;
        *dz = 2.0 * x + 3.0 * p[1] * x * x / rr;
    }
    if (r < rp) {
        double y = r - rp;
        double q = p[2] + p[3] * r + p[4] * r * r;
        *ph = y * y * q;
        *dph = 2.0 * y * q + y * y * (p[3] + 2.0 * p[4] * r);
    }
}

static void embed(double A, double z, double *f, double *df) {
    /* xi(z) = -A sqrt(z); an atom without neighbours (z == 0) has no embedding term. */
    if (z > 0.0) {
        double s = sqrt(z);
        *f = -A * s;
        *df = -0.5 * A / s;
    } else {
        *f = 0.0;
        *df = 0.0;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* ACE ingredients                                                                              */
/* ------------------------------------------------------------------------------------------ */
/* Chebyshev radial channels g_n(r) = T_n(2r/rc - 1) * fc(r), fc = (1 + cos(pi r/rc))/2. */
void ora_radial(int n_max, double rc, double r, double *g, double *dg) {
    if (r >= rc) {
        for (int n = 0; n < n_max; n++) g[n] = dg[n] = 0.0;
        return;
    }
    double x = 2.0 * r / rc - 1.0, dxdr = 2.0 / rc;
    double fc = 0.5 * (1.0 + cos(PI * r / rc));
    double dfc = -0.5 * PI / rc * sin(PI * r / rc);
    double T[32], dT[32];
    T[0] = 1.0;
    dT[0] = 0.0;
    if (n_max > 1) {
        T[1] = x;
        dT[1] = 1.0;
    }
    for (int n = 2; n < n_max; n++) {
        T[n] = 2.0 * x * T[n - 1] - T[n - 2];
        dT[n] = 2.0 * T[n - 1] + 2.0 * x * dT[n - 1] - dT[n - 2];
    }
    for (int n = 0; n < n_max; n++) {
        g[n] = T[n] * fc;
        dg[n] = dT[n] * dxdr * fc + T[n] * dfc;
    }
}

static double fact(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= i;
    return f;
}

static double binom(int a, int b) { return fact(a) / (fact(b) * fact(a - b)); }

/* Complex spherical harmonics Y_l^m(u/|u|) with the Condon-Shortley phase, orthonormal on the
 * sphere, for 0 <= l <= l_max, stored at index l*l + l + m; and their gradients with respect to
 * the unnormalised vector u (dY[3*idx + a] = d Y / d u_a).
 * Written as polynomials in the unit-vector components:
 *   Y_l^m = K_lm (-1)^m (x + i y)^m Q_lm(z),  m >= 0,
 *   Q_lm(z) = d^m/dz^m P_l(z) with Rodrigues' expansion of the Legendre polynomial P_l,
 *   K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),  Y_l^{-m} = (-1)^m conj(Y_l^m).
 * The gradient is (I - uhat uhat^T) grad_p / |u| of the polynomial p(x, y, z). */
void ora_ylm_c(int l_max, const double *u, double complex *Y, double complex *dY) {
    double r = sqrt(sq3(u));
    double x = u[0] / r, y = u[1] / r, z = u[2] / r;
    double complex w = x + I * y;
    for (int l = 0; l <= l_max; l++) {
        for (int m = 0; m <= l; m++) {
            /* Q(z) and Q'(z) from P_l(t) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) t^(l-2k) */
            double Q = 0.0, dQ = 0.0;
            for (int k = 0; 2 * k <= l; k++) {
                int p = l - 2 * k;
                if (p < m) continue;
                double a = ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l) / pow(2.0, l);
                double c = a * fact(p) / fact(p - m);
                int e = p - m;
                Q += c * (e > 0 ? pow(z, e) : 1.0);
                if (e > 0) dQ += c * e * (e > 1 ? pow(z, e - 1) : 1.0);
            }
            double K = sqrt((2.0 * l + 1.0) / (4.0 * PI) * fact(l - m) / fact(l + m));
            double sgn = (m & 1) ? -1.0 : 1.0;
            double complex wm = cpow(w, m), wm1 = m > 0 ? (m > 1 ? cpow(w, m - 1) : 1.0) : 0.0;
            if (m == 0) wm = 1.0;
            double complex val = K * sgn * wm * Q;
            double complex gp[3];
            gp[0] = K * sgn * (double)m * wm1 * Q;
            gp[1] = K * sgn * I * (double)m * wm1 * Q;
            gp[2] = K * sgn * wm * dQ;
            double complex radial = gp[0] * x + gp[1] * y + gp[2] * z;
            double complex g[3] = {(gp[0] - radial * x) / r, (gp[1] - radial * y) / r, (gp[2] - radial * z) / r};
            int ip = l * l + l + m, im = l * l + l - m;
            Y[ip] = val;
            if (dY)
                for (int a = 0; a < 3; a++) dY[3 * ip + a] = g[a];
            if (m > 0) {
                Y[im] = sgn * conj(val);
                if (dY)
                    for (int a = 0; a < 3; a++) dY[3 * im + a] = sgn * conj(g[a]);
            }
        }
    }
}

/* Split real/imag export of ora_ylm_c for tests. */
void ora_ylm(int l_max, const double *u, double *Yre, double *Yim, double *dYre, double *dYim) {
    int nlm = (l_max + 1) * (l_max + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nlm);
    double complex *dY = (double complex *)malloc(sizeof(double complex) * 3 * (size_t)nlm);
    ora_ylm_c(l_max, u, Y, dY);
    for (int t = 0; t < nlm; t++) {
        Yre[t] = creal(Y[t]);
        Yim[t] = cimag(Y[t]);
        if (dYre)
            for (int a = 0; a < 3; a++) {
                dYre[3 * t + a] = creal(dY[3 * t + a]);
                dYim[3 * t + a] = cimag(dY[3 * t + a]);
            }
    }
    free(Y);
    free(dY);
}

/* Wigner 3j symbol by Racah's closed form. */
double ora_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
    double pre = sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) * fact(j3 + m3) *
                      fact(j3 - m3));
    double s = 0.0;
    for (int k = 0; k <= j1 + j2 + j3; k++) {
        int d1 = j3 - j2 + k + m1, d2 = j3 - j1 + k - m2, d3 = j1 + j2 - j3 - k, d4 = j1 - k - m1,
            d5 = j2 - k + m2;
        if (d1 < 0 || d2 < 0 || d3 < 0 || d4 < 0 || d5 < 0) continue;
        double t = 1.0 / (fact(k) * fact(d1) * fact(d2) * fact(d3) * fact(d4) * fact(d5));
        s += (k & 1) ? -t : t;
    }
    int ph = j1 - j2 - m3;
    double sign = (ph % 2 == 0) ? 1.0 : -1.0;
    return sign * pre * s;
}

/* ACE potential description, shared by the ACE routines below. */
typedef struct {
    int n_max, l_max, n_funcs;
    double rc;
    const int *func;      /* [n_funcs][6] (n1,l1,n2,l2,n3,l3), -1 = unused slot */
    const double *c;      /* [n_funcs] linear coefficients of B_nu                */
    const double *b_dens; /* [n_max] coefficients of the embedded density        */
    double emb_A, E0;
    double *w3j;          /* 3j table [(l1,l2,l3)][m1][m2], built on first use     */
} ace_t;

static int ace_nlm(const ace_t *p) { return (p->l_max + 1) * (p->l_max + 1); }

static void ace_build_3j(ace_t *p) {
    int L1 = p->l_max + 1, M = 2 * p->l_max + 1;
    p->w3j = (double *)calloc((size_t)L1 * L1 * L1 * M * M, sizeof(double));
    for (int l1 = 0; l1 < L1; l1++)
        for (int l2 = 0; l2 < L1; l2++)
            for (int l3 = 0; l3 < L1; l3++)
                for (int m1 = -l1; m1 <= l1; m1++)
                    for (int m2 = -l2; m2 <= l2; m2++) {
                        int m3 = -m1 - m2;
                        if (abs(m3) > l3) continue;
                        p->w3j[((((size_t)l1 * L1 + l2) * L1 + l3) * M + (m1 + p->l_max)) * M + (m2 + p->l_max)] =
                            ora_wigner3j(l1, l2, l3, m1, m2, m3);
                    }
}

static double w3(const ace_t *p, int l1, int l2, int l3, int m1, int m2) {
    int L1 = p->l_max + 1, M = 2 * p->l_max + 1;
    return p->w3j[((((size_t)l1 * L1 + l2) * L1 + l3) * M + (m1 + p->l_max)) * M + (m2 + p->l_max)];
}

/* Site energy of one atom from its neighbour vectors u_j (|u_j| < rc):
 *   A_{nlm} = sum_j g_n(|u_j|) Y_l^m(u_j/|u_j|)
 *   B (order 1) = A_{n00};  B (order 2) = sum_m (-1)^m A_{n1 l m} A_{n2 l -m};
 *   B (order 3) = sum_{m1,m2} (l1 l2 l3; m1 m2 -m1-m2) A_{n1 l1 m1} A_{n2 l2 m2} A_{n3 l3 -m1-m2}
 *   E = E0 + sum_nu c_nu B_nu + xi(phi2),  phi2 = sum_n b_n sqrt(4 pi) A_{n00},  xi = -emb_A sqrt
 * E is a polynomial in A without conjugates (holomorphic), so dE/du = Re sum dE/dA dA/du.
 * Outputs (any may be NULL except E): dEdu [nn][3] = grad_{u_j} E (= f_ji with r_j moving);
 * B [n_funcs] (real parts); Aout [n_max*nlm] complex; phi2 out. */
static void ace_site(const ace_t *p, int nn, const double *u, double *E, double *dEdu, double *B,
                     double complex *Aout, double *phi2_out) {
    int nmax = p->n_max, nlm = ace_nlm(p), lmax = p->l_max;
    double complex *A = (double complex *)calloc((size_t)nmax * nlm, sizeof(double complex));
    double complex *G = (double complex *)calloc((size_t)nmax * nlm, sizeof(double complex));
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nlm);
    double complex *dY = (double complex *)malloc(sizeof(double complex) * 3 * (size_t)nlm);
    double g[32], dg[32];
    for (int j = 0; j < nn; j++) {
        const double *uj = u + 3 * j;
        double r = sqrt(sq3(uj));
        if (r >= p->rc) continue;
        ora_radial(nmax, p->rc, r, g, dg);
        ora_ylm_c(lmax, uj, Y, NULL);
        for (int n = 0; n < nmax; n++)
            for (int t = 0; t < nlm; t++) A[n * nlm + t] += g[n] * Y[t];
    }
#define AA(n, l, m) A[(n) * nlm + (l) * (l) + (l) + (m)]
#define GG(n, l, m) G[(n) * nlm + (l) * (l) + (l) + (m)]
    double e = p->E0;
    for (int f = 0; f < p->n_funcs; f++) {
        const int *q = p->func + 6 * f;
        double cf = p->c[f];
        double complex b = 0.0;
        if (q[2] < 0) { /* order 1 */
            b = AA(q[0], 0, 0);
            GG(q[0], 0, 0) += cf;
        } else if (q[4] < 0) { /* order 2 */
            int n1 = q[0], l = q[1], n2 = q[2];
            for (int m = -l; m <= l; m++) {
                double sg = (m & 1) ? -1.0 : 1.0;
                b += sg * AA(n1, l, m) * AA(n2, l, -m);
                GG(n1, l, m) += cf * sg * AA(n2, l, -m);
                GG(n2, l, -m) += cf * sg * AA(n1, l, m);
            }
        } else { /* order 3 */
            int n1 = q[0], l1 = q[1], n2 = q[2], l2 = q[3], n3 = q[4], l3 = q[5];
            for (int m1 = -l1; m1 <= l1; m1++)
                for (int m2 = -l2; m2 <= l2; m2++) {
                    int m3 = -m1 - m2;
                    if (m3 < -l3 || m3 > l3) continue;
                    double wv = w3(p, l1, l2, l3, m1, m2);
                    if (wv == 0.0) continue;
                    double complex a1 = AA(n1, l1, m1), a2 = AA(n2, l2, m2), a3 = AA(n3, l3, m3);
                    b += wv * a1 * a2 * a3;
                    GG(n1, l1, m1) += cf * wv * a2 * a3;
                    GG(n2, l2, m2) += cf * wv * a1 * a3;
                    GG(n3, l3, m3) += cf * wv * a1 * a2;
                }
        }
        if (B) B[f] = creal(b);
        e += cf * creal(b);
    }
    double phi2 = 0.0, s4pi = sqrt(4.0 * PI);
    for (int n = 0; n < nmax; n++) phi2 += p->b_dens[n] * s4pi * creal(AA(n, 0, 0));
    double fe, dfe;
    embed(p->emb_A, phi2, &fe, &dfe);
    e += fe;
    for (int n = 0; n < nmax; n++) GG(n, 0, 0) += dfe * p->b_dens[n] * s4pi;
    *E = e;
    if (phi2_out) *phi2_out = phi2;
    if (dEdu) {
        for (int j = 0; j < nn; j++) {
            const double *uj = u + 3 * j;
            double r = sqrt(sq3(uj));
            double out[3] = {0, 0, 0};
            if (r < p->rc) {
                ora_radial(nmax, p->rc, r, g, dg);
                ora_ylm_c(lmax, uj, Y, dY);
                for (int t = 0; t < nlm; t++) {
                    double complex sg = 0.0, sdg = 0.0;
                    for (int n = 0; n < nmax; n++) {
                        sg += G[n * nlm + t] * g[n];
                        sdg += G[n * nlm + t] * dg[n];
                    }
                    for (int a = 0; a < 3; a++)
                        out[a] += creal(sdg * Y[t] * (uj[a] / r) + sg * dY[3 * t + a]);
                }
            }
            for (int a = 0; a < 3; a++) dEdu[3 * j + a] = out[a];
        }
    }
    if (Aout) memcpy(Aout, A, sizeof(double complex) * (size_t)nmax * nlm);
#undef AA
#undef GG
    free(A);
    free(G);
    free(Y);
    free(dY);
}

/* Single-environment entry for tests: energy, gradient, B values and A (real/imag parts). */
int ora_ace_env(int nn, const double *u, int n_max, int l_max, double rc, int n_funcs, const int *func,
                const double *c, const double *b_dens, double emb_A, double E0, double *E, double *dEdu,
                double *B, double *A_re, double *A_im, double *phi2) {
    ace_t p = {n_max, l_max, n_funcs, rc, func, c, b_dens, emb_A, E0, NULL};
    if (n_max > 32 || l_max > 12) return ORA_E_ARG;
    ace_build_3j(&p);
    int nlm = ace_nlm(&p);
    double complex *A = (double complex *)malloc(sizeof(double complex) * (size_t)n_max * nlm);
    ace_site(&p, nn, u, E, dEdu, B, A, phi2);
    if (A_re)
        for (int t = 0; t < n_max * nlm; t++) {
            A_re[t] = creal(A[t]);
            A_im[t] = cimag(A[t]);
        }
    free(A);
    free(p.w3j);
    return ORA_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Learned indicator: a small network in place of CSP as the per-atom quantity g of Eq. (6)     */
/* ------------------------------------------------------------------------------------------ */
/* Eq. (6) admits any per-atom scalar g. With g_j a smooth function of the neighbourhood of j,
 * E depends on g_j only through the descriptors d_k, and dE/dg_j = -sum_k E~_k w(r_kj) = -W_j
 * with E~ of (S17); the general grad-g term of (S16) is then F_i += sum_j W_j grad_i g_j, the
 * same W_j as in the CSP part (S25), with grad_i g_j from the network instead of (S24).
 *
 * Features: sixteen rotation invariants of the neighbours inside rc, built from the same
 * Chebyshev radial channels g_n and complex harmonics as the ACE reading above:
 *   q[n]               = sum_j g_n(r_ij),                       n = 0..7
 *   q[8 + 4 n + l - 1] = sum_m |A_nlm|^2,  A_nlm = sum_j g_n(r_ij) Y_l^m(u_ij),   n = 0, 1; l = 1..4
 * Network: z = (q - mu) / sig, h1 = silu(W1 z + b1), h2 = silu(W2 h1 + b2), o = w3 . h2 + b3,
 * g = softplus(o), with silu(a) = a / (1 + e^-a). Trained on o against log(|E^ACE - E^EAM| + eps).
 * Parameter block (MLP_NP doubles): mu[16] sig[16] W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3.
 */
#define MLP_NQ 16
#define MLP_NH 64
#define MLP_MU 0
#define MLP_SIG 16
#define MLP_W1 32
#define MLP_B1 (MLP_W1 + MLP_NH * MLP_NQ)
#define MLP_W2 (MLP_B1 + MLP_NH)
#define MLP_B2 (MLP_W2 + MLP_NH * MLP_NH)
#define MLP_W3 (MLP_B2 + MLP_NH)
#define MLP_B3 (MLP_W3 + MLP_NH)
#define MLP_NP (MLP_B3 + 1)

int ora_mlp_nparams(void) { return MLP_NP; }

/* features q[16] of one environment (nn neighbour vectors u, any distance; r >= rc ignored) and,
 * if dq != NULL, dq[j][f][a] = d q_f / d u_j,a. */
static void mlp_site_features(int nn, const double *u, double rc, double *q, double *dq) {
    double complex A[2][25];
    memset(A, 0, sizeof(A));
    for (int f = 0; f < MLP_NQ; f++) q[f] = 0.0;
    for (int j = 0; j < nn; j++) {
        const double *uj = u + 3 * j;
        double r = sqrt(sq3(uj));
        if (r >= rc) continue;
        double g[8], dg[8];
        ora_radial(8, rc, r, g, dg);
        double complex Y[25];
        ora_ylm_c(4, uj, Y, NULL);
        for (int n = 0; n < 8; n++) q[n] += g[n];
        for (int n = 0; n < 2; n++)
            for (int t = 1; t < 25; t++) A[n][t] += g[n] * Y[t];
    }
    for (int n = 0; n < 2; n++)
        for (int l = 1; l <= 4; l++) {
            double s = 0.0;
            for (int m = -l; m <= l; m++) {
                double complex a = A[n][l * l + l + m];
                s += creal(a) * creal(a) + cimag(a) * cimag(a);
            }
            q[8 + 4 * n + l - 1] = s;
        }
    if (!dq) return;
    for (int j = 0; j < nn; j++) {
        const double *uj = u + 3 * j;
        double *d = dq + (size_t)j * MLP_NQ * 3;
        for (int f = 0; f < 3 * MLP_NQ; f++) d[f] = 0.0;
        double r = sqrt(sq3(uj));
        if (r >= rc) continue;
        double g[8], dg[8];
        ora_radial(8, rc, r, g, dg);
        double complex Y[25], dY[75];
        ora_ylm_c(4, uj, Y, dY);
        double e[3] = {uj[0] / r, uj[1] / r, uj[2] / r};
        for (int n = 0; n < 8; n++)
            for (int a = 0; a < 3; a++) d[3 * n + a] = dg[n] * e[a];
        /* d sum_m |A|^2 / du = 2 Re sum_m conj(A) d(g_n Y)/du */
        for (int n = 0; n < 2; n++)
            for (int l = 1; l <= 4; l++)
                for (int m = -l; m <= l; m++) {
                    int t = l * l + l + m;
                    double complex a = conj(A[n][t]);
                    for (int c = 0; c < 3; c++) {
                        double complex dgy = dg[n] * e[c] * Y[t] + g[n] * dY[3 * t + c];
                        d[3 * (8 + 4 * n + l - 1) + c] += 2.0 * creal(a * dgy);
                    }
                }
    }
}

static double sigm(double a) { return 1.0 / (1.0 + exp(-a)); }

/* one sample: o, g = softplus(o) and dg/dq (NULL allowed) */
static void mlp_forward1(const double *P, const double *q, double *o_out, double *g_out, double *dgdq) {
    double z[MLP_NQ], a1[MLP_NH], h1[MLP_NH], a2[MLP_NH], h2[MLP_NH];
    for (int f = 0; f < MLP_NQ; f++) z[f] = (q[f] - P[MLP_MU + f]) / P[MLP_SIG + f];
    for (int c = 0; c < MLP_NH; c++) {
        double s = P[MLP_B1 + c];
        for (int f = 0; f < MLP_NQ; f++) s += P[MLP_W1 + c * MLP_NQ + f] * z[f];
        a1[c] = s;
        h1[c] = s * sigm(s);
    }
    for (int c = 0; c < MLP_NH; c++) {
        double s = P[MLP_B2 + c];
        for (int k = 0; k < MLP_NH; k++) s += P[MLP_W2 + c * MLP_NH + k] * h1[k];
        a2[c] = s;
        h2[c] = s * sigm(s);
    }
    double o = P[MLP_B3];
    for (int c = 0; c < MLP_NH; c++) o += P[MLP_W3 + c] * h2[c];
    *o_out = o;
    *g_out = o > 0.0 ? o + log1p(exp(-o)) : log1p(exp(o));
    if (!dgdq) return;
    /* backward from dg/do = sigmoid(o); silu'(a) = s (1 + a (1 - s)), s = sigmoid(a) */
    double d2[MLP_NH], d1[MLP_NH];
    double go = sigm(o);
    for (int c = 0; c < MLP_NH; c++) {
        double s = sigm(a2[c]);
        d2[c] = go * P[MLP_W3 + c] * s * (1.0 + a2[c] * (1.0 - s));
    }
    for (int k = 0; k < MLP_NH; k++) {
        double t = 0.0;
        for (int c = 0; c < MLP_NH; c++) t += P[MLP_W2 + c * MLP_NH + k] * d2[c];
        double s = sigm(a1[k]);
        d1[k] = t * s * (1.0 + a1[k] * (1.0 - s));
    }
    for (int f = 0; f < MLP_NQ; f++) {
        double t = 0.0;
        for (int c = 0; c < MLP_NH; c++) t += P[MLP_W1 + c * MLP_NQ + f] * d1[c];
        dgdq[f] = t / P[MLP_SIG + f];
    }
}

/* features of every atom of a periodic cell (q[n][16]) */
int ora_mlp_features(int n, const double *pos_in, const double *L, double rc, double *q) {
    int rc_ = check_box(L, rc);
    if (rc_) return rc_;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t nb;
    rc_ = build_csr(n, pos, L, rc, &nb);
    if (!rc_) {
#pragma omp parallel
        {
            double *u = (double *)malloc(sizeof(double) * 3 * 4096);
#pragma omp for schedule(static)
            for (int i = 0; i < n; i++) {
                int nn = nb.start[i + 1] - nb.start[i];
                if (nn > 4096) nn = 4096;
                for (int k = 0; k < nn; k++) mic(pos, L, i, nb.idx[nb.start[i] + k], u + 3 * k);
                mlp_site_features(nn, u, rc, q + (size_t)i * MLP_NQ, NULL);
            }
            free(u);
        }
        csr_free(&nb);
    }
    free(pos);
    return rc_;
}

/* network outputs for m samples: o[m], g[m], dgdq[m][16] (may be NULL) */
void ora_mlp_forward(int m, const double *q, const double *P, double *o, double *g, double *dgdq) {
#pragma omp parallel for schedule(static)
    for (int s = 0; s < m; s++)
        mlp_forward1(P, q + (size_t)s * MLP_NQ, o + s, g + s, dgdq ? dgdq + (size_t)s * MLP_NQ : NULL);
}

/* training loss L = (1/m) sum_s (o_s - t_s)^2 and its gradient with respect to every parameter
 * (grad[MLP_NP]; the normalisation entries mu, sig are not trained and get 0). Written as the
 * chain rule layer by layer for each sample and summed over samples in order. */
double ora_mlp_loss_grad(int m, const double *q, const double *t, const double *P, double *grad) {
    for (int k = 0; k < MLP_NP; k++) grad[k] = 0.0;
    double loss = 0.0;
    for (int s = 0; s < m; s++) {
        const double *qs = q + (size_t)s * MLP_NQ;
        double z[MLP_NQ], a1[MLP_NH], h1[MLP_NH], a2[MLP_NH], h2[MLP_NH];
        for (int f = 0; f < MLP_NQ; f++) z[f] = (qs[f] - P[MLP_MU + f]) / P[MLP_SIG + f];
        for (int c = 0; c < MLP_NH; c++) {
            double v = P[MLP_B1 + c];
            for (int f = 0; f < MLP_NQ; f++) v += P[MLP_W1 + c * MLP_NQ + f] * z[f];
            a1[c] = v;
            h1[c] = v * sigm(v);
        }
        for (int c = 0; c < MLP_NH; c++) {
            double v = P[MLP_B2 + c];
            for (int k = 0; k < MLP_NH; k++) v += P[MLP_W2 + c * MLP_NH + k] * h1[k];
            a2[c] = v;
            h2[c] = v * sigm(v);
        }
        double o = P[MLP_B3];
        for (int c = 0; c < MLP_NH; c++) o += P[MLP_W3 + c] * h2[c];
        double r = o - t[s];
        loss += r * r / m;
        double go = 2.0 * r / m;
        double d2[MLP_NH], d1[MLP_NH];
        grad[MLP_B3] += go;
        for (int c = 0; c < MLP_NH; c++) {
            grad[MLP_W3 + c] += go * h2[c];
            double sg = sigm(a2[c]);
            d2[c] = go * P[MLP_W3 + c] * sg * (1.0 + a2[c] * (1.0 - sg));
        }
        for (int c = 0; c < MLP_NH; c++) {
            grad[MLP_B2 + c] += d2[c];
            for (int k = 0; k < MLP_NH; k++) grad[MLP_W2 + c * MLP_NH + k] += d2[c] * h1[k];
        }
        for (int k = 0; k < MLP_NH; k++) {
            double v = 0.0;
            for (int c = 0; c < MLP_NH; c++) v += P[MLP_W2 + c * MLP_NH + k] * d2[c];
            double sg = sigm(a1[k]);
            d1[k] = v * sg * (1.0 + a1[k] * (1.0 - sg));
        }
        for (int c = 0; c < MLP_NH; c++) {
            grad[MLP_B1 + c] += d1[c];
            for (int f = 0; f < MLP_NQ; f++) grad[MLP_W1 + c * MLP_NQ + f] += d1[c] * z[f];
        }
    }
    return loss;
}

/* ------------------------------------------------------------------------------------------ */
/* Descriptor, Eq. (6): d_i = sum_k g_k w(r_ik) / wbar_i - d0 with wbar_i = sum_k w(r_ik) and    */
/* the weighting function w(r) = f_trans(r, r_w - 1 A, r_w) of App. B. Both sums run over every */
/* atom k within r_w of i, the atom itself included (k = i, w(0) = 1).                           */
/* ------------------------------------------------------------------------------------------ */
static void descriptor_site(const double *pos, const double *L, const csr_t *nb, int i, const double *g, int gs,
                            double r_w, double d0, double *wbar, double *d) {
    double wsum = 1.0, gsum = g[(size_t)i * gs]; /* the term k = i */
    for (int q = nb->start[i]; q < nb->start[i + 1]; q++) {
        int k = nb->idx[q];
        double u[3];
        mic(pos, L, i, k, u);
        double r = sqrt(sq3(u));
        if (r >= r_w) continue;
        double w = ora_ftrans(r, r_w - 1.0, r_w);
        wsum += w;
        gsum += g[(size_t)k * gs] * w;
    }
    *wbar = wsum;
    *d = gsum / wsum - d0;
}

/* Eq. (6) for a given per-atom g[n] (any indicator) on one periodic cell: wbar[n] and d[n]. */
int ora_descriptor(int n, const double *pos_in, const double *L, const double *g, double r_w, double d0,
                   double *wbar, double *d) {
    if (n <= 0 || !pos_in || !L || !g || !wbar || !d || !(r_w > 0.0)) return ORA_E_ARG;
    int rc = check_box(L, r_w);
    if (rc) return rc;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t nb;
    rc = build_csr(n, pos, L, r_w, &nb);
    if (!rc) {
        for (int i = 0; i < n; i++) descriptor_site(pos, L, &nb, i, g, 1, r_w, d0, wbar + i, d + i);
        csr_free(&nb);
    }
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Full AP evaluation                                                                            */
/* ------------------------------------------------------------------------------------------ */
/* aux columns per atom */
enum { AX_G, AX_D, AX_WBAR, AX_LAM, AX_DLAM, AX_EF, AX_EP, AX_ET, AX_W, AX_XIP, AX_PHI2, AX_NNB };

/*
 * E_AP = sum_i [lam_i E^EAM_i + (1 - lam_i) E^ACE_i]            Eq. (4)
 * F    = -grad E_AP in the pair form (S5)-(S6):
 *   EAM family   F_i += sum_k (lam_i f^EAM_ki - lam_k f^EAM_ik)          (S12)
 *   ACE family   F_i += sum_k ((1-lam_i) f^ACE_ki - (1-lam_k) f^ACE_ik)  (S14)
 *   weight part  F_i += sum_j (E~_i (g_j - d_i - d0) w'(r_ij) rhat_ij
 *                              - E~_j (g_i - d_j - d0) w'(r_ji) rhat_ji)  (S19)-(S21)
 *   CSP part     F_i += sum_j W_j grad_i g_j, W_j = sum_k E~_k w(r_kj)     (S24)-(S27)
 *                (learned indicator: the same sum with grad_i g_j through the network, (S16))
 * with E~_k = (E^p_k - E^f_k) lam'_k / wbar_k                                (S17)
 * and the descriptor d_k = sum_j g_j w(r_kj) / wbar_k - d0, wbar_k = sum_j w(r_kj), where
 * both sums include j = k with w(0) = 1                                      Eq. (6)
 * Readings: r_ab = r_a - r_b, rhat_ij = (r_i - r_j)/|r_i - r_j|; the general descriptor
 * derivative uses (g_j - d_k - d0), which is the printed (g_j - d_k) when d0 = 0.
 *
 * eam_p  = {A, beta, c0, c1, c2, rc};  sw_p = {d_lo, d_hi, r_w, d0}
 * lam_mode: -1 computed from Eq. (2); 0 -> lam == 0 (pure ACE); 1 -> lam == 1 (pure EAM);
 *           lam' = 0 whenever lam is forced.
 * skip:     0 evaluates ACE on every atom; 1 only where lam < 1 (the skipped terms are exact
 *           zeros); 2 never (E^p = 0: switching quantities only, used for calibration).
 * no_gradlam: 1 drops the grad-lambda families (the non-conservative comparison force).
 * Outputs: E_tot[1], E_atom[n], F[n][3], virial[9] (W_ab = -sum_e (dE/du_e)_a (u_e)_b),
 *          aux[n][AUX_W] (may be NULL), Ffam[4][n][3] (may be NULL).
 */
/* indicator: 0 = CSP^list with the list csp; 1 = the learned indicator with parameters mlp_P
 * (MLP_NP doubles) on features inside mlp_rc (csp unused).
 * lam_fix: NULL, or per atom -1 (lambda from Eq. (2)) or 0 / 1: a constant switching parameter with
 *          dlambda/dd = 0 (App. B, the paragraph after (B4)); used only when lambda is computed.
 * force_mix: 1 replaces the conservative force by force mixing, Eq. (3):
 *          F_i = lambda_i F^f_i + (1 - lambda_i) F^p_i with the complete EAM and ACE forces
 *          F^f_i = -grad_i sum_k E^f_k and F^p_i = -grad_i sum_k E^p_k; E_atom stays Eq. (4), there
 *          are no grad-lambda terms, and the virial is not defined (returned as zeros). With skip = 1
 *          ACE runs on the atoms with lambda < 1 and every atom within the ACE cutoff of one. */
int ora_eval_full(int n, const double *pos_in, const double *L, const double *eam_p, int n_max, int l_max,
                  double ace_rc, int n_funcs, const int *func, const double *c, const double *b_dens, double emb_A,
                  double E0, const double *sw_p, int n_csp, const int *csp, int lam_mode, int skip, int no_gradlam,
                  double *E_tot, double *E_atom, double *F, double *virial, double *aux, double *Ffam, int indicator,
                  const double *mlp_P, double mlp_rc, int force_mix, const int *lam_fix) {
    if (n <= 0 || !pos_in || !L || !eam_p || !sw_p || !E_tot || !E_atom || !F || !virial) return ORA_E_ARG;
    if (lam_fix)
        for (int i = 0; i < n; i++)
            if (lam_fix[i] < -1 || lam_fix[i] > 1) return ORA_E_ARG;
    if (force_mix) no_gradlam = 1;
    if (n_max > 32 || l_max > 12) return ORA_E_ARG;
    if (indicator != 0 && (indicator != 1 || !mlp_P || !(mlp_rc > 0.0))) return ORA_E_ARG;
    double rc_eam = eam_p[5] > eam_p[6] ? eam_p[5] : eam_p[6];
    double d_lo = sw_p[0], d_hi = sw_p[1], r_w = sw_p[2], d0 = sw_p[3];
    int need_sw = (lam_mode < 0);
    double rmax = rc_eam > ace_rc ? rc_eam : ace_rc;
    if (need_sw && r_w > rmax) rmax = r_w;
    if (need_sw && indicator == 1 && mlp_rc > rmax) rmax = mlp_rc;
    int rc = check_box(L, rmax);
    if (rc) return rc;
    if (need_sw && indicator == 0) {
        if (n_csp != 8 && n_csp != 12) return ORA_E_CSP;
        for (long q = 0; q < (long)n * n_csp; q++)
            if (csp[q] < 0 || csp[q] >= n) return ORA_E_CSP;
    }
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t nb;
    rc = build_csr(n, pos, L, rmax, &nb);
    if (rc) {
        free(pos);
        return rc;
    }
    double *ax = (double *)calloc((size_t)n * AUX_W, sizeof(double));
    double *fam = (double *)calloc((size_t)4 * n * 3, sizeof(double));
    double vir[9] = {0};
    ace_t ace = {n_max, l_max, n_funcs, ace_rc, func, c, b_dens, emb_A, E0, NULL};
    ace_build_3j(&ace);
#define AX(i, k) ax[(size_t)(i) * AUX_W + (k)]

    /* 1. switching: g (B3), descriptor Eq. (6), lambda Eq. (2) */
    if (need_sw && indicator == 0) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) AX(i, AX_G) = csp_value(pos, L, i, n_csp, csp);
    } else if (need_sw) {
        for (int i = 0; i < n; i++)
            if (nb.start[i + 1] - nb.start[i] > 4096) rc = ORA_E_NBR;
#pragma omp parallel if (!rc)
        {
            double *u = (double *)malloc(sizeof(double) * 3 * 4096);
#pragma omp for schedule(static)
            for (int i = 0; i < n; i++) {
                if (rc) continue;
                int nn = nb.start[i + 1] - nb.start[i];
                for (int q = 0; q < nn; q++) mic(pos, L, i, nb.idx[nb.start[i] + q], u + 3 * q);
                double qf[MLP_NQ], o, g;
                mlp_site_features(nn, u, mlp_rc, qf, NULL);
                mlp_forward1(mlp_P, qf, &o, &g, NULL);
                AX(i, AX_G) = g;
            }
            free(u);
        }
    }
    if (need_sw) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++) {
            descriptor_site(pos, L, &nb, i, ax + AX_G, AUX_W, r_w, d0, &AX(i, AX_WBAR), &AX(i, AX_D));
            if (lam_fix && lam_fix[i] >= 0) {
                /* an atom with a constant switching parameter (App. B, after (B4)): lambda is 0 or 1
                 * for the whole run and not a function of d_i, so dlambda/dd = 0 */
                AX(i, AX_LAM) = (double)lam_fix[i];
                AX(i, AX_DLAM) = 0.0;
            } else {
                AX(i, AX_LAM) = ora_ftrans(AX(i, AX_D), d_lo, d_hi);
                AX(i, AX_DLAM) = ora_ftrans_d(AX(i, AX_D), d_lo, d_hi);
            }
        }
    } else {
        for (int i = 0; i < n; i++) {
            AX(i, AX_LAM) = lam_mode ? 1.0 : 0.0;
            AX(i, AX_DLAM) = 0.0;
            AX(i, AX_WBAR) = 1.0;
        }
    }

    /* 2. EAM energies (B1) for every atom */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        double z = 0.0, pair = 0.0;
        int cnt = 0;
        for (int q = nb.start[i]; q < nb.start[i + 1]; q++) {
            double u[3];
            mic(pos, L, i, nb.idx[q], u);
            double r = sqrt(sq3(u));
            if (r >= rc_eam) continue;
            double zz, dz, ph, dph;
            eam_pair(eam_p, r, &zz, &dz, &ph, &dph);
            z += zz;
            pair += ph;
            cnt++;
        }
        double xi, dxi;
        embed(eam_p[0], z, &xi, &dxi);
        AX(i, AX_EF) = xi + 0.5 * pair;
        AX(i, AX_XIP) = dxi;
        AX(i, AX_NNB) = cnt;
    }

    /* 3. ACE energies and pair gradients f^ACE_ki = grad_k E^ACE_i, stored per neighbour slot */
    int total_slots = nb.start[n];
    double *face = (double *)calloc((size_t)total_slots * 3 + 3, sizeof(double));
    char *do_ace = (char *)calloc((size_t)n, 1);
    for (int i = 0; i < n; i++) do_ace[i] = skip == 2 ? 0 : (skip ? (AX(i, AX_LAM) < 1.0) : 1);
    if (force_mix && skip == 1) {
        /* Eq. (3) takes the complete F^p_i of each atom with lambda_i < 1, which needs E^p_k of every
         * atom k within the ACE cutoff of i as well */
        for (int i = 0; i < n; i++) {
            if (!(AX(i, AX_LAM) < 1.0)) continue;
            for (int q = nb.start[i]; q < nb.start[i + 1]; q++) {
                double u[3];
                mic(pos, L, i, nb.idx[q], u);
                if (sqrt(sq3(u)) < ace_rc) do_ace[nb.idx[q]] = 1;
            }
        }
    }
    for (int i = 0; i < n; i++)
        if (nb.start[i + 1] - nb.start[i] > 4096) rc = ORA_E_NBR;
#pragma omp parallel if (!rc)
    {
        double *u = (double *)malloc(sizeof(double) * 3 * 4096);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; i++) {
            if (!do_ace[i] || rc) continue;
            int nn = nb.start[i + 1] - nb.start[i];
            for (int q = 0; q < nn; q++) mic(pos, L, i, nb.idx[nb.start[i] + q], u + 3 * q);
            double e, phi2;
            ace_site(&ace, nn, u, &e, face + 3 * (size_t)nb.start[i], NULL, NULL, &phi2);
            AX(i, AX_EP) = e;
            AX(i, AX_PHI2) = phi2;
        }
        free(u);
    }

    /* 4. AP energies Eq. (4) and grad-lambda scalars (S17), W_j of (S25) */
    double etot = 0.0;
    for (int i = 0; i < n; i++) {
        double lam = AX(i, AX_LAM);
        E_atom[i] = lam * AX(i, AX_EF) + (1.0 - lam) * AX(i, AX_EP);
        etot += E_atom[i];
        AX(i, AX_ET) = (AX(i, AX_EP) - AX(i, AX_EF)) * AX(i, AX_DLAM) / AX(i, AX_WBAR);
    }
    if (need_sw) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < n; j++) {
            double Wj = AX(j, AX_ET); /* k = j, w(0) = 1 */
            for (int q = nb.start[j]; q < nb.start[j + 1]; q++) {
                int k = nb.idx[q];
                double u[3];
                mic(pos, L, j, k, u);
                double r = sqrt(sq3(u));
                if (r >= r_w) continue;
                Wj += AX(k, AX_ET) * ora_ftrans(r, r_w - 1.0, r_w);
            }
            AX(j, AX_W) = Wj;
        }
    }

    /* 5. forces, family by family, in scatter form over ordered pairs (i, k) */
    double *fE = fam, *fA = fam + 3 * (size_t)n, *fW = fam + 6 * (size_t)n, *fC = fam + 9 * (size_t)n;
    if (force_mix) {
        /* Eq. (3): the complete force of each model, F^f_i = sum_k (f^EAM_ki - f^EAM_ik) and
         * F^p_i = sum_k (f^ACE_ki - f^ACE_ik), then weighted by lambda_i and 1 - lambda_i per atom */
        double *Ff = (double *)calloc((size_t)3 * n, sizeof(double));
        double *Fp = (double *)calloc((size_t)3 * n, sizeof(double));
        for (int i = 0; i < n; i++) {
            for (int q = nb.start[i]; q < nb.start[i + 1]; q++) {
                int k = nb.idx[q];
                double u[3];
                mic(pos, L, i, k, u);
                double r = sqrt(sq3(u));
                if (r < rc_eam) {
                    double zz, dz, ph, dph;
                    eam_pair(eam_p, r, &zz, &dz, &ph, &dph);
                    double s = AX(i, AX_XIP) * dz + 0.5 * dph;
                    for (int a = 0; a < 3; a++) {
                        Ff[3 * i + a] += s * u[a] / r;
                        Ff[3 * k + a] -= s * u[a] / r;
                    }
                }
                if (do_ace[i] && r < ace_rc) {
                    const double *f = face + 3 * (size_t)q;
                    for (int a = 0; a < 3; a++) {
                        Fp[3 * i + a] += f[a];
                        Fp[3 * k + a] -= f[a];
                    }
                }
            }
        }
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) {
                fE[3 * i + a] = AX(i, AX_LAM) * Ff[3 * i + a];
                fA[3 * i + a] = (1.0 - AX(i, AX_LAM)) * Fp[3 * i + a];
            }
        free(Ff);
        free(Fp);
    }
    for (int i = 0; i < n && !force_mix; i++) {
        double lam_i = AX(i, AX_LAM);
        for (int q = nb.start[i]; q < nb.start[i + 1]; q++) {
            int k = nb.idx[q];
            double u[3];
            mic(pos, L, i, k, u); /* u = r_k - r_i */
            double r = sqrt(sq3(u));
            /* EAM: f_ki = (xi'(zeta_i) zeta'(r) + Phi'(r)/2) rhat_ki, rhat_ki = u/r   (S11) */
            if (r < rc_eam && lam_i != 0.0) {
                double zz, dz, ph, dph;
                eam_pair(eam_p, r, &zz, &dz, &ph, &dph);
                double s = AX(i, AX_XIP) * dz + 0.5 * dph;
                for (int a = 0; a < 3; a++) {
                    double f = lam_i * s * u[a] / r;
                    fE[3 * i + a] += f;
                    fE[3 * k + a] -= f;
                }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) vir[3 * a + b] -= lam_i * s * u[a] / r * u[b];
            }
            /* ACE: (1 - lam_i) f^ACE_ki added to i, subtracted from k   (S14) */
            if (do_ace[i] && r < ace_rc) {
                const double *f = face + 3 * (size_t)q;
                double wgt = 1.0 - lam_i;
                for (int a = 0; a < 3; a++) {
                    fA[3 * i + a] += wgt * f[a];
                    fA[3 * k + a] -= wgt * f[a];
                }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) vir[3 * a + b] -= wgt * f[a] * u[b];
            }
            /* weight part of grad-lambda: grad_r_k of d_i through w(|r_k - r_i|)   (S18)-(S21) */
            if (need_sw && !no_gradlam && r < r_w && AX(i, AX_ET) != 0.0) {
                double dw = ora_ftrans_d(r, r_w - 1.0, r_w);
                double s = AX(i, AX_ET) * (AX(k, AX_G) - AX(i, AX_D) - d0) * dw;
                /* F_i += s rhat_ik, rhat_ik = (r_i - r_k)/r = -u/r ; F_k -= same */
                for (int a = 0; a < 3; a++) {
                    double f = -s * u[a] / r;
                    fW[3 * i + a] += f;
                    fW[3 * k + a] -= f;
                }
                /* dE/du = -s u/r  => W_ab -= (dE/du)_a u_b */
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) vir[3 * a + b] += s * u[a] / r * u[b];
            }
        }
    }
    /* CSP part: grad_i g_j = 2 sum_l Theta_jl (r_jl + r_j,opp(l)) (delta_ij - delta_il)   (S24) */
    if (need_sw && !no_gradlam && indicator == 0) {
        for (int j = 0; j < n; j++) {
            double Wj = AX(j, AX_W);
            if (Wj == 0.0) continue;
            for (int t = 0; t < n_csp; t++) {
                int l = csp[(size_t)j * n_csp + t];
                int o = csp[(size_t)j * n_csp + (t ^ 1)];
                double ul[3], uo[3];
                mic(pos, L, j, l, ul);
                mic(pos, L, j, o, uo);
                /* r_jl + r_jo = -(u_jl + u_jo) */
                for (int a = 0; a < 3; a++) {
                    double v = -(ul[a] + uo[a]);
                    fC[3 * j + a] += 2.0 * Wj * v;
                    fC[3 * l + a] -= 2.0 * Wj * v;
                }
                /* dE/du_jl = -2 W_j (u_jl + u_jo): every list entry is one edge u_jl */
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) vir[3 * a + b] += 2.0 * Wj * (ul[a] + uo[a]) * ul[b];
            }
        }
    }
    /* learned indicator: grad_i g_j through the features, h_jk = d g_j / d u_jk:
     * F_j -= W_j sum_k h_jk, F_k += W_j h_jk; the edge u_jk carries dE/du = -W_j h_jk */
    if (need_sw && !no_gradlam && indicator == 1) {
        double *u = (double *)malloc(sizeof(double) * 3 * 4096);
        double *dq = (double *)malloc(sizeof(double) * 3 * MLP_NQ * 4096);
        for (int j = 0; j < n && !rc; j++) {
            double Wj = AX(j, AX_W);
            if (Wj == 0.0) continue;
            int nn = nb.start[j + 1] - nb.start[j];
            for (int q = 0; q < nn; q++) mic(pos, L, j, nb.idx[nb.start[j] + q], u + 3 * q);
            double qf[MLP_NQ], o, g, dgdq[MLP_NQ];
            mlp_site_features(nn, u, mlp_rc, qf, dq);
            mlp_forward1(mlp_P, qf, &o, &g, dgdq);
            for (int q = 0; q < nn; q++) {
                int k = nb.idx[nb.start[j] + q];
                double h[3] = {0.0, 0.0, 0.0};
                for (int f = 0; f < MLP_NQ; f++)
                    for (int a = 0; a < 3; a++) h[a] += dgdq[f] * dq[((size_t)q * MLP_NQ + f) * 3 + a];
                for (int a = 0; a < 3; a++) {
                    fC[3 * j + a] -= Wj * h[a];
                    fC[3 * k + a] += Wj * h[a];
                }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) vir[3 * a + b] += Wj * h[a] * u[3 * q + b];
            }
        }
        free(dq);
        free(u);
    }
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++)
            F[3 * i + a] = fE[3 * i + a] + fA[3 * i + a] + fW[3 * i + a] + fC[3 * i + a];
    *E_tot = etot;
    memcpy(virial, vir, sizeof(vir));
    if (rc) *E_tot = NAN;
    if (aux) memcpy(aux, ax, sizeof(double) * (size_t)n * AUX_W);
    if (Ffam) memcpy(Ffam, fam, sizeof(double) * 12 * (size_t)n);
#undef AX
    free(face);
    free(do_ace);
    free(fam);
    free(ax);
    free(ace.w3j);
    csr_free(&nb);
    free(pos);
    return rc;
}

int ora_eval_ind(int n, const double *pos_in, const double *L, const double *eam_p, int n_max, int l_max,
                 double ace_rc, int n_funcs, const int *func, const double *c, const double *b_dens, double emb_A,
                 double E0, const double *sw_p, int n_csp, const int *csp, int lam_mode, int skip, int no_gradlam,
                 double *E_tot, double *E_atom, double *F, double *virial, double *aux, double *Ffam, int indicator,
                 const double *mlp_P, double mlp_rc) {
    return ora_eval_full(n, pos_in, L, eam_p, n_max, l_max, ace_rc, n_funcs, func, c, b_dens, emb_A, E0, sw_p, n_csp,
                         csp, lam_mode, skip, no_gradlam, E_tot, E_atom, F, virial, aux, Ffam, indicator, mlp_P,
                         mlp_rc, 0, NULL);
}

int ora_eval(int n, const double *pos_in, const double *L, const double *eam_p, int n_max, int l_max, double ace_rc,
             int n_funcs, const int *func, const double *c, const double *b_dens, double emb_A, double E0,
             const double *sw_p, int n_csp, const int *csp, int lam_mode, int skip, int no_gradlam, double *E_tot,
             double *E_atom, double *F, double *virial, double *aux, double *Ffam) {
    return ora_eval_ind(n, pos_in, L, eam_p, n_max, l_max, ace_rc, n_funcs, func, c, b_dens, emb_A, E0, sw_p, n_csp,
                        csp, lam_mode, skip, no_gradlam, E_tot, E_atom, F, virial, aux, Ffam, 0, NULL, 0.0);
}

/* Gradient of E_AP with respect to the ACE coefficients:
 *   dE/dc_nu  = sum_i (1 - lam_i) B_i,nu
 *   dE/db_n   = sum_i (1 - lam_i) xi'(phi2_i) sqrt(4 pi) A_i,n00
 * weight[i] = 1 - lam_i (NULL -> 1). Positions are one periodic cell; outputs dEdc[n_funcs],
 * dEdb[n_max] and the site energies E_atom[n] (without E0; may be NULL). */
int ora_ace_coeff_grad(int n, const double *pos_in, const double *L, int n_max, int l_max, double rc, int n_funcs,
                       const int *func, const double *c, const double *b_dens, double emb_A, const double *weight,
                       double *dEdc, double *dEdb, double *E_atom) {
    int rcode = check_box(L, rc);
    if (rcode) return rcode;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t nb;
    build_csr(n, pos, L, rc, &nb);
    ace_t ace = {n_max, l_max, n_funcs, rc, func, c, b_dens, emb_A, 0.0, NULL};
    ace_build_3j(&ace);
    int nlm = ace_nlm(&ace);
    double *acc = (double *)calloc((size_t)n * (n_funcs + n_max), sizeof(double));
#pragma omp parallel
    {
        double *u = (double *)malloc(sizeof(double) * 3 * 4096);
        double complex *A = (double complex *)malloc(sizeof(double complex) * (size_t)n_max * nlm);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; i++) {
            int nn = nb.start[i + 1] - nb.start[i];
            if (nn > 4096) nn = 4096; /* cannot happen below rc = L/2 for condensed matter */
            for (int q = 0; q < nn; q++) mic(pos, L, i, nb.idx[nb.start[i] + q], u + 3 * q);
            double e, phi2;
            double *Bi = acc + (size_t)i * (n_funcs + n_max);
            ace_site(&ace, nn, u, &e, NULL, Bi, A, &phi2);
            if (E_atom) E_atom[i] = e;
            double fe, dfe;
            embed(emb_A, phi2, &fe, &dfe);
            for (int m = 0; m < n_max; m++) Bi[n_funcs + m] = dfe * sqrt(4.0 * PI) * creal(A[m * nlm]);
        }
        free(u);
        free(A);
    }
    for (int f = 0; f < n_funcs + n_max; f++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += (weight ? weight[i] : 1.0) * acc[(size_t)i * (n_funcs + n_max) + f];
        if (f < n_funcs)
            dEdc[f] = s;
        else
            dEdb[f - n_funcs] = s;
    }
    free(acc);
    free(ace.w3j);
    csr_free(&nb);
    free(pos);
    return ORA_OK;
}

/* Tangents of one site along a motion of its neighbour vectors: every u_j moves with the velocity udot_j.
 * Product rule on the definitions of ace_site:
 *   Adot_{nlm} = sum_j grad_u [g_n(|u|) Y_l^m(u/|u|)] at u_j . udot_j
 *   Bdot (order 1) = Adot_{n00};  order 2 = sum_m (-1)^m (Adot_{n1lm} A_{n2l-m} + A_{n1lm} Adot_{n2l-m})
 *   order 3 = sum (l1 l2 l3; m1 m2 m3) (Adot1 A2 A3 + A1 Adot2 A3 + A1 A2 Adot3)
 *   the density term: d/dt [xi'(phi2) sqrt(4 pi) A_{n00}]
 *                    = xi''(phi2) phi2dot sqrt(4 pi) A_{n00} + xi'(phi2) sqrt(4 pi) Adot_{n00},
 *   phi2dot = sum_n b_n sqrt(4 pi) Adot_{n00}, xi = -emb_A sqrt (xi' = -emb_A / (2 sqrt), xi'' = emb_A / (4 phi2^1.5)).
 * Outputs: Bdot[n_funcs] (real parts), ddb[n_max] the density-term tangents. */
static void ace_site_tangent(const ace_t *p, int nn, const double *u, const double *udot, double *Bdot,
                             double *ddb) {
    int nmax = p->n_max, nlm = ace_nlm(p), lmax = p->l_max;
    double complex *A = (double complex *)calloc((size_t)nmax * nlm, sizeof(double complex));
    double complex *Ad = (double complex *)calloc((size_t)nmax * nlm, sizeof(double complex));
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)nlm);
    double complex *dY = (double complex *)malloc(sizeof(double complex) * 3 * (size_t)nlm);
    double g[32], dg[32];
    for (int j = 0; j < nn; j++) {
        const double *uj = u + 3 * j, *vj = udot + 3 * j;
        double r = sqrt(sq3(uj));
        if (r >= p->rc) continue;
        ora_radial(nmax, p->rc, r, g, dg);
        ora_ylm_c(lmax, uj, Y, dY);
        double rdot = (uj[0] * vj[0] + uj[1] * vj[1] + uj[2] * vj[2]) / r; /* d|u|/dt */
        for (int t = 0; t < nlm; t++) {
            double complex ydot = dY[3 * t] * vj[0] + dY[3 * t + 1] * vj[1] + dY[3 * t + 2] * vj[2];
            for (int n = 0; n < nmax; n++) {
                A[n * nlm + t] += g[n] * Y[t];
                Ad[n * nlm + t] += dg[n] * rdot * Y[t] + g[n] * ydot;
            }
        }
    }
#define AA(n, l, m) A[(n) * nlm + (l) * (l) + (l) + (m)]
#define AD(n, l, m) Ad[(n) * nlm + (l) * (l) + (l) + (m)]
    for (int f = 0; f < p->n_funcs; f++) {
        const int *q = p->func + 6 * f;
        double complex bd = 0.0;
        if (q[2] < 0) {
            bd = AD(q[0], 0, 0);
        } else if (q[4] < 0) {
            int n1 = q[0], l = q[1], n2 = q[2];
            for (int m = -l; m <= l; m++) {
                double sg = (m & 1) ? -1.0 : 1.0;
                bd += sg * (AD(n1, l, m) * AA(n2, l, -m) + AA(n1, l, m) * AD(n2, l, -m));
            }
        } else {
            int n1 = q[0], l1 = q[1], n2 = q[2], l2 = q[3], n3 = q[4], l3 = q[5];
            for (int m1 = -l1; m1 <= l1; m1++)
                for (int m2 = -l2; m2 <= l2; m2++) {
                    int m3 = -m1 - m2;
                    if (m3 < -l3 || m3 > l3) continue;
                    double wv = w3(p, l1, l2, l3, m1, m2);
                    if (wv == 0.0) continue;
                    bd += wv * (AD(n1, l1, m1) * AA(n2, l2, m2) * AA(n3, l3, m3) +
                                AA(n1, l1, m1) * AD(n2, l2, m2) * AA(n3, l3, m3) +
                                AA(n1, l1, m1) * AA(n2, l2, m2) * AD(n3, l3, m3));
                }
        }
        Bdot[f] = creal(bd);
    }
    double phi2 = 0.0, phi2d = 0.0, s4pi = sqrt(4.0 * PI);
    for (int n = 0; n < nmax; n++) {
        phi2 += p->b_dens[n] * s4pi * creal(AA(n, 0, 0));
        phi2d += p->b_dens[n] * s4pi * creal(AD(n, 0, 0));
    }
    double d1 = 0.0, d2 = 0.0; /* xi'(phi2), xi''(phi2) */
    if (phi2 > 0.0) {
        d1 = -0.5 * p->emb_A / sqrt(phi2);
        d2 = 0.25 * p->emb_A / (phi2 * sqrt(phi2));
    }
    for (int n = 0; n < nmax; n++)
        ddb[n] = d2 * phi2d * s4pi * creal(AA(n, 0, 0)) + d1 * s4pi * creal(AD(n, 0, 0));
#undef AA
#undef AD
    free(A);
    free(Ad);
    free(Y);
    free(dY);
}

/* Vector-Jacobian product of the ACE forces with respect to the ACE coefficients, one periodic cell with
 * constant per-atom weights w_i (the ACE weight 1 - lambda_i of Eq. (4); NULL = 1):
 *   E = sum_i w_i E^ACE_i,  F_k = -dE/dr_k,  L = sum_k G_k . F_k
 *   dL/dc_nu = -sum_i w_i Bdot_i,nu,  dL/db_n = -sum_i w_i ddb_i,n
 * with the tangents of ace_site_tangent for the motion r_k -> r_k + t G_k, i.e. udot_ij = G_j - G_i
 * (d/dc of F = -grad E is minus the gradient of dE/dc = sum_i w_i B_i). G is AoS [n][3]. */
int ora_ace_force_vjp(int n, const double *pos_in, const double *L, int n_max, int l_max, double rc, int n_funcs,
                      const int *func, const double *c, const double *b_dens, double emb_A, const double *weight,
                      const double *G, double *dLdc, double *dLdb) {
    int rcode = check_box(L, rc);
    if (rcode) return rcode;
    double *pos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(pos, pos_in, sizeof(double) * 3 * (size_t)n);
    ora_wrap(n, pos, L);
    csr_t nb;
    build_csr(n, pos, L, rc, &nb);
    ace_t ace = {n_max, l_max, n_funcs, rc, func, c, b_dens, emb_A, 0.0, NULL};
    ace_build_3j(&ace);
    double *acc = (double *)calloc((size_t)n * (n_funcs + n_max), sizeof(double));
#pragma omp parallel
    {
        double *u = (double *)malloc(sizeof(double) * 3 * 4096);
        double *ud = (double *)malloc(sizeof(double) * 3 * 4096);
#pragma omp for schedule(dynamic, 4)
        for (int i = 0; i < n; i++) {
            int nn = nb.start[i + 1] - nb.start[i];
            if (nn > 4096) nn = 4096; /* cannot happen below rc = L/2 for condensed matter */
            for (int q = 0; q < nn; q++) {
                int j = nb.idx[nb.start[i] + q];
                mic(pos, L, i, j, u + 3 * q);
                for (int a = 0; a < 3; a++) ud[3 * q + a] = G[3 * j + a] - G[3 * i + a];
            }
            double *row = acc + (size_t)i * (n_funcs + n_max);
            ace_site_tangent(&ace, nn, u, ud, row, row + n_funcs);
        }
        free(u);
        free(ud);
    }
    for (int f = 0; f < n_funcs + n_max; f++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s -= (weight ? weight[i] : 1.0) * acc[(size_t)i * (n_funcs + n_max) + f];
        if (f < n_funcs)
            dLdc[f] = s;
        else
            dLdb[f - n_funcs] = s;
    }
    free(acc);
    free(ace.w3j);
    csr_free(&nb);
    free(pos);
    return ORA_OK;
}

/* Velocity Verlet, NVE, in FP64 (metal units; F/m converted with 9648.533212):
 *   v += dt/2 F/m;  x += dt v;  wrap;  F = F(x);  v += dt/2 F/m.
 * thermo[s] = {E_pot, E_kin, E_tot, P_x, P_y, P_z} after step s. F must hold F(x) on entry. */
/* force_mix and lam_fix as in ora_eval_full. */
int ora_vv_full(int n, double *pos, double *vel, double *F, double mass, double dt, int n_steps, const double *L,
                const double *eam_p, int n_max, int l_max, double ace_rc, int n_funcs, const int *func, const double *c,
                const double *b_dens, double emb_A, double E0, const double *sw_p, int n_csp, const int *csp,
                int lam_mode, double *thermo, int force_mix, const int *lam_fix) {
    double *Ea = (double *)malloc(sizeof(double) * (size_t)n);
    double vir[9], etot = 0.0;
    int rc = ORA_OK;
    for (int s = 0; s < n_steps && !rc; s++) {
        for (int i = 0; i < 3 * n; i++) vel[i] += 0.5 * dt * F[i] / mass * CONV;
        for (int i = 0; i < 3 * n; i++) pos[i] += dt * vel[i];
        ora_wrap(n, pos, L);
        rc = ora_eval_full(n, pos, L, eam_p, n_max, l_max, ace_rc, n_funcs, func, c, b_dens, emb_A, E0, sw_p, n_csp,
                           csp, lam_mode, 1, 0, &etot, Ea, F, vir, NULL, NULL, 0, NULL, 0.0, force_mix, lam_fix);
        for (int i = 0; i < 3 * n; i++) vel[i] += 0.5 * dt * F[i] / mass * CONV;
        double ek = 0.0, P[3] = {0, 0, 0};
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) {
                ek += 0.5 * mass * vel[3 * i + a] * vel[3 * i + a] / CONV;
                P[a] += mass * vel[3 * i + a];
            }
        double *t = thermo + 6 * (size_t)s;
        t[0] = etot;
        t[1] = ek;
        t[2] = etot + ek;
        t[3] = P[0];
        t[4] = P[1];
        t[5] = P[2];
    }
    free(Ea);
    return rc;
}

int ora_vv(int n, double *pos, double *vel, double *F, double mass, double dt, int n_steps, const double *L,
           const double *eam_p, int n_max, int l_max, double ace_rc, int n_funcs, const int *func, const double *c,
           const double *b_dens, double emb_A, double E0, const double *sw_p, int n_csp, const int *csp,
           int lam_mode, double *thermo) {
    return ora_vv_full(n, pos, vel, F, mass, dt, n_steps, L, eam_p, n_max, l_max, ace_rc, n_funcs, func, c, b_dens,
                       emb_A, E0, sw_p, n_csp, csp, lam_mode, thermo, 0, NULL);
}
