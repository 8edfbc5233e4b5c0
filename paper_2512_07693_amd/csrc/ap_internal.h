// Library-internal declarations of the MI355X adaptive-precision EAM/ACE library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "ap.h"

namespace ap {

constexpr int kBlock = 256;      // threads per workgroup of the per-atom kernels (4 wavefronts)
constexpr int kAceMaxValid = 128; // neighbours within the ACE cutoff held per site in LDS
constexpr int kLanesPerAtom = 8;  // lanes that share one atom's neighbour loop in the per-atom passes
constexpr int kDensLanes = 4;     // the same in the density pass (its per-workgroup counts cover kBlock / 4 atoms)
constexpr int kForceLanes = 4;    // the same for the force assembly
// workgroups of the force kernel, each writing one row of the per-block partial sums
// Above this many atoms the one-kernel compaction (each workgroup sums all the chunk counts before it)
// gives way to count, scan and scatter.
constexpr int kCountedCompactMax = 1 << 18;
inline int force_blocks(int n) { return (int)(((long long)n * kForceLanes + kBlock - 1) / kBlock); }
constexpr double kConv = 9648.533212;  // eV / (A u) in A / ps^2
constexpr double kPi = 3.14159265358979323846;

// Error bits raised by kernels in ctx->d_flags[1].
enum : int {
    kErrOverflow = 1,
    kErrNonFinite = 2,
    kErrCsp = 4,
    kErrAceNbr = 8,
    kErrDensity = 16,
    kErrAsym = 32,
    kErrLamFix = 64
};

// Block b of nb runs on XCD (b % 8); giving each XCD a contiguous range of atoms keeps the
// neighbour gathers of one XCD inside its own L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = (nb + 7) / 8;
    const int x = b % 8, q = b / 8;
    const int full = nb - (per - 1) * 8;  // XCDs that get `per` blocks (the rest get per-1)
    const int start = x < full ? x * per : full * per + (x - full) * (per - 1);
    return start + q;
}

__device__ __forceinline__ double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
    double y = x - L * floor(x / L);
    if (y >= L) y = 0.0;
    return y;
}

__device__ __forceinline__ double min_image(double d, double L) {
#pragma clang fp contract(off)
    return d - L * rint(d / L);
}

// One thermo row of velocity Verlet from the force pass's per-block partial sums (column-major, nbf
// blocks): the potential energy (column 0), the kinetic energy and momentum after the second half-kick
// (columns 10-13), then |S| and the rebuild flag given by the caller. Run by one whole workgroup of kBlock
// threads, so that every row is summed in the same order.
__device__ inline void thermo_row_block(const double *__restrict__ partials, int nbf, int pstride, int S,
                                        int rebuild, int *flags, double *row) {
    __shared__ double sh[kBlock / 64][5];
    double t5[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nbf; b += kBlock) {
        t5[0] += partials[b];
        for (int q = 1; q < 5; q++) t5[q] += partials[(size_t)(9 + q) * pstride + b];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < 5; q++) {
        double x = t5[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[w][q] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[5] = {0, 0, 0, 0, 0};
        for (int k = 0; k < kBlock / 64; k++)
            for (int q = 0; q < 5; q++) s[q] += sh[k][q];
        if (!isfinite(s[0])) atomicOr(&flags[1], kErrNonFinite);
        row[0] = s[0];
        row[1] = s[1];
        row[2] = s[0] + s[1];
        for (int q = 0; q < 3; q++) row[3 + q] = s[2 + q];
        row[6] = (double)S;
        row[7] = (double)rebuild;
    }
}

// Minimum image of a difference of two wrapped coordinates (|d| < L): the value of min_image wherever
// |d| is not within rounding of L / 2 (never inside a cutoff below L / 2), without the division. The
// list build's distance test takes it too: within a cutoff below L / 2 both give the same bits, so the
// neighbour sets are those of min_image, and so does the per-step CSP value. The one-time CSP pair
// detection keeps min_image.
__device__ __forceinline__ double min_image_w(double d, double L) {
    const double h = 0.5 * L;
    return d > h ? d - L : (d < -h ? d + L : d);
}

// |u|^2 as the plain left-to-right sum of products, never fused: the neighbour test must give the
// same set as any IEEE implementation of the same expression.
__device__ __forceinline__ double norm2_nofma(double x, double y, double z) {
#pragma clang fp contract(off)
    return x * x + y * y + z * z;
}

// f_trans of Eq. (S1) and its derivative.
template <typename T>
__host__ __device__ __forceinline__ T ftrans(T x, T lo, T hi) {
    if (x <= lo) return T(1);
    if (x >= hi) return T(0);
    T y = (hi + lo - T(2) * x) / (hi - lo);
    T y2 = y * y;
    return T(0.5) + y * (T(0.9375) + y2 * (T(-0.625) + T(0.1875) * y2));
}
// The same with 1 / (hi - lo) given (the pair weight w(r) evaluates it per neighbour; for its unit
// window the product equals the quotient exactly).
template <typename T>
__host__ __device__ __forceinline__ T ftrans_i(T x, T lo, T hi, T inv) {
    if (x <= lo) return T(1);
    if (x >= hi) return T(0);
    T y = (hi + lo - T(2) * x) * inv;
    T y2 = y * y;
    return T(0.5) + y * (T(0.9375) + y2 * (T(-0.625) + T(0.1875) * y2));
}
template <typename T>
__host__ __device__ __forceinline__ T ftrans_d_i(T x, T lo, T hi, T inv) {
    if (x <= lo || x >= hi) return T(0);
    T y = (hi + lo - T(2) * x) * inv;
    T s = T(1) - y * y;
    return T(0.9375) * s * s * (T(-2) * inv);
}
template <typename T>
__host__ __device__ __forceinline__ T ftrans_d(T x, T lo, T hi) {
    if (x <= lo || x >= hi) return T(0);
    T y = (hi + lo - T(2) * x) / (hi - lo);
    T s = T(1) - y * y;
    return T(0.9375) * s * s * (T(-2) / (hi - lo));
}

struct AceTables {
    int n_max = 0, l_max = 0, n_funcs = 0, precision = AP_FP64;
    double rc = 0, emb_A = 0, E0 = 0;
    int nblk = 0;
    // device, element type double or float according to precision
    void *c1 = nullptr;   // [n_max]          coefficient of A_{n00}
    void *bd = nullptr;   // [n_max]          b_dens * sqrt(4 pi)
    double *c1d = nullptr, *bdd = nullptr;  // FP64 copies: the l = 0 two-body and density sums
    void *c2 = nullptr;   // [l_max+1][n][n]  symmetric order-2 matrix
    void *c3 = nullptr;   // [nblk][n][n][n]  order-3 coefficients of block (L, l1, l2)
    void *kval = nullptr; // coupling values, three orderings (by M, by m1, by m2)
    int *kidx = nullptr;  // packed (m1 + 8) | (m2 + 8) << 8 | (M + 8) << 16, same three orderings
    int *blk = nullptr;   // [nblk][kBlkInts] block descriptors
    int n0 = 0;           // leading L = 0 blocks; the parts of a split atom share out the blocks after them
    // the L = 0 blocks (0, l, l) in closed form: C0[l][n1][n2][n3] and their coupling kappa_l (null when
    // a block does not have the single-value diagonal form)
    void *c30 = nullptr, *kap0 = nullptr;
    int *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;  // coefficient-gradient lists (see ace_setup)
    int ng1 = 0, ng2 = 0;
    std::vector<int> h_blk;
    // gather map of ap_set_ace_coefficients: per element of c1, c2, c3, c30 (in that order) the function
    // (-1: none) and its factor; nmap = 0 when the basis cannot be updated that way
    int *cmap_f = nullptr;
    double *cmap_w = nullptr;
    int nmap = 0, n_c2 = 0, n_c3 = 0, n_c30 = 0;
};
// L, l1, l2, c3 offset, 3 x 14 coupling start offsets (by M, m1, m2), order-3 gradient list range
constexpr int kBlkInts = 48;

// Per-atom record read by the neighbour loops: four doubles in one 32-byte aligned slot, so that a
// gather of a neighbour's data is one pair of 16-byte loads instead of one load per quantity.
struct alignas(32) Rec4 {
    double x, y, z, w;
};

// A list-build candidate in cell order: its wrapped position rounded to FP32 and its index (16 bytes). The
// FP32 distance only sorts pairs into certainly inside, certainly outside and too close to call; the last
// are decided from the FP64 positions.
struct alignas(16) CandRec {
    float x, y, z;
    int j;
};

struct Geometry {
    double L[3];
    int nc[3];
    int ncell;
};

}  // namespace ap

struct ap_ctx {
    hipStream_t stream = nullptr;
    int n_cap = 0, max_nbr = 0;
    double skin = 0;
    std::string err;
    int device = 0;

    bool have_pot = false;
    ap_eam_params eam{};
    ap_switch_params sw{};
    ap::AceTables ace;

    // constant switching parameters (ap_set_lambda_fixed): [n_cap] -1 = computed, 0 / 1 = fixed
    int *lam_fix = nullptr;
    bool have_fix = false;

    // CSP pair list and its reverse (fixed at set-up)
    int csp_n = 0, n_csp = 0;
    int32_t *csp_t = nullptr;     // [n_csp][n] slot-major
    int32_t *rev_start = nullptr; // [n+1]
    int32_t *rev_code = nullptr;  // [n * n_csp]: j * 16 + t (atom j holds this atom in its slot t)

    // positions as used internally (wrapped), build-time positions, flags
    double *pos = nullptr;       // [3][n_cap]
    double *pos_build = nullptr; // [3][n_cap]
    int *d_flags = nullptr;      // [0] rebuild needed, [1] error bits, [2] n_precise, [3] rebuilt in step
    double list_r = -1;          // radius of the current list
    int list_n = -1;
    double list_box[3] = {0, 0, 0};

    // cell list
    int ncell_cap = 0;
    int ncell_cur = 0;  // cells of the geometry of the last list build
    int *cell_of = nullptr, *cell_cnt = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *cell_atoms = nullptr;
    ap::CandRec *cell_rec = nullptr;  // [n] the atoms in cell order (the list build's candidates)
    int *scan_tmp = nullptr;

    // neighbour list (slot-major)
    int32_t *nbr_cnt = nullptr, *nbr_idx = nullptr;
    int32_t *nbr_short = nullptr;  // [n] the first nbr_short[i] slots hold the neighbours inside max(r_rho, r_phi) + skin
    int *act = nullptr;            // [n] 1 if the atom or a neighbour has lambda < 1 (the force needs its full list)
    int *stamp = nullptr;          // [n] = stamp_gen when the atom is precise or in a precise atom's list
    // device counter of neighbour-list builds (raised where a build is committed), and per atom the slot
    // in each neighbour's list that holds it ([n][max_nbr], atom-major), valid while rstamp[i] equals the
    // counter: the ACE pair kernel searches a precise atom's reverse slots once per list
    int *list_gen = nullptr, *rslot = nullptr, *rstamp = nullptr;
    int stamp_gen = 0;             // evaluation counter of the stamps
    int *cmark = nullptr;          // [n] = stamp_gen when a CSP neighbour of the atom has W != 0
    // set by the velocity-Verlet loop around its force evaluations: the force pass then applies the
    // second half-kick v += kick_hdtm F (null: no kick)
    double *kick_vel = nullptr;
    double kick_hdtm = 0.0, kick_mass = 0.0;
    double *thermo_prev = nullptr;  // set by the same loop: the row the density pass fills for the last step
    double *drift_pos = nullptr;    // and the caller's positions, which the force pass drifts for the next step
    double drift_dt = 0.0;

    // gathered records: xg = {x, y, z, g}, xl = {x, y, z, lambda}, eb = {xi', g, d + d0, E~}
    ap::Rec4 *xg = nullptr, *xl = nullptr, *eb = nullptr;
    ap::Rec4 *xe = nullptr;  // [n] {x, y, z, xi'}: the EAM-only force gather
    // per-atom intermediates
    double *g = nullptr, *d = nullptr, *wbar = nullptr, *lam = nullptr, *dlam = nullptr;
    double *Ef = nullptr, *Ep = nullptr, *Et = nullptr, *W = nullptr, *xip = nullptr;
    int *sidx = nullptr, *slist = nullptr, *blk_cnt = nullptr, *mark = nullptr;
    int *chunk_cnt = nullptr;  // [ceil(n / (kBlock / kDensLanes))] counts of lambda < 1 from the density pass
    int *sid = nullptr;          // [n_cap] structure of each atom in a batch evaluation
    int *b_off = nullptr;        // [n_struct + 1] device copy of the batch offsets
    double *b_box = nullptr;     // [n_struct][3] device copy of the batch boxes
    int b_cap = 0;
    void *bval = nullptr;        // [n_cap][n_funcs + n_max] dE_i/dc and dE_i/db (batch gradients)
    size_t bval_bytes = 0;
    void *fpair = nullptr;       // [n_cap][max_nbr][3] ACE pair gradients (double or float)
    void *frev = nullptr;        // [3][max_nbr][n] the same pair terms at the neighbour's slot (k, j)
    void *gbuf = nullptr;        // ACE scratch of the S atoms: A, FP64 radial sums, two dE/dA parts, two energy parts
    size_t fpair_bytes = 0, gbuf_bytes = 0;
    // learned indicator
    bool have_mlp = false;
    double mlp_rc = 0;
    float *mlp_p = nullptr;      // [AP_MLP_NPARAMS]
    float *hpair = nullptr;      // [n_cap][max_nbr][3] W_j dg_j/du_jk of the atoms with W != 0
    float *hrev = nullptr;       // [3][max_nbr][n] the same terms at the neighbour's slot
    int *widx = nullptr, *wlist = nullptr;
    float *mlp_T = nullptr;      // training scratch [274][batch]
    int mlp_T_cap = 0;
    float *mlp_grad = nullptr, *mlp_m1 = nullptr, *mlp_m2 = nullptr;
    double *mlp_loss = nullptr;
    double *partials = nullptr;  // per-block partial sums, column-major [16][pstride]
    int pstride = 0;             // rows per column: the most blocks a per-atom or force launch has
    double *scalars = nullptr;   // [0] E_tot, [1..9] virial, [10] E_kin, [11..13] P

    // kernel timing with HIP events on the context stream (ap_set_profiling)
    bool prof_on = false;
    int prof_every = 1;      // ap_vv_step times the launches of every prof_every-th step
    bool prof_skip = false;  // set by ap_vv_step on the steps it does not time
    struct Pending {
        int label;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;
    std::vector<std::string> prof_names;
    std::vector<double> prof_ms;
    std::vector<long long> prof_cnt;
};

namespace ap {

int set_error(ap_ctx *c, int code, const std::string &msg);
// the error text of a call without a context (what ap_last_error(NULL) returns); returns code
int set_error_text(int code, const char *msg);
int hip_check(ap_ctx *c, hipError_t e, const char *what);

// Records HIP events around the launches made during its lifetime when profiling is on; the
// elapsed times are accumulated under `name` at the next stream synchronisation.
struct ProfScope {
    ap_ctx *c;
    int label = -1;
    hipEvent_t a = nullptr;
    ProfScope(ap_ctx *ctx, const char *name);
    ~ProfScope();
};
void prof_resolve(ap_ctx *c);

// Reverse-slot cache (rslot): the ACE pair kernel and the learned indicator's grad-g kernel, whichever
// fills an atom's entries first on a list, search every slot whose pair lies within
// max(ACE cutoff, feature cutoff) + 2 skin: a pair beyond that cannot come inside either cutoff before the
// next build (every atom stays within skin / 2 of its build position). Squared, with a rounding margin.
inline double rslot_reach2(const ap_ctx *c) {
    double r = c->ace.rc;
    if (c->have_mlp && c->mlp_rc > r) r = c->mlp_rc;
    r += 2.0 * c->skin;
    return r * r * (1.0 + 1e-9);
}

// geometry.hip
// Buffers of one neighbour-list build: wrapped positions in, build-time positions, flags ([0] gates the
// build, [1] error bits), the cell arrays, and the list out (counts, short counts, slot-major indices).
struct ListBufs {
    const double *pos;
    double *pos_build;
    int *flags;
    int *cell_of, *cell_cnt, *cell_start, *cell_fill, *cell_atoms;
    CandRec *cell_rec;
    int32_t *ncount, *nshort, *nidx;
};
// cells of edge >= r_list (one cell per axis below three); false when r_list >= half a box length
bool list_geometry(const double *box, double r_list, Geometry &g);
void launch_list_kernels(hipStream_t s, int n, const Geometry &g, double r_list, double r_short, int max_nbr,
                         const ListBufs &b);
void launch_wrap(hipStream_t s, const double *in, double *out, int n, const double *box);
void launch_fill_int_on(hipStream_t s, int *p, int v, int count);
// skin_checked: the caller's kernel already ran the skin check on these positions and cleared the
// cell counts; commit = false: the caller's next kernel commits the rebuild flag (flags[3] = flags[0],
// flags[0] = 0) instead of a kernel of its own
int ensure_list(ap_ctx *c, int n, const double *box, double r_list, bool force, bool skin_checked = false,
                bool commit = true);
int prepare_positions(ap_ctx *c, int n, const double *pos_in, const double *box);
void launch_csp_value(ap_ctx *c, int n, const double *box);
int build_csp_pairs(ap_ctx *c, int n, const double *box, int n_csp, int32_t *out);
int install_csp(ap_ctx *c, int n, int n_csp, const int32_t *list);
void launch_fill_int(ap_ctx *c, int *p, int v, int count);
void launch_fill_double(ap_ctx *c, double *p, double v, int count);
void launch_scan(ap_ctx *c, const int *in, int *out, int len, int *total, const int *gate);
int batch_lists(ap_ctx *c, int n, int n_struct, const int *d_off, const double *d_box, const double *pos_in,
                double r_list);

// ace.hip
int ace_setup(ap_ctx *c, const ap_ace_params *p);
void ace_free(ap_ctx *c);
// sbox: per-structure boxes of a batch (atom i uses sbox[3 * sid[i]]), null for the single box;
// want_bval: also write the per-atom coefficient gradients into c->bval
int launch_ace(ap_ctx *c, int n, const double *box, int grid_cap, const double *sbox = nullptr,
               bool want_bval = false);
void ace_cost(const ap_ctx *c, double *fixed, double *per_nbr_energy, double *per_nbr_force);
// new linear (device [n_funcs]) and density (device [n_max]) coefficients into the installed tables
int ace_set_coefficients(ap_ctx *c, const double *cf, const double *b);
// the atomic basis A, its tangent along the displacement field G (device [3][n]) and the tangents of every
// basis function and density term, per atom of S into c->bval
int launch_ace_vjp(ap_ctx *c, int n, const double *box, int grid_cap, const double *sbox, const double *G);

// forces.hip
struct EvalFlags {
    bool switching;   // lambda computed from the descriptor
    bool grad_lambda; // include the grad-lambda forces
    double lam_const; // value of lambda when not computed
    bool eam_forces;  // EAM family included
    bool ace_forces;  // ACE family included
    bool force_mix = false;  // force mixing, Eq. (3), instead of the conservative force
};
// count: also write the per-workgroup counts of lambda < 1 (chunk_cnt) that launch_compact(counted) uses
void launch_dens_desc(ap_ctx *c, int n, const double *box, const EvalFlags &f, const double *lam_in, bool count);
// counted: S from the density pass's chunk counts in one kernel (no subset); otherwise count, scan, scatter
void launch_compact(ap_ctx *c, int n, const int32_t *subset, int n_subset, bool counted);
// count, scan, scatter of the atoms with c->mark[i] != 0
void launch_compact_marked(ap_ctx *c, int n);
// force mixing: c->mark = the atoms that need ACE, c->act = lambda < 1
void launch_mix_mark(ap_ctx *c, int n, const double *box);
// stamped: only the atoms stamped by this evaluation's ACE pair kernel gather; csp_marks: also stamp (cmark)
// the atoms that receive terms from an atom with W != 0: its CSP neighbours, or with the learned
// indicator its list neighbours
void launch_W(ap_ctx *c, int n, const double *box, bool stamped, bool csp_marks);
// uniform_lambda: lambda is the constant of f on every atom (no per-atom lambda from the caller);
// csp_marked: the W pass wrote cmark: only marked atoms look for reverse CSP terms, and with the learned
// indicator an atom neither marked nor flagged active takes the EAM-only gather
void launch_force(ap_ctx *c, int n, const double *box, const EvalFlags &f, double *E_atom, double *F,
                  const double *sbox = nullptr, bool uniform_lambda = true, bool csp_marked = false);
// per-structure sums of sign x weight_i x (E^p_i, c->bval rows) over a batch (deterministic order): the
// coefficient gradients dE_i/dc, dE_i/db, or with sign -1 the force vector-Jacobian product from the tangents
void launch_struct_reduce(ap_ctx *c, int n, int n_struct, const int *d_off, const double *weight, double *E_struct,
                          double *dEdc, double *dEdb, double sign = 1.0);
void launch_reduce(ap_ctx *c, int nblocks, double *E_tot, double *virial9);

int sync_and_check(ap_ctx *c);

// mlp.hip
void launch_mlp_indicator(ap_ctx *c, int n, const double *box);
void launch_mlp_gradg(ap_ctx *c, int n, const double *box);
int mlp_alloc(ap_ctx *c);
void mlp_free(ap_ctx *c);

}  // namespace ap
