// ACE site energies and pair gradients on the precise set S = {i : lambda_i < 1}.
//
// Form evaluated (the paper cites ACE; this is the concrete basis of the library, see ap.h):
//   A_{n l m} = sum_j g_n(r_ij) Y_lm(rhat_ij)   with REAL orthonormal harmonics Y_lm
//   E = E0 + sum_n c1_n A_{n00} + sum_l sum_{n1 n2} C2_l[n1][n2] sum_m A_{n1 l m} A_{n2 l m}
//       + sum_blocks sum_M sum_{n1 n2 n3} C3[n1][n2][n3] P_M[n1][n2] A_{n3 L M} - emb_A sqrt(phi2)
//   P_M[n1][n2] = sum_{m1 m2} kappa(l1 m1, l2 m2, L M) A_{n1 l1 m1} A_{n2 l2 m2}
// Every order-3 function (l1,l2,l3 sorted so that L <= l1 <= l2) belongs to one block (L, l1, l2);
// kappa is the real-harmonic form of the Wigner 3j symbol, obtained here as the real Gaunt integral
// (Gauss-Legendre x uniform-phi quadrature, exact for these degrees) divided by
// sqrt((2l1+1)(2l2+1)(2L+1)/(4 pi)) (l1 l2 L; 0 0 0). Both forms give the same rotation invariants,
// so E equals the complex-harmonic definition with the 3j symbol.
//
// k_ace_energy (one workgroup per S atom): neighbours -> radial and Y tables in LDS -> A -> energy
// and G = dE/dA (adjoint of the block contractions); writes E^p, E~ of (S17) and G.
// k_ace_pairforce (one workgroup per S atom, one thread per neighbour slot):
// f_ji = dE_i/du_ij = sum_{n,lm} G_{nlm} grad_u [g_n(r) Y_lm(uhat)].
#include <type_traits>

#include "ap_internal.h"
#include "basis.h"

namespace ap {

constexpr int kAceMaxSlots = 1536;

struct AceArgs {
    const double *pos;
    int n;
    double L[3];
    double rc;
    const int32_t *ncount, *nidx;
    int max_nbr;
    const int *slist, *scount;
    const double *dlam, *wbar, *Ef;
    const double *c1d, *bdd;
    double *Ep, *Et;
    void *gbuf;     // [S][n_max * nlm] the atomic basis A
    double *s0buf;  // [S][n_max] FP64 sums of the radial channels over the neighbours
    // dE/dA [2][gstride][n_max * nlm]: row s of the first region holds atom s whole or its part 0; part
    // p >= 1 of split atom whole + r is row (p - 1) R + r of the second (R atoms split)
    void *gpart;
    double *epart;  // [kMaxParts][gstride] the site energy of each part
    int gstride;    // capacity in atoms
    int n0;         // leading L = 0 blocks (the parts share out the blocks after them)
    int slots;      // energy-kernel workgroups resident at once on the device
    int *queue;     // work-item counter of the energy kernel
    int *stamp;     // [n] set to gen for every precise atom and every atom in its list (null: not kept)
    // reverse slots kept per list build: rslot[i][slot] is the slot of i in the list of its slot-th
    // neighbour, valid while rstamp[i] == *list_gen (null rslot: searched every time)
    int *rslot, *rstamp;
    const int *list_gen;
    const void *c30, *kap0;  // the L = 0 blocks folded into order 2 (null: processed as blocks)
    int gen;
    // reverse terms: the neighbour's gather reads the term of a pair only inside rc, so it is written for
    // r^2 < rw2 = rc^2 (1 + 1e-9). When the reverse slots are cached for the list, they are searched for
    // every pair with r^2 < rrev2 (rslot_reach2: no pair beyond it comes inside rc before the next build)
    double rw2, rrev2;
    void *fpair;  // [S][max_nbr][3]
    void *frev;   // [3][max_nbr][n]: f of pair (i, j) stored at slot k of i in j's list
    const Rec4 *xl;  // [n] {x, y, z, lambda}
    Rec4 *eb;        // [n] {xi', g, d + d0, E~}: E~ written here
    const void *c1, *bd, *c2, *c3, *kval;
    const int *kidx, *blk;
    int nblk;
    double emb_A, E0;
    int *flags;
    // batches of periodic cells: box of structure sid[i] (null: the single box L)
    const double *sbox;
    const int *sid;
    // coefficient gradients: bval[s][nu] = dE_i/dc_nu, bval[s][n_funcs + n] = dE_i/db_n (null: off)
    void *bval;
    int bstride, n_funcs;
    const int *g1, *g2, *g3;
    int ng1, ng2;
};

__device__ __forceinline__ void atom_box(const AceArgs &a, int i, double &Lx, double &Ly, double &Lz) {
    if (a.sbox) {
        const double *b = a.sbox + 3 * a.sid[i];
        Lx = b[0];
        Ly = b[1];
        Lz = b[2];
    } else {
        Lx = a.L[0];
        Ly = a.L[1];
        Lz = a.L[2];
    }
}

__device__ __forceinline__ double block_sum_d(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); q++) s += sh[q];
    return s;
}

// Couplings of one (l1, l2, L) block in its three orderings, staged in LDS per block.
constexpr int kKapStage = 672;

// Stages one block's couplings (three orderings, at most kKapStage entries) and its dense
// coefficient block (NCE elements) in LDS: every load is issued before the first store, the block
// with 16-byte vector loads, so the whole stage costs about one memory latency.
template <typename T, int NCE>
__device__ __forceinline__ void stage_block(int *kc, T *kv, T *Cs, const int *__restrict__ kidx,
                                            const T *__restrict__ kval, const T *__restrict__ C, int k0, int k1) {
    constexpr int VW = 16 / sizeof(T);
    static_assert(NCE % VW == 0, "coefficient block size");
    typedef T vec __attribute__((ext_vector_type(VW)));
    constexpr int NV = NCE / VW, PER = (NV + kBlock - 1) / kBlock, KP = (kKapStage + kBlock - 1) / kBlock;
    const int tid = threadIdx.x;
    int ci[KP];
    T cv[KP];
    vec cc[PER];
#pragma unroll
    for (int u = 0; u < KP; u++) {
        const int q = k0 + tid + u * kBlock;
        if (q < k1) {
            ci[u] = kidx[q];
            cv[u] = kval[q];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = tid + u * kBlock;
        if (q < NV) cc[u] = reinterpret_cast<const vec *>(C)[q];
    }
#pragma unroll
    for (int u = 0; u < KP; u++) {
        const int q = k0 + tid + u * kBlock;
        if (q < k1) {
            kc[q - k0] = ci[u];
            kv[q - k0] = cv[u];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = tid + u * kBlock;
        if (q < NV) reinterpret_cast<vec *>(Cs)[q] = cc[u];
    }
}

// Per S atom: the neighbours inside rc, their radial channels and harmonics, and the atomic basis
// A[n][lm] (with the l = 0 sums also in FP64), written to the adjoint buffer and the sum buffer.
// Four consecutive LDS elements (16-byte aligned) into registers.
template <typename T>
__device__ __forceinline__ void ld4(const T *p, T *o) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    } else {
        const double2 v0 = reinterpret_cast<const double2 *>(p)[0], v1 = reinterpret_cast<const double2 *>(p)[1];
        o[0] = v0.x;
        o[1] = v0.y;
        o[2] = v1.x;
        o[3] = v1.y;
    }
}

// Work plan of the energy kernel. The per-atom time is a chain of dependent block steps, about as long
// with one workgroup on a CU as with four (0.20 against 0.23 ms at n_max 12, l_max 6). So the atoms
// that fill whole rounds of the resident workgroups (slots) are taken whole, and the remaining R atoms
// of a last, partial round are split into parts of their coupling blocks that fill that round: P =
// min(kMaxParts, slots / R) parts each, and the first E = slots - P R of them one part more where P + 1
// parts are allowed, so that every slot gets a part and most parts are the smaller ones. (P, and the
// extra part, are also capped so that the parts' rows fit the scratch rows.) Items: atoms s < whole one
// each; then the parts of the P-part atoms (the larger parts, handed out first), then those of the
// (P + 1)-part atoms. Computed from the device-side S alone, the same way by the energy kernel and by
// the pair kernel that adds the parts.
constexpr int kMaxParts = 4;
struct AcePlan {
    int whole, items, R, P, E;  // split atoms: whole + r for r < R; r < E has P + 1 parts, the rest P
};
__device__ __forceinline__ AcePlan ace_plan(int S, int slots, int cap) {
    AcePlan q;
    const int R = S % slots;
    int P = R > 0 ? slots / R : 1;
    if (P > kMaxParts) P = kMaxParts;
    if (P > 1 && (long long)(P - 1) * R > cap) P = 1 + cap / R;
    if (P >= 2) {
        q.whole = S - R;
        q.R = R;
        q.P = P;
        q.E = P + 1 <= kMaxParts && (long long)P * R <= cap ? min(R, slots - P * R) : 0;
        q.items = q.whole + P * R + q.E;
    } else {
        q.whole = S;
        q.items = S;
        q.R = 0;
        q.P = 1;
        q.E = 0;
    }
    return q;
}
__device__ __forceinline__ int ace_parts_of(const AcePlan &q, int r) { return r < q.E ? q.P + 1 : q.P; }
// split item u (its index after the whole atoms) -> atom whole + r, part h
__device__ __forceinline__ void ace_item(const AcePlan &q, int u, int &r, int &h) {
    const int big = (q.R - q.E) * q.P;
    if (u < big) {
        r = q.E + u / q.P;
        h = u - (r - q.E) * q.P;
    } else {
        const int v = u - big;
        r = v / (q.P + 1);
        h = v - r * (q.P + 1);
    }
}
// first coupling block of part p of P: equal shares of the blocks after the n0 leading L = 0 ones
__device__ __forceinline__ int ace_part_block(int p, int P, int n0, int nblk) {
    return p == 0 ? 0 : n0 + (nblk - n0) * p / P;
}

// (in FP32 at n_max 12 the second bound keeps it at 6 workgroups per CU: with 1,536 resident slots the S
// atoms of a mixed step take one round; the smaller bases would spill under it)
template <typename T, int NMAX, int LMAX>
__global__ __launch_bounds__(kBlock, (sizeof(T) == 4 && NMAX == 12) ? 6 : 1) void k_ace_basis(AceArgs a) {
    constexpr int NLM = (LMAX + 1) * (LMAX + 1), NA = NMAX * NLM;
    constexpr int V = kAceMaxValid, CH = 64;  // neighbours kept per site; harmonics computed CH at a time
    __shared__ alignas(16) T sR[CH * NMAX];  // (rows read as 16-byte vectors)
    __shared__ T sY[CH * NLM];
    __shared__ T sA[NA];
    __shared__ T sU[V * 4];
    __shared__ double sRd[V], sS[NMAX];
    __shared__ int sCnt[5];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = a.n;
    const int S = *a.scount;
    const double rc2 = a.rc * a.rc;
    const T rcT = (T)a.rc;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0;  // the energy kernel's work counter
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int i = a.slist[s];
        const double xi = a.pos[i], yi = a.pos[n + i], zi = a.pos[2 * n + i];
        double Lx, Ly, Lz;
        atom_box(a, i, Lx, Ly, Lz);
        const int cnt = a.ncount[i];
        if (tid == 0) sCnt[4] = 0;
        if (tid < NMAX) sS[tid] = 0.0;
        for (int o = tid; o < NA; o += kBlock) sA[o] = T(0);
        __syncthreads();
        // ---- phase 0: neighbours inside rc, compacted in list order (ballot prefix) ----
        for (int base = 0; base < cnt; base += kBlock) {
            const int slot = base + tid;
            bool valid = false;
            double ux = 0, uy = 0, uz = 0, r2 = 0;
            if (slot < cnt) {
                const int j = a.nidx[(size_t)slot * n + i];
                const Rec4 pj = a.xl[j];
                ux = min_image_w(pj.x - xi, Lx);
                uy = min_image_w(pj.y - yi, Ly);
                uz = min_image_w(pj.z - zi, Lz);
                r2 = ux * ux + uy * uy + uz * uz;
                valid = r2 < rc2;
            }
            const unsigned long long m = __ballot(valid);
            if (lane == 0) sCnt[wv] = __popcll(m);
            __syncthreads();
            int off = sCnt[4];
            for (int q = 0; q < wv; q++) off += sCnt[q];
            const int p = off + __popcll(m & ((1ull << lane) - 1ull));
            if (valid) {
                if (p < V) {
                    sU[4 * p + 0] = (T)ux;
                    sU[4 * p + 1] = (T)uy;
                    sU[4 * p + 2] = (T)uz;
                    sU[4 * p + 3] = (T)sqrt(r2);
                    sRd[p] = sqrt(r2);
                } else {
                    atomicOr(&a.flags[1], kErrAceNbr);
                }
            }
            __syncthreads();
            if (tid == 0) sCnt[4] += sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
            __syncthreads();
        }
        const int nv = min(sCnt[4], V);
        // ---- phases 1-2: radial channels and harmonics, CH neighbours at a time, into A[n][lm] ----
        for (int v0 = 0; v0 < nv; v0 += CH) {
            const int nc = min(CH, nv - v0);
            // a lane per neighbour in each wavefront: wavefront 0 evaluates the radial channels,
            // wavefronts 1-3 the harmonics of the orders m assigned to them (about 16 values each)
            static_assert(kBlock == 4 * CH, "one neighbour per lane in each of four wavefronts");
            if (wv == 0) {
                // the l = 0 radial sums feed the two-body and density terms, whose fitted coefficients
                // cancel strongly: they are kept in FP64 whatever T is, summed over the chunk's
                // neighbours by a fixed shuffle tree and added to s_n by lane 0
                double gd[NMAX];
#pragma unroll
                for (int q = 0; q < NMAX; q++) gd[q] = 0.0;
                if (lane < nc) {
                    const int v = lane, u = v0 + v;
                    const T r = sU[4 * u + 3];
                    T g[NMAX];
                    radial<T, NMAX>(r, rcT, g, (T *)nullptr);
#pragma unroll
                    for (int q = 0; q < NMAX; q++) sR[v * NMAX + q] = g[q];
                    radial<double, NMAX>(sRd[u], a.rc, gd, (double *)nullptr);
                }
#pragma unroll
                for (int q = 0; q < NMAX; q++) {
                    double x = gd[q];
                    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                    if (lane == 0) sS[q] += x;
                }
            } else if (lane < nc) {
                const int v = lane, u = v0 + v;
                const T r = sU[4 * u + 3], ir = T(1) / r;
                {
                    const T x = sU[4 * u] * ir, y = sU[4 * u + 1] * ir, z = sU[4 * u + 2] * ir;
                    T cm = T(1), sm = T(0);  // (x + iy)^m
#pragma unroll
                    for (int m = 0; m <= LMAX; m++) {
                        if (m > 0) {
                            const T c2 = x * cm - y * sm;
                            sm = x * sm + y * cm;
                            cm = c2;
                        }
                        // orders per wavefront: {1, 5}, {2, 4, 6}, {0, 3}
                        const int owner = (m == 0 || m == 3) ? 3 : ((m == 1 || m == 5) ? 1 : 2);
                        if (owner == wv) ylm_real_order<T, LMAX>(m, z, cm, sm, sY + v * NLM);
                    }
                }
            }
            __syncthreads();
            // A[n][lm] += sum_v R[v][n] Y[v][lm]: a thread per (four n, lm), so that each pair of loads (one
            // 16-byte radial row, one harmonic) feeds four FMAs
            static_assert(NMAX % 4 == 0, "radial channels in fours");
            for (int o = tid; o < (NMAX / 4) * NLM; o += kBlock) {
                const int q4 = o / NLM, lm = o - q4 * NLM;
                T acc[4];
#pragma unroll
                for (int j = 0; j < 4; j++) acc[j] = sA[(4 * q4 + j) * NLM + lm];
                for (int v = 0; v < nc; v++) {
                    const T y = sY[v * NLM + lm];
                    T r4[4];
                    ld4(sR + v * NMAX + 4 * q4, r4);
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[j] += r4[j] * y;
                }
#pragma unroll
                for (int j = 0; j < 4; j++) sA[(4 * q4 + j) * NLM + lm] = acc[j];
            }
            __syncthreads();
        }
        T *aout = (T *)a.gbuf + (size_t)s * NA;
        for (int o = tid; o < NA; o += kBlock) aout[o] = sA[o];
        if (tid < NMAX) a.s0buf[(size_t)s * NMAX + tid] = sS[tid];
        __syncthreads();
    }
}

// Per S atom, from its basis A: orders 1-3 with the embedding, the site energy, and the adjoint
// G = dE/dA (written over A in the adjoint buffer).
// sum_{q in [e0, e1)} kv[q] (row_q . At_q) for the coupling adjoints: code kc[q] = (byte offset of the row of
// At) | (byte offset of the matrix in rows) << 16, both multiples of 16 (the host writes them for the tables'
// precision): an At row address is one mask, a matrix row one add of the upper half; row_q starts roff elements
// into its matrix. The rows are read as 16-byte vectors. Two couplings per iteration, so that their row loads
// are in flight together; the sum still runs in q and k order (four per iteration take the kernel past 128
// VGPRs, to three workgroups per CU: 245 -> 324 us per mixed step).
template <typename T, int NMAX>
__device__ __forceinline__ T row_dot(const char *rb, const char *ab, unsigned code) {
    const T *r = reinterpret_cast<const T *>(rb + (code >> 16)), *at = reinterpret_cast<const T *>(ab + (code & 0xffffu));
    T s = T(0);
#pragma unroll
    for (int k = 0; k < NMAX; k += 4) {
        T r4[4], a4[4];
        ld4(r + k, r4);
        ld4(at + k, a4);
#pragma unroll
        for (int u = 0; u < 4; u++) s += r4[u] * a4[u];
    }
    return s;
}
template <typename T, int NMAX>
__device__ __forceinline__ T coupling_sum(const int *kc, const T *kv, const T *rows, int roff, const T *At, int e0,
                                          int e1) {
    static_assert(NMAX % 4 == 0, "rows of 16-byte vectors");
    const char *rb = reinterpret_cast<const char *>(rows + roff), *ab = reinterpret_cast<const char *>(At);
    T acc = T(0);
    int q = e0;
    for (; q + 1 < e1; q += 2) {
        const T s0 = row_dot<T, NMAX>(rb, ab, (unsigned)kc[q]);
        const T s1 = row_dot<T, NMAX>(rb, ab, (unsigned)kc[q + 1]);
        acc += kv[q] * s0;
        acc += kv[q + 1] * s1;
    }
    if (q < e1) acc += kv[q] * row_dot<T, NMAX>(rb, ab, (unsigned)kc[q]);
    return acc;
}

template <typename T, int NMAX, int LMAX>
__global__ __launch_bounds__(kBlock) void k_ace_energy(AceArgs a) {
    constexpr int NLM = (LMAX + 1) * (LMAX + 1), NA = NMAX * NLM, NN = NMAX * NMAX, MM = 2 * LMAX + 1;
    struct BlkBuf {
        T P[MM * NN], Q[MM * NN];
        alignas(16) T C[NN * NMAX];
        T kv[kKapStage];
        int kc[kKapStage];
    };
    __shared__ BlkBuf B;
    __shared__ T sA[NA], sAt[NA], sG[NA];  // A[n][lm], its transpose At[lm][n], dE/dA[n][lm]
    __shared__ double sS[NMAX];
    __shared__ double sRed[kBlock / 64];
    __shared__ T sEmbD;
    __shared__ double sEmbD64;
    const int tid = threadIdx.x;
    const T *c1 = (const T *)a.c1, *bd = (const T *)a.bd, *c2 = (const T *)a.c2, *c3 = (const T *)a.c3;
    const T *kval = (const T *)a.kval;
    const int S = *a.scount;
    const AcePlan pl = ace_plan(S, a.slots, a.gstride);
    const int whole = pl.whole, items = pl.items, R = pl.R;
    // a persistent grid: workgroup b takes item b, then the next items in order from a device counter
    // (zeroed by the basis kernel): whole atoms first, then the parts. Part 0 takes orders 1-2 and its
    // share of the blocks, the other parts theirs; each item writes its own dE/dA and energy, added by
    // the pair kernel in a fixed order.
    __shared__ int sItem;
    for (int w = blockIdx.x; w < items;) {
        const bool K2 = w >= whole;
        int r = 0, h = 0;
        if (K2) ace_item(pl, w - whole, r, h);
        const int parts = K2 ? ace_parts_of(pl, r) : 1;
        const int s = K2 ? whole + r : w;
        const T *ain = (const T *)a.gbuf + (size_t)s * NA;
        for (int o = tid; o < NA; o += kBlock) {
            const int q = o / NLM, lm = o - q * NLM;
            const T v = ain[o];
            sA[o] = v;
            sAt[lm * NMAX + q] = v;
            sG[o] = T(0);
        }
        if (tid < NMAX) sS[tid] = a.s0buf[(size_t)s * NMAX + tid];
        __syncthreads();
        // ---- phase 3a: orders 1 and 2, embedding ----
        double e = 0.0;
        T *bout = a.bval ? (T *)a.bval + (size_t)s * a.bstride : nullptr;
        // the L = 0 blocks folded into order 2, except when their own B values are asked for
        const bool fold0 = a.c30 != nullptr && !bout;
        if (h == 0) {
        if (tid == 0) {
            const double y00 = 0.28209479177387814;  // 1 / sqrt(4 pi)
            double phi2 = 0.0, e1 = 0.0;
            for (int q = 0; q < NMAX; q++) {
                phi2 += a.bdd[q] * sS[q];  // b_n sqrt(4 pi) A_n00 with A_n00 = s_n / sqrt(4 pi)
                e1 += a.c1d[q] * (sS[q] * y00);
            }
            double emb = 0.0, demb = 0.0;
            if (phi2 > 0.0) {
                const double sq = sqrt(phi2);
                emb = -a.emb_A * sq;
                demb = -0.5 * a.emb_A / sq;
            }
            sEmbD = (T)demb;
            sEmbD64 = demb;
            e = a.E0 + e1 + emb;
        }
        // the order-2 coefficients C2_l[n1][n2] staged in the (still unused) coefficient-block space
        static_assert(LMAX + 1 <= NMAX, "order-2 table fits the block buffer");
        for (int o = tid; o < (LMAX + 1) * NN; o += kBlock) B.C[o] = c2[o];
        if (fold0) {
            // The L = 0 blocks in closed form. With kappa_l their one coupling value (m1 = m2, M = 0),
            // block (0, l, l) contributes kappa_l sum_{n1 n2} D_l[n1][n2] R_l[n1][n2], where
            // D_l = sum_n3 C0_l[..][..][n3] A[n3][00] and R_l[n1][n2] = sum_m A[n1][l m] A[n2][l m]: an
            // order-2 term with matrix kappa_l (D_l + D_l^T) / 2, added to C2_l, plus the gradient through
            // D_l, dE/dA[n3][00] += kappa_l sum_{n1 n2} C0_l[n1][n2][n3] R_l[n1][n2]. One thread per
            // (l, n1, n2) reads the row C0_l[n1][n2][:] once for both.
            const T *c30 = (const T *)a.c30, *kap0 = (const T *)a.kap0;
            T acc[NMAX];
#pragma unroll
            for (int q = 0; q < NMAX; q++) acc[q] = T(0);
            for (int w = tid; w < (LMAX + 1) * NN; w += kBlock) {
                const int l = w / NN, r = w - l * NN, n1 = r / NMAX, n2 = r - n1 * NMAX;
                const T kap = kap0[l];
                T D = T(0);
                if (kap != T(0)) {
                    T R = T(0);
                    for (int m = l * l; m <= l * l + 2 * l; m++) R += sAt[m * NMAX + n1] * sAt[m * NMAX + n2];
                    const T kr = kap * R;
                    const T *crow = c30 + (size_t)w * NMAX;
#pragma unroll
                    for (int q = 0; q < NMAX; q++) {
                        const T cv = crow[q];
                        D += cv * sAt[q];  // A[q][00]
                        acc[q] += cv * kr;
                    }
                }
                B.P[w] = D;
            }
            // the A[n3][00] gradient: a fixed butterfly per wavefront, then the wavefronts in order
#pragma unroll
            for (int q = 0; q < NMAX; q++) {
                T v = acc[q];
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                if ((tid & 63) == 0) B.Q[(tid >> 6) * NMAX + q] = v;
            }
            __syncthreads();
            if (tid < NMAX) {
                T v = T(0);
                for (int wv = 0; wv < kBlock / 64; wv++) v += B.Q[wv * NMAX + tid];
                sG[tid * NLM] += v;
            }
            for (int o = tid; o < (LMAX + 1) * NN; o += kBlock) {
                const int l = o / NN, r = o - l * NN, n1 = r / NMAX, n2 = r - n1 * NMAX;
                B.C[o] += kap0[l] * T(0.5) * (B.P[o] + B.P[l * NN + n2 * NMAX + n1]);
            }
        }
        __syncthreads();
        if (bout) {
            // dE/dc for orders 1 and 2 (B values) and dE/db_n = xi'(phi2) s_n
            const double y00 = 0.28209479177387814;
            for (int q = tid; q < a.ng1; q += kBlock) bout[a.g1[2 * q + 1]] = (T)(sS[a.g1[2 * q]] * y00);
            for (int q = tid; q < NMAX; q += kBlock) bout[a.n_funcs + q] = (T)(sEmbD64 * sS[q]);
            for (int q = tid; q < a.ng2; q += kBlock) {
                const int code = a.g2[2 * q];
                const int q1 = code & 255, q2 = (code >> 8) & 255, l = code >> 16;
                T bsum = T(0);
                for (int m = l * l; m <= l * l + 2 * l; m++) bsum += sA[q1 * NLM + m] * sA[q2 * NLM + m];
                bout[a.g2[2 * q + 1]] = bsum;
            }
        }
        for (int o = tid; o < NA; o += kBlock) {
            const int q = o / NLM, lm = o - q * NLM;
            int l = 0;
            while ((l + 1) * (l + 1) <= lm) l++;
            const T *row = B.C + (l * NMAX + q) * NMAX;
            const T *acol = sAt + lm * NMAX;
            T g2 = T(0);
#pragma unroll
            for (int q2 = 0; q2 < NMAX; q2++) g2 += row[q2] * acol[q2];
            g2 *= T(2);
            e += 0.5 * (double)(sA[o] * g2);
            sG[o] += g2 + (lm == 0 ? c1[q] + sEmbD * bd[q] : T(0));  // order-1 and density parts of dE/dA
        }
        }
        // ---- phase 3b: order-3 blocks ----
        const int b_lo = K2 ? ace_part_block(h, parts, a.n0, a.nblk) : 0;
        const int b_hi = K2 && h + 1 < parts ? ace_part_block(h + 1, parts, a.n0, a.nblk) : a.nblk;
        // a whole atom starts its blocks a quarter, a half or three quarters of the way round, by its item
        // index, so that the workgroups that start together on a CU (items 256 apart in the first round)
        // are not in the same block at once (233.9 against 236.7 us per mixed step; the sums only change
        // their order)
        const int nrun = b_hi - b_lo, rot = K2 ? 0 : (((w + (w >> 8)) & 3) * nrun) >> 2;
        for (int t = 0; t < nrun; t++) {
            const int b = b_lo + (t + rot < nrun ? t + rot : t + rot - nrun);
            const int *bk = a.blk + b * kBlkInts;
            const int L = bk[0], l1 = bk[1], l2 = bk[2];
            if (fold0 && L == 0) continue;  // done with order 2
            const int nM = 2 * L + 1, n1m = 2 * l1 + 1, n2m = 2 * l2 + 1;
            const int bL = L * L + L, b1 = l1 * l1 + l1, b2 = l2 * l2 + l2;
            const int k0 = bk[4], k1 = bk[32 + n2m];
            // stage the block's couplings (host checks k1 - k0 <= kKapStage) and coefficients
            __syncthreads();
            stage_block<T, NN * NMAX>(B.kc, B.kv, B.C, a.kidx, kval, c3 + bk[3], k0, k1);
            __syncthreads();
            // P_M[n1][n2] = sum kappa A[n1][l1 m1] A[n2][l2 m2]; Q_M[n1][n2] = sum_n3 C A[n3][L M];
            // one thread per (M, n1, run of NS n2) holds its n2 in registers. The runs are as short as the
            // workgroup allows (NS = 4 up to 7 values of M, 6 up to 10, else all 12): most blocks have few M,
            // and a thread's chain over the couplings and C rows, not the lane count, sets the phase's time.
            auto pq = [&](auto ns) {
                constexpr int NS = decltype(ns)::value, SPL = NMAX / NS;
                for (int w = tid; w < nM * NMAX * SPL; w += kBlock) {
                    const int Mi = w / (NMAX * SPL), rem = w - Mi * (NMAX * SPL), n1 = rem / SPL;
                    const int o2 = (rem - n1 * SPL) * NS;  // first n2 of the run
                    T P[NS], Q[NS];
#pragma unroll
                    for (int q = 0; q < NS; q++) P[q] = T(0);
                    const int e0 = bk[4 + Mi] - k0, e1 = bk[4 + Mi + 1] - k0;
                    // (l1 m1 column) | (l2 m2 row of At, in units of four) << 8: the row offset stays a visible
                    // multiple of four, so its reads are vector loads; two couplings per iteration (their loads
                    // in flight together), each P entry still summed in coupling order
                    int q = e0;
                    for (; q + 1 < e1; q += 2) {
                        const int c0 = B.kc[q], c1 = B.kc[q + 1];
                        const T a10 = B.kv[q] * sA[n1 * NLM + (c0 & 255)];
                        const T a11 = B.kv[q + 1] * sA[n1 * NLM + (c1 & 255)];
                        const T *a20 = sAt + 4 * (c0 >> 8) + o2, *a21 = sAt + 4 * (c1 >> 8) + o2;
#pragma unroll
                        for (int q2 = 0; q2 < NS; q2++) {
                            P[q2] += a10 * a20[q2];
                            P[q2] += a11 * a21[q2];
                        }
                    }
                    if (q < e1) {
                        const int c0 = B.kc[q];
                        const T a10 = B.kv[q] * sA[n1 * NLM + (c0 & 255)];
                        const T *a20 = sAt + 4 * (c0 >> 8) + o2;
#pragma unroll
                        for (int q2 = 0; q2 < NS; q2++) P[q2] += a10 * a20[q2];
                    }
                    const T *a3 = sAt + (bL + Mi - L) * NMAX;
                    T A3[NMAX];
#pragma unroll
                    for (int q = 0; q < NMAX; q++) A3[q] = a3[q];
                    const T *cr = B.C + n1 * NN + o2 * NMAX;
#pragma unroll
                    for (int q2 = 0; q2 < NS; q2++) {
                        T acc = T(0);
#pragma unroll
                        for (int q3 = 0; q3 < NMAX; q3++) acc += cr[q2 * NMAX + q3] * A3[q3];
                        Q[q2] = acc;
                    }
                    T *pp = B.P + Mi * NN + n1 * NMAX + o2, *qq = B.Q + Mi * NN + n1 * NMAX + o2;
                    T ep = T(0);
#pragma unroll
                    for (int q2 = 0; q2 < NS; q2++) {
                        ep += P[q2] * Q[q2];
                        pp[q2] = P[q2];
                        qq[q2] = Q[q2];
                    }
                    e += (double)ep;
                }
            };
            if (NMAX % 4 == 0 && nM * NMAX * (NMAX / 4) <= kBlock)
                pq(std::integral_constant<int, (NMAX % 4 == 0 ? 4 : NMAX)>());
            else if (NMAX % 6 == 0 && nM * NMAX * (NMAX / 6) <= kBlock)
                pq(std::integral_constant<int, (NMAX % 6 == 0 ? 6 : NMAX)>());
            else
                pq(std::integral_constant<int, NMAX>());
            __syncthreads();
            if (bout) {
                // B of the block's basis functions: sum_M P_M[n1][n2] A_{n3 L M}
                for (int q = bk[46] + tid; q < bk[47]; q += kBlock) {
                    const int code = a.g3[2 * q];
                    const int rem = code & 0xffff, q3 = code >> 16;
                    T bsum = T(0);
                    for (int Mi = 0; Mi < nM; Mi++) bsum += B.P[Mi * NN + rem] * sA[q3 * NLM + bL + Mi - L];
                    bout[a.g3[2 * q + 1]] = bsum;
                }
            }
            // dE/dA[n3][L M] = sum_{n1 n2} C[n1][n2][n3] P_M[n1][n2]: a lane per (M, four n3, quarter of
            // the (n1, n2) range) reading 16-byte rows of C; the quarters are combined by a fixed
            // butterfly over four adjacent lanes
            {
                constexpr int NQ3 = NMAX / 4, PCH = NN / 4;
                static_assert(NMAX % 4 == 0 && PCH % 4 == 0, "tile shape");
                const int items = nM * NQ3 * 4;
                for (int base = 0; base < items; base += kBlock) {
                    const int w = base + tid, part = w & 3;
                    T acc[4] = {T(0), T(0), T(0), T(0)};
                    int col = -1, j4 = 0;
                    if (w < items) {
                        const int it = w >> 2, Mi = it / NQ3;
                        j4 = (it - Mi * NQ3) * 4;
                        col = bL + Mi - L;
                        const T *pp = B.P + Mi * NN + part * PCH;
                        const T *cc = B.C + part * PCH * NMAX + j4;
                        for (int p = 0; p < PCH; p += 4) {
                            T p4[4];
                            ld4(pp + p, p4);
#pragma unroll
                            for (int u = 0; u < 4; u++) {
                                T c4[4];
                                ld4(cc + (p + u) * NMAX, c4);
#pragma unroll
                                for (int j = 0; j < 4; j++) acc[j] += c4[j] * p4[u];
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        acc[j] += __shfl_xor(acc[j], 1, 64);
                        acc[j] += __shfl_xor(acc[j], 2, 64);
                    }
                    if (col >= 0 && part == 0) {
#pragma unroll
                        for (int j = 0; j < 4; j++) sG[(j4 + j) * NLM + col] += acc[j];
                    }
                }
            }
            __syncthreads();
            // dE/dA[n1][l1 m1] = scale sum kappa sum_n2 Q_M[n1][n2] A[n2][l2 m2]
            // (lanes in runs of n_max share m1: the same coupling list, read as a broadcast)
            auto adj1 = [&](T scale) {
                for (int w = tid; w < NMAX * n1m; w += kBlock) {
                    const int i1 = w / NMAX, q1 = w - i1 * NMAX;
                    // codes: (l2 m2 row of At) | (Q_M offset) << 16, in bytes
                    const T acc = coupling_sum<T, NMAX>(B.kc, B.kv, B.Q, q1 * NMAX, sAt, bk[18 + i1] - k0,
                                                        bk[18 + i1 + 1] - k0);
                    sG[q1 * NLM + b1 + i1 - l1] += scale * acc;
                }
            };
            if (l1 == l2) {
                // l1 = l2: the couplings are symmetric in (m1, m2), so the l2 adjoint is the l1 one taken
                // with Q_M transposed; the coefficient blocks of these (L, l, l) are stored symmetrised in
                // (n1, n2) (the same energy, as P_M is symmetric), so Q_M is symmetric and both adjoints
                // together are twice the l1 one
                adj1(T(2));
                continue;
            }
            adj1(T(1));
            // Q_M transposed into the space of P (no longer read), for the row reads below
            for (int o = tid; o < nM * NN; o += kBlock) {
                const int Mi = o / NN, r = o - Mi * NN, n1 = r / NMAX, n2 = r - n1 * NMAX;
                B.P[Mi * NN + n2 * NMAX + n1] = B.Q[o];
            }
            __syncthreads();
            // dE/dA[n2][l2 m2] = sum kappa sum_n1 Q_M[n1][n2] A[n1][l1 m1]
            for (int w = tid; w < NMAX * n2m; w += kBlock) {
                const int i2 = w / NMAX, q2 = w - i2 * NMAX;
                // codes: (l1 m1 row of At) | (Q_M offset) << 16, in bytes; rows of Q_M transposed
                const T acc = coupling_sum<T, NMAX>(B.kc, B.kv, B.P, q2 * NMAX, sAt, bk[32 + i2] - k0,
                                                    bk[32 + i2 + 1] - k0);
                sG[q2 * NLM + b2 + i2 - l2] += acc;
            }
        }
        __syncthreads();
        // ---- outputs: this part's energy and dE/dA ----
        const double E = block_sum_d(e, sRed);
        T *gout = (T *)a.gpart + (h == 0 ? (size_t)s : (size_t)a.gstride + (size_t)(h - 1) * R + r) * NA;
        for (int o = tid; o < NA; o += kBlock) gout[o] = sG[o];
        if (tid == 0) {
            a.epart[(size_t)h * a.gstride + s] = E;
            sItem = (int)gridDim.x + atomicAdd(a.queue, 1);
        }
        __syncthreads();
        w = sItem;
    }
}

// threads per precise atom in the pair kernel (two wavefronts: one alone per atom, 64 threads, was slower:
// 27.5 against 23.4 us per mixed step)
constexpr int kPairThreads = 128;

template <typename T, int NMAX, int LMAX>
__global__ __launch_bounds__(kPairThreads) void k_ace_pairforce(AceArgs a) {
    constexpr int NLM = (LMAX + 1) * (LMAX + 1), NA = NMAX * NLM, NW = kPairThreads / 64;
    __shared__ alignas(16) T sGt[NA];  // G transposed: [lm][n]
    // the pairs inside rc, compacted: slot, neighbour, u (in T), r^2 (FP64); sPC: wave counts and the total
    __shared__ int sPS[kAceMaxValid], sPJ[kAceMaxValid], sPC[NW + 1];
    __shared__ T sPU[4 * kAceMaxValid];
    __shared__ double sPR2[kAceMaxValid];
    const int n = a.n;
    const int S = *a.scount;
    const double rc2 = a.rc * a.rc;
    const T rcT = (T)a.rc;
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int i = a.slist[s];
        // G = dE/dA and the site energy from the energy kernel's parts, added in part order
        const AcePlan pl = ace_plan(S, a.slots, a.gstride);
        const int R = pl.R, r = s - pl.whole, P = s >= pl.whole ? ace_parts_of(pl, r) : 1;
        const T *g0 = (const T *)a.gpart + (size_t)s * NA;
        for (int o = threadIdx.x; o < NA; o += blockDim.x) {
            const int q = o / NLM, lm = o - q * NLM;
            T g = g0[o];
            for (int p = 1; p < P; p++) g += ((const T *)a.gpart)[((size_t)a.gstride + (size_t)(p - 1) * R + r) * NA + o];
            sGt[lm * NMAX + q] = g;
        }
        if (threadIdx.x == 0) {
            double E = a.epart[s];
            for (int p = 1; p < P; p++) E += a.epart[(size_t)p * a.gstride + s];
            a.Ep[i] = E;
            const double et = (E - a.Ef[i]) * a.dlam[i] / a.wbar[i];
            a.Et[i] = et;
            a.eb[i].w = et;
            if (!isfinite(E)) atomicOr(&a.flags[1], kErrNonFinite);
        }
        // this atom's reverse slots come from the cache when they were searched on the current list
        // (read by every thread before the barrier; rewritten only after the closing one)
        const int lgen = a.rslot ? *a.list_gen : 0;
        const bool cached = a.rslot && a.rstamp[i] == lgen;
        if (threadIdx.x == 0) sPC[NW] = 0;
        __syncthreads();
        double Lx, Ly, Lz;
        atom_box(a, i, Lx, Ly, Lz);
        const double xi = a.pos[i], yi = a.pos[n + i], zi = a.pos[2 * n + i];
        const int cnt = a.ncount[i];
        T *fo = (T *)a.fpair + (size_t)s * a.max_nbr * 3;
        if (a.stamp && threadIdx.x == 0) a.stamp[i] = a.gen;
        // the slot k of i in j's list (lists are symmetric): j's gather reads the term of the pair at (k, j),
        // coalesced over j. Searched eight entries at a time so that the search is not one long chain.
        auto reverse_slot = [&](int slot, int j) {
            if (cached) return a.rslot[(size_t)i * a.max_nbr + slot];
            int kk = -1;
            const int cj = a.ncount[j];
            for (int b0 = 0; b0 < cj && kk < 0; b0 += 8) {
                int v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) v[u] = b0 + u < cj ? a.nidx[(size_t)(b0 + u) * n + j] : -1;
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (v[u] == i && kk < 0) kk = b0 + u;
            }
            if (a.rslot) a.rslot[(size_t)i * a.max_nbr + slot] = kk;
            return kk;
        };
        // phase 0: every slot; the pairs inside rc compacted in slot order (ballot prefix) into LDS, the
        // others get a zero term here (and their reverse slot when the cache is being filled)
        for (int base = 0; base < cnt; base += kPairThreads) {
            const int slot = base + threadIdx.x;
            bool in = false;
            int j = 0;
            double ux = 0, uy = 0, uz = 0, r2 = 0;
            if (slot < cnt) {
                j = a.nidx[(size_t)slot * n + i];
                if (a.stamp) a.stamp[j] = a.gen;
                const Rec4 pj = a.xl[j];
                ux = min_image_w(pj.x - xi, Lx);
                uy = min_image_w(pj.y - yi, Ly);
                uz = min_image_w(pj.z - zi, Lz);
                r2 = ux * ux + uy * uy + uz * uz;
                in = r2 < rc2;
            }
            const unsigned long long m = __ballot(in);
            const int wv = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 0) sPC[wv] = __popcll(m);
            __syncthreads();
            int p = sPC[NW] + __popcll(m & ((1ull << (threadIdx.x & 63)) - 1ull));
            for (int q = 0; q < wv; q++) p += sPC[q];
            if (in && p < kAceMaxValid) {
                sPS[p] = slot;
                sPJ[p] = j;
                sPU[4 * p] = (T)ux;
                sPU[4 * p + 1] = (T)uy;
                sPU[4 * p + 2] = (T)uz;
                sPR2[p] = r2;
            }
            if (slot < cnt && !in) {
                fo[3 * slot] = T(0);
                fo[3 * slot + 1] = T(0);
                fo[3 * slot + 2] = T(0);
                // (outside rc the term is zero and the gather does not read it; the cache still wants the
                // reverse slot of every pair that can come inside rc before the next build)
                if (r2 < a.rw2 || (a.rslot && !cached && r2 < a.rrev2)) {
                    const int kk = reverse_slot(slot, j);
                    if (kk < 0) {
                        atomicOr(&a.flags[1], kErrAsym);
                    } else if (r2 < a.rw2) {
                        T *fr = (T *)a.frev;
                        const size_t st = (size_t)a.max_nbr * n, o = (size_t)kk * n + j;
                        fr[o] = T(0);
                        fr[st + o] = T(0);
                        fr[2 * st + o] = T(0);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x == 0)
                for (int q = 0; q < NW; q++) sPC[NW] += sPC[q];
            __syncthreads();
        }
        const int nv = min(sPC[NW], kAceMaxValid);
        // phase 1: the pair terms of the compacted pairs, every lane busy
        for (int c = threadIdx.x; c < nv; c += kPairThreads) {
            const int slot = sPS[c], j = sPJ[c];
            const double r2 = sPR2[c];
            T f0 = T(0), f1 = T(0), f2 = T(0);
            {
                const T r = (T)sqrt(r2), ir = T(1) / r;
                const T x = sPU[4 * c] * ir, y = sPU[4 * c + 1] * ir, z = sPU[4 * c + 2] * ir;
                T g[NMAX], dg[NMAX];
                radial<T, NMAX>(r, rcT, g, dg);
                // f = sum_{n, lm} G_{n lm} [g_n'(r) Y_lm uhat + g_n(r) grad_u Y_lm], the harmonics and
                // their gradients generated order by order (the recurrences of ylm_real_grad), so that
                // only the current column of the Legendre recursion is held in registers
                auto term = [&](int lm, T val, T px, T py, T pz) {
                    T sg = T(0), sdg = T(0);
#pragma unroll
                    for (int q = 0; q < NMAX; q += 4) {
                        T G4[4];
                        ld4(sGt + lm * NMAX + q, G4);
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            sg += G4[u] * g[q + u];
                            sdg += G4[u] * dg[q + u];
                        }
                    }
                    const T rad = px * x + py * y + pz * z, t = sdg * val;
                    f0 += t * x + sg * ((px - rad * x) * ir);
                    f1 += t * y + sg * ((py - rad * y) * ir);
                    f2 += t * z + sg * ((pz - rad * z) * ir);
                    // keeps the scheduler from hoisting every coefficient load to the top
                    __builtin_amdgcn_sched_barrier(0);
                };
                const T r2c = T(1.4142135623730951);
                T cp = T(1), sp = T(0), cm = T(1), sm = T(0), dfm = T(1);  // (x + iy)^(m-1), (x + iy)^m
#pragma unroll
                for (int m = 0; m <= LMAX; m++) {
                    if (m > 0) {
                        cp = cm;
                        sp = sm;
                        const T c2 = x * cm - y * sm;
                        sm = x * sm + y * cm;
                        cm = c2;
                        dfm *= T(2 * m - 1);
                    }
                    T q1 = T(0), q2 = T(0), d1 = T(0), d2 = T(0);  // Q_{l-1}^m, Q_{l-2}^m and their z-derivatives
#pragma unroll
                    for (int l = 0; l <= LMAX; l++) {
                        if (l < m) continue;
                        T q, dq;
                        if (l == m) {
                            q = dfm;
                            dq = T(0);
                        } else if (l == m + 1) {
                            q = T(2 * m + 1) * z * q1;
                            dq = T(2 * m + 1) * q1;
                        } else {
                            const T inv = T(1) / T(l - m);
                            q = (T(2 * l - 1) * z * q1 - T(l + m - 1) * q2) * inv;
                            dq = (T(2 * l - 1) * (q1 + z * d1) - T(l + m - 1) * d2) * inv;
                        }
                        q2 = q1;
                        q1 = q;
                        d2 = d1;
                        d1 = dq;
                        if (m == 0) {
                            const T k = klm<T>(l, 0);
                            term(l * l + l, k * q, T(0), T(0), k * dq);
                        } else {
                            const T k = r2c * klm<T>(l, m), kq = k * q, kd = k * dq, mm = T(m);
                            term(l * l + l + m, kq * cm, kq * mm * cp, -kq * mm * sp, kd * cm);
                            term(l * l + l - m, kq * sm, kq * mm * sp, kq * mm * cp, kd * sm);
                        }
                    }
                }
            }
            fo[3 * slot] = f0;
            fo[3 * slot + 1] = f1;
            fo[3 * slot + 2] = f2;
            const bool need = r2 < a.rw2;
            if (!need && !(a.rslot && !cached && r2 < a.rrev2)) continue;
            const int kk = reverse_slot(slot, j);
            if (kk < 0) {
                atomicOr(&a.flags[1], kErrAsym);
            } else if (need) {
                T *fr = (T *)a.frev;
                const size_t st = (size_t)a.max_nbr * n, o = (size_t)kk * n + j;
                fr[o] = f0;
                fr[st + o] = f1;
                fr[2 * st + o] = f2;
            }
        }
        __syncthreads();
        if (a.rslot && !cached && threadIdx.x == 0) a.rstamp[i] = lgen;
    }
}

// ---------------------------------------------------------------------------------------------
// Vector-Jacobian product of the forces with respect to the coefficients: for L = sum_k G_k . F_k,
// dL/dc_nu = -sum_i w_i Bdot_i,nu, where Bdot is the derivative of B_i along the motion r_k -> r_k + t G_k
// (each neighbour vector u_ij moves with G_j - G_i), and dL/db_n the same for xi'(phi2) sqrt(4 pi) A_n00.
// ---------------------------------------------------------------------------------------------
// Per atom: Adot[n][lm] = sum_j [g_n'(r) (uhat . t) Y_lm + g_n(r) (grad_u Y_lm . t)], t = G_j - G_i, into
// a.gpart (row s). One lane per neighbour inside rc evaluates its radial channels and, order by order, the
// harmonics and their derivative along t into LDS; the workgroup then sums over the chunk's neighbours.
template <typename T, int NMAX, int LMAX>
__global__ __launch_bounds__(kBlock) void k_ace_tangent(AceArgs a, const double *__restrict__ G) {
    // neighbours per chunk: 64 in FP32, 32 in FP64 (the chunk's tables stay under 64 KB of LDS)
    constexpr int NLM = (LMAX + 1) * (LMAX + 1), NA = NMAX * NLM, CH = sizeof(T) == 4 ? 64 : 32;
    __shared__ T sR0[CH * NMAX], sR1[CH * NMAX], sY[CH * NLM], sYd[CH * NLM];
    __shared__ T sAd[NA];
    __shared__ int sJ[kAceMaxValid];
    __shared__ int sCnt[5];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = a.n;
    const int S = *a.scount;
    const double rc2 = a.rc * a.rc;
    const T rcT = (T)a.rc;
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int i = a.slist[s];
        const double xi = a.pos[i], yi = a.pos[n + i], zi = a.pos[2 * n + i];
        double Lx, Ly, Lz;
        atom_box(a, i, Lx, Ly, Lz);
        const int cnt = a.ncount[i];
        if (tid == 0) sCnt[4] = 0;
        for (int o = tid; o < NA; o += kBlock) sAd[o] = T(0);
        __syncthreads();
        // neighbours inside rc, compacted in list order
        for (int base = 0; base < cnt; base += kBlock) {
            const int slot = base + tid;
            bool valid = false;
            int j = 0;
            if (slot < cnt) {
                j = a.nidx[(size_t)slot * n + i];
                const Rec4 pj = a.xl[j];
                const double ux = min_image_w(pj.x - xi, Lx), uy = min_image_w(pj.y - yi, Ly),
                             uz = min_image_w(pj.z - zi, Lz);
                valid = ux * ux + uy * uy + uz * uz < rc2;
            }
            const unsigned long long m = __ballot(valid);
            if (lane == 0) sCnt[wv] = __popcll(m);
            __syncthreads();
            int off = sCnt[4];
            for (int q = 0; q < wv; q++) off += sCnt[q];
            const int p = off + __popcll(m & ((1ull << lane) - 1ull));
            if (valid) {
                if (p < kAceMaxValid)
                    sJ[p] = j;
                else
                    atomicOr(&a.flags[1], kErrAceNbr);
            }
            __syncthreads();
            if (tid == 0) sCnt[4] += sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
            __syncthreads();
        }
        const int nv = min(sCnt[4], kAceMaxValid);
        const double gxi = G[i], gyi = G[n + i], gzi = G[2 * n + i];
        for (int v0 = 0; v0 < nv; v0 += CH) {
            const int nc = min(CH, nv - v0);
            if (wv == 0 && lane < nc) {
                const int j = sJ[v0 + lane];
                const Rec4 pj = a.xl[j];
                const double ux = min_image_w(pj.x - xi, Lx), uy = min_image_w(pj.y - yi, Ly),
                             uz = min_image_w(pj.z - zi, Lz);
                const double rd = sqrt(ux * ux + uy * uy + uz * uz);
                const T r = (T)rd, ir = (T)(1.0 / rd);
                const T x = (T)ux * ir, y = (T)uy * ir, z = (T)uz * ir;
                const T tx = (T)(G[j] - gxi), ty = (T)(G[n + j] - gyi), tz = (T)(G[2 * n + j] - gzi);
                const T rdot = x * tx + y * ty + z * tz;  // d|u|/dt
                T g[NMAX], dg[NMAX];
                radial<T, NMAX>(r, rcT, g, dg);
#pragma unroll
                for (int q = 0; q < NMAX; q++) {
                    sR0[lane * NMAX + q] = g[q];
                    sR1[lane * NMAX + q] = dg[q] * rdot;
                }
                // harmonics order by order (the recurrences of ylm_real_grad): value, and grad_u Y . t =
                // (grad_p . t - (grad_p . uhat)(uhat . t)) / r for the polynomial p
                auto put = [&](int lm, T val, T px, T py, T pz) {
                    const T rad = px * x + py * y + pz * z;
                    sY[lane * NLM + lm] = val;
                    sYd[lane * NLM + lm] = (px * tx + py * ty + pz * tz - rad * rdot) * ir;
                };
                const T r2c = T(1.4142135623730951);
                T cp = T(1), sp = T(0), cm = T(1), sm = T(0), dfm = T(1);
#pragma unroll
                for (int mm = 0; mm <= LMAX; mm++) {
                    if (mm > 0) {
                        cp = cm;
                        sp = sm;
                        const T c2 = x * cm - y * sm;
                        sm = x * sm + y * cm;
                        cm = c2;
                        dfm *= T(2 * mm - 1);
                    }
                    T q1 = T(0), q2 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
                    for (int l = 0; l <= LMAX; l++) {
                        if (l < mm) continue;
                        T q, dq;
                        if (l == mm) {
                            q = dfm;
                            dq = T(0);
                        } else if (l == mm + 1) {
                            q = T(2 * mm + 1) * z * q1;
                            dq = T(2 * mm + 1) * q1;
                        } else {
                            const T inv = T(1) / T(l - mm);
                            q = (T(2 * l - 1) * z * q1 - T(l + mm - 1) * q2) * inv;
                            dq = (T(2 * l - 1) * (q1 + z * d1) - T(l + mm - 1) * d2) * inv;
                        }
                        q2 = q1;
                        q1 = q;
                        d2 = d1;
                        d1 = dq;
                        if (mm == 0) {
                            const T k = klm<T>(l, 0);
                            put(l * l + l, k * q, T(0), T(0), k * dq);
                        } else {
                            const T k = r2c * klm<T>(l, mm), kq = k * q, kd = k * dq, fm = T(mm);
                            put(l * l + l + mm, kq * cm, kq * fm * cp, -kq * fm * sp, kd * cm);
                            put(l * l + l - mm, kq * sm, kq * fm * sp, kq * fm * cp, kd * sm);
                        }
                    }
                }
            }
            __syncthreads();
            for (int o = tid; o < NA; o += kBlock) {
                const int q = o / NLM, lm = o - q * NLM;
                T acc = sAd[o];
                for (int v = 0; v < nc; v++)
                    acc += sR1[v * NMAX + q] * sY[v * NLM + lm] + sR0[v * NMAX + q] * sYd[v * NLM + lm];
                sAd[o] = acc;
            }
            __syncthreads();
        }
        T *out = (T *)a.gpart + (size_t)s * NA;
        for (int o = tid; o < NA; o += kBlock) out[o] = sAd[o];
        __syncthreads();
    }
}

// Per atom: Bdot of every basis function from A (a.gbuf) and Adot (a.gpart), written with the density
// tangents into a.bval: orders 1 and 2 directly, order 3 per coupling block from P_M and its tangent
// Pdot_M = sum kappa (Adot1 A2 + A1 Adot2): Bdot = sum_M Pdot_M[n1 n2] A[n3][L M] + P_M[n1 n2] Adot[n3][L M].
template <typename T, int NMAX, int LMAX>
__global__ __launch_bounds__(kBlock) void k_ace_bdot(AceArgs a) {
    constexpr int NLM = (LMAX + 1) * (LMAX + 1), NA = NMAX * NLM, NN = NMAX * NMAX, MM = 2 * LMAX + 1;
    __shared__ T sA[NA], sAt[NA], sAd[NA], sAdt[NA];
    __shared__ T sP[MM * NN], sPd[MM * NN];
    __shared__ T skv[kKapStage];
    __shared__ int skc[kKapStage];
    const int tid = threadIdx.x;
    const int S = *a.scount;
    const T *kval = (const T *)a.kval;
    const double s4pi = 3.5449077018110318;  // sqrt(4 pi)
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const T *ain = (const T *)a.gbuf + (size_t)s * NA;
        const T *adin = (const T *)a.gpart + (size_t)s * NA;
        for (int o = tid; o < NA; o += kBlock) {
            const int q = o / NLM, lm = o - q * NLM;
            const T v = ain[o], vd = adin[o];
            sA[o] = v;
            sAt[lm * NMAX + q] = v;
            sAd[o] = vd;
            sAdt[lm * NMAX + q] = vd;
        }
        __syncthreads();
        T *bout = (T *)a.bval + (size_t)s * a.bstride;
        for (int q = tid; q < a.ng1; q += kBlock) bout[a.g1[2 * q + 1]] = sAd[a.g1[2 * q] * NLM];
        for (int q = tid; q < a.ng2; q += kBlock) {
            const int code = a.g2[2 * q];
            const int q1 = code & 255, q2 = (code >> 8) & 255, l = code >> 16;
            T bsum = T(0);
            for (int m = l * l; m <= l * l + 2 * l; m++)
                bsum += sAd[q1 * NLM + m] * sA[q2 * NLM + m] + sA[q1 * NLM + m] * sAd[q2 * NLM + m];
            bout[a.g2[2 * q + 1]] = bsum;
        }
        if (tid == 0) {
            // the density term's tangent (the l = 0 radial sums in FP64): s_n = sqrt(4 pi) A_n00
            const double *s0 = a.s0buf + (size_t)s * NMAX;
            double phi2 = 0.0, phi2d = 0.0;
            for (int q = 0; q < NMAX; q++) {
                phi2 += a.bdd[q] * s0[q];
                phi2d += a.bdd[q] * s4pi * (double)sAd[q * NLM];
            }
            double d1 = 0.0, d2 = 0.0;
            if (phi2 > 0.0) {
                d1 = -0.5 * a.emb_A / sqrt(phi2);
                d2 = 0.25 * a.emb_A / (phi2 * sqrt(phi2));
            }
            for (int q = 0; q < NMAX; q++)
                bout[a.n_funcs + q] = (T)(d2 * phi2d * s0[q] + d1 * s4pi * (double)sAd[q * NLM]);
        }
        for (int b = 0; b < a.nblk; b++) {
            const int *bk = a.blk + b * kBlkInts;
            const int L = bk[0];
            const int nM = 2 * L + 1, bL = L * L + L;
            const int k0 = bk[4], k1 = bk[4 + nM];
            __syncthreads();
            for (int q = k0 + tid; q < k1; q += kBlock) {
                skc[q - k0] = a.kidx[q];
                skv[q - k0] = kval[q];
            }
            __syncthreads();
            for (int w = tid; w < nM * NMAX; w += kBlock) {
                const int Mi = w / NMAX, n1 = w - Mi * NMAX;
                T P[NMAX], Pd[NMAX];
#pragma unroll
                for (int q = 0; q < NMAX; q++) P[q] = Pd[q] = T(0);
                const int e0 = bk[4 + Mi] - k0, e1 = bk[4 + Mi + 1] - k0;
                for (int q = e0; q < e1; q++) {
                    const int code = skc[q];
                    const T kv = skv[q];
                    const T a1 = kv * sA[n1 * NLM + (code & 255)], ad1 = kv * sAd[n1 * NLM + (code & 255)];
                    const T *a2 = sAt + 4 * (code >> 8), *ad2 = sAdt + 4 * (code >> 8);
#pragma unroll
                    for (int q2 = 0; q2 < NMAX; q2++) {
                        P[q2] += a1 * a2[q2];
                        Pd[q2] += ad1 * a2[q2] + a1 * ad2[q2];
                    }
                }
#pragma unroll
                for (int q2 = 0; q2 < NMAX; q2++) {
                    sP[Mi * NN + n1 * NMAX + q2] = P[q2];
                    sPd[Mi * NN + n1 * NMAX + q2] = Pd[q2];
                }
            }
            __syncthreads();
            for (int q = bk[46] + tid; q < bk[47]; q += kBlock) {
                const int code = a.g3[2 * q];
                const int rem = code & 0xffff, q3 = code >> 16;
                T bsum = T(0);
                for (int Mi = 0; Mi < nM; Mi++)
                    bsum += sPd[Mi * NN + rem] * sA[q3 * NLM + bL + Mi - L] + sP[Mi * NN + rem] * sAd[q3 * NLM + bL + Mi - L];
                bout[a.g3[2 * q + 1]] = bsum;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Host: tables
// ---------------------------------------------------------------------------------------------
static double w3j000(int l1, int l2, int l3) {
    const int J = l1 + l2 + l3;
    if (J % 2) return 0.0;
    const int g = J / 2;
    auto f = [](int k) {
        double r = 1;
        for (int q = 2; q <= k; q++) r *= q;
        return r;
    };
    const double s = (g % 2) ? -1.0 : 1.0;
    return s * std::sqrt(f(J - 2 * l1) * f(J - 2 * l2) * f(J - 2 * l3) / f(J + 1)) * f(g) /
           (f(g - l1) * f(g - l2) * f(g - l3));
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int npt, std::vector<double> &x, std::vector<double> &w) {
    x.resize(npt);
    w.resize(npt);
    for (int k = 0; k < npt; k++) {
        double t = std::cos(kPi * (k + 0.75) / (npt + 0.5));
        for (int it = 0; it < 100; it++) {
            double p0 = 1, p1 = t;
            for (int q = 2; q <= npt; q++) {
                double p2 = ((2 * q - 1) * t * p1 - (q - 1) * p0) / q;
                p0 = p1;
                p1 = p2;
            }
            const double dp = npt * (t * p1 - p0) / (t * t - 1);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1, p1 = t;
        for (int q = 2; q <= npt; q++) {
            double p2 = ((2 * q - 1) * t * p1 - (q - 1) * p0) / q;
            p0 = p1;
            p1 = p2;
        }
        const double dp = npt * (t * p1 - p0) / (t * t - 1);
        x[k] = t;
        w[k] = 2.0 / ((1 - t * t) * dp * dp);
    }
}

struct Kap {
    int m1, m2, M;
    double v;
};

// kappa(l1 m1, l2 m2, L M) for every (m1, m2, M): real Gaunt integral / (N3 (l1 l2 L; 0 0 0)).
static std::vector<Kap> coupling(int l1, int l2, int L) {
    const int nth = 16, nph = 32;
    std::vector<double> x, w;
    gauss_legendre(nth, x, w);
    constexpr int NLM = 49;
    std::vector<Kap> out;
    const double N3 = std::sqrt((2.0 * l1 + 1) * (2.0 * l2 + 1) * (2.0 * L + 1) / (4 * kPi)) * w3j000(l1, l2, L);
    std::vector<double> G((2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1), 0.0);
    for (int a = 0; a < nth; a++)
        for (int b = 0; b < nph; b++) {
            const double ph = 2 * kPi * b / nph, st = std::sqrt(1 - x[a] * x[a]);
            double Y[NLM];
            ylm_real<double, 6>(st * std::cos(ph), st * std::sin(ph), x[a], Y);
            const double wq = w[a] * 2 * kPi / nph;
            for (int m1 = -l1; m1 <= l1; m1++)
                for (int m2 = -l2; m2 <= l2; m2++)
                    for (int M = -L; M <= L; M++)
                        G[((m1 + l1) * (2 * l2 + 1) + (m2 + l2)) * (2 * L + 1) + (M + L)] +=
                            wq * Y[l1 * l1 + l1 + m1] * Y[l2 * l2 + l2 + m2] * Y[L * L + L + M];
        }
    for (int m1 = -l1; m1 <= l1; m1++)
        for (int m2 = -l2; m2 <= l2; m2++)
            for (int M = -L; M <= L; M++) {
                const double g = G[((m1 + l1) * (2 * l2 + 1) + (m2 + l2)) * (2 * L + 1) + (M + L)];
                if (std::fabs(g) > 1e-12) out.push_back({m1, m2, M, g / N3});
            }
    return out;
}

template <typename T>
static int upload(ap_ctx *c, void **dst, const std::vector<double> &src) {
    std::vector<T> h(src.begin(), src.end());
    if (h.empty()) h.push_back(T(0));
    int rc = hip_check(c, hipMalloc(dst, sizeof(T) * h.size()), "ace tables");
    if (!rc) rc = hip_check(c, hipMemcpy(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice), "ace tables");
    return rc;
}

void ace_free(ap_ctx *c) {
    AceTables &t = c->ace;
    (void)hipFree(t.c1);
    (void)hipFree(t.bd);
    (void)hipFree(t.c1d);
    (void)hipFree(t.bdd);
    (void)hipFree(t.g1);
    (void)hipFree(t.g2);
    (void)hipFree(t.g3);
    (void)hipFree(t.c2);
    (void)hipFree(t.c3);
    (void)hipFree(t.kval);
    (void)hipFree(t.kidx);
    (void)hipFree(t.blk);
    (void)hipFree(t.c30);
    (void)hipFree(t.kap0);
    (void)hipFree(t.cmap_f);
    (void)hipFree(t.cmap_w);
    t = AceTables();
}

// New coefficients into the installed tables (ap_set_ace_coefficients): every table element takes factor x
// c[function] from its gather map, in the precision of the tables; the density coefficients likewise.
template <typename T>
__global__ void k_coeff_gather(const int *__restrict__ fm, const double *__restrict__ wm, const double *__restrict__ cf,
                               int nmap, int n1, int n2, int n3, T *c1, double *c1d, T *c2, T *c3, T *c30) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nmap) return;
    const int f = fm[e];
    const double v = f >= 0 ? wm[e] * cf[f] : 0.0;
    if (e < n1) {
        c1[e] = (T)v;
        c1d[e] = v;
    } else if (e < n1 + n2) {
        c2[e - n1] = (T)v;
    } else if (e < n1 + n2 + n3) {
        c3[e - n1 - n2] = (T)v;
    } else {
        c30[e - n1 - n2 - n3] = (T)v;
    }
}

template <typename T>
__global__ void k_dens_gather(const double *__restrict__ b, int n, T *bd, double *bdd) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    bd[q] = (T)(b[q] * std::sqrt(4 * kPi));
    bdd[q] = b[q];
}

int ace_set_coefficients(ap_ctx *c, const double *cf, const double *b) {
    AceTables &t = c->ace;
    if (cf) {
        if (t.nmap == 0) return set_error(c, AP_E_ARG, "the installed basis has repeated rows: use ap_set_potential");
        const int g = (t.nmap + kBlock - 1) / kBlock;
        if (t.precision == AP_FP32)
            k_coeff_gather<float><<<g, kBlock, 0, c->stream>>>(t.cmap_f, t.cmap_w, cf, t.nmap, t.n_max, t.n_c2, t.n_c3,
                                                               (float *)t.c1, t.c1d, (float *)t.c2, (float *)t.c3,
                                                               (float *)t.c30);
        else
            k_coeff_gather<double><<<g, kBlock, 0, c->stream>>>(t.cmap_f, t.cmap_w, cf, t.nmap, t.n_max, t.n_c2,
                                                                t.n_c3, (double *)t.c1, t.c1d, (double *)t.c2,
                                                                (double *)t.c3, (double *)t.c30);
    }
    if (b) {
        if (t.precision == AP_FP32)
            k_dens_gather<float><<<1, kBlock, 0, c->stream>>>(b, t.n_max, (float *)t.bd, t.bdd);
        else
            k_dens_gather<double><<<1, kBlock, 0, c->stream>>>(b, t.n_max, (double *)t.bd, t.bdd);
    }
    return hip_check(c, hipGetLastError(), "coefficients");
}

int ace_setup(ap_ctx *c, const ap_ace_params *p) {
    const int N = p->n_max, Lm = p->l_max;
    if (!((N == 4 && Lm == 2) || (N == 8 && Lm == 4) || (N == 12 && Lm == 6)))
        return set_error(c, AP_E_ARG, "supported (n_max, l_max): (4,2), (8,4), (12,6)");
    if (p->precision != AP_FP64 && p->precision != AP_FP32) return set_error(c, AP_E_ARG, "precision");
    if (p->n_funcs < 0 || (p->n_funcs > 0 && (!p->func || !p->c)) || !p->b_dens)
        return set_error(c, AP_E_ARG, "ACE tables");
    ace_free(c);
    AceTables &t = c->ace;
    t.n_max = N;
    t.l_max = Lm;
    t.n_funcs = p->n_funcs;
    t.precision = p->precision;
    t.rc = p->rc;
    t.emb_A = p->emb_A;
    t.E0 = p->E0;
    std::vector<double> c1(N, 0.0), bd(N, 0.0), c2((size_t)(Lm + 1) * N * N, 0.0);
    for (int q = 0; q < N; q++) bd[q] = p->b_dens[q] * std::sqrt(4 * kPi);
    // blocks (L <= l1 <= l2)
    struct Blk {
        int L, l1, l2;
    };
    std::vector<Blk> blocks;
    std::vector<int> bindex((Lm + 1) * (Lm + 1) * (Lm + 1), -1);
    for (int L = 0; L <= Lm; L++)
        for (int l1 = L; l1 <= Lm; l1++)
            for (int l2 = l1; l2 <= Lm; l2++)
                if ((L + l1 + l2) % 2 == 0 && l2 <= l1 + L) {
                    bindex[(L * (Lm + 1) + l1) * (Lm + 1) + l2] = (int)blocks.size();
                    blocks.push_back({L, l1, l2});
                }
    std::vector<double> c3(blocks.size() * (size_t)N * N * N, 0.0);
    std::vector<char> used(blocks.size(), 0);
    // where every coefficient lands (for ap_set_ace_coefficients): per table element the function and its
    // factor, -1 where none (every element takes at most one function: the basis rows are distinct sorted
    // (n, l) triples)
    std::vector<int> f1(N, -1), f2((size_t)(Lm + 1) * N * N, -1), f3(blocks.size() * (size_t)N * N * N, -1);
    std::vector<double> w2((size_t)(Lm + 1) * N * N, 0.0), w3(blocks.size() * (size_t)N * N * N, 0.0);
    bool map_ok = true;  // false when two rows land on one element (repeated rows): no device update then
    // gradient lists (function index nu with where its B value lives): order 1 (n, nu),
    // order 2 (n1 | n2 << 8 | l << 16, nu), order 3 per block (n1 * N + n2 | n3 << 16, nu)
    std::vector<int> g1, g2;
    std::vector<std::vector<int>> g3(blocks.size());
    for (int f = 0; f < p->n_funcs; f++) {
        const int32_t *r = p->func + 6 * f;
        const double cf = p->c[f];
        if (r[2] < 0) {
            if (r[0] < 0 || r[0] >= N || r[1] != 0) return set_error(c, AP_E_ARG, "order-1 basis row");
            c1[r[0]] += cf;
            if (f1[r[0]] >= 0) map_ok = false;
            f1[r[0]] = f;
            g1.push_back(r[0]);
            g1.push_back(f);
        } else if (r[4] < 0) {
            const int n1 = r[0], l = r[1], n2 = r[2];
            if (r[3] != l || l < 0 || l > Lm || n1 < 0 || n2 < 0 || n1 >= N || n2 >= N)
                return set_error(c, AP_E_ARG, "order-2 basis row");
            g2.push_back(n1 | (n2 << 8) | (l << 16));
            g2.push_back(f);
            if (f2[((size_t)l * N + n1) * N + n2] >= 0) map_ok = false;
            if (n1 == n2) {
                c2[((size_t)l * N + n1) * N + n2] += cf;
                f2[((size_t)l * N + n1) * N + n2] = f;
                w2[((size_t)l * N + n1) * N + n2] = 1.0;
            } else {
                c2[((size_t)l * N + n1) * N + n2] += 0.5 * cf;
                c2[((size_t)l * N + n2) * N + n1] += 0.5 * cf;
                for (const size_t e : {((size_t)l * N + n1) * N + n2, ((size_t)l * N + n2) * N + n1}) {
                    f2[e] = f;
                    w2[e] = 0.5;
                }
            }
        } else {
            int ln[3][2] = {{r[1], r[0]}, {r[3], r[2]}, {r[5], r[4]}};
            for (int q = 0; q < 3; q++)
                if (ln[q][0] < 0 || ln[q][0] > Lm || ln[q][1] < 0 || ln[q][1] >= N)
                    return set_error(c, AP_E_ARG, "order-3 basis row");
            // stable sort of the three channels by l
            for (int a = 1; a < 3; a++)
                for (int q = a; q > 0 && ln[q][0] < ln[q - 1][0]; q--) {
                    std::swap(ln[q][0], ln[q - 1][0]);
                    std::swap(ln[q][1], ln[q - 1][1]);
                }
            const int L = ln[0][0], l1 = ln[1][0], l2 = ln[2][0];
            const int bi = bindex[(L * (Lm + 1) + l1) * (Lm + 1) + l2];
            if (bi < 0) return set_error(c, AP_E_ARG, "order-3 row violates the triangle or parity rule");
            c3[(((size_t)bi * N + ln[1][1]) * N + ln[2][1]) * N + ln[0][1]] += cf;
            if (f3[(((size_t)bi * N + ln[1][1]) * N + ln[2][1]) * N + ln[0][1]] >= 0) map_ok = false;
            f3[(((size_t)bi * N + ln[1][1]) * N + ln[2][1]) * N + ln[0][1]] = f;
            w3[(((size_t)bi * N + ln[1][1]) * N + ln[2][1]) * N + ln[0][1]] = 1.0;
            used[bi] = 1;
            g3[bi].push_back((ln[1][1] * N + ln[2][1]) | (ln[0][1] << 16));
            g3[bi].push_back(f);
        }
    }
    // (L, l, l) blocks: the coefficients symmetrised in (n1, n2), which leaves every energy unchanged (P_M
    // is symmetric there) and makes Q_M symmetric, so that the energy kernel takes both coupling adjoints
    // in one pass
    for (size_t bi = 0; bi < blocks.size(); bi++) {
        if (blocks[bi].l1 != blocks[bi].l2) continue;
        double *cb = c3.data() + bi * (size_t)N * N * N;
        for (int n1 = 0; n1 < N; n1++)
            for (int n2 = n1 + 1; n2 < N; n2++)
                for (int n3 = 0; n3 < N; n3++) {
                    const size_t eu = bi * (size_t)N * N * N + ((size_t)n1 * N + n2) * N + n3,
                                 ev = bi * (size_t)N * N * N + ((size_t)n2 * N + n1) * N + n3;
                    double &u = cb[((size_t)n1 * N + n2) * N + n3], &v = cb[((size_t)n2 * N + n1) * N + n3];
                    const double m = 0.5 * (u + v);
                    u = m;
                    v = m;
                    // both elements take half of the one function that lands on either
                    const int fu = f3[eu] >= 0 ? f3[eu] : f3[ev];
                    f3[eu] = f3[ev] = fu;
                    w3[eu] = w3[ev] = fu >= 0 ? 0.5 : 0.0;
                }
    }
    std::vector<int> g3flat;
    // keep only blocks with coefficients; build coupling tables in three orderings
    std::vector<int> hblk;
    std::vector<int> kidx;
    const int esz = p->precision == AP_FP32 ? 4 : 8;  // element size of the tables' precision
    if (N % 4 != 0 || (2 * Lm + 1) * N * N * esz >= (1 << 16))
        return set_error(c, AP_E_ARG, "n_max must be a multiple of 4 and at most 12");
    std::vector<double> c30((size_t)(Lm + 1) * N * N * N, 0.0), kap0(Lm + 1, 0.0);
    bool fold0 = true;
    std::vector<double> kval, c3u;
    std::vector<int> f3u, f30((size_t)(Lm + 1) * N * N * N, -1);
    std::vector<double> w3u, w30((size_t)(Lm + 1) * N * N * N, 0.0);
    int nb = 0;
    for (size_t bi = 0; bi < blocks.size(); bi++) {
        if (!used[bi]) continue;
        const Blk &B = blocks[bi];
        std::vector<Kap> k = coupling(B.l1, B.l2, B.L);
        if (B.L == 0) {
            // (0, l, l): one coupling value on the diagonal m1 = m2 with M = 0, or no closed form
            bool diag = (int)k.size() == 2 * B.l1 + 1;
            for (const Kap &e : k)
                diag = diag && e.M == 0 && e.m1 == e.m2 && std::fabs(e.v - k[0].v) <= 1e-14 * std::fabs(k[0].v);
            if (diag) {
                kap0[B.l1] = k[0].v;
                std::copy(c3.begin() + bi * (size_t)N * N * N, c3.begin() + (bi + 1) * (size_t)N * N * N,
                          c30.begin() + (size_t)B.l1 * N * N * N);
                std::copy(f3.begin() + bi * (size_t)N * N * N, f3.begin() + (bi + 1) * (size_t)N * N * N,
                          f30.begin() + (size_t)B.l1 * N * N * N);
                std::copy(w3.begin() + bi * (size_t)N * N * N, w3.begin() + (bi + 1) * (size_t)N * N * N,
                          w30.begin() + (size_t)B.l1 * N * N * N);
            } else {
                fold0 = false;
            }
        }
        std::vector<int> d(kBlkInts, 0);
        d[0] = B.L;
        d[1] = B.l1;
        d[2] = B.l2;
        d[3] = (int)c3u.size();
        c3u.insert(c3u.end(), c3.begin() + bi * (size_t)N * N * N, c3.begin() + (bi + 1) * (size_t)N * N * N);
        f3u.insert(f3u.end(), f3.begin() + bi * (size_t)N * N * N, f3.begin() + (bi + 1) * (size_t)N * N * N);
        w3u.insert(w3u.end(), w3.begin() + bi * (size_t)N * N * N, w3.begin() + (bi + 1) * (size_t)N * N * N);
        auto emit = [&](int base, int key_lo, int key_hi, int which) {
            for (int key = key_lo; key <= key_hi; key++) {
                d[base + key - key_lo] = (int)kidx.size();
                for (const Kap &e : k) {
                    const int kv = which == 0 ? e.M : (which == 1 ? e.m1 : e.m2);
                    if (kv != key) continue;
                    // LDS offsets the kernel uses directly: by M, the column l1 m1 of A and the row
                    // l2 m2 of its transpose (the row in units of four elements); by m1 (m2), the byte offsets
                    // of the row l2 m2 (l1 m1) of the transpose and, in the upper half, of the matrix Q_M,
                    // multiples of 16 below 2^16 (n_max is a multiple of 4 and at most 12)
                    const int c1 = B.l1 * B.l1 + B.l1 + e.m1, c2 = B.l2 * B.l2 + B.l2 + e.m2;
                    const int r2 = c2 * N / 4;
                    const int qmb = (e.M + B.L) * N * N * esz, r1b = c1 * N * esz, r2b = c2 * N * esz;
                    kidx.push_back(which == 0 ? c1 | (r2 << 8) : (which == 1 ? r2b | (qmb << 16) : r1b | (qmb << 16)));
                    kval.push_back(e.v);
                }
            }
            d[base + key_hi - key_lo + 1] = (int)kidx.size();
        };
        emit(4, -B.L, B.L, 0);
        emit(18, -B.l1, B.l1, 1);
        emit(32, -B.l2, B.l2, 2);
        if ((int)kidx.size() - d[4] > kKapStage) return set_error(c, AP_E_ARG, "coupling block too large for LDS");
        d[46] = (int)g3flat.size() / 2;
        g3flat.insert(g3flat.end(), g3[bi].begin(), g3[bi].end());
        d[47] = (int)g3flat.size() / 2;
        hblk.insert(hblk.end(), d.begin(), d.end());
        nb++;
    }
    t.nblk = nb;
    t.h_blk = hblk;
    // the parts of a split atom get equal numbers of the blocks they run (each block is about one step
    // of the per-atom chain, whatever its size; the L = 0 blocks, first in the table, are folded into
    // order 2 unless coefficient gradients are asked for); the first part also takes orders 1-2
    {
        int n0 = 0;
        while (n0 < nb && hblk[(size_t)n0 * kBlkInts] == 0) n0++;
        t.n0 = n0;
    }
    t.ng1 = (int)g1.size() / 2;
    t.ng2 = (int)g2.size() / 2;
    int rc;
    auto up_int = [&](int **dst, std::vector<int> v) {
        if (v.empty()) v.push_back(0);
        int r = hip_check(c, hipMalloc(dst, sizeof(int) * v.size()), "ace tables");
        if (!r) r = hip_check(c, hipMemcpy(*dst, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice), "ace");
        return r;
    };
    rc = up_int(&t.g1, g1);
    if (!rc) rc = up_int(&t.g2, g2);
    if (!rc) rc = up_int(&t.g3, g3flat);
    if (rc) return rc;
    if (p->precision == AP_FP32) {
        rc = upload<float>(c, &t.c1, c1);
        if (!rc) rc = upload<float>(c, &t.bd, bd);
        if (!rc) rc = upload<float>(c, &t.c2, c2);
        if (!rc) rc = upload<float>(c, &t.c3, c3u);
        if (!rc) rc = upload<float>(c, &t.kval, kval);
    } else {
        rc = upload<double>(c, &t.c1, c1);
        if (!rc) rc = upload<double>(c, &t.bd, bd);
        if (!rc) rc = upload<double>(c, &t.c2, c2);
        if (!rc) rc = upload<double>(c, &t.c3, c3u);
        if (!rc) rc = upload<double>(c, &t.kval, kval);
    }
    if (!rc && fold0) {
        if (p->precision == AP_FP32) {
            rc = upload<float>(c, &t.c30, c30);
            if (!rc) rc = upload<float>(c, &t.kap0, kap0);
        } else {
            rc = upload<double>(c, &t.c30, c30);
            if (!rc) rc = upload<double>(c, &t.kap0, kap0);
        }
    }
    // the gather maps of ap_set_ace_coefficients, in table order: c1, c2, c3 (used blocks), c30 when folded
    {
        std::vector<int> fm;
        std::vector<double> wm;
        auto add = [&](const std::vector<int> &ff, const std::vector<double> &ww) {
            fm.insert(fm.end(), ff.begin(), ff.end());
            wm.insert(wm.end(), ww.begin(), ww.end());
        };
        add(f1, std::vector<double>(N, 1.0));
        add(f2, w2);
        add(f3u, w3u);
        if (fold0) add(f30, w30);
        t.nmap = map_ok ? (int)fm.size() : 0;
        t.n_c2 = (int)f2.size();
        t.n_c3 = (int)f3u.size();
        t.n_c30 = fold0 ? (int)f30.size() : 0;
        if (!rc) rc = up_int(&t.cmap_f, fm);
        if (!rc) rc = upload<double>(c, (void **)&t.cmap_w, wm);
    }
    if (!rc) rc = upload<double>(c, (void **)&t.c1d, c1);
    if (!rc) rc = upload<double>(c, (void **)&t.bdd, std::vector<double>(p->b_dens, p->b_dens + N));
    if (rc) return rc;
    if (kidx.empty()) kidx.push_back(0);
    if (hblk.empty()) hblk.push_back(0);
    rc = hip_check(c, hipMalloc(&t.kidx, sizeof(int) * kidx.size()), "ace tables");
    if (!rc) rc = hip_check(c, hipMemcpy(t.kidx, kidx.data(), sizeof(int) * kidx.size(), hipMemcpyHostToDevice), "ace");
    if (!rc) rc = hip_check(c, hipMalloc(&t.blk, sizeof(int) * hblk.size()), "ace tables");
    if (!rc) rc = hip_check(c, hipMemcpy(t.blk, hblk.data(), sizeof(int) * hblk.size(), hipMemcpyHostToDevice), "ace");
    return rc;
}

template <typename T, int NMAX, int LMAX>
static void launch_t(ap_ctx *c, AceArgs a, int grid) {
    {
        // workgroups of the energy kernel resident at once: the rounds the split decision counts (taken
        // once per device for each instantiation)
        static int dev = -1, slots = 0;
        if (dev != c->device) {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ace_energy<T, NMAX, LMAX>, kBlock, 0) !=
                    hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
                per_cu = cus = 0;
            slots = per_cu > 0 && cus > 0 ? per_cu * cus : 1 << 30;
            dev = c->device;
        }
        a.slots = slots;
    }
    {
        ProfScope p(c, "ace_basis");
        k_ace_basis<T, NMAX, LMAX><<<grid, kBlock, 0, c->stream>>>(a);
    }
    {
        ProfScope p(c, "ace_energy");
        // a persistent grid: the resident workgroups, which take the work items from the counter
        const int eg = a.slots < (1 << 30) ? a.slots : 2 * grid;
        k_ace_energy<T, NMAX, LMAX><<<eg, kBlock, 0, c->stream>>>(a);
    }
    ProfScope p(c, "ace_pairforce");
    k_ace_pairforce<T, NMAX, LMAX><<<grid, kPairThreads, 0, c->stream>>>(a);
}

// Floating-point operations of the ACE kernels, counted from the tables: per S atom independent of
// the neighbour count (orders 2 and 3 with their adjoints), per neighbour inside rc in the energy
// kernel (radial channels, harmonics, A accumulation) and per neighbour in the pair-gradient kernel.
void ace_cost(const ap_ctx *c, double *fixed, double *per_nbr_energy, double *per_nbr_force) {
    const AceTables &t = c->ace;
    const double N = t.n_max, NLM = (t.l_max + 1.0) * (t.l_max + 1.0), NA = N * NLM, NN = N * N;
    double f = NA * (2.0 * N + 4.0);  // order 2 value and adjoint
    for (int b = 0; b < t.nblk; b++) {
        const int *d = t.h_blk.data() + b * kBlkInts;
        const int L = d[0], l1 = d[1], l2 = d[2];
        const double nkap = d[4 + 2 * L + 1] - d[4];
        f += NN * nkap * 3.0;                          // P
        f += (2 * L + 1) * NN * (2.0 * N + 2.0);       // Q and the energy P.Q
        f += N * (2 * L + 1) * NN * 2.0;               // adjoint into A_{n3 L M}
        // adjoints into A_{n1 l1} and A_{n2 l2}: one pass when l1 = l2 (symmetric couplings and
        // coefficients make the two equal)
        f += N * nkap * (2.0 * N + 2.0) * (l1 == l2 ? 1.0 : 2.0);
    }
    *fixed = f;
    *per_nbr_energy = 2.0 * NA + 8.0 * N + 10.0 * NLM;
    *per_nbr_force = NLM * (4.0 * N + 12.0) + 6.0 * N + 20.0 * NLM;
}

static AceArgs ace_args(ap_ctx *c, int n, const double *box, const double *sbox, bool want_bval);

template <typename T, int NMAX, int LMAX>
static void launch_vjp_t(ap_ctx *c, AceArgs a, int grid, const double *G) {
    {
        ProfScope p(c, "ace_basis");
        k_ace_basis<T, NMAX, LMAX><<<grid, kBlock, 0, c->stream>>>(a);
    }
    {
        ProfScope p(c, "ace_tangent");
        k_ace_tangent<T, NMAX, LMAX><<<grid, kBlock, 0, c->stream>>>(a, G);
    }
    ProfScope p(c, "ace_bdot");
    k_ace_bdot<T, NMAX, LMAX><<<grid, kBlock, 0, c->stream>>>(a);
}

int launch_ace_vjp(ap_ctx *c, int n, const double *box, int grid_cap, const double *sbox, const double *G) {
    const AceTables &t = c->ace;
    AceArgs a = ace_args(c, n, box, sbox, true);
    const int grid = grid_cap < 1 ? 1 : grid_cap;
    const bool f32 = t.precision == AP_FP32;
    if (t.n_max == 12) {
        if (f32)
            launch_vjp_t<float, 12, 6>(c, a, grid, G);
        else
            launch_vjp_t<double, 12, 6>(c, a, grid, G);
    } else if (t.n_max == 8) {
        if (f32)
            launch_vjp_t<float, 8, 4>(c, a, grid, G);
        else
            launch_vjp_t<double, 8, 4>(c, a, grid, G);
    } else {
        if (f32)
            launch_vjp_t<float, 4, 2>(c, a, grid, G);
        else
            launch_vjp_t<double, 4, 2>(c, a, grid, G);
    }
    return hip_check(c, hipGetLastError(), "ace vjp");
}

int launch_ace(ap_ctx *c, int n, const double *box, int grid_cap, const double *sbox, bool want_bval) {
    const AceTables &t = c->ace;
    AceArgs a = ace_args(c, n, box, sbox, want_bval);
    const int grid = grid_cap < 1 ? 1 : grid_cap;
    const bool f32 = t.precision == AP_FP32;
    if (t.n_max == 12) {
        if (f32)
            launch_t<float, 12, 6>(c, a, grid);
        else
            launch_t<double, 12, 6>(c, a, grid);
    } else if (t.n_max == 8) {
        if (f32)
            launch_t<float, 8, 4>(c, a, grid);
        else
            launch_t<double, 8, 4>(c, a, grid);
    } else {
        if (f32)
            launch_t<float, 4, 2>(c, a, grid);
        else
            launch_t<double, 4, 2>(c, a, grid);
    }
    return hip_check(c, hipGetLastError(), "ace");
}

static AceArgs ace_args(ap_ctx *c, int n, const double *box, const double *sbox, bool want_bval) {
    const AceTables &t = c->ace;
    AceArgs a;
    a.pos = c->pos;
    a.n = n;
    for (int q = 0; q < 3; q++) a.L[q] = box[q];
    a.rc = t.rc;
    a.ncount = c->nbr_cnt;
    a.nidx = c->nbr_idx;
    a.max_nbr = c->max_nbr;
    a.slist = c->slist;
    a.scount = c->d_flags + 2;
    a.dlam = c->dlam;
    a.wbar = c->wbar;
    a.Ef = c->Ef;
    a.Ep = c->Ep;
    a.Et = c->Et;
    a.gbuf = c->gbuf;
    {
        // scratch layout: A [n_cap][NA], radial sums [n_cap][n_max], dE/dA parts [2][n_cap][NA], energy parts
        // [kMaxParts][n_cap]
        const size_t abytes = (size_t)c->n_cap * t.n_max * (t.l_max + 1) * (t.l_max + 1) *
                              (t.precision == AP_FP32 ? 4 : 8);
        char *base = (char *)c->gbuf;
        a.s0buf = (double *)(base + abytes);
        a.gpart = base + abytes + (size_t)c->n_cap * t.n_max * sizeof(double);
        a.epart = (double *)(base + 3 * abytes + (size_t)c->n_cap * t.n_max * sizeof(double));
        a.gstride = c->n_cap;
        a.n0 = t.n0;
        a.queue = c->d_flags + 6;
        a.c30 = t.c30;
        a.kap0 = t.kap0;
        a.stamp = sbox ? nullptr : c->stamp;
        a.gen = c->stamp_gen;
        a.rslot = sbox ? nullptr : c->rslot;
        a.rstamp = c->rstamp;
        a.list_gen = c->list_gen;
        a.rw2 = t.rc * t.rc * (1.0 + 1e-9);
        a.rrev2 = rslot_reach2(c);
    }

    a.fpair = c->fpair;
    a.frev = c->frev;
    a.xl = c->xl;
    a.eb = c->eb;
    a.c1 = t.c1;
    a.bd = t.bd;
    a.c2 = t.c2;
    a.c3 = t.c3;
    a.kval = t.kval;
    a.kidx = t.kidx;
    a.blk = t.blk;
    a.nblk = t.nblk;
    a.emb_A = t.emb_A;
    a.E0 = t.E0;
    a.c1d = t.c1d;
    a.bdd = t.bdd;
    a.flags = c->d_flags;
    a.sbox = sbox;
    a.sid = sbox ? c->sid : nullptr;
    a.bval = want_bval ? c->bval : nullptr;
    a.bstride = t.n_funcs + t.n_max;
    a.n_funcs = t.n_funcs;
    a.g1 = t.g1;
    a.g2 = t.g2;
    a.g3 = t.g3;
    a.ng1 = t.ng1;
    a.ng2 = t.ng2;
    return a;
}

}  // namespace ap
