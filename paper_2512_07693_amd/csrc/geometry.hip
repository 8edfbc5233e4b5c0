// Periodic geometry, cell lists, neighbour lists and the CSP pair list of (B3).
//
// Neighbour lists are slot-major (nbr_idx[k * n + i] is the k-th neighbour of atom i) so that a
// wavefront of consecutive atoms reads one coalesced row per slot. All lists are deterministic:
// atoms inside a cell are sorted by index and the 27 cells are visited in a fixed order.
#include "ap_internal.h"

namespace ap {

__global__ void k_fill_int(int *p, int v, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}
__global__ void k_fill_double(double *p, double v, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}
void launch_fill_int(ap_ctx *c, int *p, int v, int count) {
    if (count > 0) k_fill_int<<<(count + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(p, v, count);
}
void launch_fill_double(ap_ctx *c, double *p, double v, int count) {
    if (count > 0) k_fill_double<<<(count + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(p, v, count);
}

// Wrapped copy of the caller's positions into the context (x - L floor(x/L), L -> 0).
__global__ void k_wrap_copy(const double *__restrict__ in, double *__restrict__ out, int n, double Lx, double Ly,
                            double Lz) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = wrap_coord(in[i], Lx);
    out[n + i] = wrap_coord(in[n + i], Ly);
    out[2 * n + i] = wrap_coord(in[2 * n + i], Lz);
}

int prepare_positions(ap_ctx *c, int n, const double *pos_in, const double *box) {
    k_wrap_copy<<<(n + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(pos_in, c->pos, n, box[0], box[1], box[2]);
    return hip_check(c, hipGetLastError(), "wrap");
}

// ------------------------------------------------------------------------------------------
// Exclusive scan of len ints in one workgroup of 1024 threads; total written to *total.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan_excl(const int *__restrict__ in, int *__restrict__ out, int len,
                                                    int *total, const int *gate) {
    if (gate && gate[0] == 0) return;
    __shared__ int sh[1024];
    const int t = threadIdx.x;
    const int chunk = (len + 1023) / 1024;
    const int b = t * chunk, e = min(len, b + chunk);
    int s = 0;
    for (int q = b; q < e; q++) s += in[q];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int run = sh[t] - s;
    for (int q = b; q < e; q++) {
        int v = in[q];
        out[q] = run;
        run += v;
    }
    if (t == 1023 && total) *total = sh[1023];
}

void launch_scan(ap_ctx *c, const int *in, int *out, int len, int *total, const int *gate) {
    k_scan_excl<<<1, 1024, 0, c->stream>>>(in, out, len, total, gate);
}

// ------------------------------------------------------------------------------------------
// Cell list (rebuilt only when d_flags[0] != 0)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
    int q = (int)floor(x / L * nc);
    return q < 0 ? 0 : (q >= nc ? nc - 1 : q);
}

__global__ void k_cell_clear(int *cnt, int *fill, int ncell, const int *flags) {
    if (flags[0] == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncell) {
        cnt[i] = 0;
        fill[i] = 0;
    }
}

__global__ void k_cell_assign(const double *__restrict__ pos, int n, Geometry g, int *cell_of, int *cnt,
                              const int *flags) {
    if (flags[0] == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(pos[i], g.L[0], g.nc[0]);
    int cy = cell_coord(pos[n + i], g.L[1], g.nc[1]);
    int cz = cell_coord(pos[2 * n + i], g.L[2], g.nc[2]);
    int cc = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = cc;
    atomicAdd(&cnt[cc], 1);
}

__global__ void k_cell_fill(int n, const int *cell_of, const int *start, int *fill, int *atoms, const int *flags) {
    if (flags[0] == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cc = cell_of[i];
    atoms[start[cc] + atomicAdd(&fill[cc], 1)] = i;
}

// Every cell's atoms sorted by index (the fill order above is not deterministic), a wavefront per cell:
// each lane ranks its atom against the others of the cell. The sorted cell also gets its candidate
// records (FP32 position, index), which the list build reads in cell order. A cell of more than 64 atoms is
// insertion-sorted by its first lane.
__global__ void k_cell_sort(int ncell, const int *start, const int *cnt, int *atoms, const double *__restrict__ pos,
                            int n, CandRec *__restrict__ rec, const int *flags) {
    if (flags[0] == 0) return;
    const int lane = threadIdx.x & 63;
    const int cc = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (cc >= ncell) return;  // whole wavefronts
    const int b = start[cc], m = cnt[cc];
    int *a = atoms + b;
    if (m <= 64) {
        const int v = lane < m ? a[lane] : 0;
        int rank = 0;
        for (int u = 0; u < m; u++) rank += __shfl(v, u, 64) < v;
        if (lane < m) {
            a[rank] = v;
            rec[b + rank] = CandRec{(float)pos[v], (float)pos[n + v], (float)pos[2 * n + v], v};
        }
        return;
    }
    if (lane == 0) {
        for (int p = 1; p < m; p++) {
            int v = a[p], q = p - 1;
            while (q >= 0 && a[q] > v) {
                a[q + 1] = a[q];
                q--;
            }
            a[q + 1] = v;
        }
    }
    __threadfence_block();
    for (int p = lane; p < m; p += 64) {
        const int v = a[p];
        rec[b + p] = CandRec{(float)pos[v], (float)pos[n + v], (float)pos[2 * n + v], v};
    }
}

// One pass over the 27 cells per atom, SUB lanes per atom: in each round the SUB lanes test SUB
// consecutive candidates of a column of cells (the three cells of a (dx, dy) column are consecutive in
// the cell order), and a ballot gives every hit its rank among the group's hits, so the slots fill in the
// order of a sequential scan (columns in a fixed order, cells by z, atoms of a cell by index). The
// neighbours inside r_short are written from the front of the slot array, those between r_short and
// r_list from its back; the back part is then moved down behind the front part (a forward
// copy: it only moves to lower slots). ncount_short = the front part.
// The test runs on the candidates' FP32 records with the periodic image of the cell (a shift of the
// atom's position by a box length where the stencil wraps): a squared distance below r^2 - delta is
// inside, one at or above r^2 + delta outside (delta bounds the FP32 error, Thresh below); the rare pair
// in between is decided in FP64 from the positions with the minimum-image difference, the same test as
// the oracle's, so the sets are exact. A dimension with a single cell takes the FP32 minimum image per
// candidate instead of the cell's (WRAP).
// STAGE: the workgroup's lists are assembled in LDS ([max_nbr][kBlock / SUB] ints, dynamic shared memory),
// and each of the two parts goes out to the slot-major array in ascending atom index. Without STAGE (more
// than 256 slots per atom) the lists stay in scan order.
struct Thresh {
    float lo, hi;    // r_list^2 -/+ delta
    float slo, shi;  // r_short^2 -/+ delta
    double r2, rs2;  // the exact squares
};

template <int SUB, bool STAGE, bool WRAP>
__global__ __launch_bounds__(kBlock) void k_nbr_build(const double *__restrict__ pos, int n, Geometry g, Thresh th,
                                                      const int *__restrict__ start,
                                                      const int *__restrict__ cnt, const CandRec *__restrict__ rec,
                                                      const int *__restrict__ cell_of, int max_nbr,
                                                      int32_t *__restrict__ ncount, int32_t *__restrict__ ncount_short,
                                                      int32_t *__restrict__ nidx, double *__restrict__ pos_build,
                                                      int *flags) {
    static_assert(SUB > 0 && 64 % SUB == 0, "lane groups inside a wavefront");
    constexpr int APB = kBlock / SUB;  // atoms per workgroup
    extern __shared__ int tile[];      // STAGE: slot s of local atom a at tile[s * APB + a]
    if (flags[0] == 0) return;         // the same for every workgroup
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int t = lb * blockDim.x + threadIdx.x;
    const int i = t / SUB, sub = t - i * SUB;
    const int al = (int)threadIdx.x / SUB;
    auto put = [&](int slot, int v) {
        if (STAGE)
            tile[slot * APB + al] = v;
        else
            nidx[(size_t)slot * n + i] = v;
    };
    auto get = [&](int slot) { return STAGE ? tile[slot * APB + al] : nidx[(size_t)slot * n + i]; };
    const int gbase = (threadIdx.x & 63) - sub;  // first lane of this atom's group in the wavefront
    const unsigned long long grp = (SUB == 64 ? ~0ull : ((1ull << SUB) - 1ull)) << gbase;
    const unsigned long long below = ((1ull << (threadIdx.x & 63)) - 1ull) & grp;
    const bool live = i < n;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    int c0 = 0, c1 = 0, c2 = 0;
    if (live) {
        xi = pos[i];
        yi = pos[n + i];
        zi = pos[2 * n + i];
        const int cc = cell_of[i];
        c0 = cc / (g.nc[1] * g.nc[2]);
        c1 = (cc / g.nc[2]) % g.nc[1];
        c2 = cc % g.nc[2];
    }
    const float Lf[3] = {(float)g.L[0], (float)g.L[1], (float)g.L[2]};
    const float hLf[3] = {0.5f * Lf[0], 0.5f * Lf[1], 0.5f * Lf[2]};
    int ks = 0, kl = 0;  // front (short) and back (long) counts, the same on every lane of the group
    const int rx = g.nc[0] > 1 ? 1 : 0, ry = g.nc[1] > 1 ? 1 : 0, rz = g.nc[2] > 1 ? 1 : 0;
    // one candidate against the atom's image (xs, ys, zs): inside the short radius, between it and r_list
    auto test = [&](const CandRec &cr, bool valid, float xs, float ys, float zs, bool &hs, bool &hl) {
        hs = hl = false;
        if (!valid) return;
        float ux = cr.x - xs, uy = cr.y - ys, uz = cr.z - zs;
        if (WRAP) {
            if (!rx) ux = ux > hLf[0] ? ux - Lf[0] : (ux < -hLf[0] ? ux + Lf[0] : ux);
            if (!ry) uy = uy > hLf[1] ? uy - Lf[1] : (uy < -hLf[1] ? uy + Lf[1] : uy);
            if (!rz) uz = uz > hLf[2] ? uz - Lf[2] : (uz < -hLf[2] ? uz + Lf[2] : uz);
        }
        const float d2 = ux * ux + uy * uy + uz * uz;
        const bool other = cr.j != i;
        const bool in = other && d2 < th.lo, maybe = other && d2 < th.hi;
        const bool sin = d2 < th.slo, smaybe = d2 < th.shi;
        hs = in && sin;
        hl = in && !smaybe;
        if (__builtin_expect((maybe && !in) || (in && smaybe && !sin), 0)) {
            // too close to call in FP32: the FP64 test on the positions
            const int j = cr.j;
            const double vx = min_image_w(pos[j] - xi, g.L[0]);
            const double vy = min_image_w(pos[n + j] - yi, g.L[1]);
            const double vz = min_image_w(pos[2 * n + j] - zi, g.L[2]);
            const double d2x = norm2_nofma(vx, vy, vz);
            hs = d2x < th.r2 && d2x < th.rs2;
            hl = d2x < th.r2 && !(d2x < th.rs2);
        }
    };
    // the group's hits of one round into their slots, in lane order
    auto record = [&](bool hs, bool hl, int j) {
        const unsigned long long ms = __ballot(hs), ml = __ballot(hl);
        // a slot outside [0, max_nbr) only happens on overflow, which is flagged below
        if (hs) {
            const int sl = ks + __popcll(ms & below);
            if (sl < max_nbr) put(sl, j);
        }
        if (hl) {
            const int sl = max_nbr - 1 - kl - __popcll(ml & below);
            if (sl >= 0) put(sl, j);
        }
        ks += __popcll(ms & grp);
        kl += __popcll(ml & grp);
    };
    // the candidates [b, e) of consecutive cells, two rounds per iteration (two loads in flight)
    auto scan = [&](int b, int e, float xs, float ys, float zs) {
        for (int p0 = b; p0 < e; p0 += 2 * SUB) {
            const int pa = p0 + sub, pb = p0 + SUB + sub;
            // both loads unconditional (clamped into [p0, e)), so that they are in flight together
            const CandRec ca = rec[pa < e ? pa : e - 1];
            const CandRec cb = rec[pb < e ? pb : e - 1];
            bool hs, hl;
            test(ca, pa < e, xs, ys, zs, hs, hl);
            record(hs, hl, ca.j);
            if (p0 + SUB < e) {  // the group's second round
                test(cb, pb < e, xs, ys, zs, hs, hl);
                record(hs, hl, cb.j);
            }
        }
    };
    // columns (dx, dy) of the stencil; a column's cells are consecutive in z and so in the cell order, one
    // range of candidates, or two where the column wraps in z (each with its own image)
    for (int dx = -rx; dx <= rx; dx++) {
        int x = c0 + dx;
        double sx = 0.0;  // the atom's image relative to the cell's candidates
        if (x < 0) {
            x += g.nc[0];
            sx = g.L[0];
        } else if (x >= g.nc[0]) {
            x -= g.nc[0];
            sx = -g.L[0];
        }
        const float xs = (float)(xi + sx);
        for (int dy = -ry; dy <= ry; dy++) {
            int y = c1 + dy;
            double sy = 0.0;
            if (y < 0) {
                y += g.nc[1];
                sy = g.L[1];
            } else if (y >= g.nc[1]) {
                y -= g.nc[1];
                sy = -g.L[1];
            }
            const float ys = (float)(yi + sy);
            const int q0 = (x * g.nc[1] + y) * g.nc[2];  // the column's first cell
            int z0 = c2 - rz, z1 = c2 + rz;
            if (z0 < 0) {
                // cell nc - 1 (seen through the lower face) first, then cells 0 .. z1
                int b = 0, e = 0;
                if (live) {
                    b = start[q0 + g.nc[2] - 1];
                    e = b + cnt[q0 + g.nc[2] - 1];
                }
                scan(b, e, xs, ys, (float)(zi + g.L[2]));
                z0 = 0;
            }
            const int zt = z1 < g.nc[2] ? z1 : g.nc[2] - 1;
            {
                int b = 0, e = 0;
                if (live) {
                    b = start[q0 + z0];
                    e = start[q0 + zt] + cnt[q0 + zt];
                }
                scan(b, e, xs, ys, (float)zi);
            }
            if (z1 >= g.nc[2]) {
                // cell 0 seen through the upper face
                int b = 0, e = 0;
                if (live) {
                    b = start[q0];
                    e = b + cnt[q0];
                }
                scan(b, e, xs, ys, (float)(zi - g.L[2]));
            }
        }
    }
    int k = ks + kl;
    if (live && k <= max_nbr) {
        // the back part [max_nbr - kl, max_nbr) moves down to [ks, ks + kl), ks <= max_nbr - kl, in
        // increasing slot order: a store only hits a slot read in the same round or an earlier one
        for (int q = sub; q < kl; q += SUB) {
            const int v = get(max_nbr - kl + q);
            put(ks + q, v);
        }
    }
    if (STAGE) {
        __syncthreads();
        // each part of the list, [0, ks) and [ks, k), goes out in ascending atom index: a lane counts, for
        // each of its entries, the entries of the same part before it in that order (the index, then the
        // slot), and stores the entry at that rank. Atoms numbered along the lattice then have their lists
        // in step: a slot of consecutive atoms names consecutive records, which the gathers of every pass
        // over the lists read as a few cache lines. (An overflowed list is written as it stands.)
        if (live && k <= max_nbr) {
            if (n <= (1 << 24)) {
                // one unsigned key per slot, the index above the slot (slots < 256 here), so that a single
                // compare orders the entries and no two share a rank (the group's lanes are one wavefront,
                // whose LDS accesses complete in program order)
                for (int p = sub; p < k; p += SUB)
                    tile[p * APB + al] = (int)(((unsigned)tile[p * APB + al] << 8) | p);
                // a lane ranks four entries of a part per pass over that part
                auto rank_part = [&](int lo, int hi) {
                    for (int p0 = lo + sub; p0 < hi; p0 += 4 * SUB) {
                        unsigned key[4];
                        int r[4];
#pragma unroll
                        for (int j = 0; j < 4; j++) {
                            const int p = p0 + j * SUB;
                            key[j] = p < hi ? (unsigned)tile[p * APB + al] : 0u;
                            r[j] = lo;
                        }
#pragma unroll 4
                        for (int q = lo; q < hi; q++) {
                            const unsigned u = (unsigned)tile[q * APB + al];
#pragma unroll
                            for (int j = 0; j < 4; j++) r[j] += (int)(u < key[j]);
                        }
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            if (p0 + j * SUB < hi) nidx[(size_t)r[j] * n + i] = (int)(key[j] >> 8);
                    }
                };
                rank_part(0, ks);
                rank_part(ks, k);
            } else {
                for (int p = sub; p < k; p += SUB) {
                    const int lo = p < ks ? 0 : ks, hi = p < ks ? ks : k;
                    const int v = tile[p * APB + al];
                    int r = lo;
                    for (int q = lo; q < hi; q++) {
                        const int u = tile[q * APB + al];
                        r += (u < v || (u == v && q < p)) ? 1 : 0;
                    }
                    nidx[(size_t)r * n + i] = v;
                }
            }
        } else if (live) {
            for (int p = sub; p < max_nbr; p += SUB) nidx[(size_t)p * n + i] = tile[p * APB + al];
        }
    }
    if (!live || sub != 0) return;
    ncount_short[i] = ks < max_nbr ? ks : max_nbr;
    if (k > max_nbr) {
        atomicOr(&flags[1], kErrOverflow);
        k = max_nbr;
    }
    ncount[i] = k;
    pos_build[i] = xi;
    pos_build[n + i] = yi;
    pos_build[2 * n + i] = zi;
}

__global__ void k_commit(int *flags, int *list_gen) {
    if (flags[0]) list_gen[0]++;
    flags[3] = flags[0];
    flags[0] = 0;
}
__global__ void k_bump(int *list_gen) { list_gen[0]++; }

// Marks a rebuild when any atom moved more than skin/2 from its position at the last build.
__global__ void k_skin_check(const double *__restrict__ pos, const double *__restrict__ pos_build, int n,
                             double Lx, double Ly, double Lz, double half_skin2, int *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ux = min_image_w(pos[i] - pos_build[i], Lx);
    double uy = min_image_w(pos[n + i] - pos_build[n + i], Ly);
    double uz = min_image_w(pos[2 * n + i] - pos_build[2 * n + i], Lz);
    if (!(ux * ux + uy * uy + uz * uz <= half_skin2)) atomicOr(&flags[0], 1);  // (non-finite: rebuild too)
}

bool list_geometry(const double *box, double r_list, Geometry &g) {
    for (int a = 0; a < 3; a++) {
        g.L[a] = box[a];
        if (!(r_list < 0.5 * box[a])) return false;
        g.nc[a] = (int)floor(box[a] / r_list);
        if (g.nc[a] < 3) g.nc[a] = 1;  // one cell spans the box: every atom is a candidate
    }
    g.ncell = g.nc[0] * g.nc[1] * g.nc[2];
    return true;
}

static int make_geometry(ap_ctx *c, const double *box, double r_list, Geometry &g) {
    if (!list_geometry(box, r_list, g))
        return set_error(c, AP_E_BOX, "list radius (cutoff + skin) must be below half the box");
    return AP_OK;
}

// The FP32 test's margins. Each coordinate of a record is within half an FP32 ulp of L of its FP64 value,
// the shifted atom position (below 2 L) within one ulp of L, and the difference and, for a single-cell
// dimension, its wrap by the rounded box length add at most another ulp of L: e <= 3 ulp(L) per component.
// The squared distance then errs by at most 2 e (|ux| + |uy| + |uz|) + 3 e^2 <= 2 sqrt(3) r e + 3 e^2, plus
// the rounding of the three products and two sums (<= 3 ulp(r^2) with FMA contraction); delta is twice that
// bound, and the FP32 thresholds are rounded outward.
static float ulp32(double v) { return (float)std::ldexp(1.0, std::ilogb(v) - 23); }
static Thresh list_thresholds(const Geometry &g, double r_list, double r_short) {
    const double Lm = std::max(g.L[0], std::max(g.L[1], g.L[2]));
    auto margin = [&](double r) {
        const double e = 3.0 * ulp32(Lm);
        return 2.0 * (2.0 * std::sqrt(3.0) * r * e + 3.0 * e * e + 3.0 * ulp32(std::max(r * r, 1e-30)));
    };
    const double r2 = r_list * r_list, rs2 = r_short * r_short, dl = margin(r_list), ds = margin(r_short);
    Thresh th;
    th.lo = std::nextafter((float)(r2 - dl), 0.0f);
    th.hi = std::nextafter((float)(r2 + dl), INFINITY);
    th.slo = std::nextafter((float)(rs2 - ds), 0.0f);
    th.shi = std::nextafter((float)(rs2 + ds), INFINITY);
    th.r2 = r2;
    th.rs2 = rs2;
    return th;
}

// The cell binning and list kernels of one build of the wrapped positions b.pos, gated by b.flags[0]
// (nothing happens unless it is set; the caller has cleared the cell counts and fills): cell ids and
// counts, their exclusive scan, the cells' atoms sorted by index with their records, then the lists.
void launch_list_kernels(hipStream_t s, int n, const Geometry &g, double r_list, double r_short, int max_nbr,
                         const ListBufs &b) {
    const int nb = (n + kBlock - 1) / kBlock;
    k_cell_assign<<<nb, kBlock, 0, s>>>(b.pos, n, g, b.cell_of, b.cell_cnt, b.flags);
    k_scan_excl<<<1, 1024, 0, s>>>(b.cell_cnt, b.cell_start, g.ncell, nullptr, b.flags);
    k_cell_fill<<<nb, kBlock, 0, s>>>(n, b.cell_of, b.cell_start, b.cell_fill, b.cell_atoms, b.flags);
    k_cell_sort<<<(int)(((size_t)g.ncell * 64 + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        g.ncell, b.cell_start, b.cell_cnt, b.cell_atoms, b.pos, n, b.cell_rec, b.flags);
    constexpr int SUB = 8;  // lanes per atom in the list build
    const int lgrid = (int)(((size_t)n * SUB + kBlock - 1) / kBlock);
    const Thresh th = list_thresholds(g, r_list, r_short);
    const size_t lds = (size_t)max_nbr * (kBlock / SUB) * sizeof(int);
    const bool wrap = g.nc[0] == 1 || g.nc[1] == 1 || g.nc[2] == 1;
    // (at most 32 KB of staged lists per workgroup)
#define AP_NBR_ARGS b.pos, n, g, th, b.cell_start, b.cell_cnt, b.cell_rec, b.cell_of, max_nbr, b.ncount, b.nshort, \
                    b.nidx, b.pos_build, b.flags
    if (max_nbr <= 256 && !wrap)
        k_nbr_build<SUB, true, false><<<lgrid, kBlock, lds, s>>>(AP_NBR_ARGS);
    else if (max_nbr <= 256)
        k_nbr_build<SUB, true, true><<<lgrid, kBlock, lds, s>>>(AP_NBR_ARGS);
    else if (!wrap)
        k_nbr_build<SUB, false, false><<<lgrid, kBlock, 0, s>>>(AP_NBR_ARGS);
    else
        k_nbr_build<SUB, false, true><<<lgrid, kBlock, 0, s>>>(AP_NBR_ARGS);
#undef AP_NBR_ARGS
}

// The stream-ordered pieces of a context-free list build: wrapped positions and fills.
void launch_wrap(hipStream_t s, const double *in, double *out, int n, const double *box) {
    k_wrap_copy<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(in, out, n, box[0], box[1], box[2]);
}
void launch_fill_int_on(hipStream_t s, int *p, int v, int count) {
    if (count > 0) k_fill_int<<<(count + kBlock - 1) / kBlock, kBlock, 0, s>>>(p, v, count);
}

static int grow_cells(ap_ctx *c, int ncell) {
    if (ncell <= c->ncell_cap) return AP_OK;
    (void)hipFree(c->cell_cnt);
    (void)hipFree(c->cell_start);
    (void)hipFree(c->cell_fill);
    int rc = hip_check(c, hipMalloc(&c->cell_cnt, sizeof(int) * ncell), "cells");
    if (!rc) rc = hip_check(c, hipMalloc(&c->cell_start, sizeof(int) * (ncell + 1)), "cells");
    if (!rc) rc = hip_check(c, hipMalloc(&c->cell_fill, sizeof(int) * ncell), "cells");
    if (!rc) c->ncell_cap = ncell;
    return rc;
}

// (Re)builds the neighbour list of the positions in c->pos at radius r_list when forced, when the
// list parameters changed, or when the device-side skin check flagged it.
int ensure_list(ap_ctx *c, int n, const double *box, double r_list, bool force, bool skin_checked, bool commit) {
    Geometry g;
    int rc = make_geometry(c, box, r_list, g);
    if (rc) return rc;
    rc = grow_cells(c, g.ncell);
    if (rc) return rc;
    bool changed = force || r_list != c->list_r || n != c->list_n || box[0] != c->list_box[0] ||
                   box[1] != c->list_box[1] || box[2] != c->list_box[2];
    const int nb = (n + kBlock - 1) / kBlock;
    const int cb = (g.ncell + kBlock - 1) / kBlock;
    if (changed) {
        launch_fill_int(c, c->d_flags, 1, 1);
        k_cell_clear<<<cb, kBlock, 0, c->stream>>>(c->cell_cnt, c->cell_fill, g.ncell, c->d_flags);
    } else if (!skin_checked) {
        k_skin_check<<<nb, kBlock, 0, c->stream>>>(c->pos, c->pos_build, n, box[0], box[1], box[2],
                                                   0.25 * c->skin * c->skin, c->d_flags);
        k_cell_clear<<<cb, kBlock, 0, c->stream>>>(c->cell_cnt, c->cell_fill, g.ncell, c->d_flags);
    }
    c->ncell_cur = g.ncell;
    const double rs = std::max(c->eam.r_rho, c->eam.r_phi) + c->skin;  // the EAM pairs first
    const ListBufs b{c->pos,        c->pos_build, c->d_flags,   c->cell_of, c->cell_cnt, c->cell_start,
                     c->cell_fill,  c->cell_atoms, c->cell_rec, c->nbr_cnt, c->nbr_short, c->nbr_idx};
    launch_list_kernels(c->stream, n, g, r_list, rs, c->max_nbr, b);
    if (commit) k_commit<<<1, 1, 0, c->stream>>>(c->d_flags, c->list_gen);
    c->list_r = r_list;
    c->list_n = n;
    for (int a = 0; a < 3; a++) c->list_box[a] = box[a];
    return hip_check(c, hipGetLastError(), "neighbour list");
}

// ------------------------------------------------------------------------------------------
// Ragged batch of periodic cells: structure id per atom, wrapped positions and, for every atom,
// the neighbours inside its own cell (every atom of the cell is a candidate).
// ------------------------------------------------------------------------------------------
__global__ void k_batch_prepare(const double *__restrict__ pos_in, int n, int n_struct, const int *__restrict__ off,
                                const double *__restrict__ sbox, int *__restrict__ sid, double *__restrict__ pos) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_struct - 1;  // the structure s with off[s] <= i < off[s+1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    sid[i] = lo;
    for (int a = 0; a < 3; a++) pos[(size_t)a * n + i] = wrap_coord(pos_in[(size_t)a * n + i], sbox[3 * lo + a]);
}

__global__ __launch_bounds__(kBlock) void k_batch_nbr(const double *__restrict__ pos, int n,
                                                      const int *__restrict__ off, const double *__restrict__ sbox,
                                                      const int *__restrict__ sid, double r2, int max_nbr,
                                                      int32_t *__restrict__ ncount, int32_t *__restrict__ nidx,
                                                      int *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = sid[i];
    const double Lx = sbox[3 * s], Ly = sbox[3 * s + 1], Lz = sbox[3 * s + 2];
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int k = 0;
    for (int j = off[s]; j < off[s + 1]; j++) {
        if (j == i) continue;
        const double ux = min_image(pos[j] - xi, Lx), uy = min_image(pos[n + j] - yi, Ly),
                     uz = min_image(pos[2 * n + j] - zi, Lz);
        if (norm2_nofma(ux, uy, uz) < r2) {
            if (k < max_nbr) nidx[(size_t)k * n + i] = j;
            k++;
        }
    }
    if (k > max_nbr) {
        atomicOr(&flags[1], kErrOverflow);
        k = max_nbr;
    }
    ncount[i] = k;
}

int batch_lists(ap_ctx *c, int n, int n_struct, const int *d_off, const double *d_box, const double *pos_in,
                double r_list) {
    const int nb = (n + kBlock - 1) / kBlock;
    k_batch_prepare<<<nb, kBlock, 0, c->stream>>>(pos_in, n, n_struct, d_off, d_box, c->sid, c->pos);
    k_batch_nbr<<<nb, kBlock, 0, c->stream>>>(c->pos, n, d_off, d_box, c->sid, r_list * r_list, c->max_nbr, c->nbr_cnt,
                                              c->nbr_idx, c->d_flags);
    k_bump<<<1, 1, 0, c->stream>>>(c->list_gen);  // the lists changed outside a committed build
    c->list_r = -1;  // not a list of the single-box evaluation
    return hip_check(c, hipGetLastError(), "batch lists");
}

// ------------------------------------------------------------------------------------------
// CSP^list of (B3)
// ------------------------------------------------------------------------------------------
// One-time pair detection: n_csp nearest by (d2, index) via repeated minimum search; greedy
// pairing by the smallest |u_a + u_b|^2 with index tie-breaks; written in choice order.
// NC (8 or 12) is a compile-time constant so that every loop over the selected neighbours unrolls
// and the per-thread tables stay in registers.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_csp_pairs(const double *__restrict__ pos, int n, Geometry g,
                                                      const int32_t *__restrict__ ncount,
                                                      const int32_t *__restrict__ nidx, int32_t *__restrict__ out,
                                                      int *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cnt = ncount[i];
    if (cnt < NC) {
        atomicOr(&flags[1], kErrCsp);
        return;
    }
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    int sel[NC];
    double sx_[NC], sy_[NC], sz_[NC];
    // the s-th nearest is the smallest key (d2, j) above the (s-1)-th one: keys are unique
    double pd = -1.0;
    int pj = -1;
#pragma unroll
    for (int s = 0; s < NC; s++) {
        int bj = -1;
        double bd = 0;
        for (int q = 0; q < cnt; q++) {
            const int j = nidx[(size_t)q * n + i];
            double ux = min_image(pos[j] - xi, g.L[0]);
            double uy = min_image(pos[n + j] - yi, g.L[1]);
            double uz = min_image(pos[2 * n + j] - zi, g.L[2]);
            double d2 = norm2_nofma(ux, uy, uz);
            const bool above = d2 > pd || (d2 == pd && j > pj);
            if (above && (bj < 0 || d2 < bd || (d2 == bd && j < bj))) {
                bd = d2;
                bj = j;
            }
        }
        pd = bd;
        pj = bj;
        sel[s] = bj;
        sx_[s] = min_image(pos[bj] - xi, g.L[0]);
        sy_[s] = min_image(pos[n + bj] - yi, g.L[1]);
        sz_[s] = min_image(pos[2 * n + bj] - zi, g.L[2]);
    }
    unsigned used = 0u;
#pragma unroll
    for (int p = 0; p < NC / 2; p++) {
        int ba = 0, bb = 0, blo = 0, bhi = 0;
        bool have = false;
        double bs = 0;
#pragma unroll
        for (int a = 0; a < NC; a++) {
#pragma unroll
            for (int b = a + 1; b < NC; b++) {
                const bool avail = ((used >> a) & 1u) == 0u && ((used >> b) & 1u) == 0u;
                double s;
                {
#pragma clang fp contract(off)
                    const double px = sx_[a] + sx_[b], py = sy_[a] + sy_[b], pz = sz_[a] + sz_[b];
                    s = px * px + py * py + pz * pz;
                }
                const int lo = sel[a] < sel[b] ? sel[a] : sel[b], hi = sel[a] < sel[b] ? sel[b] : sel[a];
                const bool better = !have || s < bs || (s == bs && (lo < blo || (lo == blo && hi < bhi)));
                if (avail && better) {
                    have = true;
                    ba = a;
                    bb = b;
                    bs = s;
                    blo = lo;
                    bhi = hi;
                }
            }
        }
        used |= (1u << ba) | (1u << bb);
        out[(size_t)i * NC + 2 * p] = blo;
        out[(size_t)i * NC + 2 * p + 1] = bhi;
    }
}

int build_csp_pairs(ap_ctx *c, int n, const double *box, int n_csp, int32_t *out) {
    const double r_search = 5.0;
    int rc = ensure_list(c, n, box, r_search, true);
    if (rc) return rc;
    Geometry g;
    rc = make_geometry(c, box, r_search, g);
    if (rc) return rc;
    const int nb = (n + kBlock - 1) / kBlock;
    if (n_csp == 8)
        k_csp_pairs<8><<<nb, kBlock, 0, c->stream>>>(c->pos, n, g, c->nbr_cnt, c->nbr_idx, out, c->d_flags);
    else
        k_csp_pairs<12><<<nb, kBlock, 0, c->stream>>>(c->pos, n, g, c->nbr_cnt, c->nbr_idx, out, c->d_flags);
    c->list_r = -1;  // the list at r_search is not the evaluation list
    return hip_check(c, hipGetLastError(), "csp pairs");
}

__global__ void k_csp_check_transpose(const int32_t *__restrict__ list, int n, int n_csp, int32_t *__restrict__ lt,
                                      int *rcnt, int *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int t = 0; t < n_csp; t++) {
        int j = list[(size_t)i * n_csp + t];
        if (j < 0 || j >= n || j == i) {
            atomicOr(&flags[1], kErrCsp);
            j = i;
        }
        lt[(size_t)t * n + i] = j;
        atomicAdd(&rcnt[j], 1);
    }
}

__global__ void k_csp_rev_fill(int n, int n_csp, const int32_t *__restrict__ lt, const int *rstart, int *rfill,
                               int32_t *rcode) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int t = 0; t < n_csp; t++) {
        int i = lt[(size_t)t * n + j];
        rcode[rstart[i] + atomicAdd(&rfill[i], 1)] = j * 16 + t;
    }
}

__global__ void k_csp_rev_sort(int n, const int *rstart, int32_t *rcode) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = rstart[i], m = rstart[i + 1] - b;
    int32_t *a = rcode + b;
    for (int p = 1; p < m; p++) {
        int v = a[p], q = p - 1;
        while (q >= 0 && a[q] > v) {
            a[q + 1] = a[q];
            q--;
        }
        a[q + 1] = v;
    }
}

int install_csp(ap_ctx *c, int n, int n_csp, const int32_t *list) {
    if (n_csp != 8 && n_csp != 12) return set_error(c, AP_E_CSP, "n_csp must be 8 or 12");
    (void)hipFree(c->csp_t);
    (void)hipFree(c->rev_start);
    (void)hipFree(c->rev_code);
    c->csp_t = nullptr;
    c->rev_start = nullptr;
    c->rev_code = nullptr;
    int rc = hip_check(c, hipMalloc(&c->csp_t, sizeof(int32_t) * (size_t)n * n_csp), "csp");
    if (!rc) rc = hip_check(c, hipMalloc(&c->rev_start, sizeof(int32_t) * (size_t)(n + 1)), "csp");
    if (!rc) rc = hip_check(c, hipMalloc(&c->rev_code, sizeof(int32_t) * (size_t)n * n_csp), "csp");
    if (rc) return rc;
    const int nb = (n + kBlock - 1) / kBlock;
    int *cnt = c->cell_of;  // scratch [n_cap] ints, free outside of list builds
    int *fill = c->sidx;
    launch_fill_int(c, cnt, 0, n + 1);
    launch_fill_int(c, fill, 0, n);
    launch_fill_int(c, c->d_flags + 1, 0, 1);
    k_csp_check_transpose<<<nb, kBlock, 0, c->stream>>>(list, n, n_csp, c->csp_t, cnt, c->d_flags);
    k_scan_excl<<<1, 1024, 0, c->stream>>>(cnt, c->rev_start, n + 1, nullptr, nullptr);
    k_csp_rev_fill<<<nb, kBlock, 0, c->stream>>>(n, n_csp, c->csp_t, c->rev_start, fill, c->rev_code);
    k_csp_rev_sort<<<nb, kBlock, 0, c->stream>>>(n, c->rev_start, c->rev_code);
    rc = hip_check(c, hipGetLastError(), "csp reverse");
    if (rc) return rc;
    rc = sync_and_check(c);
    if (rc) return rc;
    c->csp_n = n;
    c->n_csp = n_csp;
    c->list_r = -1;  // cell_of was used as scratch
    return AP_OK;
}

// g_i = sum over the stored pairs (a, b) of |u_ia + u_ib|^2 (division-free minimum images: the pairs are
// nearest neighbours, far from |d| = L / 2). NC, the list width (8 or 12, the widths the library accepts),
// is a constant so that the loop unrolls and all of an atom's gathers are in flight at once (the sum keeps
// its order).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_csp_value(const double *__restrict__ pos, int n, double Lx, double Ly,
                                                      double Lz, const int32_t *__restrict__ lt,
                                                      double *__restrict__ g, Rec4 *__restrict__ xg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < NC / 2; p++) {
        const int a = lt[(size_t)(2 * p) * n + i], b = lt[(size_t)(2 * p + 1) * n + i];
        double vx = min_image_w(pos[a] - xi, Lx) + min_image_w(pos[b] - xi, Lx);
        double vy = min_image_w(pos[n + a] - yi, Ly) + min_image_w(pos[n + b] - yi, Ly);
        double vz = min_image_w(pos[2 * n + a] - zi, Lz) + min_image_w(pos[2 * n + b] - zi, Lz);
        s += vx * vx + vy * vy + vz * vz;
    }
    g[i] = s;
    xg[i] = Rec4{xi, yi, zi, s};
}

void launch_csp_value(ap_ctx *c, int n, const double *box) {
    const int nb = (n + kBlock - 1) / kBlock;
    if (c->n_csp == 12)
        k_csp_value<12><<<nb, kBlock, 0, c->stream>>>(c->pos, n, box[0], box[1], box[2], c->csp_t, c->g, c->xg);
    else
        k_csp_value<8><<<nb, kBlock, 0, c->stream>>>(c->pos, n, box[0], box[1], box[2], c->csp_t, c->g, c->xg);
}

}  // namespace ap
