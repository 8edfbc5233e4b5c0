// Learned switching indicator: a small network as the per-atom g of Eq. (6).
//
// With g_j a smooth function of j's neighbourhood, the energy depends on g_j only through the
// descriptors d_k, dE/dg_j = -W_j (W_j = sum_k E~_k w(r_kj) of (S25), computed by k_W), and the
// force is the general grad-g term of (S16): F_i += sum_j W_j grad_i g_j.
//
// Features (sixteen rotation invariants of the neighbours inside rc, FP32):
//   q[n]               = sum_j g_n(r_ij),                         n = 0..7
//   q[8 + 4 n + l - 1] = sum_m A_nlm^2, A_nlm = sum_j g_n(r_ij) Y_lm(uhat_ij),   n = 0, 1; l = 1..4
// with the Chebyshev channels and real harmonics of basis.h. Network (FP32):
//   z = (q - mu) / sig, h1 = silu(W1 z + b1), h2 = silu(W2 h1 + b2), o = w3 . h2 + b3, g = softplus(o).
// Parameter block (AP_MLP_NPARAMS floats): mu[16] sig[16] W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3.
//
// Kernels:
//   k_mlp_indicator  one thread per atom for the features, then the forward pass of the wavefront's 64
//                    atoms on the matrix cores; g (or the features alone)
//   k_mlp_eval       one thread per sample: g and dg/dq from given features
//   k_mlp_gradg      one wavefront per atom with W_j != 0, four per workgroup: features, backward pass
//                    (a hidden unit per lane), and h_jk = W_j dg_j/du_jk per neighbour slot, stored at
//                    (j, slot) and slot-major at (slot of j in k's list, k) for the gather-only force kernel
//   k_mlp_fb         one thread per training sample: forward and backward, activations written
//                    feature-major for the weight-gradient reduction
//   k_mlp_wgrad      one wavefront per parameter: sums over the batch in a fixed order
//   k_mlp_adam       Adam step
#include "ap_internal.h"
#include "basis.h"

namespace ap {

constexpr int kNQ = 16, kNH = 64;
constexpr int kMU = 0, kSIG = 16, kW1 = 32, kB1 = kW1 + kNH * kNQ, kW2 = kB1 + kNH, kB2 = kW2 + kNH * kNH,
              kW3 = kB2 + kNH, kB3 = kW3 + kNH, kNP = kB3 + 1;
static_assert(kNP == AP_MLP_NPARAMS, "parameter block layout");
// rows of the training scratch T[kTRows][B]: z, h1, d1, h2, d2, dL/do, loss term
constexpr int kTZ = 0, kTH1 = 16, kTD1 = 80, kTH2 = 144, kTD2 = 208, kTGO = 272, kTLOSS = 273, kTRows = 274;

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }
// the logistic function with the hardware exponential and reciprocal (about 1e-6 relative), for the
// indicator's forward pass; training and the input gradient keep the library's expf and division
__device__ __forceinline__ float sigm_fast(float a) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * a));
}
__device__ __forceinline__ float silu_d(float a) {
    const float s = sigm(a);
    return s * (1.0f + a * (1.0f - s));
}
__device__ __forceinline__ float softplus(float o) { return o > 0.0f ? o + log1pf(expf(-o)) : log1pf(expf(o)); }

// Features of atom i from its slot-major neighbour list: q[16] and A[2][24] (l = 1..4).
__device__ __forceinline__ void site_features(const double *__restrict__ pos, int n, int i, double Lx, double Ly,
                                              double Lz, const int32_t *__restrict__ ncount,
                                              const int32_t *__restrict__ nidx, double rc, float *q, float *A) {
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    const double rc2 = rc * rc;
    const float rcf = (float)rc;
#pragma unroll
    for (int f = 0; f < kNQ; f++) q[f] = 0.0f;
#pragma unroll
    for (int t = 0; t < 48; t++) A[t] = 0.0f;
    const int cnt = ncount[i];
    for (int k = 0; k < cnt; k++) {
        const int j = nidx[(size_t)k * n + i];
        const double ux = min_image_w(pos[j] - xi, Lx), uy = min_image_w(pos[n + j] - yi, Ly),
                     uz = min_image_w(pos[2 * n + j] - zi, Lz);
        const double r2 = ux * ux + uy * uy + uz * uz;
        if (!(r2 < rc2)) continue;
        const double rd = sqrt(r2);
        const float r = (float)rd, ir = (float)(1.0 / rd);
        float g[8], Y[25];
        radial<float, 8>(r, rcf, g, (float *)nullptr);
        ylm_real<float, 4>((float)ux * ir, (float)uy * ir, (float)uz * ir, Y);
#pragma unroll
        for (int c = 0; c < 8; c++) q[c] += g[c];
#pragma unroll
        for (int t = 1; t < 25; t++) {
            A[t - 1] += g[0] * Y[t];
            A[24 + t - 1] += g[1] * Y[t];
        }
    }
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int l = 1; l <= 4; l++) {
            float s = 0.0f;
#pragma unroll
            for (int t = l * l; t <= l * l + 2 * l; t++) s += A[24 * c + t - 1] * A[24 * c + t - 1];
            q[8 + 4 * c + l - 1] = s;
        }
}

__device__ __forceinline__ void load_params(float *sP, const float *__restrict__ P) {
    for (int q = threadIdx.x; q < kNP; q += blockDim.x) sP[q] = P[q];
    __syncthreads();
}

struct MlpArgs {
    const double *pos;
    int n;
    double L[3];
    double rc;
    const int32_t *ncount, *nidx;
    int max_nbr;
    const float *P;
    double *g;        // [n] indicator (k_mlp_indicator)
    Rec4 *xg;         // [n] {x, y, z, g}
    const Rec4 *xl;   // [n] {x, y, z, lambda} (after the density pass)
    // reverse slots kept per list build (shared with the ACE pair kernel): rslot[j][slot] is the slot of j
    // in its slot-th neighbour's list, valid while rstamp[j] == *list_gen
    int *rslot, *rstamp;
    const int *list_gen;
    double rrev2;     // slots searched when an atom's reverse slots are cached (rslot_reach2)
    float *q;         // [n][16] features (feature mode)
    const double *W;  // [n]
    const int *wlist, *wcount;
    float *hpair, *hrev;
    int *flags;
};

// The indicator kernel's copy of the parameters in LDS: the weight matrices transposed with rows of 68
// floats, so that a matrix-core operand read (16 consecutive outputs per row, four rows apart by 68) touches
// 64 different banks.
constexpr int kTS = 68;
constexpr int kMmu = 0, kMsig = 16, kMb1 = 32, kMb2 = kMb1 + kNH, kMw3 = kMb2 + kNH, kMb3 = kMw3 + kNH,
              kMW1t = 228, kMW2t = kMW1t + kNQ * kTS, kMNP = kMW2t + kNH * kTS;
static_assert(kMb3 < kMW1t, "indicator parameter layout");
__device__ __forceinline__ void load_params_t(float *sM, const float *__restrict__ P) {
    for (int q = threadIdx.x; q < kNQ; q += blockDim.x) {
        sM[kMmu + q] = P[kMU + q];
        sM[kMsig + q] = P[kSIG + q];
    }
    for (int q = threadIdx.x; q < kNH; q += blockDim.x) {
        sM[kMb1 + q] = P[kB1 + q];
        sM[kMb2 + q] = P[kB2 + q];
        sM[kMw3 + q] = P[kW3 + q];
    }
    if (threadIdx.x == 0) sM[kMb3] = P[kB3];
    for (int q = threadIdx.x; q < kNH * kNQ; q += blockDim.x) {  // W1[h][f] -> W1t[f][h]
        const int h = q / kNQ, f = q - h * kNQ;
        sM[kMW1t + f * kTS + h] = P[kW1 + q];
    }
    for (int q = threadIdx.x; q < kNH * kNH; q += blockDim.x) {  // W2[o][h] -> W2t[h][o]
        const int o = q / kNH, h = q - o * kNH;
        sM[kMW2t + h * kTS + o] = P[kW2 + q];
    }
    __syncthreads();
}

// The network on the wavefront's 64 atoms at once, on the matrix cores (16x16x4 FP32 tiles), transposed so
// that the first layer's accumulators serve directly as the second layer's operand:
//   H1^T[h][a] = silu(W1 Z^T + b1)   (4 x 4 tiles of (h, a), k = feature)
//   H2^T[o][a] = silu(W2 H1^T + b2)  (per output tile, k = h taken in the accumulators' row order)
//   o_a = w3 . H2^T[:, a] + b3
// Z (64 x 16) goes through LDS (each lane holds its own atom's row); the weights are read from LDS. Lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives C[4 (l / 16) + j][l % 16].
__device__ __forceinline__ float mlp_forward_wave(const float *__restrict__ P, float *__restrict__ sZ,
                                                  const float *z) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, lc = lane & 15, lr = lane >> 4;
    constexpr int ZS = kNQ + 1;  // padded row of Z in LDS
#pragma unroll
    for (int f = 0; f < kNQ; f++) sZ[lane * ZS + f] = z[f];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f4 h1[4][4];  // [h tile][atom tile]
#pragma unroll
    for (int rt = 0; rt < 4; rt++) {
        // the four atom tiles share each weight operand and are independent chains
        f4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ct++) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kNQ / 4; ks++) {
            const float x = P[kMW1t + (4 * ks + lr) * kTS + 16 * rt + lc];
#pragma unroll
            for (int ct = 0; ct < 4; ct++)
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, sZ[(16 * ct + lc) * ZS + 4 * ks + lr], acc[ct], 0,
                                                               0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ct++) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float v = acc[ct][j] + P[kMb1 + 16 * rt + 4 * lr + j];
                acc[ct][j] = v * sigm_fast(v);
            }
            h1[rt][ct] = acc[ct];
        }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};  // per atom tile: this lane's share of w3 . h2
#pragma unroll
    for (int ot = 0; ot < 4; ot++) {
        f4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ct++) acc[ct] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int rt = 0; rt < 4; rt++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float x = P[kMW2t + (16 * rt + 4 * lr + j) * kTS + 16 * ot + lc];
#pragma unroll
                for (int ct = 0; ct < 4; ct++)
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, h1[rt][ct][j], acc[ct], 0, 0, 0);
            }
#pragma unroll
        for (int ct = 0; ct < 4; ct++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int o = 16 * ot + 4 * lr + j;
                const float v = acc[ct][j] + P[kMb2 + o];
                part[ct] += P[kMw3 + o] * (v * sigm_fast(v));
            }
    }
    // the four lanes of a column hold the partial sums of the same atom: a fixed butterfly over them, then
    // lane l takes its own atom's (atom l = 16 lr + lc sits in tile ct = lr)
    float mine = 0.f;
#pragma unroll
    for (int ct = 0; ct < 4; ct++) {
        float v = part[ct];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        mine = ct == lr ? v : mine;
    }
    return mine + P[kMb3];
}

__global__ __launch_bounds__(kBlock, 4) void k_mlp_indicator(MlpArgs a, int features_only) {
    __shared__ float sP[kMNP];
    __shared__ float sZ[kBlock / 64][64 * (kNQ + 1)];
    if (!features_only) load_params_t(sP, a.P);
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    // every lane stays to the end: the network runs on whole wavefronts
    float q[kNQ], A[48];
    if (i < a.n) {
        site_features(a.pos, a.n, i, a.L[0], a.L[1], a.L[2], a.ncount, a.nidx, a.rc, q, A);
    } else {
#pragma unroll
        for (int f = 0; f < kNQ; f++) q[f] = features_only ? 0.f : sP[kMmu + f];  // a finite filler row (z = 0)
    }
    if (features_only) {
        if (i < a.n)
#pragma unroll
            for (int f = 0; f < kNQ; f++) a.q[(size_t)i * kNQ + f] = q[f];
        return;
    }
    float z[kNQ];
#pragma unroll
    for (int f = 0; f < kNQ; f++) z[f] = (q[f] - sP[kMmu + f]) / sP[kMsig + f];
    const float o = mlp_forward_wave(sP, sZ[threadIdx.x >> 6], z);
    if (i >= a.n) return;
    const float g = softplus(o);
    if (!isfinite(g)) atomicOr(&a.flags[1], kErrNonFinite);
    a.g[i] = (double)g;
    a.xg[i] = Rec4{a.pos[i], a.pos[a.n + i], a.pos[2 * a.n + i], (double)g};
}

// g and dg/dq of m samples (one thread per sample, the backward pass in registers)
__global__ __launch_bounds__(kBlock) void k_mlp_eval(int m, const float *__restrict__ qin, const float *__restrict__ P,
                                                     float *__restrict__ gout, float *__restrict__ dgdq) {
    __shared__ float sP[kNP];
    load_params(sP, P);
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    float z[kNQ];
#pragma unroll
    for (int f = 0; f < kNQ; f++) z[f] = (qin[(size_t)s * kNQ + f] - sP[kMU + f]) / sP[kSIG + f];
    float h1[kNH], a2[kNH];
#pragma unroll
    for (int c = 0; c < kNH; c++) {
        float a = sP[kB1 + c];
#pragma unroll
        for (int f = 0; f < kNQ; f++) a += sP[kW1 + c * kNQ + f] * z[f];
        h1[c] = a * sigm(a);
    }
    float o = sP[kB3];
#pragma unroll
    for (int c = 0; c < kNH; c++) {
        float a = sP[kB2 + c];
#pragma unroll
        for (int k = 0; k < kNH; k++) a += sP[kW2 + c * kNH + k] * h1[k];
        a2[c] = a;
        o += sP[kW3 + c] * (a * sigm(a));
    }
    gout[s] = softplus(o);
    if (!dgdq) return;
    const float go = sigm(o);
    float dh1[kNH];
#pragma unroll
    for (int k = 0; k < kNH; k++) dh1[k] = 0.0f;
#pragma unroll
    for (int c = 0; c < kNH; c++) {
        const float d2 = go * sP[kW3 + c] * silu_d(a2[c]);
#pragma unroll
        for (int k = 0; k < kNH; k++) dh1[k] += sP[kW2 + c * kNH + k] * d2;
    }
    float dz[kNQ];
#pragma unroll
    for (int f = 0; f < kNQ; f++) dz[f] = 0.0f;
#pragma unroll
    for (int c = 0; c < kNH; c++) {
        float a = sP[kB1 + c];
#pragma unroll
        for (int f = 0; f < kNQ; f++) a += sP[kW1 + c * kNQ + f] * z[f];
        const float d1 = dh1[c] * silu_d(a);
#pragma unroll
        for (int f = 0; f < kNQ; f++) dz[f] += sP[kW1 + c * kNQ + f] * d1;
    }
#pragma unroll
    for (int f = 0; f < kNQ; f++) dgdq[(size_t)s * kNQ + f] = dz[f] / sP[kSIG + f];
}

__device__ __forceinline__ float wave_sum(float v) {
    // xor butterfly: the same pairs are combined on every lane, so all lanes hold the same sum
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// grad-g terms of the atoms with W_j != 0: kGradgWaves wavefronts per workgroup, one atom each, sharing one
// copy of the parameters in LDS. Every wavefront of a workgroup runs the same number of rounds (a wavefront
// without an atom in the last one only takes part in its barriers).
constexpr int kGradgWaves = 4;
__global__ __launch_bounds__(64 * kGradgWaves) void k_mlp_gradg(MlpArgs a) {
    __shared__ float sP[kNP];
    // W1 and W2 transposed as well ([f][c] and [k][c]): the forward pass reads them across the lanes
    // (hidden unit c per lane) like the backward pass reads the originals, each without bank conflicts
    __shared__ float sW1t[kNQ * kNH], sW2t[kNH * kNH];
    __shared__ float sHw[kGradgWaves][kNH], sDw[kGradgWaves][kNH], sQw[kGradgWaves][kNQ],
        sDQw[kGradgWaves][kNQ], sAw[kGradgWaves][48];
    for (int q = threadIdx.x; q < kNH * kNQ; q += blockDim.x) {
        const int c = q / kNQ, f = q - c * kNQ;
        sW1t[f * kNH + c] = a.P[kW1 + q];
    }
    for (int q = threadIdx.x; q < kNH * kNH; q += blockDim.x) {
        const int c = q / kNH, k = q - c * kNH;
        sW2t[k * kNH + c] = a.P[kW2 + q];
    }
    load_params(sP, a.P);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float *sH = sHw[wv], *sD = sDw[wv], *sQ = sQw[wv], *sDQ = sDQw[wv], *sA = sAw[wv];
    const int n = a.n;
    const double rc2 = a.rc * a.rc;
    const float rcf = (float)a.rc;
    const int nw = *a.wcount;
    const int lgen = *a.list_gen;
    for (int base = blockIdx.x * kGradgWaves; base < nw; base += gridDim.x * kGradgWaves) {
        const int w = base + wv;
        const bool act = w < nw;
        const int j = act ? a.wlist[w] : 0;
        // j's reverse slots from the cache when searched on the current list (read before the barriers
        // below; rewritten only after the closing one)
        const bool cached = a.rstamp[j] == lgen;
        const double xj = a.pos[j], yj = a.pos[n + j], zj = a.pos[2 * n + j];
        const int cnt = act ? a.ncount[j] : 0;
        // 1. features: per-lane partial sums over its slots, then a butterfly over the wavefront
        float q8[8], A[48];
#pragma unroll
        for (int c = 0; c < 8; c++) q8[c] = 0.0f;
#pragma unroll
        for (int t = 0; t < 48; t++) A[t] = 0.0f;
        for (int slot = lane; slot < cnt; slot += 64) {
            const int k = a.nidx[(size_t)slot * n + j];
            const Rec4 pk = a.xl[k];
            const double ux = min_image_w(pk.x - xj, a.L[0]), uy = min_image_w(pk.y - yj, a.L[1]),
                         uz = min_image_w(pk.z - zj, a.L[2]);
            const double r2 = ux * ux + uy * uy + uz * uz;
            if (!(r2 < rc2)) continue;
            const double rd = sqrt(r2);
            const float r = (float)rd, ir = (float)(1.0 / rd);
            float g[8], Y[25];
            radial<float, 8>(r, rcf, g, (float *)nullptr);
            ylm_real<float, 4>((float)ux * ir, (float)uy * ir, (float)uz * ir, Y);
#pragma unroll
            for (int c = 0; c < 8; c++) q8[c] += g[c];
#pragma unroll
            for (int t = 1; t < 25; t++) {
                A[t - 1] += g[0] * Y[t];
                A[24 + t - 1] += g[1] * Y[t];
            }
        }
#pragma unroll
        for (int c = 0; c < 8; c++) q8[c] = wave_sum(q8[c]);
#pragma unroll
        for (int t = 0; t < 48; t++) A[t] = wave_sum(A[t]);
        if (lane < 48) {
            float v = 0.0f;
#pragma unroll
            for (int t = 0; t < 48; t++) v = t == lane ? A[t] : v;
            sA[lane] = v;
        }
        if (lane < 8) {
            float v = 0.0f;
#pragma unroll
            for (int c = 0; c < 8; c++) v = c == lane ? q8[c] : v;
            sQ[lane] = v;
        }
        __syncthreads();
        if (lane >= 8 && lane < kNQ) {
            const int c = (lane - 8) >> 2, l = ((lane - 8) & 3) + 1;
            float s = 0.0f;
            for (int t = l * l; t <= l * l + 2 * l; t++) s += sA[24 * c + t - 1] * sA[24 * c + t - 1];
            sQ[lane] = s;
        }
        __syncthreads();
        if (lane < kNQ) sQ[lane] = (sQ[lane] - sP[kMU + lane]) / sP[kSIG + lane];  // z
        __syncthreads();
        // 2. network forward and backward, hidden unit `lane` per lane
        float a1 = sP[kB1 + lane];
#pragma unroll
        for (int f = 0; f < kNQ; f++) a1 += sW1t[f * kNH + lane] * sQ[f];
        sH[lane] = a1 * sigm(a1);
        __syncthreads();
        float a2 = sP[kB2 + lane];
        for (int k = 0; k < kNH; k++) a2 += sW2t[k * kNH + lane] * sH[k];
        const float o = wave_sum(sP[kW3 + lane] * (a2 * sigm(a2))) + sP[kB3];
        const float go = sigm(o);
        sD[lane] = go * sP[kW3 + lane] * silu_d(a2);
        __syncthreads();
        float dh = 0.0f;
        for (int c = 0; c < kNH; c++) dh += sP[kW2 + c * kNH + lane] * sD[c];
        const float d1 = dh * silu_d(a1);
        __syncthreads();
        sH[lane] = d1;
        __syncthreads();
        if (lane < kNQ) {
            float t = 0.0f;
            for (int c = 0; c < kNH; c++) t += sP[kW1 + c * kNQ + lane] * sH[c];
            sDQ[lane] = t / sP[kSIG + lane];
        }
        __syncthreads();
        // 3. h_jk = W_j dg_j/du_jk for every slot; written at (w, slot) and at (slot of j in k's list, k)
        const float Wj = (float)a.W[j];
        float *hp = a.hpair + (size_t)(act ? w : 0) * a.max_nbr * 3;
        for (int slot = lane; slot < cnt; slot += 64) {
            const int k = a.nidx[(size_t)slot * n + j];
            const Rec4 pk = a.xl[k];
            const double ux = min_image_w(pk.x - xj, a.L[0]), uy = min_image_w(pk.y - yj, a.L[1]),
                         uz = min_image_w(pk.z - zj, a.L[2]);
            const double r2 = ux * ux + uy * uy + uz * uz;
            float h0 = 0.0f, h1 = 0.0f, h2 = 0.0f;
            if (r2 < rc2) {
                const double rd = sqrt(r2);
                const float r = (float)rd, ir = (float)(1.0 / rd);
                const float ex = (float)ux * ir, ey = (float)uy * ir, ez = (float)uz * ir;
                float g[8], dg[8], Y[25], dY[75];
                radial<float, 8>(r, rcf, g, dg);
                ylm_real_grad<float, 4>(ex, ey, ez, ir, Y, dY);
                // radial sums: d q_c / du = g_c' uhat
                float sr = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; c++) sr += sDQ[c] * dg[c];
                h0 = sr * ex;
                h1 = sr * ey;
                h2 = sr * ez;
                // sum_m A^2: d/du = 2 sum_m A_clm (g_c' uhat Y_lm + g_c grad Y_lm)
#pragma unroll
                for (int c = 0; c < 2; c++)
#pragma unroll
                    for (int t = 1; t < 25; t++) {
                        const int l = t < 4 ? 1 : (t < 9 ? 2 : (t < 16 ? 3 : 4));
                        const float wq = 2.0f * sDQ[8 + 4 * c + l - 1] * sA[24 * c + t - 1];
                        const float rad = wq * dg[c] * Y[t], ang = wq * g[c];
                        h0 += rad * ex + ang * dY[3 * t];
                        h1 += rad * ey + ang * dY[3 * t + 1];
                        h2 += rad * ez + ang * dY[3 * t + 2];
                    }
                h0 *= Wj;
                h1 *= Wj;
                h2 *= Wj;
            }
            hp[3 * slot] = h0;
            hp[3 * slot + 1] = h1;
            hp[3 * slot + 2] = h2;
            // k's gather reads this term only inside the feature cutoff; the cache covers every slot
            // that can come inside it before the next list build
            const bool need = r2 < rc2 * (1.0 + 1e-9);
            if (!need && !(!cached && r2 < a.rrev2)) continue;
            int kk = -1;
            if (cached) {
                kk = a.rslot[(size_t)j * a.max_nbr + slot];
            } else {
                const int ck = a.ncount[k];
                for (int b0 = 0; b0 < ck && kk < 0; b0 += 8) {
                    int v[8];
#pragma unroll
                    for (int u = 0; u < 8; u++) v[u] = b0 + u < ck ? a.nidx[(size_t)(b0 + u) * n + k] : -1;
#pragma unroll
                    for (int u = 0; u < 8; u++)
                        if (v[u] == j && kk < 0) kk = b0 + u;
                }
                a.rslot[(size_t)j * a.max_nbr + slot] = kk;
            }
            if (kk < 0) {
                atomicOr(&a.flags[1], kErrAsym);
            } else if (need) {
                const size_t st = (size_t)a.max_nbr * n, o2 = (size_t)kk * n + k;
                a.hrev[o2] = h0;
                a.hrev[st + o2] = h1;
                a.hrev[2 * st + o2] = h2;
            }
        }
        __syncthreads();
        if (act && !cached && lane == 0) a.rstamp[j] = lgen;
    }
}

// ---- compaction of the atoms with W_j != 0 (ordered) ----
__global__ __launch_bounds__(kBlock) void k_wcount(int n, const double *__restrict__ W, int *__restrict__ bcnt) {
    __shared__ int sh[kBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long m = __ballot(i < n && W[i] != 0.0);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kBlock / 64; w++) s += sh[w];
        bcnt[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_wscatter(int n, const double *__restrict__ W, const int *__restrict__ boff,
                                                     int *__restrict__ widx, int *__restrict__ wlist) {
    __shared__ int sh[kBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool f = i < n && W[i] != 0.0;
    const unsigned long long m = __ballot(f);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = __popcll(m);
    __syncthreads();
    int off = boff[blockIdx.x];
    for (int q = 0; q < w; q++) off += sh[q];
    if (i < n) {
        const int r = off + __popcll(m & ((1ull << lane) - 1ull));
        widx[i] = f ? r : -1;
        if (f) wlist[r] = i;
    }
}

// ---- training ----
// forward and backward of B samples starting at s0; dL/do = 2 (o - t) / m_norm. The second-layer
// pre-activations are parked in the d2 rows of T between the two passes.
__global__ __launch_bounds__(kBlock) void k_mlp_fb(int B, int s0, const float *__restrict__ qin,
                                                   const float *__restrict__ tin, const float *__restrict__ P,
                                                   float m_norm, float *__restrict__ T) {
    __shared__ float sP[kNP];
    load_params(sP, P);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int s = s0 + b;
    float z[kNQ];
#pragma unroll
    for (int f = 0; f < kNQ; f++) {
        z[f] = (qin[(size_t)s * kNQ + f] - sP[kMU + f]) / sP[kSIG + f];
        T[(size_t)(kTZ + f) * B + b] = z[f];
    }
    float o = sP[kB3];
    {
        float h1[kNH];
#pragma unroll
        for (int c = 0; c < kNH; c++) {
            float a = sP[kB1 + c];
#pragma unroll
            for (int f = 0; f < kNQ; f++) a += sP[kW1 + c * kNQ + f] * z[f];
            h1[c] = a * sigm(a);
            T[(size_t)(kTH1 + c) * B + b] = h1[c];
        }
        for (int c = 0; c < kNH; c++) {
            float a = sP[kB2 + c];
#pragma unroll
            for (int k = 0; k < kNH; k++) a += sP[kW2 + c * kNH + k] * h1[k];
            const float h2 = a * sigm(a);
            T[(size_t)(kTH2 + c) * B + b] = h2;
            T[(size_t)(kTD2 + c) * B + b] = a;
            o += sP[kW3 + c] * h2;
        }
    }
    const float r = o - tin[s];
    const float go = 2.0f * r / m_norm;
    T[(size_t)kTGO * B + b] = go;
    T[(size_t)kTLOSS * B + b] = r * r / m_norm;
    float dh1[kNH];
#pragma unroll
    for (int k = 0; k < kNH; k++) dh1[k] = 0.0f;
    for (int c = 0; c < kNH; c++) {
        float *t2 = T + (size_t)(kTD2 + c) * B + b;
        const float d2 = go * sP[kW3 + c] * silu_d(*t2);
        *t2 = d2;
#pragma unroll
        for (int k = 0; k < kNH; k++) dh1[k] += sP[kW2 + c * kNH + k] * d2;
    }
#pragma unroll
    for (int c = 0; c < kNH; c++) {
        float a = sP[kB1 + c];
#pragma unroll
        for (int f = 0; f < kNQ; f++) a += sP[kW1 + c * kNQ + f] * z[f];
        T[(size_t)(kTD1 + c) * B + b] = dh1[c] * silu_d(a);
    }
}

// gradient of parameter p (p in [kW1, kNP)) and, for p == kNP, the batch loss: a wavefront sums
// over the batch in lane-strided order, then a fixed butterfly
__global__ __launch_bounds__(kBlock) void k_mlp_wgrad(int B, const float *__restrict__ T, float *__restrict__ grad,
                                                      double *__restrict__ loss_acc) {
    const int p = kW1 + blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p > kNP) return;
    int ra, rb = -1;  // sum_b T[ra][b] * T[rb][b]  (rb < 0: sum_b T[ra][b])
    if (p < kB1) {
        const int c = (p - kW1) / kNQ, f = (p - kW1) % kNQ;
        ra = kTD1 + c;
        rb = kTZ + f;
    } else if (p < kW2) {
        ra = kTD1 + (p - kB1);
    } else if (p < kB2) {
        const int c = (p - kW2) / kNH, k = (p - kW2) % kNH;
        ra = kTD2 + c;
        rb = kTH1 + k;
    } else if (p < kW3) {
        ra = kTD2 + (p - kB2);
    } else if (p < kB3) {
        ra = kTGO;
        rb = kTH2 + (p - kW3);
    } else if (p == kB3) {
        ra = kTGO;
    } else {
        ra = kTLOSS;
    }
    const float *A = T + (size_t)ra * B;
    const float *Bv = rb >= 0 ? T + (size_t)rb * B : nullptr;
    float acc = 0.0f;
    for (int b = lane; b < B; b += 64) acc += Bv ? A[b] * Bv[b] : A[b];
    acc = wave_sum(acc);
    if (lane == 0) {
        if (p < kNP)
            grad[p] = acc;
        else if (loss_acc)
            *loss_acc += (double)acc;
    }
}

__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m1,
                           float *__restrict__ m2, float lr, float bc1, float bc2) {
    const int p = kW1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    const float g = grad[p];
    const float a = 0.9f * m1[p] + 0.1f * g, v = 0.999f * m2[p] + 0.001f * g * g;
    m1[p] = a;
    m2[p] = v;
    P[p] -= lr * (a / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

// feature statistics of m samples: mu_f and sig_f = std_f (population), fixed-order sums in FP64
__global__ __launch_bounds__(kBlock) void k_mlp_norm(int m, const float *__restrict__ qin, float *__restrict__ P) {
    __shared__ double sh[kBlock];
    const int f = blockIdx.x;
    double s = 0.0;
    for (int q = threadIdx.x; q < m; q += kBlock) s += (double)qin[(size_t)q * kNQ + f];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double mu = sh[0] / m;
    __syncthreads();
    s = 0.0;
    for (int q = threadIdx.x; q < m; q += kBlock) {
        const double d = (double)qin[(size_t)q * kNQ + f] - mu;
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P[kMU + f] = (float)mu;
        P[kSIG + f] = (float)(sqrt(sh[0] / m) + 1e-6);
    }
}

__global__ void k_zero_double(double *p) { *p = 0.0; }

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
static MlpArgs mlp_args(ap_ctx *c, int n, const double *box) {
    MlpArgs a;
    a.pos = c->pos;
    a.n = n;
    for (int q = 0; q < 3; q++) a.L[q] = box[q];
    a.rc = c->mlp_rc;
    a.ncount = c->nbr_cnt;
    a.nidx = c->nbr_idx;
    a.max_nbr = c->max_nbr;
    a.P = c->mlp_p;
    a.g = c->g;
    a.xg = c->xg;
    a.xl = c->xl;
    a.rslot = c->rslot;
    a.rstamp = c->rstamp;
    a.list_gen = c->list_gen;
    a.rrev2 = rslot_reach2(c);
    a.q = nullptr;
    a.W = c->W;
    a.wlist = c->wlist;
    a.wcount = c->d_flags + 4;
    a.hpair = c->hpair;
    a.hrev = c->hrev;
    a.flags = c->d_flags;
    return a;
}

void launch_mlp_indicator(ap_ctx *c, int n, const double *box) {
    MlpArgs a = mlp_args(c, n, box);
    k_mlp_indicator<<<(n + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(a, 0);
}

void launch_mlp_gradg(ap_ctx *c, int n, const double *box) {
    const int nb = (n + kBlock - 1) / kBlock;
    k_wcount<<<nb, kBlock, 0, c->stream>>>(n, c->W, c->blk_cnt);
    launch_scan(c, c->blk_cnt, c->blk_cnt + nb, nb, c->d_flags + 4, nullptr);
    k_wscatter<<<nb, kBlock, 0, c->stream>>>(n, c->W, c->blk_cnt + nb, c->widx, c->wlist);
    MlpArgs a = mlp_args(c, n, box);
    // enough workgroups to fill the GPU (each loads the parameters once), not one per atom
    k_mlp_gradg<<<std::max(1, std::min((n + kGradgWaves - 1) / kGradgWaves, 2048)), 64 * kGradgWaves, 0,
                  c->stream>>>(a);
}

int mlp_alloc(ap_ctx *c) {
    if (c->mlp_p) return AP_OK;
    const size_t np = (size_t)c->n_cap * c->max_nbr * 3;
    int rc = hip_check(c, hipMalloc(&c->mlp_p, sizeof(float) * kNP), "network parameters");
    if (!rc) rc = hip_check(c, hipMalloc(&c->hpair, sizeof(float) * np), "indicator pair buffer");
    if (!rc) rc = hip_check(c, hipMalloc(&c->hrev, sizeof(float) * np), "indicator reverse buffer");
    if (!rc) rc = hip_check(c, hipMalloc(&c->widx, sizeof(int) * c->n_cap), "indicator list");
    if (!rc) rc = hip_check(c, hipMalloc(&c->wlist, sizeof(int) * c->n_cap), "indicator list");
    return rc;
}

void mlp_free(ap_ctx *c) {
    void *b[] = {c->mlp_p, c->hpair, c->hrev, c->widx, c->wlist, c->mlp_T, c->mlp_grad, c->mlp_m1, c->mlp_m2,
                 c->mlp_loss};
    for (void *p : b) (void)hipFree(p);
    c->mlp_p = nullptr;
    c->hpair = c->hrev = nullptr;
    c->widx = c->wlist = nullptr;
    c->mlp_T = c->mlp_grad = c->mlp_m1 = c->mlp_m2 = nullptr;
    c->mlp_loss = nullptr;
    c->mlp_T_cap = 0;
}

static int ensure_train_scratch(ap_ctx *c, int B) {
    if (!c->mlp_grad) {
        int rc = hip_check(c, hipMalloc(&c->mlp_grad, sizeof(float) * kNP), "network gradient");
        if (!rc) rc = hip_check(c, hipMalloc(&c->mlp_m1, sizeof(float) * kNP), "Adam state");
        if (!rc) rc = hip_check(c, hipMalloc(&c->mlp_m2, sizeof(float) * kNP), "Adam state");
        if (!rc) rc = hip_check(c, hipMalloc(&c->mlp_loss, sizeof(double)), "loss");
        if (rc) return rc;
    }
    if (B > c->mlp_T_cap) {
        (void)hipFree(c->mlp_T);
        c->mlp_T = nullptr;
        int rc = hip_check(c, hipMalloc(&c->mlp_T, sizeof(float) * (size_t)kTRows * B), "training scratch");
        if (rc) return rc;
        c->mlp_T_cap = B;
    }
    return AP_OK;
}

// one batch: activations, then every parameter gradient (and the batch loss added to *mlp_loss)
static void batch_grad(ap_ctx *c, int B, int s0, const float *q, const float *t, const float *P, float m_norm) {
    k_mlp_fb<<<(B + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(B, s0, q, t, P, m_norm, c->mlp_T);
    const int npar = kNP - kW1 + 1;  // parameters and the loss
    k_mlp_wgrad<<<(npar + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, c->stream>>>(B, c->mlp_T, c->mlp_grad,
                                                                                   c->mlp_loss);
}

}  // namespace ap

using namespace ap;

extern "C" {

int ap_set_mlp(ap_ctx *c, const float *params, double rc) {
    if (!c) return AP_E_ARG;
    if (!params || !(rc > 0.0)) return set_error(c, AP_E_ARG, "network parameters and a feature cutoff > 0 needed");
    int r = mlp_alloc(c);
    if (r) return r;
    r = hip_check(c, hipMemcpyAsync(c->mlp_p, params, sizeof(float) * kNP, hipMemcpyDeviceToDevice, c->stream),
                  "network parameters");
    if (r) return r;
    c->mlp_rc = rc;
    c->have_mlp = true;
    c->list_r = -1;
    return sync_and_check(c);
}

int ap_mlp_features(ap_ctx *c, int n, const double *pos, const ap_box *box, double rc, float *q) {
    if (!c) return AP_E_ARG;
    if (n <= 0 || n > c->n_cap || !pos || !box || !q || !(rc > 0.0)) return set_error(c, AP_E_ARG, "mlp_features");
    for (int a = 0; a < 3; a++)
        if (!(rc < 0.5 * box->L[a])) return set_error(c, AP_E_BOX, "feature cutoff must be below half the box");
    int r = prepare_positions(c, n, pos, box->L);
    if (!r) r = ensure_list(c, n, box->L, rc, true);
    if (r) return r;
    MlpArgs a = mlp_args(c, n, box->L);
    a.rc = rc;
    a.q = q;
    k_mlp_indicator<<<(n + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(a, 1);
    c->list_r = -1;  // this list is not the evaluation's list
    return sync_and_check(c);
}

int ap_mlp_eval(ap_ctx *c, int m, const float *q, const float *params, float *g, float *dgdq) {
    if (!c) return AP_E_ARG;
    if (m <= 0 || !q || !params || !g) return set_error(c, AP_E_ARG, "mlp_eval");
    k_mlp_eval<<<(m + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(m, q, params, g, dgdq);
    return sync_and_check(c);
}

int ap_mlp_loss_grad(ap_ctx *c, int m, const float *q, const float *target, const float *params, float *grad,
                     double *loss) {
    if (!c) return AP_E_ARG;
    if (m <= 0 || !q || !target || !params || !grad) return set_error(c, AP_E_ARG, "mlp_loss_grad");
    int r = ensure_train_scratch(c, m);
    if (r) return r;
    k_zero_double<<<1, 1, 0, c->stream>>>(c->mlp_loss);
    batch_grad(c, m, 0, q, target, params, (float)m);
    r = hip_check(c, hipMemsetAsync(grad, 0, sizeof(float) * kW1, c->stream), "gradient");
    if (!r)
        r = hip_check(c, hipMemcpyAsync(grad + kW1, c->mlp_grad + kW1, sizeof(float) * (kNP - kW1),
                                        hipMemcpyDeviceToDevice, c->stream), "gradient");
    double l = 0.0;
    if (!r) r = hip_check(c, hipMemcpyAsync(&l, c->mlp_loss, sizeof(double), hipMemcpyDeviceToHost, c->stream), "loss");
    if (!r) r = sync_and_check(c);
    if (!r && loss) *loss = l;
    return r;
}

int ap_mlp_train(ap_ctx *c, int m, const float *q, const float *target, int batch, int epochs, double lr,
                 int fit_norm, float *params, double *loss_hist) {
    if (!c) return AP_E_ARG;
    if (m <= 0 || !q || !target || !params || batch <= 0 || epochs < 0 || !(lr > 0.0))
        return set_error(c, AP_E_ARG, "mlp_train");
    const int B = std::min(batch, m);
    int r = ensure_train_scratch(c, B);
    if (r) return r;
    if (fit_norm) k_mlp_norm<<<kNQ, kBlock, 0, c->stream>>>(m, q, params);
    r = hip_check(c, hipMemsetAsync(c->mlp_m1, 0, sizeof(float) * kNP, c->stream), "Adam state");
    if (!r) r = hip_check(c, hipMemsetAsync(c->mlp_m2, 0, sizeof(float) * kNP, c->stream), "Adam state");
    if (r) return r;
    const int nbat = m / B;  // the ragged tail of each epoch is left out
    long long step = 0;
    for (int e = 0; e < epochs; e++) {
        k_zero_double<<<1, 1, 0, c->stream>>>(c->mlp_loss);
        for (int bt = 0; bt < nbat; bt++) {
            batch_grad(c, B, bt * B, q, target, params, (float)B);
            step++;
            const float bc1 = (float)(1.0 - std::pow(0.9, (double)step)),
                        bc2 = (float)(1.0 - std::pow(0.999, (double)step));
            k_mlp_adam<<<(kNP - kW1 + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(params, c->mlp_grad, c->mlp_m1,
                                                                                   c->mlp_m2, (float)lr, bc1, bc2);
        }
        if (loss_hist) {
            double l = 0.0;
            r = hip_check(c, hipMemcpyAsync(&l, c->mlp_loss, sizeof(double), hipMemcpyDeviceToHost, c->stream),
                          "loss");
            if (!r) r = hip_check(c, hipStreamSynchronize(c->stream), "loss");
            if (r) return r;
            loss_hist[e] = l / nbat;
        }
    }
    return sync_and_check(c);
}

}  // extern "C"
