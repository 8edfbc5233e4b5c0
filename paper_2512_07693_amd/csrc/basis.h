// Radial channels and real spherical harmonics shared by the ACE and learned-indicator kernels.
#pragma once

#include "ap_internal.h"

namespace ap {

// ---------------------------------------------------------------------------------------------
// Basis functions (shared by the host table builder and the kernels)
// ---------------------------------------------------------------------------------------------
template <typename T>
__host__ __device__ __forceinline__ T klm(int l, int m) {
    double f = 1.0;
    for (int q = l - m + 1; q <= l + m; q++) f *= q;  // (l+m)!/(l-m)!
    return (T)sqrt((2.0 * l + 1.0) / (4.0 * kPi) / f);
}

// Real orthonormal harmonics at the unit vector (x, y, z), index l*l + l + m:
//   Y_l0 = K Q_l^0(z);  Y_lm = sqrt2 K Q_l^m(z) Re(x+iy)^m;  Y_l,-m = sqrt2 K Q_l^m(z) Im(x+iy)^m
// with Q_l^m(z) = d^m P_l / dz^m from the Legendre recurrence (no Condon-Shortley phase).
template <typename T, int LMAX>
__host__ __device__ __forceinline__ void ylm_real(T x, T y, T z, T *Y) {
    T C[LMAX + 1], S[LMAX + 1], Q[LMAX + 1][LMAX + 1];
    C[0] = T(1);
    S[0] = T(0);
#pragma unroll
    for (int m = 1; m <= LMAX; m++) {
        C[m] = x * C[m - 1] - y * S[m - 1];
        S[m] = x * S[m - 1] + y * C[m - 1];
    }
    T dfm = T(1);
#pragma unroll
    for (int m = 0; m <= LMAX; m++) {
        if (m > 0) dfm *= T(2 * m - 1);
        Q[m][m] = dfm;
        if (m + 1 <= LMAX) Q[m + 1][m] = T(2 * m + 1) * z * Q[m][m];
#pragma unroll
        for (int l = m + 2; l <= LMAX; l++)
            Q[l][m] = (T(2 * l - 1) * z * Q[l - 1][m] - T(l + m - 1) * Q[l - 2][m]) / T(l - m);
    }
    const T r2 = T(1.4142135623730951);
#pragma unroll
    for (int l = 0; l <= LMAX; l++) {
        Y[l * l + l] = klm<T>(l, 0) * Q[l][0];
#pragma unroll
        for (int m = 1; m <= l; m++) {
            const T k = r2 * klm<T>(l, m) * Q[l][m];
            Y[l * l + l + m] = k * C[m];
            Y[l * l + l - m] = k * S[m];
        }
    }
}

// The harmonics of one order m >= 0 at the unit vector (x, y, z), by the same recurrences as ylm_real:
// Y_lm and Y_l,-m for l = m..LMAX, stored at index l*l + l +- m of Y; cm, sm = Re, Im (x + iy)^m.
template <typename T, int LMAX>
__device__ __forceinline__ void ylm_real_order(int m, T z, T cm, T sm, T *Y) {
    T dfm = T(1);
#pragma unroll
    for (int k = 1; k <= LMAX; k++)
        if (k <= m) dfm *= T(2 * k - 1);
    const T r2 = T(1.4142135623730951);
    T qm2 = T(0), qm1 = T(0);
#pragma unroll
    for (int l = 0; l <= LMAX; l++) {
        if (l < m) continue;
        T q;
        if (l == m)
            q = dfm;
        else if (l == m + 1)
            q = T(2 * m + 1) * z * qm1;
        else
            q = (T(2 * l - 1) * z * qm1 - T(l + m - 1) * qm2) / T(l - m);
        qm2 = qm1;
        qm1 = q;
        if (m == 0) {
            Y[l * l + l] = klm<T>(l, 0) * q;
        } else {
            const T k = r2 * klm<T>(l, m) * q;
            Y[l * l + l + m] = k * cm;
            Y[l * l + l - m] = k * sm;
        }
    }
}

// Same harmonics and their gradient with respect to the unnormalised vector u (|u| = r):
// grad_u Y = (grad_p - (uhat . grad_p) uhat) / r for the polynomial p(x, y, z).
template <typename T, int LMAX>
__device__ __forceinline__ void ylm_real_grad(T x, T y, T z, T ir, T *Y, T *dY) {
    T C[LMAX + 1], S[LMAX + 1], Q[LMAX + 1][LMAX + 1], dQ[LMAX + 1][LMAX + 1];
    C[0] = T(1);
    S[0] = T(0);
#pragma unroll
    for (int m = 1; m <= LMAX; m++) {
        C[m] = x * C[m - 1] - y * S[m - 1];
        S[m] = x * S[m - 1] + y * C[m - 1];
    }
    T dfm = T(1);
#pragma unroll
    for (int m = 0; m <= LMAX; m++) {
        if (m > 0) dfm *= T(2 * m - 1);
        Q[m][m] = dfm;
        dQ[m][m] = T(0);
        if (m + 1 <= LMAX) {
            Q[m + 1][m] = T(2 * m + 1) * z * Q[m][m];
            dQ[m + 1][m] = T(2 * m + 1) * Q[m][m];
        }
#pragma unroll
        for (int l = m + 2; l <= LMAX; l++) {
            const T inv = T(1) / T(l - m);
            Q[l][m] = (T(2 * l - 1) * z * Q[l - 1][m] - T(l + m - 1) * Q[l - 2][m]) * inv;
            dQ[l][m] = (T(2 * l - 1) * (Q[l - 1][m] + z * dQ[l - 1][m]) - T(l + m - 1) * dQ[l - 2][m]) * inv;
        }
    }
    const T r2 = T(1.4142135623730951);
#pragma unroll
    for (int l = 0; l <= LMAX; l++) {
#pragma unroll
        for (int m = 0; m <= l; m++) {
            T px[2], py[2], pz[2], val[2];
            int idx[2];
            int cnt = 1;
            if (m == 0) {
                const T k = klm<T>(l, 0);
                val[0] = k * Q[l][0];
                px[0] = T(0);
                py[0] = T(0);
                pz[0] = k * dQ[l][0];
                idx[0] = l * l + l;
            } else {
                const T k = r2 * klm<T>(l, m);
                const T q = k * Q[l][m], dq = k * dQ[l][m], mm = T(m);
                val[0] = q * C[m];
                px[0] = q * mm * C[m - 1];
                py[0] = -q * mm * S[m - 1];
                pz[0] = dq * C[m];
                idx[0] = l * l + l + m;
                val[1] = q * S[m];
                px[1] = q * mm * S[m - 1];
                py[1] = q * mm * C[m - 1];
                pz[1] = dq * S[m];
                idx[1] = l * l + l - m;
                cnt = 2;
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                if (h >= cnt) break;
                const T rad = px[h] * x + py[h] * y + pz[h] * z;
                Y[idx[h]] = val[h];
                dY[3 * idx[h] + 0] = (px[h] - rad * x) * ir;
                dY[3 * idx[h] + 1] = (py[h] - rad * y) * ir;
                dY[3 * idx[h] + 2] = (pz[h] - rad * z) * ir;
            }
        }
    }
}

// Chebyshev radial channels g_n = T_n(2r/rc - 1) fc(r), fc = (1 + cos(pi r/rc))/2, and derivatives.
template <typename T, int NMAX>
__device__ __forceinline__ void radial(T r, T rc, T *g, T *dg) {
    const T x = T(2) * r / rc - T(1), dx = T(2) / rc;
    const T a = T(kPi) * r / rc;
    const T fc = T(0.5) * (T(1) + cos(a)), dfc = -T(0.5) * T(kPi) / rc * sin(a);
    T t0 = T(1), t1 = x, d0 = T(0), d1 = T(1);
    g[0] = fc;
    if (dg) dg[0] = dfc;
#pragma unroll
    for (int n = 1; n < NMAX; n++) {
        if (n > 1) {
            const T t2 = T(2) * x * t1 - t0, d2 = T(2) * t1 + T(2) * x * d1 - d0;
            t0 = t1;
            t1 = t2;
            d0 = d1;
            d1 = d2;
        }
        g[n] = t1 * fc;
        if (dg) dg[n] = d1 * dx * fc + t1 * dfc;
    }
}

}  // namespace ap
