// Device math for the short-range four-centre integrals: McMurchie-Davidson
// Hermite expansion coefficients (Sec. 2.2 recurrences), the Hermite
// auxiliary integrals R_{tuv} (Sec. 2.3, eq. R_recursion) and the Boys
// function from an LDS-resident table.  Everything is templated on the
// angular momenta so that the loops unroll into registers.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace pbcjk {

// Cartesian component exponents, order x^l, x^(l-1)y, ... (xx xy xz yy yz zz).
__host__ __device__ constexpr int cx(int l, int k) { return l == 0 ? 0 : l == 1 ? (k == 0) : (k == 0 ? 2 : (k == 1 || k == 2) ? 1 : 0); }
__host__ __device__ constexpr int cy(int l, int k) { return l == 0 ? 0 : l == 1 ? (k == 1) : (k == 3 ? 2 : (k == 1 || k == 4) ? 1 : 0); }
__host__ __device__ constexpr int cz(int l, int k) { return l == 0 ? 0 : l == 1 ? (k == 2) : (k == 5 ? 2 : (k == 2 || k == 4) ? 1 : 0); }

// One axis of Hermite coefficients with E^{00}_0 = 1 (the Gaussian factor
// exp(-ab/p X_AB^2) is carried by the pair prefactor).
template <int LA, int LB>
struct EAxis {
    double v[LA + 1][LB + 1][LA + LB + 1];
};

template <int LA, int LB>
__device__ __forceinline__ void herm_axis(double h, double xa, double xb, EAxis<LA, LB> &E)
{
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int t = 0; t <= LA + LB; ++t) E.v[i][j][t] = 0.0;
    E.v[0][0][0] = 1.0;
#pragma unroll
    for (int i = 0; i < LA; ++i)
#pragma unroll
        for (int t = 0; t <= i + 1; ++t) {
            double r = 0.0;
            if (t >= 1) r += h * E.v[i][0][t - 1];
            if (t <= i) r += xa * E.v[i][0][t];
            if (t + 1 <= i) r += (t + 1) * E.v[i][0][t + 1];
            E.v[i + 1][0][t] = r;
        }
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j < LB; ++j)
#pragma unroll
            for (int t = 0; t <= i + j + 1; ++t) {
                double r = 0.0;
                if (t >= 1) r += h * E.v[i][j][t - 1];
                if (t <= i + j) r += xb * E.v[i][j][t];
                if (t + 1 <= i + j) r += (t + 1) * E.v[i][j][t + 1];
                E.v[i][j + 1][t] = r;
            }
}

// R_{tuv} = R^0_{tuv} for t+u+v <= L from R^m_{000}, m = 0..L.
template <int L>
__device__ __forceinline__ void herm_R(const double (&R0)[L + 1], double X, double Y, double Z,
                                       double (&R)[L + 1][L + 1][L + 1])
{
    double T[L + 1][L + 1][L + 1][L + 1];
#pragma unroll
    for (int n = L; n >= 0; --n)
#pragma unroll
        for (int t = 0; t <= L - n; ++t)
#pragma unroll
            for (int u = 0; u <= L - n - t; ++u)
#pragma unroll
                for (int v = 0; v <= L - n - t - u; ++v) {
                    double r;
                    if (t == 0 && u == 0 && v == 0) r = R0[n];
                    else if (t > 0) r = (t >= 2 ? (t - 1) * T[n + 1][t - 2][u][v] : 0.0) + X * T[n + 1][t - 1][u][v];
                    else if (u > 0) r = (u >= 2 ? (u - 1) * T[n + 1][0][u - 2][v] : 0.0) + Y * T[n + 1][0][u - 1][v];
                    else r = (v >= 2 ? (v - 1) * T[n + 1][0][0][v - 2] : 0.0) + Z * T[n + 1][0][0][v - 1];
                    T[n][t][u][v] = r;
                }
#pragma unroll
    for (int t = 0; t <= L; ++t)
#pragma unroll
        for (int u = 0; u <= L - t; ++u)
#pragma unroll
            for (int v = 0; v <= L - t - u; ++v) R[t][u][v] = T[0][t][u][v];
}

// F_m(T), m = 0..L, FP64.  tab: LDS copy of rows L..L+kBoysTerms-1,
// layout [k][j].  Below kBoysTmax: Taylor expansion of F_L about the
// nearest grid point, then downward recursion; above: asymptotic F_0 and
// upward recursion.
template <int L>
__device__ __forceinline__ void boys_f64(double T, const double *__restrict__ tab, double (&F)[L + 1])
{
    if (T < kBoysTmax) {
        int k = __double2int_rn(T * (1.0 / kBoysStep));
        double x = k * kBoysStep - T;
        const double *r = tab + k * kBoysTerms;
        double s = r[kBoysTerms - 1];
#pragma unroll
        for (int j = kBoysTerms - 2; j >= 0; --j) s = r[j] + s * x * (1.0 / (j + 1));
        F[L] = s;
        if (L > 0) {
            double e = exp(-T);
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) * (1.0 / (2 * m + 1));
        }
    } else {
        double it = 1.0 / T;
        F[0] = 0.88622692545275801365 * sqrt(it);   // sqrt(pi)/2 / sqrt(T)
        if (L > 0) {
            double e = exp(-T);
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * (0.5 * it);
        }
    }
}

// R^m_{000} of the short-range kernel erfc(w r)/r at reduced exponent rho,
// T = |L|^2 (Sec. 2.3 Boys split):
//   (-2 rho)^m F_m(rho T) - c (-2 a')^m F_m(a' T),
//   a' = rho w^2/(rho + w^2), c = w/sqrt(rho + w^2).
template <int L>
__device__ __forceinline__ void sr_R0(double rho, double w2, double T, const double *__restrict__ tab,
                                      double (&R0)[L + 1])
{
    double den = 1.0 / (rho + w2);
    double ap = rho * w2 * den;
    double c = sqrt(w2 * den);
    double F1[L + 1], F2[L + 1];
    boys_f64<L>(rho * T, tab, F1);
    boys_f64<L>(ap * T, tab, F2);
    double f1 = 1.0, f2 = c;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        R0[m] = f1 * F1[m] - f2 * F2[m];
        f1 *= -2.0 * rho;
        f2 *= -2.0 * ap;
    }
}

}  // namespace pbcjk
