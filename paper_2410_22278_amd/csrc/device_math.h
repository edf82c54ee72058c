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
// exp(-ab/p X_AB^2) is carried by the pair prefactor), in the value type T
// (FP32 for the quartets of the single-precision work lists).
template <int LA, int LB, typename T = double>
struct EAxis {
    T v[LA + 1][LB + 1][LA + LB + 1];
};

template <int LA, int LB, typename T = double>
__device__ __forceinline__ void herm_axis(T h, T xa, T xb, EAxis<LA, LB, T> &E)
{
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int t = 0; t <= LA + LB; ++t) E.v[i][j][t] = T(0);
    E.v[0][0][0] = T(1);
#pragma unroll
    for (int i = 0; i < LA; ++i)
#pragma unroll
        for (int t = 0; t <= i + 1; ++t) {
            T r = T(0);
            if (t >= 1) r += h * E.v[i][0][t - 1];
            if (t <= i) r += xa * E.v[i][0][t];
            if (t + 1 <= i) r += T(t + 1) * E.v[i][0][t + 1];
            E.v[i + 1][0][t] = r;
        }
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j < LB; ++j)
#pragma unroll
            for (int t = 0; t <= i + j + 1; ++t) {
                T r = T(0);
                if (t >= 1) r += h * E.v[i][j][t - 1];
                if (t <= i + j) r += xb * E.v[i][j][t];
                if (t + 1 <= i + j) r += T(t + 1) * E.v[i][j][t + 1];
                E.v[i][j + 1][t] = r;
            }
}

// R_{tuv} = R^0_{tuv} for t+u+v <= L from R^m_{000}, m = 0..L.
template <int L, typename V>
__device__ __forceinline__ void herm_R(const V (&R0)[L + 1], V X, V Y, V Z, V (&R)[L + 1][L + 1][L + 1])
{
    V T[L + 1][L + 1][L + 1][L + 1];
#pragma unroll
    for (int n = L; n >= 0; --n)
#pragma unroll
        for (int t = 0; t <= L - n; ++t)
#pragma unroll
            for (int u = 0; u <= L - n - t; ++u)
#pragma unroll
                for (int v = 0; v <= L - n - t - u; ++v) {
                    V r;
                    if (t == 0 && u == 0 && v == 0) r = R0[n];
                    else if (t > 0) r = (t >= 2 ? V(t - 1) * T[n + 1][t - 2][u][v] : V(0)) + X * T[n + 1][t - 1][u][v];
                    else if (u > 0) r = (u >= 2 ? V(u - 1) * T[n + 1][0][u - 2][v] : V(0)) + Y * T[n + 1][0][u - 1][v];
                    else r = (v >= 2 ? V(v - 1) * T[n + 1][0][0][v - 2] : V(0)) + Z * T[n + 1][0][0][v - 1];
                    T[n][t][u][v] = r;
                }
#pragma unroll
    for (int t = 0; t <= L; ++t)
#pragma unroll
        for (int u = 0; u <= L - t; ++u)
#pragma unroll
            for (int v = 0; v <= L - t - u; ++v) R[t][u][v] = T[0][t][u][v];
}

// FP64 reciprocal and reciprocal square root: the hardware approximation
// refined by two Newton steps (correct to about one unit in the last place,
// which is all the kernels need; no IEEE-rounded division sequence).
__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double fast_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    // y <- y (3 - x y^2) / 2, twice
    double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// Natural logarithm for screening radii only: exponent by frexp, log2 of the
// mantissa from the FP32 hardware logarithm, plus 1e-6, which bounds the
// error of the rest (about 1.5e-7 absolute), so the result is never below
// ln x.  A radius from it is at least the exact one and larger by a relative
// 1e-6 / ln(x) at most, so a screen built on it keeps every term the exact
// screen keeps and adds only terms at the threshold.
__device__ __forceinline__ double screen_log(double x)
{
    const int e = __builtin_amdgcn_frexp_exp(x);
    const float m = (float)__builtin_amdgcn_frexp_mant(x);   // [0.5, 1)
    return ((double)e + (double)__builtin_amdgcn_logf(m)) * 0.69314718055994530942 + 1e-6;
}

// F_m(T), m = 0..L, FP64.  tab: LDS copy of rows L..L+kBoysTerms-1,
// layout [k][j].  Below kBoysTmax: Taylor expansion of F_L about the
// nearest grid point, then downward recursion; above: asymptotic F_0 and
// upward recursion.
// PREDIV: the table row holds F_{L+j}(T_k) / j! (the per-lane kernels
// divide while copying the table to LDS), so Horner needs one FMA a term.
template <int L, int STRIDE = kBoysTerms, bool PREDIV = false>
__device__ __forceinline__ void boys_f64(double T, const double *__restrict__ tab, const double *__restrict__ etab,
                                         double (&F)[L + 1])
{
    if (T < kBoysTmax) {
        int k = __double2int_rn(T * (1.0 / kBoysStep));
        double x = k * kBoysStep - T;
        const double *r = tab + k * STRIDE;
        double s = r[kBoysTerms - 1];
        if (PREDIV) {
#pragma unroll
            for (int j = kBoysTerms - 2; j >= 0; --j) s = fma(s, x, r[j]);
        } else {
#pragma unroll
            for (int j = kBoysTerms - 2; j >= 0; --j) s = r[j] + s * x * (1.0 / (j + 1));
        }
        F[L] = s;
        if (L > 0) {
            // e^{-T} = e^{-T_k} e^{x}, |x| <= h/2: e^{x} by its Taylor series
            constexpr double c[9] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040,
                                     1.0 / 40320};
            double ex = c[8];
#pragma unroll
            for (int j = 7; j >= 0; --j) ex = fma(ex, x, c[j]);
            const double e = etab[k] * ex;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) * (1.0 / (2 * m + 1));
        }
    } else {
        const double rs = fast_rsqrt(T);
        F[0] = 0.88622692545275801365 * rs;   // sqrt(pi)/2 / sqrt(T)
        if (L > 0) {
            const double it = rs * rs;
            // above kBoysTmax e^{-T} changes F_m, m <= 8, by a relative 3e-8 at
            // most, so its FP32 value (hardware exp2) is ample
            const double e = (double)__builtin_amdgcn_exp2f((float)(-1.44269504088896340736 * T));
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * (0.5 * it);
        }
    }
}

// R^m_{000} of the short-range kernel erfc(w r)/r at reduced exponent rho,
// T = |L|^2 (Sec. 2.3 Boys split):
//   (-2 rho)^m F_m(rho T) - c (-2 a')^m F_m(a' T),
//   a' = rho w^2/(rho + w^2), c = w/sqrt(rho + w^2).
template <int L, int STRIDE = kBoysTerms, bool PREDIV = false>
__device__ __forceinline__ void sr_R0(double rho, double w2, double T, const double *__restrict__ tab,
                                      const double *__restrict__ etab, double (&R0)[L + 1])
{
    const double rs = fast_rsqrt(rho + w2);
    const double den = rs * rs;
    const double ap = rho * w2 * den;
    const double c = sqrt(w2) * rs;
    double F1[L + 1], F2[L + 1];
    boys_f64<L, STRIDE, PREDIV>(rho * T, tab, etab, F1);
    boys_f64<L, STRIDE, PREDIV>(ap * T, tab, etab, F2);
    double f1 = 1.0, f2 = c;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        R0[m] = f1 * F1[m] - f2 * F2[m];
        f1 *= -2.0 * rho;
        f2 *= -2.0 * ap;
    }
}

// FP32 F_m(T) from the same table, pre-divided by j! as for PREDIV (six
// Taylor terms suffice in single precision); the offset from the grid point
// is formed in FP64.
template <int L>
__device__ __forceinline__ void boys_f32(double Td, const double *__restrict__ tab, float (&F)[L + 1])
{
    const float T = (float)Td;
    if (Td < kBoysTmax) {
        int k = __double2int_rn(Td * (1.0 / kBoysStep));
        float x = (float)(k * kBoysStep - Td);
        const double *r = tab + k * kBoysTerms;   // F_{L+j}(T_k) / j!
        float s = (float)r[5];
#pragma unroll
        for (int j = 4; j >= 0; --j) s = fmaf(s, x, (float)r[j]);
        F[L] = s;
        if (L > 0) {
            float e = __expf(-T);
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = (2.0f * T * F[m + 1] + e) * (1.0f / (2 * m + 1));
        }
    } else {
        float it = 1.0f / T;
        F[0] = 0.88622692545f * sqrtf(it);
        if (L > 0) {
            float e = __expf(-T);
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * (0.5f * it);
        }
    }
}

// Short-range R^m_{000} in FP32 for the quartets of the FP32 work lists.
// Their entries are chosen so that rho T >= 1 for every quartet and shift:
// both Boys arguments are then outside the small-argument region, where the
// difference of the two terms cancels (that region is evaluated in FP64, on
// the FP64 lists).  The Boys arguments are formed in FP64.
template <int L>
__device__ __forceinline__ void sr_R0_f32(double rho, double w2, double T, const double *__restrict__ tab,
                                          float (&R0)[L + 1])
{
    const float rf = (float)rho, w2f = (float)w2;
    const float s = __builtin_amdgcn_rsqf(rf + w2f);
    const float apf = rf * w2f * (s * s);
    float F1[L + 1], F2[L + 1];
    boys_f32<L>(rho * T, tab, F1);
    boys_f32<L>((double)apf * T, tab, F2);
    float f1 = 1.0f, f2 = __builtin_amdgcn_sqrtf(w2f) * s;
    const float r2 = -2.0f * rf, a2 = -2.0f * apf;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        R0[m] = f1 * F1[m] - f2 * F2[m];
        f1 *= r2;
        f2 *= a2;
    }
}

constexpr double kTwoPi52 = 34.98683665524972497;   // 2 pi^{5/2}

// Real-space sphere of one primitive quartet (Sec. 2.4, eq.
// pbc_eri_real_cutoff_implementation): false when C2e (1 - c) <= delta, else
// rad2 = (1/p + 1/q + 1/w^2) ln(C2e (1 - c)/delta).  Shared by the
// neighbour-list builder and the build kernels so that both take the same
// decisions.
__device__ __forceinline__ bool quartet_sphere(const PairRec &b, const PairRec &k, double w2, double dR,
                                               double &rad2)
{
    const double p = b.p, q = k.p;
    const double ip = b.pad[0], iq = k.pad[0];          // 1/p, 1/q
    const double rho = fast_rcp(ip + iq);
    const double c = sqrt(w2) * fast_rsqrt(rho + w2);
    const double C2e = b.Cb * k.Cb * kTwoPi52 * ip * iq * fast_rsqrt(p + q);
    const double arg = C2e * (1.0 - c) * fast_rcp(dR);
    if (!(arg > 1.0)) return false;
    rad2 = (ip + iq + fast_rcp(w2)) * screen_log(arg);
    return true;
}

__device__ __forceinline__ void lat_image(const LatArgs &lat, const double cen[3], double n0, double n1, double n2,
                                          double L[3])
{
#pragma unroll
    for (int x = 0; x < 3; ++x) L[x] = cen[x] - (n0 * lat.M[x] + n1 * lat.M[3 + x] + n2 * lat.M[6 + x]);
}

// The nearest lattice translate of cen (its rounded fractional coordinates).
__device__ __forceinline__ void nearest_translate(const LatArgs &lat, const double cen[3], double n[3])
{
#pragma unroll
    for (int x = 0; x < 3; ++x)
        n[x] = rint(cen[0] * lat.Minv[x] + cen[1] * lat.Minv[3 + x] + cen[2] * lat.Minv[6 + x]);
}

// Calls f(L, |L|^2) for every translate L = cen - R1 in the box of lattice
// points that covers the sphere |L|^2 < rad2 (and |L|^2 <= rcap2 when
// rcap2 > 0), testing each.  A translate n inside the sphere has
// |f_x - n_x| = |sum_j L_j Minv[j][x]| <= |L| span_x < rad span_x for the
// fractional coordinates f of cen, so the box holds the integers strictly
// within rad span_x of f_x (rad slightly raised against rounding).
template <class F>
__device__ __forceinline__ void for_images_box(const LatArgs &lat, const double cen[3], double rad2, double rcap2,
                                               F &&f)
{
    double fr[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) fr[x] = cen[0] * lat.Minv[x] + cen[1] * lat.Minv[3 + x] + cen[2] * lat.Minv[6 + x];
    const double rad = rad2 * fast_rsqrt(rad2);
    const double r = rad * (1.0 + 1e-9) + 1e-9;
    int lo[3], hi[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        lo[x] = (int)ceil(fr[x] - r * lat.span[x]);
        hi[x] = (int)floor(fr[x] + r * lat.span[x]);
    }
    for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
        for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
            for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
                double Lb[3];
                lat_image(lat, cen, (double)n0, (double)n1, (double)n2, Lb);
                const double Lb2 = Lb[0] * Lb[0] + Lb[1] * Lb[1] + Lb[2] * Lb[2];
                if (Lb2 < rad2 && !(rcap2 > 0 && Lb2 > rcap2)) f(Lb, Lb2);
            }
}

// A radius at least sqrt(rad2): the FP32 square root (within a few units of
// 2^-24 of it, rad2 rounded to FP32 included) raised by a relative 1e-6.
__device__ __forceinline__ double radius_above(double rad2)
{
    return (double)(__builtin_amdgcn_sqrtf((float)rad2) * 1.000001f);
}

// Calls f(L, |L|^2) for every lattice translate L = cen - R1 with
// |L|^2 < rad2 (and |L|^2 <= rcap2 when rcap2 > 0).  Fast path: when
// |L0| <= Rmin - sqrt(rad2) for the rounded image L0, no other translate can
// lie inside the sphere.
template <class F>
__device__ __forceinline__ void for_images(const LatArgs &lat, const double cen[3], double rad2, double rcap2,
                                           F &&f)
{
    if (!(rad2 > 0.0)) return;   // empty sphere (also keeps the box below finite)
    double n[3], L[3];
    nearest_translate(lat, cen, n);
    lat_image(lat, cen, n[0], n[1], n[2], L);
    const double L2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    const double gap = lat.Rmin - radius_above(rad2);
    if (gap >= 0.0 && L2 <= gap * gap) {
        if (L2 < rad2 && !(rcap2 > 0 && L2 > rcap2)) f(L, L2);
        return;
    }
    for_images_box(lat, cen, rad2, rcap2, f);
}

// As for_images, starting from the translate by the lattice vector S (an
// integer combination of the lattice vectors) instead of the rounded image:
// the caller passes the nearest translate of a nearby point (the group
// centres of a work-list entry), which is that of most of its quartets, so
// the fast path skips the rounding.  |cen - S| <= Rmin - sqrt(rad2) again
// leaves no other translate inside the sphere, whatever S is.
template <class F>
__device__ __forceinline__ void for_images_from(const LatArgs &lat, const double cen[3], const double S[3],
                                                double rad2, double rcap2, F &&f)
{
    if (!(rad2 > 0.0)) return;
    double L[3] = {cen[0] - S[0], cen[1] - S[1], cen[2] - S[2]};
    const double L2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    const double gap = lat.Rmin - radius_above(rad2);
    if (gap >= 0.0 && L2 <= gap * gap) {
        if (L2 < rad2 && !(rcap2 > 0 && L2 > rcap2)) f(L, L2);
        return;
    }
    for_images_box(lat, cen, rad2, rcap2, f);
}

}  // namespace pbcjk
