/*
 * oracle.c -- plain FP64 CPU evaluation of the Gamma-point periodic Coulomb
 * (J) and exchange (K) matrices over contracted Cartesian Gaussians with
 * Ewald splitting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Written from the paper (Wang, Hait, Unzueta, Zhang, Martinez, "Fast and
 * Scalable GPU-Accelerated Quantum Chemistry for Periodic Systems with
 * Gaussian Orbitals"):
 *   - primitive normalisation                      Sec. 2.1, eq. local_normalization
 *   - Hermite expansion and E recurrences          Sec. 2.2, eqs. E_recursion_i/j/0/out
 *   - Gamma overlap                                Sec. 2.2, eq. pbc_overlap_formula
 *   - Boys split and short-range difference        Sec. 2.3, eq. boys_function_split
 *   - R auxiliary integrals and recurrence         Sec. 2.3, eqs. R_definition, R_recursion
 *   - periodic ERI (real + reciprocal + self)      Sec. 2.4, eq. pbc_eri_general_final
 *   - local-pair cutoffs                           Sec. 2.4, eqs. pbc_eri_pair_cutoff_*,
 *                                                   pbc_eri_cauchy_schwarz_cutoff_*
 *   - quartet screen: short-range Cauchy-Schwarz   Sec. 2.4, eq. local_cauchy_schwarz_bound
 *     factors from the pairs' own (ab|ab)_SR
 *   - real-space Ewald sphere per quartet          Sec. 2.4, eq. pbc_eri_real_cutoff_*
 *   - J and K at the Gamma point                   Sec. 2.5-2.6
 *   - point-charge Ewald energy (test utility)     Sec. 2.8, eq. nuclear_repulsion_energy
 *   - lattice sphere enumeration, minimum image    Sec. 3.3
 *
 * Everything is evaluated in the plainest order: ordered bra and ket local
 * primitive pairs (no permutational symmetry), one primitive quartet at a
 * time, one lattice image at a time.  The reciprocal-space sum is exposed as
 * pair structure factors so that the Python side can form the G sums with
 * matrix products; the self term needs only the Gamma overlap.
 *
 * Readings of the paper that this file adopts (the paper is silent, garbled
 * or inconsistent there) are stated at the point of use: the pair-R bound
 * prefactor, the constant C per primitive, the density-weighted quartet
 * screen and the global G sphere.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXL 2                  /* s, p, d */
#define ORC_MAXNC 6                 /* Cartesian components of a d shell */
#define ORC_MAXLQ (4 * ORC_MAXL)    /* total angular momentum of a quartet */
#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* public input description (mirrored by a ctypes Structure)              */
/* ---------------------------------------------------------------------- */
typedef struct {
    double cell[9];        /* rows: lattice vectors a, b, c (bohr)          */
    int natom;
    const double *xyz;     /* natom*3                                       */
    int nshell;
    const int *sh_atom, *sh_l, *sh_pure, *sh_nprim;
    const double *exps;    /* concatenated per shell                        */
    const double *coefs;   /* raw contraction coefficients                  */
    double omega;
    double d_pair_R, d_pair_cs, d_ewald_R, d_ewald_K, d_schwarz;
    double r_cut;          /* > 0: cap on |A-B(R2)| and on |P-Q-R1|          */
    double g_cut;          /* > 0: cap on |G|                                */
} orc_sys;

/* ---------------------------------------------------------------------- */
/* small helpers                                                          */
/* ---------------------------------------------------------------------- */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* k-th Cartesian component of angular momentum l, order x^l, x^(l-1)y, ... */
static void cart_comp(int l, int k, int c[3])
{
    int n = 0;
    c[0] = c[1] = c[2] = 0;
    for (int lx = l; lx >= 0; --lx)
        for (int ly = l - lx; ly >= 0; --ly) {
            if (n == k) { c[0] = lx; c[1] = ly; c[2] = l - lx - ly; return; }
            ++n;
        }
}

static double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* Sec. 2.1, eq. local_normalization: normalises one Cartesian primitive. */
static double prim_norm(double a, const int c[3])
{
    int l = c[0] + c[1] + c[2];
    double num = pow(8.0 * a, l) * fact(c[0]) * fact(c[1]) * fact(c[2]);
    double den = fact(2 * c[0]) * fact(2 * c[1]) * fact(2 * c[2]);
    return pow(2.0 * a / ORC_PI, 0.75) * sqrt(num / den);
}

/* The single constant C per primitive used in the screening bounds (the
 * paper folds normalisation and contraction into one number per pGTO, Sec.
 * 2.1).  Reading: the largest component normalisation of the shell,
 * |c| (2a/pi)^{3/4} (4a)^{l/2}. */
static double bound_const(double a, int l, double c)
{
    return fabs(c) * pow(2.0 * a / ORC_PI, 0.75) * pow(4.0 * a, 0.5 * l);
}

/* ---------------------------------------------------------------------- */
/* Boys function F_m(T), m = 0..mmax                                       */
/* Series F_m = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) and        */
/* downward recursion below T = 35; erf form of F_0 (Sec. 2.3, eq.          */
/* boys_function_erf_form) and upward recursion above.                     */
/* ---------------------------------------------------------------------- */
void orc_boys(int mmax, double T, double *F)
{
    if (T < 35.0) {
        double term = 1.0 / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= 2.0 * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        double et = exp(-T);
        F[mmax] = et * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + et) / (2 * m + 1);
    } else {
        double st = sqrt(T), et = exp(-T);
        F[0] = 0.5 * sqrt(ORC_PI) * erf(st) / st;
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - et) / (2.0 * T);
    }
}

/* ---------------------------------------------------------------------- */
/* Hermite expansion coefficients for one axis (Sec. 2.2, E recurrences).  */
/* E[(i*(lb+1)+j)*(la+lb+1)+t], i<=la, j<=lb, t<=la+lb.                     */
/* ---------------------------------------------------------------------- */
static void hermite_E(int la, int lb, double p, double XPA, double XPB, double E00, double *E)
{
    int nt = la + lb + 1;
#define EIDX(i, j, t) (((i) * (lb + 1) + (j)) * nt + (t))
    memset(E, 0, sizeof(double) * (la + 1) * (lb + 1) * nt);
    double h = 0.5 / p;
    E[EIDX(0, 0, 0)] = E00;
    for (int i = 0; i < la; ++i)
        for (int t = 0; t <= i + 1; ++t) {
            double v = XPA * (t <= i ? E[EIDX(i, 0, t)] : 0.0);
            if (t >= 1) v += h * E[EIDX(i, 0, t - 1)];
            if (t + 1 <= i) v += (t + 1) * E[EIDX(i, 0, t + 1)];
            E[EIDX(i + 1, 0, t)] = v;
        }
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j < lb; ++j)
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = XPB * (t <= i + j ? E[EIDX(i, j, t)] : 0.0);
                if (t >= 1) v += h * E[EIDX(i, j, t - 1)];
                if (t + 1 <= i + j) v += (t + 1) * E[EIDX(i, j, t + 1)];
                E[EIDX(i, j + 1, t)] = v;
            }
#undef EIDX
}

/* ---------------------------------------------------------------------- */
/* Hermite auxiliary integrals R_{tuv} = R^0_{tuv} for t+u+v <= L from      */
/* R^m_{000}, m = 0..L (Sec. 2.3, eq. R_recursion).  Out: (L+1)^3 array.    */
/* ---------------------------------------------------------------------- */
static void hermite_R(int L, const double *R000, const double X[3], double *out)
{
    int n1 = L + 1;
    static __thread double Rn[(ORC_MAXLQ + 1) * (ORC_MAXLQ + 1) * (ORC_MAXLQ + 1) * (ORC_MAXLQ + 1)];
#define RI(n, t, u, v) ((((n) * n1 + (t)) * n1 + (u)) * n1 + (v))
    for (int n = L; n >= 0; --n)
        for (int t = 0; t <= L - n; ++t)
            for (int u = 0; u <= L - n - t; ++u)
                for (int v = 0; v <= L - n - t - u; ++v) {
                    double r;
                    if (t == 0 && u == 0 && v == 0) r = R000[n];
                    else if (t > 0) r = (t >= 2 ? (t - 1) * Rn[RI(n + 1, t - 2, u, v)] : 0.0)
                                        + X[0] * Rn[RI(n + 1, t - 1, u, v)];
                    else if (u > 0) r = (u >= 2 ? (u - 1) * Rn[RI(n + 1, 0, u - 2, v)] : 0.0)
                                        + X[1] * Rn[RI(n + 1, 0, u - 1, v)];
                    else r = (v >= 2 ? (v - 1) * Rn[RI(n + 1, 0, 0, v - 2)] : 0.0)
                             + X[2] * Rn[RI(n + 1, 0, 0, v - 1)];
                    Rn[RI(n, t, u, v)] = r;
                }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L; ++u)
            for (int v = 0; v <= L; ++v)
                out[(t * n1 + u) * n1 + v] = (t + u + v <= L) ? Rn[RI(0, t, u, v)] : 0.0;
#undef RI
}

/* kernel selector for R^m_000 */
enum { KER_COULOMB = 0, KER_SR = 1, KER_LR = 2 };

/* R^m_000 for the chosen two-electron kernel at reduced exponent rho and
 * T = |L|^2 (Sec. 2.3, eq. boys_function_split; Sec. 2.4 real-space term):
 *   Coulomb: (-2 rho)^m F_m(rho T)
 *   LR     : c (-2 a')^m F_m(a' T),   a' = rho w^2/(rho+w^2), c = w/sqrt(rho+w^2)
 *   SR     : Coulomb - LR                                                  */
static void kernel_R000(int kind, int L, double rho, double omega, double T, double *R000)
{
    double F[ORC_MAXLQ + 1], G[ORC_MAXLQ + 1];
    if (kind != KER_LR) orc_boys(L, rho * T, F);
    if (kind != KER_COULOMB) {
        double w2 = omega * omega;
        double ap = rho * w2 / (rho + w2);
        orc_boys(L, ap * T, G);
        double c = omega / sqrt(rho + w2);
        double f1 = 1.0, f2 = 1.0;
        for (int m = 0; m <= L; ++m) {
            double lr = c * f2 * G[m];
            R000[m] = (kind == KER_SR) ? f1 * F[m] - lr : lr;
            f1 *= -2.0 * rho; f2 *= -2.0 * ap;
        }
    } else {
        double f1 = 1.0;
        for (int m = 0; m <= L; ++m) { R000[m] = f1 * F[m]; f1 *= -2.0 * rho; }
    }
}

/* ---------------------------------------------------------------------- */
/* molecular primitive integrals (test entry points)                       */
/* ---------------------------------------------------------------------- */

/* One element of a primitive quartet block for monomial Gaussians (Sec. 2.4
 * McMurchie-Davidson form): components ca, cb (bra) and cc, cd (ket) given
 * as exponent triples, Eab/Ecd the three axes of Hermite coefficients with
 * tables of width la+lb+1 and lc+ld+1, R the Hermite integrals in an
 * (L+1)^3 array.  Without the 2 pi^{5/2}/(pq sqrt(p+q)) prefactor. */
static double quartet_elem(int lb, int ld, int ntab, int ntcd, const int ca[3], const int cb[3],
                           const int cc[3], const int cd[3], const double *Eab[3], const double *Ecd[3],
                           const double *R, int n1)
{
    const double *ex = Eab[0] + (ca[0] * (lb + 1) + cb[0]) * ntab;
    const double *ey = Eab[1] + (ca[1] * (lb + 1) + cb[1]) * ntab;
    const double *ez = Eab[2] + (ca[2] * (lb + 1) + cb[2]) * ntab;
    const double *fx = Ecd[0] + (cc[0] * (ld + 1) + cd[0]) * ntcd;
    const double *fy = Ecd[1] + (cc[1] * (ld + 1) + cd[1]) * ntcd;
    const double *fz = Ecd[2] + (cc[2] * (ld + 1) + cd[2]) * ntcd;
    double sum = 0.0;
    for (int t = 0; t <= ca[0] + cb[0]; ++t)
    for (int u = 0; u <= ca[1] + cb[1]; ++u)
    for (int v = 0; v <= ca[2] + cb[2]; ++v) {
        double eab = ex[t] * ey[u] * ez[v];
        if (eab == 0.0) continue;
        double inner = 0.0;
        for (int tt = 0; tt <= cc[0] + cd[0]; ++tt)
        for (int uu = 0; uu <= cc[1] + cd[1]; ++uu)
        for (int vv = 0; vv <= cc[2] + cd[2]; ++vv) {
            double s = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
            inner += s * fx[tt] * fy[uu] * fz[vv] * R[((t + tt) * n1 + (u + uu)) * n1 + (v + vv)];
        }
        sum += eab * inner;
    }
    return sum;
}

/* Cartesian block of one primitive quartet for monomial (not normalised)
 * Gaussians, any kernel (Sec. 2.4 McMurchie-Davidson form):
 *   (ab|cd) = 2 pi^{5/2}/(pq sqrt(p+q)) sum_t E^{ab}_t sum_s (-1)^{|s|} E^{cd}_s R_{t+s}(P-Q)
 * out[((ia*nb+ib)*nc+ic)*nd+id]. */
static void quartet_block(int la, int lb, int lc, int ld,
                          double p, const double *Eab[3], double q, const double *Ecd[3],
                          const double PQ[3], int kind, double omega, double *out)
{
    int L = la + lb + lc + ld, n1 = L + 1;
    double rho = p * q / (p + q);
    double T = PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2];
    double R000[ORC_MAXLQ + 1];
    kernel_R000(kind, L, rho, omega, T, R000);
    static __thread double R[(ORC_MAXLQ + 1) * (ORC_MAXLQ + 1) * (ORC_MAXLQ + 1)];
    hermite_R(L, R000, PQ, R);
    double pref = 2.0 * pow(ORC_PI, 2.5) / (p * q * sqrt(p + q));
    int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    int ntab = la + lb + 1, ntcd = lc + ld + 1;
    for (int ia = 0; ia < na; ++ia) {
        int ca[3]; cart_comp(la, ia, ca);
        for (int ib = 0; ib < nb; ++ib) {
            int cb[3]; cart_comp(lb, ib, cb);
            for (int ic = 0; ic < nc; ++ic) {
                int cc[3]; cart_comp(lc, ic, cc);
                for (int id = 0; id < nd; ++id) {
                    int cd[3]; cart_comp(ld, id, cd);
                    out[((ia * nb + ib) * nc + ic) * nd + id] =
                        pref * quartet_elem(lb, ld, ntab, ntcd, ca, cb, cc, cd, Eab, Ecd, R, n1);
                }
            }
        }
    }
}

/* Largest diagonal element (ab|ab), over the Cartesian components ab, of the
 * short-range (erfc) self-integral of one primitive pair whose components
 * carry the normalisations Na, Nb (the pair's E tables include its Gaussian
 * factor).  Its square root bounds every short-range integral of the pair
 * by the Cauchy-Schwarz inequality (Sec. 2.4, eq. local_cauchy_schwarz_bound;
 * the erfc kernel is positive definite). */
static double sr_self_max(int la, int lb, double p, const double *Eab[3], const double *Na, const double *Nb,
                          double omega)
{
    int L = 2 * (la + lb), n1 = L + 1;
    double R000[ORC_MAXLQ + 1], zero[3] = {0.0, 0.0, 0.0};
    kernel_R000(KER_SR, L, 0.5 * p, omega, 0.0, R000);
    double *R = (double *)malloc(sizeof(double) * n1 * n1 * n1);
    hermite_R(L, R000, zero, R);
    double pref = 2.0 * pow(ORC_PI, 2.5) / (p * p * sqrt(2.0 * p));
    double best = 0.0;
    for (int ia = 0; ia < ncart(la); ++ia) {
        int ca[3]; cart_comp(la, ia, ca);
        for (int ib = 0; ib < ncart(lb); ++ib) {
            int cb[3]; cart_comp(lb, ib, cb);
            double v = pref * quartet_elem(lb, lb, la + lb + 1, la + lb + 1, ca, cb, ca, cb, Eab, Eab, R, n1);
            v *= Na[ia] * Na[ia] * Nb[ib] * Nb[ib];
            if (v > best) best = v;
        }
    }
    free(R);
    return best;
}

/* E tables of one primitive pair (three axes) for centres A, B. */
static void pair_E(int la, int lb, double a, double b, const double A[3], const double B[3],
                   double *E /* 3 * (la+1)(lb+1)(la+lb+1) */, double P[3])
{
    double p = a + b, mu = a * b / p;
    int sz = (la + 1) * (lb + 1) * (la + lb + 1);
    for (int x = 0; x < 3; ++x) {
        P[x] = (a * A[x] + b * B[x]) / p;
        double XAB = A[x] - B[x];
        hermite_E(la, lb, p, P[x] - A[x], P[x] - B[x], exp(-mu * XAB * XAB), E + x * sz);
    }
}

/* Test entry point: molecular primitive ERI block for monomial Gaussians.
 * kind: 0 = 1/r, 1 = erfc(w r)/r, 2 = erf(w r)/r. */
void orc_eri_prim(int kind, int la, int lb, int lc, int ld,
                  double a, double b, double c, double d,
                  const double *A, const double *B, const double *C, const double *D,
                  double omega, double *out)
{
    double Eab[3 * 3 * 3 * 5], Ecd[3 * 3 * 3 * 5], P[3], Q[3], PQ[3];
    pair_E(la, lb, a, b, A, B, Eab, P);
    pair_E(lc, ld, c, d, C, D, Ecd, Q);
    int sab = (la + 1) * (lb + 1) * (la + lb + 1), scd = (lc + 1) * (ld + 1) * (lc + ld + 1);
    const double *eab[3] = {Eab, Eab + sab, Eab + 2 * sab};
    const double *ecd[3] = {Ecd, Ecd + scd, Ecd + 2 * scd};
    for (int x = 0; x < 3; ++x) PQ[x] = P[x] - Q[x];
    quartet_block(la, lb, lc, ld, a + b, eab, c + d, ecd, PQ, kind, omega, out);
}

/* Test entry point: primitive overlap block for monomial Gaussians
 * (Sec. 2.2, eq. pbc_overlap_formula for one local pair). */
void orc_overlap_prim(int la, int lb, double a, double b, const double *A, const double *B,
                      double *out)
{
    double E[3 * 3 * 3 * 5], P[3];
    pair_E(la, lb, a, b, A, B, E, P);
    int sz = (la + 1) * (lb + 1) * (la + lb + 1), nt = la + lb + 1;
    double f = pow(ORC_PI / (a + b), 1.5);
    for (int ia = 0; ia < ncart(la); ++ia) {
        int ca[3]; cart_comp(la, ia, ca);
        for (int ib = 0; ib < ncart(lb); ++ib) {
            int cb[3]; cart_comp(lb, ib, cb);
            double v = f;
            for (int x = 0; x < 3; ++x) v *= E[x * sz + (ca[x] * (lb + 1) + cb[x]) * nt];
            out[ia * ncart(lb) + ib] = v;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* lattice (Sec. 3.3)                                                      */
/* ---------------------------------------------------------------------- */
typedef struct {
    double M[9];      /* rows: a, b, c                          */
    double Minv[9];   /* inverse of M                           */
    double V;         /* cell volume                            */
    double B[9];      /* rows: reciprocal vectors, a_i.b_j = 2pi delta */
} lattice_t;

static void lattice_init(const double *cell, lattice_t *L)
{
    memcpy(L->M, cell, 9 * sizeof(double));
    const double *m = cell;
    double det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6])
               + m[2] * (m[3] * m[7] - m[4] * m[6]);
    double *iv = L->Minv;
    iv[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    iv[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    iv[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    iv[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    iv[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    iv[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    iv[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    iv[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    iv[8] = (m[0] * m[4] - m[1] * m[3]) / det;
    L->V = fabs(det);
    /* B = 2 pi M^{-T}: row i of B = 2 pi * column i of Minv */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) L->B[i * 3 + j] = 2.0 * ORC_PI * iv[j * 3 + i];
}

/* lattice vector n0 a + n1 b + n2 c */
static void lat_vec(const double *rows, const int n[3], double out[3])
{
    for (int x = 0; x < 3; ++x) out[x] = n[0] * rows[x] + n[1] * rows[3 + x] + n[2] * rows[6 + x];
}

/* fractional index f with x = f0 a + f1 b + f2 c: f = x M^{-1} */
static void frac(const double *Minv, const double x[3], double f[3])
{
    for (int j = 0; j < 3; ++j) f[j] = x[0] * Minv[j] + x[1] * Minv[3 + j] + x[2] * Minv[6 + j];
}

/* Minimum-image offset (Sec. 3.3, eq. lattice_image_min_norm): x - R round(R^{-1} x). */
static void min_image(const lattice_t *L, const double x[3], double out[3])
{
    double f[3], R[3]; int n[3];
    frac(L->Minv, x, f);
    for (int j = 0; j < 3; ++j) n[j] = (int)lround(f[j]);
    lat_vec(L->M, n, R);
    for (int j = 0; j < 3; ++j) out[j] = x[j] - R[j];
}

/* Enumerate lattice vectors of `rows` (inverse `rinv`) inside the sphere
 * |R - c| < r: bounding parallelepiped from the floor/ceil of the fractional
 * indices of the corners of the bounding cube, then the sphere test (Sec.
 * 3.3).  Calls cb(R, n, user) for each vector; returns the count. */
typedef void (*lat_cb)(const double R[3], const int n[3], void *user);
static long enum_sphere(const double *rows, const double *rinv, const double c[3], double r,
                        lat_cb cb, void *user)
{
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (int k = 0; k < 8; ++k) {
        double corner[3] = {c[0] + ((k & 1) ? r : -r), c[1] + ((k & 2) ? r : -r),
                            c[2] + ((k & 4) ? r : -r)};
        double f[3];
        frac(rinv, corner, f);
        for (int j = 0; j < 3; ++j) {
            int fl = (int)floor(f[j]), ce = (int)ceil(f[j]);
            if (fl < lo[j]) lo[j] = fl;
            if (ce > hi[j]) hi[j] = ce;
        }
    }
    long cnt = 0;
    int n[3];
    for (n[0] = lo[0]; n[0] <= hi[0]; ++n[0])
        for (n[1] = lo[1]; n[1] <= hi[1]; ++n[1])
            for (n[2] = lo[2]; n[2] <= hi[2]; ++n[2]) {
                double R[3];
                lat_vec(rows, n, R);
                double d2 = 0;
                for (int x = 0; x < 3; ++x) d2 += (R[x] - c[x]) * (R[x] - c[x]);
                if (d2 < r * r) { if (cb) cb(R, n, user); ++cnt; }
            }
    return cnt;
}

/* ---------------------------------------------------------------------- */
/* basis and local primitive pairs (Sec. 2.4 cutoffs, Sec. 3.1 layout)     */
/* ---------------------------------------------------------------------- */
typedef struct {
    int atom, l, nprim, ao;     /* ao: first Cartesian AO index             */
    const double *a;            /* exponents                                */
    double *c;                  /* renormalised contraction coefficients    */
} shell_t;

typedef struct {
    int sa, sb, ia, ib;          /* shells and primitive indices             */
    int la, lb;
    double a, b, p;
    double A[3], B[3], P[3];     /* B is the image position B + R2           */
    double ca, cb;               /* contraction coefficients                 */
    double Ca, Cb;               /* bound constants                          */
    double Kab;                  /* exp(-ab/p |A - B(R2)|^2)                 */
    double Q;                    /* short-range Cauchy-Schwarz factor (quartet screen) */
    double *E;                   /* 3 axes of Hermite coefficients            */
    int n2[3];                   /* lattice index of the image offset         */
    double Na[ORC_MAXNC], Nb[ORC_MAXNC];  /* component normalisations         */
    double S0;                   /* c_a c_b (pi/p)^{3/2}                      */
} pair_t;

typedef struct {
    lattice_t lat;
    int nshell, nbfc;
    shell_t *sh;
    double *cstore;
    double amin;
    long npair;
    pair_t *pair;
    double *Epool;
    const orc_sys *in;
} ctx_t;

/* Contracted shell rescaled to unit single-centre self-overlap; the
 * crystalline function itself stays unnormalised (Sec. 2.1). */
static void renormalise(int l, int n, const double *a, const double *c_in, double *c)
{
    double s = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            s += c_in[i] * c_in[j] * pow(2.0 * sqrt(a[i] * a[j]) / (a[i] + a[j]), l + 1.5);
    for (int i = 0; i < n; ++i) c[i] = c_in[i] / sqrt(s);
}

typedef struct { ctx_t *X; int sa, sb, ia, ib; double dmin[3]; double X0, Y0, mu, rcap2;
                 pair_t *out; long n; long cap; } pair_user;

static void pair_cb(const double R[3], const int n[3], void *u_)
{
    pair_user *u = (pair_user *)u_;
    double d[3], r2 = 0;
    for (int x = 0; x < 3; ++x) { d[x] = u->dmin[x] - R[x]; r2 += d[x] * d[x]; }
    double g = exp(-u->mu * r2);
    /* keep iff both local-pair bounds exceed their thresholds (strict), and
     * the optional image cap holds */
    if (!(u->X0 * g > u->X->in->d_pair_R)) return;
    if (!(u->Y0 * g > u->X->in->d_pair_cs)) return;
    if (u->rcap2 > 0 && r2 > u->rcap2) return;
    if (u->out) {
        if (u->n >= u->cap) { u->n++; return; }
        pair_t *P = &u->out[u->n];
        const shell_t *A = &u->X->sh[u->sa], *B = &u->X->sh[u->sb];
        P->sa = u->sa; P->sb = u->sb; P->ia = u->ia; P->ib = u->ib;
        P->la = A->l; P->lb = B->l;
        P->a = A->a[u->ia]; P->b = B->a[u->ib]; P->p = P->a + P->b;
        const double *xa = u->X->in->xyz + 3 * A->atom;
        for (int x = 0; x < 3; ++x) { P->A[x] = xa[x]; P->B[x] = xa[x] - d[x]; }
        P->ca = A->c[u->ia]; P->cb = B->c[u->ib];
        P->Ca = bound_const(P->a, A->l, P->ca);
        P->Cb = bound_const(P->b, B->l, P->cb);
        P->Kab = g;
        for (int x = 0; x < 3; ++x) P->n2[x] = n[x];
    }
    u->n++;
}

static void comp_norms(int l, double a, double *N);

static void ctx_free(ctx_t *X)
{
    if (!X) return;
    free(X->sh); free(X->cstore); free(X->pair); free(X->Epool);
    memset(X, 0, sizeof(*X));
}

static int ctx_build(const orc_sys *in, ctx_t *X)
{
    memset(X, 0, sizeof(*X));
    X->in = in;
    lattice_init(in->cell, &X->lat);
    X->nshell = in->nshell;
    X->sh = (shell_t *)calloc(in->nshell, sizeof(shell_t));
    int ntot = 0;
    for (int s = 0; s < in->nshell; ++s) ntot += in->sh_nprim[s];
    X->cstore = (double *)malloc(sizeof(double) * (ntot > 0 ? ntot : 1));
    int off = 0, ao = 0;
    X->amin = 1e300;
    for (int s = 0; s < in->nshell; ++s) {
        shell_t *S = &X->sh[s];
        S->atom = in->sh_atom[s]; S->l = in->sh_l[s]; S->nprim = in->sh_nprim[s];
        if (S->l < 0 || S->l > ORC_MAXL) return -1;
        S->a = in->exps + off; S->c = X->cstore + off;
        renormalise(S->l, S->nprim, S->a, in->coefs + off, S->c);
        for (int i = 0; i < S->nprim; ++i) if (S->a[i] < X->amin) X->amin = S->a[i];
        S->ao = ao; ao += ncart(S->l);
        off += S->nprim;
    }
    X->nbfc = ao;

    /* two passes: count, then fill */
    long total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        long n = 0;
        for (int sa = 0; sa < X->nshell; ++sa)
        for (int sb = 0; sb < X->nshell; ++sb) {
            const shell_t *A = &X->sh[sa], *B = &X->sh[sb];
            const double *xa = in->xyz + 3 * A->atom, *xb = in->xyz + 3 * B->atom;
            double d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]}, dmin[3];
            min_image(&X->lat, d, dmin);
            for (int ia = 0; ia < A->nprim; ++ia)
            for (int ib = 0; ib < B->nprim; ++ib) {
                double a = A->a[ia], b = B->a[ib], p = a + b, mu = a * b / p;
                double Ca = bound_const(a, A->l, A->c[ia]), Cb = bound_const(b, B->l, B->c[ib]);
                /* pair-R bound prefactor.  Reading: the separable bound of
                 * 2 pi^{5/2}/(pq sqrt(p+q)) using p+q >= sqrt((p+2amin)(q+2amin)),
                 * i.e. sqrt2 pi^{5/4} |Ca Cb| / (p (p+2 amin)^{1/4}) (the printed
                 * p sqrt(p+2amin) is dimensionally inconsistent). */
                double X0 = sqrt(2.0) * pow(ORC_PI, 1.25) * Ca * Cb / (p * pow(p + 2.0 * X->amin, 0.25));
                /* Cauchy-Schwarz local-pair value 2^{1/4} pi^{5/4} |Ca Cb| / p^{5/4} */
                double Y0 = pow(2.0, 0.25) * pow(ORC_PI, 1.25) * Ca * Cb / pow(p, 1.25);
                double l1 = log(X0 / in->d_pair_R), l2 = log(Y0 / in->d_pair_cs);
                double lm = l1 < l2 ? l1 : l2;
                if (!(lm > 0)) continue;
                double r = sqrt(lm / mu) * (1.0 + 1e-9) + 1e-9;   /* search superset */
                if (in->r_cut > 0 && r > in->r_cut * (1.0 + 1e-9) + 1e-9) r = in->r_cut * (1.0 + 1e-9) + 1e-9;
                pair_user u = {X, sa, sb, ia, ib, {dmin[0], dmin[1], dmin[2]}, X0, Y0, mu,
                               in->r_cut > 0 ? in->r_cut * in->r_cut : 0.0,
                               pass ? X->pair + n : NULL, 0, pass ? total - n : 0};
                enum_sphere(X->lat.M, X->lat.Minv, dmin, r, pair_cb, &u);
                n += u.n;
            }
        }
        if (pass == 0) {
            total = n;
            X->npair = n;
            X->pair = (pair_t *)calloc(n > 0 ? n : 1, sizeof(pair_t));
        }
    }
    /* Hermite tables per pair */
    long esz = 0;
    for (long i = 0; i < X->npair; ++i) {
        pair_t *P = &X->pair[i];
        esz += 3 * (P->la + 1) * (P->lb + 1) * (P->la + P->lb + 1);
    }
    X->Epool = (double *)malloc(sizeof(double) * (esz > 0 ? esz : 1));
    long eo = 0;
    for (long i = 0; i < X->npair; ++i) {
        pair_t *P = &X->pair[i];
        double Pc[3];
        P->E = X->Epool + eo;
        pair_E(P->la, P->lb, P->a, P->b, P->A, P->B, P->E, Pc);
        comp_norms(P->la, P->a, P->Na);
        comp_norms(P->lb, P->b, P->Nb);
        P->S0 = P->ca * P->cb * pow(ORC_PI / P->p, 1.5);
        for (int x = 0; x < 3; ++x) P->P[x] = Pc[x];
        eo += 3 * (P->la + 1) * (P->lb + 1) * (P->la + P->lb + 1);
    }
    /* short-range Cauchy-Schwarz factor of every pair, for the quartet screen:
     * sqrt of the largest normalised diagonal element (ab|ab)_SR */
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < X->npair; ++i) {
        pair_t *P = &X->pair[i];
        int sz = (P->la + 1) * (P->lb + 1) * (P->la + P->lb + 1);
        const double *e[3] = {P->E, P->E + sz, P->E + 2 * sz};
        P->Q = fabs(P->ca * P->cb) * sqrt(sr_self_max(P->la, P->lb, P->p, e, P->Na, P->Nb, in->omega));
    }
    return 0;
}

/* Cartesian normalisations of every component of a shell for exponent a. */
static void comp_norms(int l, double a, double *N)
{
    for (int k = 0; k < ncart(l); ++k) { int c[3]; cart_comp(l, k, c); N[k] = prim_norm(a, c); }
}

/* ---------------------------------------------------------------------- */
/* short-range sum of one ordered (bra, ket) primitive pair over R1        */
/* ---------------------------------------------------------------------- */
typedef struct { const ctx_t *X; const pair_t *b, *k; double *acc; int nab, ncd;
                 double *blk; long nimg; double rcap2; double center[3]; double rad2; } r1_user;

static void r1_cb(const double R[3], const int n[3], void *u_)
{
    (void)n;
    r1_user *u = (r1_user *)u_;
    double L[3];
    for (int x = 0; x < 3; ++x) L[x] = u->center[x] - R[x];
    double L2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    if (!(L2 < u->rad2)) return;
    if (u->rcap2 > 0 && L2 > u->rcap2) return;
    const pair_t *b = u->b, *k = u->k;
    int sab = (b->la + 1) * (b->lb + 1) * (b->la + b->lb + 1);
    int scd = (k->la + 1) * (k->lb + 1) * (k->la + k->lb + 1);
    const double *eab[3] = {b->E, b->E + sab, b->E + 2 * sab};
    const double *ecd[3] = {k->E, k->E + scd, k->E + 2 * scd};
    quartet_block(b->la, b->lb, k->la, k->lb, b->p, eab, k->p, ecd, L, KER_SR,
                  u->X->in->omega, u->blk);
    int nn = u->nab * u->ncd;
    for (int i = 0; i < nn; ++i) u->acc[i] += u->blk[i];
    u->nimg++;
}

/* Sum over R1 of the SR block of (bra | ket shifted by R1) with the
 * real-space sphere of Sec. 2.4 (eq. pbc_eri_real_cutoff_implementation):
 *   |R1 - (P - Q)|^2 < (1/p + 1/q + 1/w^2) ln(C2e (1 - c) / delta_EwaldR),
 * C2e = Ca Cb Cc Cd 2 pi^{5/2}/(pq sqrt(p+q)) Kab Kcd.
 * acc: monomial block (no normalisation).  Returns the number of images. */
static long sr_sum(const ctx_t *X, const pair_t *b, const pair_t *k, double *acc, double *blk)
{
    const orc_sys *in = X->in;
    int nab = ncart(b->la) * ncart(b->lb), ncd = ncart(k->la) * ncart(k->lb);
    memset(acc, 0, sizeof(double) * nab * ncd);
    double p = b->p, q = k->p, w2 = in->omega * in->omega;
    double rho = p * q / (p + q);
    double c = in->omega / sqrt(rho + w2);
    double C2e = b->Ca * b->Cb * k->Ca * k->Cb * 2.0 * pow(ORC_PI, 2.5) / (p * q * sqrt(p + q))
                 * b->Kab * k->Kab;
    double arg = C2e * (1.0 - c) / in->d_ewald_R;
    if (!(arg > 1.0)) return 0;
    double rad2 = (1.0 / p + 1.0 / q + 1.0 / w2) * log(arg);
    r1_user u = {X, b, k, acc, nab, ncd, blk, 0, in->r_cut > 0 ? in->r_cut * in->r_cut : 0.0,
                 {b->P[0] - k->P[0], b->P[1] - k->P[1], b->P[2] - k->P[2]}, rad2};
    /* exact test |center - R1|^2 < rad2 inside a superset search */
    double r = sqrt(rad2) * (1.0 + 1e-9) + 1e-9;
    enum_sphere(X->lat.M, X->lat.Minv, u.center, r, r1_cb, &u);
    return u.nimg;
}

/* Density weight of a shell quartet.  Reading of the density-weighted
 * Schwarz screen: the largest |D| block among the six shell pairs the
 * quartet couples, so that one decision serves J and K and every
 * permutation of the quartet. */
static double dens_weight(const double *Dmax, int ns, int A, int B, int C, int D)
{
    double w = Dmax[A * ns + B];
    double v;
    v = Dmax[C * ns + D]; if (v > w) w = v;
    v = Dmax[A * ns + C]; if (v > w) w = v;
    v = Dmax[A * ns + D]; if (v > w) w = v;
    v = Dmax[B * ns + C]; if (v > w) w = v;
    v = Dmax[B * ns + D]; if (v > w) w = v;
    return w;
}

/* ---------------------------------------------------------------------- */
/* public: short-range J and K                                              */
/* ---------------------------------------------------------------------- */
/* Dc: Cartesian density (nbfc x nbfc).  bra_mask: NULL or per-shell flags;
 * only bra pairs whose first shell is flagged are visited, which makes the
 * J and K rows of the flagged shells exact and leaves other rows partial.
 * J, K: nbfc x nbfc outputs (overwritten).  counts[0] = ordered primitive
 * quartets kept by the screen, counts[1] = (quartet, R1) terms evaluated,
 * counts[2] = local primitive pairs.  Returns 0 or a negative error. */
int orc_sr_jk(const orc_sys *in, const double *Dc, const unsigned char *bra_mask,
              double *J, double *K, double *counts)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    int nb = X.nbfc, ns = X.nshell;
    double *Dmax = (double *)calloc((size_t)ns * ns, sizeof(double));
    for (int A = 0; A < ns; ++A)
        for (int B = 0; B < ns; ++B) {
            double m = 0;
            for (int i = 0; i < ncart(X.sh[A].l); ++i)
                for (int j = 0; j < ncart(X.sh[B].l); ++j) {
                    double v = fabs(Dc[(X.sh[A].ao + i) * nb + X.sh[B].ao + j]);
                    if (v > m) m = v;
                }
            Dmax[A * ns + B] = m;
        }
    memset(J, 0, sizeof(double) * nb * nb);
    memset(K, 0, sizeof(double) * nb * nb);
    double nq = 0, nimg = 0;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *Jt = (double *)calloc((size_t)nthr * nb * nb, sizeof(double));
    double *Kt = (double *)calloc((size_t)nthr * nb * nb, sizeof(double));
    double *qt = (double *)calloc(2 * (size_t)nthr, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *Jl = Jt + (size_t)tid * nb * nb, *Kl = Kt + (size_t)tid * nb * nb;
        double acc[ORC_MAXNC * ORC_MAXNC * ORC_MAXNC * ORC_MAXNC];
        double blk[ORC_MAXNC * ORC_MAXNC * ORC_MAXNC * ORC_MAXNC];
        double Na[ORC_MAXNC], Nb[ORC_MAXNC], Nc[ORC_MAXNC], Nd[ORC_MAXNC];
#pragma omp for schedule(dynamic, 16)
        for (long ib = 0; ib < X.npair; ++ib) {
            const pair_t *b = &X.pair[ib];
            if (bra_mask && !bra_mask[b->sa]) continue;
            comp_norms(b->la, b->a, Na); comp_norms(b->lb, b->b, Nb);
            int na = ncart(b->la), nbb = ncart(b->lb);
            int aoA = X.sh[b->sa].ao, aoB = X.sh[b->sb].ao;
            for (long ik = 0; ik < X.npair; ++ik) {
                const pair_t *k = &X.pair[ik];
                double wD = dens_weight(Dmax, ns, b->sa, b->sb, k->sa, k->sb);
                if (!(b->Q * k->Q * wD > in->d_schwarz)) continue;
                qt[2 * tid] += 1;
                long ni = sr_sum(&X, b, k, acc, blk);
                qt[2 * tid + 1] += ni;
                if (ni == 0) continue;
                comp_norms(k->la, k->a, Nc); comp_norms(k->lb, k->b, Nd);
                int nc = ncart(k->la), nd = ncart(k->lb);
                int aoC = X.sh[k->sa].ao, aoD = X.sh[k->sb].ao;
                double cc = b->ca * b->cb * k->ca * k->cb;
                for (int i = 0; i < na; ++i)
                for (int j = 0; j < nbb; ++j)
                for (int m = 0; m < nc; ++m)
                for (int n = 0; n < nd; ++n) {
                    double val = cc * Na[i] * Nb[j] * Nc[m] * Nd[n] * acc[((i * nbb + j) * nc + m) * nd + n];
                    /* Gamma point: J_{mu nu} += (mu nu|la si) D_{la si};
                     * K_{mu nu} += (mu la|nu si) D_{la si}  (Sec. 2.5) */
                    Jl[(aoA + i) * nb + aoB + j] += val * Dc[(aoC + m) * nb + aoD + n];
                    Kl[(aoA + i) * nb + aoC + m] += val * Dc[(aoB + j) * nb + aoD + n];
                }
            }
        }
    }
    for (int t = 0; t < nthr; ++t) {
        for (long i = 0; i < (long)nb * nb; ++i) { J[i] += Jt[(size_t)t * nb * nb + i]; K[i] += Kt[(size_t)t * nb * nb + i]; }
        nq += qt[2 * t]; nimg += qt[2 * t + 1];
    }
    if (counts) { counts[0] = nq; counts[1] = nimg; counts[2] = (double)X.npair; }
    free(Jt); free(Kt); free(qt); free(Dmax);
    ctx_free(&X);
    return 0;
}

/* Short-range part of the Gamma ERI tensor (nbfc^4, Cartesian), screened by
 * the Schwarz product alone (no density), for tiny systems. */
int orc_sr_tensor(const orc_sys *in, double *T)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    long nb = X.nbfc;
    memset(T, 0, sizeof(double) * nb * nb * nb * nb);
#pragma omp parallel
    {
        double acc[ORC_MAXNC * ORC_MAXNC * ORC_MAXNC * ORC_MAXNC];
        double blk[ORC_MAXNC * ORC_MAXNC * ORC_MAXNC * ORC_MAXNC];
        double Na[ORC_MAXNC], Nb[ORC_MAXNC], Nc[ORC_MAXNC], Nd[ORC_MAXNC];
        /* each thread owns the rows mu of its bra shells: iterate shells */
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < X.nshell; ++s)
            for (long ib = 0; ib < X.npair; ++ib) {
                const pair_t *b = &X.pair[ib];
                if (b->sa != s) continue;
                comp_norms(b->la, b->a, Na); comp_norms(b->lb, b->b, Nb);
                int na = ncart(b->la), nbb = ncart(b->lb);
                long aoA = X.sh[b->sa].ao, aoB = X.sh[b->sb].ao;
                for (long ik = 0; ik < X.npair; ++ik) {
                    const pair_t *k = &X.pair[ik];
                    if (!(b->Q * k->Q > in->d_schwarz)) continue;
                    if (sr_sum(&X, b, k, acc, blk) == 0) continue;
                    comp_norms(k->la, k->a, Nc); comp_norms(k->lb, k->b, Nd);
                    int nc = ncart(k->la), nd = ncart(k->lb);
                    long aoC = X.sh[k->sa].ao, aoD = X.sh[k->sb].ao;
                    double cc = b->ca * b->cb * k->ca * k->cb;
                    for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nbb; ++j)
                    for (int m = 0; m < nc; ++m)
                    for (int n = 0; n < nd; ++n)
                        T[(((aoA + i) * nb + aoB + j) * nb + aoC + m) * nb + aoD + n] +=
                            cc * Na[i] * Nb[j] * Nc[m] * Nd[n] * acc[((i * nbb + j) * nc + m) * nd + n];
                }
            }
    }
    ctx_free(&X);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* reciprocal space                                                         */
/* ---------------------------------------------------------------------- */
typedef struct { double *G, *w; int n, cap; double V, omega, dK, gcap; } g_user;

static double g_weight(double G2, double V, double omega)
{
    return 4.0 * ORC_PI / V * exp(-G2 / (4.0 * omega * omega)) / G2;
}

static void g_cb(const double R[3], const int n[3], void *u_)
{
    (void)n;
    g_user *u = (g_user *)u_;
    double G2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    if (!(G2 > 0)) return;
    double w = g_weight(G2, u->V, u->omega);
    if (!(w > u->dK)) return;
    if (u->gcap > 0 && G2 > u->gcap * u->gcap) return;
    if (u->n < u->cap) {
        for (int x = 0; x < 3; ++x) u->G[3 * u->n + x] = R[x];
        u->w[u->n] = w;
    }
    u->n++;
}

/* Reciprocal vectors G != 0 with (4 pi/V) e^{-G^2/4w^2}/G^2 > delta_EwaldK
 * (one global sphere; the weight is the form of Sec. 2.8, eq.
 * nuclear_repulsion_energy_reciprocal_cutoff) and |G| <= g_cut when set.
 * Writes up to cap vectors and returns the total count. */
int orc_glist(const orc_sys *in, int cap, double *G, double *w)
{
    lattice_t L;
    lattice_init(in->cell, &L);
    /* radius: bisection on the decreasing weight */
    double lo = 1e-6, hi = 1.0;
    while (g_weight(hi * hi, L.V, in->omega) > in->d_ewald_K) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (g_weight(mid * mid, L.V, in->omega) > in->d_ewald_K) lo = mid; else hi = mid;
    }
    double r = hi * (1.0 + 1e-9);
    if (in->g_cut > 0 && in->g_cut < r) r = in->g_cut * (1.0 + 1e-9);
    /* reciprocal rows B; inverse of B is M^T / (2 pi) */
    double Binv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Binv[i * 3 + j] = L.M[j * 3 + i] / (2.0 * ORC_PI);
    g_user u = {G, w, 0, cap, L.V, in->omega, in->d_ewald_K, in->g_cut};
    double c[3] = {0, 0, 0};
    enum_sphere(L.B, Binv, c, r, g_cb, &u);
    return u.n;
}

/* Cartesian AO count of the system. */
int orc_nbf_cart(const orc_sys *in)
{
    int n = 0;
    for (int s = 0; s < in->nshell; ++s) n += ncart(in->sh_l[s]);
    return n;
}

/* Pair structure factors rho_{mu nu}(G) = sum over local pairs of
 *   int e^{-iG.r} mu(r) nu(r - R2) dr
 *   = c_a c_b N N (pi/p)^{3/2} e^{-G^2/4p} e^{-iG.P} sum_t E_t (-iG)^t
 * (the reciprocal factor of Sec. 2.4, eq. pbc_eri_general_final, split into
 * bra and ket).  F_re/F_im: nG x nbfc x nbfc. */
static void sfac_ctx(const ctx_t *X, int nG, const double *G, double *Fre, double *Fim)
{
    long nb = X->nbfc;
    memset(Fre, 0, sizeof(double) * nG * nb * nb);
    memset(Fim, 0, sizeof(double) * nG * nb * nb);
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < nG; ++g) {
        const double *Gv = G + 3 * g;
        double G2 = Gv[0] * Gv[0] + Gv[1] * Gv[1] + Gv[2] * Gv[2];
        double *fr = Fre + (size_t)g * nb * nb, *fi = Fim + (size_t)g * nb * nb;
        for (long ip = 0; ip < X->npair; ++ip) {
            const pair_t *P = &X->pair[ip];
            const double *Na = P->Na, *Nb = P->Nb;
            double pre = P->S0 * exp(-G2 / (4.0 * P->p));
            double ph = -(Gv[0] * P->P[0] + Gv[1] * P->P[1] + Gv[2] * P->P[2]);
            double complex phase = cexp(I * ph);
            int sz = (P->la + 1) * (P->lb + 1) * (P->la + P->lb + 1), nt = P->la + P->lb + 1;
            long aoA = X->sh[P->sa].ao, aoB = X->sh[P->sb].ao;
            for (int i = 0; i < ncart(P->la); ++i) {
                int ca[3]; cart_comp(P->la, i, ca);
                for (int j = 0; j < ncart(P->lb); ++j) {
                    int cb[3]; cart_comp(P->lb, j, cb);
                    double complex h[3];
                    for (int x = 0; x < 3; ++x) {
                        const double *e = P->E + x * sz + (ca[x] * (P->lb + 1) + cb[x]) * nt;
                        double complex sm = 0, f = 1;
                        for (int t = 0; t <= ca[x] + cb[x]; ++t) {
                            sm += e[t] * f;
                            f *= -I * Gv[x];
                        }
                        h[x] = sm;
                    }
                    double complex v = pre * Na[i] * Nb[j] * h[0] * h[1] * h[2] * phase;
                    fr[(aoA + i) * nb + aoB + j] += creal(v);
                    fi[(aoA + i) * nb + aoB + j] += cimag(v);
                }
            }
        }
    }
}

/* Pair structure factors rho_{mu nu}(G) = sum over local pairs of
 *   int e^{-iG.r} mu(r) nu(r - R2) dr
 *   = c_a c_b N N (pi/p)^{3/2} e^{-G^2/4p} e^{-iG.P} sum_t E_t (-iG)^t
 * (the reciprocal factor of Sec. 2.4, eq. pbc_eri_general_final, split into
 * bra and ket).  F_re/F_im: nG x nbfc x nbfc. */
int orc_sfac(const orc_sys *in, int nG, const double *G, double *Fre, double *Fim)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    sfac_ctx(&X, nG, G, Fre, Fim);
    ctx_free(&X);
    return 0;
}

/* The same with a context kept between calls (pair list built once). */
void *orc_ctx_new(const orc_sys *in)
{
    ctx_t *X = (ctx_t *)malloc(sizeof(ctx_t));
    if (!X) return NULL;
    if (ctx_build(in, X)) { ctx_free(X); free(X); return NULL; }
    return X;
}
void orc_ctx_free(void *X)
{
    if (!X) return;
    ctx_free((ctx_t *)X);
    free(X);
}
void orc_ctx_sfac(void *X, int nG, const double *G, double *Fre, double *Fim)
{
    sfac_ctx((const ctx_t *)X, nG, G, Fre, Fim);
}

/* Gamma overlap over the local pair list (Sec. 2.2, eq. pbc_overlap_formula). */
int orc_overlap(const orc_sys *in, double *S)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    long nb = X.nbfc;
    memset(S, 0, sizeof(double) * nb * nb);
    for (long ip = 0; ip < X.npair; ++ip) {
        const pair_t *P = &X.pair[ip];
        double Na[ORC_MAXNC], Nb[ORC_MAXNC];
        comp_norms(P->la, P->a, Na); comp_norms(P->lb, P->b, Nb);
        int sz = (P->la + 1) * (P->lb + 1) * (P->la + P->lb + 1), nt = P->la + P->lb + 1;
        double pre = P->ca * P->cb * pow(ORC_PI / P->p, 1.5);
        long aoA = X.sh[P->sa].ao, aoB = X.sh[P->sb].ao;
        for (int i = 0; i < ncart(P->la); ++i) {
            int ca[3]; cart_comp(P->la, i, ca);
            for (int j = 0; j < ncart(P->lb); ++j) {
                int cb[3]; cart_comp(P->lb, j, cb);
                double v = pre * Na[i] * Nb[j];
                for (int x = 0; x < 3; ++x) v *= P->E[x * sz + (ca[x] * (P->lb + 1) + cb[x]) * nt];
                S[(aoA + i) * nb + aoB + j] += v;
            }
        }
    }
    ctx_free(&X);
    return 0;
}

/* Local primitive pair list (for enumeration tests).  Writes up to cap
 * entries: shells, primitive indices and the image lattice index n2 with
 * B(R2) = B + (n2 lattice vector); returns the total count. */
long orc_pair_list(const orc_sys *in, long cap, int *sa, int *sb, int *ia, int *ib, int *n2,
                   double *Q)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    for (long i = 0; i < X.npair && i < cap; ++i) {
        const pair_t *P = &X.pair[i];
        sa[i] = P->sa; sb[i] = P->sb; ia[i] = P->ia; ib[i] = P->ib;
        /* image index relative to the raw positions: B(R2) - B = R2 */
        const double *xb = in->xyz + 3 * X.sh[P->sb].atom;
        double d[3] = {P->B[0] - xb[0], P->B[1] - xb[1], P->B[2] - xb[2]}, f[3];
        frac(X.lat.Minv, d, f);
        for (int x = 0; x < 3; ++x) n2[3 * i + x] = (int)lround(f[x]);
        Q[i] = P->Q;
    }
    long n = X.npair;
    ctx_free(&X);
    return n;
}

/* Minimum image of a vector (test entry point). */
void orc_min_image(const double *cell, const double *x, double *out)
{
    lattice_t L;
    lattice_init(cell, &L);
    min_image(&L, x, out);
}

/* Lattice vectors inside a sphere (test entry point); writes up to cap
 * integer triples, returns the count. */
typedef struct { int *n; long k, cap; } ls_user;
static void ls_cb(const double R[3], const int n[3], void *u_)
{
    (void)R;
    ls_user *u = (ls_user *)u_;
    if (u->k < u->cap) for (int x = 0; x < 3; ++x) u->n[3 * u->k + x] = n[x];
    u->k++;
}
long orc_lattice_sphere(const double *cell, const double *c, double r, long cap, int *n)
{
    lattice_t L;
    lattice_init(cell, &L);
    ls_user u = {n, 0, cap};
    enum_sphere(L.M, L.Minv, c, r, ls_cb, &u);
    return u.k;
}

/* ---------------------------------------------------------------------- */
/* point-charge Ewald energy (Sec. 2.8, eq. nuclear_repulsion_energy)       */
/* ---------------------------------------------------------------------- */
typedef struct { double sum, omega, dx[3]; int skip0; double rcap2; } er_user;
static void er_cb(const double R[3], const int n[3], void *u_)
{
    er_user *u = (er_user *)u_;
    if (u->skip0 && n[0] == 0 && n[1] == 0 && n[2] == 0) return;
    double d[3] = {u->dx[0] + R[0], u->dx[1] + R[1], u->dx[2] + R[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    u->sum += erfc(u->omega * r) / r;
}
typedef struct { double sum, omega, V, dx[3], dK; } ek_user;
static void ek_cb(const double K[3], const int n[3], void *u_)
{
    (void)n;
    ek_user *u = (ek_user *)u_;
    double K2 = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
    if (!(K2 > 0)) return;
    double w = g_weight(K2, u->V, u->omega);
    u->sum += w * cos(K[0] * u->dx[0] + K[1] * u->dx[1] + K[2] * u->dx[2]);
}

/* Real-space radius from erfc(x) < (2/sqrt(pi)) e^{-x^2}/x, i.e.
 * (2/sqrt(pi)) e^{-w^2 r^2}/(w r^2) = delta (reading: the printed cutoff
 * equation omits the 1/w); reciprocal radius from (4 pi/V) e^{-k^2/4w^2}/k^2
 * = delta. */
double orc_ewald_energy(int natom, const double *xyz, const double *q, const double *cell,
                        double omega, double dR, double dK)
{
    lattice_t L;
    lattice_init(cell, &L);
    double lo = 1e-3, hi = 1.0;
    while (2.0 / sqrt(ORC_PI) * exp(-omega * omega * hi * hi) / (omega * hi * hi) > dR) hi *= 2;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (2.0 / sqrt(ORC_PI) * exp(-omega * omega * m * m) / (omega * m * m) > dR) lo = m; else hi = m;
    }
    double rR = hi;
    lo = 1e-6; hi = 1.0;
    while (g_weight(hi * hi, L.V, omega) > dK) hi *= 2;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (g_weight(m * m, L.V, omega) > dK) lo = m; else hi = m;
    }
    double rK = hi;
    double Binv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Binv[i * 3 + j] = L.M[j * 3 + i] / (2.0 * ORC_PI);
    double self_bg = ORC_PI / (L.V * omega * omega);   /* (4 pi/V)(1/4w^2) */
    double E = 0;
    for (int A = 0; A < natom; ++A)
        for (int B = A; B < natom; ++B) {
            double dx[3];
            for (int x = 0; x < 3; ++x) dx[x] = xyz[3 * A + x] - xyz[3 * B + x];
            double zero[3] = {0, 0, 0}, c[3] = {-dx[0], -dx[1], -dx[2]};
            er_user ur = {0, omega, {dx[0], dx[1], dx[2]}, A == B, 0};
            enum_sphere(L.M, L.Minv, c, rR, er_cb, &ur);
            ek_user uk = {0, omega, L.V, {dx[0], dx[1], dx[2]}, dK};
            enum_sphere(L.B, Binv, zero, rK, ek_cb, &uk);
            if (A == B)
                E += 0.5 * q[A] * q[A] * (uk.sum - self_bg + ur.sum - 2.0 * omega / sqrt(ORC_PI));
            else
                E += q[A] * q[B] * (uk.sum - self_bg + ur.sum);
        }
    return E;
}

/* ---------------------------------------------------------------------- */
/* one-electron matrices at the Gamma point                                 */
/* ---------------------------------------------------------------------- */
typedef struct { int lab; double p, omega, rad2, rcap2, P[3], C[3]; const double *e[3]; int nt;
                 int la, lb; double *acc; long nimg; } v_user;

/* One lattice image R_C of the short-range point-charge sum: adds
 * sum_t E^{ab}_t R^SR_t(p, L), L = P - C + R_C, to every component of the
 * pair's block. */
static void v_cb(const double R[3], const int n[3], void *u_)
{
    (void)n;
    v_user *u = (v_user *)u_;
    double L[3];
    for (int x = 0; x < 3; ++x) L[x] = u->P[x] - u->C[x] + R[x];
    double L2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    if (!(L2 < u->rad2)) return;
    if (u->rcap2 > 0 && L2 > u->rcap2) return;
    int n1 = u->lab + 1;
    double R000[ORC_MAXLQ + 1];
    /* short-range point-charge kernel: the Boys split of Sec. 2.3 (eq.
     * boys_function_split) with the pair exponent p in place of rho */
    kernel_R000(KER_SR, u->lab, u->p, u->omega, L2, R000);
    double Rt[(ORC_MAXLQ + 1) * (ORC_MAXLQ + 1) * (ORC_MAXLQ + 1)];
    hermite_R(u->lab, R000, L, Rt);
    for (int i = 0; i < ncart(u->la); ++i) {
        int ca[3]; cart_comp(u->la, i, ca);
        for (int j = 0; j < ncart(u->lb); ++j) {
            int cb[3]; cart_comp(u->lb, j, cb);
            const double *ex = u->e[0] + (ca[0] * (u->lb + 1) + cb[0]) * u->nt;
            const double *ey = u->e[1] + (ca[1] * (u->lb + 1) + cb[1]) * u->nt;
            const double *ez = u->e[2] + (ca[2] * (u->lb + 1) + cb[2]) * u->nt;
            double s = 0.0;
            for (int t = 0; t <= ca[0] + cb[0]; ++t)
            for (int v = 0; v <= ca[1] + cb[1]; ++v)
            for (int w = 0; w <= ca[2] + cb[2]; ++w)
                s += ex[t] * ey[v] * ez[w] * Rt[(t * n1 + v) * n1 + w];
            u->acc[i * ncart(u->lb) + j] += s;
        }
    }
    u->nimg++;
}

/* Gamma-point overlap S, kinetic T and the real-space part of the
 * point-charge potential matrix Vsr over the local primitive pairs of the
 * ERI pair list (ordered pairs, contracted and normalised components):
 *   S   += c_a c_b N_i N_j (pi/p)^{3/2} E^{ix jx}_0 E^{iy jy}_0 E^{iz jz}_0
 *          (Sec. 2.2, eq. pbc_overlap_formula);
 *   T   += c_a c_b N_i N_j (pi/p)^{3/2} t_local, t_local of the SI
 *          (eq. kinetic_formula), whose E^{i, j+-2}_0 come from the same
 *          E recurrences with the second index raised by two;
 *   Vsr += q_C c_a c_b N_i N_j (2 pi/p) sum_{R_C} sum_t E^{ab}_t
 *          [R^0_t(p, L) - w/sqrt(p + w^2) R^0_t(p w^2/(p + w^2), L)],
 *          L = P - C + R_C, the real-space term of Sec. 2.3 (eq.
 *          pbc_v1e_general_final), with R_C inside the sphere of eq.
 *          pbc_v1e_real_cutoff_implementation (C1e = C_a C_b (2 pi/p) K_ab)
 *          and, when set, |L| <= r_cut.
 * q: natom point charges (the potential of charge q_C is q_C/|r - C|); q
 * NULL skips Vsr.  Outputs nbfc x nbfc, overwritten.  Returns 0 or -1. */
int orc_one_electron(const orc_sys *in, const double *q, double *S, double *T, double *Vsr)
{
    ctx_t X;
    if (ctx_build(in, &X)) { ctx_free(&X); return -1; }
    long nb = X.nbfc;
    memset(S, 0, sizeof(double) * nb * nb);
    memset(T, 0, sizeof(double) * nb * nb);
    memset(Vsr, 0, sizeof(double) * nb * nb);
    const double w = in->omega, w2 = w * w;
#pragma omp parallel
    {
        double *Sl = (double *)calloc((size_t)nb * nb, sizeof(double));
        double *Tl = (double *)calloc((size_t)nb * nb, sizeof(double));
        double *Vl = (double *)calloc((size_t)nb * nb, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (long ip = 0; ip < X.npair; ++ip) {
            const pair_t *P = &X.pair[ip];
            const int la = P->la, lb = P->lb, na = ncart(la), nbb = ncart(lb);
            double Na[ORC_MAXNC], Nb[ORC_MAXNC];
            comp_norms(la, P->a, Na); comp_norms(lb, P->b, Nb);
            const double cc = P->ca * P->cb, pp = P->p;
            const double ov = pow(ORC_PI / pp, 1.5);
            /* E tables with the second index up to lb + 2 (kinetic) */
            int ntk = la + lb + 3;
            double Ek[3][3 * 5 * 7];
            for (int x = 0; x < 3; ++x) {
                double dab = P->A[x] - P->B[x];
                hermite_E(la, lb + 2, pp, P->P[x] - P->A[x], P->P[x] - P->B[x],
                          exp(-P->a * P->b / pp * dab * dab), Ek[x]);
            }
#define E0(x, i, j) Ek[x][((i) * (lb + 3) + (j)) * ntk]
            long aoA = X.sh[P->sa].ao, aoB = X.sh[P->sb].ao;
            for (int i = 0; i < na; ++i) {
                int ca[3]; cart_comp(la, i, ca);
                for (int j = 0; j < nbb; ++j) {
                    int cb[3]; cart_comp(lb, j, cb);
                    double e[3], kin = 0.0;
                    for (int x = 0; x < 3; ++x) e[x] = E0(x, ca[x], cb[x]);
                    for (int x = 0; x < 3; ++x) {
                        int jx = cb[x];
                        double d2 = (jx >= 2 ? -0.5 * jx * (jx - 1) * E0(x, ca[x], jx - 2) : 0.0)
                                    + (2 * jx + 1) * P->b * E0(x, ca[x], jx)
                                    - 2.0 * P->b * P->b * E0(x, ca[x], jx + 2);
                        kin += d2 * e[(x + 1) % 3] * e[(x + 2) % 3];
                    }
                    double f = cc * Na[i] * Nb[j] * ov;
                    Sl[(aoA + i) * nb + aoB + j] += f * e[0] * e[1] * e[2];
                    Tl[(aoA + i) * nb + aoB + j] += f * kin;
                }
            }
#undef E0
            if (q) {
                int sz = (la + 1) * (lb + 1) * (la + lb + 1);
                const double *ep[3] = {P->E, P->E + sz, P->E + 2 * sz};
                double c = w / sqrt(pp + w2);
                double C1e = P->Ca * P->Cb * 2.0 * ORC_PI / pp * P->Kab;
                double arg = C1e * (1.0 - c) / in->d_ewald_R;
                if (arg > 1.0) {
                    double rad2 = (1.0 / pp + 1.0 / w2) * log(arg);
                    double acc[ORC_MAXNC * ORC_MAXNC];
                    for (int C = 0; C < in->natom; ++C) {
                        if (q[C] == 0.0) continue;
                        memset(acc, 0, sizeof acc);
                        v_user u = {la + lb, pp, w, rad2, in->r_cut > 0 ? in->r_cut * in->r_cut : 0.0,
                                    {P->P[0], P->P[1], P->P[2]},
                                    {in->xyz[3 * C], in->xyz[3 * C + 1], in->xyz[3 * C + 2]},
                                    {ep[0], ep[1], ep[2]}, la + lb + 1, la, lb, acc, 0};
                        /* R_C with |R_C - (C - P)| < r */
                        double cen[3] = {u.C[0] - u.P[0], u.C[1] - u.P[1], u.C[2] - u.P[2]};
                        enum_sphere(X.lat.M, X.lat.Minv, cen, sqrt(rad2) * (1.0 + 1e-9) + 1e-9, v_cb, &u);
                        if (!u.nimg) continue;
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nbb; ++j)
                                Vl[(aoA + i) * nb + aoB + j] +=
                                    q[C] * cc * Na[i] * Nb[j] * 2.0 * ORC_PI / pp * acc[i * nbb + j];
                    }
                }
            }
        }
#pragma omp critical
        {
            for (long k = 0; k < nb * nb; ++k) { S[k] += Sl[k]; T[k] += Tl[k]; Vsr[k] += Vl[k]; }
        }
        free(Sl); free(Tl); free(Vl);
    }
    ctx_free(&X);
    return 0;
}
