// Host-side setup of a periodic J/K handle: validation, basis normalisation,
// lattice, unique local primitive pairs grouped by (shell pair, image) and
// sorted by angular-momentum class and Cauchy-Schwarz value, the half-space
// reciprocal vectors, the Gamma overlap and the Boys table.
//
// The paper builds this pair data once per geometry on the CPU (Sec. 3.1);
// so does this file.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <tuple>

#include "internal.h"

namespace pbcjk {

namespace {

double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

// Cartesian component k of angular momentum l (x^l first).
void comp(int l, int k, int c[3])
{
    int n = 0;
    c[0] = c[1] = c[2] = 0;
    for (int lx = l; lx >= 0; --lx)
        for (int ly = l - lx; ly >= 0; --ly) {
            if (n++ == k) { c[0] = lx; c[1] = ly; c[2] = l - lx - ly; return; }
        }
}

// Normalisation of a Cartesian primitive (Sec. 2.1, eq. local_normalization)
// split as Nbase(a, l) * rho(c): Nbase = (2a/pi)^{3/4} (4a)^{l/2} and
// rho(c) = sqrt(2^l prod c! / prod (2c)!), which is 1 for s, p and the
// mixed d components and 1/sqrt3 for xx, yy, zz.
double nbase(double a, int l) { return std::pow(2.0 * a / kPi, 0.75) * std::pow(4.0 * a, 0.5 * l); }
double rho_comp(const int c[3])
{
    int l = c[0] + c[1] + c[2];
    return std::sqrt(std::pow(2.0, l) * fact(c[0]) * fact(c[1]) * fact(c[2]) /
                     (fact(2 * c[0]) * fact(2 * c[1]) * fact(2 * c[2])));
}

void lattice_setup(const double *cell, Lattice &L)
{
    std::memcpy(L.M, cell, 9 * sizeof(double));
    const double *m = cell;
    double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
    double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    double inv[9] = {c00, m[2] * m[7] - m[1] * m[8], m[1] * m[5] - m[2] * m[4],
                     c01, m[0] * m[8] - m[2] * m[6], m[2] * m[3] - m[0] * m[5],
                     c02, m[1] * m[6] - m[0] * m[7], m[0] * m[4] - m[1] * m[3]};
    for (int i = 0; i < 9; ++i) L.Minv[i] = inv[i] / det;
    L.V = std::fabs(det);
    for (int j = 0; j < 3; ++j)
        L.span[j] = std::fabs(L.Minv[j]) + std::fabs(L.Minv[3 + j]) + std::fabs(L.Minv[6 + j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) L.B[3 * i + j] = 2.0 * kPi * L.Minv[3 * j + i];
    // any non-zero lattice vector has some index n_i != 0 and is then at least
    // one interplanar spacing 1/|Minv[:, i]| long
    L.Rmin = 1e300;
    for (int j = 0; j < 3; ++j) {
        double c2 = L.Minv[j] * L.Minv[j] + L.Minv[3 + j] * L.Minv[3 + j] + L.Minv[6 + j] * L.Minv[6 + j];
        L.Rmin = std::min(L.Rmin, 1.0 / std::sqrt(c2));
    }
}

void to_frac(const double *Minv, const double x[3], double f[3])
{
    for (int j = 0; j < 3; ++j) f[j] = x[0] * Minv[j] + x[1] * Minv[3 + j] + x[2] * Minv[6 + j];
}

// Lattice vectors (rows `rows`, fractional map `inv`, span of `inv`) within
// a superset sphere around c; the caller applies the exact test.
template <class F>
void for_lattice_box(const double *rows, const double *inv, const double span[3], const double c[3],
                     double r, F &&fn)
{
    double f[3];
    to_frac(inv, c, f);
    int lo[3], hi[3];
    for (int j = 0; j < 3; ++j) {
        lo[j] = (int)std::floor(f[j] - r * span[j]);
        hi[j] = (int)std::ceil(f[j] + r * span[j]);
    }
    for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
        for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
            for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
                double R[3];
                for (int x = 0; x < 3; ++x) R[x] = n0 * rows[x] + n1 * rows[3 + x] + n2 * rows[6 + x];
                fn(R, n0, n1, n2);
            }
}

// One-axis Hermite coefficients with E^{00}_0 = 1 (Sec. 2.2 recurrences);
// E[(i*(lb+1)+j)*(la+lb+1)+t].
void herm1(int la, int lb, double p, double xa, double xb, double *E)
{
    int nt = la + lb + 1;
    auto at = [&](int i, int j, int t) -> double & { return E[(i * (lb + 1) + j) * nt + t]; };
    std::fill(E, E + (la + 1) * (lb + 1) * nt, 0.0);
    double h = 0.5 / p;
    at(0, 0, 0) = 1.0;
    for (int i = 0; i < la; ++i)
        for (int t = 0; t <= i + 1; ++t)
            at(i + 1, 0, t) = (t >= 1 ? h * at(i, 0, t - 1) : 0.0) + (t <= i ? xa * at(i, 0, t) : 0.0) +
                              (t + 1 <= i ? (t + 1) * at(i, 0, t + 1) : 0.0);
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j < lb; ++j)
            for (int t = 0; t <= i + j + 1; ++t)
                at(i, j + 1, t) = (t >= 1 ? h * at(i, j, t - 1) : 0.0) + (t <= i + j ? xb * at(i, j, t) : 0.0) +
                                  (t + 1 <= i + j ? (t + 1) * at(i, j, t + 1) : 0.0);
}

bool finite(double x) { return std::isfinite(x); }

// Largest component of the short-range self-integral of one primitive pair,
// (ab|ab) with the erfc(w r)/r kernel, for monomial Gaussians with
// E^{00}_0 = 1 (the pair's Gaussian factor and normalisation are applied by
// the caller), times the square of the component normalisation ratios.
// At zero separation the Hermite integrals reduce to
//   R_{tuv}(0) = (t-1)!! (u-1)!! (v-1)!! R^{(t+u+v)/2}_{000}(0)   (t, u, v even),
//   R^m_{000}(0) = ((-2 rho)^m - c (-2 a')^m) / (2m + 1),  rho = p/2,
// (eq. R_recursion at X = Y = Z = 0, and F_m(0) = 1/(2m+1)), and the
// four-index sum factorises per axis into S[k] = sum_{t+s=k} (-1)^s E_t E_s.
// By the Cauchy-Schwarz inequality of Sec. 2.4 (eq. local_cauchy_schwarz_bound,
// which holds for the positive definite erfc kernel) the square root bounds
// every short-range quartet term of the pair.
double sr_self_max(int la, int lb, double a, double b, const double PA[3], const double PB[3], double omega)
{
    const double p = a + b, rho = 0.5 * p, w2 = omega * omega;
    const double ap = rho * w2 / (rho + w2), c = omega / std::sqrt(rho + w2);
    const int lab = la + lb, nt = lab + 1;
    double R0[2 * 2 * kMaxL + 1];
    for (int m = 0; m <= 2 * lab; ++m)
        R0[m] = (std::pow(-2.0 * rho, m) - c * std::pow(-2.0 * ap, m)) / (2 * m + 1);
    const double dfact[9] = {1.0, 1.0, 1.0, 3.0, 3.0, 15.0, 15.0, 105.0, 105.0};   // (k-1)!! for even k
    double E[3][(kMaxL + 1) * (kMaxL + 1) * (2 * kMaxL + 1)];
    for (int x = 0; x < 3; ++x) herm1(la, lb, p, PA[x], PB[x], E[x]);
    double best = 0.0;
    for (int ia = 0; ia < ncart(la); ++ia)
        for (int ib = 0; ib < ncart(lb); ++ib) {
            int cA[3], cB[3];
            comp(la, ia, cA);
            comp(lb, ib, cB);
            double Sx[3][2 * 2 * kMaxL + 1];
            for (int x = 0; x < 3; ++x) {
                const int nx = cA[x] + cB[x];
                const double *e = E[x] + (cA[x] * (lb + 1) + cB[x]) * nt;
                for (int k = 0; k <= 2 * nx; ++k) Sx[x][k] = 0.0;
                for (int t = 0; t <= nx; ++t)
                    for (int u = 0; u <= nx; ++u) Sx[x][t + u] += ((u & 1) ? -1.0 : 1.0) * e[t] * e[u];
            }
            double I = 0.0;
            for (int kx = 0; kx <= 2 * (cA[0] + cB[0]); kx += 2)
                for (int ky = 0; ky <= 2 * (cA[1] + cB[1]); ky += 2)
                    for (int kz = 0; kz <= 2 * (cA[2] + cB[2]); kz += 2)
                        I += Sx[0][kx] * Sx[1][ky] * Sx[2][kz] * dfact[kx] * dfact[ky] * dfact[kz] *
                             R0[(kx + ky + kz) / 2];
            I *= 2.0 * std::pow(kPi, 2.5) / (p * p * std::sqrt(2.0 * p));
            const double r = rho_comp(cA) * rho_comp(cB);
            best = std::max(best, I * r * r);
        }
    return best;
}

}  // namespace

double boys_host(int m, double T)
{
    // series sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) times e^{-T}
    long double term = 1.0L / (2 * m + 1), sum = term;
    for (int k = 1; k < 4000; ++k) {
        term *= 2.0L * T / (2 * m + 2 * k + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
    }
    return (double)(std::exp(-(long double)T) * sum);
}

// e^{-T_k} on the Boys grid (the kernels form e^{-T} from it)
void boys_exp_table(std::vector<double> &etab)
{
    etab.resize(kBoysNT);
    for (int k = 0; k < kBoysNT; ++k) etab[k] = (double)std::exp(-(long double)(k * (long double)kBoysStep));
}

void boys_table(std::vector<double> &tab)
{
    tab.assign((size_t)kBoysNT * kBoysM, 0.0);
    for (int k = 0; k < kBoysNT; ++k) {
        long double T = k * (long double)kBoysStep;
        // highest order by series, lower orders by downward recursion
        int mt = kBoysM - 1;
        long double term = 1.0L / (2 * mt + 1), sum = term;
        for (int i = 1; i < 4000; ++i) {
            term *= 2.0L * T / (2 * mt + 2 * i + 1);
            sum += term;
            if (term < 1e-24L * sum) break;
        }
        long double et = std::exp(-T);
        long double F = et * sum;
        tab[(size_t)k * kBoysM + mt] = (double)F;
        for (int m = mt - 1; m >= 0; --m) {
            F = (2.0L * T * F + et) / (2 * m + 1);
            tab[(size_t)k * kBoysM + m] = (double)F;
        }
    }
}

int build_setup(const double *cell, int natom, const double *xyz, const double *charge, int nshell, const int *atom,
                const int *l, const int *pure, const int *nprim, const double *exps,
                const double *coefs, double omega, const double thr[8], Setup &S, std::string &err)
{
    // ---------------- validation
    for (int i = 0; i < 9; ++i)
        if (!finite(cell[i])) { err = "cell has a non-finite entry"; return -1; }
    lattice_setup(cell, S.lat);
    if (!(S.lat.V > 1e-8) || !finite(S.lat.V)) { err = "cell is singular"; return -1; }
    if (natom <= 0 || !xyz) { err = "no atoms"; return -1; }
    for (int i = 0; i < 3 * natom; ++i)
        if (!finite(xyz[i])) { err = "atom position is not finite"; return -1; }
    if (nshell <= 0 || !atom || !l || !nprim || !exps || !coefs) { err = "empty basis"; return -1; }
    const char *names[5] = {"pair_R", "pair_cs", "ewald_R", "ewald_K", "schwarz"};
    for (int i = 0; i < 5; ++i)
        if (!(thr[i] > 0) || !finite(thr[i])) { err = std::string("threshold ") + names[i] + " must be > 0"; return -1; }
    for (int i = 5; i < 8; ++i)
        if (!(thr[i] >= 0) || !finite(thr[i])) { err = "fp32_below, r_cut, g_cut must be >= 0"; return -1; }
    S.d_pair_R = thr[0]; S.d_pair_cs = thr[1]; S.d_ewald_R = thr[2]; S.d_ewald_K = thr[3];
    S.d_schwarz = thr[4]; S.fp32_below = thr[5]; S.r_cut = thr[6]; S.g_cut = thr[7];
    if (!finite(omega)) { err = "omega is not finite"; return -1; }
    // Sec. 3.4, eq. omega_implementation with w = 10
    S.omega = omega > 0 ? omega : std::pow(10.0 * kPi * kPi * kPi / (S.lat.V * S.lat.V), 1.0 / 6.0);

    S.natom = natom;
    S.xyz.assign(xyz, xyz + 3 * natom);
    S.charge.clear();
    if (charge) {
        for (int i = 0; i < natom; ++i)
            if (!finite(charge[i])) { err = "atom charge is not finite"; return -1; }
        S.charge.assign(charge, charge + natom);
    }
    S.nshell = nshell;
    S.sh_l.resize(nshell); S.sh_pure.resize(nshell); S.sh_atom.resize(nshell);
    S.sh_aoc.resize(nshell); S.sh_ao.resize(nshell); S.sh_nprim.resize(nshell);
    std::vector<int> poff(nshell + 1, 0);
    for (int s = 0; s < nshell; ++s) {
        if (l[s] < 0 || l[s] > kMaxL) { err = "angular momentum must be 0, 1 or 2"; return -1; }
        if (atom[s] < 0 || atom[s] >= natom) { err = "shell atom index out of range"; return -1; }
        if (nprim[s] < 1 || nprim[s] > 64) { err = "primitive count must be in 1..64"; return -1; }
        poff[s + 1] = poff[s] + nprim[s];
    }
    std::vector<double> cnorm(poff[nshell]);
    S.amin = 1e300;
    int aoc = 0, ao = 0;
    for (int s = 0; s < nshell; ++s) {
        S.sh_l[s] = l[s];
        S.sh_pure[s] = (pure && pure[s] && l[s] == 2) ? 1 : 0;
        S.sh_atom[s] = atom[s];
        S.sh_nprim[s] = nprim[s];
        S.sh_aoc[s] = aoc; S.sh_ao[s] = ao;
        aoc += ncart(l[s]);
        ao += S.sh_pure[s] ? 2 * l[s] + 1 : ncart(l[s]);
        const double *a = exps + poff[s], *c = coefs + poff[s];
        for (int i = 0; i < nprim[s]; ++i) {
            if (!(a[i] > 0) || !finite(a[i])) { err = "exponents must be positive and finite"; return -1; }
            if (!finite(c[i])) { err = "contraction coefficient is not finite"; return -1; }
            S.amin = std::min(S.amin, a[i]);
        }
        // unit single-centre self-overlap of the contracted shell
        double ss = 0;
        for (int i = 0; i < nprim[s]; ++i)
            for (int j = 0; j < nprim[s]; ++j)
                ss += c[i] * c[j] * std::pow(2.0 * std::sqrt(a[i] * a[j]) / (a[i] + a[j]), l[s] + 1.5);
        if (!(ss > 0)) { err = "contracted shell has zero norm"; return -1; }
        for (int i = 0; i < nprim[s]; ++i) cnorm[poff[s] + i] = c[i] / std::sqrt(ss);
    }
    S.nbfc = aoc; S.nbf = ao;

    // ---------------- output transform T' = T diag(rho)
    S.tr_ao.assign(2 * S.nbfc, -1);
    S.tr_c.assign(2 * S.nbfc, 0.0);
    S.dscale.assign(S.nbfc, 1.0);
    const double h3 = std::sqrt(3.0) / 2.0;
    for (int s = 0; s < nshell; ++s) {
        for (int k = 0; k < ncart(l[s]); ++k) {
            int c[3]; comp(l[s], k, c);
            int i = S.sh_aoc[s] + k;
            double r = rho_comp(c);
            S.dscale[i] = r;
            if (!S.sh_pure[s]) { S.tr_ao[2 * i] = S.sh_ao[s] + k; S.tr_c[2 * i] = r; continue; }
            int o = S.sh_ao[s];
            // columns of the 5 x 6 solid-harmonic matrix (xx, xy, xz, yy, yz, zz)
            switch (k) {
                case 0: S.tr_ao[2*i] = o + 2; S.tr_c[2*i] = -0.5 * r; S.tr_ao[2*i+1] = o + 4; S.tr_c[2*i+1] = h3 * r; break;
                case 1: S.tr_ao[2*i] = o + 0; S.tr_c[2*i] = r; break;
                case 2: S.tr_ao[2*i] = o + 3; S.tr_c[2*i] = r; break;
                case 3: S.tr_ao[2*i] = o + 2; S.tr_c[2*i] = -0.5 * r; S.tr_ao[2*i+1] = o + 4; S.tr_c[2*i+1] = -h3 * r; break;
                case 4: S.tr_ao[2*i] = o + 1; S.tr_c[2*i] = r; break;
                case 5: S.tr_ao[2*i] = o + 2; S.tr_c[2*i] = r; break;
            }
        }
    }

    // ---------------- unique local primitive pairs
    struct Tmp { int cls, first, second, n0, n1, n2; PairRec rec; double Z; };
    std::vector<Tmp> tmp;
    const Lattice &L = S.lat;
    const double rcap2 = S.r_cut > 0 ? S.r_cut * S.r_cut : 0.0;
    long ordered = 0;
    for (int A = 0; A < nshell; ++A)
        for (int B = A; B < nshell; ++B) {
            // orientation: the higher angular momentum first; ties by index
            int first = A, second = B;
            if (l[B] > l[A]) std::swap(first, second);
            const double *xf = xyz + 3 * atom[first], *xs = xyz + 3 * atom[second];
            double d[3] = {xf[0] - xs[0], xf[1] - xs[1], xf[2] - xs[2]}, f[3], dmin[3];
            to_frac(L.Minv, d, f);
            double nr[3] = {(double)std::lround(f[0]), (double)std::lround(f[1]), (double)std::lround(f[2])};
            for (int x = 0; x < 3; ++x)
                dmin[x] = d[x] - (nr[0] * L.M[x] + nr[1] * L.M[3 + x] + nr[2] * L.M[6 + x]);
            int la = l[first], lb = l[second];
            for (int i = 0; i < nprim[first]; ++i)
                for (int j = 0; j < nprim[second]; ++j) {
                    if (first == second && j < i) continue;   // (i,j,R) ~ (j,i,-R)
                    double a = exps[poff[first] + i], b = exps[poff[second] + j];
                    double ca = cnorm[poff[first] + i], cb = cnorm[poff[second] + j];
                    double p = a + b, mu = a * b / p;
                    double Cab = std::fabs(ca * cb) * nbase(a, la) * nbase(b, lb);
                    double X0 = std::sqrt(2.0) * std::pow(kPi, 1.25) * Cab / (p * std::pow(p + 2.0 * S.amin, 0.25));
                    double Y0 = std::pow(2.0, 0.25) * std::pow(kPi, 1.25) * Cab / std::pow(p, 1.25);
                    double lm = std::min(std::log(X0 / S.d_pair_R), std::log(Y0 / S.d_pair_cs));
                    if (!(lm > 0)) continue;
                    double r = std::sqrt(lm / mu) * (1.0 + 1e-9) + 1e-9;
                    if (S.r_cut > 0) r = std::min(r, S.r_cut * (1.0 + 1e-9) + 1e-9);
                    for_lattice_box(L.M, L.Minv, L.span, dmin, r, [&](const double R[3], int n0, int n1, int n2) {
                        double v[3] = {dmin[0] - R[0], dmin[1] - R[1], dmin[2] - R[2]};
                        double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                        double g = std::exp(-mu * r2);
                        if (!(X0 * g > S.d_pair_R) || !(Y0 * g > S.d_pair_cs)) return;
                        if (rcap2 > 0 && r2 > rcap2) return;
                        double fw = 1.0;
                        if (first == second) {
                            if (i == j) {
                                bool zero = (n0 == 0 && n1 == 0 && n2 == 0);
                                bool pos = n0 > 0 || (n0 == 0 && (n1 > 0 || (n1 == 0 && n2 > 0)));
                                if (zero) fw = 0.5;
                                else if (!pos) return;
                            }
                            ordered += (i == j && fw == 0.5) ? 1 : 2;
                        } else {
                            ordered += 2;
                        }
                        Tmp t;
                        t.cls = class_of(la, lb); t.first = first; t.second = second;
                        t.n0 = n0; t.n1 = n1; t.n2 = n2;
                        double Bi[3];
                        for (int x = 0; x < 3; ++x) {
                            Bi[x] = xf[x] - v[x];
                            t.rec.P[x] = (a * xf[x] + b * Bi[x]) / p;
                            t.rec.PA[x] = t.rec.P[x] - xf[x];
                            t.rec.PB[x] = t.rec.P[x] - Bi[x];
                        }
                        t.rec.p = p;
                        t.rec.cpre = ca * cb * nbase(a, la) * nbase(b, lb) * g * fw;
                        // short-range Cauchy-Schwarz factor of the pair (quartet screen)
                        double pa[3] = {t.rec.PA[0], t.rec.PA[1], t.rec.PA[2]};
                        double pb[3] = {t.rec.PB[0], t.rec.PB[1], t.rec.PB[2]};
                        t.rec.Q = std::fabs(ca * cb) * nbase(a, la) * nbase(b, lb) * g *
                                  std::sqrt(sr_self_max(la, lb, a, b, pa, pb, S.omega));
                        t.rec.Cb = Cab * g;
                        t.rec.pad[0] = 1.0 / p;
                        t.rec.pad[1] = b;
                        t.rec.pad[2] = 0.0;
                        // Separable real-space bound: C2e (1 - c) <= Z_bra Z_ket, using
                        // 2pi^{5/2}/(pq sqrt(p+q)) <= prod sqrt2 pi^{5/4}/(p (p+2amin)^{1/4})
                        // and 1 - w/sqrt(rho+w^2) <= sqrt(prod (1 - w/sqrt(p+w^2))).
                        t.Z = std::sqrt(2.0) * std::pow(kPi, 1.25) * Cab * g / (p * std::pow(p + 2.0 * S.amin, 0.25)) *
                              std::sqrt(1.0 - S.omega / std::sqrt(p + S.omega * S.omega));
                        tmp.push_back(t);
                    });
                }
        }
    S.n_pairs_ordered = ordered;

    // ---------------- groups: (class, first, second, image); class asc, Qmax desc
    std::vector<size_t> idx(tmp.size());
    std::iota(idx.begin(), idx.end(), 0);
    auto gkey = [&](const Tmp &t) { return std::make_tuple(t.cls, t.first, t.second, t.n0, t.n1, t.n2); };
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        auto kx = gkey(tmp[x]), ky = gkey(tmp[y]);
        if (kx != ky) return kx < ky;
        return tmp[x].rec.Q > tmp[y].rec.Q;
    });
    struct G0 { size_t b, e; double qmax, zmax, pmin; int cls; };
    std::vector<G0> gl;
    for (size_t k = 0; k < idx.size();) {
        size_t e = k;
        double qm = 0, zm = 0, pm = 1e300;
        while (e < idx.size() && gkey(tmp[idx[e]]) == gkey(tmp[idx[k]])) {
            qm = std::max(qm, tmp[idx[e]].rec.Q);
            zm = std::max(zm, tmp[idx[e]].Z);
            pm = std::min(pm, tmp[idx[e]].rec.p);
            ++e;
        }
        gl.push_back({k, e, qm, zm, pm, tmp[idx[k]].cls});
        k = e;
    }
    // within a class: more primitive pairs first (similar loop lengths on
    // neighbouring lanes), then descending Cauchy-Schwarz value
    std::vector<size_t> gord(gl.size());
    std::iota(gord.begin(), gord.end(), 0);
    std::stable_sort(gord.begin(), gord.end(), [&](size_t x, size_t y) {
        if (gl[x].cls != gl[y].cls) return gl[x].cls < gl[y].cls;
        size_t nx = gl[x].e - gl[x].b, ny = gl[y].e - gl[y].b;
        if (nx != ny) return nx > ny;
        return gl[x].qmax > gl[y].qmax;
    });
    S.pairs.clear(); S.groups.clear();
    S.pairs.reserve(tmp.size()); S.groups.reserve(gl.size());
    for (int c = 0; c <= kNumClass; ++c) S.class_start[c] = 0;
    for (size_t gi : gord) {
        const G0 &g = gl[gi];
        const Tmp &t0 = tmp[idx[g.b]];
        GroupRec G;
        G.shA = t0.first; G.shB = t0.second;
        G.aoA = S.sh_aoc[t0.first]; G.aoB = S.sh_aoc[t0.second];
        G.pstart = (int)S.pairs.size();
        for (size_t k = g.b; k < g.e; ++k) S.pairs.push_back(tmp[idx[k]].rec);
        G.pend = (int)S.pairs.size();
        G.Qmax = g.qmax; G.Zmax = g.zmax; G.pmin = g.pmin;
        const PairRec &P0 = S.pairs[G.pstart];
        G.C[0] = P0.P[0]; G.C[1] = P0.P[1]; G.C[2] = P0.P[2];
        G.ext = 0.0;
        for (int k = G.pstart; k < G.pend; ++k) {
            const PairRec &Pk = S.pairs[k];
            double dx = Pk.P[0] - G.C[0], dy = Pk.P[1] - G.C[1], dz = Pk.P[2] - G.C[2];
            G.ext = std::max(G.ext, std::sqrt(dx * dx + dy * dy + dz * dz));
        }
        S.groups.push_back(G);
        S.class_start[g.cls + 1]++;
    }
    for (int c = 0; c < kNumClass; ++c) S.class_start[c + 1] += S.class_start[c];

    // unique shell pairs with their pair indices (for the structure factors)
    {
        // (class, first shell, second shell) -> pair indices
        std::vector<std::pair<std::tuple<int, int, int>, int>> sp;
        sp.reserve(S.pairs.size());
        for (const GroupRec &G : S.groups)
            for (int k = G.pstart; k < G.pend; ++k)
                sp.push_back({{class_of(l[G.shA], l[G.shB]), G.shA, G.shB}, k});
        std::sort(sp.begin(), sp.end());
        S.sp_start.clear(); S.sp_pairs.clear(); S.sp_shA.clear(); S.sp_shB.clear();
        for (int c = 0; c <= kNumClass; ++c) S.sp_class_start[c] = 0;
        for (size_t k = 0; k < sp.size(); ++k) {
            if (k == 0 || sp[k].first != sp[k - 1].first) {
                S.sp_start.push_back((int)k);
                S.sp_shA.push_back(std::get<1>(sp[k].first));
                S.sp_shB.push_back(std::get<2>(sp[k].first));
                S.sp_class_start[std::get<0>(sp[k].first) + 1]++;
            }
            S.sp_pairs.push_back(sp[k].second);
        }
        S.sp_start.push_back((int)sp.size());
        for (int c = 0; c < kNumClass; ++c) S.sp_class_start[c + 1] += S.sp_class_start[c];
    }

    // ---------------- reciprocal vectors (half space), weights 2 w_G
    {
        auto wfun = [&](double G2) { return 4.0 * kPi / L.V * std::exp(-G2 / (4.0 * S.omega * S.omega)) / G2; };
        double lo = 1e-6, hi = 1.0;
        while (wfun(hi * hi) > S.d_ewald_K) hi *= 2.0;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (wfun(mid * mid) > S.d_ewald_K) lo = mid; else hi = mid;
        }
        double r = hi * (1.0 + 1e-9);
        if (S.g_cut > 0 && S.g_cut < r) r = S.g_cut * (1.0 + 1e-9);
        double Binv[9], bspan[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Binv[3 * i + j] = L.M[3 * j + i] / (2.0 * kPi);
        for (int j = 0; j < 3; ++j) bspan[j] = std::fabs(Binv[j]) + std::fabs(Binv[3 + j]) + std::fabs(Binv[6 + j]);
        double zero[3] = {0, 0, 0};
        S.G.clear(); S.Gw.clear(); S.Gs.clear();
        for_lattice_box(L.B, Binv, bspan, zero, r, [&](const double Gv[3], int n0, int n1, int n2) {
            bool pos = n0 > 0 || (n0 == 0 && (n1 > 0 || (n1 == 0 && n2 > 0)));
            if (!pos) return;
            double G2 = Gv[0] * Gv[0] + Gv[1] * Gv[1] + Gv[2] * Gv[2];
            double w = wfun(G2);
            if (!(w > S.d_ewald_K)) return;
            if (S.g_cut > 0 && G2 > S.g_cut * S.g_cut) return;
            S.G.push_back(Gv[0]); S.G.push_back(Gv[1]); S.G.push_back(Gv[2]);
            S.Gw.push_back(2.0 * w);
            S.Gs.push_back(std::sqrt(2.0 * w));
        });
    }

    // ---------------- Gamma overlap in the scaled Cartesian basis (Sec. 2.2)
    S.S.assign((size_t)S.nbfc * S.nbfc, 0.0);
    {
        std::vector<double> Sh((size_t)S.nbfc * S.nbfc, 0.0);
        double Ex[45], Ey[45], Ez[45];   // (lmax+1)^2 (2 lmax+1) entries per axis
        for (const GroupRec &G : S.groups) {
            int la = l[G.shA], lb = l[G.shB], nt = la + lb + 1;
            for (int k = G.pstart; k < G.pend; ++k) {
                const PairRec &P = S.pairs[k];
                herm1(la, lb, P.p, P.PA[0], P.PB[0], Ex);
                herm1(la, lb, P.p, P.PA[1], P.PB[1], Ey);
                herm1(la, lb, P.p, P.PA[2], P.PB[2], Ez);
                double pre = P.cpre * std::pow(kPi / P.p, 1.5);
                for (int ia = 0; ia < ncart(la); ++ia) {
                    int ca[3]; comp(la, ia, ca);
                    for (int ib = 0; ib < ncart(lb); ++ib) {
                        int cb[3]; comp(lb, ib, cb);
                        double v = pre * Ex[(ca[0] * (lb + 1) + cb[0]) * nt] * Ey[(ca[1] * (lb + 1) + cb[1]) * nt] *
                                   Ez[(ca[2] * (lb + 1) + cb[2]) * nt];
                        Sh[(size_t)(G.aoA + ia) * S.nbfc + G.aoB + ib] += v;
                    }
                }
            }
        }
        for (int i = 0; i < S.nbfc; ++i)
            for (int j = 0; j < S.nbfc; ++j)
                S.S[(size_t)i * S.nbfc + j] = Sh[(size_t)i * S.nbfc + j] + Sh[(size_t)j * S.nbfc + i];
    }
    boys_table(S.boys);
    boys_exp_table(S.bexp);
    return 0;
}

}  // namespace pbcjk
