// Internal data layout shared by the host setup and the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pbcjk {

constexpr int kMaxL = 2;
constexpr int kNumClass = 6;               // (la, lb) with la >= lb, la <= 2
constexpr double kPi = 3.14159265358979323846;

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int class_of(int la, int lb) { return la * (la + 1) / 2 + lb; }

// Boys-function table: F_m(k h) for k < kBoysNT, m < kBoysM.  Values of
// F_L(T) come from a Taylor expansion about the nearest grid point with
// kBoysTerms terms, lower orders from downward recursion; above kBoysTmax
// the asymptotic F_0 and upward recursion are used.
constexpr double kBoysStep = 0.1;
constexpr int kBoysNT = 401;
constexpr double kBoysTmax = 40.0;
constexpr int kBoysTerms = 9;
constexpr int kBoysM = 4 * kMaxL + kBoysTerms;   // 17 rows: m = 0..16

// One unique local primitive pair (first shell in the home cell, second at
// an image).  128 bytes, read with four 32-byte loads.
struct alignas(32) PairRec {
    double P[3];    // pair centre
    double p;       // a + b
    double PA[3];   // P - A
    double cpre;    // c_a c_b Nb(a) Nb(b) exp(-ab/p |A-B|^2) * symmetry weight f
    double PB[3];   // P - B(image)
    double Q;       // short-range Cauchy-Schwarz factor: sqrt of the largest normalised
                    // component of the pair's (ab|ab) with the erfc kernel
    double Cb;      // |Ca Cb| K without the symmetry weight (real-space sphere bound)
    double pad[3];   // pad[0] = 1/p, pad[1] = b (exponent of the second primitive)
};

// A group: one (first shell, second shell, image) with its primitive pairs.
struct GroupRec {
    int shA, shB;       // shells (first in the home cell)
    int aoA, aoB;       // first scaled-Cartesian AO of each shell
    int pstart, pend;   // range in the pair array
    double Qmax;        // max Q over the group's pairs
    double C[3];        // centre: P of the group's first pair
    double ext;         // max |P - C| over the group's pairs
    double Zmax;        // max Z (separable real-space bound, see setup.cpp)
    double pmin;        // min p over the group's pairs
};

struct Lattice {
    double M[9];       // rows a, b, c
    double Minv[9];    // M^{-1}: fractional f = x Minv
    double span[3];    // sum_i |Minv[i][j]|
    double V;
    double B[9];       // reciprocal rows, a_i . b_j = 2 pi delta_ij
    double Rmin;       // lower bound on the shortest non-zero lattice vector
};

// Lattice data passed by value to kernels.
struct LatArgs {
    double M[9], Minv[9], span[3];
    double Rmin;
};

// Host-side description built once per handle.
struct Setup {
    Lattice lat;
    double omega = 0;
    double amin = 0;
    double d_pair_R = 0, d_pair_cs = 0, d_ewald_R = 0, d_ewald_K = 0, d_schwarz = 0;
    double fp32_below = 0, r_cut = 0, g_cut = 0;
    int nshell = 0, nbf = 0, nbfc = 0, natom = 0;
    std::vector<int> sh_l, sh_pure, sh_atom, sh_aoc, sh_ao, sh_nprim;
    std::vector<double> xyz;
    std::vector<double> charge;    // nuclear charges Z (empty when none were given)
    // Output transform: for each scaled-Cartesian AO i, up to two
    // (output AO, coefficient) entries: J_out = T' J~ T'^T with T' = T diag(rho).
    std::vector<int> tr_ao;        // 2 * nbfc
    std::vector<double> tr_c;      // 2 * nbfc
    std::vector<double> dscale;    // rho_i (component normalisation ratio)
    std::vector<PairRec> pairs;
    std::vector<GroupRec> groups;
    int class_start[kNumClass + 1] = {0};   // group ranges per class
    std::vector<double> G;          // 3 * nG, half space
    std::vector<double> Gs;         // nG: sqrt of the weights (F_G is stored scaled by it)
    std::vector<double> Gw;         // 2 w_G (both signs folded)
    std::vector<double> S;          // scaled-Cartesian Gamma overlap, nbfc^2
    std::vector<double> boys;       // kBoysNT * kBoysM
    std::vector<double> bexp;       // kBoysNT: e^{-k h}
    std::vector<int> sp_start;      // unique shell pairs: ranges into sp_pairs
    std::vector<int> sp_pairs;      // pair indices grouped by shell pair
    std::vector<int> sp_shA, sp_shB;
    int sp_class_start[kNumClass + 1] = {0};   // shell pairs sorted by class
    long n_pairs_ordered = 0;
};

// setup.cpp
int build_setup(const double *cell, int natom, const double *xyz, const double *charge, int nshell, const int *atom,
                const int *l, const int *pure, const int *nprim, const double *exps,
                const double *coefs, double omega, const double thr[8], Setup &S,
                std::string &err);
void boys_table(std::vector<double> &tab);
double boys_host(int m, double T);

}  // namespace pbcjk
