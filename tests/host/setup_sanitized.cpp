// Host setup (lattice, local pairs and groups, G list, overlap, Boys table)
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py: a skewed cell with s, p and spherical and
// Cartesian d shells, then invalid inputs, each through build_setup.
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

using namespace pbcjk;

static int run(const double *cell, int natom, const double *xyz, const std::vector<int> &atom,
               const std::vector<int> &l, const std::vector<int> &pure, const std::vector<int> &nprim,
               const std::vector<double> &exps, const std::vector<double> &coefs, double omega, bool expect_ok)
{
    const double thr[8] = {1e-10, 1e-10, 1e-10, 1e-10, 1e-10, 1e-6, 0.0, 0.0};
    Setup S;
    std::string err;
    const int rc = build_setup(cell, natom, xyz, nullptr, (int)l.size(), atom.data(), l.data(), pure.data(),
                               nprim.data(), exps.data(), coefs.data(), omega, thr, S, err);
    if ((rc == 0) != expect_ok) {
        std::printf("unexpected rc %d (%s)\n", rc, err.c_str());
        return 1;
    }
    if (rc == 0)
        std::printf("ok: nbf %d nbfc %d pairs %zu groups %zu G %zu\n", S.nbf, S.nbfc, S.pairs.size(),
                    S.groups.size(), S.Gw.size());
    else
        std::printf("rejected as expected: %s\n", err.c_str());
    return 0;
}

int main()
{
    const double cell[9] = {7.1, 0.0, 0.0, 1.3, 6.4, 0.0, -0.6, 0.9, 6.9};
    const double xyz[9] = {0.1, 0.2, 0.3, 2.9, 2.1, 1.6, 4.4, 5.0, 3.3};
    // per atom: s (3 prims), p (2 prims), d (1 prim); spherical d on atom 0, Cartesian elsewhere
    std::vector<int> atom, l, pure, nprim;
    std::vector<double> exps, coefs;
    for (int a = 0; a < 3; ++a) {
        const int ls[3] = {0, 1, 2}, np[3] = {3, 2, 1};
        for (int k = 0; k < 3; ++k) {
            atom.push_back(a);
            l.push_back(ls[k]);
            pure.push_back(k == 2 && a == 0 ? 1 : 0);
            nprim.push_back(np[k]);
            for (int p = 0; p < np[k]; ++p) {
                exps.push_back(0.15 * (p + 1) * (k + 1) + 0.05 * a);
                coefs.push_back(0.3 + 0.2 * p);
            }
        }
    }
    int bad = 0;
    bad |= run(cell, 3, xyz, atom, l, pure, nprim, exps, coefs, 0.3, true);
    bad |= run(cell, 3, xyz, atom, l, pure, nprim, exps, coefs, 0.0, true);    // automatic omega
    const double flat[9] = {7.0, 0.0, 0.0, 14.0, 0.0, 0.0, 0.0, 0.0, 7.0};
    bad |= run(flat, 3, xyz, atom, l, pure, nprim, exps, coefs, 0.3, false);   // singular cell
    std::vector<int> l3 = l;
    l3[2] = 3;
    bad |= run(cell, 3, xyz, atom, l3, pure, nprim, exps, coefs, 0.3, false);  // l > 2
    std::vector<double> e0 = exps;
    e0[0] = -1.0;
    bad |= run(cell, 3, xyz, atom, l, pure, nprim, e0, coefs, 0.3, false);     // negative exponent
    return bad;
}
