/* The CPU oracle's C loops (oracle/oracle.c, included whole) under
 * AddressSanitizer and UndefinedBehaviorSanitizer, driven by
 * tests/test_host_sanitizers.py: G list, pair list, overlap, structure
 * factors, short-range J/K (all bra shells and a subset), one-electron terms
 * and the Ewald energy, on a skewed cell with s, p and spherical d shells. */
#include <stdio.h>
#include <stdlib.h>

#include "oracle.c"

int main(void)
{
    static const double cell[9] = {6.0, 0.0, 0.0, 0.8, 5.7, 0.0, -0.4, 0.6, 6.3};
    static const double xyz[6] = {0.1, 0.2, 0.3, 2.4, 1.9, 1.5};
    static const int sh_atom[4] = {0, 0, 1, 1}, sh_l[4] = {0, 1, 0, 2}, sh_pure[4] = {0, 0, 0, 1};
    static const int sh_nprim[4] = {2, 1, 2, 1};
    static const double exps[6] = {0.4, 1.3, 0.8, 0.5, 1.1, 0.7}, coefs[6] = {0.6, 0.4, 1.0, 0.5, 0.5, 1.0};
    orc_sys s = {{0}, 2, xyz, 4, sh_atom, sh_l, sh_pure, sh_nprim, exps, coefs, 0.4,
                 1e-8, 1e-8, 1e-8, 1e-8, 1e-8, 0.0, 0.0};
    for (int i = 0; i < 9; ++i) s.cell[i] = cell[i];
    const int nb = orc_nbf_cart(&s);
    const size_t n2 = (size_t)nb * nb;
    double dummy3[3] = {0}, dummy1[1] = {0};
    const int nG = orc_glist(&s, 0, dummy3, dummy1);
    double *G = calloc(3 * (size_t)(nG > 0 ? nG : 1), sizeof(double));
    double *w = calloc((size_t)(nG > 0 ? nG : 1), sizeof(double));
    orc_glist(&s, nG, G, w);
    int z[1] = {0};
    double q1[1] = {0};
    const long np = orc_pair_list(&s, 0, z, z, z, z, z, q1);
    const size_t npp = (size_t)(np > 0 ? np : 1);
    int *sa = calloc(npp, sizeof(int)), *sb = calloc(npp, sizeof(int)), *ia = calloc(npp, sizeof(int));
    int *ib = calloc(npp, sizeof(int)), *n3 = calloc(3 * npp, sizeof(int));
    double *Q = calloc(npp, sizeof(double));
    orc_pair_list(&s, np, sa, sb, ia, ib, n3, Q);
    double *S = calloc(n2, sizeof(double)), *T = calloc(n2, sizeof(double)), *V = calloc(n2, sizeof(double));
    double *D = calloc(n2, sizeof(double)), *J = calloc(n2, sizeof(double)), *K = calloc(n2, sizeof(double));
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) D[(size_t)i * nb + j] = 0.1 / (1.0 + abs(i - j));
    double counts[3] = {0};
    int bad = 0;
    bad |= orc_overlap(&s, S) != 0;
    bad |= orc_sr_jk(&s, D, NULL, J, K, counts) != 0;
    unsigned char mask[4] = {0, 1, 0, 1};
    bad |= orc_sr_jk(&s, D, mask, J, K, counts) != 0;
    const int ng = nG < 4 ? nG : 4;
    double *Fr = calloc((size_t)(ng > 0 ? ng : 1) * n2, sizeof(double));
    double *Fi = calloc((size_t)(ng > 0 ? ng : 1) * n2, sizeof(double));
    if (ng) bad |= orc_sfac(&s, ng, G, Fr, Fi) != 0;
    const double q[2] = {-6.0, -8.0}, Z[2] = {6.0, 8.0};
    bad |= orc_one_electron(&s, q, S, T, V) != 0;
    const double e = orc_ewald_energy(2, xyz, Z, cell, 0.4, 1e-12, 1e-12);
    printf("nbf_cart %d G %d pairs %ld J00 %.6f K00 %.6f E_nuc %.6f bad %d\n", nb, nG, np, J[0], K[0], e, bad);
    free(G); free(w); free(sa); free(sb); free(ia); free(ib); free(n3); free(Q);
    free(S); free(T); free(V); free(D); free(J); free(K); free(Fr); free(Fi);
    return bad;
}
