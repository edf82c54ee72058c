/*
 * pbcjk.h -- C ABI of the MI355X (gfx950) Gamma-point periodic Coulomb (J)
 * and exact-exchange (K) matrix build over contracted Gaussians with Ewald
 * splitting.
 *
 * The quantity (paper: Wang et al., periodic Gaussian integrals on GPUs):
 *   J_{mu nu} = sum_{la si} (mu nu|la si) D_{la si}
 *   K_{mu nu} = sum_{la si} (mu la|nu si) D_{la si}
 * at the Gamma point (Sec. 2.5 eqs. pbc_j_definition_k_sample and
 * pbc_k_definition with k = 0 and weight 1; Sec. 2.6), where (mu nu|la si)
 * is the periodic electron repulsion integral of Sec. 2.4 (eq.
 * pbc_eri_general_final with every k = 0): a real-space sum of erfc(w r)/r
 * four-centre integrals over lattice images R1, a reciprocal-space sum over
 * G != 0, and the self (G = 0 difference) term.  E_J = 1/2 sum D J,
 * E_K = -1/4 sum D K (closed shell, D spin-summed).
 *
 * Conventions
 *   - Units: bohr for lengths, bohr^-2 for exponents, bohr^-1 for omega.
 *   - Matrices are dense, row-major, double precision, nbf x nbf.
 *   - AO order: shells in input order; Cartesian components x^l, x^(l-1)y,
 *     ... (xx, xy, xz, yy, yz, zz for d); spherical d (pure = 1) as real
 *     solid harmonics m = -2..2: xy, yz, z^2 - (x^2+y^2)/2, xz,
 *     (sqrt3/2)(x^2 - y^2), unit-normalised.
 *   - Primitives are normalised as in Sec. 2.1 (eq. local_normalization);
 *     the library rescales each contracted shell to unit single-centre
 *     self-overlap (the crystalline function itself is not normalised).
 *   - Angular momentum l <= 2.
 *
 * Ownership: pbc_jk_create deep-copies every input; the caller may free them
 * when it returns.  The handle owns all device memory it allocates.  Build
 * calls never retain D, J or K pointers.
 *
 * Errors: functions return 0 on success or a negative PBC_JK_E* code and set
 * a thread-local message readable with pbc_jk_last_error().  A handle whose
 * call returned PBC_JK_EDEVICE must only be destroyed.
 *
 * Threads: one handle per concurrent caller; distinct handles are
 * independent.  Calls on one handle must not overlap.
 */
#ifndef PBCJK_H
#define PBCJK_H

#ifdef __cplusplus
extern "C" {
#endif

#define PBC_JK_OK 0
#define PBC_JK_EINVAL (-1)   /* bad argument: shape, value, NaN/Inf, l > 2, asymmetric D */
#define PBC_JK_ENOMEM (-2)   /* device or host allocation failed, or over the HBM budget */
#define PBC_JK_EDEVICE (-3)  /* HIP runtime error; the handle is unusable                 */
#define PBC_JK_ENOTSUP (-4)  /* request outside what the library implements             */

typedef struct pbc_jk pbc_jk; /* opaque handle */

/* Lattice: rows are the vectors a, b, c (bohr); must be non-singular. */
typedef struct {
    double a[9];
} pbc_cell;

/* Atoms: natom positions (natom*3, bohr); charge is not used by J/K and
 * may be NULL. */
typedef struct {
    int natom;
    const double *xyz;
    const double *charge;
} pbc_atoms;

/* Basis: nshell shells; per shell the atom index, angular momentum l
 * (0..2), pure flag (1 = spherical, honoured for l = 2) and primitive count;
 * exps/coefs are concatenated over shells (sum nprim entries).  Exponents
 * must be positive; coefficients multiply normalised primitives. */
typedef struct {
    int nshell;
    const int *atom;
    const int *l;
    const int *pure;
    const int *nprim;
    const double *exps;
    const double *coefs;
} pbc_basis;

/* Truncation thresholds (Sec. 3.6 names four; all strictly positive):
 *   pair_R, pair_cs : local-pair image cutoffs of Sec. 2.4 (eqs.
 *                     pbc_eri_pair_cutoff_definition with the separable
 *                     prefactor sqrt2 pi^{5/4}|CaCb|/(p (p+2 a_min)^{1/4}),
 *                     and pbc_eri_cauchy_schwarz_cutoff_definition);
 *   ewald_R         : real-space image sphere per primitive quartet (eq.
 *                     pbc_eri_real_cutoff_definition);
 *   ewald_K         : global reciprocal sphere, (4 pi/V) e^{-G^2/4w^2}/G^2
 *                     > ewald_K;
 *   schwarz         : a primitive quartet is kept iff
 *                     Q_bra Q_ket max|D over the six shell-pair blocks it
 *                     couples| > schwarz, Q = the local-pair
 *                     Cauchy-Schwarz value of Sec. 2.4;
 *   fp32_below      : 0 = all quartets in FP64; otherwise quartets whose
 *                     density-weighted bound is below it run in FP32
 *                     (Sec. 3.5), accumulation stays FP64;
 *   r_cut, g_cut    : optional caps (0 = none) on |A - B(R2)| and
 *                     |P - Q - R1| (bohr) and on |G| (bohr^-1). */
typedef struct {
    double pair_R, pair_cs, ewald_R, ewald_K, schwarz;
    double fp32_below;
    double r_cut, g_cut;
} pbc_jk_thresholds;

/* Counters of one handle (filled by pbc_jk_stats). */
typedef struct {
    int nbf;             /* output AOs (spherical d counted as 5)            */
    int nbf_cart;        /* Cartesian AOs                                    */
    long n_pairs;        /* unique local primitive pairs                     */
    long n_groups;       /* unique (shell pair, image) groups                */
    int n_gvec;          /* reciprocal vectors in the half space             */
    double omega;        /* the Ewald parameter in use                       */
    double quartets;     /* last build: unique primitive quartets evaluated  */
    double terms;        /* last build: (quartet, R1 image) terms evaluated  */
    double terms_fp32;   /* last build: of which in FP32                     */
    double t_setup_ms;   /* create wall time                                 */
    double t_build_ms;   /* last build wall time                             */
    double t_sr_ms, t_lr_ms, t_other_ms; /* last build, device stage times   */
    double t_gemm_ms;    /* last build: summed durations of the FP64 matrix-core GEMM launches */
    double gemm_flops;   /* last build: algorithmic FLOPs of those launches (2 M N K each)     */
    int n_gemm;          /* last build: number of those launches                                */
    double t_sfac_ms;    /* last build: summed durations of the structure-factor launches      */
    double terms_class[21]; /* last build: short-range terms per class pair, in the order
                               (bra class, ket class) = (0,0),(0,1),..,(0,5),(1,1),..,(5,5)
                               with classes ss, ps, pp, ds, dp, dd                      */
    double n_group_pairs; /* entries of the real-space neighbour lists (group pairs that can
                               have a term for some density)                            */
} pbc_jk_counters;

/* Creates a handle: validates and copies the inputs, builds the local pair
 * lists, the reciprocal vector list, the Gamma overlap and the device-
 * resident setup data.  omega <= 0 selects omega = (10 pi^3/V^2)^{1/6}
 * (Sec. 3.4, eq. omega_implementation with weight 10).  thr may be NULL
 * (all deltas 1e-14, no caps, FP64). */
int pbc_jk_create(const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis,
                  double omega, const pbc_jk_thresholds *thr, pbc_jk **out);

/* One build from host memory: D (nbf x nbf, symmetric within 1e-10 max|D|)
 * in, J and K (nbf x nbf, caller-owned, either may be NULL to skip) and the
 * energies (either pointer may be NULL) out.  Synchronous. */
int pbc_jk_build(pbc_jk *h, const double *D, double *J, double *K, double *E_J, double *E_K);

/* One build on device memory: dD, dJ, dK are device pointers (nbf x nbf);
 * dJ or dK may be NULL to skip.  Work is queued on `stream` (a hipStream_t,
 * NULL = the default stream).  E_J/E_K are host pointers (may be NULL); when
 * given, the call waits for the stream before returning.  D is not checked
 * for symmetry on this path. */
int pbc_jk_build_device(pbc_jk *h, const double *dD, double *dJ, double *dK,
                        double *E_J, double *E_K, void *stream);

/* Releases the handle and its device memory.  NULL is accepted. */
void pbc_jk_destroy(pbc_jk *h);

/* Number of output AOs, or a negative code for a NULL handle. */
int pbc_jk_nbf(const pbc_jk *h);

/* Copies the handle's counters and timings into *out. */
int pbc_jk_stats(const pbc_jk *h, pbc_jk_counters *out);

/* Parts of the sum to evaluate (bit mask, default all): 1 = real-space
 * erfc sum, 2 = reciprocal sum, 4 = self term.  For per-part testing. */
#define PBC_JK_PART_SR 1
#define PBC_JK_PART_LR 2
#define PBC_JK_PART_SELF 4
int pbc_jk_set_parts(pbc_jk *h, int mask);

/* Message of the last error on this thread ("" if none). */
const char *pbc_jk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PBCJK_H */
