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

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBC_JK_OK 0
#define PBC_JK_EINVAL (-1)   /* bad argument: shape, value, NaN/Inf, l > 2, asymmetric D */
#define PBC_JK_ENOMEM (-2)   /* device or host allocation failed, or over the HBM budget */
#define PBC_JK_EDEVICE (-3)  /* HIP runtime error; the handle is unusable                 */
#define PBC_JK_ENOTSUP (-4)  /* request outside what the library implements             */
#define PBC_JK_ECANCELED (-5) /* server request cancelled before its build started       */
#define PBC_JK_EBUSY (-6)    /* server request already running: too late to cancel       */

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
 *                     couples| > schwarz, Q = the square root of the
 *                     largest component of the primitive pair's own
 *                     short-range integral (ab|ab) with the erfc(w r)/r
 *                     kernel (the Cauchy-Schwarz bound of Sec. 2.4, eq.
 *                     local_cauchy_schwarz_bound, for the real-space terms);
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
    double t_sr_ms, t_lr_ms, t_other_ms; /* last build, device stage times: density
                            preparation, the density factor of the low-rank exchange and the
                            short range on the build stream; reciprocal part and self term on
                            a second stream of the handle, concurrently with the short range;
                            final assembly after both                                         */
    double t_gemm_ms;    /* last build: summed durations of the launches of the GEMM kernel that
                            formed the reciprocal exchange (gemm_kernel), self term included
                            when that kernel is the plain one                                  */
    double gemm_flops;   /* last build: algorithmic FLOPs of those launches (2 M N K each; the
                            upper-triangle accumulations count M (M + 1) K)                    */
    int n_gemm;          /* last build: number of those launches                                */
    double t_sfac_ms;    /* last build: summed durations of the structure-factor launches      */
    double terms_class[21]; /* last build: short-range terms per class pair, in the order
                               (bra class, ket class) = (0,0),(0,1),..,(0,5),(1,1),..,(5,5)
                               with classes ss, ps, pp, ds, dp, dd                      */
    double n_group_pairs; /* entries of the real-space neighbour lists (group pairs that can
                               have a term for some density)                            */
    double lr_rank;      /* last build: rank of the density factor used by the reciprocal
                            exchange, or -1 when the dense form was used                */
    double t_chol_ms;    /* last build: duration of the density factorisation and of its
                            residual check                                                     */
    int gemm_kernel;     /* kernel of t_gemm_ms: 0 k_dgemm<0> (dense exchange T_G = F_G D,
                            K += T_G F_G, and the self term), 3 k_dgemm<3> (low-rank
                            accumulation K += sum_G Y_G Y_G^T, Y_G = sqrt(W_G) F_G L, FLOPs
                            counted on the upper triangle)                                     */
    double t_sr_class_ms[21]; /* last build: duration of the short-range launches per class
                            pair (same order as terms_class)                                   */
    double t_y_ms;       /* last build: duration of the low-rank products Y_G^T = L^T F_G
                            (k_dgemm<2>)                                                       */
    double y_flops;      /* last build: their FLOPs (2 n^2 rank per F matrix)                  */
    int n_y;             /* last build: number of those launches                               */
    int sr_fold_mask;    /* last build: bit k set when class pair k summed its lattice shifts
                            before the transforms                                              */
    int sr_kernel_mask;  /* last build: bit k set when class pair k ran one wavefront per group
                            pair (else one lane per group pair, in component slices for the
                            large d pairs)                                                     */
    int sr_jengine_mask; /* last build: bit k set when class pair k ran the J-engine (builds
                            without K: Hermite densities of the pairs, no Cartesian block)     */
    int y_kernel;        /* kernel of t_y_ms: 1 k_ygemm (512-row panels, when the reciprocal part
                            runs without the short range beside it), 0 k_dgemm<2>            */
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
 * NULL = the default stream): the reciprocal part runs on streams of the
 * handle that start after the work already queued on `stream` and that
 * `stream` waits for before the final assembly, so the build is ordered on
 * `stream` like a single launch.  Nothing in the build waits on the host:
 * the density factor's rank and the choice of exchange form stay on the
 * device.  E_J/E_K are host pointers (may be NULL); when given, the call
 * synchronises `stream` once at the end to read them, otherwise it returns
 * with the build queued.  D is not checked for symmetry on this path. */
int pbc_jk_build_device(pbc_jk *h, const double *dD, double *dJ, double *dK,
                        double *E_J, double *E_K, void *stream);

/* The same build as pbc_jk_build_device without any device allocation,
 * for callers that cannot allocate (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the per-build work buffers
 * (densities and J/K halves in the scaled Cartesian basis, the reciprocal
 * structure-factor chunk and products, the density factor, counters) come
 * from one static device array of 256 MiB per GPU, held until the process
 * ends; the handle keeps only its setup data and neighbour lists in use.
 * The reciprocal chunk is shrunk to fit; a cell whose work buffers do not
 * fit even with one reciprocal vector per chunk (about 94 nbf_cart^2 bytes:
 * nbf_cart up to about 1600) fails with PBC_JK_ENOMEM.  The call allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.  Every call
 * on one GPU shares that GPU's array: calls whose work overlaps on the device
 * (two streams, two threads) race and give wrong results; calls queued on
 * one stream are ordered.  The counters of pbc_jk_stats then describe this
 * build.  Arguments, stream ordering and errors as pbc_jk_build_device. */
int pbc_jk_build_device_static(pbc_jk *h, const double *dD, double *dJ, double *dK,
                               double *E_J, double *E_K, void *stream);

/* Gamma-point one-electron terms on the handle's pair list, lattice and
 * reciprocal vectors (host outputs, nbf x nbf, each may be NULL):
 *   S     overlap (Sec. 2.2, eq. pbc_overlap_formula);
 *   T     kinetic energy (supporting information, eq. kinetic_formula);
 *   V     nuclear attraction -sum_C Z_C <mu| v(r - C) |nu>, v the periodic
 *         Coulomb potential of a unit point charge with its G = 0 term
 *         removed, Ewald-split as in Sec. 2.3 (eq. pbc_v1e_general_final:
 *         real-space erfc sum inside the sphere of eq.
 *         pbc_v1e_real_cutoff_implementation, reciprocal sum over the
 *         handle's G sphere, self term -(pi/(V w^2)) sum_C q_C S);
 *   E_nuc nuclear repulsion energy (Sec. 2.9, eq. nuclear_repulsion_energy),
 *         real-space radius from erfc(x) < (2/sqrt(pi)) e^{-x^2}/x and the
 *         handle's G sphere.
 * Z are the charges given in pbc_atoms.charge at creation; V or E_nuc
 * without them is PBC_JK_EINVAL.  Uses the handle's work buffers and its own
 * stream; synchronous.  Calls on one handle must not overlap (builds
 * included). */
int pbc_jk_one_electron(pbc_jk *h, double *S, double *T, double *V, double *E_nuc);

/* Releases the handle and its device memory.  NULL is accepted. */
void pbc_jk_destroy(pbc_jk *h);

/* Number of output AOs, or a negative code for a NULL handle. */
int pbc_jk_nbf(const pbc_jk *h);

/* Copies the handle's counters and timings into *out. */
int pbc_jk_stats(const pbc_jk *h, pbc_jk_counters *out);

/* Graph mode of the host-memory build (pbc_jk_build): when enabled, the
 * first build captures its device work on the handle's stream (with the
 * fork to and join from the handle's side streams) into a HIP graph, and
 * later builds copy D in, replay the graph and copy J, K and the energies
 * out.  The graph fixes the host-side choices of the captured build (kernel
 * and lattice-sum order per class pair, the columns queued for the density
 * factor); the factor's rank and the exchange form are still decided on the
 * device at every replay.  Changing parts, class pairs or the exchange form,
 * or disabling graph mode, drops the graph.  Device builds
 * (pbc_jk_build_device, pbc_jk_build_device_static) are not affected. */
int pbc_jk_set_graph(pbc_jk *h, int enable);

/* Parts of the sum to evaluate (bit mask, default all): 1 = real-space
 * erfc sum, 2 = reciprocal sum, 4 = self term.  For per-part testing. */
#define PBC_JK_PART_SR 1
#define PBC_JK_PART_LR 2
#define PBC_JK_PART_SELF 4
int pbc_jk_set_parts(pbc_jk *h, int mask);

/* Restricts the real-space part to the class pairs whose bits are set in
 * mask21 (bit k = k-th (bra class, ket class) pair in the order of
 * terms_class; default all 21).  For per-class testing and for timing a
 * large cell one class pair at a time.  EINVAL for a NULL handle or bits
 * above 2^21. */
int pbc_jk_set_sr_classes(pbc_jk *h, int mask21);

/* Form of the reciprocal exchange K_LR = sum_G W_G (A_G D A_G + B_G D B_G)
 * (Sec. 2.4; A, B the real and imaginary pair structure factors):
 *   PBC_JK_LR_AUTO  (default) factor D = L L^T by pivoted Cholesky on the
 *                   device, stopping when every remaining diagonal entry is
 *                   <= tol * max diag(D), and use K_LR = sum_G W_G (Y Y^T)
 *                   with Y = A_G L and B_G L; the factor is accepted only if
 *                   max |D - L L^T| <= 2 tol max diag(D) + 4 n eps max diag(D)
 *                   and its rank is at most 3/4 of the Cartesian AO count,
 *                   otherwise the dense form runs.  Both forms are queued
 *                   and gated on the device by that decision, so the host
 *                   never waits for it; the columns queued for the factor
 *                   are the last finished build's rank plus 64 (the limit
 *                   when unknown), and a factor needing more falls back to
 *                   the dense form for that build.
 *   PBC_JK_LR_DENSE always the dense form T_G = A_G D, K_LR += W_G T_G A_G.
 * tol <= 0 keeps the current tolerance (default 1e-13).  EINVAL for an
 * unknown mode or a NULL handle. */
#define PBC_JK_LR_AUTO 0
#define PBC_JK_LR_DENSE 1
int pbc_jk_set_lr(pbc_jk *h, int mode, double tol);

/* ------------------------------------------------------------------------
 * Request server: Fock builds for many cells, as an SCF or MD driver issues
 * them.  Requests are queued in arrival order and run on `slots` worker
 * threads, each build on its own HIP stream, so builds of different cells
 * overlap on the device.  All device memory of the server comes from one
 * arena of `hbm_budget` bytes allocated at creation (no hipMalloc/hipFree per
 * request).  A request for a new cell is admitted when its footprint (setup
 * data, work buffers and neighbour lists) fits in the free part of the arena;
 * the first new-cell request (in queue order, see `policy`) that does not
 * fit blocks later new-cell requests (no starvation), while requests for
 * cells already resident run
 * as soon as their cell is idle.  With cache_cells set, a cell's setup data
 * stays resident after its build and later requests with identical cell,
 * atoms, basis, omega and thresholds reuse it; idle cells are evicted
 * least-recently-used when memory is needed.  A request whose footprint
 * exceeds the whole budget fails with PBC_JK_ENOMEM; a bad input fails only
 * its own request.
 * ------------------------------------------------------------------------ */
typedef struct pbc_jk_server pbc_jk_server;

typedef struct {
    size_t hbm_budget;    /* arena bytes; 0 = half of the device's free memory           */
    int slots;            /* concurrent builds (worker threads / streams); 0 = 4            */
    int cache_cells;      /* keep idle cells resident for reuse (0/1)                       */
    double lr_budget_mb;  /* per-cell reciprocal-sum chunk budget; 0 = 1024 MB              */
    int use_graphs;       /* with cache_cells: builds of a resident cell after its first one
                             replay a captured HIP graph (pbc_jk_set_graph)                 */
    int policy;           /* queue order: PBC_JK_SERVE_ARRIVAL (0) by submission;
                             PBC_JK_SERVE_DEADLINE (1) by submission time plus an estimate
                             of the build time from the cell's AO count (c nbf^2), so that
                             small requests pass large ones queued a little earlier while
                             every request still comes first once it has waited its own
                             estimate longer than later arrivals                            */
} pbc_jk_server_config;
#define PBC_JK_SERVE_ARRIVAL 0
#define PBC_JK_SERVE_DEADLINE 1

typedef struct {
    int status;           /* 0 or the request's error code                                  */
    int cache_hit;        /* 1 when the cell's setup data was already resident              */
    int retries;          /* admissions retried after the budget was short                  */
    int nbf;              /* output AOs                                                     */
    double queue_ms;      /* submit -> start of work on a worker                            */
    double setup_ms;      /* host setup + device creation (0 on a cache hit)                */
    double build_ms;      /* the build itself, D in to J, K, E out                          */
    double latency_ms;    /* submit -> completion                                           */
    size_t device_bytes;  /* device bytes the cell holds                                    */
    char error[160];      /* message when status != 0                                       */
} pbc_jk_request_info;

typedef struct {
    long submitted, completed, failed, cancelled, cache_hits, evictions, retries;
    int slots;
    int peak_running;     /* most requests in work (setup or build) at once                 */
    size_t budget;        /* arena bytes                                                    */
    size_t in_use;        /* arena bytes held now                                           */
    size_t peak_in_use;   /* most arena bytes held at once                                  */
} pbc_jk_server_counters;

/* cfg may be NULL (defaults).  ENOMEM when the arena cannot be allocated. */
int pbc_jk_server_create(const pbc_jk_server_config *cfg, pbc_jk_server **out);

/* Queues one build.  The cell, atoms, basis, thresholds and D (nbf x nbf,
 * host) are copied before the call returns; J and K (host, nbf x nbf, either
 * may be NULL) and E_J/E_K (may be NULL) must stay valid until
 * pbc_jk_server_wait returns for the ticket.  EINVAL for missing inputs. */
int pbc_jk_server_submit(pbc_jk_server *s, const pbc_cell *cell, const pbc_atoms *atoms,
                         const pbc_basis *basis, double omega, const pbc_jk_thresholds *thr,
                         const double *D, double *J, double *K, double *E_J, double *E_K,
                         unsigned long long *ticket);

/* Blocks until the request is done; fills *info (may be NULL) and returns the
 * request's status.  Each ticket is waited for once; EINVAL for an unknown
 * ticket. */
int pbc_jk_server_wait(pbc_jk_server *s, unsigned long long ticket, pbc_jk_request_info *info);

/* Cancels a request that has not started its build: it completes with
 * PBC_JK_ECANCELED.  A build already running finishes normally.  Returns 0
 * when the request will be cancelled, PBC_JK_EBUSY when it is too late,
 * EINVAL for an unknown ticket. */
int pbc_jk_server_cancel(pbc_jk_server *s, unsigned long long ticket);

int pbc_jk_server_stats(pbc_jk_server *s, pbc_jk_server_counters *out);

/* Cancels queued requests, waits for running builds, releases everything.
 * Tickets not yet waited for become invalid.  NULL is accepted. */
void pbc_jk_server_destroy(pbc_jk_server *s);

/* ---------------------------------------------------------------------
 * Periodic Becke partition weights of atom-centred integration-grid points
 * (Sec. 2.8, "Becke weights": eqs. becke_weight_definition,
 * becke_vicinity_definition, becke_mu_definition, becke_switch_definition).
 * For a point r whose origin atom is A, with X, Y running over the atom
 * images within rcut of A's home position (the paper's radius is 17 bohr):
 *   w(r) = P(A, r) / sum_X P(X, r),   P(X, r) = prod_{Y != X} s(X, Y, r),
 *   s = (1 - f(f(f(u)))) / 2, f(x) = x (3 - x^2) / 2,
 *   u = (|r - X| - |r - Y|) / |X - Y|.
 * P(X, r) is zero once one switching factor is below delta; w is zero when
 * P(A, r) is below delta.  The printed denominator's product over images is
 * read as a sum over the atom images within the sphere.  The quadrature
 * weight of a point (eq. total_weight_definition) is the caller's to apply.
 */
typedef struct pbc_becke pbc_becke; /* opaque plan: the image lists of a cell */

/* Builds the plan for natom atoms at xyz (natom*3, bohr) in `cell`: for
 * every atom, the list of atom images within rcut (> 0) of it, on the
 * current device.  delta >= 0.  Inputs are copied. */
int pbc_becke_create(const pbc_cell *cell, int natom, const double *xyz, double rcut, double delta,
                     pbc_becke **out);

/* Weights of npts points: d_pts (npts*3 doubles), d_origin (npts ints, the
 * origin atom index of each point) and d_w (npts doubles, written) are device
 * pointers; the kernel is queued on `stream` (a hipStream_t, NULL = default)
 * and the call returns without waiting.  Points grouped by origin atom run
 * fastest.  A point whose origin index is outside [0, natom) gets a NaN
 * weight.  Calls on one plan may overlap (the plan is read only). */
int pbc_becke_weights(pbc_becke *b, long npts, const double *d_pts, const int *d_origin, double *d_w,
                      void *stream);

/* Largest and total number of images in the plan's lists (NULL skips). */
int pbc_becke_info(const pbc_becke *b, int *max_images, long *total_images);

/* Switching factors s(X, Y, r) evaluated by the plan's last pbc_becke_weights
 * call (the work the kernel did: at most M (M - 1) a point for M images, fewer
 * where a factor fell below delta).  Waits for that call's stream. */
int pbc_becke_evaluations(pbc_becke *b, double *evaluations);

/* Frees the plan (NULL is accepted). */
void pbc_becke_destroy(pbc_becke *b);

/* Message of the last error on this thread ("" if none). */
const char *pbc_jk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PBCJK_H */
