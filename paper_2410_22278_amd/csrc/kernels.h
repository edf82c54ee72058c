// Kernel argument blocks and launchers (host-callable).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace pbcjk {

struct SRArgs {
    const PairRec *pairs;
    const GroupRec *groups;
    int gb0, gk0;         // first group of the bra and ket classes
    int tri;              // same class: the diagonal group pair has weight 1/2
    const int *nbr_bra;   // work list of this class pair (bra, ket indices within
    const int *nbr_ket;   //   their classes): the density-screened part of the
                          //   neighbour list in one precision
    const unsigned long long *count;   // device: entries in the work list
    long max_entries;     // host: upper bound of *count (sizes the grid)
    int max_prim_pairs;   // host: most primitive pairs in one group of either class
    const double *Dt;     // scaled Cartesian density, nbfc x nbfc
    const double *Dmax;   // nshell x nshell block maxima of the Cartesian density
    double *X, *Y;        // J and K halves, nbfc x nbfc
    int nbfc, nshell;
    LatArgs lat;
    double w2, d_schwarz, d_ewald_R, rcap2;
    double fp32_below;    // > 0: quartets with Q Q w_D below it are evaluated in FP32
    const double *boys;   // kBoysNT x kBoysM
    const double *bexp;   // kBoysNT: e^{-k h} on the Boys grid
    unsigned long long *counters;   // [0] primitive quartets, [1] (quartet, R1) terms,
                                    // [2 + slot] terms of this class pair, [23] FP32 terms,
                                    // [24 + slot] primitive quartets of this class pair
    int slot;             // class-pair index (0..20)
    int want_k;           // 0: builds without K skip the K half's contractions and atomics
    // J-engine only: Hermite densities of the bra and ket classes' pairs, the
    // densities of pair k at hd + (k - hd_p0) n_h(l_a + l_b)
    const double *hd_b, *hd_k;
    int hd_p0b, hd_p0k;
};

// Hermite densities of one class's primitive pairs (B2 of the J-engine):
// hd[(k - p0) n_h + h] = cpre_k sum_{a,b} E^{ab}_h(k) Dt[a][b] for the pairs k
// of groups g0 .. g0 + ngroups - 1 (pairs p0 onwards).
struct HdensArgs {
    const PairRec *pairs;
    const GroupRec *groups;
    int g0, ngroups, p0;
    const double *Dt;
    int nbfc;
    double *hd;
};
hipError_t launch_hdens(int cls, const HdensArgs &a, hipStream_t st);
// Short-range J alone (J-engine) of class pair (cb, ck); hipErrorNotSupported
// for the class pairs it does not cover (total angular momentum above 5).
hipError_t launch_sr_j(int cb, int ck, const SRArgs &a, hipStream_t st);

// Neighbour list of one class pair: every (bra group, ket group) that has at
// least one real-space term for some density (mode 0 counts per bra and
// distance bucket, mode 1 writes the ket indices at the given per-(bra,
// bucket) offsets, in ket order inside a bucket).
struct NbrArgs {
    const PairRec *pairs;
    const GroupRec *groups;
    int gb0, nb, gk0, nk, tri;
    LatArgs lat;
    double w2, d_ewald_R, rcap2;
    int mode;
    double inv_bw;        // 1 / width (bohr) of the distance buckets; 0: one bucket
    int *counts;          // nb * kNbrBuckets
    const long *offsets;  // nb * kNbrBuckets
    int *out_bra, *out_ket;
};
// A bra group's entries are written in buckets of the distance between the two
// group centres (nearest translate), nearest first: lanes of a wavefront then
// hold ket groups at similar distances, whose quartets pass the real-space
// sphere and the shift search alike.
constexpr int kNbrBuckets = 16;
hipError_t launch_nbr(const NbrArgs &a, hipStream_t st);

// Per-build density screen of one class pair's neighbour list: entries with
// Qmax_b Qmax_k w_D > d_schwarz are appended (in chunks of 256 that keep
// their order) to the FP64 list, or to the FP32 list when `split` and the
// same bound is below fp32_below.  counts[0], counts[1]: list lengths (must
// be zero on entry).
struct PartArgs {
    LatArgs lat;
    const GroupRec *groups;
    int gb0, gk0;
    const int *bra, *ket;
    long n;
    const double *Dmax;
    int nshell;
    double d_schwarz, fp32_below;
    int split;
    int *b64, *k64, *b32, *k32;
    unsigned long long *counts;   // out: entries of the FP64 and of the FP32 list
    long long *chunk_counts;      // work: 2 per chunk of kPartChunk entries
};
constexpr int kPartChunk = 4096;  // entries per counted chunk of the order-preserving split
hipError_t launch_partition(const PartArgs &a, hipStream_t st);

hipError_t launch_sr_jk(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st);
// large d class pairs in the per-lane kernel, one launch per component slice
hipError_t launch_sr_slices(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st);
hipError_t launch_sr_slices_dp(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st);
// class pairs with total angular momentum >= 5 (one wavefront per group pair)
hipError_t launch_sr_coop(int cb, int ck, const SRArgs &a, hipStream_t st);

// ---- one-electron terms (one_e.hip)

// S, T and the short-range part of V of the pairs of one class's groups, into
// halves in the scaled Cartesian basis (M = X + X^T).
struct OneEArgs {
    const PairRec *pairs;
    const GroupRec *groups;
    int g0, ngroups;
    int nbfc;
    const double *xyz, *q;   // natom positions, point charges (potential q_C / |r - C|)
    int natom;
    LatArgs lat;
    double w2, d_ewald_R, rcap2;
    const double *boys, *bexp;
    double *XS, *XT, *XV;
};
hipError_t launch_one_e(int cls, const OneEArgs &a, hipStream_t st);
// Nuclear structure factor on ng half-space vectors, scaled by Gs: rho[g] real
// parts, rho[ng + g] imaginary parts of sum_C q_C e^{-i G.C}.
hipError_t launch_rho_nuc(const double *G, const double *Gs, int ng, const double *xyz, const double *q, int natom,
                          double *rho, hipStream_t st);
// *out += real-space part of the point-charge Ewald energy (images within
// sqrt(rb2) of each atom pair).
hipError_t launch_enuc_real(const double *xyz, const double *q, int natom, const LatArgs &lat, double w,
                            double rb2, double *out, hipStream_t st);

// ---- long range and utilities (lr.hip)

// Structure factors of a chunk of reciprocal vectors: F[b][mu][nu] for
// b < ng the real parts, b in [ng, 2ng) the imaginary parts.
struct SfacArgs {
    const PairRec *pairs;
    const int *sp_start, *sp_pairs, *sp_shA, *sp_shB;
    const int *sh_l, *sh_aoc;
    int sp0, nsp;         // shell-pair range of one class
    const double *G;      // 3 * ng
    const double *Gs;     // ng scale factors applied to F_G (sqrt of the weights), or NULL
    int ng;
    double *F;            // 2 ng x nbfc x nbfc
    int nbfc;
};
hipError_t launch_sfac(int cls, const SfacArgs &a, hipStream_t st);

// rho[b] = sum_{mu nu} Dt[mu nu] F[b][mu nu] for b < nb.
hipError_t launch_dot_batched(const double *F, const double *Dt, int n2, int nb, double *rho, hipStream_t st);

// Jt[mu nu] += sum_g Gw[g] (F[g][mu nu] rho[g] + F[ng+g][mu nu] rho[ng+g]).
// K[r][c] += sum_k P[k][r][c] for k < nc (n x n matrices), skipping the block
// r >= bs, c < bs.
hipError_t launch_sum_partials(const double *P, int nc, int n, int bs, double *K, hipStream_t st);
// Jt += sum_g Gw[g] (Re F_g rho_g + Im F_g rho'_g); Gw NULL: unit weights.
hipError_t launch_jlr(const double *F, const double *rho, const double *Gw, int ng, int n2, double *Jt,
                      hipStream_t st);

// C_b = alpha_b A_b B_b (mode 0) or C += sum_b alpha_b A_b B_b (mode 1,
// batches split into `slices` partial sums added atomically).  Row-major.
struct GemmArgs {
    int M, N, K;
    const double *A; long lda, sA;
    const double *B; long ldb, sB;
    double *C; long ldc, sC;
    int nbatch;
    const double *alpha;  // device, per batch; NULL = 1
    double alpha0;        // scalar factor applied on top
    int reduce;
    int slices;
    int transA;           // A element (m, k) read from A[k * lda + m]
    int transB;           // B element (k, j) read from B[j * ldb + k]
    int upper;            // compute only output tiles on or above the diagonal (M == N)
    // Device-side gating by the low-rank control block ctl = {rank, use_dense}:
    // 0 none; 1 skip if use_dense, N = rank; 2 skip if use_dense, K = rank;
    // 3 skip unless use_dense; 4 skip if use_dense, M = rank.  The host sizes
    // the grid for the upper bound of the rank; tiles beyond it return.
    const int *ctl;
    int ctl_mode;
    // Instantiation (one per role, so that profiles tell them apart):
    // 0 plain products (self term, dense exchange), 1 residual check of the
    // density factor, 2 Y_b^T = L^T F_b, 3 K += sum_b Y_b Y_b^T.
    int role;
    int tile;             // output tile edge, 64 or 128 (0: kGemmTile); products that
                          // accumulate the upper tiles of K always use kGemmTile
};
hipError_t launch_dgemm(const GemmArgs &a, hipStream_t st);
// C_b = alpha0 A B_b for the low-rank exchange factors (row-major A, B_b, C_b;
// no transposes, no reduction), M gated by ctl_mode 4 as in launch_dgemm:
// 64-column panels of up to 512 rows per workgroup (k_ygemm).
hipError_t launch_ygemm(const GemmArgs &a, hipStream_t st);

// Sets the thread's last-error message read by pbc_jk_last_error; returns code.
int set_error(int code, const char *msg);
// Edge of the upper blocks in which K is accumulated (and read back by the
// final assembly), and the default GEMM output tile.
constexpr int kGemmTile = 64;

// Pivoted Cholesky of a symmetric n x n matrix D ~= L L^T, L stored by
// columns (column j at L + j * n), with the rank and the stop decision kept
// on the device: nothing is read back to the host.  With a work matrix Aw
// (n x n, overwritten) it runs in panels of 32 columns (one launch for the
// panel's columns, one for the trailing update); without, one launch per
// column.  Launches after the stop return at once.  Stops when the largest
// remaining diagonal entry is <= tol * max diag(D) or after rmax columns.
// ctl (4 ints): {rank, use_dense, done, -}.  work: n + 2 * ceil(n / 64) + 4
// doubles and 2 * ceil(n / 64) ints (wi).  use_dense is set when the factor
// did not converge within rmax columns or D has a diagonal entry below
// -tol * max.
hipError_t launch_pchol(const double *D, int n, double tol, int rmax, double *L, double *work, int *wi,
                        int *ctl, double *Aw, hipStream_t st);
// After R = L L^T: sets ctl[1] when max |D - R| exceeds 2 tol max diag(D)
// plus the rounding allowance 4 n eps max diag(D).
hipError_t launch_lowrank_check(const double *D, const double *R, int n, const double *work, int *ctl,
                                hipStream_t st);

hipError_t launch_fill(double *p, long n, double v, hipStream_t st);

// Density preparation: Dt (scaled Cartesian), Dc block maxima per shell pair
// and their global maximum (as the bit pattern of a non-negative double).
struct DprepArgs {
    const double *D;      // nbf x nbf
    int nbf, nbfc, nshell;
    const int *tr_ao;     // 2 * nbfc
    const double *tr_c;   // 2 * nbfc
    const double *dscale; // nbfc
    const int *sh_aoc, *sh_l;
    double *Dt;           // nbfc^2
    double *Dmax;         // nshell^2
    unsigned long long *dmax_glob;
};
hipError_t launch_dprep(const DprepArgs &a, hipStream_t st);

// sum_{ij} A[i] B[i] into out (atomic add).
hipError_t launch_dot(const double *A, const double *B, long n, double *out, hipStream_t st);

// Jt += f * s * S where s = *sdot (device scalar).
hipError_t launch_axpy_scaled(double *Y, const double *X, long n, double f, const double *sdot, hipStream_t st);

// Finalise: Jc = X + X^T + Jt, out[a][b] = sum T'[a][i] T'[b][j] Jc[i][j]
// using the inverse transform lists (up to 3 entries per output AO).
struct FinalArgs {
    const double *X, *Jt;  // Jt may be NULL (no full-matrix part)
    int nbfc, nbf;
    int jt_block;          // > 0: Jt holds only its upper blocks of this size (block row <= block column); 0: whole
    const int *inv_ci;     // 3 * nbf scaled-Cartesian indices (-1 = none)
    const double *inv_cc;  // 3 * nbf coefficients
    double *out;           // nbf^2
};
hipError_t launch_final(const FinalArgs &a, hipStream_t st);

}  // namespace pbcjk
