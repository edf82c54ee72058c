// Reciprocal-space (long-range) part, the self term and the utility kernels.
//
// With pair structure factors F_G[mu nu] = sum over local pairs of
//   int e^{-iG.r} mu(r) nu(r - R2) dr = c (pi/p)^{3/2} e^{-G^2/4p} e^{-iG.P} sum_t E_t (-iG)^t
// the reciprocal term of the periodic ERI (Sec. 2.4, eq.
// pbc_eri_general_final) becomes, over the half space of G with
// W_G = 2 (4 pi/V) e^{-G^2/4w^2}/G^2 and F = A + iB (A, B symmetric):
//   J_LR = sum_G W_G (A_G Re rho_D(G) + B_G Im rho_D(G)),  rho_D(G) = sum D F_G
//   K_LR = sum_G W_G (A_G D A_G + B_G D B_G)
// K_LR is a dense contraction and runs on the FP64 matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- structure factors
template <int LA, int LB>
__device__ __forceinline__ void sfac_pairs(const SfacArgs &a, int sp, double Gx, double Gy, double Gz,
                                           double (&re)[ncart(LA)][ncart(LB)], double (&im)[ncart(LA)][ncart(LB)])
{
    constexpr int NA = ncart(LA), NB = ncart(LB), LT = LA + LB;
    const double G2 = Gx * Gx + Gy * Gy + Gz * Gz;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) { re[i][j] = 0.0; im[i][j] = 0.0; }
    for (int k = a.sp_start[sp]; k < a.sp_start[sp + 1]; ++k) {
        const PairRec P = a.pairs[a.sp_pairs[k]];
        const double ip = P.pad[0];   // 1/p
        const double pre = P.cpre * exp(-0.25 * G2 * ip) * (kPi * ip) * sqrt(kPi * ip);
        double s, c;
        sincos(Gx * P.P[0] + Gy * P.P[1] + Gz * P.P[2], &s, &c);
        // e^{-i G.P} = c - i s
        EAxis<LA, LB> Ex, Ey, Ez;
        const double h = 0.5 * ip;
        herm_axis<LA, LB>(h, P.PA[0], P.PB[0], Ex);
        herm_axis<LA, LB>(h, P.PA[1], P.PB[1], Ey);
        herm_axis<LA, LB>(h, P.PA[2], P.PB[2], Ez);
        // powers (-iG)^t as (real, imag)
        double px_r[LT + 1], px_i[LT + 1], py_r[LT + 1], py_i[LT + 1], pz_r[LT + 1], pz_i[LT + 1];
        px_r[0] = py_r[0] = pz_r[0] = 1.0;
        px_i[0] = py_i[0] = pz_i[0] = 0.0;
#pragma unroll
        for (int t = 1; t <= LT; ++t) {
            // (r + i m)(-i g) = m g - i r g
            px_r[t] = px_i[t - 1] * Gx; px_i[t] = -px_r[t - 1] * Gx;
            py_r[t] = py_i[t - 1] * Gy; py_i[t] = -py_r[t - 1] * Gy;
            pz_r[t] = pz_i[t - 1] * Gz; pz_i[t] = -pz_r[t - 1] * Gz;
        }
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                double hxr = 0, hxi = 0, hyr = 0, hyi = 0, hzr = 0, hzi = 0;
#pragma unroll
                for (int t = 0; t <= cx(LA, ia) + cx(LB, ib); ++t) {
                    hxr += Ex.v[cx(LA, ia)][cx(LB, ib)][t] * px_r[t];
                    hxi += Ex.v[cx(LA, ia)][cx(LB, ib)][t] * px_i[t];
                }
#pragma unroll
                for (int t = 0; t <= cy(LA, ia) + cy(LB, ib); ++t) {
                    hyr += Ey.v[cy(LA, ia)][cy(LB, ib)][t] * py_r[t];
                    hyi += Ey.v[cy(LA, ia)][cy(LB, ib)][t] * py_i[t];
                }
#pragma unroll
                for (int t = 0; t <= cz(LA, ia) + cz(LB, ib); ++t) {
                    hzr += Ez.v[cz(LA, ia)][cz(LB, ib)][t] * pz_r[t];
                    hzi += Ez.v[cz(LA, ia)][cz(LB, ib)][t] * pz_i[t];
                }
                // h = hx hy hz (complex), times (c - i s)
                double xyr = hxr * hyr - hxi * hyi, xyi = hxr * hyi + hxi * hyr;
                double hr = xyr * hzr - xyi * hzi, hi = xyr * hzi + xyi * hzr;
                re[ia][ib] += pre * (hr * c + hi * s);
                im[ia][ib] += pre * (hi * c - hr * s);
            }
    }
}

template <int LA, int LB>
__device__ __forceinline__ void sfac_store(const SfacArgs &a, int sp, int g, double Gx, double Gy, double Gz)
{
    constexpr int NA = ncart(LA), NB = ncart(LB);
    double re[NA][NB], im[NA][NB];
    sfac_pairs<LA, LB>(a, sp, Gx, Gy, Gz, re, im);
    if (a.Gs) {
        const double w = a.Gs[g];
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) { re[ia][ib] *= w; im[ia][ib] *= w; }
    }
    const int A = a.sp_shA[sp], B = a.sp_shB[sp];
    const long n = a.nbfc;
    double *Fr = a.F + (long)g * n * n;
    double *Fi = a.F + (long)(a.ng + g) * n * n;
    const int aoA = a.sh_aoc[A], aoB = a.sh_aoc[B];
    if (A == B) {
        // F = F_h + F_h^T inside one shell
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                Fr[(aoA + ia) * n + aoB + ib] = re[ia][ib] + re[ib < NA ? ib : 0][ia < NB ? ia : 0];
                Fi[(aoA + ia) * n + aoB + ib] = im[ia][ib] + im[ib < NA ? ib : 0][ia < NB ? ia : 0];
            }
    } else {
#pragma unroll
        for (int ia = 0; ia < NA; ++ia)
#pragma unroll
            for (int ib = 0; ib < NB; ++ib) {
                Fr[(aoA + ia) * n + aoB + ib] = re[ia][ib];
                Fr[(aoB + ib) * n + aoA + ia] = re[ia][ib];
                Fi[(aoA + ia) * n + aoB + ib] = im[ia][ib];
                Fi[(aoB + ib) * n + aoA + ia] = im[ia][ib];
            }
    }
}

// one block per shell pair of one class, threads over reciprocal vectors
template <int LA, int LB>
__global__ __launch_bounds__(64) void k_sfac(SfacArgs a)
{
    const int sp = a.sp0 + blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.ng) return;
    const double Gx = a.G[3 * g], Gy = a.G[3 * g + 1], Gz = a.G[3 * g + 2];
    sfac_store<LA, LB>(a, sp, g, Gx, Gy, Gz);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// rho[b] += sum_i F[b][i] Dt[i]: blockIdx.y = b, blockIdx.x = slice of the
// matrix (enough blocks per matrix to stream it at full bandwidth); rho must
// be zero on entry.
__global__ __launch_bounds__(256) void k_dot_batched(const double *F, const double *Dt, long n2, double *rho)
{
    __shared__ double sh[4];
    const double *f = F + (long)blockIdx.y * n2;
    double s = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x)
        s += f[i] * Dt[i];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(&rho[blockIdx.y], t);
}

__global__ __launch_bounds__(256) void k_dot(const double *A, const double *B, long n, double *out)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        s += A[i] * B[i];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) atomicAdd(out, t);
}

__global__ __launch_bounds__(256) void k_jlr(const double *F, const double *rho, const double *Gw, int ng, long n2,
                                            double *Jt)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    double s = 0.0;
    for (int g = 0; g < ng; ++g)
        s += (Gw ? Gw[g] : 1.0) * (F[(long)g * n2 + i] * rho[g] + F[(long)(ng + g) * n2 + i] * rho[ng + g]);
    Jt[i] += s;
}

// K[r][c] += sum_k P[k][r][c], k < nc (partial products of the split
// reduction), except in the block r >= bs, c < bs, which the partial
// products do not form.
__global__ __launch_bounds__(256) void k_sum_partials(const double *P, int nc, int n, int bs, double *K)
{
    const long n2 = (long)n * n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
        if (i / n >= bs && i % n < bs) continue;
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s += P[(long)c * n2 + i];
        K[i] += s;
    }
}

__global__ __launch_bounds__(256) void k_fill(double *p, long n, double v)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void k_axpy_scaled(double *Y, const double *X, long n, double f, const double *sdot)
{
    const double s = f * (*sdot);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        Y[i] += s * X[i];
}

// ---------------------------------------------------------------- density preparation
__global__ __launch_bounds__(256) void k_dtransform(DprepArgs a)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nc = a.nbfc;
    if (e >= nc * nc) return;
    int i = (int)(e / nc), j = (int)(e % nc);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int ai = a.tr_ao[2 * i + u];
        if (ai < 0) continue;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            int bj = a.tr_ao[2 * j + v];
            if (bj < 0) continue;
            s += a.tr_c[2 * i + u] * a.tr_c[2 * j + v] * a.D[(long)ai * a.nbf + bj];
        }
    }
    a.Dt[e] = s;
}

__global__ __launch_bounds__(256) void k_dmax(DprepArgs a)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int ns = a.nshell;
    if (e >= ns * ns) return;
    int A = e / ns, B = e % ns;
    int na = ncart(a.sh_l[A]), nb = ncart(a.sh_l[B]);
    double m = 0.0;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            int ii = a.sh_aoc[A] + i, jj = a.sh_aoc[B] + j;
            // block maxima of the unscaled Cartesian density
            double v = fabs(a.Dt[(long)ii * a.nbfc + jj] / (a.dscale[ii] * a.dscale[jj]));
            m = fmax(m, v);
        }
    a.Dmax[e] = m;
    atomicMax(a.dmax_glob, (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------- finalise
__global__ __launch_bounds__(256) void k_final(FinalArgs a)
{
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long nb = a.nbf, nc = a.nbfc;
    if (e >= nb * nb) return;
    int p = (int)(e / nb), q = (int)(e % nb);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        int i = a.inv_ci[3 * p + u];
        if (i < 0) continue;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            int j = a.inv_ci[3 * q + v];
            if (j < 0) continue;
            long jt = (long)i * nc + j;
            if (a.jt_block > 0 && i / a.jt_block > j / a.jt_block) jt = (long)j * nc + i;
            double x = a.X[(long)i * nc + j] + a.X[(long)j * nc + i] + (a.Jt ? a.Jt[jt] : 0.0);
            s += a.inv_cc[3 * p + u] * a.inv_cc[3 * q + v] * x;
        }
    }
    a.out[e] = s;
}

// ---------------------------------------------------------------- FP64 MFMA GEMM
// Block tile T x T (T = 64 or 128), four waves in a 2 x 2 arrangement, each
// owning a T/2 x T/2 sub-tile as (T/32) x (T/32) MFMA 16x16x4 accumulators;
// K staged through LDS in slabs of 16 with the next slab prefetched into
// registers.  Small tiles keep more workgroups resident per CU, which hides
// the barrier and load latency behind the other workgroups' matrix work.
// Operand layout of v_mfma_f64_16x16x4f64 (lane l): A[l & 15][l >> 4],
// B[l >> 4][l & 15]; result register r holds D[(l >> 4) + 4 r][l & 15].
constexpr int GBK = 16, GPAD = 2;

// ROLE (separate instantiations, so that profiles tell the roles apart):
// 0 plain (self term, dense exchange), 1 residual check of the density
// factor, 2 Y_b^T = L^T F_b, 3 K += sum_b Y_b Y_b^T (low-rank exchange).
template <int ROLE, int T>
__global__ __launch_bounds__(256) void k_dgemm(GemmArgs g)
{
    constexpr int VEC = T * GBK / 256;   // values staged per thread and operand
    constexpr int WT = T / 2;            // wave sub-tile edge
    constexpr int NF = WT / 16;          // MFMA tiles per wave and dimension
    __shared__ double As[GBK][T + GPAD];
    __shared__ double Bs[GBK][T + GPAD];
    int M = g.M, N = g.N, K = g.K;
    if (g.ctl_mode) {
        const int use_dense = g.ctl[1];
        if (g.ctl_mode == 3 ? !use_dense : use_dense) return;
        if (g.ctl_mode == 1) N = min(N, g.ctl[0]);
        if (g.ctl_mode == 2) K = min(K, g.ctl[0]);
        if (g.ctl_mode == 4) M = min(M, g.ctl[0]);
    }
    // persistent grid: each workgroup strides over the (tile column, tile
    // row, batch or slice) space sized by the host's upper bounds; skipped
    // tiles are uniform over the workgroup.  Consecutive workgroups (dealt
    // round-robin to the XCDs) take consecutive column tiles of one row tile:
    // the row panel of A is shared through every XCD's L2, and the column
    // panels of B spread over the memory channels.  (Grouping the row tiles
    // of one column panel on one XCD cut the L2 misses but ran the low-rank
    // products at 39 instead of 47 TFLOP/s.)
    const int nx = (g.N + T - 1) / T, ny = (g.M + T - 1) / T;
    const long nxy = (long)nx * ny, total = nxy * (g.reduce ? g.slices : g.nbatch);
    for (long vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int tx = (int)(vb % nx), ty = (int)((vb / nx) % ny), tz = (int)(vb / nxy);
    if (g.upper && ty > tx) continue;
    const int m0 = ty * T, n0 = tx * T;
    if (n0 >= N || m0 >= M) continue;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    int b0, b1;
    if (g.reduce) {
        int per = (g.nbatch + g.slices - 1) / g.slices;
        b0 = tz * per;
        b1 = min(g.nbatch, b0 + per);
    } else {
        b0 = tz;
        b1 = b0 + 1;
    }
    dbl4 acc[NF][NF];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    // staging maps: VEC consecutive values along the contiguous dimension
    const int am = tid / (GBK / VEC), ak = (tid % (GBK / VEC)) * VEC;     // A (m, k), k contiguous
    const int tak = tid / (T / VEC), tam = (tid % (T / VEC)) * VEC;      // A (m, k), m contiguous
    const int bk = tid / (T / VEC), bn = (tid % (T / VEC)) * VEC;        // B (k, n), n contiguous
    const int tn = tid / (GBK / VEC), tk = (tid % (GBK / VEC)) * VEC;    // B (k, n), k contiguous
    double ra[VEC], rb[VEC];
    const int nk = (K + GBK - 1) / GBK;
    for (int b = b0; b < b1; ++b) {
        const double *A = g.A + (long)b * g.sA;
        const double *B = g.B + (long)b * g.sB;
        const double alpha = (g.alpha ? g.alpha[b] : 1.0) * g.alpha0;
        auto load = [&](int kt) {
            const int k0 = kt * GBK;
            if (g.transA) {
                const int gk = k0 + tak;
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    int gm = m0 + tam + u;
                    ra[u] = (gm < M && gk < K) ? A[(long)gk * g.lda + gm] : 0.0;
                }
            } else {
                const int gm = m0 + am;
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    int gk = k0 + ak + u;
                    ra[u] = (gm < M && gk < K) ? A[(long)gm * g.lda + gk] : 0.0;
                }
            }
            if (g.transB) {
                const int gn = n0 + tn;
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    int gk2 = k0 + tk + u;
                    rb[u] = (gk2 < K && gn < N) ? B[(long)gn * g.ldb + gk2] : 0.0;
                }
            } else {
                const int gk = k0 + bk;
#pragma unroll
                for (int u = 0; u < VEC; ++u) {
                    int gn = n0 + bn + u;
                    rb[u] = (gk < K && gn < N) ? B[(long)gk * g.ldb + gn] : 0.0;
                }
            }
        };
        load(0);
        for (int kt = 0; kt < nk; ++kt) {
            __syncthreads();
            if (g.transA) {
#pragma unroll
                for (int u = 0; u < VEC; ++u) As[tak][tam + u] = alpha * ra[u];
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u) As[ak + u][am] = alpha * ra[u];
            }
            if (g.transB) {
#pragma unroll
                for (int u = 0; u < VEC; ++u) Bs[tk + u][tn] = rb[u];
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u) Bs[bk][bn + u] = rb[u];
            }
            __syncthreads();
            if (kt + 1 < nk) load(kt + 1);
#pragma unroll
            for (int kk = 0; kk < GBK; kk += 4) {
                double af[NF], bf[NF];
#pragma unroll
                for (int i = 0; i < NF; ++i) af[i] = As[kk + lk][wm * WT + i * 16 + lr];
#pragma unroll
                for (int j = 0; j < NF; ++j) bf[j] = Bs[kk + lk][wn * WT + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < NF; ++i)
#pragma unroll
                    for (int j = 0; j < NF; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
        }
        if (!g.reduce) {
            double *C = g.C + (long)b * g.sC;
#pragma unroll
            for (int i = 0; i < NF; ++i)
#pragma unroll
                for (int j = 0; j < NF; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        int gm = m0 + wm * WT + i * 16 + lk + 4 * r;
                        int gn = n0 + wn * WT + j * 16 + lr;
                        if (gm < M && gn < N) C[(long)gm * g.ldc + gn] = acc[i][j][r];
                    }
#pragma unroll
            for (int i = 0; i < NF; ++i)
#pragma unroll
                for (int j = 0; j < NF; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    }
    if (g.reduce && b1 > b0) {
#pragma unroll
        for (int i = 0; i < NF; ++i)
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int gm = m0 + wm * WT + i * 16 + lk + 4 * r;
                    int gn = n0 + wn * WT + j * 16 + lr;
                    if (gm < M && gn < N) atomicAdd(&g.C[(long)gm * g.ldc + gn], acc[i][j][r]);
                }
    }
    }
}

// ---------------------------------------------------------------- Y_b^T = L^T F_b, tall tiles
// The low-rank exchange products (C_b = A B_b with A the M x K factor rows,
// M the rank read from the control block).  One workgroup of eight
// wavefronts forms 64 columns of C_b for up to 512 rows, so that each F_b
// column panel is read once per 512 rows of the factor (64 x 64 tiles read it
// once per 64 rows).  The 16-row MFMA tiles are dealt to the wavefronts round
// robin (wavefront w takes tiles w, w + 8, w + 16, w + 24): the two
// wavefronts of a SIMD then carry about the same number.  K is staged in
// slabs of 16 through two LDS buffers: the next slab is loaded into
// registers while the current one is multiplied, and one barrier a slab
// separates the buffers' reads from their next writes.
constexpr int kYRows = 512, kYCols = 64, kYK = 16, kYThreads = 512;

__global__ __launch_bounds__(kYThreads) void k_ygemm(GemmArgs g)
{
    __shared__ double As[2][kYK][kYRows + GPAD];
    __shared__ double Bs[2][kYK][kYCols + GPAD];
    int M = g.M;
    if (g.ctl_mode) {
        if (g.ctl[1]) return;
        M = min(M, g.ctl[0]);
    }
    const int N = g.N, K = g.K;
    // grid: (column tile, row chunk, batch) from the host's upper bounds
    const int nx = (N + kYCols - 1) / kYCols, nch = (g.M + kYRows - 1) / kYRows;
    const long vb = blockIdx.x;
    const int tx = (int)(vb % nx), ch = (int)((vb / nx) % nch);
    const int b = (int)(vb / ((long)nx * nch));
    const int m0 = ch * kYRows, n0 = tx * kYCols;
    if (m0 >= M || b >= g.nbatch) return;
    const int rows = min(kYRows, M - m0);
    const int mt = (rows + 15) / 16;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int my = mt > wave ? (mt - wave + 7) / 8 : 0;   // this wavefront's m-tiles (<= 4)
    dbl4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const double *A = g.A;
    const double *B = g.B + (long)b * g.sB;
    // staging: thread t loads row m0 + t of the A slab (16 values along K)
    // and two neighbouring values of row t / 32 of the B slab
    double ra[kYK], rb[2];
    const int bk = tid >> 5, bn = 2 * (tid & 31);
    auto load = [&](int kt) {
        const int k0 = kt * kYK;
        if (tid < rows) {
            const double *src = A + (long)(m0 + tid) * g.lda + k0;
            if (k0 + kYK <= K) {
#pragma unroll
                for (int u = 0; u < kYK; ++u) ra[u] = src[u];
            } else {
#pragma unroll
                for (int u = 0; u < kYK; ++u) ra[u] = k0 + u < K ? src[u] : 0.0;
            }
        } else {
#pragma unroll
            for (int u = 0; u < kYK; ++u) ra[u] = 0.0;
        }
        const int gk = k0 + bk, gn = n0 + bn;
        rb[0] = (gk < K && gn < N) ? B[(long)gk * g.ldb + gn] : 0.0;
        rb[1] = (gk < K && gn + 1 < N) ? B[(long)gk * g.ldb + gn + 1] : 0.0;
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < kYK; ++u) As[buf][u][tid] = ra[u];
        Bs[buf][bk][bn] = rb[0];
        Bs[buf][bk][bn + 1] = rb[1];
    };
    const int nk = (K + kYK - 1) / kYK;
    load(0);
    stash(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load(kt + 1);
#pragma unroll
        for (int kk = 0; kk < kYK; kk += 4) {
            double bf[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][kk + lk][j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i < my) {
                    const double af = As[cur][kk + lk][(wave + 8 * i) * 16 + lr];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[j], acc[i][j], 0, 0, 0);
                }
            }
        }
        if (kt + 1 < nk) stash(cur ^ 1);
        __syncthreads();
    }
    double *C = g.C + (long)b * g.sC;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= my) break;
        const int rt = m0 + (wave + 8 * i) * 16;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = rt + lk + 4 * r, gn = n0 + j * 16 + lr;
                if (gm < M && gn < N) C[(long)gm * g.ldc + gn] = g.alpha0 * acc[i][j][r];
            }
    }
}

// ---------------------------------------------------------------- pivoted Cholesky
// Step k: every block reduces the per-block maxima of the remaining diagonal
// left by step k - 1 to the pivot p, then forms rows [64 b, 64 b + 64) of
// column k, L_ik = (D_ip - sum_{j<k} L_ij L_pj) / sqrt(d_p), and the new
// remaining diagonal d_i -= L_ik^2, with its block maximum for step k + 1.
// Work layout: diag[n] | pv[2][nblk] | stop, max0; wi: pi[2][nblk].
constexpr int kCholRows = 64;
constexpr int kCholSingleMax = 256;    // one-workgroup factorisation up to this n

__device__ inline void argmax_merge(double &v, int &i, double ov, int oi)
{
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

__global__ __launch_bounds__(1024) void k_pchol_init(const double *D, int n, double tol, double *work, int *wi,
                                                    int *ctl)
{
    __shared__ double sm[16], sn[16];
    const int nblk = (n + kCholRows - 1) / kCholRows;
    double *diag = work, *pv = work + n, *par = work + n + 2 * nblk;
    int *pi = wi;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, nw = blockDim.x >> 6;
    double mx = 0.0, mn = 0.0;
    for (int i = tid; i < n; i += blockDim.x) {
        const double d = D[(long)i * n + i];
        diag[i] = d;
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off, 64));
        mn = fmin(mn, __shfl_xor(mn, off, 64));
    }
    if (l == 0) { sm[w] = mx; sn[w] = mn; }
    __syncthreads();
    mx = 0.0; mn = 0.0;
    for (int u = 0; u < nw; ++u) { mx = fmax(mx, sm[u]); mn = fmin(mn, sn[u]); }
    // block maxima of the diagonal for step 0
    for (int b = w; b < nblk; b += nw) {
        const int i = b * kCholRows + l;
        double v = i < n ? diag[i] : -1e300;
        int ii = i;
        for (int off = 32; off > 0; off >>= 1) argmax_merge(v, ii, __shfl_xor(v, off, 64), __shfl_xor(ii, off, 64));
        if (l == 0) { pv[b] = v; pi[b] = ii; }
    }
    if (tid == 0) {
        par[0] = tol * mx;
        par[1] = mx;
        ctl[0] = 0;
        ctl[1] = (mn < -tol * mx) ? 1 : 0;
        ctl[2] = (mx > 0.0) ? 0 : 1;
        ctl[3] = 0;
    }
}

// One workgroup of four wavefronts per 64 rows: the dot products over the
// previous columns are split over the wavefronts, four independent loads in
// flight each, so that a step waits on about k / 16 L2 round trips.
constexpr int kCholWaves = 4;

__global__ __launch_bounds__(64 * kCholWaves) void k_pchol_step(const double *D, int n, int k, double *L,
                                                               double *work, int *wi, int *ctl)
{
    __shared__ double sred[kCholWaves][kCholRows];
    __shared__ double s_piv;
    __shared__ int s_p, s_done;
    if (threadIdx.x == 0) s_done = ctl[2];
    __syncthreads();
    if (s_done) return;
    const int nblk = (n + kCholRows - 1) / kCholRows;
    double *diag = work, *par = work + n + 2 * nblk;
    const double *pv_in = work + n + (k & 1) * nblk;
    double *pv_out = work + n + ((k + 1) & 1) * nblk;
    const int *pi_in = wi + (k & 1) * nblk;
    int *pi_out = wi + ((k + 1) & 1) * nblk;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    if (w == 0) {
        double v = -1e300;
        int ii = 0x7fffffff;
        for (int b = l; b < nblk; b += 64) argmax_merge(v, ii, pv_in[b], pi_in[b]);
        for (int off = 32; off > 0; off >>= 1) argmax_merge(v, ii, __shfl_xor(v, off, 64), __shfl_xor(ii, off, 64));
        if (l == 0) { s_piv = v; s_p = ii; }
    }
    __syncthreads();
    const double piv = s_piv;
    const int p = s_p;
    if (!(piv > par[0])) {
        if (blockIdx.x == 0 && tid == 0) { ctl[0] = k; ctl[2] = 1; }
        return;
    }
    const int i = blockIdx.x * kCholRows + l;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < n) {
        constexpr int W = kCholWaves;
        int j = w;
        for (; j + 3 * W < k; j += 4 * W) {
            s0 += L[(long)j * n + i] * L[(long)j * n + p];
            s1 += L[(long)(j + W) * n + i] * L[(long)(j + W) * n + p];
            s2 += L[(long)(j + 2 * W) * n + i] * L[(long)(j + 2 * W) * n + p];
            s3 += L[(long)(j + 3 * W) * n + i] * L[(long)(j + 3 * W) * n + p];
        }
        for (; j < k; j += W) s0 += L[(long)j * n + i] * L[(long)j * n + p];
    }
    sred[w][l] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (w == 0) {
        double v = -1e300;
        if (i < n) {
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < kCholWaves; ++u) s += sred[u][l];
            const double x = (D[(long)p * n + i] - s) / sqrt(piv);
            L[(long)k * n + i] = x;
            const double d = (i == p) ? 0.0 : diag[i] - x * x;
            diag[i] = d;
            v = d;
        }
        int ii = i;
        for (int off = 32; off > 0; off >>= 1) argmax_merge(v, ii, __shfl_xor(v, off, 64), __shfl_xor(ii, off, 64));
        if (l == 0) { pv_out[blockIdx.x] = v; pi_out[blockIdx.x] = ii; }
    }
}

// Blocked form (right-looking): panels of kCholPanel columns.  One workgroup
// takes the panel's columns one after the other from the trailing matrix A
// (D minus the outer products of all earlier panels): pivot p = the largest
// remaining diagonal entry, L_ki = (A_pi - sum over the panel's earlier
// columns j of L_ji L_jp) / sqrt(d_p), d_i -= L_ki^2.  Each thread owns rows
// tid + 512 q and keeps, in registers, their remaining diagonal and their
// values in the panel's columns; the pivot row's values reach the other
// threads through LDS from the thread that owns it, so a step reads only the
// pivot row of A from memory.  Then k_pchol_update subtracts the panel's
// outer products from the trailing matrix.  Same columns as the
// one-launch-per-column steps, up to the order of the sums.
constexpr int kCholPanel = 16;
constexpr int kCholPanelThreads = 512;
constexpr int kCholPanelRows = 4;      // rows per thread
// Larger matrices take the per-column steps: there the trailing updates (a
// pass over the n x n matrix per panel) cost more than the launches saved.
constexpr int kCholPanelMaxN = kCholPanelRows * kCholPanelThreads;

__global__ __launch_bounds__(kCholPanelThreads) void k_pchol_panel(const double *A, int n, int k0, int kend,
                                                                  double *L, double *work, int *ctl)
{
    constexpr int T = kCholPanelThreads, NW = T / 64, R = kCholPanelRows, P = kCholPanel;
    __shared__ double s_v[NW];
    __shared__ int s_i[NW];
    __shared__ double s_lp[P];
    __shared__ double s_piv;
    __shared__ int s_p, s_done;
    if (threadIdx.x == 0) s_done = ctl[2];
    __syncthreads();
    if (s_done) return;
    const int nblk = (n + kCholRows - 1) / kCholRows;
    double *diag = work;
    const double stop = work[n + 2 * nblk];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    double d[R], pl[R][P];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int i = tid + q * T;
        d[q] = i < n ? diag[i] : -1e300;
#pragma unroll
        for (int t = 0; t < P; ++t) pl[q][t] = 0.0;
    }
    int k = k0;
    bool stopped = false;
    for (; k < kend; ++k) {
        double bv = -1e300;
        int bi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int i = tid + q * T;
            if (i < n) argmax_merge(bv, bi, d[q], i);
        }
        for (int off = 32; off > 0; off >>= 1) argmax_merge(bv, bi, __shfl_xor(bv, off, 64), __shfl_xor(bi, off, 64));
        if (l == 0) { s_v[w] = bv; s_i[w] = bi; }
        __syncthreads();
        if (tid == 0) {
            double t = s_v[0];
            int ti = s_i[0];
            for (int u = 1; u < NW; ++u) argmax_merge(t, ti, s_v[u], s_i[u]);
            s_piv = t;
            s_p = ti;
        }
        __syncthreads();
        const double piv = s_piv;
        const int p = s_p;
        if (!(piv > stop)) {
            stopped = true;
            break;
        }
        const int kk = k - k0;
        // the pivot row's panel values (zero beyond column kk) from its owner
        if (tid == p % T) {
            const int qp = p / T;
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (q == qp)
#pragma unroll
                    for (int t = 0; t < P; ++t) s_lp[t] = pl[q][t];
        }
        __syncthreads();
        const double inv = 1.0 / sqrt(piv);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int i = tid + q * T;
            if (i < n) {
                double v0 = A[(long)p * n + i], v1 = 0.0;
#pragma unroll
                for (int t = 0; t < P; t += 2) {
                    v0 -= pl[q][t] * s_lp[t];
                    v1 -= pl[q][t + 1] * s_lp[t + 1];
                }
                const double x = (v0 + v1) * inv;
                L[(long)k * n + i] = x;
#pragma unroll
                for (int t = 0; t < P; ++t)
                    if (t == kk) pl[q][t] = x;
                d[q] = (i == p) ? 0.0 : d[q] - x * x;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int i = tid + q * T;
        if (i < n) diag[i] = d[q];
    }
    if (stopped && tid == 0) {
        ctl[0] = k;
        ctl[2] = 1;
    }
}

// dst = src - sum_{k0 <= j < k0 + kb} L_j L_j^T (full matrix, 64 x 64 tiles,
// 4 x 4 outputs a thread); nothing once the factor has stopped.
__global__ __launch_bounds__(256) void k_pchol_update(const double *src, double *dst, int n, int k0, int kb,
                                                     const double *L, const int *ctl)
{
    __shared__ double Li[kCholPanel][64], Lj[kCholPanel][64];
    if (ctl[2]) return;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    for (int e = tid; e < kb * 64; e += 256) {
        const int t = e >> 6, c = e & 63;
        Li[t][c] = i0 + c < n ? L[(long)(k0 + t) * n + i0 + c] : 0.0;
        Lj[t][c] = j0 + c < n ? L[(long)(k0 + t) * n + j0 + c] : 0.0;
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            acc[a][b] = (i < n && j < n) ? src[(long)i * n + j] : 0.0;
        }
    for (int t = 0; t < kb; ++t) {
        double x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = Li[t][ty * 4 + a];
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = Lj[t][tx * 4 + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] -= x[a] * y[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            if (i < n && j < n) dst[(long)i * n + j] = acc[a][b];
        }
}

// After the last step: rank = rmax when the factor did not stop by itself;
// use_dense when it did not converge or a remaining diagonal entry is below
// -tol * max diag.
__global__ __launch_bounds__(256) void k_pchol_fin(int n, int rmax, const double *work, const int *wi, int *ctl)
{
    __shared__ int s_bad;
    const int nblk = (n + kCholRows - 1) / kCholRows;
    const double *diag = work, *par = work + n + 2 * nblk;
    const double stop = par[0];
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const bool done = ctl[2] != 0;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = diag[i];
        if (d < -stop || (!done && d > stop)) bad = 1;
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!done) { ctl[0] = rmax; ctl[2] = 1; }
        if (s_bad) ctl[1] = 1;
    }
}

// The whole factorisation in one workgroup (for small n, where one launch per
// column would be launch-bound).  Same outputs as init + steps + fin.
__global__ __launch_bounds__(1024) void k_pchol_single(const double *D, int n, double tol, int rmax, double *L,
                                                      double *work, int *ctl)
{
    __shared__ double sv[16];
    __shared__ int si[16];
    __shared__ double s_mx, s_mn, s_piv;
    __shared__ int s_p, s_bad;
    const int nblk = (n + kCholRows - 1) / kCholRows;
    double *diag = work, *par = work + n + 2 * nblk;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, nw = blockDim.x >> 6;
    double mx = 0.0, mn = 0.0;
    for (int i = tid; i < n; i += blockDim.x) {
        const double d = D[(long)i * n + i];
        diag[i] = d;
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off, 64));
        mn = fmin(mn, __shfl_xor(mn, off, 64));
    }
    if (l == 0) sv[w] = mx;
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        for (int u = 0; u < nw; ++u) a = fmax(a, sv[u]);
        s_mx = a;
        s_bad = 0;
    }
    __syncthreads();
    if (l == 0) sv[w] = mn;
    __syncthreads();
    if (tid == 0) {
        double b = 0.0;
        for (int u = 0; u < nw; ++u) b = fmin(b, sv[u]);
        s_mn = b;
    }
    __syncthreads();
    const double max0 = s_mx, stop = tol * max0;
    int k = 0;
    bool stopped = !(max0 > 0.0);
    for (; k < rmax && !stopped; ++k) {
        double bv = -1e300;
        int bi = 0x7fffffff;
        for (int i = tid; i < n; i += blockDim.x) argmax_merge(bv, bi, diag[i], i);
        for (int off = 32; off > 0; off >>= 1) argmax_merge(bv, bi, __shfl_xor(bv, off, 64), __shfl_xor(bi, off, 64));
        if (l == 0) { sv[w] = bv; si[w] = bi; }
        __syncthreads();
        if (tid == 0) {
            double t = sv[0];
            int ti = si[0];
            for (int u = 1; u < nw; ++u) argmax_merge(t, ti, sv[u], si[u]);
            s_piv = t;
            s_p = ti;
        }
        __syncthreads();
        const double piv = s_piv;
        const int p = s_p;
        if (!(piv > stop)) {
            stopped = true;
            break;
        }
        const double inv = 1.0 / sqrt(piv);
        for (int i = tid; i < n; i += blockDim.x) {
            double v = D[(long)p * n + i];
            for (int j = 0; j < k; ++j) v -= L[(long)j * n + i] * L[(long)j * n + p];
            v *= inv;
            L[(long)k * n + i] = v;
            diag[i] = (i == p) ? 0.0 : diag[i] - v * v;
        }
        __syncthreads();
    }
    int bad = 0;
    for (int i = tid; i < n; i += blockDim.x) {
        const double d = diag[i];
        if (d < -stop || (!stopped && d > stop)) bad = 1;
    }
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (tid == 0) {
        par[0] = stop;
        par[1] = max0;
        ctl[0] = k;
        ctl[1] = (s_bad || s_mn < -stop) ? 1 : 0;
        ctl[2] = 1;
        ctl[3] = 0;
    }
}

__global__ __launch_bounds__(256) void k_lowrank_check(const double *D, const double *R, int n, const double *work,
                                                      int *ctl)
{
    if (ctl[1]) return;
    const int nblk = (n + kCholRows - 1) / kCholRows;
    const double *par = work + n + 2 * nblk;
    const double thr = 2.0 * par[0] + 4.0 * n * 2.220446049250313e-16 * par[1];
    const long n2 = (long)n * n;
    int bad = 0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += (long)gridDim.x * blockDim.x)
        if (!(fabs(D[e] - R[e]) <= thr)) bad = 1;
    if (bad) atomicOr(&ctl[1], 1);
}

}  // namespace

hipError_t launch_pchol(const double *D, int n, double tol, int rmax, double *L, double *work, int *wi,
                        int *ctl, double *Aw, hipStream_t st)
{
    const int nblk = (n + kCholRows - 1) / kCholRows;
    if (n <= kCholSingleMax) {
        hipLaunchKernelGGL(k_pchol_single, dim3(1), dim3(1024), 0, st, D, n, tol, rmax, L, work, ctl);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pchol_init, dim3(1), dim3(1024), 0, st, D, n, tol, work, wi, ctl);
    if (Aw && n <= kCholPanelMaxN) {
        // panels: the trailing matrix lives in Aw (D itself for the first panel)
        const int nt = (n + 63) / 64;
        for (int k0 = 0; k0 < rmax; k0 += kCholPanel) {
            const int kb = std::min(kCholPanel, rmax - k0);
            hipLaunchKernelGGL(k_pchol_panel, dim3(1), dim3(kCholPanelThreads), 0, st, k0 == 0 ? D : (const double *)Aw,
                               n, k0, k0 + kb, L, work, ctl);
            if (k0 + kb < rmax)
                hipLaunchKernelGGL(k_pchol_update, dim3(nt, nt), dim3(256), 0, st, k0 == 0 ? D : (const double *)Aw, Aw,
                                   n, k0, kb, (const double *)L, (const int *)ctl);
        }
        hipLaunchKernelGGL(k_pchol_fin, dim3(1), dim3(256), 0, st, n, rmax, (const double *)work, (const int *)wi, ctl);
        return hipGetLastError();
    }
    // every column up to rmax is queued; the steps after the stop return at
    // their first instruction (the caller keeps rmax near the expected rank)
    for (int k = 0; k < rmax; ++k)
        hipLaunchKernelGGL(k_pchol_step, dim3(nblk), dim3(64 * kCholWaves), 0, st, D, n, k, L, work, wi, ctl);
    hipLaunchKernelGGL(k_pchol_fin, dim3(1), dim3(256), 0, st, n, rmax, (const double *)work, (const int *)wi, ctl);
    return hipGetLastError();
}

hipError_t launch_lowrank_check(const double *D, const double *R, int n, const double *work, int *ctl,
                                hipStream_t st)
{
    const long n2 = (long)n * n;
    const unsigned blocks = (unsigned)std::min<long>(2048, (n2 + 255) / 256);
    hipLaunchKernelGGL(k_lowrank_check, dim3(std::max(1u, blocks)), dim3(256), 0, st, D, R, n, work, ctl);
    return hipGetLastError();
}

hipError_t launch_sfac(int cls, const SfacArgs &a, hipStream_t st)
{
    if (a.nsp <= 0 || a.ng <= 0) return hipSuccess;
    dim3 grid((a.ng + 63) / 64, a.nsp), block(64);
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_sfac<0, 0>), grid, block, 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_sfac<1, 0>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_sfac<1, 1>), grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_sfac<2, 0>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_sfac<2, 1>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((k_sfac<2, 2>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_dot_batched(const double *F, const double *Dt, int n2, int nb, double *rho, hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    hipError_t e = launch_fill(rho, nb, 0.0, st);
    if (e != hipSuccess) return e;
    // about 2048 blocks in all, at most one per 256 x 16 elements of a matrix
    const long per = std::max(1L, std::min<long>((n2 + 4095) / 4096, (2048 + nb - 1) / nb));
    hipLaunchKernelGGL(k_dot_batched, dim3((unsigned)per, nb), dim3(256), 0, st, F, Dt, (long)n2, rho);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *P, int nc, int n, int bs, double *K, hipStream_t st)
{
    const long n2 = (long)n * n;
    if (nc <= 0 || n2 <= 0) return hipSuccess;
    const long blocks = std::min<long>(4096, (n2 + 255) / 256);
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)blocks), dim3(256), 0, st, P, nc, n, bs, K);
    return hipGetLastError();
}

hipError_t launch_jlr(const double *F, const double *rho, const double *Gw, int ng, int n2, double *Jt,
                      hipStream_t st)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jlr, dim3((n2 + 255) / 256), dim3(256), 0, st, F, rho, Gw, ng, (long)n2, Jt);
    return hipGetLastError();
}

// Workgroups of the persistent grid of device-gated products.
constexpr long kGemmGrid = 1024;

template <int T>
hipError_t launch_dgemm_t(const GemmArgs &a, hipStream_t st)
{
    const long z = a.reduce ? a.slices : a.nbatch;
    const long tiles = (long)((a.N + T - 1) / T) * ((a.M + T - 1) / T) * z;
    // one tile per workgroup, except for products that run only when the
    // device-side decision falls back to them: a capped persistent grid, so
    // that the usual case (gated off) costs few workgroups
    dim3 grid((unsigned)(a.ctl_mode == 3 ? std::min(tiles, kGemmGrid) : tiles));
    switch (a.role) {
        case 1: hipLaunchKernelGGL((k_dgemm<1, T>), grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_dgemm<2, T>), grid, dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_dgemm<3, T>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_dgemm<0, T>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_ygemm(const GemmArgs &a, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0 || a.nbatch <= 0) return hipSuccess;
    if (a.transA || a.transB || a.reduce || a.upper || a.alpha || (a.ctl_mode != 0 && a.ctl_mode != 4))
        return hipErrorInvalidValue;
    const long blocks = (long)((a.N + kYCols - 1) / kYCols) * ((a.M + kYRows - 1) / kYRows) * a.nbatch;
    hipLaunchKernelGGL(k_ygemm, dim3((unsigned)blocks), dim3(kYThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dgemm(const GemmArgs &a, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0 || a.nbatch <= 0) return hipSuccess;
    // products that write the upper tiles of K use the K block size
    const int t = (a.upper || a.tile == 0) ? kGemmTile : a.tile;
    return t == 64 ? launch_dgemm_t<64>(a, st) : launch_dgemm_t<128>(a, st);
}

hipError_t launch_fill(double *p, long n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_dprep(const DprepArgs &a, hipStream_t st)
{
    long n2 = (long)a.nbfc * a.nbfc;
    hipLaunchKernelGGL(k_dtransform, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ns2 = a.nshell * a.nshell;
    hipLaunchKernelGGL(k_dmax, dim3((ns2 + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dot(const double *A, const double *B, long n, double *out, hipStream_t st)
{
    long blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_dot, dim3((unsigned)blocks), dim3(256), 0, st, A, B, n, out);
    return hipGetLastError();
}

hipError_t launch_axpy_scaled(double *Y, const double *X, long n, double f, const double *sdot, hipStream_t st)
{
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_axpy_scaled, dim3((unsigned)blocks), dim3(256), 0, st, Y, X, n, f, sdot);
    return hipGetLastError();
}

hipError_t launch_final(const FinalArgs &a, hipStream_t st)
{
    long n2 = (long)a.nbf * a.nbf;
    hipLaunchKernelGGL(k_final, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace pbcjk
