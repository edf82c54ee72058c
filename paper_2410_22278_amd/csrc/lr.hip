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
        const double ip = 1.0 / P.p;
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

__global__ __launch_bounds__(256) void k_dot_batched(const double *F, const double *Dt, long n2, double *rho)
{
    __shared__ double sh[4];
    const double *f = F + (long)blockIdx.x * n2;
    double s = 0.0;
    for (long i = threadIdx.x; i < n2; i += blockDim.x) s += f[i] * Dt[i];
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) rho[blockIdx.x] = t;
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
        s += Gw[g] * (F[(long)g * n2 + i] * rho[g] + F[(long)(ng + g) * n2 + i] * rho[ng + g]);
    Jt[i] += s;
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
            double x = a.X[(long)i * nc + j] + a.X[(long)j * nc + i] + a.Jt[(long)i * nc + j];
            s += a.inv_cc[3 * p + u] * a.inv_cc[3 * q + v] * x;
        }
    }
    a.out[e] = s;
}

// ---------------------------------------------------------------- FP64 MFMA GEMM
// Block tile 128 x 128, four waves in a 2 x 2 arrangement, each owning a
// 64 x 64 sub-tile as 4 x 4 MFMA 16x16x4 accumulators; K staged through LDS
// in slabs of 16 with the next slab prefetched into registers.
// Operand layout of v_mfma_f64_16x16x4f64 (lane l): A[l & 15][l >> 4],
// B[l >> 4][l & 15]; result register r holds D[(l >> 4) + 4 r][l & 15].
constexpr int GBM = 128, GBN = 128, GBK = 16, GPAD = 2;

__global__ __launch_bounds__(256) void k_dgemm(GemmArgs g)
{
    __shared__ double As[GBK][GBM + GPAD];
    __shared__ double Bs[GBK][GBN + GPAD];
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    int b0, b1;
    if (g.reduce) {
        int per = (g.nbatch + g.slices - 1) / g.slices;
        b0 = blockIdx.z * per;
        b1 = min(g.nbatch, b0 + per);
    } else {
        b0 = blockIdx.z;
        b1 = b0 + 1;
    }
    dbl4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    // each thread stages 8 A values (one row, 8 consecutive k) and 8 B values
    const int am = tid >> 1, ak = (tid & 1) * 8;
    const int bk = tid >> 4, bn = (tid & 15) * 8;
    double ra[8], rb[8];
    const int nk = (g.K + GBK - 1) / GBK;
    for (int b = b0; b < b1; ++b) {
        const double *A = g.A + (long)b * g.sA;
        const double *B = g.B + (long)b * g.sB;
        const double alpha = (g.alpha ? g.alpha[b] : 1.0) * g.alpha0;
        auto load = [&](int kt) {
            const int k0 = kt * GBK;
            const int gm = m0 + am;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                int gk = k0 + ak + u;
                ra[u] = (gm < g.M && gk < g.K) ? A[(long)gm * g.lda + gk] : 0.0;
            }
            const int gk = k0 + bk;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                int gn = n0 + bn + u;
                rb[u] = (gk < g.K && gn < g.N) ? B[(long)gk * g.ldb + gn] : 0.0;
            }
        };
        load(0);
        for (int kt = 0; kt < nk; ++kt) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u) As[ak + u][am] = alpha * ra[u];
#pragma unroll
            for (int u = 0; u < 8; ++u) Bs[bk][bn + u] = rb[u];
            __syncthreads();
            if (kt + 1 < nk) load(kt + 1);
#pragma unroll
            for (int kk = 0; kk < GBK; kk += 4) {
                double af[4], bf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) af[i] = As[kk + lk][wm * 64 + i * 16 + lr];
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[j] = Bs[kk + lk][wn * 64 + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
        }
        if (!g.reduce) {
            double *C = g.C + (long)b * g.sC;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        int gm = m0 + wm * 64 + i * 16 + lk + 4 * r;
                        int gn = n0 + wn * 64 + j * 16 + lr;
                        if (gm < g.M && gn < g.N) C[(long)gm * g.ldc + gn] = acc[i][j][r];
                    }
        }
    }
    if (g.reduce && b1 > b0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    int gm = m0 + wm * 64 + i * 16 + lk + 4 * r;
                    int gn = n0 + wn * 64 + j * 16 + lr;
                    if (gm < g.M && gn < g.N) atomicAdd(&g.C[(long)gm * g.ldc + gn], acc[i][j][r]);
                }
    }
}

}  // namespace

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
    hipLaunchKernelGGL(k_dot_batched, dim3(nb), dim3(256), 0, st, F, Dt, (long)n2, rho);
    return hipGetLastError();
}

hipError_t launch_jlr(const double *F, const double *rho, const double *Gw, int ng, int n2, double *Jt,
                      hipStream_t st)
{
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jlr, dim3((n2 + 255) / 256), dim3(256), 0, st, F, rho, Gw, ng, (long)n2, Jt);
    return hipGetLastError();
}

hipError_t launch_dgemm(const GemmArgs &a, hipStream_t st)
{
    if (a.M <= 0 || a.N <= 0 || a.K <= 0 || a.nbatch <= 0) return hipSuccess;
    int z = a.reduce ? a.slices : a.nbatch;
    dim3 grid((a.N + GBN - 1) / GBN, (a.M + GBM - 1) / GBM, z);
    hipLaunchKernelGGL(k_dgemm, grid, dim3(256), 0, st, a);
    return hipGetLastError();
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
