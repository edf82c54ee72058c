// Neighbour lists of (shell pair, image) groups for the real-space sum.
//
// Built once per cell.  A group pair is kept iff some primitive quartet of
// it has a lattice shift R1 inside its real-space sphere (Sec. 2.4, eq.
// pbc_eri_real_cutoff_implementation); that does not depend on the density,
// so the per-build density-weighted screen is applied afterwards.  A cheap
// rigorous group-level test runs first: with the separable bound
// C2e (1 - c) <= Z_bra Z_ket, every sphere of the group pair has radius at
// most sqrt((1/p_min + 1/q_min + 1/w^2) ln(Z Z/delta)), and every pair
// centre lies within `ext` of its group centre.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "kernels.h"

namespace pbcjk {

namespace {

__device__ bool group_pair_test(const NbrArgs &a, const GroupRec &gb, const GroupRec &gk)
{
    const double zz = gb.Zmax * gk.Zmax;
    if (!(zz > a.d_ewald_R)) return false;
    double rad = sqrt((1.0 / gb.pmin + 1.0 / gk.pmin + 1.0 / a.w2) * log(zz / a.d_ewald_R));
    if (a.rcap2 > 0) rad = fmin(rad, sqrt(a.rcap2));
    const double R = (rad + gb.ext + gk.ext) * (1.0 + 1e-9) + 1e-9;
    const double cen[3] = {gb.C[0] - gk.C[0], gb.C[1] - gk.C[1], gb.C[2] - gk.C[2]};
    bool any = false;
    for_images(a.lat, cen, R * R, 0.0, [&](const double *, double) { any = true; });
    return any;
}

__device__ bool group_pair_has_term(const NbrArgs &a, const GroupRec &gb, const GroupRec &gk)
{
    for (int pb = gb.pstart; pb < gb.pend; ++pb) {
        const PairRec Pb = a.pairs[pb];
        for (int pk = gk.pstart; pk < gk.pend; ++pk) {
            const PairRec Pk = a.pairs[pk];
            double rad2;
            if (!quartet_sphere(Pb, Pk, a.w2, a.d_ewald_R, rad2)) continue;
            const double cen[3] = {Pb.P[0] - Pk.P[0], Pb.P[1] - Pk.P[1], Pb.P[2] - Pk.P[2]};
            bool any = false;
            for_images(a.lat, cen, rad2, a.rcap2, [&](const double *, double) { any = true; });
            if (any) return true;
        }
    }
    return false;
}

// Distance bucket of a group pair: |C_b - C_k - R| for the rounded translate R.
__device__ __forceinline__ int nbr_bucket(const NbrArgs &a, const GroupRec &gb, const GroupRec &gk)
{
    const double x[3] = {gb.C[0] - gk.C[0], gb.C[1] - gk.C[1], gb.C[2] - gk.C[2]};
    double n[3], L[3];
    nearest_translate(a.lat, x, n);
    lat_image(a.lat, x, n[0], n[1], n[2], L);
    const double t = sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]) * a.inv_bw;
    return t < (double)(kNbrBuckets - 1) ? (int)t : kNbrBuckets - 1;
}

// One wavefront per bra group.  Lane b < kNbrBuckets keeps bucket b's count
// (mode 0) or its next write position (mode 1).
__global__ __launch_bounds__(256) void k_nbr(NbrArgs a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi = blockIdx.x * (blockDim.x >> 6) + wave;
    if (bi >= a.nb) return;
    const GroupRec gb = a.groups[a.gb0 + bi];
    const int jlo = a.tri ? bi : 0;
    long mine = (a.mode && lane < kNbrBuckets) ? a.offsets[(long)bi * kNbrBuckets + lane] : 0;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int j0 = jlo; j0 < a.nk; j0 += 64) {
        const int j = j0 + lane;
        bool keep = false;
        int bk = 0;
        if (j < a.nk) {
            const GroupRec gk = a.groups[a.gk0 + j];
            keep = group_pair_test(a, gb, gk) && group_pair_has_term(a, gb, gk);
            if (keep) bk = nbr_bucket(a, gb, gk);
        }
        if (__ballot(keep) == 0) continue;
        for (int b = 0; b < kNbrBuckets; ++b) {
            const unsigned long long m = __ballot(keep && bk == b);
            if (m == 0) continue;
            // read with every lane active: lane b need not be among the writers
            const long start = __shfl(mine, b, 64);
            if (a.mode && keep && bk == b) {
                const long pos = start + __popcll(m & below);
                a.out_bra[pos] = bi;
                a.out_ket[pos] = j;
            }
            if (lane == b) mine += __popcll(m);
        }
    }
    if (!a.mode && lane < kNbrBuckets) a.counts[(long)bi * kNbrBuckets + lane] = (int)mine;
}

// Screen flags of one entry: bit 0 keep in FP64, bit 1 keep in FP32.
// 0: no quartet of the entry passes the density-weighted screen; 1: FP64
// list; 2: FP32 list.  An entry goes to FP32 when its bound is below
// fp32_below and every quartet has rho T >= 1 for every lattice shift, so
// that no short-range Boys value of the FP32 kernels falls in the
// small-argument region (which stays FP64): rho >= rho_min of the two
// groups' smallest exponent sums, and |P - Q - R1| >= d - ext_b - ext_k
// with d a lower bound on the distance from the group centres' difference
// to the lattice, min(|x - R0|, R_min - |x - R0|) for its rounded image R0
// (any other translate R has |x - R| >= |R - R0| - |x - R0| >= R_min -
// |x - R0|).
__device__ __forceinline__ int entry_class(const PartArgs &a, long e)
{
    const GroupRec &gb = a.groups[a.gb0 + a.bra[e]];
    const GroupRec &gk = a.groups[a.gk0 + a.ket[e]];
    const int ns = a.nshell;
    const int A = gb.shA, B = gb.shB, C = gk.shA, D = gk.shB;
    double wD = a.Dmax[A * ns + B];
    wD = fmax(wD, a.Dmax[C * ns + D]);
    wD = fmax(wD, a.Dmax[A * ns + C]);
    wD = fmax(wD, a.Dmax[A * ns + D]);
    wD = fmax(wD, a.Dmax[B * ns + C]);
    wD = fmax(wD, a.Dmax[B * ns + D]);
    const double bound = gb.Qmax * gk.Qmax * wD;
    if (!(bound > a.d_schwarz)) return 0;
    if (!(a.split && bound < a.fp32_below)) return 1;
    const double x[3] = {gb.C[0] - gk.C[0], gb.C[1] - gk.C[1], gb.C[2] - gk.C[2]};
    double n[3], L[3];
    nearest_translate(a.lat, x, n);
    lat_image(a.lat, x, n[0], n[1], n[2], L);
    const double d0 = sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    const double dmin = fmax(0.0, fmin(d0, a.lat.Rmin - d0) - gb.ext - gk.ext);
    const double rho_min = gb.pmin * gk.pmin / (gb.pmin + gk.pmin);
    // a relative margin covers the rounding of these bounds
    return rho_min * dmin * dmin * (1.0 - 1e-9) >= 1.0 ? 2 : 1;
}

// Order-preserving split of a class pair's neighbour list into the FP64 and
// FP32 work lists, in three launches: entry counts per chunk of
// kPartChunk entries, an exclusive scan of those counts, then the scatter,
// each chunk writing from its scanned offsets in list order.  The lists so
// keep the bra order of the neighbour list, and a wavefront of the build
// kernels mostly shares one bra group.
__device__ __forceinline__ int block_sum_256(int v, int *s4)
{
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (l == 0) s4[w] = v;
    __syncthreads();
    const int t = s4[0] + s4[1] + s4[2] + s4[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_part_count(PartArgs a, long long *cc)
{
    __shared__ int s4[4];
    const int tid = threadIdx.x;
    const long nch = (a.n + kPartChunk - 1) / kPartChunk;
    for (long c = blockIdx.x; c < nch; c += gridDim.x) {
        int c64 = 0, c32 = 0;
        for (int r = 0; r < kPartChunk / 256; ++r) {
            const long e = c * kPartChunk + r * 256 + tid;
            const int f = e < a.n ? entry_class(a, e) : 0;
            c64 += f == 1;
            c32 += f == 2;
        }
        const int t64 = block_sum_256(c64, s4);
        const int t32 = block_sum_256(c32, s4);
        if (tid == 0) {
            cc[2 * c] = t64;
            cc[2 * c + 1] = t32;
        }
    }
}

// One workgroup: in-place exclusive scan of the two interleaved count
// sequences; the totals go to counts[0] (FP64 list) and counts[1] (FP32).
__global__ __launch_bounds__(1024) void k_part_scan(long long *cc, long nch, unsigned long long *counts)
{
    __shared__ long long s[2][16];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    long long carry0 = 0, carry1 = 0;
    for (long base = 0; base < nch; base += 1024) {
        const long c = base + tid;
        const long long v0 = c < nch ? cc[2 * c] : 0, v1 = c < nch ? cc[2 * c + 1] : 0;
        long long x0 = v0, x1 = v1;
        for (int d = 1; d < 64; d <<= 1) {
            const long long y0 = __shfl_up(x0, d, 64), y1 = __shfl_up(x1, d, 64);
            if (l >= d) { x0 += y0; x1 += y1; }
        }
        if (l == 63) { s[0][w] = x0; s[1][w] = x1; }
        __syncthreads();
        if (w == 0) {
            long long t0 = l < 16 ? s[0][l] : 0, t1 = l < 16 ? s[1][l] : 0;
            for (int d = 1; d < 16; d <<= 1) {
                const long long y0 = __shfl_up(t0, d, 64), y1 = __shfl_up(t1, d, 64);
                if (l >= d) { t0 += y0; t1 += y1; }
            }
            if (l < 16) { s[0][l] = t0; s[1][l] = t1; }
        }
        __syncthreads();
        const long long p0 = carry0 + (w > 0 ? s[0][w - 1] : 0) + x0 - v0;
        const long long p1 = carry1 + (w > 0 ? s[1][w - 1] : 0) + x1 - v1;
        if (c < nch) {
            cc[2 * c] = p0;
            cc[2 * c + 1] = p1;
        }
        carry0 += s[0][15];
        carry1 += s[1][15];
        __syncthreads();   // s is rewritten by the next tile
    }
    if (tid == 0) {
        counts[0] = (unsigned long long)carry0;
        counts[1] = (unsigned long long)carry1;
    }
}

__global__ __launch_bounds__(256) void k_part_scatter(PartArgs a, const long long *cc)
{
    __shared__ int s_cnt[2][4];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const unsigned long long below = (l == 0) ? 0ull : (~0ull >> (64 - l));
    const long nch = (a.n + kPartChunk - 1) / kPartChunk;
    for (long c = blockIdx.x; c < nch; c += gridDim.x) {
        long long base0 = cc[2 * c], base1 = cc[2 * c + 1];
        for (int r = 0; r < kPartChunk / 256; ++r) {
            const long e = c * kPartChunk + r * 256 + tid;
            const int f = e < a.n ? entry_class(a, e) : 0;
            const unsigned long long m64 = __ballot(f == 1), m32 = __ballot(f == 2);
            if (l == 0) {
                s_cnt[0][w] = __popcll(m64);
                s_cnt[1][w] = __popcll(m32);
            }
            __syncthreads();
            if (f) {
                const int k = f - 1;
                const unsigned long long m = k ? m32 : m64;
                long long pos = (k ? base1 : base0) + __popcll(m & below);
                for (int u = 0; u < w; ++u) pos += s_cnt[k][u];
                if (k == 0) { a.b64[pos] = a.bra[e]; a.k64[pos] = a.ket[e]; }
                else { a.b32[pos] = a.bra[e]; a.k32[pos] = a.ket[e]; }
            }
            base0 += s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3];
            base1 += s_cnt[1][0] + s_cnt[1][1] + s_cnt[1][2] + s_cnt[1][3];
            __syncthreads();   // s_cnt is rewritten by the next round
        }
    }
}

}  // namespace

hipError_t launch_nbr(const NbrArgs &a, hipStream_t st)
{
    if (a.nb <= 0 || a.nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nbr, dim3((a.nb + 3) / 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_partition(const PartArgs &a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const long nch = (a.n + kPartChunk - 1) / kPartChunk;
    const unsigned grid = (unsigned)(nch < 8192 ? nch : 8192);
    hipLaunchKernelGGL(k_part_count, dim3(grid), dim3(256), 0, st, a, a.chunk_counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_part_scan, dim3(1), dim3(1024), 0, st, a.chunk_counts, nch, a.counts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_part_scatter, dim3(grid), dim3(256), 0, st, a, (const long long *)a.chunk_counts);
    return hipGetLastError();
}

}  // namespace pbcjk
