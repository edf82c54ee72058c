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

__global__ __launch_bounds__(256) void k_nbr(NbrArgs a)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int bi = blockIdx.x * (blockDim.x >> 6) + wave;
    if (bi >= a.nb) return;
    const GroupRec gb = a.groups[a.gb0 + bi];
    const int jlo = a.tri ? bi : 0;
    long base = a.mode ? a.offsets[bi] : 0;
    int cnt = 0;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int j0 = jlo; j0 < a.nk; j0 += 64) {
        const int j = j0 + lane;
        bool keep = false;
        if (j < a.nk) {
            const GroupRec gk = a.groups[a.gk0 + j];
            keep = group_pair_test(a, gb, gk) && group_pair_has_term(a, gb, gk);
        }
        const unsigned long long m = __ballot(keep);
        if (a.mode && keep) {
            const long pos = base + cnt + __popcll(m & below);
            a.out_bra[pos] = bi;
            a.out_ket[pos] = j;
        }
        cnt += __popcll(m);
    }
    if (!a.mode && lane == 0) a.counts[bi] = cnt;
}

// Screen flags of one entry: bit 0 keep in FP64, bit 1 keep in FP32.
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
    return (a.split && bound < a.fp32_below) ? 2 : 1;
}

__global__ __launch_bounds__(256) void k_partition(PartArgs a)
{
    __shared__ int s_cnt[2][4];
    __shared__ unsigned long long s_base[2];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (long c0 = (long)blockIdx.x * 256; c0 < a.n; c0 += (long)gridDim.x * 256) {
        const long e = c0 + tid;
        const int f = e < a.n ? entry_class(a, e) : 0;
        const unsigned long long m64 = __ballot(f == 1), m32 = __ballot(f == 2);
        const unsigned long long below = (l == 0) ? 0ull : (~0ull >> (64 - l));
        if (l == 0) {
            s_cnt[0][w] = __popcll(m64);
            s_cnt[1][w] = __popcll(m32);
        }
        __syncthreads();
        if (tid == 0) {
            const int t64 = s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3];
            const int t32 = s_cnt[1][0] + s_cnt[1][1] + s_cnt[1][2] + s_cnt[1][3];
            s_base[0] = t64 ? atomicAdd(&a.counts[0], (unsigned long long)t64) : 0ull;
            s_base[1] = t32 ? atomicAdd(&a.counts[1], (unsigned long long)t32) : 0ull;
        }
        __syncthreads();
        if (f) {
            const int k = f - 1;
            const unsigned long long m = k ? m32 : m64;
            long pos = (long)s_base[k] + __popcll(m & below);
            for (int u = 0; u < w; ++u) pos += s_cnt[k][u];
            if (k == 0) { a.b64[pos] = a.bra[e]; a.k64[pos] = a.ket[e]; }
            else { a.b32[pos] = a.bra[e]; a.k32[pos] = a.ket[e]; }
        }
        __syncthreads();   // s_cnt and s_base are rewritten by the next chunk
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
    const long chunks = (a.n + 255) / 256;
    const unsigned grid = (unsigned)(chunks < 8192 ? chunks : 8192);
    hipLaunchKernelGGL(k_partition, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace pbcjk
