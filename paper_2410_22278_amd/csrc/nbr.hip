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

}  // namespace

hipError_t launch_nbr(const NbrArgs &a, hipStream_t st)
{
    if (a.nb <= 0 || a.nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nbr, dim3((a.nb + 3) / 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace pbcjk
