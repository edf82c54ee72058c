// Short-range (real-space erfc) part of the Gamma-point J and K builds.
//
// For each unique pair of (shell pair, image) groups the kernel sums the
// primitive quartets and the lattice shifts R1 of the ket (Sec. 2.4, eq.
// pbc_eri_general_final, real-space term) into a contracted Cartesian
// integral block held in registers, then contracts the block with the
// density into the J and K halves:
//   X[a,b] += 2w I D[c,d],  X[c,d] += 2w I D[a,b]          (J = X + X^T)
//   Y[a,c] += w I D[b,d], Y[b,c] += w I D[a,d],
//   Y[a,d] += w I D[b,c], Y[b,d] += w I D[a,c]              (K = Y + Y^T)
// with w = 1/2 on the diagonal group pair and 1 otherwise (the primitive
// symmetry weights are folded into the pair prefactors).
//
// Mapping: one lane per entry of the class pair's work list (the group pairs
// of the neighbour list that pass this build's density-weighted screen, in
// one precision; entries of one bra group are consecutive, so a wavefront
// mostly shares its bra data).  Each lane screens the primitive quartets of
// its group pair and finds the lattice shifts R1 inside each quartet's
// real-space sphere.  With FOLD the Hermite integrals R_{tuv} of the shifts
// are summed in FP64 before the Hermite -> Cartesian transforms, which then
// run once per quartet (the better order when quartets have several shifts,
// as in small cells); without it the transforms run per shift.
// In the FP32 variant R_{tuv} of each shift and the transforms are FP32
// (the Boys values stay FP64 for small arguments); the lattice sum and the
// block accumulation are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sr_lane.h"

namespace pbcjk {

namespace {

// Grid: enough blocks of 256 lanes for the work list's upper bound, capped;
// the kernel strides over the actual device-side count.
inline dim3 sr_grid(long max_entries)
{
    return dim3((unsigned)std::max(1L, (max_entries + 255) / 256));
}

template <int LA, int LB, int LC, int LD>
hipError_t launch_one(const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
    if (a.max_entries <= 0) return hipSuccess;
    const dim3 g = sr_grid(a.max_entries), b(256);
    if (f32 && fold) hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, float, true>), g, b, 0, st, a);
    else if (f32) hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, float, false>), g, b, 0, st, a);
    else if (fold) hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, double, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_sr_jk<LA, LB, LC, LD, double, false>), g, b, 0, st, a);
    return hipGetLastError();
}

constexpr int kLa[kNumClass] = {0, 1, 1, 2, 2, 2};
constexpr int kLb[kNumClass] = {0, 0, 1, 0, 1, 2};

template <int CB, int CK>
hipError_t launch_pair(const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
    return launch_one<kLa[CB], kLb[CB], kLa[CK], kLb[CK]>(a, f32, fold, st);
}

}  // namespace

// Launches the kernel of bra class cb and ket class ck (cb <= ck) on one
// work list, in FP32 (f32) or FP64, with or without the lattice sum folded
// into the Hermite integrals.
hipError_t launch_sr_jk(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
#define PBCJK_CASE(X, Y) \
    if (cb == X && ck == Y) return launch_pair<X, Y>(a, f32, fold, st);
    PBCJK_CASE(0, 0) PBCJK_CASE(0, 1) PBCJK_CASE(0, 2) PBCJK_CASE(1, 1) PBCJK_CASE(1, 2) PBCJK_CASE(2, 2)
#if PBCJK_WITH_D
    // d-shell class pairs whose block and E coefficients fit in registers;
    // the others run in the cooperative kernel
    PBCJK_CASE(0, 3) PBCJK_CASE(0, 4) PBCJK_CASE(1, 3)
    PBCJK_CASE(1, 4) PBCJK_CASE(2, 3) PBCJK_CASE(3, 3)
#endif
#undef PBCJK_CASE
    return hipErrorNotSupported;
}

}  // namespace pbcjk
