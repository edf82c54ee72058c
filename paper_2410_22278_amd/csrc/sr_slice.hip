// Short-range J and K for the large d class pairs in the per-lane kernel,
// one launch per slice of the first ket shell's Cartesian components (the
// slice's block fits in one lane's registers; each launch recomputes the
// Hermite integrals of its quartets and shifts).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sr_lane.h"

namespace pbcjk {

namespace {

constexpr int kLa[kNumClass] = {0, 1, 1, 2, 2, 2};
constexpr int kLb[kNumClass] = {0, 0, 1, 0, 1, 2};

}  // namespace

// Class pairs (cb <= ck) run in slices; hipErrorNotSupported for the others.
hipError_t launch_sr_slices(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
    if (a.max_entries <= 0) return hipSuccess;
#define PBCJK_SLICE(X, Y, W) \
    if (cb == X && ck == Y) return launch_slices<kLa[X], kLb[X], kLa[Y], kLb[Y], W>(a, f32, fold, st);
#if PBCJK_WITH_D
    PBCJK_SLICE(0, 5, 3) PBCJK_SLICE(1, 5, 2) PBCJK_SLICE(2, 4, 3) PBCJK_SLICE(2, 5, 1)
    PBCJK_SLICE(3, 4, 3) PBCJK_SLICE(3, 5, 2)
#endif
#undef PBCJK_SLICE
    return launch_sr_slices_dp(cb, ck, a, f32, fold, st);
}

}  // namespace pbcjk
