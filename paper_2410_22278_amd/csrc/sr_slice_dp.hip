// Component-slice launches of the (dp|dp) and (dp|dd) class pairs (their own
// translation unit, to compile in parallel with the other slices).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sr_lane.h"

namespace pbcjk {

hipError_t launch_sr_slices_dp(int cb, int ck, const SRArgs &a, bool f32, bool fold, hipStream_t st)
{
#if PBCJK_WITH_D
    if (cb == 4 && ck == 4) return launch_slices<2, 1, 2, 1, 2>(a, f32, fold, st);
    if (cb == 4 && ck == 5) return launch_slices<2, 1, 2, 2, 1>(a, f32, fold, st);
#endif
    return hipErrorNotSupported;
}

}  // namespace pbcjk
