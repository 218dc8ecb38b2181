// k_dft.hip -- split-precision DFT-matrix transform (placeholder until the
// MFMA kernels land).
#include "internal.hpp"

namespace epic {

epic_status launch_dft2_split(int, int, int64_t, int, const float2 *, float2 *, int, hipStream_t)
{
    return fail(EPIC_ERR_UNSUPPORTED, "split-precision transform not built yet");
}

}  // namespace epic
