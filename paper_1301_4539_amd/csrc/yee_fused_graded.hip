// Fused Yee kernels with graded (per-index) cell sizes, FP32 storage (their
// own translation unit, compiled in parallel with the uniform ones).
#include "yee_fused.hpp"

namespace yee {

hipError_t launch_fused_f32_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                   hipStream_t st)
{
    return launch_codec<CodecF32, true>(T, a, n, batch, variant, zc, st);
}

}  // namespace yee
