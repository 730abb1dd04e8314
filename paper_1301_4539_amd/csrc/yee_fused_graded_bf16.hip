// Fused Yee kernels with graded (per-index) cell sizes, bfloat16 storage (a
// translation unit of their own, compiled in parallel with the others).
#include "yee_fused.hpp"

namespace yee {

hipError_t launch_fused_bf16_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                   hipStream_t st)
{
    return launch_codec<CodecBF16, true>(T, a, n, batch, variant, zc, st);
}

}  // namespace yee
