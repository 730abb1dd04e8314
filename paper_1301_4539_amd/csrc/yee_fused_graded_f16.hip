// Fused Yee kernels with graded (per-index) cell sizes, binary16 storage (a
// translation unit of their own, compiled in parallel with the others).
#include "yee_fused.hpp"

namespace yee {

hipError_t launch_fused_f16_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                   hipStream_t st)
{
    return launch_codec<CodecF16, true>(T, a, n, batch, variant, zc, st);
}

}  // namespace yee
