// Fused Yee kernels instantiated for one storage format (one translation
// unit per format, so the three compile in parallel).
#include "yee_fused.hpp"

namespace yee {

hipError_t launch_fused_f32(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st)
{
    return launch_codec<CodecF32>(T, a, n, batch, variant, zc, st);
}

}  // namespace yee
