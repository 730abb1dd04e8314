// Fused Yee kernels with CPML absorbing layers: graded FP32 storage, one row
// per lane (their own translation unit, compiled in parallel with the others).
#include "yee_fused.hpp"

namespace yee {

hipError_t launch_fused_cpml(int T, const FusedArgs &a, const CpmlFused &c, int zc, hipStream_t st)
{
    constexpr Tiling tl = kCpmlTiling;
    if (c.pml.n < 1 || !a.gc || !c.pml.cp || !c.pml.psi || !c.psi_out) return hipErrorInvalidValue;
    switch (T) {
    case 1: return launch_shape<1, tl.ry, tl.nw, CodecF32, true, true>(a, zc, st, c);
    case 2: return launch_shape<2, tl.ry, tl.nw, CodecF32, true, true>(a, zc, st, c);
    case 3: return launch_shape<3, tl.ry, tl.nw, CodecF32, true, true>(a, zc, st, c);
    }
    return hipErrorInvalidValue;
}

}  // namespace yee
