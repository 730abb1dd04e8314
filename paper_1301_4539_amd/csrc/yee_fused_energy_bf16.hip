// Fused Yee kernels that also sum the energy of one time level's input state,
// uniform spacing, BF16 storage (their own translation unit, compiled in
// parallel with the others).
#include "yee_fused.hpp"

namespace yee {

namespace {

template <int T>
hipError_t launch_t_energy(const FusedArgs &a, const EnergyFused &en, int variant, int zc, hipStream_t st)
{
    switch (variant) {
    case 1: return launch_shape<T, kTilings[T][1].ry, kTilings[T][1].nw, CodecBF16, false, false, true>(a, zc, st, {}, en);
    case 2: return launch_shape<T, kTilings[T][2].ry, kTilings[T][2].nw, CodecBF16, false, false, true>(a, zc, st, {}, en);
    default: return launch_shape<T, kTilings[T][0].ry, kTilings[T][0].nw, CodecBF16, false, false, true>(a, zc, st, {}, en);
    }
}

}  // namespace

hipError_t launch_fused_energy_bf16(int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
                                  hipStream_t st)
{
    if (a.gc || en.level < 1 || en.level > T || !en.partial || !en.half_eps || !en.out) return hipErrorInvalidValue;
    switch (T) {
    case 1: return launch_t_energy<1>(a, en, variant, zc, st);
    case 2: return launch_t_energy<2>(a, en, variant, zc, st);
    case 3: return launch_t_energy<3>(a, en, variant, zc, st);
    case 4: return launch_t_energy<4>(a, en, variant, zc, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace yee
