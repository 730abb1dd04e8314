// Fused Yee kernels that also sum the energy of one time level's input state,
// uniform spacing, F32 storage (their own translation unit, compiled in
// parallel with the others).
#include "yee_fused.hpp"

namespace yee {

namespace {

template <int T>
hipError_t launch_t_energy(const FusedArgs &a, const EnergyFused &en, int variant, int zc, hipStream_t st)
{
    switch (variant) {
    case 1: return launch_shape<T, kTilings[T][1].ry, kTilings[T][1].nw, CodecF32, false, false, true>(a, zc, st, {}, en);
    case 2: return launch_shape<T, kTilings[T][2].ry, kTilings[T][2].nw, CodecF32, false, false, true>(a, zc, st, {}, en);
    default: return launch_shape<T, kTilings[T][0].ry, kTilings[T][0].nw, CodecF32, false, false, true>(a, zc, st, {}, en);
    }
}

}  // namespace

hipError_t launch_fused_energy_f32(int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
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

namespace yee {

hipError_t launch_fused_energy_f16(int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
                                  hipStream_t st);
hipError_t launch_fused_energy_bf16(int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
                                   hipStream_t st);

hipError_t launch_fused_energy(int storage, int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
                               hipStream_t st)
{
    switch (storage) {
    case 0: return launch_fused_energy_f32(T, a, en, variant, zc, st);
    case 1: return launch_fused_energy_f16(T, a, en, variant, zc, st);
    case 2: return launch_fused_energy_bf16(T, a, en, variant, zc, st);
    }
    return hipErrorInvalidValue;
}

long long fused_tiles_bound(const Layout &L)
{
    long long most = 0;
    for (int T = 1; T <= MAX_T_ENERGY; ++T)
        for (int v = 0; v < 3; ++v) {
            const Tiling tl = kTilings[T][v];
            const long long ox = 64 - 2 * T, oy = tl.ry * tl.nw - 2 * T;
            most = std::max(most, ((L.nx + 1 + ox - 1) / ox) * ((L.ny + 1 + oy - 1) / oy) * (long long)(L.nz + 1));
        }
    return most;
}

}  // namespace yee
