// Device-side helpers: storage codecs, the scale rule and cross-lane moves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "yee_internal.hpp"

namespace yee {

// ---- storage codecs --------------------------------------------------------
// A stored value q of component c represents q * 2^-s_c.  Encoding rounds
// x * 2^s_c to nearest-even; a result beyond the largest finite value
// saturates to +-max and raises the flag, a NaN raises the flag.
// enc_max tracks the largest encoded magnitude (bits), excluding NaN.

struct CodecF32 {
    using T = float;
    static constexpr bool scaled = false;
    __device__ static inline float load(const float *p, float) { return *p; }
    __device__ static inline void store(float *p, float v, float, uint32_t &, uint32_t &) { *p = v; }
    __device__ static inline float decode_mag(uint32_t, float) { return 0.0f; }
};

struct CodecF16 {
    using T = uint16_t;
    static constexpr bool scaled = true;
    __device__ static inline float load(const uint16_t *p, float down)
    {
        return (float)__builtin_bit_cast(_Float16, *p) * down;
    }
    __device__ static inline void store(uint16_t *p, float v, float up, uint32_t &mx, uint32_t &flag)
    {
        uint16_t h = __builtin_bit_cast(uint16_t, (_Float16)(v * up));
        uint32_t a = h & 0x7fffu;
        if (a == 0x7c00u) { h = (uint16_t)((h & 0x8000u) | 0x7bffu); a = 0x7bffu; flag = 1u; }
        if (a > 0x7c00u) flag = 1u;
        else mx = a > mx ? a : mx;
        *p = h;
    }
    __device__ static inline float decode_mag(uint32_t a, float down)
    {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)a) * down;
    }
};

struct CodecBF16 {
    using T = uint16_t;
    static constexpr bool scaled = true;
    __device__ static inline float load(const uint16_t *p, float down)
    {
        return __builtin_bit_cast(float, (uint32_t)(*p) << 16) * down;
    }
    __device__ static inline void store(uint16_t *p, float v, float up, uint32_t &mx, uint32_t &flag)
    {
        uint32_t u = __builtin_bit_cast(uint32_t, v * up);
        uint16_t h;
        if ((u & 0x7fffffffu) > 0x7f800000u) h = (uint16_t)((u >> 16) | 0x40u);
        else h = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        uint32_t a = h & 0x7fffu;
        if (a == 0x7f80u) { h = (uint16_t)((h & 0x8000u) | 0x7f7fu); a = 0x7f7fu; flag = 1u; }
        if (a > 0x7f80u) flag = 1u;
        else mx = a > mx ? a : mx;
        *p = h;
    }
    __device__ static inline float decode_mag(uint32_t a, float down)
    {
        return __builtin_bit_cast(float, a << 16) * down;
    }
};

// ---- scale rule --------------------------------------------------------------
// s = 10 - ceil(log2 m), clamped to [-64, 64]; m = max(M_c, A), or the
// largest M over the components when that is zero; s = 0 when all are zero.
__device__ inline int scale_from(float m)
{
    if (!(m > 0.0f) || __builtin_isinf(m)) return 0;
    int e;
    float fr = frexpf(m, &e);
    int cl = fr == 0.5f ? e - 1 : e;
    int s = 10 - cl;
    return s > 64 ? 64 : (s < -64 ? -64 : s);
}

__device__ inline void choose_scales(const float *mprev, float a_max, int *s)
{
    float all = 0.0f;
    for (int c = 0; c < 6; ++c) all = mprev[c] > all ? mprev[c] : all;
    for (int c = 0; c < 6; ++c) {
        float m = mprev[c] > a_max ? mprev[c] : a_max;
        if (!(m > 0.0f)) m = all;
        s[c] = scale_from(m);
    }
}

// ---- cross-lane moves (wave64) ---------------------------------------------
// DPP wave shifts: one VALU op, no LDS traffic.  Lanes with no source lane
// (lane 63 for from_right, lane 0 for from_left) get 0; they are halo lanes.
// Value held by lane+1 (wave_shl:1).
__device__ inline float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
// Value held by lane-1 (wave_shr:1).
__device__ inline float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}

}  // namespace yee
