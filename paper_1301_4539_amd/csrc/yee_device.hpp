// Device-side helpers: storage codecs, the scale rule and cross-lane moves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "yee_internal.hpp"

namespace yee {

// ---- storage codecs --------------------------------------------------------
// A stored value q of component c represents q * 2^-s_c.  Encoding rounds
// y = x * 2^s_c to nearest-even after clamping y to +-(largest finite value):
// for every finite y this equals rounding and then saturating what would
// overflow.  Stores track the largest |x| (as bits; NaN compares above every
// number); finish_max() turns it into the largest stored magnitude (scaling
// by 2^s and rounding are monotone, so max |Q(y)| = Q(max |x| 2^s)), the
// overflow test (|y| at or above the first value that would round beyond the
// largest finite one) and the NaN test.

struct CodecF32 {
    using T = float;
    static constexpr bool scaled = false;
    __device__ static inline float load(const float *p, float) { return *p; }
};

struct CodecF16 {
    using T = uint16_t;
    static constexpr bool scaled = true;
    static constexpr float kMax = 65504.0f;        // largest finite binary16
    static constexpr float kOver = 65520.0f;       // rounds to infinity from here on
    __device__ static inline float load(const uint16_t *p, float down)
    {
        return (float)__builtin_bit_cast(_Float16, *p) * down;
    }
    __device__ static inline uint16_t encode(float y)
    {
        return __builtin_bit_cast(uint16_t, (_Float16)__builtin_amdgcn_fmed3f(y, -kMax, kMax));
    }
    // Encode v * 2^s; fold |v| into mx when `track` (owned values only).
    __device__ static inline uint16_t encode_tracked(float v, float up, uint32_t &mx, bool track)
    {
        const uint32_t a = __builtin_bit_cast(uint32_t, v) & 0x7fffffffu;
        mx = (track && a > mx) ? a : mx;
        return encode(v * up);
    }
    __device__ static inline float stored_mag(float ymax)
    {
        return (float)__builtin_bit_cast(_Float16, encode(ymax));
    }
};

struct CodecBF16 {
    using T = uint16_t;
    static constexpr bool scaled = true;
    static constexpr uint32_t kMaxBits = 0x7f7f0000u;   // largest finite bfloat16
    static constexpr uint32_t kOverBits = 0x7f7f8000u;  // rounds to infinity from here on
    __device__ static inline float load(const uint16_t *p, float down)
    {
        return __builtin_bit_cast(float, (uint32_t)(*p) << 16) * down;
    }
    __device__ static inline uint16_t encode(float y)
    {
        const float m = __builtin_bit_cast(float, kMaxBits);
        const uint32_t u = __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(y, -m, m));
        return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
    // Encode v * 2^s; fold |v| into mx when `track` (owned values only).
    __device__ static inline uint16_t encode_tracked(float v, float up, uint32_t &mx, bool track)
    {
        const uint32_t a = __builtin_bit_cast(uint32_t, v) & 0x7fffffffu;
        mx = (track && a > mx) ? a : mx;
        return encode(v * up);
    }
    __device__ static inline float stored_mag(float ymax)
    {
        return __builtin_bit_cast(float, (uint32_t)encode(ymax) << 16);
    }
};

// From the largest |x| bits a thread saw (values before encoding, scale
// 2^s = up): the largest stored magnitude (in field units), whether a NaN was
// stored, whether |x| 2^s would round beyond the largest finite value
// (overflow), and the largest |x| itself.
template <class Codec>
__device__ inline void finish_max(uint32_t xbits, float up, float *m, bool *nan, bool *over, float *pre)
{
    *nan = xbits > 0x7f800000u;
    if (*nan) { *over = false; *m = 0.0f; *pre = 0.0f; return; }
    *pre = __builtin_bit_cast(float, xbits);
    const float ymax = *pre * up;
    if constexpr (std::is_same<Codec, CodecF16>::value) *over = ymax >= CodecF16::kOver;
    else *over = __builtin_bit_cast(uint32_t, ymax) >= CodecBF16::kOverBits;
    *m = Codec::stored_mag(ymax) * (1.0f / up);   // 2^-s: exact
}

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
// DPP wave shifts: one VALU op (often folded into the subtraction that uses
// it), no LDS traffic.  Lanes with no source lane (lane 63 for from_right,
// lane 0 for from_left) read 0 (bound_ctrl); they are halo lanes.
// Value held by lane+1 (wave_shl:1).
__device__ inline float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
// Value held by lane-1 (wave_shr:1).
__device__ inline float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}

}  // namespace yee
