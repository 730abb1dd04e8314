// Dispatch of the fused Yee kernel by storage format, and the size limits of
// its addressing.
#include <algorithm>

#include "yee_internal.hpp"

namespace yee {

hipError_t launch_fused_f32(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);
hipError_t launch_fused_f16(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);
hipError_t launch_fused_bf16(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);

namespace {

hipError_t launch_any(int storage, int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                      hipStream_t st)
{
    switch (storage) {
    case 0: return launch_fused_f32(T, a, n, batch, variant, zc, st);
    case 1: return launch_fused_f16(T, a, n, batch, variant, zc, st);
    case 2: return launch_fused_bf16(T, a, n, batch, variant, zc, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

bool fused_fits(const Layout &L, int storage, int T)
{
    // a chunk's buffer resource spans (planes * kstride * es) bytes, below 2^31
    const int es = storage == 0 ? 4 : 2;
    const long long planes = ((1LL << 31) - 1) / ((long long)L.kstride * es);
    return planes >= 2 * T + 2 && (long long)L.pitch * es < (1LL << 31);
}

hipError_t launch_fused(int storage, int T, const FusedArgs &a, int variant, int zc, hipStream_t st)
{
    return launch_any(storage, T, &a, 1, false, variant, zc, st);
}

hipError_t launch_fused_batch(int storage, int T, const FusedArgs *args, int n, int variant, int zc,
                              hipStream_t st)
{
    if (n < 1 || n > MAX_BATCH) return hipErrorInvalidValue;
    return launch_any(storage, T, args, n, true, variant, zc, st);
}

}  // namespace yee
