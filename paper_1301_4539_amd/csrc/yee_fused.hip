// Dispatch of the fused Yee kernel by storage format, and the size limits of
// its addressing.
#include <algorithm>

#include "yee_internal.hpp"

namespace yee {

hipError_t launch_fused_f32(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);
hipError_t launch_fused_f16(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);
hipError_t launch_fused_bf16(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st);
hipError_t launch_fused_f32_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                   hipStream_t st);
hipError_t launch_fused_f16_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                   hipStream_t st);
hipError_t launch_fused_bf16_graded(int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                                    hipStream_t st);

namespace {

hipError_t launch_any(int storage, int T, const FusedArgs *a, int n, bool batch, int variant, int zc,
                      hipStream_t st)
{
    if (a->gc) {   // graded spacing: one solve per launch
        if (batch) return hipErrorInvalidValue;
        switch (storage) {
        case 0: return launch_fused_f32_graded(T, a, n, batch, variant, zc, st);
        case 1: return launch_fused_f16_graded(T, a, n, batch, variant, zc, st);
        case 2: return launch_fused_bf16_graded(T, a, n, batch, variant, zc, st);
        }
        return hipErrorInvalidValue;
    }
    switch (storage) {
    case 0: return launch_fused_f32(T, a, n, batch, variant, zc, st);
    case 1: return launch_fused_f16(T, a, n, batch, variant, zc, st);
    case 2: return launch_fused_bf16(T, a, n, batch, variant, zc, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Fastest tile shape per (storage, T) measured on MI355X with the 256^3 and
// 512^3 dielectric workloads (shape indices of the fused kernel's tile table:
// 0 = 2 rows x 16 waves, 1 = 4 x 8, 2 = 3 x 12; 4 x 4, 2 x 8, 2 x 16 for T=1).
// With FP32 storage at T = 4 and 5 the 8-wave shape is the faster one on
// grids of 64 M cells and more (512^3: 250 against 240 G/s at T = 4, 254
// against 248 at T = 5) and the 16-wave one below (256^3: 216 against 205 at
// T = 4).  Graded spacing (FP32) was measured on its own 256^3 workload.
int auto_shape(int storage, int T, bool graded, long long cells)
{
    static const int f32[MAX_T + 1] = {0, 2, 1, 1, 0, 0, 0};
    static const int f32g[MAX_T_GRADED + 1] = {0, 0, 1, 0, 2};
    static const int f16[MAX_T + 1] = {0, 2, 0, 0, 0, 1, 1};
    static const int bf16[MAX_T + 1] = {0, 2, 0, 0, 0, 1, 1};
    if (T < 1 || T > MAX_T || (graded && T > MAX_T_GRADED)) return 0;
    if (storage == 0) {
        if (graded) return f32g[T];
        if ((T == 4 || T == 5) && cells >= (64LL << 20)) return 1;
        return f32[T];
    }
    return storage == 1 ? f16[T] : bf16[T];
}

// Fastest steps per pass on MI355X for the storage format (FP32 storage is
// compute-bound at 4, 16-bit storage at 3; graded spacing at 3, where its
// extra registers push T = 4 into spills), lowered while the grid's planes
// are too large for the fused kernel's addressing.
int fastest_T(const Layout &L, int storage, bool graded)
{
    int T = storage == 0 && !graded ? 4 : 3;
    while (T > 1 && !fused_fits(L, storage, T)) --T;
    return T;
}

bool cpml_fused_fits(const Layout &L, long long psi_elems, int T)
{
    return T >= 1 && T <= MAX_T_CPML && fused_fits(L, 0, T) && psi_elems * 4 < (1LL << 31);
}

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
