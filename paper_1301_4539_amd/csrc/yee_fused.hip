// Fused, temporally blocked Yee kernel: one pass over HBM advances T steps.
//
// This is the GPU form of the cache-reuse ideas of Sec. 3: Ampere and
// Faraday interleaved per sub-domain (Sec. 3.2), plane by plane along z
// (Sec. 3.3), several time steps gathered per pass (Sec. 3.4, generalised
// to T steps as suggested in the conclusion).  On a GPU the "cache" is the
// register file: a workgroup owns an x-y tile, marches z, and keeps T+1 time
// levels of the six fields in registers; level t runs one plane behind level
// t-1.  Overlapped tiles (a halo of T cells on every side in x and y, T
// planes at both ends of a z chunk) replace the paper's surface routines:
// halo cells are recomputed redundantly instead of being exchanged, so each
// owned value depends only on data this workgroup computed itself, in the
// same operation order as the plain kernel -- results are bit-identical for
// every T and tile shape.
//
// Thread layout: lane = x (64 consecutive points, coalesced), each lane holds
// RY consecutive rows in y, NW waves stack in y.  x neighbours move between
// lanes with cross-lane shuffles; the y neighbour across a wave boundary goes
// through a small LDS slot.  Fields are read from buffer fin and the advanced
// state is written to buffer fout (ping-pong): an in-place update would race
// with neighbouring tiles still reading the old time level.

#include "yee_device.hpp"
#include "yee_internal.hpp"

namespace yee {

namespace {

template <int T>
struct Shape;
// rows per lane, waves per workgroup
template <> struct Shape<1> { static constexpr int RY = 4, NW = 4; };
template <> struct Shape<2> { static constexpr int RY = 4, NW = 8; };
template <> struct Shape<3> { static constexpr int RY = 4, NW = 8; };
template <> struct Shape<4> { static constexpr int RY = 4, NW = 8; };

template <int T, class Codec>
__global__ __launch_bounds__(64 * Shape<T>::NW) void yee_fused(FusedArgs a)
{
    constexpr int RY = Shape<T>::RY, NW = Shape<T>::NW;
    constexpr int OX = 64 - 2 * T;      // owned points per tile in x
    constexpr int NR = NW * RY;         // rows per tile
    constexpr int OY = NR - 2 * T;      // owned rows per tile
    using S = typename Codec::T;

    __shared__ float4 s_coef[256];
    __shared__ float2 s_e[NW + 1][64];  // (Ex, Ez) of each wave's first row; slot NW stays zero
    __shared__ float2 s_h[NW + 1][64];  // (Hx, Hz) of each wave's last row, in slot w+1; slot 0 stays zero

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int q = tid; q < a.n_mat; q += 64 * NW) s_coef[q] = a.coef[q];
    if (tid < 64) {
        s_e[NW][tid] = make_float2(0.0f, 0.0f);
        s_h[0][tid] = make_float2(0.0f, 0.0f);
    }

    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so that halo re-reads hit its own L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (b & 7) * (nb >> 3) + (b >> 3);

    float dn[6], up[6];
    if constexpr (Codec::scaled) {
        float mprev[6];
        int s_in[6], s_out[6];
        for (int c = 0; c < 6; ++c) {
            mprev[c] = __uint_as_float(a.sb.ctrl->maxbits[a.sb.slot_in][c]);
            s_in[c] = a.sb.ctrl->scale[a.sb.par][c];
        }
        choose_scales(mprev, a.sb.a_max, s_out);
        for (int c = 0; c < 6; ++c) {
            dn[c] = ldexpf(1.0f, -s_in[c]);
            up[c] = ldexpf(1.0f, s_out[c]);
        }
        if (logical == 0 && tid < 6) {
            a.sb.ctrl->scale[a.sb.par ^ 1][tid] = s_out[tid];
            a.sb.ctrl->maxbits[a.sb.slot_clear][tid] = 0u;
        }
    } else {
        for (int c = 0; c < 6; ++c) dn[c] = up[c] = 1.0f;
    }
    __syncthreads();
    if (logical >= a.nwg) return;   // uniform per workgroup

    const Layout L = a.L;
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int tx = logical % a.ntx;
    const int rem = logical / a.ntx;
    const int ty = rem % a.nty, tz = rem / a.nty;
    const int x0 = tx * OX, y0 = ty * OY, z0 = tz * a.zc;
    const int z1 = min(z0 + a.zc, nz + 1);
    const int xl = x0 - T;              // x of lane 0
    const int x = xl + lane;
    const int yt = y0 - T;              // y of the tile's first row
    const int yw = yt + w * RY;         // y of this wave's first row
    const int kb = max(0, z0 - T);      // first plane the pipeline loads
    const int ke = min(nz, z1 - 1 + T); // last plane the pipeline loads

    const bool xin = x >= 0 && x <= nx;
    const bool xlt = x < nx;
    const bool xint = x > 0 && x < nx;
    const bool xown = lane >= T && lane < T + OX && x <= nx;

    const S *fin = static_cast<const S *>(a.fin);
    S *fout = static_cast<S *>(a.fout);
    const long long cs = L.cstride;

    float E[T + 1][3][RY], H[T + 1][3][RY];
    int M[T + 1][RY];
#pragma unroll
    for (int t = 0; t <= T; ++t)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            M[t][r] = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) E[t][c][r] = H[t][c][r] = 0.0f;
        }

    // prefetched next level-0 plane
    float PE[3][RY], PH[3][RY];
    int PM[RY];

#define YEE_LOAD_PLANE(KK)                                                              \
    do {                                                                                \
        const int kk_ = (KK);                                                           \
        _Pragma("unroll") for (int r = 0; r < RY; ++r) {                                \
            const int y = yw + r;                                                       \
            const bool in = xin && y >= 0 && y <= ny && kk_ <= ke;                      \
            const long long off = (long long)kk_ * L.plane + (long long)y * L.pitch + x; \
            _Pragma("unroll") for (int c = 0; c < 3; ++c) {                             \
                PE[c][r] = in ? Codec::load(fin + c * cs + off, dn[c]) : 0.0f;          \
                PH[c][r] = in ? Codec::load(fin + (3 + c) * cs + off, dn[3 + c]) : 0.0f; \
            }                                                                           \
            PM[r] = in ? (int)a.mat[off] : 0;                                           \
        }                                                                               \
    } while (0)

    YEE_LOAD_PLANE(kb);

    uint32_t mx[6] = {0u, 0u, 0u, 0u, 0u, 0u};
    uint32_t flag = 0u;

    for (int K = kb; K <= ke + T; ++K) {
        // Level 0 takes plane K; plane K-1 of level 0 becomes level 1's input.
        float Eo[3][RY], Ho[3][RY];
        int Mo[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            Mo[r] = M[0][r];
            M[0][r] = PM[r];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Eo[c][r] = E[0][c][r];
                Ho[c][r] = H[0][c][r];
                E[0][c][r] = PE[c][r];
                H[0][c][r] = PH[c][r];
            }
        }
        YEE_LOAD_PLANE(K + 1);

#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int p = K - t;                      // plane of time level t
            if (p >= kb && p <= ke) {                 // uniform over the workgroup
                const bool plt = p < nz, pint = p > 0 && p < nz;
                // ---- Faraday: H^(t) at plane p from E^(t-1) at p and p+1 ----
                if constexpr (NW > 1) {
                    s_e[w][lane] = make_float2(Eo[0][0], Eo[2][0]);
                    __syncthreads();
                }
                const float2 eup = NW > 1 ? s_e[w + 1][lane] : make_float2(0.0f, 0.0f);
                float Hn[3][RY];
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int y = yw + r;
                    const bool in = xin && y >= 0 && y <= ny;
                    const float exu = r + 1 < RY ? Eo[0][(r + 1) % RY] : eup.x;
                    const float ezu = r + 1 < RY ? Eo[2][(r + 1) % RY] : eup.y;
                    const float ezr = from_right(Eo[2][r]);
                    const float eyr = from_right(Eo[1][r]);
                    const float dey_z = E[t - 1][1][r] - Eo[1][r];
                    const float dez_y = ezu - Eo[2][r];
                    const float hx = __builtin_fmaf(-a.chy, dez_y, __builtin_fmaf(a.chz, dey_z, Ho[0][r]));
                    const float dez_x = ezr - Eo[2][r];
                    const float dex_z = E[t - 1][0][r] - Eo[0][r];
                    const float hy = __builtin_fmaf(-a.chz, dex_z, __builtin_fmaf(a.chx, dez_x, Ho[1][r]));
                    const float dex_y = exu - Eo[0][r];
                    const float dey_x = eyr - Eo[1][r];
                    const float hz = __builtin_fmaf(-a.chx, dey_x, __builtin_fmaf(a.chy, dex_y, Ho[2][r]));
                    Hn[0][r] = (in && y < ny && plt) ? hx : Ho[0][r];
                    Hn[1][r] = (in && xlt && plt) ? hy : Ho[1][r];
                    Hn[2][r] = (in && xlt && y < ny) ? hz : Ho[2][r];
                }
                // ---- Ampere: E^(t) at plane p from H^(t) at p and p-1 ----
                if constexpr (NW > 1) {
                    s_h[w + 1][lane] = make_float2(Hn[0][RY - 1], Hn[2][RY - 1]);
                    __syncthreads();
                }
                const float2 hdn = NW > 1 ? s_h[w][lane] : make_float2(0.0f, 0.0f);
                float En[3][RY];
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int y = yw + r;
                    const bool in = xin && y >= 0 && y <= ny;
                    const bool yint = y > 0 && y < ny;
                    const float hxd = r > 0 ? Hn[0][(r + RY - 1) % RY] : hdn.x;
                    const float hzd = r > 0 ? Hn[2][(r + RY - 1) % RY] : hdn.y;
                    const float hzl = from_left(Hn[2][r]);
                    const float hyl = from_left(Hn[1][r]);
                    const float4 cf = s_coef[Mo[r]];
                    const float dhz_y = Hn[2][r] - hzd;
                    const float dhy_z = Hn[1][r] - H[t][1][r];
                    const float ex = __builtin_fmaf(-cf.w, dhy_z, __builtin_fmaf(cf.z, dhz_y, cf.x * Eo[0][r]));
                    const float dhx_z = Hn[0][r] - H[t][0][r];
                    const float dhz_x = Hn[2][r] - hzl;
                    const float ey = __builtin_fmaf(-cf.y, dhz_x, __builtin_fmaf(cf.w, dhx_z, cf.x * Eo[1][r]));
                    const float dhy_x = Hn[1][r] - hyl;
                    const float dhx_y = Hn[0][r] - hxd;
                    const float ez = __builtin_fmaf(-cf.z, dhx_y, __builtin_fmaf(cf.y, dhy_x, cf.x * Eo[2][r]));
                    En[0][r] = (in && xlt && yint && pint) ? ex : Eo[0][r];
                    En[1][r] = (in && y < ny && xint && pint) ? ey : Eo[1][r];
                    En[2][r] = (in && plt && xint && yint) ? ez : Eo[2][r];
                }
                // ---- soft sources of step step0+t-1, on every tile computing the edge ----
                const long long n = a.step0 + (t - 1);
                for (int q = 0; q < a.src.n; ++q) {
                    const int4 d = a.src.pos[q];
                    if (d.w != p) continue;
                    const int2 wv = a.src.wave[q];
                    if (n >= wv.y) continue;
                    const int lx = d.y - xl, ry = d.z - yt;
                    if (lx < 0 || lx >= 64 || ry < 0 || ry >= NR || ry / RY != w) continue;
                    const float val = a.src.samples[wv.x + n];
                    if (lane == lx) {
#pragma unroll
                        for (int r = 0; r < RY; ++r)
                            if (r == ry - w * RY) {
                                if (d.x == 0) En[0][r] = En[0][r] + val;
                                else if (d.x == 1) En[1][r] = En[1][r] + val;
                                else En[2][r] = En[2][r] + val;
                            }
                    }
                }
                // ---- probes, recorded by the owning tile only: planes outside
                // [z0, z1) are this chunk's warm-up/drain halo, where upper time
                // levels are incomplete ----
                for (int q = 0; q < a.probe.n; ++q) {
                    const int4 d = a.probe.pos[q];
                    if (d.w != p || p < z0 || p >= z1) continue;
                    const int lx = d.y - xl, ry = d.z - yt;
                    if (lx < T || lx >= T + OX || ry < T || ry >= T + OY || ry / RY != w) continue;
                    if (lane == lx) {
                        float v = 0.0f;
#pragma unroll
                        for (int r = 0; r < RY; ++r)
                            if (r == ry - w * RY) {
                                v = d.x == 0 ? En[0][r] : d.x == 1 ? En[1][r] : d.x == 2 ? En[2][r]
                                  : d.x == 3 ? Hn[0][r] : d.x == 4 ? Hn[1][r] : Hn[2][r];
                            }
                        a.probe.out[(n - a.probe.base) * a.probe.n + q] = (double)v;
                    }
                }
                // ---- rotate: level t's previous plane becomes level t+1's input ----
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int mt = M[t][r];
                    M[t][r] = Mo[r];
                    Mo[r] = mt;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float et = E[t][c][r], ht = H[t][c][r];
                        E[t][c][r] = En[c][r];
                        H[t][c][r] = Hn[c][r];
                        Eo[c][r] = et;
                        Ho[c][r] = ht;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    Mo[r] = M[t][r];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Eo[c][r] = E[t][c][r];
                        Ho[c][r] = H[t][c][r];
                    }
                }
            }
        }

        // ---- store the owned part of level T (plane K-T) ----
        const int q = K - T;
        if (q >= z0 && q < z1) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int row = w * RY + r;
                const int y = yw + r;
                if (xown && row >= T && row < T + OY && y <= ny) {
                    const long long off = (long long)q * L.plane + (long long)y * L.pitch + x;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Codec::store(fout + c * cs + off, E[T][c][r], up[c], mx[c], flag);
                        Codec::store(fout + (3 + c) * cs + off, H[T][c][r], up[3 + c], mx[3 + c], flag);
                    }
                }
            }
        }
    }
#undef YEE_LOAD_PLANE

    if constexpr (Codec::scaled) {
        // largest stored magnitude per component and the saturation flag
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float m = Codec::decode_mag(mx[c], 1.0f / up[c]);
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
            if (lane == 0 && m > 0.0f) atomicMax(&a.sb.ctrl->maxbits[a.sb.slot_out][c], __float_as_uint(m));
        }
        const unsigned long long any = __ballot(flag != 0u);
        if (lane == 0 && any) atomicOr(&a.sb.ctrl->flag, 1u);
    }
}

template <int T>
void geometry(const Layout &L, int *ntx, int *nty, int *ntz, int *zc, int *threads)
{
    constexpr int OX = 64 - 2 * T, OY = Shape<T>::NW * Shape<T>::RY - 2 * T;
    *ntx = (L.nx + 1 + OX - 1) / OX;
    *nty = (L.ny + 1 + OY - 1) / OY;
    // Enough z chunks for ~8 workgroups per CU, each chunk at least 8T planes deep.
    const int per_plane = *ntx * *nty;
    int want = (2048 + per_plane - 1) / per_plane;
    int maxc = (L.nz + 1) / (8 * T);
    if (maxc < 1) maxc = 1;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    *zc = (L.nz + 1 + want - 1) / want;
    *ntz = (L.nz + 1 + *zc - 1) / *zc;
    *threads = 64 * Shape<T>::NW;
}

template <int T, class Codec>
hipError_t launch_t(const FusedArgs &a0, hipStream_t st)
{
    FusedArgs a = a0;
    int threads;
    geometry<T>(a.L, &a.ntx, &a.nty, &a.ntz, &a.zc, &threads);
    a.nwg = a.ntx * a.nty * a.ntz;
    const int grid = (a.nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((yee_fused<T, Codec>), dim3(grid), dim3(threads), 0, st, a);
    return hipGetLastError();
}

template <class Codec>
hipError_t launch_codec(int T, const FusedArgs &a, hipStream_t st)
{
    switch (T) {
    case 1: return launch_t<1, Codec>(a, st);
    case 2: return launch_t<2, Codec>(a, st);
    case 3: return launch_t<3, Codec>(a, st);
    case 4: return launch_t<4, Codec>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

void fused_geometry(int T, const Layout &L, int *ntx, int *nty, int *ntz, int *zc, int *threads)
{
    switch (T) {
    case 1: geometry<1>(L, ntx, nty, ntz, zc, threads); break;
    case 2: geometry<2>(L, ntx, nty, ntz, zc, threads); break;
    case 3: geometry<3>(L, ntx, nty, ntz, zc, threads); break;
    default: geometry<4>(L, ntx, nty, ntz, zc, threads); break;
    }
}

hipError_t launch_fused(int storage, int T, const FusedArgs &a, hipStream_t st)
{
    switch (storage) {
    case 0: return launch_codec<CodecF32>(T, a, st);
    case 1: return launch_codec<CodecF16>(T, a, st);
    case 2: return launch_codec<CodecBF16>(T, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace yee
