// Fused, temporally blocked Yee kernel: one pass over HBM advances T steps.
//
// This is the GPU form of the cache-reuse ideas of Sec. 3: Ampere and
// Faraday interleaved per sub-domain (Sec. 3.2), plane by plane along z
// (Sec. 3.3), several time steps gathered per pass (Sec. 3.4, generalised
// to T steps as the conclusion suggests).  On a GPU the "cache" is the
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
// lanes with DPP wave shifts; the y neighbour across a wave boundary goes
// through LDS, with one barrier per time level.  Each level computes only
// the planes of its dependency cone within the chunk.  Fields are read from
// buffer fin and the advanced state is written to buffer fout (ping-pong):
// an in-place update would race with neighbouring tiles still reading the
// old time level.
//
// Graded spacing (GR): the c dt / size factors come from per-index arrays --
// x per lane and y per row, both fixed for the tile and held in registers,
// and z per plane, loaded with the plane prefetch and shifted through the
// levels like the material indices.  An E coefficient is the material's G
// times the dual-size factor, formed in FP32 before its fma.
//
// Zero tiles (Sec. 4.2 leaves out sub-domains whose fields are all zero):
// the host tracks a box holding every value that may differ from
// +0 in the input state (it grows by one node per step on each axis, the
// reach of the stencil) and every source point active in the launch.  A tile
// whose loaded region misses that box would compute +0 everywhere -- every
// difference is +0, and fma(c, +0, +0) and Ca * (+0) round to zeros that the
// next fma turns into +0 -- and its owned region of the output buffer already
// holds +0 (an older state, inside a smaller box).  Such tiles are not
// launched: the grid covers only the box of tiles meeting the value box
// (offsets tx0, ty0, tz0), and the probe rows of the others keep the 0 they
// were allocated with.
// Dead tiles: inside a perfect conductor, a node whose E edges are all
// conductor-owned (Ca = Cb = 0, so every update writes +0) and whose H values
// see only such edges (a zero curl) keeps +0 for good once it holds +0.  The
// host lists the tiles owning a node that is not dead; the launch walks that
// list, and a listed tile missing the value box exits at once.
//
// Addressing: every array is read through a buffer resource based at the
// chunk's first plane; the per-lane x offset lives in one VGPR and the plane
// and row offsets are scalar, so a load costs one instruction.  Halo lanes
// and rows outside the grid read clamped (in-grid) addresses: their values
// only ever feed other halo values, never an owned output.

#pragma once

#include <algorithm>
#include <type_traits>

#include "yee_device.hpp"
#include "yee_internal.hpp"

namespace yee {

namespace {

constexpr int BUF_FLAGS = 0x00020000;   // raw (untyped) dword buffer, gfx9 word 3

// Read-only data at wave-uniform addresses, read through the constant address
// space so that the loads are scalar (s_load) and leave the vector memory
// counter to the plane prefetch.
typedef __attribute__((address_space(4))) const float ConstFloat;

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, long long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, BUF_FLAGS);
}

// Loads return the stored payload (Raw); decode() turns it into an FP32 field
// value.  The prefetched plane is held raw and decoded only when it enters the
// pipeline one z step later, so the decode does not wait for the load.
template <class Codec> struct Buf;
template <> struct Buf<CodecF32> {
    using Raw = float;
    __device__ static inline Raw load(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static inline float decode(Raw v, float) { return v; }
    __device__ static inline void store(__amdgpu_buffer_rsrc_t r, int vo, int so, float v, float, uint32_t &, bool)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, 0);
    }
};
template <class Codec> struct Buf16 {
    using Raw = uint16_t;
    __device__ static inline Raw load(__amdgpu_buffer_rsrc_t r, int vo, int so)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    }
    __device__ static inline float decode(Raw q, float down) { return Codec::load(&q, down); }
    __device__ static inline void store(__amdgpu_buffer_rsrc_t r, int vo, int so, float v, float up, uint32_t &mx,
                                        bool own)
    {
        __builtin_amdgcn_raw_buffer_store_b16(Codec::encode_tracked(v, up, mx, own), r, vo, so, 0);
    }
};
template <> struct Buf<CodecF16> : Buf16<CodecF16> {};
template <> struct Buf<CodecBF16> : Buf16<CodecBF16> {};

constexpr int MAX_LOCAL = 256;   // sources / probes per solver

template <int T, int NW>
struct TileShared {
    // The exchange rows come first, so that every access is one per-lane base
    // register plus an immediate offset.
    // (Hx, Hz) of each wave's last row, in slot w+1, in buffer t % NHB at level
    // t: consecutive levels, also across z steps, use different buffers, so
    // one barrier per level orders both the write and the reuse; slot 0 stays
    // zero.
    static constexpr int NHB = (T & 1) ? 3 : 2;
    float2 h[NHB][NW + 1][64];
    // (Ex, Ez) of each wave's first row, per time level 0..T-1: level t's row
    // of z step K is written once level t+1 has read step K-1's row (after
    // that level's barrier) and read by level t+1 in step K+1; slot NW stays
    // zero.
    float2 e[T][NW + 1][64];
    float4 coef[256];
    int4 src[MAX_LOCAL];     // sources this workgroup computes: (comp, lane, row, plane)
    int srcn[MAX_LOCAL];     // how many of this launch's T steps have a sample
    float srcv[MAX_LOCAL][T];  // those samples, staged so the z march issues no
                               // global loads besides the plane prefetch
    int4 prb[MAX_LOCAL];     // probes this workgroup owns: (comp, lane, row, plane)
    int prbid[MAX_LOCAL];
    int nsrc, nprb;
    uint32_t vmax[6];        // largest |value| per component over the tile, as bits
};

// One tile (x-y tile x z chunk) of one solve: T steps of the owned region.
// `logical` is the tile index within the solve.  Starts and ends with every
// thread of the workgroup in step, so a workgroup may run several tiles in a
// row (the batched kernel does).
// Tile coordinates of work item `logical`: from the launched range of tiles,
// or from a list of the tiles owning a live node (indices into the full
// tiling).  False for a listed tile outside the range -- it misses the value
// box, so it would only rewrite +0 -- except item 0, which runs anyway: it
// publishes the next block's scales.
__device__ __forceinline__ bool tile_coords(const FusedArgs &a, const int logical, int &tx, int &ty, int &tz)
{
    if (!a.tiles) {
        const int rem = logical / a.ntx;
        tx = a.tx0 + logical % a.ntx;
        ty = a.ty0 + rem % a.nty;
        tz = a.tz0 + rem / a.nty;
        return true;
    }
    const int t = a.tiles[logical];
    const int rem = t / a.ltx;
    tx = t % a.ltx;
    ty = rem % a.lty;
    tz = rem / a.lty;
    return logical == 0 || (tx >= a.tx0 && tx < a.tx0 + a.ntx && ty >= a.ty0 && ty < a.ty0 + a.nty &&
                            tz >= a.tz0 && tz < a.tz0 + a.ntz);
}

// EN: the pass also sums the energy of its input state at one time level
// (EnergyFused), over the values this tile owns, into en.partial[logical];
// s_en holds half of each material's eps_r, then the per-wave sums.
template <int T, int RY, int NW, class Codec, bool GR = false, bool CP = false, bool EN = false>
__device__ __forceinline__ void fused_tile(const FusedArgs &a, const int logical, const int tx, const int ty,
                                           const int tz, TileShared<T, NW> &sm, const CpmlFused &cpa = {},
                                           const EnergyFused &en = {}, double *s_en = nullptr)
{
    constexpr int OX = 64 - 2 * T;      // owned points per tile in x
    constexpr int NR = NW * RY;         // rows per tile
    constexpr int OY = NR - 2 * T;      // owned rows per tile
    using S = typename Codec::T;
    using B = Buf<Codec>;
    constexpr int ES = sizeof(S);
    float4 *const s_coef = sm.coef;
    auto &s_e = sm.e;
    auto &s_h = sm.h;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int q = tid; q < a.n_mat; q += 64 * NW) s_coef[q] = a.coef[q];
    if constexpr (EN)
        for (int q = tid; q < a.n_mat; q += 64 * NW) s_en[q] = en.half_eps[q];
    if (tid < 64) {
        for (int t = 0; t < T; ++t) s_e[t][NW][tid] = make_float2(0.0f, 0.0f);
        for (int b = 0; b < TileShared<T, NW>::NHB; ++b) s_h[b][0][tid] = make_float2(0.0f, 0.0f);
    }

    float dn[6], up[6];
    if constexpr (Codec::scaled) {
        float mprev[6];
        int s_in[6], s_out[6];
        Ctrl *const ctrl = a.sb.ctrl;
        // the stored maxima of the input: of its block's second pass if it ran
        const bool retried_in = ctrl->ovf[a.sb.slot_in] != 0u;
        for (int c = 0; c < 6; ++c) {
            mprev[c] = __uint_as_float(retried_in ? ctrl->rmaxbits[a.sb.slot_in][c] : ctrl->maxbits[a.sb.slot_in][c]);
            s_in[c] = ctrl->scale[a.sb.par][c];
        }
        choose_scales(mprev, a.sb.a_max, s_out);
        if (a.sb.retry) {                // the components that overflowed take their own block's scale
            const uint32_t ov = ctrl->ovf[a.sb.slot_out];
            for (int c = 0; c < 6; ++c)
                if ((ov >> c) & 1u) {
                    const float pm = __uint_as_float(ctrl->premax[a.sb.slot_out][c]);
                    s_out[c] = scale_from(pm > a.sb.a_max ? pm : a.sb.a_max);
                }
        }
        for (int c = 0; c < 6; ++c) {   // uniform: keep them in scalar registers
            dn[c] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                        __builtin_bit_cast(int, ldexpf(1.0f, -s_in[c]))));
            up[c] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                        __builtin_bit_cast(int, ldexpf(1.0f, s_out[c]))));
        }
        if (logical == 0 && tid < 6) {
            ctrl->scale[a.sb.par ^ 1][tid] = s_out[tid];
            if (!a.sb.retry) {
                ctrl->maxbits[a.sb.slot_clear][tid] = 0u;
                ctrl->rmaxbits[a.sb.slot_clear][tid] = 0u;
                ctrl->premax[a.sb.slot_clear][tid] = 0u;
                if (tid == 0) ctrl->ovf[a.sb.slot_clear] = 0u;
            }
        }
    } else {
        for (int c = 0; c < 6; ++c) dn[c] = up[c] = 1.0f;
    }

    const Layout L = a.L;
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int x0 = tx * OX, y0 = ty * OY, z0 = tz * a.zc;
    const int z1 = min(z0 + a.zc, nz + 1);
    const int xl = x0 - T;              // x of lane 0
    const int x = xl + lane;
    const int yt = y0 - T;              // y of the tile's first row
    const int yw = yt + w * RY;         // y of this wave's first row
    const int kb = max(0, z0 - T);      // first plane the pipeline loads
    const int ke = min(nz, z1 - 1 + T); // last plane the pipeline loads

    // sources on points this tile computes, probes on points it owns
    if (tid == 0) {
        int ns = 0, np = 0;
        for (int q = 0; q < a.src.n; ++q) {
            const int4 d = a.src.pos[q];
            const int lx = d.y - xl, ry = d.z - yt;
            if (lx >= 0 && lx < 64 && ry >= 0 && ry < NR && d.w >= kb && d.w <= ke && ns < MAX_LOCAL) {
                sm.src[ns] = make_int4(d.x, lx, ry, d.w);
                const int2 wv = a.src.wave[q];     // (sample offset, n_samples)
                const long long left = (long long)wv.y - a.step0;
                const int nv = left < 0 ? 0 : (left > T ? T : (int)left);
                sm.srcn[ns] = nv;
                for (int t = 0; t < nv; ++t) sm.srcv[ns][t] = a.src.samples[wv.x + a.step0 + t];
                ++ns;
            }
        }
        for (int q = 0; q < a.probe.n; ++q) {
            const int4 d = a.probe.pos[q];
            const int lx = d.y - xl, ry = d.z - yt;
            if (lx >= T && lx < T + OX && ry >= T && ry < T + OY && d.w >= z0 && d.w < z1 && np < MAX_LOCAL) {
                sm.prb[np] = make_int4(d.x, lx, ry, d.w);
                sm.prbid[np] = q;
                ++np;
            }
        }
        sm.nsrc = ns;
        sm.nprb = np;
    }
    if (tid < 6) sm.vmax[tid] = 0u;
    __syncthreads();
    const int nsrc = sm.nsrc, nprb = sm.nprb;

    // lane and row predicates
    // Walls.  Values at positions outside their component's range (Hy, Hz
    // and Ex at x = nx; Hx, Hz and Ey at y = ny) and on lanes and rows beyond
    // the walls are computed like the rest and never feed a value in range:
    // every difference that reaches across a wall ends on a tangential E of
    // that wall, which is held at its stored zero.  So the updates mask only
    // the walls' tangential E (and the z walls, per plane), and the stores
    // write zero at the positions outside each component's range.
    const bool xwall = x == 0 || x == nx;
    const bool xlt = x < nx;
    const bool xint = x > 0 && x < nx;
    const bool xown = lane >= T && lane < T + OX && x <= nx;
    const int xc = min(max(x, 0), nx);
    const int vo = xc * ES;             // per-lane byte offset of the field arrays
    // The material index's per-lane byte offset, xc, is formed from vo at each
    // load (one shift; the asm keeps the compiler from hoisting it into a
    // register of its own, one more live value through the whole march).
    auto mat_offset = [&]() __attribute__((always_inline)) -> int {
        int m;
        asm volatile("v_lshrrev_b32 %0, %1, %2" : "=v"(m) : "n"(ES == 4 ? 2 : 1), "v"(vo));
        return m;
    };

    // buffer resources based at this chunk's first plane
    const long long cs = L.cstride, ks = L.kstride;
    const __amdgpu_buffer_rsrc_t rin = rsrc(static_cast<const S *>(a.fin) + (long long)kb * ks,
                                            (long long)(ke - kb + 1) * ks * ES);
    const __amdgpu_buffer_rsrc_t rout = rsrc(static_cast<S *>(a.fout) + (long long)kb * ks,
                                             (long long)(ke - kb + 1) * ks * ES);
    const __amdgpu_buffer_rsrc_t rmat = rsrc(a.mat + (long long)kb * L.plane, (long long)(ke - kb + 1) * L.plane);
    int rowoff[RY];                     // clamped row offsets (elements), uniform per wave
#pragma unroll
    for (int r = 0; r < RY; ++r) rowoff[r] = min(max(yw + r, 0), ny) * L.pitch;

    // graded spacing: (c dt / primal size, c dt / dual size) of this lane's x,
    // of each row's y (uniform per wave) and of each level's z plane
    float gxh = 0.0f, gxe = 0.0f, gyh[RY], gye[RY], gzh[T + 1], gze[T + 1];
    float2 PZ = make_float2(0.0f, 0.0f);
    ConstFloat *const gcu = (ConstFloat *)a.gc;   // pairs: element 2q, 2q+1
    if constexpr (GR) {
        const float2 gx = a.gc[xc];
        gxh = gx.x;
        gxe = gx.y;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int q = 2 * (nx + 1 + min(max(yw + r, 0), ny));
            gyh[r] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, gcu[q])));
            gye[r] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, gcu[q + 1])));
        }
#pragma unroll
        for (int t = 0; t <= T; ++t) gzh[t] = gze[t] = 0.0f;
    }

    // CPML layers (CP): membership of this lane's x, of each row's y (uniform)
    // and, per level, of its plane (uniform) in the slabs of the auxiliary
    // state psi.  H values at a cell q < n belong when q < N or q >= n - N, E
    // values at a node when 0 < q < N or n - N < q < n; the slab slot of q is
    // q (lower layer) or q - n + 2N (upper).  The x-type psi offsets of lanes
    // outside a slab (and, for stores, of lanes this tile does not own) lie
    // 2^31 beyond the array, where loads read 0 and stores are dropped.
    static_assert(!CP || (GR && std::is_same<Codec, CodecF32>::value), "CPML layers: graded FP32 kernels");
    constexpr int NPS = CP ? 12 : 1;
    const int N = CP ? cpa.pml.n : 0;
    bool xph = false, xpe = false, tile_x = false, tile_xy = false;
    int vpx = 0, vpxs = 0;
    float cxp[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // {b_h, a_h, c dt/d, b_e, a_e, c dt/d'} of x
    bool yph[RY], ype[RY];
    int ysl[RY];
    const __amdgpu_buffer_rsrc_t rpsi = rsrc(CP ? cpa.pml.psi : nullptr, CP ? cpa.pml.elems * 4 : 0);
    const __amdgpu_buffer_rsrc_t rpso = rsrc(CP ? cpa.psi_out : nullptr, CP ? cpa.pml.elems * 4 : 0);
    ConstFloat *const cpu = (ConstFloat *)cpa.pml.cp;
    if constexpr (CP) {
        xph = x >= 0 && x < nx && (x < N || x >= nx - N);
        xpe = (x > 0 && x < N) || (x > nx - N && x < nx);
        const int slot = x < N ? x : x - nx + 2 * N;
        vpx = xph ? slot * 16 : (int)0x80000000u;
        vpxs = (xph && xown) ? slot * 16 : (int)0x80000000u;
        tile_x = xl < N || xl + 63 >= nx - N;            // some lane in an x slab
        tile_xy = tile_x || yt < N || yt + NR - 1 >= ny - N;
        if (tile_x) {
#pragma unroll
            for (int c = 0; c < 6; ++c) cxp[c] = cpa.pml.cp[6 * xc + c];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = yw + r;
            yph[r] = y >= 0 && y < ny && (y < N || y >= ny - N);
            ype[r] = (y > 0 && y < N) || (y > ny - N && y < ny);
            ysl[r] = y < N ? y : y - ny + 2 * N;
        }
    }
    // psi of level t at its latest plane (level 0: loaded, plane K), and the
    // level below's previous plane, handed up one level per z step
    float PS[CP ? T : 1][NPS][RY], PSo[NPS][RY];
#pragma unroll
    for (int c = 0; c < NPS; ++c)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            PSo[c][r] = 0.0f;
#pragma unroll
            for (int t = 0; t < (CP ? T : 1); ++t) PS[t][c][r] = 0.0f;
        }
    // psi of plane K into PS[0]: one 16-byte group per type, zero outside the
    // slabs
    const int vg = vo * 4;              // per-lane byte offset of a group at index x
    auto group = [&](const int axis, const int g) __attribute__((always_inline)) -> int {
        return (int)(cpa.pml.base[axis] + 4LL * g) * 4;   // bytes; the arrays fit 2^31
    };
    auto load_psi = [&](const int K) __attribute__((always_inline)) {
        const bool zin = K < nz && (K < N || K >= nz - N);
        const int zsl = K < N ? K : K - nz + 2 * N;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yc = min(max(yw + r, 0), ny);
            auto put = [&](const int first, const uint4 v) __attribute__((always_inline)) {
                PS[0][first + 0][r] = __builtin_bit_cast(float, v.x);
                PS[0][first + 1][r] = __builtin_bit_cast(float, v.y);
                PS[0][first + 2][r] = __builtin_bit_cast(float, v.z);
                PS[0][first + 3][r] = __builtin_bit_cast(float, v.w);
            };
            const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
            auto ld = [&](const int vofs, const int so) __attribute__((always_inline)) -> uint4 {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(rpsi, vofs, so, 0);
                return make_uint4(v[0], v[1], v[2], v[3]);
            };
            put(PS_HYX, tile_x ? ld(vpx, group(0, (K * (ny + 1) + yc) * 2 * N)) : zero);
            put(PS_HXY, yph[r] ? ld(vg, group(1, (K * 2 * N + ysl[r]) * (nx + 1))) : zero);
            put(PS_HXZ, zin ? ld(vg, group(2, (zsl * (ny + 1) + yc) * (nx + 1))) : zero);
        }
    };
    // level T's psi of plane q: the values this tile owns (every slab entry of
    // an owned node is written, updated or passed through)
    const int vgs = xown ? vg : (int)((uint32_t)vg | 0x80000000u);
    auto store_psi = [&](const int q, const float (&V)[NPS][RY]) __attribute__((always_inline)) {
        const bool zin = q < nz && (q < N || q >= nz - N);
        const int zsl = q < N ? q : q - nz + 2 * N;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int row = w * RY + r;
            const int y = yw + r;
            if (!(row >= T && row < NR - T && y <= ny)) continue;    // uniform
            auto st = [&](const int first, const int vofs, const int so) __attribute__((always_inline)) {
                typedef unsigned int u4 __attribute__((ext_vector_type(4)));
                const u4 v = {__builtin_bit_cast(uint32_t, V[first][r]), __builtin_bit_cast(uint32_t, V[first + 1][r]),
                              __builtin_bit_cast(uint32_t, V[first + 2][r]), __builtin_bit_cast(uint32_t, V[first + 3][r])};
                __builtin_amdgcn_raw_buffer_store_b128(v, rpso, vofs, so, 0);
            };
            if (tile_x) st(PS_HYX, vpxs, group(0, (q * (ny + 1) + y) * 2 * N));
            if (yph[r]) st(PS_HXY, vgs, group(1, (q * 2 * N + ysl[r]) * (nx + 1)));
            if (zin) st(PS_HXZ, vgs, group(2, (zsl * (ny + 1) + y) * (nx + 1)));
        }
    };

    float E[T + 1][3][RY], H[T + 1][3][RY];
    // Material indices of the planes the levels are on, one byte per level:
    // byte t-1 of MP[r] is the index of plane K-t (level t's plane) in row r,
    // for t = 1..T.  The material of plane K-1 is loaded during step K-1 and
    // shifted in at step K.
    using MPack = typename std::conditional<(T >= 5), uint64_t, uint32_t>::type;
    MPack MP[RY];
#pragma unroll
    for (int t = 0; t <= T; ++t)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (t == 0) MP[r] = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) E[t][c][r] = H[t][c][r] = 0.0f;
        }

    // prefetched next level-0 plane
    typename B::Raw PE[3][RY], PH[3][RY];
    uint32_t PM[RY];

#define YEE_LOAD_PLANE(KK)                                                                  \
    do {                                                                                    \
        const int pofs_ = ((KK) - kb) * (int)ks;                                            \
        const int mofs_ = (max((KK) - 1, kb) - kb) * (int)L.plane;                         \
        _Pragma("unroll") for (int r = 0; r < RY; ++r) {                                    \
            const int so_ = pofs_ + rowoff[r];                                              \
            _Pragma("unroll") for (int c = 0; c < 3; ++c) {                                 \
                PE[c][r] = B::load(rin, vo, (so_ + c * (int)cs) * ES);                      \
                PH[c][r] = B::load(rin, vo, (so_ + (3 + c) * (int)cs) * ES);                \
            }                                                                               \
            PM[r] = __builtin_amdgcn_raw_buffer_load_b8(rmat, mat_offset(), mofs_ + rowoff[r], 0); \
        }                                                                                   \
        if constexpr (GR) PZ = make_float2(gcu[2 * (nx + ny + 2 + (KK))],                   \
                                           gcu[2 * (nx + ny + 2 + (KK)) + 1]);              \
    } while (0)


    uint32_t mx[6] = {0u, 0u, 0u, 0u, 0u, 0u};   // largest |value| stored, as bits

    // Store the owned part of level T, which holds plane q.  Every lane and row
    // issues its stores, without branches: a value this tile does not own gets
    // an offset 2^31 beyond its address, which the buffer range check drops.
    // (Loads and stores share one completion counter; stores inside branches
    // make the compiler's wait for the next plane's loads also wait for them.)
    // INNER tiles own no position outside a component's range; elsewhere those
    // positions are stored as zero (Ex, Hy at x = nx; Ey, Hx at y = ny; Hz on
    // both; the z walls keep their zeros through the plane masks).
    auto store_plane = [&](const int q, auto inner_c) __attribute__((always_inline)) {
        constexpr bool INNER = decltype(inner_c)::value;
        const int pofs = (q - kb) * (int)ks;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int row = w * RY + r;
            const int y = yw + r;
            const bool own = xown && row >= T && row < T + OY && y <= ny;
            const int vs = own ? vo : (int)((uint32_t)vo | 0x80000000u);
            const int so = (pofs + rowoff[r]) * ES;
            float ev[3] = {E[T][0][r], E[T][1][r], E[T][2][r]};
            float hv[3] = {H[T][0][r], H[T][1][r], H[T][2][r]};
            if constexpr (!INNER) {
                const bool ylt = y < ny;                // uniform over the wave
                ev[0] = xlt ? ev[0] : 0.0f;
                ev[1] = ylt ? ev[1] : 0.0f;
                hv[0] = ylt ? hv[0] : 0.0f;
                hv[1] = xlt ? hv[1] : 0.0f;
                hv[2] = (xlt && ylt) ? hv[2] : 0.0f;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                B::store(rout, vs, so + c * (int)cs * ES, ev[c], up[c], mx[c], own);
                B::store(rout, vs, so + (3 + c) * (int)cs * ES, hv[c], up[3 + c], mx[3 + c], own);
            }
        }
    };

    // One z step of the pipeline.  ALL: every time level is active, the next
    // plane is loaded and an owned plane is stored (steady state), so no
    // per-level branches remain.
    // INNER: every lane and row of the tile lies strictly inside the grid in
    // x and y (no wall in reach), so only the plane tests remain in the masks.
    // Otherwise only the tangential E of the x and y walls is held.
    // energy of the recorded level's input state over the owned values (EN)
    double eacc = 0.0;

    // PSI: a step that carries psi (CP kernels only; steps of a tile outside
    // every slab leave the all-zero psi registers alone).
    auto iterate = [&](const int K, auto all_c, auto inner_c, auto psi_c) __attribute__((always_inline)) {
        constexpr bool ALL = decltype(all_c)::value;
        constexpr bool INNER = decltype(inner_c)::value;
        constexpr bool PSI = CP && decltype(psi_c)::value;
        // Level 0 takes plane K; plane K-1 of level 0 becomes level 1's input.
        float Eo[3][RY], Ho[3][RY];
        if constexpr (GR) {
#pragma unroll
            for (int t = T; t > 0; --t) {
                gzh[t] = gzh[t - 1];
                gze[t] = gze[t - 1];
            }
            gzh[0] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, PZ.x)));
            gze[0] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, PZ.y)));
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            MP[r] = (MP[r] << 8) | (MPack)PM[r];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Eo[c][r] = E[0][c][r];
                Ho[c][r] = H[0][c][r];
                E[0][c][r] = B::decode(PE[c][r], dn[c]);
                H[0][c][r] = B::decode(PH[c][r], dn[3 + c]);
            }
        }
        if (ALL || K + 1 <= ke) YEE_LOAD_PLANE(K + 1);
        if constexpr (PSI) {
            // level 1 takes plane K-1's psi; plane K's is loaded for the next step
#pragma unroll
            for (int c = 0; c < NPS; ++c)
#pragma unroll
                for (int r = 0; r < RY; ++r) PSo[c][r] = PS[0][c][r];
            if (ALL || K <= ke) load_psi(K);
        }

#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int p = K - t;                      // plane of time level t
            // Level t is computed on planes [lo, hi]: its dependency cone.  Its
            // values are exact on [kb+t, ke-t] (walls aside), and level t+1 needs
            // one plane below that for its own first exact plane.
            const int lo = kb > 0 ? kb + t - 1 : 0;
            const int hi = ke < nz ? ke - t : nz;
            if (ALL || (p >= lo && p <= hi)) {        // uniform over the workgroup
                // steady steps keep every level off the z walls (0 < p < nz)
                const bool plt = ALL || p < nz, pint = ALL || (p > 0 && p < nz);
                // ---- Faraday: H^(t) at plane p from E^(t-1) at p and p+1 ----
                // E^(t-1) at plane p was computed in the previous z step, so the
                // row above is read from the exchange rows without a barrier.
                const float2 eup = NW > 1 ? s_e[t - 1][w + 1][lane] : make_float2(0.0f, 0.0f);
                float Hn[3][RY];
                const float chz = GR ? gzh[t] : a.chz;
                // CPML: the plane's layer membership and its z coefficients
                // {b_h, a_h, c dt/d, b_e, a_e, c dt/d'} (uniform)
                float PSn[NPS][RY];
                const bool zph = CP && p < nz && (p < N || p >= nz - N);
                const bool zpe = CP && ((p > 0 && p < N) || (p > nz - N && p < nz));
                float czp[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (CP && (zph || zpe)) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) czp[c] = cpu[6 * (nx + ny + 2 + p) + c];
                }
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int y = yw + r;
                    const float chx = GR ? gxh : a.chx, chy = GR ? gyh[r] : a.chy;
                    const float exu = r + 1 < RY ? Eo[0][(r + 1) % RY] : eup.x;
                    const float ezu = r + 1 < RY ? Eo[2][(r + 1) % RY] : eup.y;
                    const float ezr = from_right(Eo[2][r]);
                    const float eyr = from_right(Eo[1][r]);
                    const float dey_z = E[t - 1][1][r] - Eo[1][r];
                    const float dez_y = ezu - Eo[2][r];
                    float hx = __builtin_fmaf(-chy, dez_y, __builtin_fmaf(chz, dey_z, Ho[0][r]));
                    const float dez_x = ezr - Eo[2][r];
                    const float dex_z = E[t - 1][0][r] - Eo[0][r];
                    float hy = __builtin_fmaf(-chz, dex_z, __builtin_fmaf(chx, dez_x, Ho[1][r]));
                    const float dex_y = exu - Eo[0][r];
                    const float dey_x = eyr - Eo[1][r];
                    float hz = __builtin_fmaf(-chx, dey_x, __builtin_fmaf(chy, dex_y, Ho[2][r]));
                    if constexpr (PSI) {
                        // psi terms of each H value in a layer, in the order of its
                        // update (Hx: z then y, Hy: x then z, Hz: y then x), psi first:
                        // psi = b psi + a diff, then H +- (c dt/d) psi
                        const bool ylt = y < ny;
                        float cyp[3] = {0.0f, 0.0f, 0.0f};
                        if (yph[r]) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) cyp[c] = cpu[6 * (nx + 1 + y) + c];
                        }
                        auto keep = [&](const int c) __attribute__((always_inline)) { PSn[c][r] = PSo[c][r]; };
                        if (zph && ylt) {
                            const float ps = __builtin_fmaf(czp[0], PSo[PS_HXZ][r], czp[1] * dey_z);
                            hx = __builtin_fmaf(czp[2], ps, hx);
                            PSn[PS_HXZ][r] = ps;
                        } else keep(PS_HXZ);
                        if (yph[r] && plt) {
                            const float ps = __builtin_fmaf(cyp[0], PSo[PS_HXY][r], cyp[1] * dez_y);
                            hx = __builtin_fmaf(-cyp[2], ps, hx);
                            PSn[PS_HXY][r] = ps;
                        } else keep(PS_HXY);
                        if (tile_x && plt) {
                            const float ps = __builtin_fmaf(cxp[0], PSo[PS_HYX][r], cxp[1] * dez_x);
                            const float h2 = __builtin_fmaf(cxp[2], ps, hy);
                            hy = xph ? h2 : hy;
                            PSn[PS_HYX][r] = xph ? ps : PSo[PS_HYX][r];
                        } else keep(PS_HYX);
                        if (zph) {
                            const float ps = __builtin_fmaf(czp[0], PSo[PS_HYZ][r], czp[1] * dex_z);
                            const float h2 = __builtin_fmaf(-czp[2], ps, hy);
                            hy = xlt ? h2 : hy;
                            PSn[PS_HYZ][r] = xlt ? ps : PSo[PS_HYZ][r];
                        } else keep(PS_HYZ);
                        if (yph[r]) {
                            const float ps = __builtin_fmaf(cyp[0], PSo[PS_HZY][r], cyp[1] * dex_y);
                            const float h2 = __builtin_fmaf(cyp[2], ps, hz);
                            hz = xlt ? h2 : hz;
                            PSn[PS_HZY][r] = xlt ? ps : PSo[PS_HZY][r];
                        } else keep(PS_HZY);
                        if (tile_x && ylt) {
                            const float ps = __builtin_fmaf(cxp[0], PSo[PS_HZX][r], cxp[1] * dey_x);
                            const float h2 = __builtin_fmaf(-cxp[2], ps, hz);
                            hz = xph ? h2 : hz;
                            PSn[PS_HZX][r] = xph ? ps : PSo[PS_HZX][r];
                        } else keep(PS_HZX);
                    }
                    Hn[0][r] = plt ? hx : Ho[0][r];
                    Hn[1][r] = plt ? hy : Ho[1][r];
                    Hn[2][r] = hz;
                }
                // ---- energy W^n of level t's input state n = step0 + t - 1 ----
                // 1/2 eps_r E^n.E^n on interior edges (eps of the owner cell)
                // plus 1/2 H^(n-1/2).H^(n+1/2) on every H value in range: E^n and
                // H^(n-1/2) are level t-1's values at plane p, H^(n+1/2) the ones
                // just computed.  FP64 products and sums.
                if constexpr (EN) {
                    // owned planes only: in steady steps the lower levels also
                    // run on the halo planes past z1
                    if (t == en.level && p >= z0 && p < z1) {                // uniform
                        const bool zin = ALL || (p > 0 && p < nz), zlt = ALL || p < nz;
#pragma unroll
                        for (int r = 0; r < RY; ++r) {
                            const int row = w * RY + r;
                            const int y = yw + r;
                            if (!(row >= T && row < T + OY && y <= ny)) continue;   // uniform
                            const bool yin = y > 0 && y < ny, ylt = y < ny;
                            const double he = s_en[(uint32_t)(MP[r] >> (8 * (t - 1))) & 0xffu];
                            const double e0 = Eo[0][r], e1 = Eo[1][r], e2 = Eo[2][r];
                            double v = 0.0;
                            v = (xlt && yin && zin) ? __builtin_fma(he * e0, e0, v) : v;
                            v = (xint && ylt && zin) ? __builtin_fma(he * e1, e1, v) : v;
                            v = (xint && yin && zlt) ? __builtin_fma(he * e2, e2, v) : v;
                            v = (ylt && zlt) ? __builtin_fma(0.5 * (double)Ho[0][r], (double)Hn[0][r], v) : v;
                            v = (xlt && zlt) ? __builtin_fma(0.5 * (double)Ho[1][r], (double)Hn[1][r], v) : v;
                            v = (xlt && ylt) ? __builtin_fma(0.5 * (double)Ho[2][r], (double)Hn[2][r], v) : v;
                            eacc += xown ? v : 0.0;
                        }
                    }
                }
                // ---- Ampere: E^(t) at plane p from H^(t) at p and p-1 ----
                // Only row 0 needs the H row of the wave below: rows 1..RY-1 are
                // updated before the level's barrier, row 0 after it.
                // Consecutive levels alternate buffers (also across z steps), so
                // one barrier per level orders both the write and the reuse.
                float En[3][RY];
                auto e_row = [&](const int r, const float hxd, const float hzd) __attribute__((always_inline)) {
                    const int y = yw + r;
                    const bool ywall = y == 0 || y == ny;   // uniform over the wave
                    const float hzl = from_left(Hn[2][r]);
                    const float hyl = from_left(Hn[1][r]);
                    const float4 cf = s_coef[(uint32_t)(MP[r] >> (8 * (t - 1))) & 0xffu];
                    float cbx = cf.y, cby = cf.z, cbz = cf.w;
                    if constexpr (GR) {   // cf.y holds G
                        cbx = cf.y * gxe;
                        cby = cf.y * gye[r];
                        cbz = cf.y * gze[t];
                    }
                    const float dhz_y = Hn[2][r] - hzd;
                    const float dhy_z = Hn[1][r] - H[t][1][r];
                    float ex = __builtin_fmaf(-cbz, dhy_z, __builtin_fmaf(cby, dhz_y, cf.x * Eo[0][r]));
                    const float dhx_z = Hn[0][r] - H[t][0][r];
                    const float dhz_x = Hn[2][r] - hzl;
                    float ey = __builtin_fmaf(-cbx, dhz_x, __builtin_fmaf(cbz, dhx_z, cf.x * Eo[1][r]));
                    const float dhy_x = Hn[1][r] - hyl;
                    const float dhx_y = Hn[0][r] - hxd;
                    float ez = __builtin_fmaf(-cby, dhx_y, __builtin_fmaf(cbx, dhy_x, cf.x * Eo[2][r]));
                    if constexpr (PSI) {
                        // psi terms of each interior E edge in a layer (Ex: y then z,
                        // Ey: z then x, Ez: x then y), the factor G * (c dt/d') formed
                        // in FP32 before its fma
                        const float G = cf.y;
                        const bool ylt = y < ny, yint = y > 0 && y < ny;
                        float cye[3] = {0.0f, 0.0f, 0.0f};
                        if (ype[r]) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) cye[c] = cpu[6 * (nx + 1 + y) + 3 + c];
                        }
                        auto keep = [&](const int c) __attribute__((always_inline)) { PSn[c][r] = PSo[c][r]; };
                        if (ype[r] && pint) {
                            const float ps = __builtin_fmaf(cye[0], PSo[PS_EXY][r], cye[1] * dhz_y);
                            const float e2 = __builtin_fmaf(G * cye[2], ps, ex);
                            ex = xlt ? e2 : ex;
                            PSn[PS_EXY][r] = xlt ? ps : PSo[PS_EXY][r];
                        } else keep(PS_EXY);
                        if (zpe && yint) {
                            const float ps = __builtin_fmaf(czp[3], PSo[PS_EXZ][r], czp[4] * dhy_z);
                            const float e2 = __builtin_fmaf(-(G * czp[5]), ps, ex);
                            ex = xlt ? e2 : ex;
                            PSn[PS_EXZ][r] = xlt ? ps : PSo[PS_EXZ][r];
                        } else keep(PS_EXZ);
                        if (zpe && ylt) {
                            const float ps = __builtin_fmaf(czp[3], PSo[PS_EYZ][r], czp[4] * dhx_z);
                            const float e2 = __builtin_fmaf(G * czp[5], ps, ey);
                            ey = xint ? e2 : ey;
                            PSn[PS_EYZ][r] = xint ? ps : PSo[PS_EYZ][r];
                        } else keep(PS_EYZ);
                        if (tile_x && ylt && pint) {
                            const float ps = __builtin_fmaf(cxp[3], PSo[PS_EYX][r], cxp[4] * dhz_x);
                            const float e2 = __builtin_fmaf(-(G * cxp[5]), ps, ey);
                            ey = xpe ? e2 : ey;
                            PSn[PS_EYX][r] = xpe ? ps : PSo[PS_EYX][r];
                        } else keep(PS_EYX);
                        if (tile_x && plt && yint) {
                            const float ps = __builtin_fmaf(cxp[3], PSo[PS_EZX][r], cxp[4] * dhy_x);
                            const float e2 = __builtin_fmaf(G * cxp[5], ps, ez);
                            ez = xpe ? e2 : ez;
                            PSn[PS_EZX][r] = xpe ? ps : PSo[PS_EZX][r];
                        } else keep(PS_EZX);
                        if (ype[r] && plt) {
                            const float ps = __builtin_fmaf(cye[0], PSo[PS_EZY][r], cye[1] * dhx_y);
                            const float e2 = __builtin_fmaf(-(G * cye[2]), ps, ez);
                            ez = xint ? e2 : ez;
                            PSn[PS_EZY][r] = xint ? ps : PSo[PS_EZY][r];
                        } else keep(PS_EZY);
                    }
                    if constexpr (INNER) {
                        En[0][r] = pint ? ex : Eo[0][r];
                        En[1][r] = pint ? ey : Eo[1][r];
                        En[2][r] = plt ? ez : Eo[2][r];
                    } else {
                        En[0][r] = (!ywall && pint) ? ex : Eo[0][r];
                        En[1][r] = (!xwall && pint) ? ey : Eo[1][r];
                        En[2][r] = (!xwall && !ywall && plt) ? ez : Eo[2][r];
                    }
                };
                constexpr int NHB = TileShared<T, NW>::NHB;
                if constexpr (NW > 1) s_h[t % NHB][w + 1][lane] = make_float2(Hn[0][RY - 1], Hn[2][RY - 1]);
#pragma unroll
                for (int r = 1; r < RY; ++r) e_row(r, Hn[0][r - 1], Hn[2][r - 1]);
                if constexpr (NW > 1) {
                    __syncthreads();
                    const float2 hdn = s_h[t % NHB][w][lane];
                    // every wave has read level t-1's previous row: publish this step's
                    if constexpr (ALL) s_e[t - 1][w][lane] = make_float2(E[t - 1][0][0], E[t - 1][2][0]);
                    e_row(0, hdn.x, hdn.y);
                } else {
                    e_row(0, 0.0f, 0.0f);
                }
                // ---- soft sources of step step0+t-1, on every tile computing the edge ----
                const long long n = a.step0 + (t - 1);
                for (int q = 0; q < nsrc; ++q) {
                    const int4 d = sm.src[q];
                    if (d.w != p || t - 1 >= sm.srcn[q] || d.z / RY != w) continue;
                    const float val = sm.srcv[q][t - 1];
                    if (lane == d.y) {
#pragma unroll
                        for (int r = 0; r < RY; ++r)
                            if (r == d.z - w * RY) {
                                if (d.x == 0) En[0][r] = En[0][r] + val;
                                else if (d.x == 1) En[1][r] = En[1][r] + val;
                                else En[2][r] = En[2][r] + val;
                            }
                    }
                }
                // ---- probes, recorded by the owning tile only (planes outside
                // [z0, z1) are this chunk's halo, where upper levels are incomplete) ----
                for (int q = 0; q < nprb; ++q) {
                    const int4 d = sm.prb[q];
                    if (d.w != p || d.z / RY != w) continue;
                    if (lane == d.y) {
                        float v = 0.0f;
#pragma unroll
                        for (int r = 0; r < RY; ++r)
                            if (r == d.z - w * RY) {
                                v = d.x == 0 ? En[0][r] : d.x == 1 ? En[1][r] : d.x == 2 ? En[2][r]
                                  : d.x == 3 ? Hn[0][r] : d.x == 4 ? Hn[1][r] : Hn[2][r];
                            }
                        a.probe.out[(n - a.probe.base) * a.probe.n + sm.prbid[q]] = (double)v;
                    }
                }
                // ---- rotate: level t's previous plane becomes level t+1's input ----
#pragma unroll
                for (int r = 0; r < RY; ++r) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float et = E[t][c][r], ht = H[t][c][r];
                        E[t][c][r] = En[c][r];
                        H[t][c][r] = Hn[c][r];
                        Eo[c][r] = et;
                        Ho[c][r] = ht;
                    }
                }
                if constexpr (PSI) {
                    if (t < T) {
#pragma unroll
                        for (int c = 0; c < NPS; ++c)
#pragma unroll
                            for (int r = 0; r < RY; ++r) {
                                const float pt = PS[t < T ? t : 0][c][r];
                                PS[t < T ? t : 0][c][r] = PSn[c][r];
                                PSo[c][r] = pt;
                            }
                    } else if (ALL || (p >= z0 && p < z1)) {
                        store_psi(p, PSn);      // level T: the owned values of plane p
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < RY; ++r) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Eo[c][r] = E[t][c][r];
                        Ho[c][r] = H[t][c][r];
                    }
                }
                if constexpr (PSI) {
                    if (t < T) {
#pragma unroll
                        for (int c = 0; c < NPS; ++c)
#pragma unroll
                            for (int r = 0; r < RY; ++r) PSo[c][r] = PS[t < T ? t : 0][c][r];
                    }
                }
            }
        }

        // ---- store the owned part of level T (plane K-T) ----
        if constexpr (ALL) store_plane(K - T, inner_c);
        else if (K - T >= z0 && K - T < z1) store_plane(K - T, inner_c);
        // With some levels idle, every level's exchange row is published at the
        // end of the step (an active level t+1 has read the previous one before
        // its barrier), and a barrier separates them from the next step's
        // reads.  T = 1 has no level between the write and the next read.
        if constexpr (!ALL && NW > 1) {
#pragma unroll
            for (int t = 0; t < T; ++t) s_e[t][w][lane] = make_float2(E[t][0][0], E[t][2][0]);
        }
        if constexpr ((!ALL || T == 1) && NW > 1) __syncthreads();
    };

    // warm-up (upper levels not yet in their cone), steady state (every level
    // active, off the z walls, an owned plane to store and one to prefetch),
    // drain
    auto march = [&](auto inner_c) __attribute__((always_inline)) {
        using F = std::false_type;
        using Tr = std::true_type;
        YEE_LOAD_PLANE(kb);   // here, so that its registers are live on one branch only
        int K = kb;
        const int kw = min(max(kb > 0 ? kb + 2 * T - 1 : T + 1, z0 + T), ke);
        const int kend = ke < nz ? ke : nz + T;
        for (; K < kw; ++K) iterate(K, F{}, inner_c, Tr{});
        // Drain every outstanding load and store once before the steady loop
        // (s_waitcnt vmcnt(0)): the compiler's wait counts at the loop head
        // then only account for the loop's own traffic.
        __builtin_amdgcn_s_waitcnt(0x0f70);
        if (!CP || tile_xy) {
            for (; K < ke; ++K) iterate(K, Tr{}, inner_c, Tr{});
        } else {
            // Only the z slabs: psi enters with the plane loaded at step K and
            // leaves with level T's, so steps K in [0, N + T) and
            // [nz - N, nz + T) carry it.
            while (K < ke) {
                const bool in = K < N + T || (K >= nz - N && K < nz + T);
                const int next = min(ke, K < N + T ? N + T : K < nz - N ? nz - N : nz + T);
                if (in) for (; K < next; ++K) iterate(K, Tr{}, inner_c, Tr{});
                else for (; K < next; ++K) iterate(K, Tr{}, inner_c, F{});
            }
        }
        for (; K <= kend; ++K) iterate(K, F{}, inner_c, Tr{});
    };
    const bool inner = xl >= 1 && xl + 63 <= nx - 1 && yt >= 1 && yt + NR - 1 <= ny - 1;
    if (inner) march(std::true_type{});
    else march(std::false_type{});
#undef YEE_LOAD_PLANE

    if constexpr (EN) {
        // the tile's energy: a fixed butterfly over each wave, then the waves
        // in order (the partials are summed in tile order afterwards)
        double v = eacc;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) s_en[256 + w] = v;
        __syncthreads();
        if (tid == 0) {
            double sum = s_en[256];
            for (int q = 1; q < NW; ++q) sum += s_en[256 + q];
            en.partial[logical] = sum;
        }
    }

    if constexpr (Codec::scaled) {
        // Largest stored magnitude per component and the saturation flag:
        // reduce over the wave, then over the workgroup in LDS, and only then
        // touch the six global words (one atomic per component per workgroup;
        // per-wave atomics on the same six addresses serialise at the cache).
        // The maxima are bit patterns of |value| >= 0, so unsigned order is
        // float order, and a NaN (bits above infinity) wins and raises the flag.
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            uint32_t b = mx[c];
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t ob = __shfl_xor(b, o, 64);
                b = ob > b ? ob : b;
            }
            if (lane == 0 && b != 0u) atomicMax(&sm.vmax[c], b);
        }
        __syncthreads();
        if (tid < 6) {
            const uint32_t b = sm.vmax[tid];
            float m, pre;
            bool nan, over;
            float upc = up[0];
#pragma unroll
            for (int c = 1; c < 6; ++c) upc = tid == c ? up[c] : upc;
            finish_max<Codec>(b, upc, &m, &nan, &over, &pre);
            Ctrl *const ctrl = a.sb.ctrl;
            const int so = a.sb.slot_out;
            if (!a.sb.retry) {           // first pass: an overflow asks for the second pass
                if (m > 0.0f) atomicMax(&ctrl->maxbits[so][tid], __float_as_uint(m));
                if (pre > 0.0f) atomicMax(&ctrl->premax[so][tid], __float_as_uint(pre));
                if (over) atomicOr(&ctrl->ovf[so], 1u << tid);
                if (nan) atomicOr(&ctrl->flag, 1u);
            } else {
                if (m > 0.0f) atomicMax(&ctrl->rmaxbits[so][tid], __float_as_uint(m));
                if (nan || over) atomicOr(&ctrl->flag, 1u);
            }
        }
    }
    __syncthreads();   // LDS is reused by the next tile of a batched launch
}

template <int T, int RY, int NW, class Codec, bool GR, bool CP = false, bool EN = false>
__global__ __launch_bounds__(64 * NW) void yee_fused(FusedArgs a, CpmlFused cpa, EnergyFused en)
{
    __shared__ TileShared<T, NW> sm;
    __shared__ double s_en[EN ? 256 + NW : 1];
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of tiles so that halo re-reads hit its own L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (b & 7) * (nb >> 3) + (b >> 3);
    int tx, ty, tz;
    if (logical >= a.nwg) return;                                           // uniform per workgroup
    if (!tile_coords(a, logical, tx, ty, tz)) {       // a listed tile that only rewrites +0
        if constexpr (EN)
            if (threadIdx.x == 0) en.partial[logical] = 0.0;
        return;
    }
    if constexpr (Codec::scaled)         // a second pass runs only after an overflow
        if (a.sb.retry && a.sb.ctrl->ovf[a.sb.slot_out] == 0u) return;
    fused_tile<T, RY, NW, Codec, GR, CP, EN>(a, logical, tx, ty, tz, sm, cpa, en, s_en);
}

// Several solves in one launch: the workgroups take the concatenated tile
// lists of up to MAX_BATCH solves (same storage format and block length), one
// tile each, so small grids that could not fill the GPU alone share it.  A
// solve with dead tiles contributes its list of live tiles (as fdtd_step).
template <int T, int RY, int NW, class Codec>
__global__ __launch_bounds__(64 * NW) void yee_fused_batch(BatchArgs a)
{
    __shared__ TileShared<T, NW> sm;
    const int nb = gridDim.x, b = blockIdx.x;
    const int item = (b & 7) * (nb >> 3) + (b >> 3);      // contiguous runs per XCD
    if (item >= a.start[a.n]) return;
    int i = 0;
    while (i + 1 < a.n && item >= a.start[i + 1]) ++i;
    if constexpr (Codec::scaled)         // a second pass runs only after an overflow
        if (a.s[i].sb.retry && a.s[i].sb.ctrl->ovf[a.s[i].sb.slot_out] == 0u) return;
    int tx, ty, tz;
    if (!tile_coords(a.s[i], item - a.start[i], tx, ty, tz)) return;   // a listed tile that only rewrites +0
    fused_tile<T, RY, NW, Codec>(a.s[i], item - a.start[i], tx, ty, tz, sm);
}

// ---- tilings ---------------------------------------------------------------
// (RY rows per lane, NW waves) per time-block length; variant 0 is the default.
// At 16 waves a lane has 128 VGPRs, at 12 waves 168, at 8 waves 256.  The
// shapes the library picks by itself (T <= 4 for FP32, T <= 3 for 16-bit
// storage; auto_shape) fit without spilling; 16-bit storage at T = 4, the
// 3 x 12 shapes and T = 5, 6 at every shape exceed the register file (the
// 8-wave shapes least: T = 5 FP32 at 4 x 8 spills 7 VGPRs).  T = 5 and 6
// serve uniform-spacing solves alone (no batches, no graded sizes).
struct Tiling { int ry, nw; };
constexpr Tiling kTilings[MAX_T + 1][3] = {
    {},
    {{4, 4}, {2, 8}, {2, 16}},    // T = 1
    {{2, 16}, {4, 8}, {3, 12}},   // T = 2
    {{2, 16}, {4, 8}, {3, 12}},   // T = 3
    {{2, 16}, {4, 8}, {3, 12}},   // T = 4
    {{2, 16}, {4, 8}, {3, 12}},   // T = 5
    {{4, 8}, {2, 16}, {3, 12}},   // T = 6
};
// With CPML layers the kernel holds twelve psi values per row and time level
// besides the fields: one row per lane keeps them within 128 VGPRs at T <= 3.
constexpr Tiling kCpmlTiling = {1, 16};

int planes_fit(const Layout &L, int es)
{
    // a chunk's buffer resource spans (planes * kstride * es) bytes, below 2^31
    long long p = ((1LL << 31) - 1) / ((long long)L.kstride * es);
    return (int)std::min<long long>(p, 1 << 20);
}

// Tile counts and z-chunk length.  `slots` is the number of workgroups the
// GPU holds at once (0: unknown, as for the persistent batched launch).  With
// slots known the chunk length minimises  rounds * (zc + 1.5 T):  a tile's
// time grows with its planes plus the cone overhead at its two ends, and the
// launch takes ceil(workgroups / slots) rounds -- a few workgroups spilling
// into another round cost a whole round.
void geometry_for(int T, Tiling tl, int zc_req, int es, const Layout &L, int slots, int *ntx, int *nty, int *ntz,
                  int *zc, int *threads, LiveNodes *live = nullptr)
{
    const int OX = 64 - 2 * T, OY = tl.nw * tl.ry - 2 * T;
    *ntx = (L.nx + 1 + OX - 1) / OX;
    *nty = (L.ny + 1 + OY - 1) / OY;
    const int zmax = std::max(1, planes_fit(L, es) - 2 * T - 1);
    const int per_plane = *ntx * *nty;
    int z = zc_req;
    if (z <= 0 && slots > 0 && live)            // the same model over the listed tiles only
        z = live_best_zc(live, OX, OY, *ntx, *nty, T, slots, zmax);
    if (z <= 0 && slots > 0) {
        double best = 0.0;
        for (int n = 1; n <= L.nz + 1; ++n) {
            const int zz = (L.nz + 1 + n - 1) / n;
            if (zz > zmax || (n > 1 && zz == (L.nz + 1 + n - 2) / (n - 1))) continue;
            const long long wgs = (long long)per_plane * ((L.nz + 1 + zz - 1) / zz);
            const double cost = (double)((wgs + slots - 1) / slots) * (zz + 1.5 * T);
            if (z <= 0 || cost < best) { best = cost; z = zz; }
            if (wgs > 64LL * slots) break;
        }
    } else if (z <= 0) {
        // chunks of ~64 planes, fewer when that leaves the GPU short of workgroups
        const int want = std::max(1, (1024 + per_plane - 1) / per_plane);
        z = std::max(8 * T, std::min(64, (L.nz + 1 + want - 1) / want));
    }
    z = std::min(z, zmax);
    z = std::max(1, std::min(z, L.nz + 1));
    *zc = z;
    *ntz = (L.nz + 1 + z - 1) / z;
    *threads = 64 * tl.nw;
}

// Workgroups of this kernel the current device holds at once (all CUs).
template <class K>
int resident_slots(K kernel, int threads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
    return cus * per_cu;
}

// Restrict a's tiling (ntx x nty x ntz tiles of OX x OY points and zc planes)
// to the tiles whose loaded region meets the value box; false when none does.
template <int T, int NR>
bool restrict_to_box(FusedArgs &a)
{
    constexpr int OX = 64 - 2 * T, OY = NR - 2 * T;
    auto range = [](int lo, int hi, int own, int load_lo, int load_len, int n, int *t0, int *t1) {
        // tile t loads [t own + load_lo, t own + load_lo + load_len - 1]
        const long long a0 = (long long)lo - load_lo - load_len + 1, b0 = (long long)hi - load_lo;
        long long first = a0 <= 0 ? 0 : (a0 + own - 1) / own;
        long long last = b0 < 0 ? -1 : b0 / own;
        *t0 = (int)std::max(0LL, first);
        *t1 = (int)std::min((long long)n - 1, last);
        return *t0 <= *t1;
    };
    int x0, x1, y0, y1, z0, z1;
    const bool any = range(a.box_lo.x, a.box_hi.x, OX, -T, 64, a.ntx, &x0, &x1) &&
                     range(a.box_lo.y, a.box_hi.y, OY, -T, NR, a.nty, &y0, &y1) &&
                     range(a.box_lo.z, a.box_hi.z, a.zc, -T, a.zc + 2 * T, a.ntz, &z0, &z1);
    if (!any) return false;
    a.tx0 = x0;
    a.ty0 = y0;
    a.tz0 = z0;
    a.ntx = x1 - x0 + 1;
    a.nty = y1 - y0 + 1;
    a.ntz = z1 - z0 + 1;
    return true;
}

template <int T, int RY, int NW, class Codec, bool GR, bool CP = false, bool EN = false>
hipError_t launch_shape(const FusedArgs &a0, int zc_req, hipStream_t st, const CpmlFused &cpa = {},
                        const EnergyFused &en = {})
{
    constexpr Tiling tl = {RY, NW};
    static const int slots = resident_slots(yee_fused<T, tl.ry, tl.nw, Codec, GR, CP, EN>, 64 * tl.nw);
    FusedArgs a = a0;
    int threads;
    geometry_for(T, tl, zc_req, sizeof(typename Codec::T), a.L, slots, &a.ntx, &a.nty, &a.ntz, &a.zc, &threads, a.live);
    const long long full = (long long)a.ntx * a.nty * a.ntz;
    int listed = 0;
    a.tiles = nullptr;
    if (a.live) {
        a.tiles = live_tile_list(a.live, 64 - 2 * T, tl.ry * tl.nw - 2 * T, a.zc, a.ntx, a.nty, a.ntz, &listed, st);
        a.ltx = a.ntx;
        a.lty = a.nty;
    }
    if (!restrict_to_box<T, tl.ry * tl.nw>(a) || (a.tiles && listed == 0)) {
        if (!Codec::scaled) {                       // all +0 and stays so
            if (a.tile_stats) a.tile_stats[1] += full;
            if constexpr (EN) return launch_energy_sum(en.partial, 0, en.out, st);   // W = 0
            return hipSuccess;
        }
        a.ntx = a.nty = a.ntz = 1;                  // one tile publishes the next block's scales
        a.tx0 = a.ty0 = a.tz0 = 0;
        a.tiles = nullptr;
    }
    a.nwg = a.tiles ? listed : a.ntx * a.nty * a.ntz;
    if (a.tile_stats) {
        a.tile_stats[0] += a.nwg;
        a.tile_stats[1] += full;
    }
    const int grid = (a.nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((yee_fused<T, tl.ry, tl.nw, Codec, GR, CP, EN>), dim3(grid), dim3(threads), 0, st, a, cpa, en);
    if constexpr (Codec::scaled) {       // the block again, with new scales, if it overflowed
        if (hipError_t e = hipGetLastError()) return e;
        a.sb.retry = 1;
        a.tile_stats = nullptr;
        hipLaunchKernelGGL((yee_fused<T, tl.ry, tl.nw, Codec, GR, CP, EN>), dim3(grid), dim3(threads), 0, st, a, cpa,
                           en);
    }
    if constexpr (EN) {                  // the tiles' partials, in tile order
        if (hipError_t e = hipGetLastError()) return e;
        return launch_energy_sum(en.partial, a.nwg, en.out, st);
    }
    return hipGetLastError();
}

template <int T, int V, class Codec, bool GR>
hipError_t launch_tv(const FusedArgs &a0, int zc_req, hipStream_t st)
{
    return launch_shape<T, kTilings[T][V].ry, kTilings[T][V].nw, Codec, GR>(a0, zc_req, st);
}

template <int T, int V, class Codec>
hipError_t launch_batch_tv(const FusedArgs *args, int n, int zc_req, hipStream_t st)
{
    static_assert(sizeof(BatchArgs) <= 4000, "batch descriptors must fit the kernel argument segment");
    constexpr Tiling tl = kTilings[T][V];
    BatchArgs b;
    b.n = n;
    b.start[0] = 0;
    int threads = 64 * tl.nw;
    for (int i = 0; i < n; ++i) {
        FusedArgs &a = b.s[i];
        a = args[i];
        a.tiles = nullptr;
        geometry_for(T, tl, zc_req, sizeof(typename Codec::T), a.L, 0, &a.ntx, &a.nty, &a.ntz, &a.zc, &threads);
        const long long full = (long long)a.ntx * a.nty * a.ntz;
        int listed = 0;
        if (a.live) {                               // the tiles owning a live node
            a.tiles = live_tile_list(a.live, 64 - 2 * T, tl.ry * tl.nw - 2 * T, a.zc, a.ntx, a.nty, a.ntz, &listed, st);
            a.ltx = a.ntx;
            a.lty = a.nty;
        }
        a.live = nullptr;
        if (!restrict_to_box<T, tl.ry * tl.nw>(a) || (a.tiles && listed == 0)) {
            a.ntx = a.nty = a.ntz = Codec::scaled ? 1 : 0;   // one tile publishes the next block's scales
            a.tx0 = a.ty0 = a.tz0 = 0;
            a.tiles = nullptr;
        }
        a.nwg = a.tiles ? listed : a.ntx * a.nty * a.ntz;
        if (a.tile_stats) {
            a.tile_stats[0] += a.nwg;
            a.tile_stats[1] += full;
        }
        b.start[i + 1] = b.start[i] + a.nwg;
    }
    if (b.start[n] == 0) return hipSuccess;        // every solve all +0 (unscaled storage)
    const int grid = (b.start[n] + 7) / 8 * 8;
    hipLaunchKernelGGL((yee_fused_batch<T, tl.ry, tl.nw, Codec>), dim3(grid), dim3(threads), 0, st, b);
    if constexpr (Codec::scaled) {       // solves whose block overflowed run it again
        if (hipError_t e = hipGetLastError()) return e;
        for (int i = 0; i < n; ++i) b.s[i].sb.retry = 1;
        hipLaunchKernelGGL((yee_fused_batch<T, tl.ry, tl.nw, Codec>), dim3(grid), dim3(threads), 0, st, b);
    }
    return hipGetLastError();
}

template <int T, class Codec, bool GR>
hipError_t launch_t(const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st)
{
    if constexpr (GR || T > MAX_T_BATCH) {
        if (batch) return hipErrorInvalidValue;   // batches are uniform-spacing solves of short blocks
    } else if (batch) {
        switch (variant) {
        case 1: return launch_batch_tv<T, 1, Codec>(a, n, zc, st);
        case 2: return launch_batch_tv<T, 2, Codec>(a, n, zc, st);
        default: return launch_batch_tv<T, 0, Codec>(a, n, zc, st);
        }
    }
    switch (variant) {
    case 1: return launch_tv<T, 1, Codec, GR>(*a, zc, st);
    case 2: return launch_tv<T, 2, Codec, GR>(*a, zc, st);
    default: return launch_tv<T, 0, Codec, GR>(*a, zc, st);
    }
}

template <class Codec, bool GR = false>
hipError_t launch_codec(int T, const FusedArgs *a, int n, bool batch, int variant, int zc, hipStream_t st)
{
    switch (T) {
    case 1: return launch_t<1, Codec, GR>(a, n, batch, variant, zc, st);
    case 2: return launch_t<2, Codec, GR>(a, n, batch, variant, zc, st);
    case 3: return launch_t<3, Codec, GR>(a, n, batch, variant, zc, st);
    case 4: return launch_t<4, Codec, GR>(a, n, batch, variant, zc, st);
    }
    if constexpr (!GR) {                          // deeper blocks: uniform spacing only
        switch (T) {
        case 5: return launch_t<5, Codec, false>(a, n, batch, variant, zc, st);
        case 6: return launch_t<6, Codec, false>(a, n, batch, variant, zc, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

}  // namespace yee
