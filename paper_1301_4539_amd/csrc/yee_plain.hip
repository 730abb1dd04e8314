// Plain two-pass Yee step: an in-place H pass over the whole grid, then an
// in-place E pass (the standard loop structure of Sec. 2.2, one thread per
// node-box point updating all three components there).  FP32 storage only.
// Each pass streams its fields from HBM once; the E pass also reads the
// uint8 material index and looks the coefficients up in an LDS table.
// With graded spacing (GR) the c dt / size factors come per index from the
// one-dimensional arrays a.gc (primal sizes for H, dual sizes for E), and an
// E coefficient is the material's G times the dual factor, one FP32 product.
// With CPML layers (CP) each value inside a layer then adds its psi terms in
// the order of its own update, psi first updated by its recursion
// psi = b psi + a diff (the convolutional PML of Roden and Gedney cited in
// Sec. 3.3; the stretch kappa is already folded into the a.gc factors).

#include "yee_device.hpp"
#include "yee_internal.hpp"

namespace yee {

namespace {

constexpr int BX = 64, BY = 4;

// layer membership and slab slot of index q along an axis of n cells
__device__ inline bool h_in(int n, int N, int q) { return q < N || q >= n - N; }
__device__ inline bool e_in(int n, int N, int q) { return (q > 0 && q < N) || (q > n - N && q < n); }
__device__ inline int slot(int n, int N, int q) { return q < N ? q : q - n + 2 * N; }

// psi entry of array `arr` for a value at (i, j, k)
__device__ inline float &psi_at(const Cpml &c, const Layout &L, int arr, int i, int j, int k)
{
    const int N = c.n, axis = arr >> 2;
    long long g;
    if (axis == 0) g = ((long long)k * (L.ny + 1) + j) * (2 * N) + slot(L.nx, N, i);
    else if (axis == 1) g = ((long long)k * (2 * N) + slot(L.ny, N, j)) * (L.nx + 1) + i;
    else g = ((long long)slot(L.nz, N, k) * (L.ny + 1) + j) * (L.nx + 1) + i;
    return c.psi[c.base[axis] + 4 * g + (arr & 3)];
}

// one psi term of an H value: psi <- b psi + a diff, then v + sign (c dt/d) psi
__device__ inline float h_term(const float *cpq, float &ps, float diff, float v, bool neg)
{
    ps = __builtin_fmaf(cpq[0], ps, cpq[1] * diff);
    return __builtin_fmaf(neg ? -cpq[2] : cpq[2], ps, v);
}

// one psi term of an E value, with the material factor G
__device__ inline float e_term(const float *cpq, float g, float &ps, float diff, float v, bool neg)
{
    ps = __builtin_fmaf(cpq[3], ps, cpq[4] * diff);
    const float c = g * cpq[5];
    return __builtin_fmaf(neg ? -c : c, ps, v);
}

template <bool GR, bool CP>
__global__ __launch_bounds__(BX *BY) void h_plain(PlainArgs a)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const Layout &L = a.L;
    if (i > L.nx || j > L.ny) return;
    float *ex = a.f, *ey = a.f + L.cstride, *ez = a.f + 2 * L.cstride;
    float *hx = a.f + 3 * L.cstride, *hy = a.f + 4 * L.cstride, *hz = a.f + 5 * L.cstride;
    const long long p = k * L.kstride + (long long)j * L.pitch + i;
    float chx = a.chx, chy = a.chy, chz = a.chz;
    if constexpr (GR) {
        chx = a.gc[i].x;
        chy = a.gc[L.nx + 1 + j].x;
        chz = a.gc[L.nx + L.ny + 2 + k].x;
    }
    const float *cpx = nullptr, *cpy = nullptr, *cpz = nullptr;
    if constexpr (CP) {
        cpx = a.pml.cp + 6 * i;
        cpy = a.pml.cp + 6 * (L.nx + 1 + j);
        cpz = a.pml.cp + 6 * (L.nx + L.ny + 2 + k);
    }
    const int N = a.pml.n;
    // Faraday: H -= c dt curl E, z-difference term first, then y (cyclic).
    if (j < L.ny && k < L.nz) {
        float dey_z = ey[p + L.kstride] - ey[p];
        float dez_y = ez[p + L.pitch] - ez[p];
        float h = __builtin_fmaf(-chy, dez_y, __builtin_fmaf(chz, dey_z, hx[p]));
        if constexpr (CP) {
            if (h_in(L.nz, N, k)) h = h_term(cpz, psi_at(a.pml, L, PS_HXZ, i, j, k), dey_z, h, false);
            if (h_in(L.ny, N, j)) h = h_term(cpy, psi_at(a.pml, L, PS_HXY, i, j, k), dez_y, h, true);
        }
        hx[p] = h;
    }
    if (i < L.nx && k < L.nz) {
        float dez_x = ez[p + 1] - ez[p];
        float dex_z = ex[p + L.kstride] - ex[p];
        float h = __builtin_fmaf(-chz, dex_z, __builtin_fmaf(chx, dez_x, hy[p]));
        if constexpr (CP) {
            if (h_in(L.nx, N, i)) h = h_term(cpx, psi_at(a.pml, L, PS_HYX, i, j, k), dez_x, h, false);
            if (h_in(L.nz, N, k)) h = h_term(cpz, psi_at(a.pml, L, PS_HYZ, i, j, k), dex_z, h, true);
        }
        hy[p] = h;
    }
    if (i < L.nx && j < L.ny) {
        float dex_y = ex[p + L.pitch] - ex[p];
        float dey_x = ey[p + 1] - ey[p];
        float h = __builtin_fmaf(-chx, dey_x, __builtin_fmaf(chy, dex_y, hz[p]));
        if constexpr (CP) {
            if (h_in(L.ny, N, j)) h = h_term(cpy, psi_at(a.pml, L, PS_HZY, i, j, k), dex_y, h, false);
            if (h_in(L.nx, N, i)) h = h_term(cpx, psi_at(a.pml, L, PS_HZX, i, j, k), dey_x, h, true);
        }
        hz[p] = h;
    }
}

template <bool GR, bool CP>
__global__ __launch_bounds__(BX *BY) void e_plain(PlainArgs a)
{
    __shared__ float4 s_coef[256];
    const int t = threadIdx.y * BX + threadIdx.x;
    for (int q = t; q < a.n_mat; q += BX * BY) s_coef[q] = a.coef[q];
    __syncthreads();
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    const Layout &L = a.L;
    if (i > L.nx || j > L.ny) return;
    float *ex = a.f, *ey = a.f + L.cstride, *ez = a.f + 2 * L.cstride;
    const float *hx = a.f + 3 * L.cstride, *hy = a.f + 4 * L.cstride, *hz = a.f + 5 * L.cstride;
    const long long p = k * L.kstride + (long long)j * L.pitch + i;
    const float4 cf = s_coef[a.mat[k * L.plane + (long long)j * L.pitch + i]];   // owner cell's Ca, Cbx, Cby, Cbz
    float cbx = cf.y, cby = cf.z, cbz = cf.w;
    if constexpr (GR) {   // cf.y holds G
        cbx = cf.y * a.gc[i].y;
        cby = cf.y * a.gc[L.nx + 1 + j].y;
        cbz = cf.y * a.gc[L.nx + L.ny + 2 + k].y;
    }
    const bool kin = k > 0 && k < L.nz, jin = j > 0 && j < L.ny, iin = i > 0 && i < L.nx;
    const float *cpx = nullptr, *cpy = nullptr, *cpz = nullptr;
    if constexpr (CP) {
        cpx = a.pml.cp + 6 * i;
        cpy = a.pml.cp + 6 * (L.nx + 1 + j);
        cpz = a.pml.cp + 6 * (L.nx + L.ny + 2 + k);
    }
    const int N = a.pml.n;
    // Ampere with loss: E = Ca E + Cb curl H on edges not tangential to a wall.
    if (i < L.nx && jin && kin) {
        float dhz_y = hz[p] - hz[p - L.pitch];
        float dhy_z = hy[p] - hy[p - L.kstride];
        float e = __builtin_fmaf(-cbz, dhy_z, __builtin_fmaf(cby, dhz_y, cf.x * ex[p]));
        if constexpr (CP) {
            if (e_in(L.ny, N, j)) e = e_term(cpy, cf.y, psi_at(a.pml, L, PS_EXY, i, j, k), dhz_y, e, false);
            if (e_in(L.nz, N, k)) e = e_term(cpz, cf.y, psi_at(a.pml, L, PS_EXZ, i, j, k), dhy_z, e, true);
        }
        ex[p] = e;
    }
    if (j < L.ny && iin && kin) {
        float dhx_z = hx[p] - hx[p - L.kstride];
        float dhz_x = hz[p] - hz[p - 1];
        float e = __builtin_fmaf(-cbx, dhz_x, __builtin_fmaf(cbz, dhx_z, cf.x * ey[p]));
        if constexpr (CP) {
            if (e_in(L.nz, N, k)) e = e_term(cpz, cf.y, psi_at(a.pml, L, PS_EYZ, i, j, k), dhx_z, e, false);
            if (e_in(L.nx, N, i)) e = e_term(cpx, cf.y, psi_at(a.pml, L, PS_EYX, i, j, k), dhz_x, e, true);
        }
        ey[p] = e;
    }
    if (k < L.nz && iin && jin) {
        float dhy_x = hy[p] - hy[p - 1];
        float dhx_y = hx[p] - hx[p - L.pitch];
        float e = __builtin_fmaf(-cby, dhx_y, __builtin_fmaf(cbx, dhy_x, cf.x * ez[p]));
        if constexpr (CP) {
            if (e_in(L.nx, N, i)) e = e_term(cpx, cf.y, psi_at(a.pml, L, PS_EZX, i, j, k), dhy_x, e, false);
            if (e_in(L.ny, N, j)) e = e_term(cpy, cf.y, psi_at(a.pml, L, PS_EZY, i, j, k), dhx_y, e, true);
        }
        ez[p] = e;
    }
}

// Soft sources of step `step`, added in source order by one thread.
__global__ void src_plain(float *f, Layout L, SourceTable s, long long step)
{
    for (int q = 0; q < s.n; ++q) {
        int4 d = s.pos[q];
        int2 w = s.wave[q];
        if (step < w.y) {
            long long p = d.x * L.cstride + d.w * L.kstride + (long long)d.z * L.pitch + d.y;
            f[p] = f[p] + s.samples[w.x + step];
        }
    }
}

__global__ void probe_plain(const float *f, Layout L, ProbeTable pt, long long step)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= pt.n) return;
    int4 d = pt.pos[q];
    long long p = d.x * L.cstride + d.w * L.kstride + (long long)d.z * L.pitch + d.y;
    pt.out[(step - pt.base) * pt.n + q] = (double)f[p];
}

}  // namespace

hipError_t launch_plain_step(const PlainArgs &a, const SourceTable &src, const ProbeTable &probe,
                             long long step, hipStream_t st)
{
    dim3 block(BX, BY, 1);
    dim3 grid((a.L.nx + 1 + BX - 1) / BX, (a.L.ny + 1 + BY - 1) / BY, a.L.nz + 1);
    if (a.pml.n > 0) {
        if (!a.gc || !a.pml.cp || !a.pml.psi) return hipErrorInvalidValue;
        hipLaunchKernelGGL((h_plain<true, true>), grid, block, 0, st, a);
        hipLaunchKernelGGL((e_plain<true, true>), grid, block, 0, st, a);
    } else if (a.gc) {
        hipLaunchKernelGGL((h_plain<true, false>), grid, block, 0, st, a);
        hipLaunchKernelGGL((e_plain<true, false>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((h_plain<false, false>), grid, block, 0, st, a);
        hipLaunchKernelGGL((e_plain<false, false>), grid, block, 0, st, a);
    }
    if (src.n > 0) hipLaunchKernelGGL(src_plain, dim3(1), dim3(1), 0, st, a.f, a.L, src, step);
    if (probe.n > 0)
        hipLaunchKernelGGL(probe_plain, dim3((probe.n + 63) / 64), dim3(64), 0, st, (const float *)a.f, a.L,
                           probe, step);
    return hipGetLastError();
}

}  // namespace yee
