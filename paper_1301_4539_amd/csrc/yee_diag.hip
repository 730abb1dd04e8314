// FP64 diagnostics of a state (E^n, H^{n-1/2}):
//   energy W^n = 1/2 sum eps_r E^n.E^n + 1/2 sum H^{n-1/2}.H^{n+1/2}, the
//     quantity the leapfrog conserves in a lossless PEC box (consequence of
//     the discrete antisymmetry noted in Sec. 2.1); H^{n+1/2} is recomputed
//     in registers with the same FP32 operation order as the update kernels;
//   div(eps_r E) at interior nodes and div(H) at cell centres: largest
//     magnitude and sum of squares (both constant in time without sources
//     and losses);
//   largest |value| per component.
// Reduction is deterministic: each thread accumulates its (i, j) column over
// a fixed run of planes in ascending k; each wave combines its 64 lanes in a
// fixed butterfly of cross-lane moves (no LDS, no barrier per quantity), the
// block adds its 4 wave results in wave order, and one block then sums the
// block partials the same way.  The plane runs keep the partials few (a few
// thousand), so the final single-block pass is short.
// Graded spacing (GR): every term is weighted by its volume (edge length x
// dual face area for E, face area x dual edge length for H; dual sizes are
// half cells on the walls), the energy is then in units of eps0 with volumes
// in m^3, differences are divided by the per-index sizes, and H^{n+1/2} uses
// the per-index update factors.

#include <algorithm>
#include <mutex>

#include "yee_device.hpp"
#include "yee_internal.hpp"

namespace yee {

namespace {

constexpr int DBX = 64, DBY = 4, DT = DBX * DBY;

// Sum or maximum over the 64 lanes of a wave, the same on every lane: a
// fixed butterfly of xor shuffles, so the result does not depend on timing.
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Quantities 0..2 are sums, the rest maxima.  Combines v over the block
// (nwave waves of 64 lanes, in wave order) into out[q] on thread 0.
template <int NWAVE>
__device__ inline void block_reduce(const double *v, double (*s_w)[DIAG_W], int t, double *out)
{
    const int lane = t & 63, wv = t >> 6;
#pragma unroll
    for (int q = 0; q < DIAG_W; ++q) {
        const double r = q <= 2 ? wave_sum(v[q]) : wave_max(v[q]);
        if (lane == 0) s_w[wv][q] = r;
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < DIAG_W; ++q) {
            double r = s_w[0][q];
            for (int w = 1; w < NWAVE; ++w) r = q <= 2 ? r + s_w[w][q] : fmax(r, s_w[w][q]);
            out[q] = r;
        }
    }
}
constexpr int DZ = 8;   // plane runs per grid (fewer for thin grids)

template <class Codec, bool GR>
__global__ __launch_bounds__(DT) void diag_points(DiagArgs a)
{
    using S = typename Codec::T;
    __shared__ double s_eps[256];
    __shared__ double s_w[DT / 64][DIAG_W];
    const int t = threadIdx.y * DBX + threadIdx.x;
    for (int q = t; q < a.n_mat; q += DT) s_eps[q] = a.eps[q];
    __syncthreads();

    const Layout &L = a.L;
    const int i = blockIdx.x * DBX + threadIdx.x;
    const int j = blockIdx.y * DBY + threadIdx.y;
    const int run = (L.nz + 1 + gridDim.z - 1) / gridDim.z;
    const int k0 = blockIdx.z * run, k1 = min(L.nz + 1, k0 + run);
    const S *f = static_cast<const S *>(a.f);
    float dn[6];
    for (int c = 0; c < 6; ++c) dn[c] = Codec::scaled ? ldexpf(1.0f, -a.sb.ctrl->scale[a.sb.par][c]) : 1.0f;
    auto F = [&](int c, long long p) -> float { return Codec::load(f + c * L.cstride + p, dn[c]); };

    double v[DIAG_W];
    for (int q = 0; q < DIAG_W; ++q) v[q] = 0.0;
    for (int k = k0; k < k1 && i <= L.nx && j <= L.ny; ++k) {
        const int nx = L.nx, ny = L.ny, nz = L.nz;
        const long long p = k * L.kstride + (long long)j * L.pitch + i;
        // owner-cell permittivity of an E edge, zero on wall (PEC) edges
        auto eps_edge = [&](int c, int ii, int jj, int kk) -> double {
            bool interior = c == 0 ? (ii < nx && jj > 0 && jj < ny && kk > 0 && kk < nz)
                          : c == 1 ? (jj < ny && ii > 0 && ii < nx && kk > 0 && kk < nz)
                                   : (kk < nz && ii > 0 && ii < nx && jj > 0 && jj < ny);
            if (!interior) return 0.0;
            return s_eps[a.mat[kk * L.plane + (long long)jj * L.pitch + ii]];
        };
        const float ex = F(0, p), ey = F(1, p), ez = F(2, p);
        const float hx = F(3, p), hy = F(4, p), hz = F(5, p);
        float chx = a.chx, chy = a.chy, chz = a.chz;
        // volume weights (1 on uniform grids) and sizes of this node
        double we[3] = {1.0, 1.0, 1.0}, wh[3] = {1.0, 1.0, 1.0};
        double2 sx = make_double2(0.0, 0.0), sy = sx, sz = sx;
        if constexpr (GR) {
            chx = a.gc[i].x;
            chy = a.gc[nx + 1 + j].x;
            chz = a.gc[nx + ny + 2 + k].x;
            sx = a.gsz[i];                    // (cell size, dual size)
            sy = a.gsz[nx + 1 + j];
            sz = a.gsz[nx + ny + 2 + k];
            we[0] = sx.x * sy.y * sz.y;
            we[1] = sx.y * sy.x * sz.y;
            we[2] = sx.y * sy.y * sz.x;
            wh[0] = sx.y * sy.x * sz.x;
            wh[1] = sx.x * sy.y * sz.x;
            wh[2] = sx.x * sy.x * sz.y;
        }
        // electric energy
        v[0] += 0.5 * eps_edge(0, i, j, k) * (double)ex * (double)ex * we[0];
        v[0] += 0.5 * eps_edge(1, i, j, k) * (double)ey * (double)ey * we[1];
        v[0] += 0.5 * eps_edge(2, i, j, k) * (double)ez * (double)ez * we[2];
        // magnetic energy with H^{n+1/2} from the Faraday half-step
        if (j < ny && k < nz) {
            const float h1 = __builtin_fmaf(-chy, F(2, p + L.pitch) - ez, __builtin_fmaf(chz, F(1, p + L.kstride) - ey, hx));
            v[0] += 0.5 * (double)hx * (double)h1 * wh[0];
        }
        if (i < nx && k < nz) {
            const float h1 = __builtin_fmaf(-chz, F(0, p + L.kstride) - ex, __builtin_fmaf(chx, F(2, p + 1) - ez, hy));
            v[0] += 0.5 * (double)hy * (double)h1 * wh[1];
        }
        if (i < nx && j < ny) {
            const float h1 = __builtin_fmaf(-chx, F(1, p + 1) - ey, __builtin_fmaf(chy, F(0, p + L.pitch) - ex, hz));
            v[0] += 0.5 * (double)hz * (double)h1 * wh[2];
        }
        // div(eps_r E) at interior nodes
        if (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz) {
            const double tx = eps_edge(0, i, j, k) * ex - eps_edge(0, i - 1, j, k) * F(0, p - 1);
            const double ty = eps_edge(1, i, j, k) * ey - eps_edge(1, i, j - 1, k) * F(1, p - L.pitch);
            const double tz = eps_edge(2, i, j, k) * ez - eps_edge(2, i, j, k - 1) * F(2, p - L.kstride);
            double d;
            if constexpr (GR) d = tx / sx.y + ty / sy.y + tz / sz.y;
            else d = tx * a.idx + ty * a.idy + tz * a.idz;
            v[1] += d * d;
            v[3] = fmax(v[3], fabs(d));
        }
        // div(H) at cell centres
        if (i < nx && j < ny && k < nz) {
            const double tx = (double)F(3, p + 1) - hx, ty = (double)F(4, p + L.pitch) - hy;
            const double tz = (double)F(5, p + L.kstride) - hz;
            double d;
            if constexpr (GR) d = tx / sx.x + ty / sy.x + tz / sz.x;
            else d = tx * a.idx + ty * a.idy + tz * a.idz;
            v[2] += d * d;
            v[4] = fmax(v[4], fabs(d));
        }
        v[5] = fmax(v[5], fabs(ex)); v[6] = fmax(v[6], fabs(ey)); v[7] = fmax(v[7], fabs(ez));
        v[8] = fmax(v[8], fabs(hx)); v[9] = fmax(v[9], fabs(hy)); v[10] = fmax(v[10], fabs(hz));
    }
    // wave butterflies, then the block's waves in order
    const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_reduce<DT / 64>(v, s_w, t, a.partial + blk * DIAG_W);
}

__global__ __launch_bounds__(256) void diag_final(const double *partial, long long nblk, double *out)
{
    __shared__ double s_w[4][DIAG_W];
    const int t = threadIdx.x;
    double v[DIAG_W];
#pragma unroll
    for (int q = 0; q < DIAG_W; ++q) v[q] = 0.0;
    for (long long b = t; b < nblk; b += 256) {      // each thread its strided partials, in order
#pragma unroll
        for (int q = 0; q < DIAG_W; ++q) {
            const double x = partial[b * DIAG_W + q];
            v[q] = q <= 2 ? v[q] + x : fmax(v[q], x);
        }
    }
    block_reduce<4>(v, s_w, t, out);
}

// Sum of n partials in a fixed order: each thread its strided partials in
// order, then the wave butterflies, then the waves in order.
__global__ __launch_bounds__(256) void energy_sum(const double *partial, long long n, double *out)
{
    __shared__ double s_w[4];
    const int t = threadIdx.x;
    double v = 0.0;
    for (long long b = t; b < n; b += 256) v += partial[b];
    v = wave_sum(v);
    if ((t & 63) == 0) s_w[t >> 6] = v;
    __syncthreads();
    if (t == 0) *out = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

template <class Codec>
hipError_t launch_diag_t(const DiagArgs &a, double *out, hipStream_t st)
{
    dim3 block(DBX, DBY, 1);
    dim3 grid((a.L.nx + 1 + DBX - 1) / DBX, (a.L.ny + 1 + DBY - 1) / DBY, std::min(DZ, a.L.nz + 1));
    if (a.gc) {
        if (!a.gsz) return hipErrorInvalidValue;
        hipLaunchKernelGGL((diag_points<Codec, true>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((diag_points<Codec, false>), grid, block, 0, st, a);
    }
    const long long nblk = (long long)grid.x * grid.y * grid.z;
    hipLaunchKernelGGL(diag_final, dim3(1), dim3(256), 0, st, (const double *)a.partial, nblk, out);
    return hipGetLastError();
}

// Scratch of the diagnostics entry point that allocates nothing: 11 result
// doubles at the start (padded to 256 bytes), then the per-block partials.
// One copy per GPU, held until the process ends; host code never names it
// directly (its host-side name is not a device address) but only through the
// per-device address that diag_static_scratch() looks up.
constexpr size_t DIAG_SCRATCH_BYTES = size_t(4) << 20;
constexpr size_t DIAG_OUT_DOUBLES = 32;   // 256 bytes ahead of the partials
static __device__ __align__(256) double scratch[DIAG_SCRATCH_BYTES / sizeof(double)];

}  // namespace

long long diag_static_max_blocks()
{
    return (long long)((DIAG_SCRATCH_BYTES / sizeof(double) - DIAG_OUT_DOUBLES) / DIAG_W);
}

hipError_t diag_static_scratch(double **out, double **partial)
{
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static double *per_dev[MAX_DEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!per_dev[dev]) {            // once per device, with that device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        per_dev[dev] = static_cast<double *>(p);
    }
    *out = per_dev[dev];
    *partial = per_dev[dev] + DIAG_OUT_DOUBLES;
    return hipSuccess;
}

int diag_blocks(const Layout &L)
{
    return ((L.nx + 1 + DBX - 1) / DBX) * ((L.ny + 1 + DBY - 1) / DBY) * std::min(DZ, L.nz + 1);
}

hipError_t launch_energy_sum(const double *partial, long long n, double *out, hipStream_t st)
{
    if (!out || (n > 0 && !partial)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(energy_sum, dim3(1), dim3(256), 0, st, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_diag(int storage, const DiagArgs &a, double *out, hipStream_t st)
{
    switch (storage) {
    case 0: return launch_diag_t<CodecF32>(a, out, st);
    case 1: return launch_diag_t<CodecF16>(a, out, st);
    case 2: return launch_diag_t<CodecBF16>(a, out, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace yee
