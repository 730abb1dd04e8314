// Host runtime of the Yee FDTD library: the C ABI declared in include/fdtd.h.
//
// Responsibilities: argument validation, coefficient precompute (FP64,
// rounded once to FP32), device workspace layout, upload/readback of fields
// (with the reduced-storage codec), source/probe tables, and the step
// scheduler, which cuts fdtd_step(n) into blocks of at most T steps -- full
// blocks from the current step with FP32 storage, blocks ending at absolute
// step counts that are multiples of T with 16-bit storage (a pin-point output never
// forces an extra block: probes are recorded inside the kernels, the GPU
// counterpart of Sec. 3.4's advice not to start a multi-step block the step
// before an output is needed).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "yee_internal.hpp"

namespace {

constexpr double C0 = 299792458.0;
constexpr double EPS0 = 8.8541878128e-12;

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FDTD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

int elem_size(int storage) { return storage == FDTD_FP32 ? 4 : 2; }

struct Dims {
    int pitch;
    long long plane, kstride;
    size_t fbytes, matbytes, total;
};

// Plane-interleaved field buffers: the six components of one z plane are
// consecutive, each plane of one component pitch*(ny+1) elements.
Dims dims_for(int nx, int ny, int nz, int storage)
{
    Dims d;
    const int es = elem_size(storage);
    d.pitch = (int)round_up((size_t)nx + 1, 128 / es);          // rows start on 128-byte lines
    d.plane = (long long)d.pitch * (ny + 1);
    d.kstride = 6 * d.plane;
    d.fbytes = round_up((size_t)d.kstride * (nz + 1) * es, 256);
    d.matbytes = round_up((size_t)d.plane * (nz + 1), 256);
    d.total = 2 * d.fbytes + d.matbytes + round_up(sizeof(yee::Ctrl), 256);   // then the control block
    return d;
}

// 1 if component c exists at (i,j,k) of the node box
bool in_range(int nx, int ny, int nz, int c, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i > nx || j > ny || k > nz) return false;
    switch (c) {
    case 0: return i < nx;
    case 1: return j < ny;
    case 2: return k < nz;
    case 3: return j < ny && k < nz;
    case 4: return i < nx && k < nz;
    case 5: return i < nx && j < ny;
    }
    return false;
}

// 1 if E component c at (i,j,k) is not tangential to a wall
bool e_interior(int nx, int ny, int nz, int c, int i, int j, int k)
{
    switch (c) {
    case 0: return i < nx && j > 0 && j < ny && k > 0 && k < nz;
    case 1: return j < ny && i > 0 && i < nx && k > 0 && k < nz;
    case 2: return k < nz && i > 0 && i < nx && j > 0 && j < ny;
    }
    return false;
}

// Stored range of component c on row (j,k): true and [i0, i1) if the row holds
// values (inside the component's range, and not tangential E on a wall).
bool row_span(int nx, int ny, int nz, int c, int j, int k, int *i0, int *i1)
{
    switch (c) {
    case 0: *i0 = 0; *i1 = nx; return j > 0 && j < ny && k > 0 && k < nz;
    case 1: *i0 = 1; *i1 = nx; return j < ny && k > 0 && k < nz;
    case 2: *i0 = 1; *i1 = nx; return k < nz && j > 0 && j < ny;
    case 3: *i0 = 0; *i1 = nx + 1; return j < ny && k < nz;
    case 4: *i0 = 0; *i1 = nx; return k < nz;
    case 5: *i0 = 0; *i1 = nx; return j < ny;
    }
    return false;
}

// ---- reduced-storage codec on the host (upload and readback) ---------------
uint16_t enc_f16(float y)
{
    _Float16 h = (_Float16)y;                  // round to nearest even, subnormals kept
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

float dec_f16(uint16_t b)
{
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return (float)h;
}

uint16_t enc_bf16(float y)
{
    uint32_t u;
    std::memcpy(&u, &y, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

float dec_bf16(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Encode y (already scaled); saturate at the largest finite value.
uint16_t encode(int storage, float y, bool *sat)
{
    if (storage == FDTD_FP16) {
        uint16_t h = enc_f16(y);
        if ((h & 0x7fffu) == 0x7c00u) { h = (uint16_t)((h & 0x8000u) | 0x7bffu); *sat = true; }
        else if ((h & 0x7fffu) > 0x7c00u) *sat = true;
        return h;
    }
    uint16_t h = enc_bf16(y);
    if ((h & 0x7fffu) == 0x7f80u) { h = (uint16_t)((h & 0x8000u) | 0x7f7fu); *sat = true; }
    else if ((h & 0x7fffu) > 0x7f80u) *sat = true;
    return h;
}

float decode(int storage, uint16_t h) { return storage == FDTD_FP16 ? dec_f16(h) : dec_bf16(h); }

int scale_from(float m)
{
    if (!(m > 0.0f) || std::isinf(m)) return 0;
    int e;
    float fr = std::frexp(m, &e);
    int cl = fr == 0.5f ? e - 1 : e;
    int s = 10 - cl;
    return std::max(-64, std::min(64, s));
}

void choose_scales(const float *m, float a_max, int *s)
{
    float all = 0.0f;
    for (int c = 0; c < 6; ++c) all = std::max(all, m[c]);
    for (int c = 0; c < 6; ++c) {
        float v = m[c] > a_max ? m[c] : a_max;
        if (!(v > 0.0f)) v = all;
        s[c] = scale_from(v);
    }
}

}  // namespace

// CPML layer parameters (Roden and Gedney's CFS-CPML; see fdtd_set_cpml).
struct CpmlParams {
    int n = 0;                          // cells per layer; 0 = no layers
    int order = 3;
    double sigma_factor = 1.0, kappa_max = 1.0, alpha_max = 0.0;
};

struct fdtd_solver {
    yee::Layout L{};
    double dx = 0, dy = 0, dz = 0, dt = 0;
    int storage = FDTD_FP32;
    int kernel = FDTD_KERNEL_AUTO;
    int T = 1;                          // set by fdtd_create (automatic) or fdtd_set_kernel
    bool T_auto = true;                 // T chosen automatically (re-chosen by fdtd_set_spacing)
    int tiling = 0;                     // fused-kernel tile shape: 0 = auto, 1..3 = explicit
    // Zero-tile skipping: every value that may differ from +0, in both field
    // buffers, lies in the node box [box_lo, box_hi] (empty when lo > hi)
    bool zero_skip = true;
    bool poison = false;                // debug: fill each fused launch's output buffer with NaN first
    int box_lo[3] = {1, 1, 1}, box_hi[3] = {0, 0, 0};
    int zchunk = 0;                     // planes per z chunk (0 = automatic)
    hipStream_t st = nullptr;
    Dims d{};
    char *ws = nullptr;
    bool own_ws = false;
    char *fbuf[2] = {nullptr, nullptr};
    uint8_t *mat = nullptr;
    yee::Ctrl *ctrl = nullptr;
    int n_mat = 0;
    float coef_h[256 * 4];
    float ch[3];
    double eps_h[256];
    double sig_h[256];
    // perfect-conductor entries (sigma = +inf) and, when there are any, the
    // host copy of the cell material index (fdtd_set_fields zeroes the edges
    // those cells own)
    bool pec[256] = {};
    std::vector<uint8_t> mat_h;
    float4 *coef_d = nullptr;
    double *eps_d = nullptr;
    // graded spacing (fdtd_set_spacing) and CPML layers (fdtd_set_cpml):
    // per-index (c dt / (kappa primal size), c dt / (kappa dual size)) pairs,
    // x then y then z; null while the grid is uniform without layers
    float2 *gc_d = nullptr;
    std::vector<double> sizes[3];       // per-index cell sizes (empty: uniform dx, dy, dz)
    CpmlParams pml;                     // layers (pml.n == 0: none)
    float *cp_d = nullptr;              // per axis and index {b_h, a_h, c dt/d, b_e, a_e, c dt/d'}
    double2 *gsz_d = nullptr;           // per axis and node (cell size or 0, dual size; half on walls)
    float *psi_d = nullptr;             // CPML auxiliary state in the layers
    size_t psi_bytes = 0;
    long long psi_off[3] = {};          // x-, y-, z-type blocks (floats)
    int cur = 0;
    long long steps = 0;
    long long block = 0;                // reduced-storage blocks run since the last upload
    // sources
    std::vector<int4> src_pos;
    std::vector<int2> src_wave;
    std::vector<float> samples;
    int4 *src_pos_d = nullptr;
    int2 *src_wave_d = nullptr;
    float *samples_d = nullptr;
    float a_max = 0.0f;
    // probes
    std::vector<int4> probe_pos;
    int4 *probe_pos_d = nullptr;
    double *probe_out_d = nullptr;
    long long probe_cap = 0;            // rows
    // diagnostics scratch
    double *diag_part_d = nullptr;
    double *diag_out_d = nullptr;
    // energy trace (fdtd_set_energy_trace): record k is W^n of the state
    // n = k * energy_every, written when a step starts from that state
    int energy_every = 0;
    double *energy_d = nullptr;         // records (all-ones bits, a NaN, until written)
    long long energy_cap = 0;           // records
    double *epart_d = nullptr;          // per-tile partials of one fused launch
    double *half_eps_d = nullptr;       // eps_r / 2 per material
    // pinned host staging for uploads and read-backs: two buffers of one
    // z-plane of all six components in device layout, used alternately so
    // that host work on one plane overlaps the copy of the other
    char *stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    // live nodes (only when a material is a perfect conductor): conductor
    // interiors whose values are +0 for good are not launched
    yee::LiveNodes *live = nullptr;
    // fused launches since create: workgroups dispatched, tiles of the full tiling
    long long tile_stats[2] = {0, 0};
    // recorded on the stream after the solver's last enqueued steps, so that
    // reading its probes waits for its own work only; the copy then runs on
    // a stream of the library's own (created on first use)
    hipEvent_t done_ev = nullptr;
    bool done_pending = false;
    hipStream_t priv = nullptr;
};

namespace yee {

// One bit per node, 1 = live; row (j, k) is `words` 64-bit words from
// ((k (ny+1) + j) words).  Tile lists are made on first use per geometry.
struct LiveNodes {
    int nx = 0, ny = 0, nz = 0, words = 0;
    std::vector<uint64_t> bits;
    struct List {
        int ox, oy, zc, ntx, nty, ntz;
        int count;
        int *dev;                       // null: every tile is live
        std::vector<int> host;          // source of the (asynchronous) upload
    };
    std::vector<List> lists;
    struct Chunk {
        int ox, oy, T, slots, zmax, zc;
    };
    std::vector<Chunk> chunks;          // chosen z chunk per geometry

    void drop_lists()
    {
        for (List &l : lists)
            if (l.dev) (void)hipFree(l.dev);
        lists.clear();
        chunks.clear();
    }
    void mark(int i, int j, int k)
    {
        if (i < 0 || j < 0 || k < 0 || i > nx || j > ny || k > nz) return;
        bits[((size_t)k * (ny + 1) + j) * words + (i >> 6)] |= 1ULL << (i & 63);
    }
};

const int *live_tile_list(LiveNodes *d, int ox, int oy, int zc, int ntx, int nty, int ntz, int *count,
                          hipStream_t st)
{
    *count = 0;
    for (const LiveNodes::List &l : d->lists)
        if (l.ox == ox && l.oy == oy && l.zc == zc && l.ntx == ntx && l.nty == nty && l.ntz == ntz) {
            *count = l.count;
            return l.dev;
        }
    // a tile (tx, ty, tz) owns x in [tx ox, tx ox + ox), y in [ty oy, ..),
    // z in [tz zc, ..): mark the owner of every live node, skipping the rest
    // of a tile's bits once it is marked
    std::vector<uint8_t> flag((size_t)ntx * nty * ntz, 0);
    for (int k = 0; k <= d->nz; ++k)
        for (int j = 0; j <= d->ny; ++j) {
            const uint64_t *row = &d->bits[((size_t)k * (d->ny + 1) + j) * d->words];
            uint8_t *f = &flag[((size_t)(k / zc) * nty + j / oy) * ntx];
            for (int w = 0; w < d->words; ++w) {
                uint64_t b = row[w];
                while (b) {
                    const int tx = (w * 64 + __builtin_ctzll(b)) / ox;
                    f[tx] = 1;
                    const int next = (tx + 1) * ox - w * 64;    // next tile's first bit in this word
                    if (next >= 64) break;
                    b &= ~0ULL << next;
                }
            }
        }
    LiveNodes::List l{ox, oy, zc, ntx, nty, ntz, 0, nullptr, {}};
    for (size_t t = 0; t < flag.size(); ++t)
        if (flag[t]) l.host.push_back((int)t);
    l.count = (int)l.host.size();
    if (l.host.size() < flag.size()) {
        if (hipMalloc(&l.dev, std::max<size_t>(1, l.host.size()) * sizeof(int)) != hipSuccess) {
            l.dev = nullptr;            // no list: every tile runs
            return nullptr;
        }
        if (!l.host.empty() &&
            hipMemcpyAsync(l.dev, l.host.data(), l.host.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipFree(l.dev);
            return nullptr;
        }
    }
    d->lists.push_back(std::move(l));
    *count = d->lists.back().count;
    return d->lists.back().dev;
}

int live_best_zc(LiveNodes *d, int ox, int oy, int ntx, int nty, int T, int slots, int zmax)
{
    for (const LiveNodes::Chunk &c : d->chunks)
        if (c.ox == ox && c.oy == oy && c.T == T && c.slots == slots && c.zmax == zmax) return c.zc;
    // col[k][ty][tx]: plane k holds a live node in the owned columns of tile (tx, ty)
    const int np = d->nz + 1;
    std::vector<uint8_t> col((size_t)np * nty * ntx, 0);
    for (int k = 0; k < np; ++k)
        for (int j = 0; j <= d->ny; ++j) {
            const uint64_t *row = &d->bits[((size_t)k * (d->ny + 1) + j) * d->words];
            uint8_t *f = &col[((size_t)k * nty + j / oy) * ntx];
            for (int w = 0; w < d->words; ++w) {
                uint64_t b = row[w];
                while (b) {
                    const int tx = (w * 64 + __builtin_ctzll(b)) / ox;
                    f[tx] = 1;
                    const int next = (tx + 1) * ox - w * 64;
                    if (next >= 64) break;
                    b &= ~0ULL << next;
                }
            }
        }
    const int per_plane = ntx * nty;
    std::vector<uint8_t> any(per_plane);
    int best_z = 0;
    double best = 0.0;
    for (int n = 1; n <= np; ++n) {
        const int zz = (np + n - 1) / n;
        if (zz > zmax || (n > 1 && zz == (np + n - 2) / (n - 1))) continue;
        long long listed = 0;
        for (int k0 = 0; k0 < np; k0 += zz) {
            std::fill(any.begin(), any.end(), 0);
            for (int k = k0; k < std::min(np, k0 + zz); ++k)
                for (int t = 0; t < per_plane; ++t) any[t] |= col[(size_t)k * per_plane + t];
            for (int t = 0; t < per_plane; ++t) listed += any[t];
        }
        const double cost = (double)((listed + slots - 1) / slots) * (zz + 1.5 * T);
        if (best_z == 0 || cost < best) { best = cost; best_z = zz; }
    }
    d->chunks.push_back({ox, oy, T, slots, zmax, best_z});
    return best_z;
}

}  // namespace yee

namespace {

void free_dev(void *p)
{
    if (p) (void)hipFree(p);
}

void live_drop(fdtd_solver *s)
{
    if (!s->live) return;
    (void)hipStreamSynchronize(s->st);  // no launch in flight still reads a list
    s->live->drop_lists();
    delete s->live;
    s->live = nullptr;
}

// A source at node (i, j, k) unpins its edge: every node whose E or H
// involves that edge, within {i-1, i} x {j-1, j} x {k-1, k}, becomes live.
void live_mark_source(yee::LiveNodes *d, int i, int j, int k)
{
    for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) d->mark(i + di, j + dj, k + dk);
}

void live_source(fdtd_solver *s, int i, int j, int k)
{
    if (!s->live) return;
    (void)hipStreamSynchronize(s->st);
    s->live->drop_lists();
    live_mark_source(s->live, i, j, k);
}

// A node is dead when its E edges are all pinned -- walls, or owned by a
// perfect-conductor cell, with no source -- each of its H values sees only
// pinned edges, and its six stored values are +0: then every update rewrites
// +0 there (Ca = Cb = 0 for pinned E, a zero curl for H).  pec(i, j, k) tells
// whether cell (i, j, k) is a perfect conductor; nonzero(c, i, j, k) whether
// stored component c is not +0; src holds the sources as (comp, i, j, k).
template <class Pec, class NonZero>
void live_fill(yee::LiveNodes *d, int nx, int ny, int nz, Pec pec, NonZero nonzero, const int4 *src, size_t n_src)
{
    d->nx = nx; d->ny = ny; d->nz = nz;
    d->words = (nx + 1 + 63) / 64;
    d->bits.assign((size_t)(nz + 1) * (ny + 1) * d->words, 0);
    // bit c of P[k & 1][j (nx+1) + i]: E component c at node (i, j, k) is pinned
    const size_t np = (size_t)(nx + 1) * (ny + 1);
    std::vector<uint8_t> P[2] = {std::vector<uint8_t>(np), std::vector<uint8_t>(np)};
    // (the interior tests of e_interior, split into their row and x parts)
    auto pinned_plane = [&](int k, uint8_t *p) {
        const bool kin = k > 0 && k < nz, klt = k < nz;
        for (int j = 0; j <= ny; ++j) {
            const bool jin = j > 0 && j < ny, jlt = j < ny;
            const bool rx = jin && kin, ry = jlt && kin, rz = klt && jin, rc = jlt && klt;
            uint8_t *q = p + (size_t)j * (nx + 1);
            for (int i = 0; i <= nx; ++i) {
                const bool iin = i > 0 && i < nx;
                const bool pc = rc && i < nx && pec(i, j, k);
                q[i] = (uint8_t)((pc || !(rx && i < nx)) | ((pc || !(ry && iin)) << 1) | ((pc || !(rz && iin)) << 2));
            }
        }
    };
    pinned_plane(0, P[0].data());
    for (int k = 0; k <= nz; ++k) {
        const uint8_t *p0 = P[k & 1].data();
        if (k < nz) pinned_plane(k + 1, P[(k + 1) & 1].data());
        const uint8_t *p1 = P[(k + 1) & 1].data();     // read only when k < nz
        for (int j = 0; j <= ny; ++j) {
            uint64_t *row = &d->bits[((size_t)k * (ny + 1) + j) * d->words];
            const uint8_t *a = p0 + (size_t)j * (nx + 1);
            for (int i = 0; i <= nx; ++i) {
                bool dead = a[i] == 7;
                if (dead && j < ny && k < nz)    // Hx: Ez at j and j+1, Ey at k and k+1
                    dead = (a[i + nx + 1] & 4) && (p1[(size_t)j * (nx + 1) + i] & 2);
                if (dead && i < nx && k < nz)    // Hy: Ex at k and k+1, Ez at i and i+1
                    dead = (p1[(size_t)j * (nx + 1) + i] & 1) && (a[i + 1] & 4);
                if (dead && i < nx && j < ny)    // Hz: Ey at i and i+1, Ex at j and j+1
                    dead = (a[i + 1] & 2) && (a[i + nx + 1] & 1);
                for (int c = 0; c < 6 && dead; ++c)
                    dead = !(in_range(nx, ny, nz, c, i, j, k) && nonzero(c, i, j, k));
                if (!dead) row[i >> 6] |= 1ULL << (i & 63);
            }
        }
    }
    for (size_t q = 0; q < n_src; ++q) live_mark_source(d, src[q].y, src[q].z, src[q].w);
}

// The solver's map (none without perfect-conductor cells).
template <class NonZero>
void live_build(fdtd_solver *s, NonZero nonzero)
{
    live_drop(s);
    if (s->mat_h.empty()) return;
    const int nx = s->L.nx, ny = s->L.ny;
    auto *d = new yee::LiveNodes;
    live_fill(
        d, nx, ny, s->L.nz, [&](int i, int j, int k) { return s->pec[s->mat_h[((size_t)k * ny + j) * nx + i]]; },
        nonzero, s->src_pos.data(), s->src_pos.size());
    s->live = d;
}

int upload_sources(fdtd_solver *s)
{
    free_dev(s->src_pos_d);
    free_dev(s->src_wave_d);
    free_dev(s->samples_d);
    s->src_pos_d = nullptr;
    s->src_wave_d = nullptr;
    s->samples_d = nullptr;
    const size_t n = s->src_pos.size();
    if (n == 0) return FDTD_OK;
    hipError_t e;
    if ((e = hipMalloc(&s->src_pos_d, n * sizeof(int4))) != hipSuccess) return hip_fail(e, "hipMalloc(sources)");
    if ((e = hipMalloc(&s->src_wave_d, n * sizeof(int2))) != hipSuccess) return hip_fail(e, "hipMalloc(sources)");
    const size_t ns = std::max<size_t>(1, s->samples.size());
    if ((e = hipMalloc(&s->samples_d, ns * sizeof(float))) != hipSuccess) return hip_fail(e, "hipMalloc(samples)");
    if ((e = hipMemcpyAsync(s->src_pos_d, s->src_pos.data(), n * sizeof(int4), hipMemcpyHostToDevice, s->st)) ||
        (e = hipMemcpyAsync(s->src_wave_d, s->src_wave.data(), n * sizeof(int2), hipMemcpyHostToDevice, s->st)))
        return hip_fail(e, "hipMemcpy(sources)");
    if (!s->samples.empty() &&
        (e = hipMemcpyAsync(s->samples_d, s->samples.data(), s->samples.size() * sizeof(float),
                            hipMemcpyHostToDevice, s->st)))
        return hip_fail(e, "hipMemcpy(samples)");
    if ((e = hipStreamSynchronize(s->st))) return hip_fail(e, "hipStreamSynchronize");
    return FDTD_OK;
}

int ensure_probe_rows(fdtd_solver *s, long long rows)
{
    if (s->probe_pos.empty() || rows <= s->probe_cap) return FDTD_OK;
    long long cap = std::max(rows, 2 * s->probe_cap);
    cap = std::max(cap, 256LL);
    double *p = nullptr;
    hipError_t e;
    const size_t np = s->probe_pos.size();
    if ((e = hipMalloc(&p, (size_t)cap * np * sizeof(double)))) return hip_fail(e, "hipMalloc(probes)");
    // rows start as 0: a tile skipped as all-zero leaves its probes' rows alone
    const size_t keep = (size_t)s->probe_cap * np * sizeof(double);
    if ((e = hipMemsetAsync((char *)p + keep, 0, (size_t)cap * np * sizeof(double) - keep, s->st)) ||
        (s->probe_out_d && (e = hipMemcpyAsync(p, s->probe_out_d, keep, hipMemcpyDeviceToDevice, s->st))) ||
        (e = hipStreamSynchronize(s->st))) {
        free_dev(p);
        return hip_fail(e, "initialise probe rows");
    }
    free_dev(s->probe_out_d);
    s->probe_out_d = p;
    s->probe_cap = cap;
    return FDTD_OK;
}

// Energy records for every state a step may start from below `steps`.
int ensure_energy_rows(fdtd_solver *s, long long steps)
{
    if (s->energy_every <= 0 || steps <= 0) return FDTD_OK;
    const long long need = (steps - 1) / s->energy_every + 1;
    if (need <= s->energy_cap) return FDTD_OK;
    const long long cap = std::max(std::max(need, 2 * s->energy_cap), 64LL);
    double *p = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&p, (size_t)cap * sizeof(double)))) return hip_fail(e, "hipMalloc(energy records)");
    const size_t keep = (size_t)s->energy_cap * sizeof(double);
    if ((e = hipMemsetAsync((char *)p + keep, 0xff, (size_t)cap * sizeof(double) - keep, s->st)) ||
        (s->energy_d && (e = hipMemcpyAsync(p, s->energy_d, keep, hipMemcpyDeviceToDevice, s->st))) ||
        (e = hipStreamSynchronize(s->st))) {
        free_dev(p);
        return hip_fail(e, "initialise energy records");
    }
    free_dev(s->energy_d);
    s->energy_d = p;
    s->energy_cap = cap;
    return FDTD_OK;
}

yee::SourceTable src_table(const fdtd_solver *s)
{
    yee::SourceTable t;
    t.n = (int)s->src_pos.size();
    t.pos = s->src_pos_d;
    t.wave = s->src_wave_d;
    t.samples = s->samples_d;
    return t;
}

yee::ProbeTable probe_table(const fdtd_solver *s)
{
    yee::ProbeTable t;
    t.n = (int)s->probe_pos.size();
    t.pos = s->probe_pos_d;
    t.out = s->probe_out_d;
    t.base = 0;
    return t;
}

yee::StorageBlock storage_block(const fdtd_solver *s)
{
    yee::StorageBlock b;
    b.ctrl = s->ctrl;
    b.slot_in = (int)(s->block % 3);
    b.slot_out = (int)((s->block + 1) % 3);
    b.slot_clear = (int)((s->block + 2) % 3);
    b.par = (int)(s->block % 2);
    b.a_max = s->a_max;
    b.retry = 0;
    return b;
}


// CPML psi arrays: two copies of psi_bytes (the fused kernel reads one and
// writes the other, like the field buffers; the plain kernels update copy
// `cur` in place).
float *psi_buf(const fdtd_solver *s, int which)
{
    return s->psi_d ? s->psi_d + (size_t)which * (s->psi_bytes / sizeof(float)) : nullptr;
}

long long psi_elems(const fdtd_solver *s) { return (long long)(s->psi_bytes / sizeof(float)); }

// Steps per fused pass with CPML layers: T = 2 keeps the twelve psi values
// of every level in registers without spilling (T = 3 spills).
constexpr int CPML_T = 2;

int auto_T(const fdtd_solver *s)
{
    if (s->pml.n > 0) {
        int T = CPML_T;
        while (T > 1 && !yee::cpml_fused_fits(s->L, psi_elems(s), T)) --T;
        return T;
    }
    return yee::fastest_T(s->L, s->storage, s->gc_d != nullptr);
}

// Allocate the pinned staging buffers on first use (freed by fdtd_destroy).
int ensure_staging(fdtd_solver *s)
{
    if (s->stage[0]) return FDTD_OK;
    const size_t bytes = (size_t)s->L.kstride * elem_size(s->storage);
    hipError_t e;
    for (int b = 0; b < 2; ++b) {
        if ((e = hipHostMalloc((void **)&s->stage[b], bytes, hipHostMallocDefault)))
            return hip_fail(e, "hipHostMalloc(staging)");
        if ((e = hipEventCreateWithFlags(&s->stage_ev[b], hipEventDisableTiming)))
            return hip_fail(e, "hipEventCreate(staging)");
    }
    return FDTD_OK;
}

// Staging buffers above 64 MiB (grids with very large planes) are not kept
// pinned between calls.
void release_large_staging(fdtd_solver *s)
{
    if (!s->stage[0] || (size_t)s->L.kstride * elem_size(s->storage) <= (64u << 20)) return;
    for (int b = 0; b < 2; ++b) {
        (void)hipHostFree(s->stage[b]);
        (void)hipEventDestroy(s->stage_ev[b]);
        s->stage[b] = nullptr;
        s->stage_ev[b] = nullptr;
    }
}

int read_ctrl(fdtd_solver *s, yee::Ctrl *out)
{
    hipError_t e = hipMemcpyAsync(out, s->ctrl, sizeof(yee::Ctrl), hipMemcpyDeviceToHost, s->st);
    if (!e) e = hipStreamSynchronize(s->st);
    return e ? hip_fail(e, "hipMemcpy(ctrl)") : FDTD_OK;
}

// Mark the end of the solver's enqueued work (after fdtd_step, fdtd_step_batch).
int record_done(fdtd_solver *s)
{
    hipError_t e = hipSuccess;
    if (!s->done_ev) e = hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming);
    if (!e) e = hipEventRecord(s->done_ev, s->st);
    if (e) return hip_fail(e, "hipEventRecord");
    s->done_pending = true;
    return FDTD_OK;
}

// Length of the next block.  With FP32 storage the result does not depend on
// where blocks fall, so full blocks of T are packed from the current step;
// 16-bit storage re-encodes at every block end, so its blocks end at absolute
// multiples of T (a run split over several calls then rounds where one call
// would).
int next_block(const fdtd_solver *s, int left)
{
    // CPML layers (FP32 storage only) run blocks of at most MAX_T_CPML steps
    const int T = s->pml.n > 0 ? std::min(s->T, yee::MAX_T_CPML) : s->T;
    const int len = s->storage == FDTD_FP32 ? T : T - (int)(s->steps % T);
    return std::min(len, left);
}

// Launch arguments of the next block of solver s (tile geometry excluded).
void fill_fused(const fdtd_solver *s, yee::FusedArgs *a)
{
    std::memset(a, 0, sizeof(*a));
    a->L = s->L;
    a->mat = s->mat;
    a->coef = s->coef_d;
    a->n_mat = s->n_mat;
    a->chx = s->ch[0];
    a->chy = s->ch[1];
    a->chz = s->ch[2];
    a->gc = s->gc_d;
    a->src = src_table(s);
    a->probe = probe_table(s);
    a->fin = s->fbuf[s->cur];
    a->fout = s->fbuf[s->cur ^ 1];
    a->step0 = s->steps;
    a->sb = storage_block(s);
    a->tile_stats = const_cast<long long *>(s->tile_stats);
    a->box_lo = make_int4(-(1 << 28), -(1 << 28), -(1 << 28), 0);   // no tile skipped unless set
    a->box_hi = make_int4(1 << 28, 1 << 28, 1 << 28, 0);
}

// fdtd_step runs the plain kernels: asked for, or the planes (or, with
// CPML layers, the psi arrays) too large for the fused kernel's 32-bit
// addressing.
bool runs_plain(const fdtd_solver *s)
{
    return s->kernel == FDTD_KERNEL_PLAIN ||
           (s->pml.n > 0 && !yee::cpml_fused_fits(s->L, psi_elems(s), std::min(s->T, yee::MAX_T_CPML))) ||
           (s->kernel == FDTD_KERNEL_AUTO && !yee::fused_fits(s->L, s->storage, 1));
}

void advance(fdtd_solver *s, int len)
{
    s->cur ^= 1;
    s->steps += len;
    s->block += 1;
}

// The box after `len` more steps from step s->steps: the current box and the
// points of the sources that still have samples, widened by len nodes on
// every axis (the stencil reaches one node per step), clipped to the grid.
void box_add_point(fdtd_solver *s, const int p[3])
{
    const bool empty = s->box_lo[0] > s->box_hi[0];
    for (int ax = 0; ax < 3; ++ax) {
        s->box_lo[ax] = empty ? p[ax] : std::min(s->box_lo[ax], p[ax]);
        s->box_hi[ax] = empty ? p[ax] : std::max(s->box_hi[ax], p[ax]);
    }
}

// Take in the stored values q[i0..i1) of row (j, k) that are not +0 (any bit set).
template <class Q>
void box_add_row(fdtd_solver *s, const Q *q, int i0, int i1, int j, int k)
{
    int first = i0;
    while (first < i1 && q[first] == 0 && !std::signbit((double)q[first])) ++first;
    if (first == i1) return;
    int last = i1 - 1;
    while (q[last] == 0 && !std::signbit((double)q[last])) --last;
    const int a[3] = {first, j, k}, b[3] = {last, j, k};
    box_add_point(s, a);
    box_add_point(s, b);
}

void box_take_sources(fdtd_solver *s)
{
    for (size_t q = 0; q < s->src_pos.size(); ++q) {
        if (s->src_wave[q].y <= s->steps) continue;     // no samples left
        const int p[3] = {s->src_pos[q].y, s->src_pos[q].z, s->src_pos[q].w};
        box_add_point(s, p);
    }
}

void box_grow(fdtd_solver *s, int len)
{
    if (s->box_lo[0] > s->box_hi[0]) return;
    const int n[3] = {s->L.nx, s->L.ny, s->L.nz};
    for (int ax = 0; ax < 3; ++ax) {
        s->box_lo[ax] = std::max(0, s->box_lo[ax] - len);
        s->box_hi[ax] = std::min(n[ax], s->box_hi[ax] + len);
    }
}

// Kernel form of the box: outside the grid when empty, covering everything
// when skipping is off.
void box_args(const fdtd_solver *s, yee::FusedArgs *a)
{
    constexpr int FAR = 1 << 28;
    if (!s->zero_skip) {
        a->box_lo = make_int4(-FAR, -FAR, -FAR, 0);
        a->box_hi = make_int4(FAR, FAR, FAR, 0);
    } else if (s->box_lo[0] > s->box_hi[0]) {
        a->box_lo = a->box_hi = make_int4(-FAR, -FAR, -FAR, 0);
    } else {
        a->box_lo = make_int4(s->box_lo[0], s->box_lo[1], s->box_lo[2], 0);
        a->box_hi = make_int4(s->box_hi[0], s->box_hi[1], s->box_hi[2], 0);
    }
}

// Per-index tables of graded spacing (sizes d[axis][q], q < n[axis]) with
// CPML layers of p.n cells folded in: cag = n_mat x {Ca, G}; gc = per axis
// and node q {c dt / (kappa_h d[q]), c dt / (kappa_e d'[q])} (0 past the
// last cell, and on the walls for the dual one); cp (if not null) = per axis
// and node q {b_h, a_h, c dt / d[q], b_e, a_e, c dt / d'[q]}, the CFS-CPML
// recursion coefficients of the H value at cell q and the E value at node q
// (zero outside the layers).  Profiles at depth rho cells into a layer,
// x = rho / n: sigma = sigma_max x^m, kappa = 1 + (kappa_max - 1) x^m,
// alpha = alpha_max (1 - x), b = exp(-(sigma/kappa + alpha) dt / eps0),
// a = sigma (b - 1) / (kappa (sigma + kappa alpha)), with
// sigma_max = sigma_factor 0.8 (m + 1) / (eta0 d_out) for the outermost cell
// size d_out of the face.  All in FP64, each table value rounded once.
int graded_tables(const fdtd_material *table, int n_mat, const int n[3], const double *const d[3], double dt,
                  const CpmlParams &p, float *cag, float *gc, float *cp)
{
    if (!table || !cag || !gc || n_mat < 1 || n_mat > 256) return fail(FDTD_EINVAL, "NULL argument or bad table");
    if (n[0] < 2 || n[1] < 2 || n[2] < 2 || !(dt > 0)) return fail(FDTD_EINVAL, "bad dimensions or dt");
    for (int m = 0; m < n_mat; ++m) {
        const double eps = table[m].eps_r, sig = table[m].sigma;
        if (!(eps > 0) || !(sig >= 0) || table[m].mu_r != 1.0 || !std::isfinite(eps))
            return fail(FDTD_EINVAL, "material " + std::to_string(m) + ": need eps_r > 0, sigma >= 0, mu_r = 1");
        if (std::isinf(sig)) {              // perfect conductor
            cag[2 * m + 0] = cag[2 * m + 1] = 0.0f;
            continue;
        }
        const double a = (sig * dt) / (2.0 * EPS0 * eps);
        cag[2 * m + 0] = (float)((1.0 - a) / (1.0 + a));
        cag[2 * m + 1] = (float)((1.0 / eps) / (1.0 + a));
    }
    const int N = p.n;
    if (N < 0 || (N > 0 && (p.order < 1 || p.order > 8 || !(p.sigma_factor >= 0) || !(p.kappa_max >= 1) ||
                            !(p.alpha_max >= 0) || !std::isfinite(p.sigma_factor) || !std::isfinite(p.kappa_max) ||
                            !std::isfinite(p.alpha_max))))
        return fail(FDTD_EINVAL, "CPML: need order 1..8, sigma_factor >= 0, kappa_max >= 1, alpha_max >= 0");
    const double cdt = C0 * dt;
    const double eta0 = 1.0 / (EPS0 * C0);
    int off = 0;
    for (int ax = 0; ax < 3; ++ax) {
        const int nn = n[ax];
        const double *dd = d[ax];
        if (!dd) return fail(FDTD_EINVAL, "NULL cell sizes");
        if (N > 0 && 2 * N >= nn) return fail(FDTD_EINVAL, "CPML layers must leave an interior on every axis");
        for (int q = 0; q < nn; ++q)
            if (!(dd[q] > 0) || !std::isfinite(dd[q])) return fail(FDTD_EINVAL, "cell sizes must be > 0");
        const double smax_lo = N > 0 ? p.sigma_factor * 0.8 * (p.order + 1) / (eta0 * dd[0]) : 0.0;
        const double smax_hi = N > 0 ? p.sigma_factor * 0.8 * (p.order + 1) / (eta0 * dd[nn - 1]) : 0.0;
        for (int q = 0; q <= nn; ++q) {
            float *g = gc + 2 * (off + q);
            float *c = cp ? cp + 6 * (off + q) : nullptr;
            g[0] = g[1] = 0.0f;
            if (c) for (int v = 0; v < 6; ++v) c[v] = 0.0f;
            for (int half = 0; half < 2; ++half) {      // 0: H at cell q (q + 1/2), 1: E at node q
                if (half == 0 && q == nn) continue;
                if (half == 1 && (q == 0 || q == nn)) continue;
                const double pos = half == 0 ? q + 0.5 : (double)q;
                double rho = 0.0, smax = 0.0;
                if (N > 0 && pos < N) { rho = N - pos; smax = smax_lo; }
                else if (N > 0 && pos > nn - N) { rho = pos - (nn - N); smax = smax_hi; }
                const bool inside = half == 0 ? (q < N || q >= nn - N) : ((q > 0 && q < N) || (q > nn - N && q < nn));
                double kappa = 1.0, b = 0.0, a = 0.0;
                if (rho > 0.0) {
                    const double x = rho / N, xm = std::pow(x, p.order);
                    const double sg = smax * xm, al = p.alpha_max * (1.0 - x);
                    kappa = 1.0 + (p.kappa_max - 1.0) * xm;
                    b = std::exp(-(sg / kappa + al) * dt / EPS0);
                    a = sg > 0.0 ? sg * (b - 1.0) / (kappa * (sg + kappa * al)) : 0.0;
                }
                const double size = half == 0 ? dd[q] : (dd[q - 1] + dd[q]) / 2.0;
                g[half] = (float)(kappa != 1.0 ? cdt / (kappa * size) : cdt / size);
                if (c && N > 0 && inside) {
                    c[3 * half + 0] = (float)b;
                    c[3 * half + 1] = (float)a;
                }
                if (c) c[3 * half + 2] = (float)(cdt / size);
            }
        }
        off += nn + 1;
    }
    return FDTD_OK;
}

// Courant bound of the smallest size per axis.  Sufficient: along an axis
// the second difference through node q (dual size = mean of cells q-1 and
// q) has row sum 4 / (d[q-1] d[q]) <= 4 / min d^2, the curl-curl operator of
// a tensor-product grid is bounded by the sum over axes, and CPML stretching
// (kappa >= 1) only lowers the coefficients.
double graded_courant_limit(const int n[3], const double *const d[3])
{
    double sum = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double m = *std::min_element(d[ax], d[ax] + n[ax]);
        sum += 1.0 / (m * m);
    }
    return 1.0 / (C0 * std::sqrt(sum));
}

// Build and upload the per-index tables for cell sizes sz (empty: uniform)
// and layers p; on success the solver adopts both.
int apply_graded(fdtd_solver *s, const std::vector<double> *sz, const CpmlParams &p)
{
    const int n[3] = {s->L.nx, s->L.ny, s->L.nz};
    const double uni[3] = {s->dx, s->dy, s->dz};
    std::vector<double> full[3];
    const double *d[3];
    for (int ax = 0; ax < 3; ++ax) {
        if (sz[ax].empty()) full[ax].assign(n[ax], uni[ax]);
        else full[ax] = sz[ax];
        d[ax] = full[ax].data();
    }
    fdtd_material table[256];
    for (int m = 0; m < s->n_mat; ++m) {
        table[m].eps_r = s->eps_h[m];
        table[m].mu_r = 1.0;
        table[m].sigma = s->sig_h[m];
    }
    const size_t nidx = (size_t)n[0] + n[1] + n[2] + 3;
    float cag[2 * 256];
    std::vector<float> gc(2 * nidx), cp(6 * nidx);
    std::vector<double2> gsz(nidx);     // sizes for the diagnostics' volume weights
    for (int ax = 0, off = 0; ax < 3; off += n[ax] + 1, ++ax)
        for (int q = 0; q <= n[ax]; ++q) {
            const double *dd = d[ax];
            const double dual = q == 0 ? dd[0] / 2.0 : (q == n[ax] ? dd[n[ax] - 1] / 2.0 : (dd[q - 1] + dd[q]) / 2.0);
            gsz[off + q] = make_double2(q < n[ax] ? dd[q] : 0.0, dual);
        }
    int rc = graded_tables(table, s->n_mat, n, d, s->dt, p, cag, gc.data(), cp.data());
    if (rc) return rc;
    const double limit = graded_courant_limit(n, d);
    if (s->dt > limit)
        return fail(FDTD_ECFL, "dt exceeds the Courant limit " + std::to_string(limit) + " of the smallest cells");
    if (!s->T_auto && s->T > yee::MAX_T_GRADED)
        return fail(FDTD_EINVAL, "graded spacing runs blocks of at most " + std::to_string(yee::MAX_T_GRADED) +
                                     " steps; lower time_block first");
    float coef[256 * 4];
    for (int m = 0; m < s->n_mat; ++m) {
        coef[4 * m + 0] = cag[2 * m + 0];
        coef[4 * m + 1] = cag[2 * m + 1];
        coef[4 * m + 2] = coef[4 * m + 3] = 0.0f;
    }
    // psi blocks of 4-float groups: x-type 2n (ny+1)(nz+1) groups, y-type
    // 2n (nx+1)(nz+1), z-type 2n (nx+1)(ny+1)
    long long off[3] = {};
    size_t psi_bytes = 0;
    if (p.n > 0) {
        const long long per[3] = {2LL * p.n * (n[1] + 1) * (n[2] + 1), 2LL * p.n * (n[0] + 1) * (n[2] + 1),
                                  2LL * p.n * (n[0] + 1) * (n[1] + 1)};
        long long at = 0;
        for (int ax = 0; ax < 3; ++ax) {
            off[ax] = at;
            at += 4 * per[ax];
        }
        psi_bytes = (size_t)at * sizeof(float);
    }
    // Fill fresh device buffers and adopt them only once every copy has
    // completed, so that a failure leaves the solver exactly as it was.
    hipError_t e = hipSuccess;
    float2 *gc_d = nullptr;
    double2 *gsz_d = nullptr;
    float *cp_d = nullptr, *psi_d = nullptr;
    float4 *coef_d = nullptr;
    auto drop = [&]() {
        free_dev(gc_d);
        free_dev(gsz_d);
        free_dev(cp_d);
        free_dev(psi_d);
        free_dev(coef_d);
    };
    if ((e = hipMalloc(&gc_d, gc.size() * sizeof(float))) || (e = hipMalloc(&gsz_d, gsz.size() * sizeof(double2))) ||
        (e = hipMalloc(&coef_d, 256 * sizeof(float4))) ||
        (p.n > 0 && (e = hipMalloc(&cp_d, cp.size() * sizeof(float)))) ||
        (psi_bytes && (e = hipMalloc(&psi_d, 2 * psi_bytes)))) {
        drop();
        return hip_fail(e, "hipMalloc(graded tables)");
    }
    if ((e = hipMemcpyAsync(gc_d, gc.data(), gc.size() * sizeof(float), hipMemcpyHostToDevice, s->st)) ||
        (e = hipMemcpyAsync(gsz_d, gsz.data(), gsz.size() * sizeof(double2), hipMemcpyHostToDevice, s->st)) ||
        (e = hipMemcpyAsync(coef_d, coef, s->n_mat * sizeof(float4), hipMemcpyHostToDevice, s->st)) ||
        (p.n > 0 && (e = hipMemcpyAsync(cp_d, cp.data(), cp.size() * sizeof(float), hipMemcpyHostToDevice, s->st))) ||
        (psi_bytes && (e = hipMemsetAsync(psi_d, 0, 2 * psi_bytes, s->st))) ||
        (e = hipStreamSynchronize(s->st))) {
        drop();
        return hip_fail(e, "upload graded tables");
    }
    std::swap(s->gc_d, gc_d);
    std::swap(s->gsz_d, gsz_d);
    std::swap(s->coef_d, coef_d);
    std::swap(s->cp_d, cp_d);
    std::swap(s->psi_d, psi_d);
    drop();                             // the solver's previous buffers
    s->psi_bytes = psi_bytes;
    std::memcpy(s->coef_h, coef, s->n_mat * 4 * sizeof(float));
    for (int ax = 0; ax < 3; ++ax) s->sizes[ax] = sz[ax];
    s->pml = p;
    std::memcpy(s->psi_off, off, sizeof(off));
    if (s->T_auto) s->T = auto_T(s);
    return FDTD_OK;
}

hipError_t launch_diagnostics(fdtd_solver *s, double *partial, double *dout);
int ensure_diag_buffers(fdtd_solver *s);

yee::Cpml cpml_args(const fdtd_solver *s)
{
    yee::Cpml c;
    c.n = s->pml.n;
    c.cp = s->cp_d;
    c.psi = psi_buf(s, s->cur);
    std::memcpy(c.base, s->psi_off, sizeof(c.base));
    c.elems = (long long)(s->psi_bytes / sizeof(float));
    return c;
}

}  // namespace

extern "C" {

const char *fdtd_last_error(void) { return g_err.c_str(); }

size_t fdtd_workspace_bytes(int nx, int ny, int nz, int storage)
{
    if (nx < 2 || ny < 2 || nz < 2 || storage < 0 || storage > 2) return 0;
    if ((long long)(nx + 1) * (ny + 1) >= (1LL << 31)) return 0;
    return dims_for(nx, ny, nz, storage).total;
}

int fdtd_coefficients(const fdtd_material *table, int n_materials, double dx, double dy, double dz, double dt,
                      float *out, float *ch)
{
    if (!table || !out || !ch || n_materials < 1 || n_materials > 256) return fail(FDTD_EINVAL, "bad table");
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !(dt > 0)) return fail(FDTD_EINVAL, "bad spacing or dt");
    for (int m = 0; m < n_materials; ++m) {
        const double eps = table[m].eps_r, sig = table[m].sigma;
        if (!(eps > 0) || !(sig >= 0) || table[m].mu_r != 1.0 || !std::isfinite(eps))
            return fail(FDTD_EINVAL, "material " + std::to_string(m) + ": need eps_r > 0, sigma >= 0, mu_r = 1");
        if (std::isinf(sig)) {              // perfect conductor: the owned edges stay zero
            for (int v = 0; v < 4; ++v) out[4 * m + v] = 0.0f;
            continue;
        }
        // semi-implicit loss: a = sigma dt / (2 eps0 eps_r)
        const double a = (sig * dt) / (2.0 * EPS0 * eps);
        const double cb = ((C0 * dt) / eps) / (1.0 + a);
        out[4 * m + 0] = (float)((1.0 - a) / (1.0 + a));
        out[4 * m + 1] = (float)(cb / dx);
        out[4 * m + 2] = (float)(cb / dy);
        out[4 * m + 3] = (float)(cb / dz);
    }
    ch[0] = (float)((C0 * dt) / dx);
    ch[1] = (float)((C0 * dt) / dy);
    ch[2] = (float)((C0 * dt) / dz);
    return FDTD_OK;
}

int fdtd_graded_coefficients(const fdtd_material *table, int n_materials, int nx, int ny, int nz,
                             const double *dx, const double *dy, const double *dz, double dt,
                             float *cag, float *gc)
{
    const int n[3] = {nx, ny, nz};
    const double *d[3] = {dx, dy, dz};
    return graded_tables(table, n_materials, n, d, dt, CpmlParams(), cag, gc, nullptr);
}

int fdtd_live_nodes(const fdtd_material *table, int n_materials, const uint8_t *mat_index, int nx, int ny, int nz,
                    const int *sources, int n_sources, uint8_t *live)
{
    if (!table || !mat_index || !live || (n_sources > 0 && !sources)) return fail(FDTD_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || nz < 1 || n_materials < 1 || n_materials > 256 || n_sources < 0)
        return fail(FDTD_EINVAL, "bad sizes");
    const size_t ncell = (size_t)nx * ny * nz;
    for (size_t q = 0; q < ncell; ++q)
        if (mat_index[q] >= n_materials) return fail(FDTD_EINVAL, "material index out of range");
    std::vector<int4> src(n_sources);
    for (int q = 0; q < n_sources; ++q) {
        src[q] = make_int4(sources[4 * q], sources[4 * q + 1], sources[4 * q + 2], sources[4 * q + 3]);
        if (!e_interior(nx, ny, nz, src[q].x, src[q].y, src[q].z, src[q].w))
            return fail(FDTD_EINVAL, "source must sit on an interior E edge");
    }
    bool pt[256] = {};
    for (int m = 0; m < n_materials; ++m) pt[m] = std::isinf(table[m].sigma);
    yee::LiveNodes d;
    live_fill(
        &d, nx, ny, nz, [&](int i, int j, int k) { return pt[mat_index[((size_t)k * ny + j) * nx + i]]; },
        [](int, int, int, int) { return false; }, src.data(), src.size());
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j) {
            const uint64_t *row = &d.bits[((size_t)k * (ny + 1) + j) * d.words];
            for (int i = 0; i <= nx; ++i)
                live[((size_t)k * (ny + 1) + j) * (nx + 1) + i] = (uint8_t)((row[i >> 6] >> (i & 63)) & 1u);
        }
    return FDTD_OK;
}

int fdtd_cpml_coefficients(const fdtd_material *table, int n_materials, int nx, int ny, int nz,
                           const double *dx, const double *dy, const double *dz, double dt,
                           int thickness, int order, double sigma_factor, double kappa_max, double alpha_max,
                           float *cag, float *gc, float *cp)
{
    if (!cp) return fail(FDTD_EINVAL, "NULL argument");
    if (thickness < 1) return fail(FDTD_EINVAL, "CPML thickness must be >= 1");
    CpmlParams p;
    p.n = thickness;
    p.order = order;
    p.sigma_factor = sigma_factor;
    p.kappa_max = kappa_max;
    p.alpha_max = alpha_max;
    const int n[3] = {nx, ny, nz};
    const double *d[3] = {dx, dy, dz};
    return graded_tables(table, n_materials, n, d, dt, p, cag, gc, cp);
}

int fdtd_create(fdtd_solver **out, int nx, int ny, int nz, double dx, double dy, double dz, double dt,
                const fdtd_material *table, int n_materials, const uint8_t *mat_index, int storage,
                void *device_workspace, size_t workspace_bytes, void *hip_stream)
{
    if (!out) return fail(FDTD_EINVAL, "out is NULL");
    if (nx < 2 || ny < 2 || nz < 2) return fail(FDTD_EINVAL, "need at least 2 cells per axis");
    if ((long long)(nx + 1) * (ny + 1) >= (1LL << 31)) return fail(FDTD_EINVAL, "plane too large");
    if (storage < 0 || storage > 2) return fail(FDTD_EINVAL, "bad storage format");
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !(dt > 0)) return fail(FDTD_EINVAL, "bad spacing or dt");
    const double limit = 1.0 / (C0 * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz)));
    if (dt > limit) return fail(FDTD_ECFL, "dt exceeds the Courant limit " + std::to_string(limit));

    fdtd_solver *s = new (std::nothrow) fdtd_solver();
    if (!s) return fail(FDTD_ENOMEM, "host allocation failed");
    int rc = fdtd_coefficients(table, n_materials, dx, dy, dz, dt, s->coef_h, s->ch);
    if (rc) { delete s; return rc; }
    const size_t ncell = (size_t)nx * ny * nz;
    if (mat_index)
        for (size_t q = 0; q < ncell; ++q)
            if (mat_index[q] >= n_materials) {
                delete s;
                return fail(FDTD_EINVAL, "material index " + std::to_string(mat_index[q]) + " >= n_materials");
            }
    s->n_mat = n_materials;
    bool any_pec = false;
    for (int m = 0; m < n_materials; ++m) {
        s->eps_h[m] = table[m].eps_r;
        s->sig_h[m] = table[m].sigma;
        s->pec[m] = std::isinf(table[m].sigma);
        any_pec = any_pec || s->pec[m];
    }
    if (any_pec && mat_index) s->mat_h.assign(mat_index, mat_index + ncell);
    else if (any_pec && s->pec[0]) s->mat_h.assign(ncell, 0);
    s->dx = dx; s->dy = dy; s->dz = dz; s->dt = dt;
    s->storage = storage;
    s->st = (hipStream_t)hip_stream;
    s->d = dims_for(nx, ny, nz, storage);
    s->L.nx = nx; s->L.ny = ny; s->L.nz = nz;
    s->L.pitch = s->d.pitch;
    s->L.plane = s->d.plane;
    s->L.cstride = s->d.plane;
    s->L.kstride = s->d.kstride;
    s->T = auto_T(s);
    if (!yee::fused_fits(s->L, storage, 1) && storage != FDTD_FP32) {
        delete s;
        return fail(FDTD_EINVAL, "grid planes too large for the fused kernel, and the plain kernel needs FP32 storage");
    }

    hipError_t e;
    if (device_workspace) {
        if (workspace_bytes < s->d.total || ((uintptr_t)device_workspace & 255u)) {
            delete s;
            return fail(FDTD_ENOMEM, "workspace smaller than fdtd_workspace_bytes or not 256-byte aligned");
        }
        s->ws = (char *)device_workspace;
    } else {
        if ((e = hipMalloc(&s->ws, s->d.total))) { delete s; return fail(FDTD_ENOMEM, std::string("hipMalloc(workspace): ") + hipGetErrorString(e)); }
        s->own_ws = true;
    }
    s->fbuf[0] = s->ws;
    s->fbuf[1] = s->ws + s->d.fbytes;
    s->mat = (uint8_t *)(s->ws + 2 * s->d.fbytes);
    s->ctrl = (yee::Ctrl *)(s->ws + 2 * s->d.fbytes + s->d.matbytes);

    // material index in the padded box layout (zero outside the cells)
    {
        std::vector<uint8_t> box((size_t)s->d.plane * (nz + 1), 0);
        if (mat_index)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    std::memcpy(&box[(size_t)k * s->d.plane + (size_t)j * s->d.pitch],
                                mat_index + ((size_t)k * ny + j) * nx, nx);
        if ((e = hipMemcpyAsync(s->mat, box.data(), box.size(), hipMemcpyHostToDevice, s->st)) ||
            (e = hipStreamSynchronize(s->st))) {
            fdtd_destroy(s);
            return hip_fail(e, "upload material index");
        }
    }
    if ((e = hipMalloc(&s->coef_d, 256 * sizeof(float4))) || (e = hipMalloc(&s->eps_d, 256 * sizeof(double)))) {
        fdtd_destroy(s);
        return hip_fail(e, "hipMalloc(tables)");
    }
    if ((e = hipMemcpyAsync(s->coef_d, s->coef_h, n_materials * sizeof(float4), hipMemcpyHostToDevice, s->st)) ||
        (e = hipMemcpyAsync(s->eps_d, s->eps_h, n_materials * sizeof(double), hipMemcpyHostToDevice, s->st))) {
        fdtd_destroy(s);
        return hip_fail(e, "upload tables");
    }
    rc = fdtd_set_fields(s, nullptr);
    if (rc) { fdtd_destroy(s); return rc; }
    *out = s;
    return FDTD_OK;
}

int fdtd_set_spacing(fdtd_solver *s, const double *dx, const double *dy, const double *dz)
{
    if (!s || !dx || !dy || !dz) return fail(FDTD_EINVAL, "NULL argument");
    if (s->steps > 0) return fail(FDTD_ESTATE, "spacing must be set before the first step");
    std::vector<double> sz[3] = {std::vector<double>(dx, dx + s->L.nx), std::vector<double>(dy, dy + s->L.ny),
                                 std::vector<double>(dz, dz + s->L.nz)};
    return apply_graded(s, sz, s->pml);
}

int fdtd_set_cpml(fdtd_solver *s, int thickness, int order, double sigma_factor, double kappa_max,
                  double alpha_max)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (s->steps > 0) return fail(FDTD_ESTATE, "CPML layers must be set before the first step");
    if (s->storage != FDTD_FP32) return fail(FDTD_EINVAL, "CPML layers need FP32 storage");
    if (thickness < 0) return fail(FDTD_EINVAL, "negative CPML thickness");
    if (thickness > 0 && s->kernel == FDTD_KERNEL_FUSED) {
        const long long nx = s->L.nx, ny = s->L.ny, nz = s->L.nz;
        const long long elems = 8LL * thickness * ((ny + 1) * (nz + 1) + (nx + 1) * (nz + 1) + (nx + 1) * (ny + 1));
        if ((!s->T_auto && s->T > yee::MAX_T_CPML) || !yee::cpml_fused_fits(s->L, elems, 1))
            return fail(FDTD_EINVAL, "CPML layers run fused blocks of at most " + std::to_string(yee::MAX_T_CPML) +
                                         " steps (and arrays below 2 GiB); lower time_block first");
    }
    CpmlParams p;
    p.n = thickness;
    p.order = order;
    p.sigma_factor = sigma_factor;
    p.kappa_max = kappa_max;
    p.alpha_max = alpha_max;
    return apply_graded(s, s->sizes, p);
}

int fdtd_set_kernel(fdtd_solver *s, int kernel, int time_block)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (kernel < 0 || kernel > 2) return fail(FDTD_EINVAL, "bad kernel family");
    if (time_block < 0 || time_block > yee::MAX_T)
        return fail(FDTD_EINVAL, "time_block must be 0 (automatic) or 1.." + std::to_string(yee::MAX_T));
    if (s->gc_d && time_block > yee::MAX_T_GRADED)
        return fail(FDTD_EINVAL, "graded spacing runs blocks of at most " + std::to_string(yee::MAX_T_GRADED) + " steps");
    const bool automatic = time_block == 0;
    if (automatic) time_block = auto_T(s);
    if (kernel == FDTD_KERNEL_AUTO)   // AUTO lowers T to what the grid allows (plain if nothing fits)
        while (time_block > 1 && !yee::fused_fits(s->L, s->storage, time_block)) --time_block;
    if (kernel == FDTD_KERNEL_PLAIN && s->storage != FDTD_FP32)
        return fail(FDTD_EINVAL, "the plain kernel needs FP32 storage");
    if (kernel == FDTD_KERNEL_FUSED && !yee::fused_fits(s->L, s->storage, time_block))
        return fail(FDTD_EINVAL, "grid planes too large for the fused kernel; use the plain kernel");
    if (kernel == FDTD_KERNEL_FUSED && s->pml.n > 0 && !yee::cpml_fused_fits(s->L, psi_elems(s), time_block))
        return fail(FDTD_EINVAL, "CPML layers run fused blocks of at most " + std::to_string(yee::MAX_T_CPML) +
                                     " steps (and arrays below 2 GiB)");
    s->kernel = kernel;
    s->T = time_block;
    s->T_auto = automatic;
    return FDTD_OK;
}

int fdtd_tile_stats(const fdtd_solver *s, long long *dispatched, long long *full)
{
    if (!s || !dispatched || !full) return fail(FDTD_EINVAL, "NULL argument");
    *dispatched = s->tile_stats[0];
    *full = s->tile_stats[1];
    return FDTD_OK;
}

int fdtd_set_zero_skip(fdtd_solver *s, int enable)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    s->zero_skip = enable != 0;
    return FDTD_OK;
}

int fdtd_set_poison(fdtd_solver *s, int enable)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (!enable && s->poison) {
        // the second buffer now holds NaN outside what the last launch wrote
        // (its padding): restore +0 there for the zero-tile invariant
        hipError_t e = hipMemsetAsync(s->fbuf[s->cur ^ 1], 0, s->d.fbytes, s->st);
        if (!e && s->psi_d) e = hipMemsetAsync(psi_buf(s, s->cur ^ 1), 0, s->psi_bytes, s->st);
        if (e) return hip_fail(e, "clear poison");
    }
    s->poison = enable != 0;
    return FDTD_OK;
}

int fdtd_set_tiling(fdtd_solver *s, int variant, int z_chunk)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (variant < 0 || variant > 3) return fail(FDTD_EINVAL, "tiling variant must be 0 (auto) or 1..3");
    if (z_chunk < 0) return fail(FDTD_EINVAL, "negative z chunk");
    s->tiling = variant;
    s->zchunk = z_chunk;
    return FDTD_OK;
}

int fdtd_set_fields(fdtd_solver *s, const float *host)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    const int nx = s->L.nx, ny = s->L.ny, nz = s->L.nz;
    const size_t nbox = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int es = elem_size(s->storage);
    hipError_t e;
    if ((e = hipStreamSynchronize(s->st))) return hip_fail(e, "hipStreamSynchronize");
    yee::Ctrl ctrl;
    std::memset(&ctrl, 0, sizeof(ctrl));
    s->cur = 0;
    s->block = 0;
    s->box_lo[0] = 1;                   // empty box: filled below from the uploaded values
    s->box_hi[0] = 0;
    // both buffers start as +0 outside the uploaded values (the zero-tile skip
    // relies on the older buffer too)
    if ((e = hipMemsetAsync(s->fbuf[1], 0, s->d.fbytes, s->st))) return hip_fail(e, "hipMemset");
    if (s->psi_d && (e = hipMemsetAsync(s->psi_d, 0, 2 * s->psi_bytes, s->st)))
        return hip_fail(e, "clear CPML state");
    if (!host) {
        if ((e = hipMemsetAsync(s->fbuf[0], 0, s->d.fbytes, s->st)) ||
            (e = hipMemcpyAsync(s->ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice, s->st)) ||
            (e = hipStreamSynchronize(s->st)))
            return hip_fail(e, "zero fields");
        live_build(s, [](int, int, int, int) { return false; });
        return FDTD_OK;
    }
    // Stored values per component and row: positions outside the component's
    // range, tangential E on the walls and E on edges owned by perfect-conductor
    // cells are zero.  Pass 1: maxima (for the reduced-storage scales); pass 2:
    // clean, encode and upload plane by plane.
    const size_t nplane = (size_t)(nx + 1) * (ny + 1);
    const bool has_pec = !s->mat_h.empty();
    auto pec_owned = [&](int c, int i, int j, int k) {
        return c < 3 && i < nx && j < ny && k < nz && s->pec[s->mat_h[((size_t)k * ny + j) * nx + i]];
    };
    float m[6] = {0, 0, 0, 0, 0, 0};
    int sc[6] = {0, 0, 0, 0, 0, 0};
    if (s->storage != FDTD_FP32) {
        for (int c = 0; c < 6; ++c)
            for (int k = 0; k <= nz; ++k)
                for (int j = 0; j <= ny; ++j) {
                    int i0, i1;
                    if (!row_span(nx, ny, nz, c, j, k, &i0, &i1)) continue;
                    const float *row = host + (size_t)c * nbox + (size_t)k * nplane + (size_t)j * (nx + 1);
                    for (int i = i0; i < i1; ++i)
                        if (!(has_pec && pec_owned(c, i, j, k))) m[c] = std::max(m[c], std::fabs(row[i]));
                }
        choose_scales(m, s->a_max, sc);
    }
    if (int rc = ensure_staging(s)) return rc;
    if ((e = hipMemsetAsync(s->fbuf[0], 0, s->d.fbytes, s->st))) return hip_fail(e, "hipMemset");
    // One copy per z plane: the six components of plane k are contiguous on
    // the device (kstride = 6 planes), so they are laid out in a pinned buffer
    // exactly as on the device (pitched rows, zeros in the padding) and sent in
    // one transfer; the other buffer is filled meanwhile.
    float mx[6] = {0, 0, 0, 0, 0, 0};
    bool sat = false;
    float upf[6], dnf[6];
    for (int c = 0; c < 6; ++c) {
        upf[c] = std::ldexp(1.0f, sc[c]);
        dnf[c] = std::ldexp(1.0f, -sc[c]);
    }
    const size_t pitch = (size_t)s->d.pitch;
    for (int k = 0; k <= nz; ++k) {
        const int b = k & 1;
        if (k >= 2 && (e = hipEventSynchronize(s->stage_ev[b]))) return hip_fail(e, "upload fields");
        char *buf = s->stage[b];
        std::memset(buf, 0, (size_t)s->L.kstride * es);
        for (int c = 0; c < 6; ++c) {
            const float *src = host + (size_t)c * nbox + (size_t)k * nplane;
            for (int j = 0; j <= ny; ++j) {
                int i0 = 0, i1 = 0;
                if (!row_span(nx, ny, nz, c, j, k, &i0, &i1)) continue;
                const float *row = src + (size_t)j * (nx + 1);
                const size_t at = (size_t)c * s->L.cstride + (size_t)j * pitch;
                if (s->storage == FDTD_FP32) {
                    float *q = (float *)buf + at;
                    std::memcpy(q + i0, row + i0, (size_t)(i1 - i0) * sizeof(float));
                    if (has_pec && c < 3)
                        for (int i = i0; i < i1; ++i)
                            if (pec_owned(c, i, j, k)) q[i] = 0.0f;
                    box_add_row(s, q, i0, i1, j, k);
                } else {
                    uint16_t *q = (uint16_t *)buf + at;
                    for (int i = i0; i < i1; ++i) {
                        const float v = has_pec && pec_owned(c, i, j, k) ? 0.0f : row[i];
                        const uint16_t h = encode(s->storage, v * upf[c], &sat);
                        q[i] = h;
                        const float d = std::fabs(decode(s->storage, h) * dnf[c]);
                        if (d > mx[c]) mx[c] = d;        // NaN never compares greater
                    }
                    box_add_row(s, q, i0, i1, j, k);
                }
            }
        }
        if ((e = hipMemcpyAsync(s->fbuf[0] + (size_t)k * s->L.kstride * es, buf, (size_t)s->L.kstride * es,
                                hipMemcpyHostToDevice, s->st)) ||
            (e = hipEventRecord(s->stage_ev[b], s->st)))
            return hip_fail(e, "upload fields");
    }
    if (s->storage != FDTD_FP32) {
        for (int c = 0; c < 6; ++c) {
            ctrl.scale[0][c] = sc[c];
            std::memcpy(&ctrl.maxbits[0][c], &mx[c], 4);
        }
        ctrl.flag = sat ? 1u : 0u;
    }
    if ((e = hipMemcpyAsync(s->ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice, s->st)) ||
        (e = hipStreamSynchronize(s->st)))
        return hip_fail(e, "upload fields");
    release_large_staging(s);
    live_build(s, [&](int c, int i, int j, int k) {
        if (c < 3) return false;        // pinned E edges were stored as +0
        uint32_t b;
        std::memcpy(&b, host + (size_t)c * nbox + (size_t)k * nplane + (size_t)j * (nx + 1) + i, 4);
        return b != 0;                  // -0 and values a 16-bit format rounds to +0 count as live
    });
    return FDTD_OK;
}

int fdtd_set_source(fdtd_solver *s, int comp, int i, int j, int k, const float *waveform, int n_samples, int *id)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (comp < 0 || comp > 2) return fail(FDTD_EINVAL, "sources act on E components only");
    if (!e_interior(s->L.nx, s->L.ny, s->L.nz, comp, i, j, k))
        return fail(FDTD_EINVAL, "source must sit on an interior (non-PEC) edge");
    if (n_samples < 0 || (n_samples > 0 && !waveform)) return fail(FDTD_EINVAL, "bad waveform");
    if (s->src_pos.size() >= 256) return fail(FDTD_EINVAL, "at most 256 sources per solver");
    const int off = (int)s->samples.size();
    float amax = s->a_max;
    for (int n = 0; n < n_samples; ++n) {
        if (!std::isfinite(waveform[n])) return fail(FDTD_EINVAL, "non-finite waveform sample");
        amax = std::max(amax, std::fabs(waveform[n]));
    }
    s->samples.insert(s->samples.end(), waveform, waveform + n_samples);
    s->src_pos.push_back(make_int4(comp, i, j, k));
    s->src_wave.push_back(make_int2(off, n_samples));
    live_source(s, i, j, k);
    s->a_max = amax;
    int rc = upload_sources(s);
    if (rc) return rc;
    if (id) *id = (int)s->src_pos.size() - 1;
    return FDTD_OK;
}

int fdtd_set_probe(fdtd_solver *s, int comp, int i, int j, int k, int *id)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (s->steps > 0) return fail(FDTD_ESTATE, "probes must be added before the first step");
    if (comp < 0 || comp > 5 || !in_range(s->L.nx, s->L.ny, s->L.nz, comp, i, j, k))
        return fail(FDTD_EINVAL, "probe outside the component's range");
    if (s->probe_pos.size() >= 256) return fail(FDTD_EINVAL, "at most 256 probes per solver");
    s->probe_pos.push_back(make_int4(comp, i, j, k));
    free_dev(s->probe_pos_d);
    free_dev(s->probe_out_d);
    s->probe_pos_d = nullptr;
    s->probe_out_d = nullptr;
    s->probe_cap = 0;
    hipError_t e;
    if ((e = hipMalloc(&s->probe_pos_d, s->probe_pos.size() * sizeof(int4))) ||
        (e = hipMemcpyAsync(s->probe_pos_d, s->probe_pos.data(), s->probe_pos.size() * sizeof(int4),
                            hipMemcpyHostToDevice, s->st)) ||
        (e = hipStreamSynchronize(s->st)))
        return hip_fail(e, "upload probes");
    if (id) *id = (int)s->probe_pos.size() - 1;
    return FDTD_OK;
}

int fdtd_step(fdtd_solver *s, int n_steps)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (n_steps < 0) return fail(FDTD_EINVAL, "negative step count");
    if (n_steps == 0) return FDTD_OK;
    const long long every = s->energy_every;
    if (every > 0 && (s->gc_d || s->pml.n > 0))
        return fail(FDTD_EINVAL, "the energy trace needs uniform spacing and no CPML layers");
    int rc = ensure_probe_rows(s, s->steps + n_steps);
    if (rc) return rc;
    if ((rc = ensure_energy_rows(s, s->steps + n_steps))) return rc;
    const yee::SourceTable src = src_table(s);
    const yee::ProbeTable probe = probe_table(s);
    hipError_t e;
    // AUTO is the fused kernel, or the plain one for grids whose planes (or
    // CPML arrays) are too large for the fused kernel's 32-bit addressing
    // (FP32 only: create rejects 16-bit storage for such grids).
    const bool cpml = s->pml.n > 0;
    if (runs_plain(s)) {
        yee::PlainArgs a;
        a.L = s->L;
        a.f = (float *)s->fbuf[s->cur];
        a.mat = s->mat;
        a.coef = s->coef_d;
        a.n_mat = s->n_mat;
        a.chx = s->ch[0]; a.chy = s->ch[1]; a.chz = s->ch[2];
        a.gc = s->gc_d;
        a.pml = cpml_args(s);
        box_take_sources(s);
        for (int q = 0; q < n_steps; ++q) {
            const long long n = s->steps + q;
            if (every > 0 && n % every == 0) {       // the energy of state n, by the diagnostics pass
                if ((rc = ensure_diag_buffers(s))) return rc;
                if ((e = launch_diagnostics(s, s->diag_part_d, s->diag_out_d)) ||
                    (e = hipMemcpyAsync(s->energy_d + n / every, s->diag_out_d, sizeof(double),
                                        hipMemcpyDeviceToDevice, s->st)))
                    return hip_fail(e, "energy trace");
            }
            if ((e = yee::launch_plain_step(a, src, probe, n, s->st))) return hip_fail(e, "plain step");
        }
        box_grow(s, n_steps);
        s->steps += n_steps;
        return record_done(s);
    }
    if (every > 0) {           // the fused energy kernels: blocks of at most MAX_T_ENERGY steps
        if (s->T > yee::MAX_T_ENERGY)
            return fail(FDTD_EINVAL, "the energy trace runs fused blocks of at most " +
                                         std::to_string(yee::MAX_T_ENERGY) + " steps");
        if (s->storage != FDTD_FP32 && every < s->T)
            return fail(FDTD_EINVAL, "with 16-bit storage the energy trace needs every >= T");
    }
    int left = n_steps;
    while (left > 0) {
        int len = next_block(s, left);
        // the recorded state of this block, if any: at most one per launch
        // (FP32 blocks end before a second; 16-bit blocks hold at most one
        // since every >= T)
        int level = 0;
        long long rec = 0;
        if (every > 0) {
            const long long n0 = (s->steps + every - 1) / every * every;
            if (n0 < s->steps + len) {
                if (n0 + every < s->steps + len) len = (int)(n0 + every - s->steps);
                level = (int)(n0 - s->steps) + 1;
                rec = n0 / every;
            }
        }
        yee::FusedArgs a;
        fill_fused(s, &a);
        const int shape = s->tiling > 0 ? s->tiling - 1
                                        : yee::auto_shape(s->storage, len, s->gc_d != nullptr,
                                                          (long long)s->L.nx * s->L.ny * s->L.nz);
        if (!yee::fused_fits(s->L, s->storage, len))      // never launch a chunk beyond its addressing
            return fail(FDTD_EINVAL, "grid planes too large for the fused kernel at this T");
        box_take_sources(s);
        box_args(s, &a);
        // Conductor interiors keep their fields at +0 but, in a layer, not
        // their psi (it follows the curl next door): no dead-tile list there.
        a.live = s->zero_skip && !cpml ? s->live : nullptr;
        yee::CpmlFused cp{};
        if (cpml) {
            cp.pml = cpml_args(s);
            cp.psi_out = psi_buf(s, s->cur ^ 1);
        }
        if (s->poison) {     // every value the launch owns must be rewritten: nothing may rely on the old buffer
            a.box_lo = make_int4(-(1 << 28), -(1 << 28), -(1 << 28), 0);
            a.box_hi = make_int4(1 << 28, 1 << 28, 1 << 28, 0);
            a.live = nullptr;
            if ((e = hipMemsetAsync(s->fbuf[s->cur ^ 1], 0xff, s->d.fbytes, s->st)) ||
                (cpml && (e = hipMemsetAsync(cp.psi_out, 0xff, s->psi_bytes, s->st))))
                return hip_fail(e, "poison");
        }
        if (cpml) {
            e = yee::launch_fused_cpml(len, a, cp, s->zchunk, s->st);
        } else if (level > 0) {
            yee::EnergyFused en;
            en.level = level;
            en.partial = s->epart_d;
            en.half_eps = s->half_eps_d;
            en.out = s->energy_d + rec;
            e = yee::launch_fused_energy(s->storage, len, a, en, shape, s->zchunk, s->st);
        } else {
            e = yee::launch_fused(s->storage, len, a, shape, s->zchunk, s->st);
        }
        if (e) return hip_fail(e, "fused step");
        box_grow(s, len);
        advance(s, len);
        left -= len;
    }
    return record_done(s);
}

int fdtd_step_batch(fdtd_solver *const *solvers, int count, const int *n_steps)
{
    if (!solvers || !n_steps || count < 0) return fail(FDTD_EINVAL, "NULL argument");
    if (count == 0) return FDTD_OK;
    const hipStream_t st = solvers[0] ? solvers[0]->st : nullptr;
    std::vector<int> left(count);
    for (int i = 0; i < count; ++i) {
        fdtd_solver *s = solvers[i];
        if (!s) return fail(FDTD_EINVAL, "solver is NULL");
        if (s->st != st) return fail(FDTD_EINVAL, "batched solvers must share one stream");
        if (s->kernel == FDTD_KERNEL_PLAIN || !yee::fused_fits(s->L, s->storage, s->T))
            return fail(FDTD_EINVAL, "batched steps use the fused kernel");
        if (s->energy_every > 0) return fail(FDTD_EINVAL, "solvers with an energy trace are stepped alone (fdtd_step)");
        if (s->gc_d) return fail(FDTD_EINVAL, "graded-spacing solvers are stepped alone (fdtd_step)");
        if (s->T > yee::MAX_T_BATCH)
            return fail(FDTD_EINVAL, "batched steps run blocks of at most " + std::to_string(yee::MAX_T_BATCH) + " steps");
        if (n_steps[i] < 0) return fail(FDTD_EINVAL, "negative step count");
        for (int j = 0; j < i; ++j)
            if (solvers[j] == s) return fail(FDTD_EINVAL, "a solver appears twice in the batch");
        left[i] = n_steps[i];
        int rc = ensure_probe_rows(s, s->steps + n_steps[i]);
        if (rc) return rc;
    }
    // Each round advances every unfinished solve by its next block; solves
    // with equal (storage, block length, tile shape) share launches.
    std::vector<int> len(count), key(count), done(count);
    for (;;) {
        bool any = false;
        for (int i = 0; i < count; ++i) {
            done[i] = 0;
            if (left[i] > 0) {
                fdtd_solver *s = solvers[i];
                len[i] = next_block(s, left[i]);
                const int shape = s->tiling > 0 ? s->tiling - 1 : yee::auto_shape(s->storage, len[i]);
                key[i] = (s->storage * 8 + len[i]) * 8 + shape;
                any = true;
            } else {
                done[i] = 1;
            }
        }
        if (!any) break;
        for (int i = 0; i < count; ++i) {
            if (done[i]) continue;
            yee::FusedArgs group[yee::MAX_BATCH];
            int members[yee::MAX_BATCH];
            int n = 0;
            for (int j = i; j < count && n < yee::MAX_BATCH; ++j)
                if (!done[j] && key[j] == key[i]) {
                    fill_fused(solvers[j], &group[n]);
                    box_take_sources(solvers[j]);
                    box_args(solvers[j], &group[n]);
                    group[n].live = solvers[j]->zero_skip ? solvers[j]->live : nullptr;
                    members[n++] = j;
                    done[j] = 1;
                }
            const fdtd_solver *s0 = solvers[i];
            const int shape = key[i] % 8;
            hipError_t e = yee::launch_fused_batch(s0->storage, len[i], group, n, shape, s0->zchunk, st);
            if (e) return hip_fail(e, "batched step");
            for (int q = 0; q < n; ++q) {
                box_grow(solvers[members[q]], len[i]);
                advance(solvers[members[q]], len[i]);
                left[members[q]] -= len[i];
            }
        }
    }
    for (int i = 0; i < count; ++i)
        if (n_steps[i] > 0)
            if (int rc = record_done(solvers[i])) return rc;
    return FDTD_OK;
}

int fdtd_set_stream(fdtd_solver *s, void *hip_stream)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    hipError_t e = hipStreamSynchronize(s->st);
    if (e) return hip_fail(e, "hipStreamSynchronize");
    s->st = (hipStream_t)hip_stream;
    s->done_pending = false;
    return FDTD_OK;
}

int fdtd_read_fields(fdtd_solver *s, int comp, float *host_dst)
{
    if (!s || !host_dst) return fail(FDTD_EINVAL, "NULL argument");
    if (comp < 0 || comp > 5) return fail(FDTD_EINVAL, "bad component");
    const int nx = s->L.nx, ny = s->L.ny, nz = s->L.nz;
    const int es = elem_size(s->storage);
    hipError_t e;
    if (int rc = ensure_staging(s)) return rc;
    float dnf = 1.0f;
    if (s->storage != FDTD_FP32) {
        yee::Ctrl c;
        if (int rc = read_ctrl(s, &c)) return rc;
        dnf = std::ldexp(1.0f, -c.scale[s->block % 2][comp]);
    }
    // Plane k of the component is one contiguous pitched block on the device:
    // copy it to a pinned buffer while the host unpacks the previous one.
    const size_t nplane = (size_t)(nx + 1) * (ny + 1);
    const size_t pbytes = (size_t)s->L.plane * es;
    auto fetch = [&](int k) {
        const int b = k & 1;
        hipError_t r = hipMemcpyAsync(s->stage[b], s->fbuf[s->cur] + ((size_t)comp * s->L.cstride +
                                      (size_t)k * s->L.kstride) * es, pbytes, hipMemcpyDeviceToHost, s->st);
        return r ? r : hipEventRecord(s->stage_ev[b], s->st);
    };
    e = fetch(0);
    for (int k = 0; k <= nz && !e; ++k) {
        if (k < nz && (e = fetch(k + 1))) break;
        if ((e = hipEventSynchronize(s->stage_ev[k & 1]))) break;
        const char *buf = s->stage[k & 1];
        float *out = host_dst + (size_t)k * nplane;
        for (int j = 0; j <= ny; ++j) {
            const size_t at = (size_t)j * s->d.pitch;
            if (s->storage == FDTD_FP32) {
                std::memcpy(out + (size_t)j * (nx + 1), (const float *)buf + at, (size_t)(nx + 1) * sizeof(float));
            } else {
                const uint16_t *q = (const uint16_t *)buf + at;
                for (int i = 0; i <= nx; ++i) out[(size_t)j * (nx + 1) + i] = decode(s->storage, q[i]) * dnf;
            }
        }
    }
    if (!e) e = hipStreamSynchronize(s->st);
    if (e) return hip_fail(e, "read fields");
    release_large_staging(s);
    return FDTD_OK;
}

int fdtd_read_probes(fdtd_solver *s, double *host_dst, long long first_step, int n_steps)
{
    if (!s || (!host_dst && n_steps > 0)) return fail(FDTD_EINVAL, "NULL argument");
    if (first_step < 0 || n_steps < 0 || first_step + n_steps > s->steps)
        return fail(FDTD_EINVAL, "requested steps have not been run");
    const size_t np = s->probe_pos.size();
    if (np == 0 || n_steps == 0) return FDTD_OK;
    // Wait for this solver's own enqueued work only (later work that other
    // solvers queued on the same stream keeps running), then copy on a
    // stream of the library's own.
    hipError_t e = hipSuccess;
    if (!s->priv) e = hipStreamCreateWithFlags(&s->priv, hipStreamNonBlocking);
    if (!e && s->done_pending) e = hipEventSynchronize(s->done_ev);
    if (!e) e = hipMemcpyAsync(host_dst, s->probe_out_d + (size_t)first_step * np,
                               (size_t)n_steps * np * sizeof(double), hipMemcpyDeviceToHost, s->priv);
    if (!e) e = hipStreamSynchronize(s->priv);
    return e ? hip_fail(e, "read probes") : FDTD_OK;
}

int fdtd_reserve_steps(fdtd_solver *s, long long total_steps)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (total_steps < 0) return fail(FDTD_EINVAL, "negative step count");
    if (int rc = ensure_probe_rows(s, total_steps)) return rc;
    return ensure_energy_rows(s, total_steps);
}

int fdtd_set_energy_trace(fdtd_solver *s, int every)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    if (every < 0) return fail(FDTD_EINVAL, "negative energy trace interval");
    if (s->steps > 0) return fail(FDTD_ESTATE, "the energy trace must be set before the first step");
    if (every > 0 && (s->gc_d || s->pml.n > 0))
        return fail(FDTD_EINVAL, "the energy trace needs uniform spacing and no CPML layers");
    free_dev(s->energy_d);
    s->energy_d = nullptr;
    s->energy_cap = 0;
    s->energy_every = 0;
    if (every == 0) return FDTD_OK;
    hipError_t e;
    if (!s->half_eps_d) {
        double half[256];
        for (int m = 0; m < 256; ++m) half[m] = m < s->n_mat ? 0.5 * s->eps_h[m] : 0.0;
        double *p = nullptr, *q = nullptr;
        const size_t nt = (size_t)yee::fused_tiles_bound(s->L);
        if ((e = hipMalloc(&p, sizeof(half))) || (e = hipMalloc(&q, nt * sizeof(double))) ||
            (e = hipMemcpyAsync(p, half, sizeof(half), hipMemcpyHostToDevice, s->st)) ||
            (e = hipStreamSynchronize(s->st))) {
            free_dev(p);
            free_dev(q);
            return hip_fail(e, "energy trace buffers");
        }
        s->half_eps_d = p;
        s->epart_d = q;
    }
    s->energy_every = every;
    return FDTD_OK;
}

int fdtd_read_energy(fdtd_solver *s, double *host_dst, long long first_record, int n_records)
{
    if (!s || (!host_dst && n_records > 0)) return fail(FDTD_EINVAL, "NULL argument");
    if (s->energy_every <= 0) return fail(FDTD_EINVAL, "no energy trace (fdtd_set_energy_trace)");
    const long long have = s->steps > 0 ? (s->steps - 1) / s->energy_every + 1 : 0;
    if (first_record < 0 || n_records < 0 || first_record + n_records > have)
        return fail(FDTD_EINVAL, "requested records have not been written");
    if (n_records == 0) return FDTD_OK;
    hipError_t e = hipSuccess;
    if (!s->priv) e = hipStreamCreateWithFlags(&s->priv, hipStreamNonBlocking);
    if (!e && s->done_pending) e = hipEventSynchronize(s->done_ev);
    if (!e) e = hipMemcpyAsync(host_dst, s->energy_d + first_record, (size_t)n_records * sizeof(double),
                               hipMemcpyDeviceToHost, s->priv);
    if (!e) e = hipStreamSynchronize(s->priv);
    return e ? hip_fail(e, "read energy") : FDTD_OK;
}

}  // extern "C"

namespace {

// Diagnostics of the current state into the 11 doubles at dout (device),
// with the block partials in `partial`.
hipError_t launch_diagnostics(fdtd_solver *s, double *partial, double *dout)
{
    yee::DiagArgs a;
    a.L = s->L;
    a.f = s->fbuf[s->cur];
    a.mat = s->mat;
    a.coef = s->coef_d;
    a.eps = s->eps_d;
    a.n_mat = s->n_mat;
    a.chx = s->ch[0]; a.chy = s->ch[1]; a.chz = s->ch[2];
    a.idx = 1.0 / s->dx; a.idy = 1.0 / s->dy; a.idz = 1.0 / s->dz;
    a.gc = s->gc_d;
    a.gsz = s->gsz_d;
    a.partial = partial;
    a.sb = storage_block(s);
    return yee::launch_diag(s->storage, a, dout, s->st);
}

int ensure_diag_buffers(fdtd_solver *s)
{
    if (s->diag_part_d) return FDTD_OK;
    const size_t nb = (size_t)yee::diag_blocks(s->L);
    hipError_t e;
    if ((e = hipMalloc(&s->diag_part_d, nb * yee::DIAG_W * sizeof(double))) ||
        (e = hipMalloc(&s->diag_out_d, yee::DIAG_W * sizeof(double))))
        return hip_fail(e, "hipMalloc(diagnostics)");
    return FDTD_OK;
}

// Diagnostics of the current state with the block partials in `partial`
// and the 11 reduced values in `dout` (device), copied to *out.
int run_diagnostics(fdtd_solver *s, double *partial, double *dout, fdtd_diag *out)
{
    hipError_t e;
    if ((e = launch_diagnostics(s, partial, dout))) return hip_fail(e, "diagnostics");
    double v[yee::DIAG_W];
    e = hipMemcpyAsync(v, dout, sizeof(v), hipMemcpyDeviceToHost, s->st);
    if (!e) e = hipStreamSynchronize(s->st);
    if (e) return hip_fail(e, "diagnostics");
    out->energy = v[0];
    out->div_e_sumsq = v[1];
    out->div_h_sumsq = v[2];
    out->div_e_max = v[3];
    out->div_h_max = v[4];
    for (int c = 0; c < 6; ++c) out->max_abs[c] = v[5 + c];
    return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_diagnostics(fdtd_solver *s, fdtd_diag *out)
{
    if (!s || !out) return fail(FDTD_EINVAL, "NULL argument");
    if (s->pml.n > 0) return fail(FDTD_EINVAL, "diagnostics are not defined with CPML layers");
    if (int rc = ensure_diag_buffers(s)) return rc;
    return run_diagnostics(s, s->diag_part_d, s->diag_out_d, out);
}

int fdtd_diagnostics_noalloc(fdtd_solver *s, fdtd_diag *out)
{
    if (!s || !out) return fail(FDTD_EINVAL, "NULL argument");
    if (s->pml.n > 0) return fail(FDTD_EINVAL, "diagnostics are not defined with CPML layers");
    const long long nb = yee::diag_blocks(s->L);
    if (nb > yee::diag_static_max_blocks())
        return fail(FDTD_EINVAL, "grid needs " + std::to_string(nb) + " diagnostics partials; the static scratch holds " +
                                     std::to_string(yee::diag_static_max_blocks()) + " (use fdtd_diagnostics)");
    double *dout = nullptr, *partial = nullptr;
    if (hipError_t e = yee::diag_static_scratch(&dout, &partial)) return hip_fail(e, "diagnostics scratch");
    return run_diagnostics(s, partial, dout, out);
}

// Saved state: a header, the current field buffer as stored on the device,
// the reduced-storage control block and the CPML psi arrays.
namespace {
struct StateHeader {
    char magic[8];                      // "FDTDSTA1"
    int32_t nx, ny, nz, storage;
    int32_t pml_n, pad;
    int64_t steps, block;
    int32_t box_lo[3], box_hi[3];
    uint64_t field_bytes, ctrl_bytes, psi_bytes;
};
constexpr char STATE_MAGIC[8] = {'F', 'D', 'T', 'D', 'S', 'T', 'A', '1'};
}  // namespace

size_t fdtd_state_bytes(const fdtd_solver *s)
{
    if (!s) return 0;
    return sizeof(StateHeader) + s->d.fbytes + sizeof(yee::Ctrl) + s->psi_bytes;
}

int fdtd_save_state(fdtd_solver *s, void *host_dst, size_t bytes)
{
    if (!s || !host_dst) return fail(FDTD_EINVAL, "NULL argument");
    if (bytes < fdtd_state_bytes(s)) return fail(FDTD_EINVAL, "buffer smaller than fdtd_state_bytes");
    StateHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, STATE_MAGIC, 8);
    h.nx = s->L.nx; h.ny = s->L.ny; h.nz = s->L.nz; h.storage = s->storage;
    h.pml_n = s->pml.n;
    h.steps = s->steps; h.block = s->block;
    for (int a = 0; a < 3; ++a) { h.box_lo[a] = s->box_lo[a]; h.box_hi[a] = s->box_hi[a]; }
    h.field_bytes = s->d.fbytes; h.ctrl_bytes = sizeof(yee::Ctrl); h.psi_bytes = s->psi_bytes;
    char *dst = (char *)host_dst;
    std::memcpy(dst, &h, sizeof(h));
    hipError_t e;
    if ((e = hipMemcpyAsync(dst + sizeof(h), s->fbuf[s->cur], s->d.fbytes, hipMemcpyDeviceToHost, s->st)) ||
        (e = hipMemcpyAsync(dst + sizeof(h) + s->d.fbytes, s->ctrl, sizeof(yee::Ctrl), hipMemcpyDeviceToHost, s->st)) ||
        (s->psi_bytes && (e = hipMemcpyAsync(dst + sizeof(h) + s->d.fbytes + sizeof(yee::Ctrl), psi_buf(s, s->cur),
                                             s->psi_bytes, hipMemcpyDeviceToHost, s->st))) ||
        (e = hipStreamSynchronize(s->st)))
        return hip_fail(e, "save state");
    return FDTD_OK;
}

int fdtd_load_state(fdtd_solver *s, const void *host_src, size_t bytes)
{
    if (!s || !host_src) return fail(FDTD_EINVAL, "NULL argument");
    StateHeader h;
    if (bytes < sizeof(h)) return fail(FDTD_EINVAL, "state too short");
    std::memcpy(&h, host_src, sizeof(h));
    if (std::memcmp(h.magic, STATE_MAGIC, 8) != 0) return fail(FDTD_EINVAL, "not a saved solver state");
    if (h.nx != s->L.nx || h.ny != s->L.ny || h.nz != s->L.nz || h.storage != s->storage || h.pml_n != s->pml.n ||
        h.field_bytes != s->d.fbytes || h.ctrl_bytes != sizeof(yee::Ctrl) || h.psi_bytes != s->psi_bytes)
        return fail(FDTD_EINVAL, "saved state does not match this solver (grid, storage or CPML layers)");
    if (bytes < fdtd_state_bytes(s)) return fail(FDTD_EINVAL, "state truncated");
    if (h.steps < 0 || h.block < 0) return fail(FDTD_EINVAL, "corrupt state");
    if (int rc = ensure_probe_rows(s, h.steps)) return rc;
    const char *src = (const char *)host_src;
    hipError_t e;
    if ((e = hipStreamSynchronize(s->st)) ||
        (e = hipMemcpyAsync(s->fbuf[0], src + sizeof(h), s->d.fbytes, hipMemcpyHostToDevice, s->st)) ||
        (e = hipMemsetAsync(s->fbuf[1], 0, s->d.fbytes, s->st)) ||
        (e = hipMemcpyAsync(s->ctrl, src + sizeof(h) + s->d.fbytes, sizeof(yee::Ctrl), hipMemcpyHostToDevice, s->st)) ||
        (s->psi_bytes && (e = hipMemcpyAsync(psi_buf(s, 0), src + sizeof(h) + s->d.fbytes + sizeof(yee::Ctrl),
                                             s->psi_bytes, hipMemcpyHostToDevice, s->st))) ||
        (s->psi_bytes && (e = hipMemsetAsync(psi_buf(s, 1), 0, s->psi_bytes, s->st))))
        return hip_fail(e, "load state");
    // Probe rows from the restored step on start again at 0: a tile that the
    // zero-tile skip or the dead-tile list leaves out never writes its probes'
    // rows, which must then read 0, not what a later history wrote there.
    if (s->probe_out_d && s->probe_cap > h.steps) {
        const size_t np = s->probe_pos.size();
        if ((e = hipMemsetAsync(s->probe_out_d + (size_t)h.steps * np, 0,
                                (size_t)(s->probe_cap - h.steps) * np * sizeof(double), s->st)))
            return hip_fail(e, "load state");
    }
    // energy records of states from the restored step on: unwritten again
    if (s->energy_every > 0 && s->energy_d) {
        const long long k0 = (h.steps + s->energy_every - 1) / s->energy_every;
        if (k0 < s->energy_cap &&
            (e = hipMemsetAsync(s->energy_d + k0, 0xff, (size_t)(s->energy_cap - k0) * sizeof(double), s->st)))
            return hip_fail(e, "load state");
    }
    if ((e = hipStreamSynchronize(s->st))) return hip_fail(e, "load state");
    s->cur = 0;
    s->steps = h.steps;
    s->block = h.block;
    for (int a = 0; a < 3; ++a) { s->box_lo[a] = h.box_lo[a]; s->box_hi[a] = h.box_hi[a]; }
    const char *fb = src + sizeof(h);
    const int es = elem_size(s->storage);
    live_build(s, [&](int c, int i, int j, int k) {
        const size_t at = ((size_t)c * s->L.cstride + (size_t)k * s->L.kstride + (size_t)j * s->L.pitch + i) * es;
        uint32_t b = 0;
        std::memcpy(&b, fb + at, es);
        return b != 0;
    });
    return FDTD_OK;
}

int fdtd_steps_done(const fdtd_solver *s, long long *n)
{
    if (!s || !n) return fail(FDTD_EINVAL, "NULL argument");
    *n = s->steps;
    return FDTD_OK;
}

int fdtd_time_block(const fdtd_solver *s, int *T)
{
    if (!s || !T) return fail(FDTD_EINVAL, "NULL argument");
    *T = runs_plain(s) ? 1 : s->pml.n > 0 ? std::min(s->T, yee::MAX_T_CPML) : s->T;
    return FDTD_OK;
}

int fdtd_tune_time_block(fdtd_solver *s, int n_steps, int *chosen, double *ns_per_step)
{
    if (!s || !chosen) return fail(FDTD_EINVAL, "NULL argument");
    if (n_steps < 1) return fail(FDTD_EINVAL, "n_steps must be positive");
    if (s->storage != FDTD_FP32 || s->gc_d || s->pml.n > 0 || s->energy_every > 0 || runs_plain(s))
        return fail(FDTD_EINVAL, "tuning T needs FP32 storage, uniform spacing, no CPML layers, no energy trace "
                                 "and the fused kernel");
    constexpr int NC = 3, cand[NC] = {3, 4, 5};
    // the steps every candidate runs: an untimed block (first-launch costs),
    // then the largest multiple of T up to n_steps
    long long total = 0;
    for (int T : cand) total += T + std::max(T, n_steps / T * T);
    int rc = ensure_probe_rows(s, s->steps + total);
    if (rc) return rc;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int q = 0; q < 2 && !e; ++q) e = hipEventCreate(&ev[q]);
    const bool skip = s->zero_skip, automatic = s->T_auto;
    const int T0 = s->T;
    s->zero_skip = false;               // full launches, as once a field fills the grid
    int best = 0;
    double best_ns = 0.0;
    for (int c = 0; c < NC && !e && !rc; ++c) {
        const int T = cand[c];
        if (ns_per_step) ns_per_step[c] = 0.0;
        if (!yee::fused_fits(s->L, s->storage, T)) continue;
        s->T = T;
        const int m = std::max(T, n_steps / T * T);
        float ms = 0.0f;
        if ((rc = fdtd_step(s, T))) break;
        if ((e = hipEventRecord(ev[0], s->st))) break;
        if ((rc = fdtd_step(s, m))) break;
        if ((e = hipEventRecord(ev[1], s->st)) || (e = hipEventSynchronize(ev[1])) ||
            (e = hipEventElapsedTime(&ms, ev[0], ev[1])))
            break;
        const double ns = 1e6 * ms / m;
        if (ns_per_step) ns_per_step[c] = ns;
        if (best == 0 || ns < best_ns) {
            best = T;
            best_ns = ns;
        }
    }
    s->zero_skip = skip;
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc || e || best == 0) {
        s->T = T0;
        s->T_auto = automatic;
        if (rc) return rc;
        return e ? hip_fail(e, "tune time block") : fail(FDTD_EINVAL, "no candidate T fits the grid");
    }
    s->T = best;
    s->T_auto = false;
    *chosen = best;
    return FDTD_OK;
}

int fdtd_storage_state(fdtd_solver *s, int scales[6], int *saturated)
{
    if (!s || !scales || !saturated) return fail(FDTD_EINVAL, "NULL argument");
    if (s->storage == FDTD_FP32) {
        hipError_t e = hipStreamSynchronize(s->st);
        if (e) return hip_fail(e, "hipStreamSynchronize");
        for (int c = 0; c < 6; ++c) scales[c] = 0;
        *saturated = 0;
        return FDTD_OK;
    }
    yee::Ctrl c;
    int rc = read_ctrl(s, &c);
    if (rc) return rc;
    for (int q = 0; q < 6; ++q) scales[q] = c.scale[s->block % 2][q];
    *saturated = c.flag ? 1 : 0;
    return FDTD_OK;
}

int fdtd_synchronize(fdtd_solver *s)
{
    if (!s) return fail(FDTD_EINVAL, "solver is NULL");
    hipError_t e = hipStreamSynchronize(s->st);
    if (e) return hip_fail(e, "hipStreamSynchronize");
    if (s->storage != FDTD_FP32) {
        yee::Ctrl c;
        int rc = read_ctrl(s, &c);
        if (rc) return rc;
        if (c.flag) return fail(FDTD_ERANGE, "reduced storage stored a non-finite value, or overflowed after its block was re-run with new scales");
    }
    return FDTD_OK;
}

void fdtd_destroy(fdtd_solver *s)
{
    if (!s) return;
    // its own work only: later work of other solvers on the stream may run on
    if (s->done_pending) (void)hipEventSynchronize(s->done_ev);
    else (void)hipStreamSynchronize(s->st);
    live_drop(s);
    if (s->own_ws) free_dev(s->ws);
    free_dev(s->coef_d);
    free_dev(s->eps_d);
    free_dev(s->gc_d);
    free_dev(s->cp_d);
    free_dev(s->gsz_d);
    free_dev(s->psi_d);
    free_dev(s->src_pos_d);
    free_dev(s->src_wave_d);
    free_dev(s->samples_d);
    free_dev(s->probe_pos_d);
    free_dev(s->probe_out_d);
    free_dev(s->diag_part_d);
    free_dev(s->diag_out_d);
    free_dev(s->energy_d);
    free_dev(s->epart_d);
    free_dev(s->half_eps_d);
    for (int b = 0; b < 2; ++b) {
        if (s->stage[b]) (void)hipHostFree(s->stage[b]);
        if (s->stage_ev[b]) (void)hipEventDestroy(s->stage_ev[b]);
    }
    if (s->done_ev) (void)hipEventDestroy(s->done_ev);
    if (s->priv) (void)hipStreamDestroy(s->priv);
    delete s;
}

}  // extern "C"
