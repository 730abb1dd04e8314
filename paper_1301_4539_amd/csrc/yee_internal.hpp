// Internal declarations shared by the host runtime and the HIP kernels of
// the Yee FDTD library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace yee {

// Device field layout, plane-interleaved: the six components of one z plane
// are stored one after another, so a z march reads one contiguous run per
// plane.  Component c of point (i,j,k) sits at
//     c*cstride + k*kstride + j*pitch + i
// with pitch >= nx+1, plane = pitch*(ny+1), cstride = plane and
// kstride = 6*plane.  The material index is a separate byte array addressed
// k*plane + j*pitch + i (bytes outside the cell range are 0).
struct Layout {
    int nx, ny, nz;
    int pitch;
    long long plane;
    long long cstride;
    long long kstride;
};

// Reduced-storage control block (device).  maxbits holds, per component,
// the largest |stored value| as float bits (non-negative floats order like
// their bit patterns); three slots rotate so that the block that reads one
// slot fills the next and clears the one after, and so do the arrays below.
// scale[par] is the scale of the currently stored fields.  Overflow retry:
// a block's first pass records in ovf (bit c) the components whose encoding
// would overflow and in premax their largest |value| before encoding; its
// second pass, which runs only when ovf is set, encodes those components with
// a scale from premax and records its stored maxima in rmaxbits, where the
// next block reads them.  flag is sticky: a NaN, or an overflow left after
// the retry.
struct Ctrl {
    uint32_t maxbits[3][6];
    uint32_t rmaxbits[3][6];
    uint32_t premax[3][6];
    uint32_t ovf[3];
    int32_t scale[2][6];
    uint32_t flag;
    uint32_t pad[2];
};

struct SourceTable {
    int n;
    const int4 *pos;      // (comp, i, j, k)
    const int2 *wave;     // (offset into samples, n_samples)
    const float *samples;
};

struct ProbeTable {
    int n;
    const int4 *pos;      // (comp, i, j, k)
    double *out;          // rows of n doubles, row = step - base
    long long base;       // step of row 0
};

struct StorageBlock {
    Ctrl *ctrl;
    int slot_in, slot_out, slot_clear, par;
    float a_max;          // largest |source sample|
    int retry;            // 1: the block's second pass (runs only if its first pass overflowed)
};

// Live nodes of a solve: a node is dead when its six values are +0 and stay
// so for good -- its E edges are walls or belong to perfect-conductor cells
// (no source on them), and each of its H values sees only such edges.  The
// runtime keeps the map; the launcher asks it, per tile geometry, for the
// tiles whose owned region holds a live node (conductor interiors drop out).
struct LiveNodes;
// Device list, ascending, of tile indices (tz nty + ty) ntx + tx of the full
// ntx x nty x ntz tiling (owned regions of ox x oy points and zc planes) that
// own a live node; *count is its length.  nullptr when every tile does (or
// the list could not be made): then every tile runs.  The list stays valid
// until the map changes.
const int *live_tile_list(LiveNodes *d, int ox, int oy, int zc, int ntx, int nty, int ntz, int *count,
                          hipStream_t st);
// The z chunk (<= zmax planes) minimising rounds * (zc + 1.5 T) when only the
// tiles owning a live node are launched, `slots` workgroups at a time; 0 when
// none qualifies.  Cached per geometry until the map changes.
int live_best_zc(LiveNodes *d, int ox, int oy, int ntx, int nty, int T, int slots, int zmax);

// CPML absorbing layers of n cells on every face.  cp: per axis (x, y, z)
// and node index q, 6 floats {b_h, a_h, c dt / d[q], b_e, a_e, c dt / d'[q]}
// (H values at cell q, E values at node q).  psi: the auxiliary state of each
// (component, derivative axis), kept only in the layers: an index q along the
// derivative axis maps to the slab slot l = q (q < n) or q - (n_axis - 2 n)
// (upper layer), l < 2 n.  The four values that share a derivative axis sit
// together, one 16-byte group per slab position, in three blocks starting at
// base[axis] (floats):
//   x-type (Hy, Hz, Ey, Ez), group ((k (ny+1) + j) 2n + l)
//   y-type (Hx, Hz, Ex, Ez), group ((k 2n + l)(nx+1) + i)
//   z-type (Hx, Hy, Ex, Ey), group ((l (ny+1) + j)(nx+1) + i)
// PsiArray numbers them axis * 4 + place in the group.
enum PsiArray { PS_HYX = 0, PS_HZX, PS_EYX, PS_EZX, PS_HXY, PS_HZY, PS_EXY, PS_EZY, PS_HXZ, PS_HYZ, PS_EXZ, PS_EYZ };
struct Cpml {
    int n;                // cells per layer (0: no layers)
    const float *cp;
    float *psi;
    long long base[3];    // start of the x-, y- and z-type blocks
    long long elems;      // floats in all three
};

struct FusedArgs {
    Layout L;
    const void *fin;
    void *fout;
    const uint8_t *mat;
    const float4 *coef;   // per material (Ca, Cbx, Cby, Cbz); graded spacing: (Ca, G, 0, 0)
    int n_mat;
    float chx, chy, chz;
    // Graded spacing (null: uniform, chx..chz and coef's Cb apply).  Per node
    // index, x (nx+1 entries) then y (ny+1) then z (nz+1): (c dt / primal
    // cell size, c dt / dual cell size); an E coefficient is G * the second.
    const float2 *gc;
    // Zero-tile skipping: every value of the input state outside the box
    // [box_lo, box_hi] (node indices x, y, z; w unused) is +0, and so is the
    // output buffer there; the launcher runs only the tiles meeting it.
    int4 box_lo, box_hi;
    int ntx, nty, ntz, nwg;   // launched tiles per axis (filled by the launcher)
    int tx0, ty0, tz0;        // index of the first launched tile per axis
    // Dead tiles: `live` (host, null: all live) is consulted by the launcher,
    // which then runs the listed `tiles` (device, full-tiling indices with ltx
    // x lty tiles per plane) instead of the range; listed tiles outside the
    // range exit at once.
    LiveNodes *live;
    const int *tiles;
    int ltx, lty;
    int zc;               // planes per z chunk
    long long step0;      // absolute step index advanced by time level 1
    SourceTable src;
    ProbeTable probe;
    StorageBlock sb;
    // host counters (null: none): += workgroups dispatched, tiles of the full
    // tiling, per launch
    long long *tile_stats;
};

// CPML layers for the fused kernel (a kernel argument of its own, so that
// batch descriptors stay small): psi of the input state in pml.psi, of the
// output state in psi_out (ping-pong, like the fields).
struct CpmlFused {
    Cpml pml;
    float *psi_out;
};

// Energy in the pass (uniform-spacing kernels, T <= MAX_T_ENERGY): time level
// `level` (1..T) sums W^n of its input state n = step0 + level - 1,
//   W^n = 1/2 sum eps_r E^n.E^n + 1/2 sum H^(n-1/2).H^(n+1/2)
// (eps_r of the edge's owner cell on interior edges; every H value in
// range), over the values each tile owns, into partial[work item] (FP64);
// launch_energy_sum then adds the partials in tile order into *out.
// half_eps[m] = eps_r(m) / 2.
struct EnergyFused {
    int level;
    double *partial;
    const double *half_eps;
    double *out;
};

// Up to MAX_BATCH solves in one launch; start[i] is the first work item
// (tile) of solve i, start[n] the total.  Passed by value as kernel
// arguments (no device copy of the descriptors).
constexpr int MAX_BATCH = 12;
// Longest time block of the fused kernel, and of its batched and
// graded-spacing forms.
constexpr int MAX_T = 6, MAX_T_BATCH = 4, MAX_T_GRADED = 4, MAX_T_CPML = 3, MAX_T_ENERGY = 4;
struct BatchArgs {
    int n;
    int start[MAX_BATCH + 1];
    FusedArgs s[MAX_BATCH];
};

struct PlainArgs {
    Layout L;
    float *f;             // in-place FP32 fields
    const uint8_t *mat;
    const float4 *coef;
    int n_mat;
    float chx, chy, chz;
    const float2 *gc;     // graded spacing, as in FusedArgs (null: uniform); with
                          // CPML, c dt / (kappa size) so the layers' stretch is folded in
    Cpml pml;
};

struct DiagArgs {
    Layout L;
    const void *f;
    const uint8_t *mat;
    const float4 *coef;
    const double *eps;    // per material eps_r
    int n_mat;
    float chx, chy, chz;
    double idx, idy, idz; // 1/dx, 1/dy, 1/dz
    // graded spacing (null: uniform): the update factors as in FusedArgs, and
    // per axis and node q the cell size d[q] (0 at q = n) and the dual size
    // (half cells on the walls), x then y then z
    const float2 *gc;
    const double2 *gsz;
    double *partial;      // per block: 11 doubles
    StorageBlock sb;      // scale[par] decodes the stored fields
};

enum { DIAG_W = 11 };     // energy, div_e_sumsq, div_h_sumsq, div_e_max, div_h_max, max_abs[6]

// Launchers (return hipError_t of the launch).
hipError_t launch_plain_step(const PlainArgs &a, const SourceTable &src, const ProbeTable &probe,
                             long long step, hipStream_t st);
// variant: tile shape (0 = default; FP32 also has 1 and 2); zc: planes per
// z chunk (0 = automatic).  a.gc set: graded spacing (FP32 storage only).
hipError_t launch_fused(int storage, int T, const FusedArgs &a, int variant, int zc, hipStream_t st);
// The fused kernel with CPML layers (graded FP32, T <= MAX_T_CPML, its own
// tile shape).
hipError_t launch_fused_cpml(int T, const FusedArgs &a, const CpmlFused &c, int zc, hipStream_t st);
// The fused kernel (uniform spacing, T <= MAX_T_ENERGY) that also sums the
// energy of one level's input state into *en.out; en.partial holds at least
// one double per launched tile (fused_tiles_bound).
hipError_t launch_fused_energy(int storage, int T, const FusedArgs &a, const EnergyFused &en, int variant, int zc,
                               hipStream_t st);
// Sum of partial[0..n) in a fixed order into *out (0 when n = 0).
hipError_t launch_energy_sum(const double *partial, long long n, double *out, hipStream_t st);
// Upper bound on the tiles of one fused launch over every T <= MAX_T_ENERGY,
// tile shape and z chunk.
long long fused_tiles_bound(const Layout &L);
// false if the psi arrays or a z chunk cannot be addressed with 32-bit offsets
bool cpml_fused_fits(const Layout &L, long long psi_elems, int T);
// One persistent launch over several solves sharing storage, T and shape;
// each args[i] is complete except for its tile geometry, which is filled in.
hipError_t launch_fused_batch(int storage, int T, const FusedArgs *args, int n, int variant, int zc,
                              hipStream_t st);
// false if a z chunk of this grid cannot be addressed with 32-bit offsets
bool fused_fits(const Layout &L, int storage, int T);
// Tile shape (index into the fused kernel's table) and steps per pass chosen
// when the caller does not: measured fastest on MI355X.
// cells: of the grid (0 for batched solves, which take the small-grid shape).
int auto_shape(int storage, int T, bool graded = false, long long cells = 0);
int fastest_T(const Layout &L, int storage, bool graded = false);
hipError_t launch_diag(int storage, const DiagArgs &a, double *out11, hipStream_t st);
int diag_blocks(const Layout &L);
// The diagnostics scratch that needs no allocation: a static device array,
// one per GPU.  Looks up the current device's copy (once per device) and
// returns where the 11 results and the block partials go; at most
// diag_static_max_blocks() partials fit.
hipError_t diag_static_scratch(double **out11, double **partial);
long long diag_static_max_blocks();

}  // namespace yee
