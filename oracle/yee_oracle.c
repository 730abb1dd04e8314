/*
 * Yee FDTD oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of the 3-D Yee
 * leapfrog scheme (Yee 1966; the update printed in Sec. 2.1 of Cessenat,
 * "Sophie, an FDTD code on the way to multicore").  It exists to check the
 * GPU library against; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it.  It shares no code with the GPU path.
 *
 * Three arithmetic modes:
 *   f64  -- the accuracy reference: every value and coefficient in double.
 *   f32  -- "operation-order" mode: float fields, coefficients rounded once
 *           from double, every product/sum in a fixed order with fmaf.  A
 *           GPU kernel that follows the same order is bit-identical to it.
 *   q    -- reduced-storage emulation: f32 arithmetic, fields quantised to
 *           binary16 or bfloat16 (per-component power-of-two scale) at the
 *           end of every block of T steps.
 *
 * Storage: six components Ex, Ey, Ez, Hx, Hy, Hz, each an array over the
 * (nx+1)(ny+1)(nz+1) node box, x fastest; entries outside a component's
 * staggered range are zero.  E is in V/m, H is stored as eta0*H (V/m).
 *
 *   Ex (i+1/2, j, k)     i<nx  j<=ny k<=nz
 *   Ey (i, j+1/2, k)     i<=nx j<ny  k<=nz
 *   Ez (i, j, k+1/2)     i<=nx j<=ny k<nz
 *   Hx (i, j+1/2, k+1/2) i<=nx j<ny  k<nz
 *   Hy (i+1/2, j, k+1/2) i<nx  j<=ny k<nz
 *   Hz (i+1/2, j+1/2, k) i<nx  j<ny  k<=nz
 *
 * One step n -> n+1 (state (E^n, H^{n-1/2}) -> (E^{n+1}, H^{n+1/2})):
 *   1. Faraday half-step on every H DoF of the ranges above.
 *   2. Ampere half-step with conductivity on every E edge that is not
 *      tangential to the outer walls; tangential E on the walls is a perfect
 *      electric conductor and stays zero (Sec. 3.3: E is zeroed on the PEC
 *      before the Faraday solve).
 *   3. Soft sources: E_c(src) += w[n]  (a current added to Ampere's law).
 *   4. Probes: record the component at (i,j,k) (pin-point outputs, Sec. 4.2).
 *
 * Materials: each interior E edge takes eps_r and sigma of its owner cell,
 * the cell whose lowest corner is the edge's lower end; mu_r = 1.  A
 * material with sigma = +infinity is a perfect electric conductor: its
 * coefficients are Ca = Cb = 0 (G = 0 on graded grids), so the edges its
 * cells own are zero after every update (the limit of the loss term, where
 * E is driven to zero, taken exactly).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#define C0 299792458.0
#define EPS0 8.8541878128e-12

enum { EX = 0, EY, EZ, HX, HY, HZ };

typedef struct {
    int nx, ny, nz;
    size_t sy, sz, n;   /* strides of j and k; points per component */
} grid_t;

static grid_t mkgrid(int nx, int ny, int nz)
{
    grid_t g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.sy = (size_t)nx + 1;
    g.sz = g.sy * ((size_t)ny + 1);
    g.n = g.sz * ((size_t)nz + 1);
    return g;
}

static size_t at(const grid_t *g, int i, int j, int k)
{
    return (size_t)i + g->sy * (size_t)j + g->sz * (size_t)k;
}

/* 1 if component c exists at storage point (i,j,k), 0 otherwise. */
static int in_range(const grid_t *g, int c, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i > g->nx || j > g->ny || k > g->nz) return 0;
    switch (c) {
    case EX: return i < g->nx;
    case EY: return j < g->ny;
    case EZ: return k < g->nz;
    case HX: return j < g->ny && k < g->nz;
    case HY: return i < g->nx && k < g->nz;
    case HZ: return i < g->nx && j < g->ny;
    }
    return 0;
}

/* 1 if E component c at (i,j,k) is an interior edge (updated by Ampere). */
static int e_interior(const grid_t *g, int c, int i, int j, int k)
{
    switch (c) {
    case EX: return i < g->nx && j > 0 && j < g->ny && k > 0 && k < g->nz;
    case EY: return j < g->ny && i > 0 && i < g->nx && k > 0 && k < g->nz;
    case EZ: return k < g->nz && i > 0 && i < g->nx && j > 0 && j < g->ny;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Coefficients (FP64).  For an edge with relative permittivity eps_r and    */
/* conductivity sigma, the semi-implicit (time-averaged) loss term gives      */
/*   a   = sigma dt / (2 eps0 eps_r)                                           */
/*   Ca  = (1 - a) / (1 + a)                                                   */
/*   Cb_d = (c dt / eps_r) / (1 + a) / d_d                                     */
/* and the Faraday coefficient is ch_d = c dt / d_d (mu_r = 1), matching the  */
/* c*dt/delta factor of the antisymmetric form of Maxwell's equations         */
/* (Sec. 2.1).                                                                */
/* ------------------------------------------------------------------------ */
void orc_coefficients(int n_mat, const double *eps_r, const double *sigma,
                      double dt, double dx, double dy, double dz,
                      double *coef /* n_mat x {Ca, Cbx, Cby, Cbz} */,
                      double *ch /* {chx, chy, chz} */)
{
    for (int m = 0; m < n_mat; m++) {
        if (isinf(sigma[m])) {              /* perfect conductor */
            for (int v = 0; v < 4; v++) coef[4 * m + v] = 0.0;
            continue;
        }
        double a = (sigma[m] * dt) / (2.0 * EPS0 * eps_r[m]);
        double cb = ((C0 * dt) / eps_r[m]) / (1.0 + a);
        coef[4 * m + 0] = (1.0 - a) / (1.0 + a);
        coef[4 * m + 1] = cb / dx;
        coef[4 * m + 2] = cb / dy;
        coef[4 * m + 3] = cb / dz;
    }
    ch[0] = (C0 * dt) / dx;
    ch[1] = (C0 * dt) / dy;
    ch[2] = (C0 * dt) / dz;
}

/* ------------------------------------------------------------------------ */
/* FP64 half-steps                                                          */
/* ------------------------------------------------------------------------ */

/* Faraday: H^{n+1/2} = H^{n-1/2} - c dt curl E^n (Sec. 2.1 prints Hx). */
void orc_h_half_f64(int nx, int ny, int nz, const double *ch, double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                if (in_range(&g, HX, i, j, k))
                    hx[p] = hx[p] + ch[2] * (ey[p + g.sz] - ey[p]) - ch[1] * (ez[p + g.sy] - ez[p]);
                if (in_range(&g, HY, i, j, k))
                    hy[p] = hy[p] + ch[0] * (ez[p + 1] - ez[p]) - ch[2] * (ex[p + g.sz] - ex[p]);
                if (in_range(&g, HZ, i, j, k))
                    hz[p] = hz[p] + ch[1] * (ex[p + g.sy] - ex[p]) - ch[0] * (ey[p + 1] - ey[p]);
            }
}

/* Ampere with conductivity on interior edges; owner-cell material. */
void orc_e_half_f64(int nx, int ny, int nz, const double *coef, const uint8_t *mat, double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const double *cf = coef + 4 * m;
                if (e_interior(&g, EX, i, j, k))
                    ex[p] = cf[0] * ex[p] + cf[2] * (hz[p] - hz[p - g.sy]) - cf[3] * (hy[p] - hy[p - g.sz]);
                if (e_interior(&g, EY, i, j, k))
                    ey[p] = cf[0] * ey[p] + cf[3] * (hx[p] - hx[p - g.sz]) - cf[1] * (hz[p] - hz[p - 1]);
                if (e_interior(&g, EZ, i, j, k))
                    ez[p] = cf[0] * ez[p] + cf[1] * (hy[p] - hy[p - 1]) - cf[2] * (hx[p] - hx[p - g.sy]);
            }
}

/* ------------------------------------------------------------------------ */
/* FP32 operation-order half-steps.                                         */
/* The order follows the printed Hx loop of Sec. 2.2 (z-difference term      */
/* first, y-difference term second, the y coefficient carrying the minus     */
/* sign of the Sec. 2.1 formula) and its cyclic permutations:                */
/*   Hx = fmaf(-chy, dEz_y, fmaf(chz, dEy_z, Hx))                            */
/*   Hy = fmaf(-chz, dEx_z, fmaf(chx, dEz_x, Hy))                            */
/*   Hz = fmaf(-chx, dEy_x, fmaf(chy, dEx_y, Hz))                            */
/*   Ex = fmaf(-Cbz, dHy_z, fmaf(Cby, dHz_y, Ca*Ex))                         */
/*   Ey = fmaf(-Cbx, dHz_x, fmaf(Cbz, dHx_z, Ca*Ey))                         */
/*   Ez = fmaf(-Cby, dHx_y, fmaf(Cbx, dHy_x, Ca*Ez))                         */
/* Each difference is a single float subtraction.                            */
/* ------------------------------------------------------------------------ */
void orc_h_half_f32(int nx, int ny, int nz, const float *ch, float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                if (in_range(&g, HX, i, j, k)) {
                    float dey_z = ey[p + g.sz] - ey[p];
                    float dez_y = ez[p + g.sy] - ez[p];
                    hx[p] = fmaf(-ch[1], dez_y, fmaf(ch[2], dey_z, hx[p]));
                }
                if (in_range(&g, HY, i, j, k)) {
                    float dez_x = ez[p + 1] - ez[p];
                    float dex_z = ex[p + g.sz] - ex[p];
                    hy[p] = fmaf(-ch[2], dex_z, fmaf(ch[0], dez_x, hy[p]));
                }
                if (in_range(&g, HZ, i, j, k)) {
                    float dex_y = ex[p + g.sy] - ex[p];
                    float dey_x = ey[p + 1] - ey[p];
                    hz[p] = fmaf(-ch[0], dey_x, fmaf(ch[1], dex_y, hz[p]));
                }
            }
}

void orc_e_half_f32(int nx, int ny, int nz, const float *coef, const uint8_t *mat, float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const float *cf = coef + 4 * m;
                if (e_interior(&g, EX, i, j, k)) {
                    float dhz_y = hz[p] - hz[p - g.sy];
                    float dhy_z = hy[p] - hy[p - g.sz];
                    float t = cf[0] * ex[p];
                    t = fmaf(cf[2], dhz_y, t);
                    ex[p] = fmaf(-cf[3], dhy_z, t);
                }
                if (e_interior(&g, EY, i, j, k)) {
                    float dhx_z = hx[p] - hx[p - g.sz];
                    float dhz_x = hz[p] - hz[p - 1];
                    float t = cf[0] * ey[p];
                    t = fmaf(cf[3], dhx_z, t);
                    ey[p] = fmaf(-cf[1], dhz_x, t);
                }
                if (e_interior(&g, EZ, i, j, k)) {
                    float dhy_x = hy[p] - hy[p - 1];
                    float dhx_y = hx[p] - hx[p - g.sy];
                    float t = cf[0] * ez[p];
                    t = fmaf(cf[1], dhy_x, t);
                    ez[p] = fmaf(-cf[2], dhx_y, t);
                }
            }
}

/* ------------------------------------------------------------------------ */
/* Whole runs: n_steps full steps starting at absolute step step0.           */
/*   src:   n_src x {comp, i, j, k}; wave: n_src x n_wave samples, w[n] is   */
/*          added during the step that produces E^{n+1} (zero for n>=n_wave) */
/*   probe: n_probe x {comp, i, j, k}; probe_out: n_steps x n_probe doubles, */
/*          the value after step step0+s completes (E^{n+1} or H^{n+1/2}).   */
/* Returns 0, or -1 for a bad source/probe descriptor.                       */
/* ------------------------------------------------------------------------ */
static int check_points(const grid_t *g, int n, const int *d, int e_only)
{
    for (int s = 0; s < n; s++) {
        int c = d[4 * s];
        if (c < 0 || c > 5 || (e_only && c > EZ)) return -1;
        if (!in_range(g, c, d[4 * s + 1], d[4 * s + 2], d[4 * s + 3])) return -1;
        if (e_only && !e_interior(g, c, d[4 * s + 1], d[4 * s + 2], d[4 * s + 3])) return -1;
    }
    return 0;
}

int orc_run_f64(int nx, int ny, int nz, const double *ch, const double *coef,
                const uint8_t *mat, double *f, long step0, int n_steps,
                int n_src, const int *src, const double *wave, int n_wave,
                int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_f64(nx, ny, nz, ch, f);
        orc_e_half_f64(nx, ny, nz, coef, mat, f);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])] += wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

int orc_run_f32(int nx, int ny, int nz, const float *ch, const float *coef,
                const uint8_t *mat, float *f, long step0, int n_steps,
                int n_src, const int *src, const float *wave, int n_wave,
                int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_f32(nx, ny, nz, ch, f);
        orc_e_half_f32(nx, ny, nz, coef, mat, f);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                size_t p = (size_t)d[0] * g.n + at(&g, d[1], d[2], d[3]);
                f[p] = f[p] + wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = (double)f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reduced-storage emulation.                                                */
/*                                                                          */
/* Storage formats: 1 = IEEE binary16 (with subnormals), 2 = bfloat16 (the   */
/* top half of binary32).  Both round to nearest, ties to even.  A value x  */
/* of component c is stored as q = RNE(x * 2^s_c) and read back as          */
/* q * 2^-s_c (exact).  If x * 2^s_c would round beyond the largest finite  */
/* value, the stored value saturates to +-max and the overflow flag is set;  */
/* a NaN sets the flag and is stored as NaN.                                 */
/*                                                                          */
/* Scale policy: s_c = 10 - ceil(log2 m) clamped to [-64, 64], with        */
/* m = max(M_c, A): M_c is the largest |stored value| of component c at the */
/* previous quantisation (at upload: the largest |uploaded value|) and A is */
/* the largest |source sample|.  If m is 0, the largest M over all six     */
/* components is used; if that is 0 too, s_c = 0.  The stored magnitudes   */
/* then stay below 2^10, 64x under the binary16 limit, so fields may grow  */
/* 64-fold within one block before overflowing.                            */
/*                                                                          */
/* Overflow retry: if some finite value of component c at a block's end    */
/* would round beyond the largest finite value with s_c, the block's end   */
/* is quantised instead with s_c = 10 - ceil(log2 max(m', A)), m' the      */
/* largest |value| of component c before quantisation (the block's own     */
/* FP32 values do not depend on the scale it ends with, so a GPU re-run of */
/* the block from its intact input gives the same values).  Only what     */
/* still overflows then saturates and raises the flag (an infinite value), */
/* as does a NaN.                                                           */
/* ------------------------------------------------------------------------ */

static uint32_t f2u(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float u2f(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }

/* binary32 -> binary16 bits, round to nearest even, subnormals kept.
 * Values that round beyond 65504 give +-inf bits (0x7c00). */
static uint16_t f32_to_f16_bits(float x)
{
    uint32_t u = f2u(x);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    uint32_t ax = u & 0x7fffffffu;
    if (ax > 0x7f800000u) return (uint16_t)(sign | 0x7e00u);   /* NaN */
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  /* >= 65520 rounds to inf */
    int e = (int)(ax >> 23) - 127;                             /* unbiased exponent */
    uint32_t mant = (ax & 0x7fffffu) | 0x800000u;              /* 24-bit significand */
    if (ax < 0x00800000u) return sign;                         /* fp32 subnormal: far below fp16 range */
    int shift;
    uint32_t h_exp;
    if (e >= -14) { shift = 13; h_exp = (uint32_t)(e + 15); }  /* normal fp16 */
    else { shift = 13 + (-14 - e); h_exp = 0; }                /* subnormal fp16 */
    if (shift > 24) return sign;                               /* rounds to zero */
    uint32_t q = mant >> shift;
    uint32_t rem = mant & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1u))) q++;
    uint32_t bits;
    if (h_exp == 0) bits = q;                       /* may carry into the normal range: correct */
    else bits = (h_exp << 10) + (q - 0x400u);       /* q in [0x400, 0x800]; carry bumps exponent */
    return (uint16_t)(sign | bits);
}

static float f16_bits_to_f32(uint16_t h)
{
    uint32_t sign = ((uint32_t)h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    if (e == 0x1f) return u2f(sign | 0x7f800000u | (m << 13));
    if (e == 0) return (sign ? -1.0f : 1.0f) * ldexpf((float)m, -24);
    return u2f(sign | ((e - 15 + 127) << 23) | (m << 13));
}

/* binary32 -> bfloat16 bits, round to nearest even. */
static uint16_t f32_to_bf16_bits(float x)
{
    uint32_t u = f2u(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

static float bf16_bits_to_f32(uint16_t h) { return u2f((uint32_t)h << 16); }

/* Exposed for the tests that pin the conversions against library routines. */
void orc_quantize_bits(int fmt, int n, const float *x, uint16_t *out)
{
    for (int i = 0; i < n; i++) out[i] = fmt == 1 ? f32_to_f16_bits(x[i]) : f32_to_bf16_bits(x[i]);
}

/* ceil(log2(m)) for finite m > 0 */
static int ceil_log2(float m)
{
    int e;
    float fr = frexpf(m, &e);      /* m = fr * 2^e, fr in [0.5, 1) */
    return fr == 0.5f ? e - 1 : e;
}

static int scale_from(float m)
{
    if (!(m > 0.0f) || isinf(m)) return 0;
    int s = 10 - ceil_log2(m);
    if (s > 64) s = 64;
    if (s < -64) s = -64;
    return s;
}

void orc_choose_scales(const float *m_prev, float a_max, int *s_out)
{
    float all = 0.0f;
    for (int c = 0; c < 6; c++) if (m_prev[c] > all) all = m_prev[c];
    for (int c = 0; c < 6; c++) {
        float m = m_prev[c] > a_max ? m_prev[c] : a_max;
        if (!(m > 0.0f)) m = all;
        s_out[c] = scale_from(m);
    }
}

/* Quantise one component array in place with scale s; returns the largest
 * |stored value| and raises *flag on overflow or NaN. */
static float quantize_array(int fmt, int s, size_t n, float *x, int *flag)
{
    float mx = 0.0f;
    int fl = 0;
    const float up = ldexpf(1.0f, s), down = ldexpf(1.0f, -s);
    /* every element is independent; the maximum and the flag do not depend
     * on the order of the reduction */
    #pragma omp parallel for schedule(static) reduction(max : mx) reduction(| : fl)
    for (size_t p = 0; p < n; p++) {
        float y = x[p] * up;
        float r;
        if (fmt == 1) {
            uint16_t h = f32_to_f16_bits(y);
            if ((h & 0x7fffu) == 0x7c00u) { h = (uint16_t)((h & 0x8000u) | 0x7bffu); fl = 1; }
            if ((h & 0x7fffu) > 0x7c00u) fl = 1;
            r = f16_bits_to_f32(h);
        } else {
            uint16_t h = f32_to_bf16_bits(y);
            if ((h & 0x7fffu) == 0x7f80u) { h = (uint16_t)((h & 0x8000u) | 0x7f7fu); fl = 1; }
            if ((h & 0x7fffu) > 0x7f80u) fl = 1;
            r = bf16_bits_to_f32(h);
        }
        x[p] = r * down;
        float a = fabsf(x[p]);
        if (a > mx) mx = a;
    }
    if (fl) *flag = 1;
    return mx;
}

/* 1 if some finite x * 2^s rounds beyond the largest finite value of the
 * format (NaN excluded). */
static int would_overflow(int fmt, int s, size_t n, const float *x)
{
    int ov = 0;
    const float up = ldexpf(1.0f, s);
    #pragma omp parallel for schedule(static) reduction(| : ov)
    for (size_t p = 0; p < n; p++) {
        if (isnan(x[p])) continue;
        const float y = x[p] * up;
        if (fmt == 1) ov |= (f32_to_f16_bits(y) & 0x7fffu) == 0x7c00u;
        else ov |= (f32_to_bf16_bits(y) & 0x7fffu) == 0x7f80u;
    }
    return ov;
}

/* largest |x| (NaN ignored) */
static float max_abs(size_t n, const float *x)
{
    float mx = 0.0f;
    #pragma omp parallel for schedule(static) reduction(max : mx)
    for (size_t p = 0; p < n; p++) if (fabsf(x[p]) > mx) mx = fabsf(x[p]);
    return mx;
}

/* Quantise all six components.  upload != 0: M comes from the values
 * themselves; otherwise from m_stored (the previous quantisation), with the
 * overflow retry above.  scales[6] and m_stored[6] are updated. */
void orc_quantize_state(int nx, int ny, int nz, int fmt, int upload, float a_max,
                        float *f, int *scales, float *m_stored, int *flag)
{
    grid_t g = mkgrid(nx, ny, nz);
    float m[6];
    for (int c = 0; c < 6; c++) {
        m[c] = m_stored[c];
        if (upload) {
            const float *x = f + (size_t)c * g.n;
            float mc = 0.0f;
            #pragma omp parallel for schedule(static) reduction(max : mc)
            for (size_t p = 0; p < g.n; p++) if (fabsf(x[p]) > mc) mc = fabsf(x[p]);
            m[c] = mc;
        }
    }
    orc_choose_scales(m, a_max, scales);
    for (int c = 0; c < 6; c++) {
        float *x = f + (size_t)c * g.n;
        if (!upload && would_overflow(fmt, scales[c], g.n, x)) {
            const float mp = max_abs(g.n, x);
            scales[c] = scale_from(mp > a_max ? mp : a_max);
        }
        m_stored[c] = quantize_array(fmt, scales[c], g.n, x, flag);
    }
}

/* f32 arithmetic with quantisation at the end of every block.  Blocks end
 * at absolute steps that are multiples of T and at the end of this run.
 * a_max: the largest |source sample| (the fallback for the scale). */
int orc_run_q(int nx, int ny, int nz, int fmt, int T, const float *ch, const float *coef,
              const uint8_t *mat, float *f, long step0, int n_steps,
              int n_src, const int *src, const float *wave, int n_wave,
              int n_probe, const int *probe, double *probe_out,
              float a_max, int *scales, float *m_stored, int *flag)
{
    for (int s = 0; s < n_steps; s++) {
        int rc = orc_run_f32(nx, ny, nz, ch, coef, mat, f, step0 + s, 1, n_src, src, wave, n_wave,
                             n_probe, probe, probe_out + (size_t)s * n_probe);
        if (rc) return rc;
        long done = step0 + s + 1;
        if (done % T == 0 || s == n_steps - 1)
            orc_quantize_state(nx, ny, nz, fmt, 0, a_max, f, scales, m_stored, flag);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics (FP64).                                                       */
/*   Energy  W^n = 1/2 sum_E eps_r E^n.E^n + 1/2 sum_H mu_r H^{n-1/2}.H^{n+1/2}*/
/*   in units of eps0*dx*dy*dz; it is the quantity conserved by the leapfrog  */
/*   in a lossless PEC box, a consequence of the discrete antisymmetry of     */
/*   Sec. 2.1.  H^{n+1/2} is computed with the same mode's H half-step on a   */
/*   copy.  Each k-plane is summed separately, then planes in order, so the  */
/*   result does not depend on the thread count.                              */
/*   div_e at interior nodes: sum_d (eps_r E_d(node) - eps_r E_d(node-e_d))/d_d */
/*   div_h at cell centres:   sum_d (H_d(cell+e_d) - H_d(cell))/d_d          */
/* ------------------------------------------------------------------------ */
static double edge_eps(const grid_t *g, const double *eps_r, const uint8_t *mat, int c, int i, int j, int k)
{
    if (!e_interior(g, c, i, j, k)) return 0.0;   /* PEC edges hold E = 0 */
    return eps_r[mat[(size_t)i + (size_t)g->nx * ((size_t)j + (size_t)g->ny * k)]];
}

static double energy_sum(const grid_t *g, const double *eps_r, const uint8_t *mat,
                         const double *e, const double *h0, const double *h1)
{
    int nz = g->nz;
    double *plane = (double *)calloc((size_t)nz + 1, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++) {
        double acc = 0.0;
        for (int j = 0; j <= g->ny; j++)
            for (int i = 0; i <= g->nx; i++) {
                size_t p = at(g, i, j, k);
                for (int c = 0; c < 3; c++) {
                    double ep = edge_eps(g, eps_r, mat, c, i, j, k);
                    double v = e[(size_t)c * g->n + p];
                    acc += 0.5 * ep * v * v;
                }
                for (int c = 0; c < 3; c++)
                    if (in_range(g, HX + c, i, j, k))
                        acc += 0.5 * h0[(size_t)c * g->n + p] * h1[(size_t)c * g->n + p];
            }
        plane[k] = acc;
    }
    double w = 0.0;
    for (int k = 0; k <= nz; k++) w += plane[k];
    free(plane);
    return w;
}

double orc_energy_f64(int nx, int ny, int nz, const double *ch, const double *eps_r,
                      const uint8_t *mat, const double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    double *tmp = (double *)malloc(6 * g.n * sizeof(double));
    memcpy(tmp, f, 6 * g.n * sizeof(double));
    orc_h_half_f64(nx, ny, nz, ch, tmp);
    double w = energy_sum(&g, eps_r, mat, f, f + 3 * g.n, tmp + 3 * g.n);
    free(tmp);
    return w;
}

double orc_energy_f32(int nx, int ny, int nz, const float *ch, const double *eps_r,
                      const uint8_t *mat, const float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    float *tmp = (float *)malloc(6 * g.n * sizeof(float));
    memcpy(tmp, f, 6 * g.n * sizeof(float));
    orc_h_half_f32(nx, ny, nz, ch, tmp);
    double *e = (double *)malloc(9 * g.n * sizeof(double));
    for (size_t p = 0; p < 6 * g.n; p++) e[p] = (double)f[p];
    for (size_t p = 0; p < 3 * g.n; p++) e[6 * g.n + p] = (double)tmp[3 * g.n + p];
    double w = energy_sum(&g, eps_r, mat, e, e + 3 * g.n, e + 6 * g.n);
    free(e);
    free(tmp);
    return w;
}

/* div_e: (nz+1)(ny+1)(nx+1) node array (zero on boundary nodes);
 * div_h: nz*ny*nx cell array. */
void orc_divergence_f64(int nx, int ny, int nz, double dx, double dy, double dz,
                        const double *eps_r, const uint8_t *mat, const double *f,
                        double *div_e, double *div_h)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                double d = 0.0;
                if (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz) {
                    d += (edge_eps(&g, eps_r, mat, EX, i, j, k) * ex[p]
                          - edge_eps(&g, eps_r, mat, EX, i - 1, j, k) * ex[p - 1]) / dx;
                    d += (edge_eps(&g, eps_r, mat, EY, i, j, k) * ey[p]
                          - edge_eps(&g, eps_r, mat, EY, i, j - 1, k) * ey[p - g.sy]) / dy;
                    d += (edge_eps(&g, eps_r, mat, EZ, i, j, k) * ez[p]
                          - edge_eps(&g, eps_r, mat, EZ, i, j, k - 1) * ez[p - g.sz]) / dz;
                }
                div_e[p] = d;
                if (i < nx && j < ny && k < nz) {
                    double dh = (hx[p + 1] - hx[p]) / dx + (hy[p + g.sy] - hy[p]) / dy
                              + (hz[p + g.sz] - hz[p]) / dz;
                    div_h[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] = dh;
                }
            }
}

/* ------------------------------------------------------------------------ */
/* Graded (non-uniform) spacing.                                              */
/*                                                                          */
/* The paper's loop takes the spacing from one-dimensional per-index        */
/* coefficient arrays (dy(j), dz(k) in Sec. 2.2).  With primal cell sizes    */
/* dx[i] (i < nx), dy[j], dz[k], Stokes' theorem on a primal face gives the  */
/* Faraday update with primal sizes, and on the dual face around an E edge   */
/* the Ampere update with dual sizes d'[idx] = (d[idx-1] + d[idx]) / 2 at    */
/* interior nodes:                                                           */
/*   hc_d[idx] = c dt / d[idx]          idx < n_d      (0 at idx = n_d)      */
/*   ec_d[idx] = c dt / d'[idx]         0 < idx < n_d  (0 on the walls)      */
/*   per material: a = sigma dt / (2 eps0 eps_r),                            */
/*                 Ca = (1 - a) / (1 + a),  G = (1 / eps_r) / (1 + a)        */
/*   Hx <- Hx + hc_z[k] (Ey(k+1) - Ey(k)) - hc_y[j] (Ez(j+1) - Ez(j))        */
/*   Ex <- Ca Ex + G ec_y[j] (Hz(j) - Hz(j-1)) - G ec_z[k] (Hy(k) - Hy(k-1)) */
/* and cyclic.  The FP32 mode forms each E coefficient as one float product  */
/* cb = G * ec_d[idx] and then follows the uniform mode's fmaf order; the H  */
/* update is the uniform one with per-index coefficients.                    */
/* hc and ec hold the x, y and z arrays one after another:                   */
/* (nx+1) + (ny+1) + (nz+1) values.                                          */
/* ------------------------------------------------------------------------ */
void orc_graded_coefficients(int n_mat, const double *eps_r, const double *sigma, double dt,
                             int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                             double *cag /* n_mat x {Ca, G} */, double *hc, double *ec)
{
    for (int m = 0; m < n_mat; m++) {
        if (isinf(sigma[m])) {              /* perfect conductor */
            cag[2 * m + 0] = cag[2 * m + 1] = 0.0;
            continue;
        }
        double a = (sigma[m] * dt) / (2.0 * EPS0 * eps_r[m]);
        cag[2 * m + 0] = (1.0 - a) / (1.0 + a);
        cag[2 * m + 1] = (1.0 / eps_r[m]) / (1.0 + a);
    }
    const int n[3] = {nx, ny, nz};
    const double *d[3] = {dx, dy, dz};
    int off = 0;
    for (int ax = 0; ax < 3; ax++) {
        for (int q = 0; q <= n[ax]; q++) {
            hc[off + q] = q < n[ax] ? (C0 * dt) / d[ax][q] : 0.0;
            ec[off + q] = (q > 0 && q < n[ax]) ? (C0 * dt) / ((d[ax][q - 1] + d[ax][q]) / 2.0) : 0.0;
        }
        off += n[ax] + 1;
    }
}

void orc_h_half_graded_f64(int nx, int ny, int nz, const double *hc, double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *hcx = hc, *hcy = hc + nx + 1, *hcz = hc + nx + 1 + ny + 1;
    const double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                if (in_range(&g, HX, i, j, k))
                    hx[p] = hx[p] + hcz[k] * (ey[p + g.sz] - ey[p]) - hcy[j] * (ez[p + g.sy] - ez[p]);
                if (in_range(&g, HY, i, j, k))
                    hy[p] = hy[p] + hcx[i] * (ez[p + 1] - ez[p]) - hcz[k] * (ex[p + g.sz] - ex[p]);
                if (in_range(&g, HZ, i, j, k))
                    hz[p] = hz[p] + hcy[j] * (ex[p + g.sy] - ex[p]) - hcx[i] * (ey[p + 1] - ey[p]);
            }
}

void orc_e_half_graded_f64(int nx, int ny, int nz, const double *cag, const double *ec, const uint8_t *mat,
                           double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *ecx = ec, *ecy = ec + nx + 1, *ecz = ec + nx + 1 + ny + 1;
    double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const double ca = cag[2 * m], gm = cag[2 * m + 1];
                if (e_interior(&g, EX, i, j, k))
                    ex[p] = ca * ex[p] + gm * ecy[j] * (hz[p] - hz[p - g.sy]) - gm * ecz[k] * (hy[p] - hy[p - g.sz]);
                if (e_interior(&g, EY, i, j, k))
                    ey[p] = ca * ey[p] + gm * ecz[k] * (hx[p] - hx[p - g.sz]) - gm * ecx[i] * (hz[p] - hz[p - 1]);
                if (e_interior(&g, EZ, i, j, k))
                    ez[p] = ca * ez[p] + gm * ecx[i] * (hy[p] - hy[p - 1]) - gm * ecy[j] * (hx[p] - hx[p - g.sy]);
            }
}

void orc_h_half_graded_f32(int nx, int ny, int nz, const float *hc, float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const float *hcx = hc, *hcy = hc + nx + 1, *hcz = hc + nx + 1 + ny + 1;
    const float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                if (in_range(&g, HX, i, j, k)) {
                    float dey_z = ey[p + g.sz] - ey[p];
                    float dez_y = ez[p + g.sy] - ez[p];
                    hx[p] = fmaf(-hcy[j], dez_y, fmaf(hcz[k], dey_z, hx[p]));
                }
                if (in_range(&g, HY, i, j, k)) {
                    float dez_x = ez[p + 1] - ez[p];
                    float dex_z = ex[p + g.sz] - ex[p];
                    hy[p] = fmaf(-hcz[k], dex_z, fmaf(hcx[i], dez_x, hy[p]));
                }
                if (in_range(&g, HZ, i, j, k)) {
                    float dex_y = ex[p + g.sy] - ex[p];
                    float dey_x = ey[p + 1] - ey[p];
                    hz[p] = fmaf(-hcx[i], dey_x, fmaf(hcy[j], dex_y, hz[p]));
                }
            }
}

void orc_e_half_graded_f32(int nx, int ny, int nz, const float *cag, const float *ec, const uint8_t *mat,
                           float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    const float *ecx = ec, *ecy = ec + nx + 1, *ecz = ec + nx + 1 + ny + 1;
    float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const float ca = cag[2 * m], gm = cag[2 * m + 1];
                if (e_interior(&g, EX, i, j, k)) {
                    float cby = gm * ecy[j], cbz = gm * ecz[k];
                    float dhz_y = hz[p] - hz[p - g.sy];
                    float dhy_z = hy[p] - hy[p - g.sz];
                    float t = ca * ex[p];
                    t = fmaf(cby, dhz_y, t);
                    ex[p] = fmaf(-cbz, dhy_z, t);
                }
                if (e_interior(&g, EY, i, j, k)) {
                    float cbz = gm * ecz[k], cbx = gm * ecx[i];
                    float dhx_z = hx[p] - hx[p - g.sz];
                    float dhz_x = hz[p] - hz[p - 1];
                    float t = ca * ey[p];
                    t = fmaf(cbz, dhx_z, t);
                    ey[p] = fmaf(-cbx, dhz_x, t);
                }
                if (e_interior(&g, EZ, i, j, k)) {
                    float cbx = gm * ecx[i], cby = gm * ecy[j];
                    float dhy_x = hy[p] - hy[p - 1];
                    float dhx_y = hx[p] - hx[p - g.sy];
                    float t = ca * ez[p];
                    t = fmaf(cbx, dhy_x, t);
                    ez[p] = fmaf(-cby, dhx_y, t);
                }
            }
}

int orc_run_graded_f64(int nx, int ny, int nz, const double *hc, const double *cag, const double *ec,
                       const uint8_t *mat, double *f, long step0, int n_steps,
                       int n_src, const int *src, const double *wave, int n_wave,
                       int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_graded_f64(nx, ny, nz, hc, f);
        orc_e_half_graded_f64(nx, ny, nz, cag, ec, mat, f);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])] += wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

int orc_run_graded_f32(int nx, int ny, int nz, const float *hc, const float *cag, const float *ec,
                       const uint8_t *mat, float *f, long step0, int n_steps,
                       int n_src, const int *src, const float *wave, int n_wave,
                       int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_graded_f32(nx, ny, nz, hc, f);
        orc_e_half_graded_f32(nx, ny, nz, cag, ec, mat, f);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                size_t p = (size_t)d[0] * g.n + at(&g, d[1], d[2], d[3]);
                f[p] = f[p] + wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = (double)f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

/* Graded energy and divergence (FP64).  Dual sizes on the walls are half    */
/* cells.  With V_e = (edge length) x (dual face area) for E and            */
/* V_f = (face area) x (dual edge length) for H,                             */
/*   W = 1/2 sum_e eps_r E_e^2 V_e + 1/2 sum_f H_f^{n-1/2} H_f^{n+1/2} V_f   */
/* in units of eps0 (volumes in m^3) is conserved by a lossless PEC box;     */
/*   div_e(node) = sum_d (eps_r E_d(node) - eps_r E_d(node - e_d)) / d'_d    */
/*   div_h(cell) = sum_d (H_d(cell + e_d) - H_d(cell)) / d_d                 */
/* stay constant without sources.                                            */
static void dual_sizes(int n, const double *d, double *dd)
{
    for (int q = 0; q <= n; q++)
        dd[q] = q == 0 ? d[0] / 2.0 : (q == n ? d[n - 1] / 2.0 : (d[q - 1] + d[q]) / 2.0);
}

/* weighted sum of the energy terms; h1 holds H^{n+1/2} (3 components) */
static double graded_energy_sum(int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                                const double *eps_r, const uint8_t *mat, const double *f, const double *h1)
{
    grid_t g = mkgrid(nx, ny, nz);
    double *dxd = (double *)malloc(((size_t)nx + ny + nz + 3) * sizeof(double));
    double *dyd = dxd + nx + 1, *dzd = dyd + ny + 1;
    dual_sizes(nx, dx, dxd);
    dual_sizes(ny, dy, dyd);
    dual_sizes(nz, dz, dzd);
    double *plane = (double *)calloc((size_t)nz + 1, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++) {
        double acc = 0.0;
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                const double ve[3] = {
                    i < nx ? dx[i] * dyd[j] * dzd[k] : 0.0,
                    j < ny ? dxd[i] * dy[j] * dzd[k] : 0.0,
                    k < nz ? dxd[i] * dyd[j] * dz[k] : 0.0};
                const double vh[3] = {
                    (j < ny && k < nz) ? dxd[i] * dy[j] * dz[k] : 0.0,
                    (i < nx && k < nz) ? dx[i] * dyd[j] * dz[k] : 0.0,
                    (i < nx && j < ny) ? dx[i] * dy[j] * dzd[k] : 0.0};
                for (int c = 0; c < 3; c++) {
                    double v = f[(size_t)c * g.n + p];
                    acc += 0.5 * edge_eps(&g, eps_r, mat, c, i, j, k) * v * v * ve[c];
                }
                for (int c = 0; c < 3; c++)
                    if (in_range(&g, HX + c, i, j, k))
                        acc += 0.5 * f[(size_t)(3 + c) * g.n + p] * h1[(size_t)c * g.n + p] * vh[c];
            }
        plane[k] = acc;
    }
    double w = 0.0;
    for (int k = 0; k <= nz; k++) w += plane[k];
    free(plane);
    free(dxd);
    return w;
}

double orc_energy_graded_f64(int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                             const double *hc, const double *eps_r, const uint8_t *mat, const double *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    double *tmp = (double *)malloc(6 * g.n * sizeof(double));
    memcpy(tmp, f, 6 * g.n * sizeof(double));
    orc_h_half_graded_f64(nx, ny, nz, hc, tmp);
    double w = graded_energy_sum(nx, ny, nz, dx, dy, dz, eps_r, mat, f, tmp + 3 * g.n);
    free(tmp);
    return w;
}

/* The same energy of FP32 fields, with H^{n+1/2} from the FP32 graded
 * half-step (the operation order of the kernels), summed in FP64. */
double orc_energy_graded_f32(int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                             const float *hc, const double *eps_r, const uint8_t *mat, const float *f)
{
    grid_t g = mkgrid(nx, ny, nz);
    float *tmp = (float *)malloc(6 * g.n * sizeof(float));
    memcpy(tmp, f, 6 * g.n * sizeof(float));
    orc_h_half_graded_f32(nx, ny, nz, hc, tmp);
    double *e = (double *)malloc(9 * g.n * sizeof(double));
    for (size_t p = 0; p < 6 * g.n; p++) e[p] = (double)f[p];
    for (size_t p = 0; p < 3 * g.n; p++) e[6 * g.n + p] = (double)tmp[3 * g.n + p];
    double w = graded_energy_sum(nx, ny, nz, dx, dy, dz, eps_r, mat, e, e + 6 * g.n);
    free(e);
    free(tmp);
    return w;
}

void orc_divergence_graded_f64(int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                               const double *eps_r, const uint8_t *mat, const double *f,
                               double *div_e, double *div_h)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    double *dxd = (double *)malloc(((size_t)nx + ny + nz + 3) * sizeof(double));
    double *dyd = dxd + nx + 1, *dzd = dyd + ny + 1;
    dual_sizes(nx, dx, dxd);
    dual_sizes(ny, dy, dyd);
    dual_sizes(nz, dz, dzd);
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                double d = 0.0;
                if (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz) {
                    d += (edge_eps(&g, eps_r, mat, EX, i, j, k) * ex[p]
                          - edge_eps(&g, eps_r, mat, EX, i - 1, j, k) * ex[p - 1]) / dxd[i];
                    d += (edge_eps(&g, eps_r, mat, EY, i, j, k) * ey[p]
                          - edge_eps(&g, eps_r, mat, EY, i, j - 1, k) * ey[p - g.sy]) / dyd[j];
                    d += (edge_eps(&g, eps_r, mat, EZ, i, j, k) * ez[p]
                          - edge_eps(&g, eps_r, mat, EZ, i, j, k - 1) * ez[p - g.sz]) / dzd[k];
                }
                div_e[p] = d;
                if (i < nx && j < ny && k < nz) {
                    double dh = (hx[p + 1] - hx[p]) / dx[i] + (hy[p + g.sy] - hy[p]) / dy[j]
                              + (hz[p + g.sz] - hz[p]) / dz[k];
                    div_h[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] = dh;
                }
            }
    free(dxd);
}

/* ------------------------------------------------------------------------ */
/* Convolutional PML (CPML) absorbing layers.                                */
/*                                                                          */
/* The paper cites the convolutional PML of Roden and Gedney (2000) as the   */
/* radiation condition its production code implements (Sec. 3.3, Sec. 4.2),  */
/* with one-dimensional coefficients so as not to add bandwidth.  The        */
/* formulation here is that published CFS-CPML (also Taflove and Hagness,    */
/* 3rd ed., Sec. 7.9-7.11).  In a layer of N                                 */
/* cells on every face each spatial derivative d/du of the curl becomes     */
/*   (1/kappa_u) d/du + psi_u,  psi_u <- b_u psi_u + a_u (difference along u) */
/* with, at depth rho (cells, measured from the inner face of the layer),   */
/*   x = rho / N,  sigma = sigma_max x^m,  kappa = 1 + (kappa_max - 1) x^m,   */
/*   alpha = alpha_max (1 - x),                                              */
/*   b = exp(-(sigma / kappa + alpha) dt / eps0),                             */
/*   a = sigma (b - 1) / (kappa (sigma + kappa alpha))   (0 when sigma = 0),  */
/*   sigma_max = sigma_factor * 0.8 (m + 1) / (eta0 d_out),                   */
/* d_out being the outermost cell size of that face.  Depths: an H value at  */
/* cell q (position q + 1/2) has rho = N - (q + 1/2) in the low layer and     */
/* (q + 1/2) - (n - N) in the high one; an E value at node q has rho = N - q */
/* and q - (n - N).  psi is kept where rho > 0: H cells q < N or q >= n - N,  */
/* E nodes 0 < q < N or n - N < q < n.                                       */
/*                                                                          */
/* Coefficients are the graded ones with kappa folded in,                    */
/*   hc[q] = c dt / (kappa_h(q) d[q]),  ec[q] = c dt / (kappa_e(q) d'[q]),     */
/* so outside the layers the update is the graded one, and per axis and      */
/* index cp holds {b_h, a_h, c dt / d[q], b_e, a_e, c dt / d'[q]}.          */
/* One step: the graded H half-step, then each H value in a layer adds its    */
/* psi terms in the order of its update (Hx: z then y, Hy: x then z, Hz: y   */
/* then x), psi updated first:                                               */
/*   psi = b psi + a diff;   Hx += (c dt/dz) psi_z,  Hx -= (c dt/dy) psi_y    */
/* then the graded E half-step and likewise for interior E edges with the    */
/* material factor G: Ex += G (c dt/dy') psi_y, Ex -= G (c dt/dz') psi_z.     */
/* FP32 mode: psi = fmaf(b, psi, a * diff); field = fmaf(+-coef, psi, field), */
/* the E coefficient formed as one float product G * (c dt / d').           */
/* psi state: 12 arrays over the node box (component c, axis u), order       */
/* (Hx,y) (Hx,z) (Hy,z) (Hy,x) (Hz,x) (Hz,y) (Ex,y) (Ex,z) (Ey,z) (Ey,x)     */
/* (Ez,x) (Ez,y); only entries in a layer are used.                          */
/* ------------------------------------------------------------------------ */
enum { PS_HXY = 0, PS_HXZ, PS_HYZ, PS_HYX, PS_HZX, PS_HZY, PS_EXY, PS_EXZ, PS_EYZ, PS_EYX, PS_EZX, PS_EZY };

static int cpml_h_in(int n, int N, int q) { return q < N || q >= n - N; }
static int cpml_e_in(int n, int N, int q) { return (q > 0 && q < N) || (q > n - N && q < n); }

int orc_cpml_coefficients(int n_mat, const double *eps_r, const double *sigma, double dt,
                          int nx, int ny, int nz, const double *dx, const double *dy, const double *dz,
                          int N, int m, double sigma_factor, double kappa_max, double alpha_max,
                          double *cag, double *hc, double *ec, double *cp /* 6 per index */)
{
    const int n[3] = {nx, ny, nz};
    const double *d[3] = {dx, dy, dz};
    if (N < 1) return -1;
    for (int ax = 0; ax < 3; ax++)
        if (2 * N >= n[ax]) return -1;
    orc_graded_coefficients(n_mat, eps_r, sigma, dt, nx, ny, nz, dx, dy, dz, cag, hc, ec);
    const double eta0 = 1.0 / (EPS0 * C0);
    int off = 0;
    for (int ax = 0; ax < 3; ax++) {
        const int nn = n[ax];
        const double smax_lo = sigma_factor * 0.8 * (m + 1) / (eta0 * d[ax][0]);
        const double smax_hi = sigma_factor * 0.8 * (m + 1) / (eta0 * d[ax][nn - 1]);
        for (int q = 0; q <= nn; q++) {
            double *c = cp + 6 * (size_t)(off + q);
            for (int v = 0; v < 6; v++) c[v] = 0.0;
            for (int half = 0; half < 2; half++) {        /* 0: H at q + 1/2, 1: E at node q */
                if (half == 0 && q == nn) continue;
                const double pos = half == 0 ? q + 0.5 : (double)q;
                double rho = 0.0, smax = 0.0;
                if (pos < N) { rho = N - pos; smax = smax_lo; }
                else if (pos > nn - N) { rho = pos - (nn - N); smax = smax_hi; }
                const int inside = half == 0 ? cpml_h_in(nn, N, q) : cpml_e_in(nn, N, q);
                double kappa = 1.0, b = 0.0, a = 0.0;
                if (rho > 0.0) {
                    const double x = rho / N, xm = pow(x, m);
                    const double sg = smax * xm, al = alpha_max * (1.0 - x);
                    kappa = 1.0 + (kappa_max - 1.0) * xm;
                    b = exp(-(sg / kappa + al) * dt / EPS0);
                    a = sg > 0.0 ? sg * (b - 1.0) / (kappa * (sg + kappa * al)) : 0.0;
                }
                if (half == 0) {
                    if (kappa != 1.0) hc[off + q] = (C0 * dt) / (kappa * d[ax][q]);
                    c[0] = inside ? b : 0.0;
                    c[1] = inside ? a : 0.0;
                    c[2] = (C0 * dt) / d[ax][q];
                } else if (q > 0 && q < nn) {
                    const double dd = (d[ax][q - 1] + d[ax][q]) / 2.0;
                    if (kappa != 1.0) ec[off + q] = (C0 * dt) / (kappa * dd);
                    c[3] = inside ? b : 0.0;
                    c[4] = inside ? a : 0.0;
                    c[5] = (C0 * dt) / dd;
                }
            }
        }
        off += nn + 1;
    }
    return 0;
}

/* psi terms after the graded half-steps (see above), FP64 */
static void cpml_h_f64(int nx, int ny, int nz, int N, const double *cp, double *f, double *psi)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *cx = cp, *cy = cp + 6 * ((size_t)nx + 1), *cz = cy + 6 * ((size_t)ny + 1);
    const double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                double *ps;
                if (in_range(&g, HX, i, j, k)) {
                    if (cpml_h_in(nz, N, k)) {
                        ps = psi + PS_HXZ * g.n + p;
                        *ps = cz[6 * k] * *ps + cz[6 * k + 1] * (ey[p + g.sz] - ey[p]);
                        hx[p] += cz[6 * k + 2] * *ps;
                    }
                    if (cpml_h_in(ny, N, j)) {
                        ps = psi + PS_HXY * g.n + p;
                        *ps = cy[6 * j] * *ps + cy[6 * j + 1] * (ez[p + g.sy] - ez[p]);
                        hx[p] -= cy[6 * j + 2] * *ps;
                    }
                }
                if (in_range(&g, HY, i, j, k)) {
                    if (cpml_h_in(nx, N, i)) {
                        ps = psi + PS_HYX * g.n + p;
                        *ps = cx[6 * i] * *ps + cx[6 * i + 1] * (ez[p + 1] - ez[p]);
                        hy[p] += cx[6 * i + 2] * *ps;
                    }
                    if (cpml_h_in(nz, N, k)) {
                        ps = psi + PS_HYZ * g.n + p;
                        *ps = cz[6 * k] * *ps + cz[6 * k + 1] * (ex[p + g.sz] - ex[p]);
                        hy[p] -= cz[6 * k + 2] * *ps;
                    }
                }
                if (in_range(&g, HZ, i, j, k)) {
                    if (cpml_h_in(ny, N, j)) {
                        ps = psi + PS_HZY * g.n + p;
                        *ps = cy[6 * j] * *ps + cy[6 * j + 1] * (ex[p + g.sy] - ex[p]);
                        hz[p] += cy[6 * j + 2] * *ps;
                    }
                    if (cpml_h_in(nx, N, i)) {
                        ps = psi + PS_HZX * g.n + p;
                        *ps = cx[6 * i] * *ps + cx[6 * i + 1] * (ey[p + 1] - ey[p]);
                        hz[p] -= cx[6 * i + 2] * *ps;
                    }
                }
            }
}

static void cpml_e_f64(int nx, int ny, int nz, int N, const double *cp, const double *cag, const uint8_t *mat,
                       double *f, double *psi)
{
    grid_t g = mkgrid(nx, ny, nz);
    const double *cx = cp, *cy = cp + 6 * ((size_t)nx + 1), *cz = cy + 6 * ((size_t)ny + 1);
    double *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const double *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const double gm = cag[2 * m + 1];
                double *ps;
                if (e_interior(&g, EX, i, j, k)) {
                    if (cpml_e_in(ny, N, j)) {
                        ps = psi + PS_EXY * g.n + p;
                        *ps = cy[6 * j + 3] * *ps + cy[6 * j + 4] * (hz[p] - hz[p - g.sy]);
                        ex[p] += gm * cy[6 * j + 5] * *ps;
                    }
                    if (cpml_e_in(nz, N, k)) {
                        ps = psi + PS_EXZ * g.n + p;
                        *ps = cz[6 * k + 3] * *ps + cz[6 * k + 4] * (hy[p] - hy[p - g.sz]);
                        ex[p] -= gm * cz[6 * k + 5] * *ps;
                    }
                }
                if (e_interior(&g, EY, i, j, k)) {
                    if (cpml_e_in(nz, N, k)) {
                        ps = psi + PS_EYZ * g.n + p;
                        *ps = cz[6 * k + 3] * *ps + cz[6 * k + 4] * (hx[p] - hx[p - g.sz]);
                        ey[p] += gm * cz[6 * k + 5] * *ps;
                    }
                    if (cpml_e_in(nx, N, i)) {
                        ps = psi + PS_EYX * g.n + p;
                        *ps = cx[6 * i + 3] * *ps + cx[6 * i + 4] * (hz[p] - hz[p - 1]);
                        ey[p] -= gm * cx[6 * i + 5] * *ps;
                    }
                }
                if (e_interior(&g, EZ, i, j, k)) {
                    if (cpml_e_in(nx, N, i)) {
                        ps = psi + PS_EZX * g.n + p;
                        *ps = cx[6 * i + 3] * *ps + cx[6 * i + 4] * (hy[p] - hy[p - 1]);
                        ez[p] += gm * cx[6 * i + 5] * *ps;
                    }
                    if (cpml_e_in(ny, N, j)) {
                        ps = psi + PS_EZY * g.n + p;
                        *ps = cy[6 * j + 3] * *ps + cy[6 * j + 4] * (hx[p] - hx[p - g.sy]);
                        ez[p] -= gm * cy[6 * j + 5] * *ps;
                    }
                }
            }
}

/* FP32 operation order */
static void cpml_h_f32(int nx, int ny, int nz, int N, const float *cp, float *f, float *psi)
{
    grid_t g = mkgrid(nx, ny, nz);
    const float *cx = cp, *cy = cp + 6 * ((size_t)nx + 1), *cz = cy + 6 * ((size_t)ny + 1);
    const float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                float *ps;
                if (in_range(&g, HX, i, j, k)) {
                    if (cpml_h_in(nz, N, k)) {
                        ps = psi + PS_HXZ * g.n + p;
                        float dey_z = ey[p + g.sz] - ey[p];
                        *ps = fmaf(cz[6 * k], *ps, cz[6 * k + 1] * dey_z);
                        hx[p] = fmaf(cz[6 * k + 2], *ps, hx[p]);
                    }
                    if (cpml_h_in(ny, N, j)) {
                        ps = psi + PS_HXY * g.n + p;
                        float dez_y = ez[p + g.sy] - ez[p];
                        *ps = fmaf(cy[6 * j], *ps, cy[6 * j + 1] * dez_y);
                        hx[p] = fmaf(-cy[6 * j + 2], *ps, hx[p]);
                    }
                }
                if (in_range(&g, HY, i, j, k)) {
                    if (cpml_h_in(nx, N, i)) {
                        ps = psi + PS_HYX * g.n + p;
                        float dez_x = ez[p + 1] - ez[p];
                        *ps = fmaf(cx[6 * i], *ps, cx[6 * i + 1] * dez_x);
                        hy[p] = fmaf(cx[6 * i + 2], *ps, hy[p]);
                    }
                    if (cpml_h_in(nz, N, k)) {
                        ps = psi + PS_HYZ * g.n + p;
                        float dex_z = ex[p + g.sz] - ex[p];
                        *ps = fmaf(cz[6 * k], *ps, cz[6 * k + 1] * dex_z);
                        hy[p] = fmaf(-cz[6 * k + 2], *ps, hy[p]);
                    }
                }
                if (in_range(&g, HZ, i, j, k)) {
                    if (cpml_h_in(ny, N, j)) {
                        ps = psi + PS_HZY * g.n + p;
                        float dex_y = ex[p + g.sy] - ex[p];
                        *ps = fmaf(cy[6 * j], *ps, cy[6 * j + 1] * dex_y);
                        hz[p] = fmaf(cy[6 * j + 2], *ps, hz[p]);
                    }
                    if (cpml_h_in(nx, N, i)) {
                        ps = psi + PS_HZX * g.n + p;
                        float dey_x = ey[p + 1] - ey[p];
                        *ps = fmaf(cx[6 * i], *ps, cx[6 * i + 1] * dey_x);
                        hz[p] = fmaf(-cx[6 * i + 2], *ps, hz[p]);
                    }
                }
            }
}

static void cpml_e_f32(int nx, int ny, int nz, int N, const float *cp, const float *cag, const uint8_t *mat,
                       float *f, float *psi)
{
    grid_t g = mkgrid(nx, ny, nz);
    const float *cx = cp, *cy = cp + 6 * ((size_t)nx + 1), *cz = cy + 6 * ((size_t)ny + 1);
    float *ex = f, *ey = f + g.n, *ez = f + 2 * g.n;
    const float *hx = f + 3 * g.n, *hy = f + 4 * g.n, *hz = f + 5 * g.n;
    #pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                size_t p = at(&g, i, j, k);
                int m = (i < nx && j < ny && k < nz) ? mat[(size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k)] : 0;
                const float gm = cag[2 * m + 1];
                float *ps;
                if (e_interior(&g, EX, i, j, k)) {
                    if (cpml_e_in(ny, N, j)) {
                        ps = psi + PS_EXY * g.n + p;
                        float dhz_y = hz[p] - hz[p - g.sy];
                        *ps = fmaf(cy[6 * j + 3], *ps, cy[6 * j + 4] * dhz_y);
                        ex[p] = fmaf(gm * cy[6 * j + 5], *ps, ex[p]);
                    }
                    if (cpml_e_in(nz, N, k)) {
                        ps = psi + PS_EXZ * g.n + p;
                        float dhy_z = hy[p] - hy[p - g.sz];
                        *ps = fmaf(cz[6 * k + 3], *ps, cz[6 * k + 4] * dhy_z);
                        ex[p] = fmaf(-(gm * cz[6 * k + 5]), *ps, ex[p]);
                    }
                }
                if (e_interior(&g, EY, i, j, k)) {
                    if (cpml_e_in(nz, N, k)) {
                        ps = psi + PS_EYZ * g.n + p;
                        float dhx_z = hx[p] - hx[p - g.sz];
                        *ps = fmaf(cz[6 * k + 3], *ps, cz[6 * k + 4] * dhx_z);
                        ey[p] = fmaf(gm * cz[6 * k + 5], *ps, ey[p]);
                    }
                    if (cpml_e_in(nx, N, i)) {
                        ps = psi + PS_EYX * g.n + p;
                        float dhz_x = hz[p] - hz[p - 1];
                        *ps = fmaf(cx[6 * i + 3], *ps, cx[6 * i + 4] * dhz_x);
                        ey[p] = fmaf(-(gm * cx[6 * i + 5]), *ps, ey[p]);
                    }
                }
                if (e_interior(&g, EZ, i, j, k)) {
                    if (cpml_e_in(nx, N, i)) {
                        ps = psi + PS_EZX * g.n + p;
                        float dhy_x = hy[p] - hy[p - 1];
                        *ps = fmaf(cx[6 * i + 3], *ps, cx[6 * i + 4] * dhy_x);
                        ez[p] = fmaf(gm * cx[6 * i + 5], *ps, ez[p]);
                    }
                    if (cpml_e_in(ny, N, j)) {
                        ps = psi + PS_EZY * g.n + p;
                        float dhx_y = hx[p] - hx[p - g.sy];
                        *ps = fmaf(cy[6 * j + 3], *ps, cy[6 * j + 4] * dhx_y);
                        ez[p] = fmaf(-(gm * cy[6 * j + 5]), *ps, ez[p]);
                    }
                }
            }
}

int orc_run_cpml_f64(int nx, int ny, int nz, int N, const double *hc, const double *cag, const double *ec,
                     const double *cp, const uint8_t *mat, double *f, double *psi, long step0, int n_steps,
                     int n_src, const int *src, const double *wave, int n_wave,
                     int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_graded_f64(nx, ny, nz, hc, f);
        cpml_h_f64(nx, ny, nz, N, cp, f, psi);
        orc_e_half_graded_f64(nx, ny, nz, cag, ec, mat, f);
        cpml_e_f64(nx, ny, nz, N, cp, cag, mat, f, psi);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])] += wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

int orc_run_cpml_f32(int nx, int ny, int nz, int N, const float *hc, const float *cag, const float *ec,
                     const float *cp, const uint8_t *mat, float *f, float *psi, long step0, int n_steps,
                     int n_src, const int *src, const float *wave, int n_wave,
                     int n_probe, const int *probe, double *probe_out)
{
    grid_t g = mkgrid(nx, ny, nz);
    if (check_points(&g, n_src, src, 1) || check_points(&g, n_probe, probe, 0)) return -1;
    for (int s = 0; s < n_steps; s++) {
        long n = step0 + s;
        orc_h_half_graded_f32(nx, ny, nz, hc, f);
        cpml_h_f32(nx, ny, nz, N, cp, f, psi);
        orc_e_half_graded_f32(nx, ny, nz, cag, ec, mat, f);
        cpml_e_f32(nx, ny, nz, N, cp, cag, mat, f, psi);
        for (int q = 0; q < n_src; q++) {
            if (n < n_wave) {
                const int *d = src + 4 * q;
                size_t p = (size_t)d[0] * g.n + at(&g, d[1], d[2], d[3]);
                f[p] = f[p] + wave[(size_t)q * n_wave + n];
            }
        }
        for (int q = 0; q < n_probe; q++) {
            const int *d = probe + 4 * q;
            probe_out[(size_t)s * n_probe + q] = (double)f[(size_t)d[0] * g.n + at(&g, d[1], d[2], d[3])];
        }
    }
    return 0;
}

/* Reduced-storage emulation on graded grids: the graded FP32 step, with the
 * state quantised at the same block ends as orc_run_q. */
int orc_run_q_graded(int nx, int ny, int nz, int fmt, int T, const float *hc, const float *cag, const float *ec,
                     const uint8_t *mat, float *f, long step0, int n_steps,
                     int n_src, const int *src, const float *wave, int n_wave,
                     int n_probe, const int *probe, double *probe_out,
                     float a_max, int *scales, float *m_stored, int *flag)
{
    for (int s = 0; s < n_steps; s++) {
        int rc = orc_run_graded_f32(nx, ny, nz, hc, cag, ec, mat, f, step0 + s, 1, n_src, src, wave, n_wave,
                                    n_probe, probe, probe_out + (size_t)s * n_probe);
        if (rc) return rc;
        long done = step0 + s + 1;
        if (done % T == 0 || s == n_steps - 1)
            orc_quantize_state(nx, ny, nz, fmt, 0, a_max, f, scales, m_stored, flag);
    }
    return 0;
}

/* Number of threads the parallel loops use (1 without OpenMP), and setting
 * it (timing only; results do not depend on it). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
