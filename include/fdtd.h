/*
 * fdtd.h -- C ABI of the MI355X (gfx950) Yee FDTD library.
 *
 * The library advances Maxwell's equations on a Cartesian Yee grid with the
 * explicit leapfrog of Cessenat, "Sophie, an FDTD code on the way to
 * multicore", Sec. 2.1: an H (Faraday) half-step from the curl of E, then an
 * E (Ampere) half-step from the curl of H, every coefficient one-dimensional
 * or table-sized (Sec. 2.2).  Materials enter through a per-cell uint8 index
 * into a small table (relative permittivity, conductivity); the outer walls
 * are perfect electric conductors (tangential E held at zero, Sec. 3.3);
 * sources are currents added to Ampere's law at pin points and probes read
 * single field values after every step (pin-point outputs, Sec. 3.4, 4.2).
 *
 * Grid and storage conventions
 * ----------------------------
 * nx, ny, nz cells of size dx, dy, dz (metres); time step dt (seconds).
 * Every component is addressed on the (nx+1)(ny+1)(nz+1) node box, x
 * fastest (index i + (nx+1)*(j + (ny+1)*k)); positions outside the
 * component's staggered range hold 0:
 *   Ex (i+1/2, j, k)      i<nx            Hx (i, j+1/2, k+1/2)  j<ny, k<nz
 *   Ey (i, j+1/2, k)      j<ny            Hy (i+1/2, j, k+1/2)  i<nx, k<nz
 *   Ez (i, j, k+1/2)      k<nz            Hz (i+1/2, j+1/2, k)  i<nx, j<ny
 * E is in V/m and H is stored as eta0*H (V/m), so both updates carry the
 * factor c*dt/delta of the antisymmetric form (Sec. 2.1).  The state after
 * n steps is (E^n, H^{n-1/2}).  Each interior E edge uses the material of
 * its owner cell, the cell whose lowest corner is the edge's lower end.
 *
 * Arithmetic: FP32 throughout, every update in a fixed fused-multiply-add
 * order (z-difference term, then y, cyclically), so results are
 * reproducible bit for bit and do not depend on the kernel variant, the
 * time-block length T or the tile shape when fields are stored in FP32.
 * Fields may instead be stored as binary16 or bfloat16 with one power-of-two
 * scale per component; they are then re-encoded at the end of every block
 * of T steps (blocks end at absolute step counts that are multiples of T and
 * at the end of each fdtd_step call), with the scale s_c = 10 -
 * ceil(log2 max(M_c, A)), M_c the largest stored |value| of the component at
 * the previous block's end and A the largest |source sample|.  A component
 * that would overflow the format at a block's end is instead encoded with
 * the scale of its own end-of-block maximum: the block runs again from its
 * input (still intact: fields ping-pong between two buffers), on the GPU,
 * without a host round trip.
 *
 * Ownership and errors
 * --------------------
 * Host inputs are copied during the call; the caller may free them on
 * return.  A caller-supplied device workspace stays owned by the caller and
 * must outlive fdtd_destroy.  The stream is never destroyed by the library.
 * Every function returns FDTD_OK (0) or a negative fdtd_status; output
 * arguments are written only on FDTD_OK.  fdtd_last_error() gives a
 * thread-local message for the last failure.  One host thread at a time may
 * use a given solver; different solvers may be used concurrently.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_solver fdtd_solver;

enum fdtd_status {
    FDTD_OK = 0,
    FDTD_EINVAL = -1,   /* bad argument: dimensions, index, component, range */
    FDTD_ENOMEM = -2,   /* device or host allocation failed, workspace too small */
    FDTD_EDEVICE = -3,  /* a HIP call or kernel launch failed */
    FDTD_ECFL = -4,     /* dt above the 3-D Courant limit */
    FDTD_ERANGE = -5,   /* reduced storage held a non-finite value, or a value beyond the format at any scale */
    FDTD_ESTATE = -6    /* call not allowed in the solver's current state */
};

enum fdtd_storage { FDTD_FP32 = 0, FDTD_FP16 = 1, FDTD_BF16 = 2 };

enum fdtd_component { FDTD_EX = 0, FDTD_EY = 1, FDTD_EZ = 2, FDTD_HX = 3, FDTD_HY = 4, FDTD_HZ = 5 };

/* Kernel families.  PLAIN: one in-place H pass then one in-place E pass per
 * step (the standard loop of Sec. 2.2; FP32 storage only).  FUSED: one pass
 * over HBM advances T steps, H and E interleaved plane by plane along z
 * with T time levels pipelined in registers (Sec. 3.2-3.4).  AUTO picks
 * FUSED, or PLAIN for grids whose z-planes are too large for the fused
 * kernel's chunk addressing (6 components x T+1 planes above 2 GiB; FP32
 * storage only -- fdtd_create rejects 16-bit storage for such grids). */
enum fdtd_kernel { FDTD_KERNEL_AUTO = 0, FDTD_KERNEL_PLAIN = 1, FDTD_KERNEL_FUSED = 2 };

/* A material.  sigma = +INFINITY makes a perfect electric conductor: the
 * coefficients of the three E edges each of its cells owns are Ca = Cb = 0,
 * so those edges are zero after every update (the loss term's limit taken
 * exactly), and fdtd_set_fields zeroes them.  Since a cell owns the edges at
 * its lowest corner, the faces of a conductor region that look towards lower
 * indices are exact staircase PEC walls (its lowest nodes hold tangential
 * E = 0): PEC cells filling i >= m (or j, k) leave exactly the cavity of the
 * cells below live.  On the faces that look towards higher indices the wall
 * lies one node inside the region, and the edges joining it to the region's
 * outer nodes are held at zero too.  A source on a PEC-owned edge is added
 * after that edge's update and cleared by the next one. */
typedef struct {
    double eps_r;   /* relative permittivity, > 0, finite */
    double mu_r;    /* relative permeability; must be 1 */
    double sigma;   /* conductivity in S/m, >= 0; +INFINITY = perfect conductor */
} fdtd_material;

/* Diagnostics of the current state (E^n, H^{n-1/2}), reduced in FP64 in a
 * fixed order (results do not depend on scheduling).
 *   energy  = 1/2 sum eps_r E^n.E^n + 1/2 sum H^{n-1/2}.H^{n+1/2}, in units of
 *             eps0*dx*dy*dz; conserved exactly by a lossless PEC box.  With
 *             graded spacing each term is weighted by its volume (edge
 *             length x dual face area for E, face area x dual edge length for
 *             H, dual sizes halved on the walls), in units of eps0 (m^3)
 *   div_e_* = div(eps_r E) at interior nodes; div_h_* = div(H) at cell
 *             centres (both in V/m^2; differences over the dual and the cell
 *             sizes): largest magnitude and sum of squares
 *   max_abs = largest |value| of each component */
typedef struct {
    double energy;
    double div_e_max, div_e_sumsq;
    double div_h_max, div_h_sumsq;
    double max_abs[6];
} fdtd_diag;

/* Device bytes fdtd_create needs for a caller-supplied workspace: two field
 * buffers (ping-pong: the fused passes read one time level and write the
 * other), the material index (the per-cell byte whose bandwidth Sec. 2.2
 * counts) and a small control block.  Probe rows, energy records, CPML psi
 * and diagnostics partials are allocated by the library on first use.
 * Returns 0 for invalid dimensions or storage. */
size_t fdtd_workspace_bytes(int nx, int ny, int nz, int storage);

/* Create a solver with all fields zero: the Yee scheme of Sec. 2.1 on a box
 * of nx x ny x nz cells with perfectly conducting walls, E on the cell edges
 * and H on the faces, one material per cell.
 *   nx, ny, nz    >= 2 cells each (and (nx+1)(ny+1) < 2^31)
 *   dx, dy, dz    > 0; dt > 0 and <= 1/(c sqrt(dx^-2+dy^-2+dz^-2)) (else FDTD_ECFL)
 *   table         n_materials entries (1..256), copied
 *   mat_index     host, nx*ny*nz bytes, x fastest (i + nx*(j + ny*k)); every
 *                 entry < n_materials (scanned; else FDTD_EINVAL); NULL = all 0
 *   storage       fdtd_storage; FP16/BF16 need z-planes small enough for the
 *                 fused kernel (6 (nx+1) (ny+1) 2 bytes x 4 planes < 2 GiB),
 *                 else FDTD_EINVAL
 *   device_workspace  NULL: the library allocates; else at least
 *                 fdtd_workspace_bytes(...) bytes of device memory, 256-byte
 *                 aligned, owned by the caller
 *   hip_stream    hipStream_t to enqueue on (NULL = the default stream) */
int fdtd_create(fdtd_solver **out, int nx, int ny, int nz,
                double dx, double dy, double dz, double dt,
                const fdtd_material *table, int n_materials,
                const uint8_t *mat_index, int storage,
                void *device_workspace, size_t workspace_bytes, void *hip_stream);

/* Graded spacing: per-index cell sizes (metres) dx[nx], dy[ny], dz[nz]
 * replace the uniform dx, dy, dz of fdtd_create.  The coefficients stay
 * one-dimensional, as in the loop of Sec. 2.2: the Faraday update of a face
 * uses c dt / (its cell sizes), and the Ampere update of an edge uses
 * c dt / (dual sizes), a dual size being the mean of the two cells that meet
 * at the node (Stokes' theorem on the dual face, Sec. 2.1).  Each E
 * coefficient is formed in FP32 as G * (c dt / dual size) with
 * G = (1/eps_r) / (1 + sigma dt / (2 eps0 eps_r)).
 *   Sizes > 0 and finite; dt must satisfy the Courant bound of the smallest
 *   size on each axis (else FDTD_ECFL; sufficient for such grids).  Any
 *   storage format (the PLAIN family needs FP32 storage as always); only
 *   before the first step (FDTD_ESTATE); may be called again to replace the
 *   sizes.  Arrays are copied.  Graded solvers run with fdtd_step (PLAIN or
 *   FUSED, any T);
 *   fdtd_step_batch rejects them (FDTD_EINVAL).  fdtd_diagnostics weights
 *   each term by its volume (see fdtd_diag). */
int fdtd_set_spacing(fdtd_solver *s, const double *dx, const double *dy, const double *dz);

/* CPML absorbing layers of `thickness` cells inside every face of the box
 * (0 removes them): the convolutional PML of Roden and Gedney that the paper
 * cites as its radiation condition (Sec. 3.3, Sec. 4.2), in its CFS form.
 * Every derivative d/du of the curl becomes (1/kappa_u) d/du + psi_u with
 * the recursion psi_u <- b_u psi_u + a_u (difference along u), kept only in
 * the layers; kappa is folded into the one-dimensional coefficients.  At
 * depth rho cells into a layer, x = rho / thickness:
 *   sigma = sigma_max x^order, kappa = 1 + (kappa_max - 1) x^order,
 *   alpha = alpha_max (1 - x)  (S/m),  sigma_max = sigma_factor
 *   0.8 (order + 1) / (eta0 d_out), d_out the outermost cell size of the face,
 *   b = exp(-(sigma/kappa + alpha) dt / eps0),
 *   a = sigma (b - 1) / (kappa (sigma + kappa alpha)).
 * H values at cell q (position q + 1/2) and E values at node q take their
 * depth from those positions.  After the (graded) update of a value in a
 * layer, its psi terms are added in the order of its update (Hx: z then y,
 * cyclically), each as psi = fmaf(b, psi, a * diff) then
 * value = fmaf(+-c dt / d, psi, value) -- times the material's G for E.
 *   thickness: 2 thickness < every one of nx, ny, nz; order 1..8;
 *   sigma_factor >= 0, kappa_max >= 1, alpha_max >= 0 (else FDTD_EINVAL).
 *   FP32 storage only; before the first step (FDTD_ESTATE); combines with
 *   fdtd_set_spacing in either order.  Both kernel families run the layers:
 *   the FUSED kernel carries the psi values of every time level through its
 *   pass (Sec. 3.3 counts absorbing layers among the per-cell work between
 *   the two half-steps, kept on one-dimensional coefficients so as not to add
 *   bandwidth) in blocks of at most 3 steps -- AUTO picks it with T = 2, the
 *   fastest; FUSED with a fixed T > 3 is rejected (FDTD_EINVAL), and so is
 *   psi state of 2 GiB or more, which the PLAIN family (and AUTO) still
 *   runs.  Conductor interiors are not skipped in solvers with layers.  The
 *   psi state starts at zero and is cleared by fdtd_set_fields.
 *   fdtd_step_batch and fdtd_diagnostics reject solvers with layers
 *   (FDTD_EINVAL). */
int fdtd_set_cpml(fdtd_solver *s, int thickness, int order, double sigma_factor, double kappa_max,
                  double alpha_max);

/* Kernel family (fdtd_kernel) and steps per HBM pass T for the FUSED family:
 * 1..6, or 0 = automatic (the default after fdtd_create): 4 for FP32
 * storage, 3 for FP16/BF16 storage and for graded spacing, 2 with CPML
 * layers, the fastest on MI355X, lowered for grids whose planes are too large
 * for that T (an automatic T is chosen again by fdtd_set_spacing and
 * fdtd_set_cpml).  T = 5 and 6 (deeper step gathering, Sec. 3.4 and the
 * conclusion) exceed the register file -- FP32 at T = 5 still runs faster
 * on some large grids (512^3) and slower on others -- and re-quantise 16-bit
 * storage less often; solvers with graded spacing and fdtd_step_batch take
 * T <= 4 (FDTD_EINVAL otherwise, also from fdtd_set_spacing on a solver with
 * a fixed T > 4), solvers with CPML layers T <= 3 with FUSED (AUTO caps its
 * blocks at 3 steps).  Allowed before the first step and between steps.
 * Results do not depend on T for FP32 storage; for FP16/BF16 storage, T sets
 * where values are re-quantised (every T steps).  fdtd_time_block reports
 * the T in use. */
int fdtd_set_kernel(fdtd_solver *s, int kernel, int time_block);

/* Zero-tile skipping of the FUSED kernel (enable != 0, the default after
 * fdtd_create); Sec. 4.2 leaves sub-domains whose fields are zero out of the
 * computation.  Two kinds of tiles are skipped:
 *  - The library tracks a node box holding every value that may differ from
 *    +0: the values fdtd_set_fields stored (or none), widened by one node per
 *    step on each axis -- the reach of the stencil -- plus the points of
 *    sources that still have samples.  A tile whose loaded region misses the
 *    box computes +0 exactly.  This saves time while a field is still
 *    spreading from its sources.
 *  - With perfect-conductor materials, a node is dead when its E edges are
 *    walls or owned by conductor cells (no source on them), its H values see
 *    only such edges, and its six stored values are +0 (as fdtd_set_fields or
 *    fdtd_load_state found them): it then stays +0 for good.  Tiles owning
 *    only dead nodes (conductor interiors) are not launched, for the whole
 *    run.  The map is made by fdtd_set_fields (and fdtd_create, with zero
 *    fields) and fdtd_load_state; fdtd_set_source wakes the nodes around its
 *    edge.  The first fused launch of each tile geometry lists the tiles and
 *    uploads the list (a small device allocation, kept until the map
 *    changes); batched steps skip them too.  Solvers with CPML layers run
 *    conductor interiors (their psi keeps following the curl next door).
 * Skipped tiles' probes record 0.  Results are bit-identical either way. */
int fdtd_set_zero_skip(fdtd_solver *s, int enable);

/* Fused-kernel tile counters since fdtd_create, summed over the fused
 * launches of fdtd_step and fdtd_step_batch: workgroups dispatched and
 * tiles of the full tiling.  Their ratio is the share of the
 * grid that ran once the zero-tile skip had its say (a listed tile that
 * misses the value box is dispatched and exits at once).  Host counters,
 * updated as steps are enqueued; no device call.  FDTD_EINVAL on NULL. */
int fdtd_tile_stats(const fdtd_solver *s, long long *dispatched, long long *full);

/* Debugging aid (enable != 0): before every FUSED launch, fill its output
 * buffer with NaN bit patterns, and launch every tile.  A launch that leaves
 * an owned value unwritten, or reads a neighbour from the buffer it writes,
 * then shows NaN in the results; correct code gives bit-identical results
 * either way.  Costs one buffer fill per launch.  Off by default. */
int fdtd_set_poison(fdtd_solver *s, int enable);

/* Tile shape of the FUSED kernel -- variant 0 = chosen per storage format and
 * T (default), 1..3 = the three rows-per-lane / waves-per-workgroup splits of
 * that T -- and planes per z chunk (0 = chosen from the grid): the sizes of
 * the sub-domains of Sec. 3.1.  Results do not depend on either; they only
 * change speed.  For tuning. */
int fdtd_set_tiling(fdtd_solver *s, int variant, int z_chunk);

/* Replace the whole state (the leapfrog's E^n and H^{n-1/2}, Sec. 2.1).
 * host: 6*(nx+1)*(ny+1)*(nz+1) floats, components
 * Ex, Ey, Ez, Hx, Hy, Hz one after another (E^n, then H^{n-1/2}); NULL sets
 * every field to zero.  Positions outside a component's range, tangential E
 * on the walls and E on edges owned by perfect-conductor cells are forced to
 * zero.  With reduced storage the
 * values are encoded here, with scales from their own maxima and from the
 * sources registered so far.  Synchronises the stream. */
int fdtd_set_fields(fdtd_solver *s, const float *host);

/* Add a soft source -- a current added to Ampere's equation, which Sec. 3.3
 * names among the work between the two half-steps: E_comp(i,j,k) +=
 * waveform[n] during step n (the step that produces E^{n+1}), for n <
 * n_samples; zero afterwards.  comp is an E
 * component and (i,j,k) must be an interior (non-PEC) edge.  waveform is
 * copied.  At most 256 sources per solver; several sources on one edge add
 * in index order.  *id receives the source index (0, 1, ...). */
int fdtd_set_source(fdtd_solver *s, int comp, int i, int j, int k,
                    const float *waveform, int n_samples, int *id);

/* Add a probe -- a pin-point output as in Sec. 3.4 and Sec. 4.2 -- of
 * component comp at storage position (i,j,k) (inside that component's
 * range).  After every step n (E^{n+1}, H^{n+1/2}) the value is
 * recorded in FP64.  Only allowed before the first step; at most 256 probes
 * per solver.  *id receives the probe index. */
int fdtd_set_probe(fdtd_solver *s, int comp, int i, int j, int k, int *id);

/* Enqueue n_steps >= 0 leapfrog steps (Sec. 2.1: the H half-step from curl
 * E, then the E half-step from curl H) on the solver's stream and return
 * without waiting.  The FUSED kernel advances T steps per pass over the
 * fields (Sec. 3.2-3.4), the PLAIN one a step per pair of passes (Sec. 2.2).
 * Saturation of reduced storage is reported by fdtd_synchronize. */
int fdtd_step(fdtd_solver *s, int n_steps);

/* Advance several solvers at once (continuous batching for serving; the
 * paper runs one problem at a time): n_steps[i] (>= 0) steps for solvers[i],
 * count >= 0, every solver distinct, all created on the same stream, none
 * set to the PLAIN kernel and none with planes too large for the FUSED one
 * (else FDTD_EINVAL).  Each block (up to T steps, ending on multiples of
 * T) is issued as one persistent launch over the tiles of up to 12 solvers
 * that share storage format, block length and tile shape, so small grids
 * share the GPU instead of each under-filling it.  Results are bit-identical
 * to fdtd_step on each solver alone.  Enqueues only (continuous batching:
 * solvers may join or leave between calls). */
int fdtd_step_batch(fdtd_solver *const *solvers, int count, const int *n_steps);

/* Bind the solver to another stream (caller-owned; NULL = the default
 * stream) after the work enqueued on its current stream has finished.  A
 * serving loop creates solvers on a side stream, so that uploads do not wait
 * for the running batch, and then moves them to the batch stream (batched
 * solvers must share one).  FDTD_EINVAL on NULL solver. */
int fdtd_set_stream(fdtd_solver *s, void *hip_stream);

/* Copy one component of the current state (E^n or H^{n-1/2}, Sec. 2.1) to host (float,
 * (nx+1)(ny+1)(nz+1), x fastest; decoded if stored in reduced precision).
 * Synchronises the stream. */
int fdtd_read_fields(fdtd_solver *s, int comp, float *host_dst);

/* Copy probe records for steps [first_step, first_step+n_steps) to host_dst
 * as n_steps rows of n_probes doubles (row = step, column = probe id), the
 * pin-point outputs of Sec. 3.4 and 4.2.  The steps must have been run.
 * Waits for the solver's own enqueued steps only, not for work enqueued on
 * the same stream afterwards (other solvers' next batch keeps the GPU busy
 * meanwhile), and copies on a stream of the library's own. */
int fdtd_read_probes(fdtd_solver *s, double *host_dst, long long first_step, int n_steps);

/* Allocate the probe rows (and energy records) of the first total_steps
 * steps now, so that fdtd_step up to that count allocates nothing and never
 * synchronises the stream; otherwise fdtd_step grows them by doubling, each
 * time with hipMalloc and a wait for the solver's stream.  A serving loop
 * calls it when it admits a request, on the stream the solver was created
 * on.  After the probes (fdtd_set_probe discards the rows) and the energy
 * trace are set.  FDTD_EINVAL for a negative count, FDTD_EDEVICE if the
 * memory cannot be allocated. */
int fdtd_reserve_steps(fdtd_solver *s, long long total_steps);

/* Energy trace: record k is the discrete energy W^n of the state n =
 * k * every (fdtd_diag's energy: 1/2 sum eps_r E^n.E^n + 1/2 sum
 * H^(n-1/2).H^(n+1/2), the quantity the leapfrog conserves by the
 * antisymmetry of its two half-steps, Sec. 2.1), written when a step starts
 * from that state.  The FUSED kernel forms it inside the pass, in the
 * Faraday half-step of the time level that takes state n -- E^n and
 * H^(n-1/2) are that level's inputs, H^(n+1/2) its result -- as FP64
 * products summed per tile (wave butterflies, then the waves in order) and
 * the tiles' sums added in tile order: the same value on every run of the
 * same launch sequence, equal to fdtd_diagnostics' energy up to the order
 * of the FP64 sums.  The PLAIN kernels take it with the diagnostics pass.
 *   every: 1.. (0 turns the trace off); before the first step (FDTD_ESTATE);
 *   uniform spacing and no CPML layers (FDTD_EINVAL, also from fdtd_step
 *   when spacing or layers are set afterwards); fused blocks of at most 4
 *   steps; with FP16/BF16 storage every >= T (a block holds at most one
 *   recorded state), with FP32 storage a block ends before a second one.
 *   fdtd_step_batch rejects solvers with a trace (FDTD_EINVAL).  The records
 *   of states from a restored step on are unwritten again after
 *   fdtd_load_state.  Memory: one double per record and one per tile of a
 *   launch, allocated here and by fdtd_step. */
int fdtd_set_energy_trace(fdtd_solver *s, int every);

/* Copy energy records [first_record, first_record + n_records) to host_dst
 * (record k: the state k * every).  Records of states no step has started
 * from are rejected (FDTD_EINVAL), and so is a solver without a trace.
 * Waits for the solver's own enqueued steps only, like fdtd_read_probes. */
int fdtd_read_energy(fdtd_solver *s, double *host_dst, long long first_record, int n_records);

/* Compute diagnostics of the current state (fdtd_diag; the energy is the
 * quantity the leapfrog conserves by the antisymmetry of its two half-steps,
 * Sec. 2.1).  FDTD_EINVAL with CPML layers.  The first call allocates the
 * block partials (kept until fdtd_destroy).  Synchronises the stream. */
int fdtd_diagnostics(fdtd_solver *s, fdtd_diag *out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * same diagnostics, bit for bit, with the block partials and the reduced
 * values in a static device array of 4 MiB that the library holds once per
 * GPU until the process ends, instead of memory allocated per solver.  No
 * device memory is allocated or freed.  Grids whose diagnostics need more
 * block partials than the array holds (about 47 000: one per 64 x 4 nodes of
 * a plane, times min(8, nz+1) plane runs -- e.g. planes up to about
 * 1500 x 1000 nodes) are rejected with FDTD_EINVAL before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (several host threads, or solvers on different streams still running)
 * race and may return each other's values.  Call with the solver's device
 * current.  Synchronises the stream. */
int fdtd_diagnostics_noalloc(fdtd_solver *s, fdtd_diag *out);

/* Number of steps enqueued so far. */
int fdtd_steps_done(const fdtd_solver *s, long long *n);

/* Steps per launch of the next fdtd_step: the FUSED kernel's T as chosen
 * (automatic or fixed; with CPML layers at most 3), 1 when the PLAIN
 * kernels run.  FDTD_EINVAL on NULL. */
int fdtd_time_block(const fdtd_solver *s, int *T);

/* Choose T by measurement (Sec. 3.4 gathers steps per pass; which count is
 * fastest depends on the grid's tile count as much as on the blocking): for
 * each of T = 3, 4, 5 the solver runs one untimed block, then the largest
 * multiple of T up to n_steps (>= 1) timed with HIP events on its stream,
 * every launch with the zero-tile skip off; it keeps the fastest T as a
 * fixed T (fdtd_set_kernel) and writes it to *chosen, and the per-step
 * times in ns to ns_per_step[0..2] (NULL: not wanted; 0 for a T the grid's
 * planes do not allow).  The solver advances by all these steps, at most
 * 3 n_steps + 12: FP32 results do not depend on T, so they are the steps of
 * any T.  Synchronises the stream.  Only for FP32 storage with uniform
 * spacing, no CPML layers, no energy trace and the fused kernel
 * (FDTD_EINVAL otherwise).  Measure where the field fills the grid: early
 * steps from zero fields run little work anyway. */
int fdtd_tune_time_block(fdtd_solver *s, int n_steps, int *chosen, double *ns_per_step);

/* Checkpoint and resume.  fdtd_save_state copies the whole evolving state
 * to host memory: the fields exactly as stored (reduced storage included),
 * the storage scales and saturation flag, the CPML psi state, the step count
 * and the zero-tile box.  fdtd_load_state restores it into a solver created
 * with the same grid, storage, CPML layers, spacing, materials, sources and
 * probes (grid, storage and layers are checked; FDTD_EINVAL otherwise), which
 * then continues bit-identically to the saved solver.  Probe records before
 * the restored step are not part of the state (a fresh restoring solver
 * reads them as 0).  host_dst / host_src hold at least fdtd_state_bytes(s)
 * bytes (0 for a NULL solver); both calls synchronise the stream. */
size_t fdtd_state_bytes(const fdtd_solver *s);
int fdtd_save_state(fdtd_solver *s, void *host_dst, size_t bytes);
int fdtd_load_state(fdtd_solver *s, const void *host_src, size_t bytes);

/* Current per-component storage scales (2^scale multiplies a value before
 * encoding; all 0 for FP32 storage) and the sticky flag of FDTD_ERANGE (a
 * non-finite value stored, or a value beyond the format even at the scale
 * its overflow retry chose, stored saturated).  Synchronises. */
int fdtd_storage_state(fdtd_solver *s, int scales[6], int *saturated);

/* Wait for all work enqueued on the solver's stream; reports FDTD_ERANGE when
 * reduced storage raised its flag (see fdtd_storage_state). */
int fdtd_synchronize(fdtd_solver *s);

/* Release the solver and everything the library allocated for it, after its
 * own enqueued work has finished. */
void fdtd_destroy(fdtd_solver *s);

/* Message for the last failed call on this thread ("" if none). */
const char *fdtd_last_error(void);

/* FP32 coefficients the library derives from a material table: out gets
 * n_materials x {Ca, Cbx, Cby, Cbz} and ch gets {c dt/dx, c dt/dy, c dt/dz}.
 * Host-only; no device is needed. */
int fdtd_coefficients(const fdtd_material *table, int n_materials,
                      double dx, double dy, double dz, double dt,
                      float *out, float *ch);

/* FP32 coefficients of graded spacing (see fdtd_set_spacing): cag gets
 * n_materials x {Ca, G}; gc gets, per node index of x (nx+1 entries), then
 * y (ny+1), then z (nz+1), the pair {c dt / d[q] (0 at q = n),
 * c dt / ((d[q-1] + d[q]) / 2) (0 at q = 0 and q = n)}, each rounded once
 * from FP64.  Host-only; no device is needed. */
int fdtd_graded_coefficients(const fdtd_material *table, int n_materials, int nx, int ny, int nz,
                             const double *dx, const double *dy, const double *dz, double dt,
                             float *cag, float *gc);

/* Host only (no device, no solver): the live-node map the zero-tile skip
 * uses for perfect conductors, for a state whose stored values are all +0.
 * A node (i, j, k) of the (nx+1)(ny+1)(nz+1) box is dead (live[...] = 0)
 * when its three E edges are walls or owned by cells whose material has
 * sigma = +INFINITY, with no source on them, and each of its in-range H
 * values (Hx from Ez at j, j+1 and Ey at k, k+1; Hy from Ex at k, k+1 and Ez
 * at i, i+1; Hz from Ey at i, i+1 and Ex at j, j+1) sees only such edges:
 * every update then leaves its six values at +0.  mat_index: nx*ny*nz cell
 * indices, x fastest; sources: n_sources x (comp, i, j, k), interior E edges
 * (a source wakes the nodes {i-1, i} x {j-1, j} x {k-1, k}); live: output,
 * (nx+1)(ny+1)(nz+1) bytes, x fastest, 1 = live.  FDTD_EINVAL on NULL
 * arguments, bad sizes, indices >= n_materials or a source off the interior
 * E edges. */
int fdtd_live_nodes(const fdtd_material *table, int n_materials, const uint8_t *mat_index, int nx, int ny, int nz,
                    const int *sources, int n_sources, uint8_t *live);

/* FP32 tables of CPML layers over graded spacing (see fdtd_set_cpml): cag
 * and gc as fdtd_graded_coefficients but with kappa folded into gc
 * (c dt / (kappa d)); cp gets, per node index of x, then y, then z, the six
 * values {b_h, a_h, c dt / d[q], b_e, a_e, c dt / d'[q]} of the H value at
 * cell q and the E value at node q (b and a zero outside the layers), each
 * rounded once from FP64.  Host-only; no device is needed. */
int fdtd_cpml_coefficients(const fdtd_material *table, int n_materials, int nx, int ny, int nz,
                           const double *dx, const double *dy, const double *dz, double dt,
                           int thickness, int order, double sigma_factor, double kappa_max, double alpha_max,
                           float *cag, float *gc, float *cp);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
