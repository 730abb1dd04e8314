"""Seeded synthetic workloads for the Yee FDTD solver.

This module only *generates inputs*: material tables, per-cell material
indices, source positions and waveforms, probe positions and initial
fields.  It contains none of the update arithmetic, so both the CPU
oracle (test infrastructure) and the GPU path can consume its output.

The paper measures synthetic N^3 cubes and cavity cases (a PEC box with a
point current and a few pin-point outputs; Sec. 4.1, Sec. 4.2).  The
workloads below stand in for those cases with the shapes, sizes and
structure of the configurations this library is benchmarked on:

* ``cavity32``  -- 32^3 vacuum PEC box, analytic TM110 mode plus noise.
* ``spheres256`` -- 256^3, 16-entry dielectric table, 40 random spheres,
  Ez soft source at the centre, 16 probes, 1000 steps.
* ``spheres512`` -- 512^3, 200 spheres, three sources (Ex, Ey, Ez).
* ``precision512``, ``precision1024`` -- 512^3 and 1024x512x256, the
  ``spheres512`` recipe with 16-bit storage, 2000 steps.
* ``cavity402`` -- the paper's case C: an empty 402^3 PEC cavity with a
  pin-point current.
* ``serving``   -- 256 requests with random anisotropic grids.
* ``graded256`` -- 256^3 with graded cell sizes (fine core, geometric growth
  to coarse cells near the walls), otherwise as ``spheres256``.
* ``open256``   -- ``spheres256`` in open space: 10-cell CPML layers on
  every face instead of reflecting walls.
* ``sphere402`` -- the paper's case S: a spherical PEC cavity of 400 cells
  diameter in a 402^3 box, a pin-point current inside.

All randomness comes from splitmix64 (Steele, Lea, Flood 2014), drawn in a
fixed order: material table, spheres (cx, cy, cz, radius, index), sources,
probes, noise.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

C0 = 299792458.0            # speed of light in vacuum, m/s
COMP_NAMES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
EX, EY, EZ, HX, HY, HZ = range(6)
FP32, FP16, BF16 = 0, 1, 2
STORAGE_NAMES = {FP32: "fp32", FP16: "fp16", BF16: "bf16"}

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 generator; scalar draws and vectorised continuation."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    @staticmethod
    def _mix(z: int) -> int:
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        return self._mix(self.state)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        u = (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in the closed range [lo, hi]."""
        u = (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)
        return lo + min(int(u * (hi - lo + 1)), hi - lo)

    def uniform_array(self, n: int, lo: float, hi: float) -> np.ndarray:
        """The next n draws as uniforms in [lo, hi) (same stream as uniform())."""
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * _GAMMA
            z = (z ^ (z >> np.uint64(30))) * _M1
            z = (z ^ (z >> np.uint64(27))) * _M2
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * 0x9E3779B97F4A7C15) & _MASK64
        u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u


def courant_dt(dx: float, dy: float, dz: float, frac: float = 0.99) -> float:
    """frac times the 3-D Courant limit 1/(c*sqrt(dx^-2+dy^-2+dz^-2))."""
    return frac / (C0 * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2))


def gaussian_sine(n: int, dt: float, dx: float, amplitude: float = 1.0) -> np.ndarray:
    """Gaussian-modulated sinusoid sampled at t=(n+1/2)dt, in float64.

    f0 = c/(20 dx) (20 cells per vacuum wavelength), tau = 1/f0, t0 = 4 tau.
    """
    f0 = C0 / (20.0 * dx)
    tau = 1.0 / f0
    t0 = 4.0 * tau
    t = (np.arange(n, dtype=np.float64) + 0.5) * dt
    return amplitude * np.exp(-((t - t0) / tau) ** 2) * np.sin(2.0 * math.pi * f0 * (t - t0))


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float
    eps_r: np.ndarray            # (n_mat,) float64
    mu_r: np.ndarray             # (n_mat,) float64 (all 1)
    sigma: np.ndarray            # (n_mat,) float64, S/m
    mat: np.ndarray              # (nz, ny, nx) uint8 cell material index
    sources: List[Tuple[int, int, int, int]]   # (comp, i, j, k)
    waveforms: np.ndarray        # (n_src, n_wave) float64
    probes: List[Tuple[int, int, int, int]]    # (comp, i, j, k)
    n_steps: int
    init_fields: Optional[np.ndarray] = None   # (6, nz+1, ny+1, nx+1) float64
    storage: int = FP32
    # graded spacing: per-index cell sizes (dx (nx,), dy (ny,), dz (nz,)) in
    # metres; None = uniform dx, dy, dz
    spacing: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None
    # CPML absorbing layers: dict(thickness, order, sigma_factor, kappa_max,
    # alpha_max); None = PEC walls only
    cpml: Optional[dict] = None

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def box_shape(self) -> Tuple[int, int, int]:
        return (self.nz + 1, self.ny + 1, self.nx + 1)


def material_table(rng: SplitMix64, n_mat: int = 16):
    """Entry 0 is vacuum; entries 1..n-1: eps_r U[1,12], sigma U[0,0.05] S/m, mu_r=1."""
    eps = np.ones(n_mat)
    sig = np.zeros(n_mat)
    for m in range(1, n_mat):
        eps[m] = rng.uniform(1.0, 12.0)
        sig[m] = rng.uniform(0.0, 0.05)
    return eps, np.ones(n_mat), sig


def paint_spheres(rng: SplitMix64, nx: int, ny: int, nz: int, n_spheres: int,
                  rmin: int, rmax: int, n_mat: int) -> np.ndarray:
    """Cell material index array; later spheres overwrite earlier ones.

    A cell (i,j,k) is inside when its centre (i+1/2, j+1/2, k+1/2) lies within
    radius r of the sphere centre.
    """
    mat = np.zeros((nz, ny, nx), dtype=np.uint8)
    for _ in range(n_spheres):
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        cz = rng.uniform(0.0, nz)
        r = rng.randint(rmin, rmax)
        idx = rng.randint(1, n_mat - 1)
        i0, i1 = max(0, int(math.floor(cx - r - 1))), min(nx, int(math.ceil(cx + r + 1)))
        j0, j1 = max(0, int(math.floor(cy - r - 1))), min(ny, int(math.ceil(cy + r + 1)))
        k0, k1 = max(0, int(math.floor(cz - r - 1))), min(nz, int(math.ceil(cz + r + 1)))
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        zi = (np.arange(k0, k1) + 0.5 - cz)[:, None, None]
        yi = (np.arange(j0, j1) + 0.5 - cy)[None, :, None]
        xi = (np.arange(i0, i1) + 0.5 - cx)[None, None, :]
        inside = (xi * xi + yi * yi + zi * zi) <= float(r * r)
        sub = mat[k0:k1, j0:j1, i0:i1]
        sub[inside] = idx
    return mat


_PROBE_CYCLE = (EZ, HX, HY, EX, EY, HZ)


def seeded_probes(rng: SplitMix64, nx: int, ny: int, nz: int, n: int):
    """n probes at interior positions; components cycle Ez, Hx, Hy, Ex, Ey, Hz."""
    out = []
    for p in range(n):
        i = rng.randint(1, nx - 2)
        j = rng.randint(1, ny - 2)
        k = rng.randint(1, nz - 2)
        out.append((_PROBE_CYCLE[p % 6], i, j, k))
    return out


def interior_e_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """(3, nz+1, ny+1, nx+1) bool: E edges not tangential to the PEC walls."""
    m = np.zeros((3, nz + 1, ny + 1, nx + 1), dtype=bool)
    m[0, 1:nz, 1:ny, 0:nx] = True
    m[1, 1:nz, 0:ny, 1:nx] = True
    m[2, 0:nz, 1:ny, 1:nx] = True
    return m


def tm110_state(nx: int, ny: int, nz: int, dx: float, dy: float, dz: float, dt: float) -> np.ndarray:
    """Closed-form discrete TM110 cavity mode, amplitude 1 (float64).

    E^0_z(i,j,k) = sin(pi i/nx) sin(pi j/ny); other E components are 0.
    H^{-1/2} is the mode's magnetic part half a time step back, chosen so
    that H^{+1/2} = -H^{-1/2} (the mode is then advanced at its exact
    discrete frequency):
        eta0 Hx(i, j+1/2) =  (c dt / dy) sin(pi/(2 ny)) cos(pi (j+1/2)/ny) sin(pi i/nx)
        eta0 Hy(i+1/2, j) = -(c dt / dx) sin(pi/(2 nx)) cos(pi (i+1/2)/nx) sin(pi j/ny)
    -- analytic expressions of the mode (each equals the difference of the
    two neighbouring sines by the sum-to-product identity), so no update of
    the scheme is evaluated here.  H is stored as eta0*H, in V/m.
    """
    f = np.zeros((6, nz + 1, ny + 1, nx + 1))
    si = np.sin(math.pi * np.arange(nx + 1) / nx)
    sj = np.sin(math.pi * np.arange(ny + 1) / ny)
    f[EZ, 0:nz, :, :] = sj[None, :, None] * si[None, None, :]
    cj = np.cos(math.pi * (np.arange(ny) + 0.5) / ny)       # j + 1/2, j in [0, ny)
    ci = np.cos(math.pi * (np.arange(nx) + 0.5) / nx)       # i + 1/2, i in [0, nx)
    ax = C0 * dt / dy * math.sin(math.pi / (2 * ny))
    ay = C0 * dt / dx * math.sin(math.pi / (2 * nx))
    f[HX, 0:nz, 0:ny, :] = ax * cj[None, :, None] * si[None, None, :]
    f[HY, 0:nz, :, 0:nx] = -ay * sj[None, :, None] * ci[None, None, :]
    return f


def cavity32(seed: int = 1000, n: int = 32, n_steps: int = 100, noise: float = 1e-4) -> Workload:
    """32^3 vacuum PEC box, TM110 mode plus seeded noise on interior E, 4 probes."""
    nx = ny = nz = n
    d = 1e-3
    dt = courant_dt(d, d, d)
    rng = SplitMix64(seed)
    probes = seeded_probes(rng, nx, ny, nz, 4)
    f = tm110_state(nx, ny, nz, d, d, d, dt)
    mask = interior_e_mask(nx, ny, nz)
    cnt = int(mask.sum())
    f[0:3][mask] += rng.uniform_array(cnt, -noise, noise)
    return Workload("cavity32", nx, ny, nz, d, d, d, dt,
                    np.ones(1), np.ones(1), np.zeros(1),
                    np.zeros((nz, ny, nx), np.uint8), [], np.zeros((0, n_steps)),
                    probes, n_steps, init_fields=f)


def spheres(nx: int, ny: int, nz: int, n_spheres: int, n_steps: int, seed: int,
            n_sources: int = 1, n_probes: int = 16, rmin: int = 8, rmax: int = 40,
            name: str = "spheres", storage: int = FP32, d: float = 1e-3) -> Workload:
    """Dielectric-scatterer cavity: 16-entry table, random spheres, soft sources.

    n_sources == 1: an Ez source at the grid centre.  n_sources == 3: Ex, Ey
    and Ez sources at seeded edges at least 16 cells (or a quarter of the
    grid, if smaller) from every wall.
    """
    dt = courant_dt(d, d, d)
    rng = SplitMix64(seed)
    eps, mu, sig = material_table(rng, 16)
    mat = paint_spheres(rng, nx, ny, nz, n_spheres, rmin, rmax, 16)
    srcs = []
    if n_sources == 1:
        srcs.append((EZ, nx // 2, ny // 2, nz // 2))
    else:
        for s in range(n_sources):
            m = [max(1, min(16, n // 4)) for n in (nx, ny, nz)]
            i = rng.randint(m[0], nx - m[0])
            j = rng.randint(m[1], ny - m[1])
            k = rng.randint(m[2], nz - m[2])
            srcs.append(((EX, EY, EZ)[s % 3], i, j, k))
    w = gaussian_sine(n_steps, dt, d)
    waves = np.tile(w, (len(srcs), 1))
    probes = seeded_probes(rng, nx, ny, nz, n_probes)
    return Workload(name, nx, ny, nz, d, d, d, dt, eps, mu, sig, mat, srcs, waves,
                    probes, n_steps, storage=storage)


def spheres256(n_steps: int = 1000) -> Workload:
    return spheres(256, 256, 256, 40, n_steps, seed=1001, n_sources=1, name="spheres256")


def spheres512(n_steps: int = 500) -> Workload:
    return spheres(512, 512, 512, 200, n_steps, seed=1002, n_sources=3, name="spheres512")


def precision512(storage: int, n_steps: int = 2000) -> Workload:
    return spheres(512, 512, 512, 200, n_steps, seed=1003, n_sources=3,
                   name="precision512", storage=storage)


def precision1024(storage: int, n_steps: int = 2000) -> Workload:
    return spheres(1024, 512, 256, 200, n_steps, seed=1003, n_sources=3,
                   name="precision1024x512x256", storage=storage)


def cavity402(n_steps: int = 1300, seed: int = 1005, storage: int = FP32) -> Workload:
    """The paper's production case C (Sec. 4.2): an empty 402^3 cavity with PEC
    walls, driven by a current at a pin point, 1300 steps, 6 outputs.

    Readings: the pin point is unplaced in the paper -- here a seeded interior
    Ez edge at least 50 cells from every wall, with the Gaussian-modulated sine
    of the other workloads; the 6 outputs are seeded probes recorded at every
    step (the paper records every 20th).  Vacuum everywhere (one material).
    """
    n = 402
    d = 1e-3
    dt = courant_dt(d, d, d)
    rng = SplitMix64(seed)
    eps, mu, sig = np.ones(1), np.ones(1), np.zeros(1)
    mat = np.zeros((n, n, n), np.uint8)
    i, j, k = (rng.randint(50, n - 50) for _ in range(3))
    srcs = [(EZ, i, j, k)]
    waves = gaussian_sine(n_steps, dt, d)[None, :]
    probes = seeded_probes(rng, n, n, n, 6)
    return Workload("cavity402", n, n, n, d, d, d, dt, eps, mu, sig, mat, srcs, waves, probes, n_steps,
                    storage=storage)


def graded_sizes(n: int, d_fine: float, d_coarse: float, ratio: float, core: int) -> np.ndarray:
    """Cell sizes along one axis: d_fine over the central `core` cells, growing
    by `ratio` per cell outwards until d_coarse, then constant."""
    q = np.arange(n) + 0.5 - n / 2.0
    steps = np.maximum(0.0, np.abs(q) - core / 2.0)
    return np.minimum(d_fine * ratio ** np.ceil(steps), d_coarse)


def courant_dt_graded(sx: np.ndarray, sy: np.ndarray, sz: np.ndarray, frac: float = 0.99) -> float:
    """frac times the Courant bound of the smallest cell size on each axis."""
    return courant_dt(float(sx.min()), float(sy.min()), float(sz.min()), frac)


def graded(n: int, n_spheres: int, n_steps: int, seed: int, d_fine: float = 0.5e-3,
           d_coarse: float = 2e-3, ratio: float = 1.05, core: int = 64, name: str = "graded") -> Workload:
    """The spheres recipe (spheres painted in index space) on a graded grid: fine
    cells around the centre, where the Ez source sits, coarse cells near the
    walls.  dt from the smallest cells; the waveform has 20 coarse cells per
    vacuum wavelength."""
    sz = graded_sizes(n, d_fine, d_coarse, ratio, core)
    wl = spheres(n, n, n, n_spheres, n_steps, seed=seed, n_sources=1, name=name)
    wl.dt = courant_dt_graded(sz, sz, sz)
    wl.dx = wl.dy = wl.dz = d_coarse
    wl.waveforms = np.tile(gaussian_sine(n_steps, wl.dt, d_coarse), (len(wl.sources), 1))
    wl.spacing = (sz.copy(), sz.copy(), sz.copy())
    return wl


def graded256(n_steps: int = 1000) -> Workload:
    return graded(256, 40, n_steps, seed=1006, name="graded256")


def sphere402(n_steps: int = 1300, seed: int = 1007, storage: int = FP32) -> Workload:
    """The paper's production case S (Sec. 4.2): a sphere of 400 cells
    diameter inside a 402^3 box, the field inside it, driven by a current at
    a pin point, 1300 steps, 6 outputs.

    Readings: the sphere is a perfect conductor enclosing the field (a cell is
    conductor when its centre lies farther than 200 cells from the box centre);
    the pin point is a seeded interior Ez edge at least 50 cells inside the
    sphere, with the Gaussian-modulated sine of the other workloads; the 6
    outputs are seeded probes inside the sphere, recorded at every step.
    """
    n, d = 402, 1e-3
    dt = courant_dt(d, d, d)
    rng = SplitMix64(seed)
    c, r = n / 2.0, 200.0
    mat = np.zeros((n, n, n), np.uint8)
    ax = np.arange(n) + 0.5 - c
    yx = ax[:, None] ** 2 + ax[None, :] ** 2
    for k in range(n):
        mat[k][yx + ax[k] ** 2 > r * r] = 1
    def inside(lo):
        while True:
            p = tuple(rng.randint(lo, n - lo) for _ in range(3))
            if sum((q + 0.5 - c) ** 2 for q in p) < (r - 50.0) ** 2:
                return p
    i, j, k = inside(60)
    srcs = [(EZ, i, j, k)]
    waves = gaussian_sine(n_steps, dt, d)[None, :]
    probes = []
    for q in range(6):
        pi, pj, pk = inside(20)
        probes.append((_PROBE_CYCLE[q % 6], pi, pj, pk))
    return Workload("sphere402", n, n, n, d, d, d, dt, np.ones(2), np.ones(2), np.array([0.0, np.inf]), mat,
                    srcs, waves, probes, n_steps, storage=storage)


CPML_LAYER = dict(thickness=10, order=3, sigma_factor=1.0, kappa_max=5.0, alpha_max=0.05)


def open256(n_steps: int = 1000) -> Workload:
    """spheres256 radiating into open space: CPML layers on every face."""
    wl = spheres(256, 256, 256, 40, n_steps, seed=1001, n_sources=1, name="open256")
    wl.cpml = dict(CPML_LAYER)
    return wl


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float               # seconds from the start of the run
    nx: int
    ny: int
    nz: int
    n_spheres: int
    n_steps: int
    storage: int

    def workload(self) -> Workload:
        wl = spheres(self.nx, self.ny, self.nz, self.n_spheres, self.n_steps,
                     seed=(1004 << 20) + self.rid, n_sources=1, n_probes=8,
                     rmin=min(8, max(1, min(self.nx, self.ny, self.nz) // 8)),
                     rmax=min(40, max(2, min(self.nx, self.ny, self.nz) // 4)),
                     name=f"req{self.rid}", storage=self.storage)
        return wl


def serving_requests(n: int = 256, rate: float = 8.0, seed: int = 1004,
                     dim_lo: int = 48, dim_hi: int = 320,
                     steps_lo: int = 200, steps_hi: int = 3000) -> List[Request]:
    """Poisson arrivals at `rate` req/s; dims, sphere counts, steps, storage seeded."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for r in range(n):
        nx, ny, nz = (rng.randint(dim_lo, dim_hi) for _ in range(3))
        ns = rng.randint(5, 60)
        steps = rng.randint(steps_lo, steps_hi)
        storage = FP16 if rng.uniform() < 0.5 else FP32
        t += -math.log(1.0 - rng.uniform()) / rate
        out.append(Request(r, t, nx, ny, nz, ns, steps, storage))
    return out


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a-b||_2/||b||_2 with float64 accumulation (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.sqrt(np.sum(b * b)))
    return float(np.sqrt(np.sum((a - b) ** 2))) / den if den > 0 else float(np.sqrt(np.sum(a * a)))
