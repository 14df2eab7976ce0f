"""Seeded synthetic inputs for the embedded-ROM FDTD solver.

This module is shared by the CPU oracle and by the GPU library's tests and
benchmark.  It only *describes* problems: grid sizes, cell sizes, time step,
per-cell material maps, reduced-region footprints with their fine-cell
material, source waveforms (additive increments per step), probe positions
and step counts.  It performs none of the method's arithmetic (no update
coefficients, no reduced models, no coupling).

The paper (Zhang, Bekmambetova, Triverio, "A Stable FDTD Method with Embedded
Reduced-Order Models") runs a 2D TEz PEC cavity (Sec. VI-A), a waveguide with
irises (Sec. VI-B) and a rod reflection test (Sec. VI-C) excited by Gaussian
pulses of stated bandwidth.  The configurations below are synthetic,
seeded stand-ins of those workloads scaled to GPU size; every random draw
comes from ``numpy.random.default_rng`` with a fixed seed.

Index conventions (shared vocabulary, not arithmetic):
  * coarse cell (i, j): x in [i*dx, (i+1)*dx), y in [j*dy, (j+1)*dy);
    i < nx, j < ny.  Maps are arrays indexed [j, i].
  * Hz(i, j) sits at the cell centre; Ex(i, j) on the horizontal edge
    y = j*dy (south edge of cell (i, j)); Ey(i, j) on the vertical edge
    x = i*dx (west edge of cell (i, j)).
  * A reduced region covers coarse cells [i0, i0+ni) x [j0, j0+nj) and is
    refined by an integer factor r; its fine material maps are indexed
    [jf, if] with jf < r*nj, if < r*ni.
  * A source adds ``incr[n]`` at step n to one field component over a
    rectangle of positions [i0, i1) x [j0, j1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Physical constants used only to turn a Courant fraction into a time step
# (an input of the problem) and to place source pulses in time.
_C0 = 299792458.0

HZ, EX, EY = 0, 1, 2
COMP_NAMES = {HZ: "Hz", EX: "Ex", EY: "Ey"}


@dataclasses.dataclass
class Source:
    comp: int
    i0: int
    i1: int
    j0: int
    j1: int
    incr: np.ndarray  # float64 [nsteps]: value added at step n


@dataclasses.dataclass
class Probe:
    comp: int
    i: int
    j: int


@dataclasses.dataclass
class RomSpec:
    """A refined region replaced by a reduced model."""
    i0: int
    j0: int
    ni: int
    nj: int
    r: int
    q: int
    eps_r: np.ndarray   # fine-cell relative permittivity [r*nj, r*ni]
    sigma: np.ndarray   # fine-cell conductivity in S/m  [r*nj, r*ni]
    f_max: float        # source bandwidth in Hz (sets the expansion point)
    group: int = -1     # regions with equal group >= 0 share one model
    pec: Optional[np.ndarray] = None   # fine cells that are perfect conductors [r*nj, r*ni]

    @property
    def n_ports(self) -> int:
        return 2 * (self.ni + self.nj)


@dataclasses.dataclass
class Pml:
    """Absorbing layers of the coarse grid (convolutional PML): thickness in
    coarse cells on each side (0: that side stays a PEC wall) and the
    grading parameters - polynomial order m, conductivity scale (1 = the
    usual optimum 0.8 (m+1)/(eta0 d)), maximum stretch kappa and the
    complex-frequency shift alpha (S/m) at the layer's inner face."""
    n_xlo: int = 0
    n_xhi: int = 0
    n_ylo: int = 0
    n_yhi: int = 0
    m: float = 3.0
    sigma_scale: float = 1.0
    kappa_max: float = 1.0
    alpha_max: float = 0.0

    @property
    def any(self) -> bool:
        return (self.n_xlo + self.n_xhi + self.n_ylo + self.n_yhi) > 0


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    eps_r: np.ndarray   # coarse-cell relative permittivity [ny, nx]
    sigma: np.ndarray   # coarse-cell conductivity [ny, nx]
    roms: List[RomSpec]
    sources: List[Source]
    probes: List[Probe]
    nsteps: int
    dtype: str          # "f64" or "f32"
    pml: Optional[Pml] = None
    pec: Optional[np.ndarray] = None   # coarse cells that are perfect conductors [ny, nx]
    pitch_pad: int = 0                  # device layout: unused columns appended to each row

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


# ----------------------------------------------------------------------------
# waveforms
# ----------------------------------------------------------------------------

def pulse_tau(f_bw: float) -> float:
    """Gaussian width whose spectrum falls to 1 % at ``f_bw``."""
    return math.sqrt(math.log(100.0)) / (math.pi * f_bw)


def gaussian_derivative(nsteps: int, dt: float, f_bw: float, amp: float = 1.0,
                        t_offset: float = 0.0) -> np.ndarray:
    """Differentiated Gaussian, peak magnitude ``amp``, sampled at n*dt + t_offset."""
    tau = pulse_tau(f_bw)
    t0 = 4.0 * tau
    t = np.arange(nsteps, dtype=np.float64) * dt + t_offset
    x = (t - t0) / tau
    return -amp * math.sqrt(2.0 * math.e) * x * np.exp(-x * x)


def gaussian(nsteps: int, dt: float, f_bw: float, amp: float = 1.0,
             t_offset: float = 0.0) -> np.ndarray:
    tau = pulse_tau(f_bw)
    t0 = 4.0 * tau
    t = np.arange(nsteps, dtype=np.float64) * dt + t_offset
    x = (t - t0) / tau
    return amp * np.exp(-x * x)


def courant_dt(dx: float, dy: float, frac: float, eps_r: float = 1.0) -> float:
    """frac times the 2D Courant limit for wave speed c0/sqrt(eps_r)."""
    c = _C0 / math.sqrt(eps_r)
    return frac / (c * math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2))


# ----------------------------------------------------------------------------
# material maps
# ----------------------------------------------------------------------------

def patch_map(rng: np.random.Generator, nx: int, ny: int, patch: int,
              lo: float, hi: float) -> np.ndarray:
    """Piecewise-constant map, uniform draw per patch x patch block (raster order)."""
    px = (nx + patch - 1) // patch
    py = (ny + patch - 1) // patch
    vals = rng.uniform(lo, hi, size=(py, px))
    full = np.repeat(np.repeat(vals, patch, axis=0), patch, axis=1)
    return np.ascontiguousarray(full[:ny, :nx])


def upsample(coarse: np.ndarray, i0: int, j0: int, ni: int, nj: int, r: int) -> np.ndarray:
    """Fine-cell map of a block: each fine cell takes its coarse cell's value."""
    blk = coarse[j0:j0 + nj, i0:i0 + ni]
    return np.ascontiguousarray(np.repeat(np.repeat(blk, r, axis=0), r, axis=1))


def uniform_fine(ni: int, nj: int, r: int, value: float) -> np.ndarray:
    return np.full((r * nj, r * ni), value, dtype=np.float64)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def cavity_c1(nsteps: int = 2000) -> Problem:
    """60x60 PEC cavity, 1 cm cells, vacuum; central 10x10 block refined 4x
    (eps_r = 4, sigma = 0.01 S/m) replaced by one order-40 model.  Source:
    differentiated Gaussian (10 GHz bandwidth) on Hz(15,15); probe Hz(45,45).
    dt = 0.99 x the vacuum Courant limit of the fine (2.5 mm) mesh.  FP64."""
    nx = ny = 60
    dx = dy = 0.01
    r = 4
    dt = courant_dt(dx / r, dy / r, 0.99)
    f_bw = 10e9
    rom = RomSpec(i0=25, j0=25, ni=10, nj=10, r=r, q=40,
                  eps_r=uniform_fine(10, 10, r, 4.0),
                  sigma=uniform_fine(10, 10, r, 0.01), f_max=f_bw)
    src = Source(HZ, 15, 16, 15, 16, gaussian_derivative(nsteps, dt, f_bw))
    return Problem("C1-cavity-60", nx, ny, dx, dy, dt,
                   np.ones((ny, nx)), np.zeros((ny, nx)), [rom], [src],
                   [Probe(HZ, 45, 45)], nsteps, "f64")


def random_media(n: int = 2048, nsteps: int = 10000, seed: int = 2,
                 block: int = 32, spacing: int = 512, offset: int = 224,
                 qs: Tuple[int, ...] = (32, 48, 64, 96), r: int = 4,
                 n_probe_side: int = 8, dtype: str = "f32",
                 eps_hi: float = 10.0, sig_hi: float = 0.05,
                 f_bw: float = 1e9) -> Problem:
    """n x n random piecewise-constant medium (eps_r in [1,eps_hi], sigma in
    [0,sig_hi] per 32x32 patch), reduced blocks of ``block`` cells on a
    regular lattice (origins offset + spacing*a), refined r-fold with the
    patch material, orders cycling through ``qs``.  dt = 0.95 x coarse
    vacuum Courant limit.  Magnetic-current source at the centre; probes on
    an n_probe_side^2 lattice.  The default is the 2048^2, 16-model FP32 run."""
    rng = np.random.default_rng(seed)
    dx = dy = 0.01
    eps = patch_map(rng, n, n, 32, 1.0, eps_hi)
    sig = patch_map(rng, n, n, 32, 0.0, sig_hi)
    dt = courant_dt(dx, dy, 0.95)
    roms = []
    nb = max(1, (n - offset) // spacing + (1 if (n - offset) % spacing >= block else 0))
    k = 0
    for a in range(nb):
        for b in range(nb):
            i0 = offset + spacing * a
            j0 = offset + spacing * b
            if i0 + block + 1 >= n or j0 + block + 1 >= n:
                continue
            roms.append(RomSpec(i0=i0, j0=j0, ni=block, nj=block, r=r,
                                q=qs[k % len(qs)],
                                eps_r=upsample(eps, i0, j0, block, block, r),
                                sigma=upsample(sig, i0, j0, block, block, r),
                                f_max=f_bw))
            k += 1
    src = Source(HZ, n // 2, n // 2 + 1, n // 2, n // 2 + 1,
                 gaussian_derivative(nsteps, dt, f_bw))
    step = n // n_probe_side
    probes = [Probe(HZ, step // 2 + step * a, step // 2 + step * b)
              for a in range(n_probe_side) for b in range(n_probe_side)]
    return Problem(f"C2-random-{n}", n, n, dx, dy, dt, eps, sig, roms, [src],
                   probes, nsteps, dtype)


def many_copies(n: int = 4096, nsteps: int = 5000, q: int = 128,
                spacing: int = 256, block: int = 32, r: int = 4,
                dtype: str = "f32", f_bw: float = 1e9) -> Problem:
    """n x n vacuum PEC guide with identical reduced blocks (fine eps_r=4,
    sigma=0.01) on a regular lattice, all sharing one model (group 0).  A
    Gaussian plane wave is injected by an additive Ey line source on column
    i=8; probes Hz(spacing*a + spacing/2, n/2)."""
    dx = dy = 0.01
    dt = courant_dt(dx, dy, 0.95)
    off = spacing // 2 - block // 2
    na = n // spacing
    roms = []
    fe = uniform_fine(block, block, r, 4.0)
    fs = uniform_fine(block, block, r, 0.01)
    for a in range(na):
        for b in range(na):
            roms.append(RomSpec(i0=off + spacing * a, j0=off + spacing * b,
                                ni=block, nj=block, r=r, q=q, eps_r=fe, sigma=fs,
                                f_max=f_bw, group=0))
    src = Source(EY, 8, 9, 0, n, gaussian(nsteps, dt, f_bw, t_offset=0.5 * dt))
    probes = [Probe(HZ, spacing * a + spacing // 2, n // 2) for a in range(na)]
    return Problem(f"C3-copies-{n}", n, n, dx, dy, dt, np.ones((n, n)),
                   np.zeros((n, n)), roms, [src], probes, nsteps, dtype)


def _place_blocks(rng, nx, ny, m, block, gap, tries=1000):
    placed = []
    for _ in range(tries):
        if len(placed) == m:
            break
        i0 = int(rng.integers(gap, nx - block - gap + 1))
        j0 = int(rng.integers(gap, ny - block - gap + 1))
        ok = True
        for (a, b) in placed:
            if not (i0 + block + gap <= a or a + block + gap <= i0 or
                    j0 + block + gap <= b or b + block + gap <= j0):
                ok = False
                break
        if ok:
            placed.append((i0, j0))
    return placed


def batch_c4(B: int = 64, nsteps: int = 3000, seed: int = 4, nmin: int = 256,
             nmax: int = 1024, block: int = 16, r: int = 4,
             qmin: int = 16, qmax: int = 96, mmax: int = 8,
             dtype: str = "f32", f_bw: float = 1e9) -> List[Problem]:
    """B independent instances: sizes uniform in [nmin, nmax] per axis, eps_r
    in [1,8], sigma in [0,0.02] per 32x32 patch, 1..mmax reduced 16x16 blocks
    (r=4, orders uniform in [qmin,qmax]) placed with >= 2-cell gaps, one
    source at a random free cell, four random probes."""
    rng = np.random.default_rng(seed)
    dx = dy = 0.01
    dt = courant_dt(dx, dy, 0.95)
    out = []
    for b in range(B):
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        eps = patch_map(rng, nx, ny, 32, 1.0, 8.0)
        sig = patch_map(rng, nx, ny, 32, 0.0, 0.02)
        m = int(rng.integers(1, mmax + 1))
        blocks = _place_blocks(rng, nx, ny, m, block, 2)
        roms = []
        for (i0, j0) in blocks:
            q = int(rng.integers(qmin, qmax + 1))
            roms.append(RomSpec(i0=i0, j0=j0, ni=block, nj=block, r=r, q=q,
                                eps_r=upsample(eps, i0, j0, block, block, r),
                                sigma=upsample(sig, i0, j0, block, block, r),
                                f_max=f_bw))

        def free_cell():
            while True:
                i = int(rng.integers(1, nx - 1))
                j = int(rng.integers(1, ny - 1))
                if all(not (i0 - 1 <= i <= i0 + block and j0 - 1 <= j <= j0 + block)
                       for (i0, j0) in blocks):
                    return i, j
        si, sj = free_cell()
        src = Source(HZ, si, si + 1, sj, sj + 1, gaussian_derivative(nsteps, dt, f_bw))
        probes = []
        for _ in range(4):
            pi, pj = free_cell()
            probes.append(Probe(HZ, pi, pj))
        out.append(Problem(f"C4-batch-{b}", nx, ny, dx, dy, dt, eps, sig, roms,
                           [src], probes, nsteps, dtype))
    return out


def adjoint_c5(n: int = 1024, nsteps: int = 4000, seed: int = 5, q: int = 64,
               block: int = 32, r: int = 4, dtype: str = "f32",
               f_bw: float = 1e9) -> Problem:
    """n x n random medium (eps_r in [1,10], sigma in [0,0.05] per 32x32
    patch), four reduced blocks at (224|736, 224|736) scaled to n, source at
    the centre, objective probe Hz(800,300) scaled to n."""
    rng = np.random.default_rng(seed)
    dx = dy = 0.01
    eps = patch_map(rng, n, n, 32, 1.0, 10.0)
    sig = patch_map(rng, n, n, 32, 0.0, 0.05)
    dt = courant_dt(dx, dy, 0.95)
    s = n / 1024.0
    roms = []
    for (a, b) in [(224, 224), (224, 736), (736, 224), (736, 736)]:
        i0 = int(round(a * s))
        j0 = int(round(b * s))
        roms.append(RomSpec(i0=i0, j0=j0, ni=block, nj=block, r=r, q=q,
                            eps_r=upsample(eps, i0, j0, block, block, r),
                            sigma=upsample(sig, i0, j0, block, block, r),
                            f_max=f_bw))
    c = n // 2
    src = Source(HZ, c, c + 1, c, c + 1, gaussian_derivative(nsteps, dt, f_bw))
    probe = Probe(HZ, int(round(800 * s)), int(round(300 * s)))
    return Problem(f"C5-adjoint-{n}", n, n, dx, dy, dt, eps, sig, roms, [src],
                   [probe], nsteps, dtype)


def fd_cells(prob: Problem, count: int = 32, seed: int = 5) -> List[Tuple[int, int]]:
    """Cells for finite-difference gradient checks: random, outside every
    reduced block and its one-cell ring, away from the walls."""
    rng = np.random.default_rng(seed + 1000)
    cells = []
    while len(cells) < count:
        i = int(rng.integers(1, prob.nx - 1))
        j = int(rng.integers(1, prob.ny - 1))
        bad = False
        for rm in prob.roms:
            if rm.i0 - 1 <= i <= rm.i0 + rm.ni and rm.j0 - 1 <= j <= rm.j0 + rm.nj:
                bad = True
        if not bad and (i, j) not in cells:
            cells.append((i, j))
    return cells


def stencil_only(n: int = 8192, nsteps: int = 200, material: bool = True,
                 dtype: str = "f32", seed: int = 2) -> Problem:
    """Large grid with no reduced regions, for the HBM-resident stencil rate."""
    rng = np.random.default_rng(seed)
    dx = dy = 0.01
    dt = courant_dt(dx, dy, 0.95)
    if material:
        eps = patch_map(rng, n, n, 32, 1.0, 10.0)
        sig = patch_map(rng, n, n, 32, 0.0, 0.05)
    else:
        eps = np.ones((n, n))
        sig = np.zeros((n, n))
    src = Source(HZ, n // 2, n // 2 + 1, n // 2, n // 2 + 1,
                 gaussian_derivative(nsteps, dt, 1e9))
    return Problem(f"S-stencil-{n}", n, n, dx, dy, dt, eps, sig, [], [src],
                   [Probe(HZ, n // 4, n // 4)], nsteps, dtype)


# Conductivity of the copper rods (Sec. VI-C).
SIGMA_COPPER = 5.8e7


def iris_waveguide(nsteps: int = 4000, q: int = 648, irises: bool = True,
                   dtype: str = "f64", aperture: int = 18, f_bw: float = 0.4e9,
                   cfl_gain: float = 2.0) -> Problem:
    """Waveguide with two thin PEC irises (Sec. VI-B): 4 m x 0.7 m, 5 cm
    coarse cells (80 x 14), PEC walls at y = 0 and 0.7 m, absorbing layers 10
    coarse cells deep at both x ends.  Two 0.5 m x 0.5 m regions (10 x 10
    coarse cells at i0 = 25 and 45, j0 = 2) refined 3-fold (30 x 30 fine
    cells, 2,760 states) are replaced by order-``q`` models.

    The iris geometry is only drawn in the paper and its thickness is not
    given; here each iris is a perfectly conducting plate one fine cell
    (1.67 cm) thick on the middle fine column of the region's middle coarse
    column (x in [1.517, 1.533] m and [2.517, 2.533] m), from both edges of
    the region to a centred aperture of ``aperture`` fine cells (0.3 m).
    Between the region and the walls the plates continue as PEC coarse
    cells of that coarse column (the coarse mesh has nothing thinner); in
    the region's first and last fine rows the plate takes the whole coarse
    column's width, so that the coarse interface edge where it meets the
    continuation is PEC over all its fine edges (eq. (15) ties them).
    Excitation: a Gaussian current pulse (``f_bw`` bandwidth) on an Ey line
    across the guide at i = 12; probes at the far end (Hz, Ey at i = 67)
    and near the source (Hz at i = 14).  dt = cfl_gain x 0.99 x the fine
    mesh's vacuum Courant limit."""
    nx, ny = 80, 14
    dx = dy = 0.05
    r = 3
    dt = cfl_gain * courant_dt(dx / r, dy / r, 0.99)
    eps = np.ones((ny, nx))
    sig = np.zeros((ny, nx))
    pec = np.zeros((ny, nx), dtype=bool)
    roms = []
    for i0 in (25, 45):
        fe = uniform_fine(10, 10, r, 1.0)
        fs = uniform_fine(10, 10, r, 0.0)
        fp = None
        if irises:
            c0 = r * (10 // 2)
            mid = c0 + r // 2
            lo = (r * 10 - aperture) // 2
            fp = np.zeros((r * 10, r * 10), dtype=bool)
            fp[:lo, mid] = True
            fp[lo + aperture:, mid] = True
            fp[0, c0:c0 + r] = True
            fp[-1, c0:c0 + r] = True
            ci = i0 + 10 // 2
            pec[:2, ci] = True
            pec[12:, ci] = True
        roms.append(RomSpec(i0=i0, j0=2, ni=10, nj=10, r=r, q=q, eps_r=fe, sigma=fs,
                            f_max=f_bw, pec=fp))
    src = Source(EY, 12, 13, 0, ny, gaussian(nsteps, dt, f_bw, t_offset=0.5 * dt))
    probes = [Probe(HZ, 67, 7), Probe(EY, 67, 7), Probe(HZ, 14, 7)]
    return Problem("E3-irises" if irises else "E3-empty", nx, ny, dx, dy, dt, eps, sig, roms,
                   [src], probes, nsteps, dtype, Pml(10, 10, 0, 0), pec if irises else None)


def rods_reflection(nsteps: int = 2000, q: int = 1920, rods: bool = True,
                    dtype: str = "f64", f_bw: float = 30e9, cfl_gain: float = 3.0) -> Problem:
    """Reflection test (Sec. VI-C): 66 mm x 40 mm waveguide, 1 mm coarse
    cells, PEC walls at y = 0 and 40 mm, absorbing layers 15 mm deep at both
    x ends.  The 8 mm x 8 mm region x in [39, 47] mm, y in [16, 24] mm is
    refined 6-fold (48 x 48 fine cells, 7,008 states) and replaced by an
    order-``q`` model.  Scatterer (``rods``): four copper rods of 1 mm
    radius centred at (41, 22), (41, 18), (45, 22), (45, 18) mm, as the fine
    cells whose centres lie within the radius; without rods the region is
    vacuum (the interface-reflection run).  Excitation: a Gaussian Jy line
    current at x = 17 mm (pulse bandwidth ``f_bw``: not given in the paper);
    line probe: Ey at x = 19 mm on every row.  dt = cfl_gain x 0.99 x the
    fine mesh's vacuum Courant limit."""
    nx, ny = 66, 40
    dx = dy = 1e-3
    r = 6
    i0, j0, nb = 39, 16, 8
    dt = cfl_gain * courant_dt(dx / r, dy / r, 0.99)
    fe = uniform_fine(nb, nb, r, 1.0)
    fs = uniform_fine(nb, nb, r, 0.0)
    if rods:
        xc = i0 + (np.arange(r * nb) + 0.5) / r          # fine cell centres in mm
        yc = j0 + (np.arange(r * nb) + 0.5) / r
        X, Y = np.meshgrid(xc, yc)
        for cx, cy in ((41.0, 22.0), (41.0, 18.0), (45.0, 22.0), (45.0, 18.0)):
            fs[(X - cx) ** 2 + (Y - cy) ** 2 <= 1.0] = SIGMA_COPPER
    rom = RomSpec(i0=i0, j0=j0, ni=nb, nj=nb, r=r, q=q, eps_r=fe, sigma=fs, f_max=f_bw)
    src = Source(EY, 17, 18, 0, ny, gaussian(nsteps, dt, f_bw, t_offset=0.5 * dt))
    probes = [Probe(EY, 19, j) for j in range(ny)]
    return Problem("E4-rods" if rods else "E4-empty", nx, ny, dx, dy, dt, np.ones((ny, nx)),
                   np.zeros((ny, nx)), [rom], [src], probes, nsteps, dtype, Pml(15, 15, 0, 0))


def iris_sweep(count: int = 64, nsteps: int = 4000, dtype: str = "f32", q: int = 648) -> List[Problem]:
    """A design sweep over the iris guide of Sec. VI-B: ``count`` guides whose
    iris apertures step through 4..26 fine cells (two sizes per even value
    repeat when count > 12), otherwise identical - the kind of parameter
    study a batch of independent runs serves."""
    out = []
    for k in range(count):
        ap = 4 + 2 * (k % 12)
        p = iris_waveguide(nsteps=nsteps, q=q, dtype=dtype, aperture=ap)
        out.append(dataclasses.replace(p, name=f"E3-irises-ap{ap}-{k}"))
    return out


# The method variants compared in Tabs. I-III, as (basis, clip, CFL number
# relative to the fine mesh's limit): "mor_only" reduces without the CFL
# extension (so its step stays within the fine limit), "cfl_only" keeps the
# whole fine model and extends the limit, "proposed" does both; "coarse" is
# the all-coarse Yee run (no regions, the coarse mesh's own limit).
ABLATIONS = {
    "coarse": dict(basis=None, clip=False),
    "mor_only": dict(basis="sprim", clip=False),
    "cfl_only": dict(basis="identity", clip=True),
    "proposed": dict(basis="sprim", clip=True),
}


def ablation(make, mode: str, proposed_steps: int, **kw) -> Problem:
    """Problem for one method variant of an experiment built by ``make``
    (``iris_waveguide`` or ``rods_reflection``), simulating the same time as
    ``proposed_steps`` steps of the proposed method: MOR only runs at 0.99x
    the fine limit, CFL extension only at the proposed step, the all-coarse
    run at 0.99x the coarse limit with each region's fine material sampled
    at the coarse cell centres."""
    base = make(nsteps=proposed_steps, **kw)
    r = base.roms[0].r
    fine_dt = courant_dt(base.dx / r, base.dy / r, 0.99)
    if mode == "proposed":
        return base
    if mode == "cfl_only":
        return dataclasses.replace(base, name=base.name + "-cfl-only")
    if mode == "mor_only":
        n = int(math.ceil(proposed_steps * base.dt / fine_dt))
        p = make(nsteps=n, cfl_gain=1.0, **kw)
        # per-step increments of a current scale with the step
        src = [dataclasses.replace(x, incr=x.incr * (p.dt / base.dt)) for x in p.sources]
        return dataclasses.replace(p, name=p.name + "-mor-only", sources=src)
    if mode == "coarse":
        dt = courant_dt(base.dx, base.dy, 0.99)
        n = int(math.ceil(proposed_steps * base.dt / dt))
        p = make(nsteps=n, **kw)
        eps, sig = p.eps_r.copy(), p.sigma.copy()
        pec = np.zeros((p.ny, p.nx), dtype=bool) if p.pec is None else p.pec.copy()
        for s in p.roms:
            c = s.r // 2
            eps[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.eps_r[c::s.r, c::s.r]
            sig[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.sigma[c::s.r, c::s.r]
            if s.pec is not None:
                pec[s.j0:s.j0 + s.nj, s.i0:s.i0 + s.ni] = s.pec[c::s.r, c::s.r]
        src = [dataclasses.replace(x, incr=_resample(x.incr, p.dt, dt, n)) for x in p.sources]
        return dataclasses.replace(p, name=p.name + "-coarse", dt=dt, eps_r=eps, sigma=sig, roms=[],
                                   sources=src, nsteps=n, pec=pec if pec.any() else None)
    raise ValueError(mode)


def _resample(incr: np.ndarray, dt_old: float, dt_new: float, n: int) -> np.ndarray:
    """A source waveform sampled at another step (linear interpolation in
    time, scaled by the step ratio so the injected charge stays the same)."""
    t_old = np.arange(len(incr)) * dt_old
    t_new = np.arange(n) * dt_new
    return np.interp(t_new, t_old, incr, right=0.0) * (dt_new / dt_old)


def pec_problem(seed: int = 1, r: int = 2, q: int = 12, nsteps: int = 150, dtype: str = "f64",
                nx: int = 20, ny: int = 18) -> Problem:
    """A small random problem with one 5 x 4 region that holds PEC fine
    cells: a plate from the region's South boundary (continued by PEC coarse
    cells down to the wall, so the port it covers carries no field), a PEC
    fine cell in the North-East corner (two more such ports) and one
    interior PEC fine cell; sources and probes stay on free samples."""
    p = random_problem(seed, nx, ny, nsteps, nroms=1, block=(5, 4), r=r, q=q, dtype=dtype)
    s = p.roms[0]
    fp = np.zeros((r * s.nj, r * s.ni), dtype=bool)
    fp[: 2 * r, 2 * r:3 * r] = True             # plate over South port 2
    fp[3 * r:, 4 * r:] = True                   # North-East corner cell: North port 4, East port 3
    fp[r, r] = True                             # an interior fine cell
    s.pec = fp
    pec = np.zeros((p.ny, p.nx), dtype=bool)
    pec[: s.j0, s.i0 + 2] = True                # the plate's coarse continuation
    p.pec = pec

    def free(comp, i, j):
        if comp == HZ:
            return not pec[j, i]
        if comp == EX:
            return not (pec[j, i] if j < p.ny else False) and not (pec[j - 1, i] if j >= 1 else False)
        return not (pec[j, i] if i < p.nx else False) and not (pec[j, i - 1] if i >= 1 else False)
    for src in p.sources:
        assert all(free(src.comp, i, j) for j in range(src.j0, src.j1) for i in range(src.i0, src.i1))
    p.probes = [pr for pr in p.probes if free(pr.comp, pr.i, pr.j)]
    assert p.probes
    return p


def random_problem(seed: int, nx: int, ny: int, nsteps: int, nroms: int = 2,
                   block: Tuple[int, int] = (6, 5), r: int = 2, q: int = 12,
                   dtype: str = "f64", lossy: bool = True,
                   dt_frac_coarse: Optional[float] = None,
                   f_bw: float = 3e9, init_fields: bool = False) -> Problem:
    """Small random test problem (parity and property tests)."""
    rng = np.random.default_rng(seed)
    dx, dy = 0.01, 0.012
    eps = rng.uniform(1.0, 4.0, size=(ny, nx))
    sig = rng.uniform(0.0, 0.05, size=(ny, nx)) if lossy else np.zeros((ny, nx))
    ni, nj = block
    blocks = _place_blocks(rng, nx, ny, nroms, max(ni, nj), 2)
    roms = []
    for (i0, j0) in blocks:
        fe = rng.uniform(1.0, 6.0, size=(r * nj, r * ni))
        fs = rng.uniform(0.0, 0.05, size=(r * nj, r * ni)) if lossy else np.zeros((r * nj, r * ni))
        roms.append(RomSpec(i0=i0, j0=j0, ni=ni, nj=nj, r=r, q=q, eps_r=fe,
                            sigma=fs, f_max=f_bw))
    if dt_frac_coarse is None:
        dt = courant_dt(dx / r, dy / r, 0.99)
    else:
        dt = courant_dt(dx, dy, dt_frac_coarse)

    def free_cell():
        while True:
            i = int(rng.integers(1, nx - 1))
            j = int(rng.integers(1, ny - 1))
            if all(not (rm.i0 - 1 <= i <= rm.i0 + rm.ni and rm.j0 - 1 <= j <= rm.j0 + rm.nj)
                   for rm in roms):
                return i, j
    si, sj = free_cell()
    srcs = [Source(HZ, si, si + 1, sj, sj + 1, gaussian_derivative(nsteps, dt, f_bw))]
    ei, ej = free_cell()
    srcs.append(Source(EY, ei, ei + 1, ej, ej + 1,
                       0.3 * gaussian(nsteps, dt, f_bw, t_offset=0.5 * dt)))
    probes = []
    for comp in (HZ, HZ, EX, EY):
        pi, pj = free_cell()
        probes.append(Probe(comp, pi, pj))
    return Problem(f"rand-{seed}-{nx}x{ny}", nx, ny, dx, dy, dt, eps, sig, roms,
                   srcs, probes, nsteps, dtype)
