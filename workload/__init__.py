"""Seeded synthetic inputs for the particle / bulk-grid / fine-grid coupling exchange.

This module only *draws* inputs: particle positions, diameters and velocities, and
the fine-grid fluid velocity and pressure sampled at fine cell centres.  It holds
none of the coupling arithmetic (binning, deposition, restriction, interpolation,
drag, prolongation); both the FP64 oracle and the GPU path receive the arrays it
returns and nothing else.

Workloads (the paper's own cases need solver runs and case files that are not
available; these synthetic stand-ins keep their shape, see Sec. 3.3 for the
10-million-particle layered bed that the largest one imitates):

* ``cube8_ngp_fp64``  unit cube, bulk 8^3, fine 32^3, 10,000 uniform spheres,
  log-normal diameters, Taylor-Green fluid of amplitude 1, FP64, containing-cell
  deposition.
* ``cube64_cic``      unit cube, bulk 64^3, fine 256^3, 2,000,000 uniform spheres,
  same distributions, cloud-in-cell deposition, 100 explicit-Euler steps of 1e-4.
* ``bed128_cic``      box 1x1x2, bulk 128x128x256, fine 512x512x1024, 10,000,000
  spheres: 7,000,000 on a jittered lattice in the bottom quarter (solid fraction
  ~0.6), 3,000,000 uniform above; bimodal diameters; upflow 0.5 plus a Taylor-Green
  perturbation of amplitude 0.1.
* ``bed128_sub2m``    the same grids and fluid with the particles whose id is a
  multiple of 5 (2,000,000), for the precision study.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in the fixed order
positions, diameters (through class labels for the bed), velocities.  Positions are drawn in FP64 and
rounded once to the working precision.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Grid description
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Grid:
    """Uniform, nested bulk/fine grid pair.

    ``box`` is (Lx, Ly, Lz); ``nb`` is bulk cells per axis (x, y, z); the fine grid
    has ``ratio`` fine cells per bulk cell along every axis.  Arrays are stored
    z-major, x fastest: a field of the fine grid has shape (nfz, nfy, nfx).
    """

    box: tuple
    nb: tuple
    ratio: int

    @property
    def nf(self):
        return tuple(n * self.ratio for n in self.nb)

    @property
    def n_bulk(self):
        return self.nb[0] * self.nb[1] * self.nb[2]

    @property
    def n_fine(self):
        nf = self.nf
        return nf[0] * nf[1] * nf[2]

    def fine_centres_1d(self, axis):
        """Fine cell-centre coordinates along ``axis`` (FP64)."""
        n = self.nf[axis]
        h = self.box[axis] / n
        return (np.arange(n, dtype=np.float64) + 0.5) * h


@dataclass
class Workload:
    name: str
    grid: Grid
    n_particles: int
    precision: str          # "fp64" | "fp32"
    deposit: str            # "ngp" | "cic"
    seed: int
    particles: str          # "uniform" | "bed"
    fluid: str              # "tg1" | "upflow"
    steps: int = 1
    dt: float = 0.0
    advect: bool = False
    rho_f: float = 1000.0
    mu_f: float = 1.0e-3
    rho_p: float = 2500.0
    eps_min: float = 0.3
    bed_diameters: tuple = (0.002630, 0.005260)
    subsample_stride: int = 1
    notes: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "cube8_ngp_fp64": Workload(
        name="cube8_ngp_fp64", grid=Grid((1.0, 1.0, 1.0), (8, 8, 8), 4),
        n_particles=10_000, precision="fp64", deposit="ngp", seed=0,
        particles="uniform", fluid="tg1"),
    "cube64_cic": Workload(
        name="cube64_cic", grid=Grid((1.0, 1.0, 1.0), (64, 64, 64), 4),
        n_particles=2_000_000, precision="fp32", deposit="cic", seed=1,
        particles="uniform", fluid="tg1", steps=100, dt=1.0e-4, advect=True),
    "bed128_cic": Workload(
        name="bed128_cic", grid=Grid((1.0, 1.0, 2.0), (128, 128, 256), 4),
        n_particles=10_000_000, precision="fp32", deposit="cic", seed=2,
        particles="bed", fluid="upflow"),
    "bed128_sub2m": Workload(
        name="bed128_sub2m", grid=Grid((1.0, 1.0, 2.0), (128, 128, 256), 4),
        n_particles=10_000_000, precision="fp32", deposit="cic", seed=2,
        particles="bed", fluid="upflow", subsample_stride=5),
}

# ---------------------------------------------------------------------------
# Particles
# ---------------------------------------------------------------------------

LOGNORMAL_MEAN = 0.02
LOGNORMAL_SIGMA = 0.2
LOGNORMAL_CLIP = (0.01, 0.04)
VELOCITY_SIGMA = 0.1


def lognormal_diameters(rng, n):
    """d = clip(exp(mu + sigma Z), 0.01, 0.04) with mu chosen so that E[d] = 0.02."""
    mu = math.log(LOGNORMAL_MEAN) - 0.5 * LOGNORMAL_SIGMA ** 2
    z = rng.standard_normal(n)
    return np.clip(np.exp(mu + LOGNORMAL_SIGMA * z), *LOGNORMAL_CLIP)


def uniform_particles(rng, n, box):
    """Positions U[0, L) per axis, log-normal diameters, N(0, 0.1^2) velocities."""
    pos = rng.random((n, 3)) * np.asarray(box, dtype=np.float64)
    d = lognormal_diameters(rng, n)
    vel = rng.normal(0.0, VELOCITY_SIGMA, size=(n, 3))
    return pos, d, vel


BED_LATTICE = (242, 242, 120)      # sites along x, y, z in the bottom quarter
BED_TOP_Z = 0.5
BED_PACKED = 7_000_000
BED_LOOSE = 3_000_000


def bed_particles(rng, box, diameters):
    """Layered packed bed: jittered lattice in z < 0.5, uniform loose particles above.

    The lattice has 242 x 242 x 120 sites with spacing (Lx/242, Ly/242, 0.5/120);
    each site is jittered uniformly by +-0.25 spacing per axis and a seeded random
    subset of 7,000,000 sites is kept (in the random order the draw returns).  The
    remaining 3,000,000 particles are uniform in [0,Lx) x [0,Ly) x [0.5, Lz).
    Diameters are bimodal, exactly half of each class, assigned by a seeded
    permutation.
    """
    nx, ny, nz = BED_LATTICE
    sp = np.array([box[0] / nx, box[1] / ny, BED_TOP_Z / nz])
    nsite = nx * ny * nz
    # positions: lattice subset, jitter, loose particles
    pick = rng.permutation(nsite)[:BED_PACKED]
    iz, rem = np.divmod(pick, nx * ny)
    iy, ix = np.divmod(rem, nx)
    lat = np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5
    jitter = rng.uniform(-0.25, 0.25, size=(BED_PACKED, 3))
    packed = (lat + jitter) * sp
    lo = np.array([0.0, 0.0, BED_TOP_Z])
    ext = np.array([box[0], box[1], box[2] - BED_TOP_Z])
    loose = lo + rng.random((BED_LOOSE, 3)) * ext
    pos = np.concatenate([packed, loose], axis=0)
    n = pos.shape[0]
    cls = rng.permutation(n) < (n // 2)
    d = np.where(cls, diameters[1], diameters[0]).astype(np.float64)
    vel = rng.normal(0.0, VELOCITY_SIGMA, size=(n, 3))
    return pos, d, vel


def particles(w: Workload, seed=None, n=None):
    """Draw the particle set of workload ``w``.

    Returns (pos [n,3], diam [n], vel [n,3]) as float32 (fp32 workloads) or float64.
    ``n`` overrides the particle count of uniform workloads (small test cases).
    """
    rng = np.random.default_rng(w.seed if seed is None else seed)
    if w.particles == "uniform":
        pos, d, vel = uniform_particles(rng, w.n_particles if n is None else n, w.grid.box)
    elif w.particles == "bed":
        pos, d, vel = bed_particles(rng, w.grid.box, w.bed_diameters)
    else:
        raise ValueError(w.particles)
    if w.subsample_stride > 1:
        sel = slice(0, None, w.subsample_stride)
        pos, d, vel = pos[sel], d[sel], vel[sel]
    dt = np.float64 if w.precision == "fp64" else np.float32
    return (np.ascontiguousarray(pos.astype(dt)), np.ascontiguousarray(d.astype(dt)),
            np.ascontiguousarray(vel.astype(dt)))


# ---------------------------------------------------------------------------
# Fluid on the fine grid (point values at fine cell centres)
# ---------------------------------------------------------------------------

TG_K = 2.0 * math.pi


def _tables(grid: Grid, xp):
    """1-D FP64 tables of the Taylor-Green factors on fine cell centres."""
    xs = [grid.fine_centres_1d(a) for a in range(3)]
    t = {}
    for a, name in enumerate("xyz"):
        v = TG_K * xs[a]
        t["s" + name] = np.sin(v)
        t["c" + name] = np.cos(v)
        t["c2" + name] = np.cos(2.0 * v)
    if xp is not np:
        t = {k: xp.as_tensor(v) for k, v in t.items()}
    return t


def _fields(grid: Grid, fluid: str, rho_f: float, t, sl=None):
    """Evaluate (u, v, w, p) from the 1-D tables with fixed multiplication order.

    ``t`` holds numpy arrays or torch tensors; the expressions below are evaluated
    identically by either library (IEEE FP64 products in the same order), so a
    field generated on the host and on the device is bitwise the same.
    """
    if fluid == "tg1":
        amp, w0 = 1.0, 0.0
    elif fluid == "upflow":
        amp, w0 = 0.1, 0.5
    else:
        raise ValueError(fluid)
    sx, cx, c2x = t["sx"][None, None, :], t["cx"][None, None, :], t["c2x"][None, None, :]
    sy, cy, c2y = t["sy"][None, :, None], t["cy"][None, :, None], t["c2y"][None, :, None]
    sz, cz, c2z = t["sz"][:, None, None], t["cz"][:, None, None], t["c2z"][:, None, None]
    if sl is not None:  # restrict the z extent (streaming generation)
        sz, cz, c2z = sz[sl], cz[sl], c2z[sl]
    u = ((amp * sx) * cy) * cz
    v = ((-amp * cx) * sy) * cz
    pc = rho_f * amp * amp / 16.0
    p = ((c2x + c2y) * (c2z + 2.0)) * pc
    w = u * 0.0 + w0
    return u, v, w, p


def fine_fields(w: Workload, dtype=None):
    """Host (numpy) fine fields u, v, w, p, each (nfz, nfy, nfx), C-contiguous."""
    dt = dtype or (np.float64 if w.precision == "fp64" else np.float32)
    t = _tables(w.grid, np)
    out = []
    for f in _fields(w.grid, w.fluid, w.rho_f, t):
        out.append(np.ascontiguousarray(np.broadcast_to(f, (w.grid.nf[2], w.grid.nf[1], w.grid.nf[0])).astype(dt)))
    return tuple(out)


def fine_fields_torch(w: Workload, device, dtype=None):
    """The same fields built on a torch device (bitwise equal to :func:`fine_fields`)."""
    import torch
    dt = dtype or (torch.float64 if w.precision == "fp64" else torch.float32)
    t = _tables(w.grid, np)
    t = {k: torch.from_numpy(v).to(device) for k, v in t.items()}
    nf = w.grid.nf
    out = []
    for f in _fields(w.grid, w.fluid, w.rho_f, t):
        out.append(f.expand(nf[2], nf[1], nf[0]).to(dt).contiguous())
    return tuple(out)


def _alpha(grid: Grid, xp, x, y, z):
    """Liquid volume fraction of a smooth, tilted free surface: liquid below
    z_s(x, y) = L_z (0.6 + 0.1 x / L_x - 0.05 y / L_y), a tanh profile two fine
    cells thick: alpha = (1 - tanh((z - z_s) / (2 h_z))) / 2."""
    L = grid.box
    zs = L[2] * (0.6 + 0.1 * x / L[0] - 0.05 * y / L[1])
    delta = 2.0 * L[2] / grid.nf[2]
    return 0.5 * (1.0 - xp.tanh((z - zs) / delta))


def fine_alpha(w: Workload, dtype=None):
    """Host (numpy) fine liquid fraction (nfz, nfy, nfx), for the two-fluid drag."""
    dt = dtype or (np.float64 if w.precision == "fp64" else np.float32)
    g = w.grid
    xs = [g.fine_centres_1d(a) for a in range(3)]
    a = _alpha(g, np, xs[0][None, None, :], xs[1][None, :, None], xs[2][:, None, None])
    return np.ascontiguousarray(a.astype(dt))


def fine_alpha_torch(w: Workload, device, dtype=None):
    """The same field built on a torch device (FP64 there, then cast; equal to
    :func:`fine_alpha` up to the last bit of tanh)."""
    import torch
    dt = dtype or (torch.float64 if w.precision == "fp64" else torch.float32)
    g = w.grid
    xs = [torch.from_numpy(g.fine_centres_1d(a)).to(device) for a in range(3)]
    out = torch.empty((g.nf[2], g.nf[1], g.nf[0]), dtype=dt, device=device)
    for k in range(g.nf[2]):   # one z-plane at a time: bounded FP64 temporaries
        out[k] = _alpha(g, torch, xs[0][None, :], xs[1][:, None], xs[2][k]).to(dt)
    return out


def fine_values_at(w: Workload, fidx, dtype=None):
    """Fine-field values (u, v, w, p) at flat fine indices ``fidx`` (host, numpy).

    Equal, element by element, to indexing the arrays of :func:`fine_fields`.
    """
    dt = dtype or (np.float64 if w.precision == "fp64" else np.float32)
    nf = w.grid.nf
    fidx = np.asarray(fidx, dtype=np.int64)
    iz, rem = np.divmod(fidx, nf[0] * nf[1])
    iy, ix = np.divmod(rem, nf[0])
    t = _tables(w.grid, np)
    tt = {}
    for k, v in t.items():
        ax = k[-1]
        idx = {"x": ix, "y": iy, "z": iz}[ax]
        tt[k] = v[idx]
    # evaluate the same expressions on 1-D gathered tables: index [None,None,:] etc.
    # would broadcast; use a flat evaluation with identical operation order instead.
    if w.fluid == "tg1":
        amp, w0 = 1.0, 0.0
    else:
        amp, w0 = 0.1, 0.5
    u = ((amp * tt["sx"]) * tt["cy"]) * tt["cz"]
    v = ((-amp * tt["cx"]) * tt["sy"]) * tt["cz"]
    pc = w.rho_f * amp * amp / 16.0
    p = ((tt["c2x"] + tt["c2y"]) * (tt["c2z"] + 2.0)) * pc
    ww = u * 0.0 + w0
    return tuple(a.astype(dt) for a in (u, v, ww, p))


def fluid_analytic(w: Workload, x, y, z):
    """The continuous fluid fields (FP64) at arbitrary points: for error bounds."""
    amp, w0 = (1.0, 0.0) if w.fluid == "tg1" else (0.1, 0.5)
    k = TG_K
    u = amp * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    v = -amp * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    ww = np.zeros_like(u) + w0
    p = w.rho_f * amp * amp / 16.0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    return u, v, ww, p


def small_workload(nb=(4, 3, 5), ratio=4, box=(1.0, 0.75, 1.25), n=200, seed=7,
                   precision="fp64", deposit="cic", fluid="tg1", advect=False, dt=0.0):
    """A tiny uniform workload for brute-force and edge-case tests."""
    return Workload(name=f"small_{nb[0]}x{nb[1]}x{nb[2]}_r{ratio}_n{n}", grid=Grid(tuple(box), tuple(nb), ratio),
                    n_particles=n, precision=precision, deposit=deposit, seed=seed,
                    particles="uniform", fluid=fluid, advect=advect, dt=dt)


# ---------------------------------------------------------------------------
# Grids made of axis-aligned cells (boxes): uniform and locally refined
# ---------------------------------------------------------------------------

def box_grid(box, n):
    """Cells of a uniform grid of n = (nx, ny, nz) cells over box, as an [N, 6]
    array of boxes (x0, x1, y0, y1, z0, z1) in raster order (x fastest)."""
    e = [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]
    z0, y0, x0 = np.meshgrid(e[2][:-1], e[1][:-1], e[0][:-1], indexing="ij")
    z1, y1, x1 = np.meshgrid(e[2][1:], e[1][1:], e[0][1:], indexing="ij")
    return np.stack([x0.ravel(), x1.ravel(), y0.ravel(), y1.ravel(), z0.ravel(), z1.ravel()], axis=1)


def refined_box_grid(box, n, region, split=2):
    """A locally refined grid: the uniform base grid of n cells over box, with
    every base cell whose centre lies inside region = (x0, x1, y0, y1, z0, z1)
    split into split^3 children.  Cells are listed in the base raster order, a
    split cell replaced in place by its children (raster order within it), so
    that neighbouring cells stay close in memory.  Returns [N, 6] boxes."""
    base = box_grid(box, n)
    cx, cy, cz = (base[:, 0] + base[:, 1]) / 2, (base[:, 2] + base[:, 3]) / 2, (base[:, 4] + base[:, 5]) / 2
    inside = ((cx > region[0]) & (cx < region[1]) & (cy > region[2]) & (cy < region[3]) &
              (cz > region[4]) & (cz < region[5]))
    t = (np.arange(split + 1, dtype=np.float64) / split)
    out = []
    for b, ref in zip(base, inside):
        if not ref:
            out.append(b[None, :])
            continue
        ex = b[0] + (b[1] - b[0]) * t
        ey = b[2] + (b[3] - b[2]) * t
        ez = b[4] + (b[5] - b[4]) * t
        k, j, i = np.meshgrid(np.arange(split), np.arange(split), np.arange(split), indexing="ij")
        k, j, i = k.ravel(), j.ravel(), i.ravel()
        out.append(np.stack([ex[i], ex[i + 1], ey[j], ey[j + 1], ez[k], ez[k + 1]], axis=1))
    return np.concatenate(out, axis=0)


def refined_box_grid_fast(box, n, region, split=2):
    """refined_box_grid for large grids (vectorised; the same cells in the same
    order)."""
    base = box_grid(box, n)
    c = np.stack([(base[:, 0] + base[:, 1]) / 2, (base[:, 2] + base[:, 3]) / 2, (base[:, 4] + base[:, 5]) / 2], 1)
    inside = ((c[:, 0] > region[0]) & (c[:, 0] < region[1]) & (c[:, 1] > region[2]) & (c[:, 1] < region[3]) &
              (c[:, 2] > region[4]) & (c[:, 2] < region[5]))
    s3 = split ** 3
    counts = np.where(inside, s3, 1)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    out = np.empty((int(counts.sum()), 6), dtype=np.float64)
    out[first[~inside]] = base[~inside]
    rb = base[inside]
    k, j, i = np.meshgrid(np.arange(split), np.arange(split), np.arange(split), indexing="ij")
    k, j, i = k.ravel(), j.ravel(), i.ravel()
    for q in range(s3):
        lo = np.stack([i[q], j[q], k[q]]) / split
        hi = (np.stack([i[q], j[q], k[q]]) + 1) / split
        child = np.empty_like(rb)
        for a in range(3):
            w = rb[:, 2 * a + 1] - rb[:, 2 * a]
            child[:, 2 * a] = rb[:, 2 * a] + w * lo[a]
            child[:, 2 * a + 1] = rb[:, 2 * a] + w * hi[a]
        out[first[inside] + q] = child
    return out
