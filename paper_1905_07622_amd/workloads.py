"""Seeded synthetic inputs for the transient heat-flow workloads.

This module only draws random numbers and lays out arrays: grids, per-element
coefficient fields, boundary-condition descriptions, initial fields and sensor
points.  It holds none of the finite element arithmetic, so both the HIP path
and the CPU oracle can be fed from it without sharing any of the method.

Conventions (stated once, used everywhere):

* A grid has ``nx*ny*nz`` hexahedral elements with spacing ``h`` per axis and
  origin 0.  Nodes are numbered ``i = ix + (nx+1)*(iy + (ny+1)*iz)`` (x
  fastest, as in the paper's fixed-grid mesh, Sec. 4.1) and elements
  ``e = ex + nx*(ey + ny*ez)``.  Numpy arrays are therefore shaped
  ``(nz, ny, nx)`` for elements and ``(nz+1, ny+1, nx+1)`` for nodes before
  being flattened in C order.
* Spacing is cubic, ``h = 1/max(nx, ny, nz)``, so the largest edge of the
  domain has length 1.
* Faces are numbered 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.  "Bottom" is z=0 (face 4)
  and "top" is z=max (face 5).
* Membership of an element in a sphere or ellipsoid is decided at its
  centroid with ``<=``.
* Every random draw comes from ``numpy.random.Generator(PCG64)``; where a
  workload needs two independent streams they are the two children of
  ``SeedSequence(seed).spawn(2)``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = range(6)


def face_bit(face: int) -> int:
    return 1 << face


@dataclasses.dataclass
class Problem:
    """One forward simulation: grid, coefficients, boundary data and run controls."""

    name: str
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    k_e: np.ndarray          # (E,) float64 conductivity per element
    rhoc_e: np.ndarray       # (E,) float64 heat capacity per element
    T0: np.ndarray           # (N,) float64 initial field
    dt: float
    theta: float
    nsteps: int
    rtol: float
    dirichlet_mask: int = 0
    dirichlet_value: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(6))
    flux_mask: int = 0
    flux: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(6))
    flux_schedule: Optional[np.ndarray] = None   # s_n for n = 1..len; None means 1 always
    sensors: Optional[np.ndarray] = None         # (S, 3) float64 points
    seed: Optional[int] = None
    element: int = 0                             # 0: trilinear hexahedra; 1: six linear tetrahedra per box

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_elems(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# geometry helpers (index layout only)
# ----------------------------------------------------------------------------

def cubic_spacing(nx: int, ny: int, nz: int) -> float:
    return 1.0 / max(nx, ny, nz)


def element_centroids(nx, ny, nz, hx, hy, hz):
    """Centroid coordinates of every element, each shaped (nz, ny, nx)."""
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (ex + 0.5) * hx, (ey + 0.5) * hy, (ez + 0.5) * hz


def node_coords(nx, ny, nz, hx, hy, hz):
    iz, iy, ix = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return ix * hx, iy * hy, iz * hz


def sensor_grid(m: int, lx: float, ly: float, z: float) -> np.ndarray:
    """m*m points ((i+1/2)/m*lx, (j+1/2)/m*ly, z), sensor index i + m*j."""
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    pts = np.stack([((i + 0.5) / m * lx).ravel(), ((j + 0.5) / m * ly).ravel(),
                    np.full(m * m, z)], axis=1)
    return np.ascontiguousarray(pts, dtype=np.float64)


def _streams(seed: int, n: int = 2) -> List[np.random.Generator]:
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


# ----------------------------------------------------------------------------
# coefficient fields
# ----------------------------------------------------------------------------

def lognormal_field(nx, ny, nz, rng: np.random.Generator) -> np.ndarray:
    """k_e = exp(Z_e): Z_e is the 3x3x3 box sum of i.i.d. N(0,1) draws W,
    clipped to the grid and divided by sqrt(count), so each Z_e is exactly
    N(0,1) and neighbours within 3 elements are correlated."""
    w = rng.standard_normal((nz, ny, nx))
    wp = np.pad(w, 1)
    cp = np.pad(np.ones_like(w), 1)
    s = np.zeros_like(w)
    c = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                s += wp[dz:dz + nz, dy:dy + ny, dx:dx + nx]
                c += cp[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    return np.exp(s / np.sqrt(c)).ravel()


def spheres_field(nx, ny, nz, h, rng: np.random.Generator):
    """Two-phase field: matrix k=1, rho*c=1; spheres of one inclusion
    conductivity k ~ U[2,50] (rho*c = 1).  Draw order: k_inc, target volume
    fraction phi ~ U[0.05,0.3], then per sphere centre (3 uniforms in the box)
    and radius U[0.05,0.15]; spheres are added until the element volume
    fraction first reaches phi."""
    k_inc = rng.uniform(2.0, 50.0)
    phi = rng.uniform(0.05, 0.3)
    cx, cy, cz = element_centroids(nx, ny, nz, h, h, h)
    lx, ly, lz = nx * h, ny * h, nz * h
    inside = np.zeros((nz, ny, nx), dtype=bool)
    n_spheres = 0
    while inside.mean() < phi and n_spheres < 10000:
        c = rng.uniform(0.0, 1.0, 3) * np.array([lx, ly, lz])
        r = rng.uniform(0.05, 0.15)
        inside |= (cx - c[0]) ** 2 + (cy - c[1]) ** 2 + (cz - c[2]) ** 2 <= r * r
        n_spheres += 1
    k = np.where(inside, k_inc, 1.0).ravel()
    return k, np.ones(nx * ny * nz), dict(k_inc=k_inc, phi=phi, n_spheres=n_spheres,
                                           fraction=float(inside.mean()))


# ----------------------------------------------------------------------------
# the workload configurations
# ----------------------------------------------------------------------------

def two_phase_sphere_cube(n: int = 16) -> Problem:
    """16^3 unit cube, centred sphere r=0.25 with k=10, rho*c=2 inside a
    k=1, rho*c=1 matrix; T0=1; T=0 on z=0, insulated elsewhere; backward
    Euler, dt=1e-3, 20 steps, rtol 1e-10."""
    h = cubic_spacing(n, n, n)
    cx, cy, cz = element_centroids(n, n, n, h, h, h)
    inside = ((cx - 0.5) ** 2 + (cy - 0.5) ** 2 + (cz - 0.5) ** 2 <= 0.25 ** 2).ravel()
    k = np.where(inside, 10.0, 1.0)
    rhoc = np.where(inside, 2.0, 1.0)
    N = (n + 1) ** 3
    return Problem(name=f"sphere{n}", nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, k_e=k, rhoc_e=rhoc,
                   T0=np.ones(N), dt=1e-3, theta=1.0, nsteps=20, rtol=1e-10,
                   dirichlet_mask=face_bit(FACE_ZM))


def lognormal_cube(n: int = 100, seed: int = 2, nsteps: int = 200) -> Problem:
    """n^3 unit cube with log-normal k_e (box-filtered, seeded) and
    rho*c_e ~ U[0.8,1.2] from a second stream; q=1 on the top face, T=0 on
    the bottom, T0=0; Crank-Nicolson, dt=5e-4, rtol 1e-8."""
    h = cubic_spacing(n, n, n)
    g1, g2 = _streams(seed)
    k = lognormal_field(n, n, n, g1)
    rhoc = g2.uniform(0.8, 1.2, n * n * n)
    flux = np.zeros(6)
    flux[FACE_ZP] = 1.0
    return Problem(name=f"lognormal{n}", nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, k_e=k, rhoc_e=rhoc,
                   T0=np.zeros((n + 1) ** 3), dt=5e-4, theta=0.5, nsteps=nsteps, rtol=1e-8,
                   dirichlet_mask=face_bit(FACE_ZM), flux_mask=face_bit(FACE_ZP), flux=flux,
                   seed=seed)


def defect_slab(nx: int = 200, ny: int = 200, nz: int = 25, seed: int = 3,
                n_defects: int = 20, nsteps: int = 300, pulse_steps: int = 10,
                n_sensor: int = 16) -> Problem:
    """Slab [0,1]^2 x [0,nz*h] (h = 1/200): k=1 in the bottom 5 element layers
    and k=5 above; 20 axis-aligned ellipsoidal defects (centres uniform in the
    slab, semi-axes U[2,8]*h drawn per axis, k=0.01, overriding the layers);
    rho*c=1; T0=0; flux q=1 on the top face for the first 10 steps, all faces
    otherwise insulated; backward Euler, dt=1e-3, rtol 1e-8; a 16x16 sensor
    grid on the top face."""
    h = cubic_spacing(nx, ny, nz)
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy, cz = element_centroids(nx, ny, nz, h, h, h)
    k = np.where(cz < 5 * h, 1.0, 5.0)
    lx, ly, lz = nx * h, ny * h, nz * h
    for _ in range(n_defects):
        c = rng.uniform(0.0, 1.0, 3) * np.array([lx, ly, lz])
        a = rng.uniform(2.0, 8.0, 3) * h
        inside = ((cx - c[0]) / a[0]) ** 2 + ((cy - c[1]) / a[1]) ** 2 + ((cz - c[2]) / a[2]) ** 2 <= 1.0
        k = np.where(inside, 0.01, k)
    flux = np.zeros(6)
    flux[FACE_ZP] = 1.0
    sched = np.zeros(nsteps)
    sched[:pulse_steps] = 1.0
    return Problem(name=f"slab{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, hx=h, hy=h, hz=h,
                   k_e=k.ravel().astype(np.float64), rhoc_e=np.ones(nx * ny * nz),
                   T0=np.zeros((nx + 1) * (ny + 1) * (nz + 1)), dt=1e-3, theta=1.0,
                   nsteps=nsteps, rtol=1e-8, flux_mask=face_bit(FACE_ZP), flux=flux,
                   flux_schedule=sched, sensors=sensor_grid(n_sensor, lx, ly, lz), seed=seed)


# The paper's performance workload (Sec. 5.1): a two-layer laminate
# [-15,15] x [-15,15] x [0,10] (mm), unit flux on the face x3 = 0, the other
# faces insulated, T0 = 0; layer x3 <= 5 mild steel, above it iron oxide,
# with the heat capacities and conductivities as printed; 50 Crank-Nicolson
# steps of dt = 0.01, rtol 1e-6.  Its mesh sizes give 10.5k to 2.00M nodes
# for n = 30 to 180 divisions across (n/3 through the thickness).
LAMINATE_RHOC = (3.724e6, 1.65e6)
LAMINATE_K = (4.9e8, 4e6)


def laminate(n: int = 30, nsteps: int = 50, element: int = 1) -> Problem:
    """The two-layer laminate on an n x n x n/3 grid of cubes of side 30/n
    (origin at the prism's corner), material by element centroid
    (x3 <= 5: steel), six tetrahedra per cube by default (the paper's element)."""
    assert n % 3 == 0
    nz = n // 3
    h = 30.0 / n
    _, _, cz = element_centroids(n, n, nz, h, h, h)
    steel = cz <= 5.0
    k = np.where(steel, LAMINATE_K[0], LAMINATE_K[1]).ravel().astype(np.float64)
    rhoc = np.where(steel, LAMINATE_RHOC[0], LAMINATE_RHOC[1]).ravel().astype(np.float64)
    flux = np.zeros(6)
    flux[FACE_ZM] = 1.0
    return Problem(name=f"laminate{n}", nx=n, ny=n, nz=nz, hx=h, hy=h, hz=h, k_e=k, rhoc_e=rhoc,
                   T0=np.zeros((n + 1) * (n + 1) * (nz + 1)), dt=0.01, theta=0.5, nsteps=nsteps, rtol=1e-6,
                   dirichlet_mask=0, flux_mask=face_bit(FACE_ZM), flux=flux, element=element)


def sphere_proposal(s: int, n: int = 48, nsteps: int = 100) -> Problem:
    """One simulation of the batched proposal workload: n^3 unit cube,
    random-sphere two-phase field from seed 4000+s, T0=1, T=0 on z=0,
    backward Euler, dt=1e-3, rtol 1e-8."""
    seed = 4000 + s
    h = cubic_spacing(n, n, n)
    rng = np.random.Generator(np.random.PCG64(seed))
    k, rhoc, _ = spheres_field(n, n, n, h, rng)
    return Problem(name=f"proposal{s}", nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, k_e=k, rhoc_e=rhoc,
                   T0=np.ones((n + 1) ** 3), dt=1e-3, theta=1.0, nsteps=nsteps, rtol=1e-8,
                   dirichlet_mask=face_bit(FACE_ZM), seed=seed)


SERVE_EDGES = (32, 48, 64, 96, 128)


def serve_request(i: int) -> Problem:
    """Request i of the serving stream (seed 5001+i): edge from
    {32,48,64,96,128}, log-normal or two-phase field (p=1/2), theta in
    {0.5,1} (p=1/2), steps U{50..300}; dt=1e-3, rtol 1e-8; boundary data and
    T0 as the sphere cube (T0=1, T=0 on z=0)."""
    seed = 5001 + i
    g_meta, g_field = _streams(seed)
    n = int(g_meta.choice(SERVE_EDGES))
    lognormal = bool(g_meta.integers(0, 2) == 0)
    theta = 0.5 if g_meta.integers(0, 2) == 0 else 1.0
    nsteps = int(g_meta.integers(50, 301))
    h = cubic_spacing(n, n, n)
    if lognormal:
        gk, gr = _streams(seed + 1_000_000)
        k = lognormal_field(n, n, n, gk)
        rhoc = gr.uniform(0.8, 1.2, n ** 3)
    else:
        k, rhoc, _ = spheres_field(n, n, n, h, g_field)
    return Problem(name=f"request{i}", nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, k_e=k, rhoc_e=rhoc,
                   T0=np.ones((n + 1) ** 3), dt=1e-3, theta=theta, nsteps=nsteps, rtol=1e-8,
                   dirichlet_mask=face_bit(FACE_ZM), seed=seed)


def poisson_arrivals(n: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of n requests at Poisson rate `rate`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))


def random_problem(nx, ny, nz, seed, *, hx=None, hy=None, hz=None, theta=1.0, dt=1e-3,
                   nsteps=3, rtol=1e-10, dirichlet_mask=face_bit(FACE_ZM), flux_mask=0,
                   flux=None, dirichlet_value=None, k_range=(0.1, 10.0),
                   rhoc_range=(0.5, 2.0), zero_k_fraction=0.0, random_T0=True) -> Problem:
    """Small test problem with i.i.d. uniform coefficients and a random T0."""
    g = np.random.Generator(np.random.PCG64(seed))
    h = cubic_spacing(nx, ny, nz)
    hx = h if hx is None else hx
    hy = h if hy is None else hy
    hz = h if hz is None else hz
    E = nx * ny * nz
    N = (nx + 1) * (ny + 1) * (nz + 1)
    k = g.uniform(*k_range, E)
    if zero_k_fraction > 0:
        k[g.uniform(0, 1, E) < zero_k_fraction] = 0.0
    rhoc = g.uniform(*rhoc_range, E)
    T0 = g.uniform(-1.0, 1.0, N) if random_T0 else np.ones(N)
    return Problem(name=f"random{nx}x{ny}x{nz}s{seed}", nx=nx, ny=ny, nz=nz, hx=hx, hy=hy, hz=hz,
                   k_e=k, rhoc_e=rhoc, T0=T0, dt=dt, theta=theta, nsteps=nsteps, rtol=rtol,
                   dirichlet_mask=dirichlet_mask,
                   dirichlet_value=np.zeros(6) if dirichlet_value is None else np.asarray(dirichlet_value, float),
                   flux_mask=flux_mask, flux=np.zeros(6) if flux is None else np.asarray(flux, float),
                   seed=seed)


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, n)


# ----------------------------------------------------------------------------
# coefficient-inverse stand-in (Section 5.4): corroded plate, camera, draws
# ----------------------------------------------------------------------------

PLATE_L = (1.0, 0.5, 0.125)      # plate extent; the front (heated, observed) face is z = 0.125
CHANNEL_Y, CHANNEL_W = 0.25, 0.15  # corrosion channel: apex line y = 0.25, zero depth at 0.25 +- 0.15
K_CORRODED = 0.01                # k and rho*c of corroded material (steel: 1)


def corroded_plate(depth: float, n: int = 32, nsteps: int = 30, pulse_steps: int = 15, flux: float = 40.0,
                   camera=(16, 8)) -> Problem:
    """Stand-in for the paper's corroded plate (its gusset geometry exists only in a missing figure):
    the plate [0,1] x [0,0.5] x [0,0.125] on n x n/2 x n/8 cubic elements, k = rho*c = 1, corroded from
    the back face z = 0 along a channel that is constant in x and parabolic in y, penetrating `depth` at
    its apex (y = 0.25) and nothing at |y - 0.25| >= 0.15.  Corroded material has k = rho*c = 0.01; an
    element mixes the two by the share of its z-extent below the profile at its centroid, so the
    coefficients move continuously with depth.  The front face is heated with q = `flux` for the first
    `pulse_steps` steps (insulated otherwise, like every other face); backward Euler, dt = 1e-3,
    rtol 1e-8; camera pixels (mx x my) centred on the front face."""
    nx, ny, nz = n, n // 2, max(1, n // 8)
    h = PLATE_L[0] / nx
    cx, cy, cz = element_centroids(nx, ny, nz, h, h, h)
    prof = depth * np.maximum(0.0, 1.0 - ((cy - CHANNEL_Y) / CHANNEL_W) ** 2)
    frac = np.clip((prof - (cz - 0.5 * h)) / h, 0.0, 1.0)
    k = (1.0 - frac) * 1.0 + frac * K_CORRODED
    flux_v = np.zeros(6)
    flux_v[FACE_ZP] = flux
    sched = np.zeros(nsteps)
    sched[:pulse_steps] = 1.0
    mx, my = camera
    j, i = np.meshgrid(np.arange(my), np.arange(mx), indexing="ij")
    cam = np.stack([((i + 0.5) / mx * PLATE_L[0]).ravel(), ((j + 0.5) / my * PLATE_L[1]).ravel(),
                    np.full(mx * my, nz * h)], axis=1)
    return Problem(name=f"plate{nx}x{ny}x{nz}_d{depth:.4f}", nx=nx, ny=ny, nz=nz, hx=h, hy=h, hz=h,
                   k_e=k.ravel().astype(np.float64), rhoc_e=k.ravel().astype(np.float64).copy(),
                   T0=np.zeros((nx + 1) * (ny + 1) * (nz + 1)), dt=1e-3, theta=1.0, nsteps=nsteps,
                   rtol=1e-8, flux_mask=face_bit(FACE_ZP), flux=flux_v, flux_schedule=sched,
                   sensors=np.ascontiguousarray(cam, dtype=np.float64))


def mh_draws(seed: int, n_iter: int, n_chains: int):
    """Random numbers of n_chains Metropolis-Hastings chains over n_iter iterations: standard normals for
    the random-walk proposals and U[0,1) for the acceptance tests, each (n_iter, n_chains)."""
    g1, g2 = _streams(seed, 2)
    return g1.standard_normal((n_iter, n_chains)), g2.uniform(0.0, 1.0, (n_iter, n_chains))


def camera_noise(seed: int, n_pixels: int) -> np.ndarray:
    """Standard normal draws for the camera's per-pixel noise."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n_pixels)
