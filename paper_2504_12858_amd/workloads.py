"""Seeded synthetic inputs for the grain-envelope step.

This module draws inputs only: nucleation sites, orientations, grain seeds and
the scalar parameters of each workload.  It holds none of the method's
arithmetic (no kinetics, no advance, no branching, no containment), so both the
HIP path and the FP64 oracle consume exactly the same arrays from it.

Random draws use numpy ``Generator(PCG64(seed))`` with a fixed draw order.

Orientation sampling follows Shoemake's uniform random rotation (Graphics Gems
III, 1992).  Nucleation undercoolings follow the normal law of the nucleation
model (Sec. 2.1.1), truncated to [0, 10] K as in the CET benchmark (Sec. 3.5,
Table S4), drawn by rejection.  Boundary nuclei get a zero nucleation
undercooling (Sec. 3.5).

Workloads (sizes in SI units):

* ``single_grain``  one cube-aligned grain whose octahedral envelope is sampled
  by the lattice points of the L1 shell of radius 50 (10 002 particles at 5 um
  spacing), uniform undercooling 5 K, 200 steps of 1e-4 s.
* ``directional``   64 grains seeded on the bottom face of a 2 x 2 x 4 mm box,
  linear undercooling field with G = 1e4 K/m along z and 10 K/s cooling.
* ``cet``           moving-source columnar-to-equiaxed workload: 4 x 2 x 1 mm
  box, Rosenthal point source plus linear background resampled onto a 256^3
  grid every step, 800 bulk nuclei (N(5, 1) K truncated to [0, 10] K) and 800
  bottom-face nuclei (zero nucleation undercooling).
* ``bicrystal``     two grains in a constant gradient (favourably oriented
  grain A versus grain B rotated 30 degrees about y).
* ``adjoint``       directional physics reduced to 16 grains, branching off
  during the differentiated window.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import Optional

import numpy as np

# Field kinds (values shared with the C headers by meaning, not by import).
FIELD_UNIFORM = 0
FIELD_LINEAR = 1
FIELD_GRID = 2
FIELD_ROSENTHAL = 3
FIELD_SOLUTE = 4


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def shoemake_quaternions(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (w, x, y, z), shape (n, 4).

    Shoemake (1992): with u1, u2, u3 ~ U[0, 1),
    q = (sqrt(1-u1) sin 2 pi u2, sqrt(1-u1) cos 2 pi u2,
         sqrt(u1) sin 2 pi u3, sqrt(u1) cos 2 pi u3).
    The components are returned in (w, x, y, z) order with w taken from the
    last entry of that tuple.
    """
    u = g.random((n, 3))
    a = np.sqrt(1.0 - u[:, 0])
    b = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    x = a * np.sin(t1)
    y = a * np.cos(t1)
    z = b * np.sin(t2)
    w = b * np.cos(t2)
    return np.stack([w, x, y, z], axis=1)


def truncated_normal(g: np.random.Generator, n: int, mu: float, sigma: float,
                     lo: float, hi: float) -> np.ndarray:
    """n draws of N(mu, sigma) restricted to [lo, hi] by rejection."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        draw = g.normal(mu, sigma, size=max(2 * (n - filled), 16))
        keep = draw[(draw >= lo) & (draw <= hi)]
        take = min(keep.size, n - filled)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def bunge_quaternion(phi1_deg: float, Phi_deg: float, phi2_deg: float) -> np.ndarray:
    """Unit quaternion (w, x, y, z) of the Bunge (z-x-z) Euler rotation that
    maps crystal axes to world axes: R = Rz(phi1) Rx(Phi) Rz(phi2)."""
    def qz(a):
        return np.array([math.cos(a / 2), 0.0, 0.0, math.sin(a / 2)])

    def qx(a):
        return np.array([math.cos(a / 2), math.sin(a / 2), 0.0, 0.0])

    def qmul(p, q):
        w1, x1, y1, z1 = p
        w2, x2, y2, z2 = q
        return np.array([
            w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
            w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
            w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
            w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
        ])

    r = math.radians
    return qmul(qmul(qz(r(phi1_deg)), qx(r(Phi_deg))), qz(r(phi2_deg)))


def axis_angle_quaternion(axis, angle_deg: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    h = math.radians(angle_deg) / 2
    return np.array([math.cos(h), *(math.sin(h) * a)])


@dataclass
class Field:
    kind: int
    dT: float = 0.0                      # UNIFORM
    dT0: float = 0.0                     # LINEAR / ROSENTHAL background
    grad: tuple = (0.0, 0.0, 0.0)        # d(dT)/dx [K/m]
    rate: float = 0.0                    # d(dT)/dt [K/s]
    # GRID / ROSENTHAL sampling grid (node-centred)
    n: tuple = (0, 0, 0)
    origin: tuple = (0.0, 0.0, 0.0)
    spacing: tuple = (0.0, 0.0, 0.0)
    data: Optional[np.ndarray] = None    # GRID values, float32, shape (nz, ny, nx)
    # ROSENTHAL source
    q: float = 0.0                       # power / conductivity [K m]
    U: float = 0.0                       # travel speed [m/s]
    alpha: float = 0.0                   # thermal diffusivity [m^2/s]
    x_start: float = 0.0                 # raster limits along x [m]
    x_end: float = 0.0
    ys: float = 0.0                      # source y, z [m]
    zs: float = 0.0
    r_min: float = 0.0                   # distance floor [m]
    dT_min: float = -1000.0              # undercooling floor [K]
    # SOLUTE: node temperature [K] and solute concentration, float64, shape
    # (nz, ny, nx); liquidus T_L(w) = liq_T + liq_m w
    T: Optional[np.ndarray] = None
    w: Optional[np.ndarray] = None
    liq_T: float = 0.0
    liq_m: float = 0.0


@dataclass
class Workload:
    name: str
    lo: tuple
    hi: tuple
    lambda0: float
    h: float
    rc: float
    a: tuple
    b: tuple
    theta: float
    dt: float
    n_steps: int
    field: Field
    branching: int = 1
    box_exit: int = 1
    periodic: int = 0       # bit a: axis a periodic with period hi - lo (Sec. 3.4)
    grain_centre: np.ndarray = dc_field(default_factory=lambda: np.zeros((0, 3)))
    grain_quat: np.ndarray = dc_field(default_factory=lambda: np.zeros((0, 4)))
    grain_shell: np.ndarray = dc_field(default_factory=lambda: np.zeros((0,), np.int32))
    site_xyz: np.ndarray = dc_field(default_factory=lambda: np.zeros((0, 3)))
    site_dTn: np.ndarray = dc_field(default_factory=lambda: np.zeros((0,)))
    site_quat: np.ndarray = dc_field(default_factory=lambda: np.zeros((0, 4)))
    notes: str = ""

    @property
    def box_size(self) -> float:
        return max(h - l for l, h in zip(self.lo, self.hi))


# Kinetics of the benchmark workloads: v = 1e-5 dT^2 + 1e-6 dT^3 (Eq. 2 with
# exponents 2 and 3).
KIN_A = (1e-5, 1e-6)
KIN_B = (2.0, 3.0)


def single_grain(shell_r: int = 50, n_steps: int = 200) -> Workload:
    """One cube-aligned grain at the centre of a 1 mm cube, envelope sampled on
    the L1 shell of radius ``shell_r`` lattice steps (lambda0 = 5 um)."""
    return Workload(
        name="single_grain", lo=(0.0, 0.0, 0.0), hi=(1e-3, 1e-3, 1e-3),
        lambda0=5e-6, h=10e-6, rc=5e-6, a=KIN_A, b=KIN_B, theta=0.0,
        dt=1e-4, n_steps=n_steps, field=Field(FIELD_UNIFORM, dT=5.0),
        grain_centre=np.array([[5e-4, 5e-4, 5e-4]]),
        grain_quat=np.array([[1.0, 0.0, 0.0, 0.0]]),
        grain_shell=np.array([shell_r], np.int32))


def nucleus_uniform(lambda0: float = 5e-6, dT: float = 5.0, quat=None) -> Workload:
    """One 6-point nucleus in a uniformly undercooled 1 mm cube."""
    q = np.array([1.0, 0, 0, 0]) if quat is None else np.asarray(quat, float)
    return Workload(
        name="nucleus_uniform", lo=(0.0, 0.0, 0.0), hi=(1e-3, 1e-3, 1e-3),
        lambda0=lambda0, h=lambda0, rc=lambda0, a=KIN_A, b=KIN_B, theta=0.0,
        dt=1e-4, n_steps=0, field=Field(FIELD_UNIFORM, dT=dT),
        grain_centre=np.array([[5e-4, 5e-4, 5e-4]]), grain_quat=q[None, :],
        grain_shell=np.array([0], np.int32))


# Undercooling at the cold face at t = 0 of the directional workload: a knob
# of the configuration (its other values are fixed), chosen so that about 2M
# particles are stored after 2000 steps of 5e-5 s (64 grains: 1.0M at 14 K,
# 2.45M at 18 K, measured on the HIP path).
DIRECTIONAL_DT0 = 17.0


def directional(seed: int = 2, n_grains: int = 64, size=(2e-3, 2e-3, 4e-3),
                lambda0: float = 5e-6, dT0: float = DIRECTIONAL_DT0, G: float = 1e4,
                rate: float = 10.0, dt: float = 5e-5, n_steps: int = 2000,
                h: Optional[float] = None) -> Workload:
    """Directional competitive growth: grains on the bottom face, linear field
    dT = dT0 - G z + rate t."""
    g = rng(seed)
    xy = g.random((n_grains, 2)) * np.array(size[:2])
    centre = np.column_stack([xy, np.zeros(n_grains)])
    quat = shoemake_quaternions(g, n_grains)
    return Workload(
        name="directional", lo=(0.0, 0.0, 0.0), hi=tuple(size),
        lambda0=lambda0, h=lambda0 if h is None else h, rc=lambda0, a=KIN_A, b=KIN_B, theta=0.0,
        dt=dt, n_steps=n_steps,
        field=Field(FIELD_LINEAR, dT0=dT0, grad=(0.0, 0.0, -G), rate=rate),
        grain_centre=centre, grain_quat=quat,
        grain_shell=np.zeros(n_grains, np.int32),
        notes=f"seed={seed}")


# Binary alloy of the solute-coupled workloads (Al-Cu-like): melting point of
# the pure solvent [K] and liquidus slope [K per wt%].
LIQ_T, LIQ_M = 933.5, -3.4


@dataclass
class SoluteSpec:
    """Temperature and solute node values of a solute-coupled field: an
    imposed temperature T = T_L(w0) - dT0 + G z - rate t and a static lateral
    segregation pattern w = w0 + amp sin(2 pi x / period) sin(2 pi y / period)
    (the local undercooling is taken with respect to the local liquidus,
    Sec. 3.4)."""
    n: tuple
    origin: tuple
    spacing: tuple
    dT0: float
    G: float
    rate: float
    w0: float
    amp: float
    period: float

    def field(self, t: float) -> Field:
        nx, ny, nz = self.n
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        x = self.origin[0] + i * self.spacing[0]
        y = self.origin[1] + j * self.spacing[1]
        z = self.origin[2] + k * self.spacing[2]
        T = (LIQ_T + LIQ_M * self.w0) - self.dT0 + self.G * z - self.rate * t
        w = self.w0 + self.amp * np.sin(2 * np.pi * x / self.period) * np.sin(2 * np.pi * y / self.period)
        return Field(FIELD_SOLUTE, n=tuple(self.n), origin=tuple(self.origin),
                     spacing=tuple(self.spacing), T=np.ascontiguousarray(T, np.float64),
                     w=np.ascontiguousarray(w, np.float64), liq_T=LIQ_T, liq_m=LIQ_M)


def directional_solute(seed: int = 2, n_grains: int = 8, size=(0.3e-3, 0.3e-3, 0.6e-3),
                       lambda0: float = 5e-6, dT0: float = 10.0, G: float = 1e4,
                       rate: float = 10.0, w0: float = 3.0, amp: float = 0.3,
                       period: float = 1e-4, grid=(16, 16, 32), dt: float = 5e-4,
                       n_steps: int = 240, h: Optional[float] = None):
    """Directional growth (grains on the bottom face) under a temperature and
    solute field on a node grid spanning the box; returns the workload (field
    at t = 0) and the spec that gives the field at any time."""
    w = directional(seed=seed, n_grains=n_grains, size=size, lambda0=lambda0, dT0=dT0, G=G,
                    rate=rate, dt=dt, n_steps=n_steps, h=h)
    spacing = tuple(s / (m - 1) for s, m in zip(size, grid))
    spec = SoluteSpec(n=tuple(grid), origin=(0.0, 0.0, 0.0), spacing=spacing, dT0=dT0, G=G,
                      rate=rate, w0=w0, amp=amp, period=period)
    w.field = spec.field(0.0)
    w.name = "directional_solute"
    return w, spec


def cet(seed: int = 3, size=(4e-3, 2e-3, 1e-3), lambda0: float = 2e-6,
        dT0: float = 4.0, G: float = 1e4, rate: float = 10.0,
        bulk_density: float = 1e11, face_density: float = 1e8,
        dTn_mu: float = 5.0, dTn_sigma: float = 1.0, grid_n: int = 256,
        U: float = 0.05, alpha: float = 4.9e-6, q: float = 0.0264,
        dt: float = 5e-5, n_steps: int = 4000, h: Optional[float] = None) -> Workload:
    """Columnar-to-equiaxed transition under a moving Rosenthal source.

    Bulk nuclei: round(density * volume) sites, uniform iid positions,
    N(dTn_mu, dTn_sigma) truncated to [0, 10] K, Shoemake orientations.
    Face nuclei: round(face_density * area) sites on z = 0 with zero
    nucleation undercooling.
    """
    g = rng(seed)
    size = np.asarray(size, float)
    vol = float(np.prod(size))
    n_bulk = int(round(bulk_density * vol))
    n_face = int(round(face_density * size[0] * size[1]))
    bulk_xyz = g.random((n_bulk, 3)) * size
    bulk_dTn = truncated_normal(g, n_bulk, dTn_mu, dTn_sigma, 0.0, 10.0)
    bulk_q = shoemake_quaternions(g, n_bulk)
    face_xy = g.random((n_face, 2)) * size[:2]
    face_xyz = np.column_stack([face_xy, np.zeros(n_face)])
    face_q = shoemake_quaternions(g, n_face)
    # Face nuclei first so that the columnar population gets the low grain ids.
    xyz = np.concatenate([face_xyz, bulk_xyz])
    dTn = np.concatenate([np.zeros(n_face), bulk_dTn])
    quat = np.concatenate([face_q, bulk_q])
    spacing = tuple(float(s) / (grid_n - 1) for s in size)
    fld = Field(FIELD_ROSENTHAL, dT0=dT0, grad=(0.0, 0.0, -G), rate=rate,
                n=(grid_n, grid_n, grid_n), origin=(0.0, 0.0, 0.0), spacing=spacing,
                q=q, U=U, alpha=alpha, x_start=0.0, x_end=float(size[0]),
                ys=float(size[1]) / 2, zs=float(size[2]), r_min=min(spacing),
                dT_min=-1000.0)
    return Workload(
        name="cet", lo=(0.0, 0.0, 0.0), hi=tuple(size), lambda0=lambda0,
        h=lambda0 if h is None else h, rc=lambda0, a=KIN_A, b=KIN_B, theta=0.0, dt=dt,
        n_steps=n_steps, field=fld, site_xyz=xyz, site_dTn=dTn, site_quat=quat,
        notes=f"seed={seed} n_face={n_face} n_bulk={n_bulk}")


def bicrystal(lambda0: float = 20e-6, dt: float = 2e-3, n_steps: int = 400,
              size=(1e-3, 0.2e-3, 2e-3), G: float = 1e4, rate: float = 10.0,
              dT0: float = 2.0) -> Workload:
    """Grain A cube-aligned at x = size/4, grain B rotated 30 deg about y at
    x = 3 size/4, both on the bottom face, linear field dT0 - G z + rate t."""
    qa = np.array([1.0, 0.0, 0.0, 0.0])
    qb = axis_angle_quaternion((0, 1, 0), 30.0)
    centre = np.array([[size[0] / 4, size[1] / 2, 0.0], [3 * size[0] / 4, size[1] / 2, 0.0]])
    return Workload(
        name="bicrystal", lo=(0.0, 0.0, 0.0), hi=tuple(size), lambda0=lambda0,
        h=lambda0, rc=lambda0, a=KIN_A, b=KIN_B, theta=0.0, dt=dt,
        n_steps=n_steps,
        field=Field(FIELD_LINEAR, dT0=dT0, grad=(0.0, 0.0, -G), rate=rate),
        grain_centre=centre, grain_quat=np.stack([qa, qb]),
        grain_shell=np.zeros(2, np.int32))


def random_cloud_state(seed: int, n_grains: int, n_per_grain: int, box: float,
                       lambda0: float, spread: float = 0.25):
    """A synthetic post-branch particle state for containment tests: grains
    with random centres and orientations, particles at random lattice sites
    within ``spread * box`` of the centre with random direction and travel.

    Returns (centre, quat, grain, site, dir, s) arrays.
    """
    g = rng(seed)
    centre = box * (0.25 + 0.5 * g.random((n_grains, 3)))
    quat = shoemake_quaternions(g, n_grains)
    m = int(round(spread * box / lambda0))
    grain = np.repeat(np.arange(n_grains, dtype=np.int32), n_per_grain)
    site = g.integers(-m, m + 1, size=(grain.size, 3)).astype(np.int32)
    d = g.integers(0, 6, size=grain.size).astype(np.int32)
    s = g.random(grain.size) * lambda0
    return centre, quat, grain, site, d, s
