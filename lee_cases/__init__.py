"""Seeded, synthetic input descriptions shared by the GPU library and the oracle.

This module only *describes* problems: grid sizes, wall geometry, impedance
parameters, initial pulses, sources and probe positions, as plain numbers.  It
holds none of the method's arithmetic (no mask, ghost, least-squares, ADE or
stencil code): both the HIP library and the FP64 oracle read these numbers and
compute everything else on their own.

The workloads restate the paper's three validation cases (flat immersed wall,
Sec. 4.1; cylinder reflecting a pulse, Sec. 4.2; cylinder scattering a
harmonic monopole, Sec. 4.3) at the grid sizes and parameters of the
benchmark configurations, plus the batched and served random mixes.  Wall
normals are stored as doubles so both sides use bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Plain description records
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class Wall:
    """Immersed wall.  kind: "none", "line" or "circle".

    line:   passes through (cx, cy); (nx, ny) is the unit normal pointing into
            the fluid (fluid is where (x-c).n > 0).
    circle: centre (cx, cy), radius rc; fluid outside.
    """

    kind: str = "none"
    cx: float = 0.0
    cy: float = 0.0
    nx: float = 0.0
    ny: float = 0.0
    rc: float = 0.0


@dataclass(frozen=True)
class Impedance:
    """Wall condition. kind: "rigid", "msd" (mass M, resistance R, stiffness K
    per unit area, Sec. 2.5) or "poles": a wall admittance given in the
    multi-pole form of Sec. 2.3 (eq. Yrational) without a direct term,
    real = ((lambda_k, A_k), ...) for the real poles and
    pairs = ((alpha_k, beta_k, B_k, C_k), ...) for the pole pairs
    s_k = alpha_k +- i beta_k with residues B_k +- i C_k (at most 8 states:
    one per real pole, two per pair)."""

    kind: str = "rigid"
    R: float = 0.0
    M: float = 0.0
    K: float = 0.0
    real: tuple = ()
    pairs: tuple = ()


@dataclass(frozen=True)
class Pulse:
    """Gaussian pressure pulse p0 = a exp(-ln2 |x-xs|^2 / w^2), u0 = v0 = 0
    (Sec. 4.2)."""

    xs: float
    ys: float
    a: float
    w: float


@dataclass(frozen=True)
class Packet:
    """Plane wave packet travelling along the unit vector (dx, dy) (Sec. 4.1):
    with s = (x-xs)dx + (y-ys)dy,
    p0 = a/2 exp(-alpha^2 s^2) cos(2 pi k s), (u0, v0) = p0 (dx, dy)."""

    xs: float
    ys: float
    dx: float
    dy: float
    a: float
    alpha: float
    k: float


@dataclass(frozen=True)
class Monopole:
    """Harmonic monopole s = a exp(-ln2 |x-xs|^2/w^2) sin(omega t) (Sec. 4.3)."""

    xs: float
    ys: float
    a: float
    w: float
    omega: float


@dataclass(frozen=True)
class Case:
    """One solve on a uniform grid x_i = x0 + i h, y_j = y0 + j h,
    0 <= i < nx, 0 <= j < ny."""

    nx: int
    ny: int
    x0: float
    y0: float
    h: float
    H: int = 5                     # DRP half-width: 5 (11-point) or 3 (7-point)
    cfl: float = 0.5               # dt = cfl * h  (c0 = 1)
    filter_sigma: float = 0.2      # selective-filter strength; 0 disables it
    filter_explicit: bool = False  # the filter once per step (q -= sigma F q) instead of in each stage's RHS
    sponge_cells: int = 0          # width of the outer damping layer
    sponge_sigma: float = 0.0      # peak damping rate at the domain edge
    wall: Wall = Wall()
    impedance: Impedance = Impedance()
    ic: Optional[object] = None    # Pulse | Packet | None
    source: Optional[Monopole] = None
    steps: int = 0
    probes: Tuple[Tuple[float, float], ...] = ()
    dft_steps: int = 0             # running DFT over the final dft_steps steps
    radiation: bool = False        # radiation condition in the outer band of H nodes
    rad_center: Tuple[float, float] = (0.0, 0.0)   # its centre (x, y)
    name: str = ""

    @property
    def dt(self) -> float:
        return self.cfl * self.h

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


def line_normal(angle_deg: float) -> Tuple[float, float]:
    """Unit normal (pointing to the fluid side) of a wall inclined angle_deg to
    the x axis: (-sin, cos)."""
    t = math.radians(angle_deg)
    return (-math.sin(t), math.cos(t))


# --------------------------------------------------------------------------
# The five benchmark workloads
# --------------------------------------------------------------------------

#: grid-unit reading of the flat-wall impedance (R, m, k) = (1, 0.05, 20):
#: the values are taken in the physical units of the 1/64 grid, so in grid
#: units M_g = 64 m, K_g = k / 64, R_g = R.
FLAT_IMPEDANCE_GRID = Impedance("msd", R=1.0, M=0.05 * 64.0, K=20.0 / 64.0)
#: the literal reading, which makes the ADE unstable under RK4 at dt = 0.5.
FLAT_IMPEDANCE_LITERAL = Impedance("msd", R=1.0, M=0.05, K=20.0)


def flat_wall_201(steps: int = 500, impedance: Impedance = FLAT_IMPEDANCE_GRID) -> Case:
    """Flat immersed wall, 201^2, dx = 1, wall through the centre at 30 deg,
    Gaussian pulse (a = 1e-3, half-width 3 dx) centred 20 dx from the wall."""
    nx_, ny_ = line_normal(30.0)
    return Case(
        nx=201, ny=201, x0=-100.0, y0=-100.0, h=1.0, H=5, cfl=0.5,
        filter_sigma=0.2,
        wall=Wall("line", 0.0, 0.0, nx_, ny_),
        impedance=impedance,
        ic=Pulse(20.0 * nx_, 20.0 * ny_, 1e-3, 3.0),
        steps=steps,
        probes=((10.0 * nx_, 10.0 * ny_), (30.0 * nx_ + 15.0, 30.0 * ny_)),
        name="flat-wall-201",
    )


def cylinder_pulse_1024(steps: int = 4000, n: int = 1024) -> Case:
    """Cylinder reflecting a pulse: n^2 on [-8, 8)^2, r_c = 0.5 with its centre
    shifted by (0.3 h, 0.3 h), pulse at (4, 0) (a = 1e-3, w = 0.2), impedance
    (R, m, k) = (0.5, 0.02, 10), 8 probes on r = 5."""
    h = 16.0 / n
    probes = tuple((5.0 * math.cos(j * math.pi / 4), 5.0 * math.sin(j * math.pi / 4))
                   for j in range(8))
    return Case(
        nx=n, ny=n, x0=-8.0, y0=-8.0, h=h, H=5, cfl=0.5, filter_sigma=0.2,
        wall=Wall("circle", 0.3 * h, 0.3 * h, rc=0.5),
        impedance=Impedance("msd", R=0.5, M=0.02, K=10.0),
        ic=Pulse(4.0, 0.0, 1e-3, 0.2),
        steps=steps, probes=probes, name=f"cylinder-pulse-{n}",
    )


def monopole_4096(steps: int = 20000, n: int = 4096) -> Case:
    """Cylinder scattering a harmonic monopole: n^2 on [-16, 16)^2, r_c = 1,
    monopole at (4, 0), omega = 4 pi, half-width 3 h, impedance
    (R, m, k) = (1, 0.01, 5) (two real poles), 64-cell sponge, amplitudes by a
    running DFT over the last 10 periods on rings r = 1.1 and r = 5."""
    h = 32.0 / n
    omega = 2.0 * math.pi * 2.0
    rings = []
    for r in (1.1, 5.0):
        for j in range(180):
            t = 2.0 * math.pi * j / 180.0
            rings.append((r * math.cos(t), r * math.sin(t)))
    dt = 0.5 * h
    steps_per_period = int(round(2.0 * math.pi / omega / dt))
    return Case(
        nx=n, ny=n, x0=-16.0, y0=-16.0, h=h, H=5, cfl=0.5, filter_sigma=0.2,
        sponge_cells=64, sponge_sigma=15.0 / (64 * h),
        wall=Wall("circle", 0.0, 0.0, rc=1.0),
        impedance=Impedance("msd", R=1.0, M=0.01, K=5.0),
        source=Monopole(4.0, 0.0, 1.0, 3.0 * h, omega),
        steps=steps, probes=tuple(rings), dft_steps=10 * steps_per_period,
        name=f"monopole-{n}",
    )


def _loguniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def random_impedance(rng) -> Impedance:
    """R, m, k log-uniform on [0.1, 10], [0.001, 0.1], [1, 100]."""
    R = _loguniform(rng, 0.1, 10.0)
    M = _loguniform(rng, 0.001, 0.1)
    K = _loguniform(rng, 1.0, 100.0)
    return Impedance("msd", R=R, M=M, K=K)


def random_cylinder(rng, side: int, steps: int) -> Case:
    """A cylinder-pulse instance on [-8, 8)^2 with a random radius in
    [0.3, 1.5] and a random impedance.  The pulse half-width is
    max(0.2, 3 h) so that coarse grids still resolve it."""
    h = 16.0 / side
    rc = float(rng.uniform(0.3, 1.5))
    imp = random_impedance(rng)
    return Case(
        nx=side, ny=side, x0=-8.0, y0=-8.0, h=h, H=5, cfl=0.5, filter_sigma=0.2,
        wall=Wall("circle", 0.3 * h, 0.3 * h, rc=rc), impedance=imp,
        ic=Pulse(4.0, 0.0, 1e-3, max(0.2, 3.0 * h)), steps=steps,
        probes=((5.0, 0.0), (0.0, 5.0), (-5.0, 0.0), (0.0, -5.0)),
        name=f"rand-cyl-{side}",
    )


def random_flat(rng, side: int, steps: int) -> Case:
    """A flat-wall instance on [-8, 8)^2: wall through the centre at a random
    angle in [0, 180) deg, pulse of half-width 3 h centred 20 h from the wall."""
    h = 16.0 / side
    ang = float(rng.uniform(0.0, 180.0))
    nx_, ny_ = line_normal(ang)
    imp = random_impedance(rng)
    return Case(
        nx=side, ny=side, x0=-8.0, y0=-8.0, h=h, H=5, cfl=0.5, filter_sigma=0.2,
        wall=Wall("line", 0.0, 0.0, nx_, ny_), impedance=imp,
        ic=Pulse(20.0 * h * nx_, 20.0 * h * ny_, 1e-3, 3.0 * h), steps=steps,
        probes=((10.0 * h * nx_, 10.0 * h * ny_), (30.0 * h * nx_, 30.0 * h * ny_)),
        name=f"rand-flat-{side}-{ang:.1f}",
    )


def batch_candidates(seed: int = 2609, steps: int = 2000):
    """Endless stream of batched cylinder-pulse candidates: side drawn from
    {128, 256, 512, 1024}.  The consumer keeps the first 256 that its own
    impedance checks accept (critical damping and RK4 stability of the ADE)."""
    rng = np.random.default_rng(seed)
    while True:
        side = int(rng.choice([128, 256, 512, 1024]))
        yield random_cylinder(rng, side, steps)


def request_stream(seed: int = 26091, rate: float = 50.0, duration: float = 120.0):
    """Poisson request arrivals: yields (arrival_time, Case candidate).  Each
    request is a flat-wall or cylinder case with probability 1/2, side uniform
    in [256, 2048], steps uniform in [1000, 5000]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            return
        side = int(rng.integers(256, 2049))
        steps = int(rng.integers(1000, 5001))
        if rng.uniform() < 0.5:
            yield t, random_flat(rng, side, steps)
        else:
            yield t, random_cylinder(rng, side, steps)


def small_cylinder(n: int = 96, steps: int = 40, impedance: Optional[Impedance] = None,
                   filter_sigma: float = 0.2, H: int = 5) -> Case:
    """A reduced cylinder-pulse case the oracle finishes in seconds (several
    tiles and a ragged tail)."""
    h = 16.0 / n
    return Case(
        nx=n, ny=n + 7, x0=-8.0, y0=-8.0 - 3 * h, h=h, H=H, cfl=0.5,
        filter_sigma=filter_sigma,
        wall=Wall("circle", 0.3 * h, 0.3 * h, rc=1.3),
        impedance=impedance if impedance is not None else Impedance("msd", R=0.5, M=0.2, K=10.0),
        ic=Pulse(1.9, 0.4, 1e-3, 0.5), steps=steps,
        probes=((2.5, 0.0), (0.0, 2.5), (-3.0, -1.0)),
        name=f"small-cyl-{n}",
    )


def coarse_cylinder(n: int = 28, rc: float = 4.0, dx: float = 0.0, dy: float = 0.0,
                    impedance: Optional[Impedance] = None, H: int = 5,
                    filter_sigma: float = 0.2) -> Case:
    """A cylinder of radius rc grid units (dx = 1) in an n x n grid centred on
    the origin, its centre shifted by (dx, dy); no initial field, no source.
    Small enough for the step map to be assembled and its eigenvalues found
    densely; the shift moves the nodes near the points where the wall is
    tangent to the grid lines."""
    c0 = -0.5 * (n - 1)
    return Case(
        nx=n, ny=n, x0=c0, y0=c0, h=1.0, H=H, cfl=0.5, filter_sigma=filter_sigma,
        wall=Wall("circle", dx, dy, rc=rc),
        impedance=impedance if impedance is not None else Impedance(),
        steps=0, name=f"coarse-cylinder-{n}-{rc:g}-{dx:g}-{dy:g}",
    )


def radiating_cylinder(n: int = 96, steps: int = 120, impedance: Optional[Impedance] = None,
                       H: int = 5, filter_sigma: float = 0.2) -> Case:
    """A reduced cylinder-pulse case truncated by the radiation condition
    instead of the zero frame (Sec. 4.2 uses non-reflecting conditions on
    all four sides): n x (n + 7) nodes on [-8, 8) in x, cylinder r_c = 1.3,
    pulse (a = 1e-3, w = 0.5) at (3, 1), radiation centre at the origin."""
    h = 16.0 / n
    return Case(
        nx=n, ny=n + 7, x0=-8.0, y0=-8.0 - 3 * h, h=h, H=H, cfl=0.5,
        filter_sigma=filter_sigma,
        wall=Wall("circle", 0.3 * h, 0.3 * h, rc=1.3),
        impedance=impedance if impedance is not None else Impedance("msd", R=0.5, M=0.2, K=10.0),
        ic=Pulse(3.0, 1.0, 1e-3, 0.5), steps=steps,
        probes=((5.0, 0.0), (0.0, 6.5), (-7.5, -7.0)),
        radiation=True, rad_center=(0.0, 0.0),
        name=f"radiating-cylinder-{n}",
    )


def paper_cylinder_pulse(steps: int = 400) -> Case:
    """The paper's own cylinder-pulse configuration (Sec. 4.2): [-6, 6]^2 at
    h = 0.04 (301^2 nodes), cylinder r_c = 0.5 at the origin, Gaussian pulse
    of amplitude 1 and half-width 0.2 at (4, 0), mass-spring-damper wall
    (M, K, R) = (0.025, 1.6, 0.2), CFL 0.5, the paper's scheme (7-point DRP,
    no filter) and the non-reflecting condition on all four sides (centre at
    the origin).  Probes on r = 2."""
    return Case(
        nx=301, ny=301, x0=-6.0, y0=-6.0, h=0.04, H=3, cfl=0.5, filter_sigma=0.0,
        wall=Wall("circle", 0.0, 0.0, rc=0.5),
        impedance=Impedance("msd", R=0.2, M=0.025, K=1.6),
        ic=Pulse(4.0, 0.0, 1.0, 0.2), steps=steps,
        probes=((2.0, 0.0), (0.0, 2.0), (-2.0, 0.0), (0.0, -2.0)),
        radiation=True, rad_center=(0.0, 0.0),
        name="paper-cylinder-pulse-301",
    )


def paper_monopole(steps: int = 1500, h: float = 0.02) -> Case:
    """The paper's harmonic-monopole configuration (Sec. 4.3): [-6, 6]^2 at
    h = 0.02 (601^2 nodes), cylinder r_c = 0.5 at the origin, monopole of
    amplitude 1 and half-width 0.2 at (4, 0) driven at omega = 8 pi, wall
    (M, K, R) = (0.025, 15.79, 1) (resonance at 8 pi), CFL 0.5, the paper's
    scheme (7-point DRP, no filter) and the non-reflecting condition on all
    four sides; t_end = 15 and a running DFT over the last two time units
    (eight periods, the paper's window [13, 15]) on rings r = 0.6 (the
    nearest ring whose probe stencils stay in the fluid at this h; the
    paper's is 0.55) and r = 5, 72 points each."""
    n = int(round(12.0 / h)) + 1
    omega = 8.0 * math.pi
    rings = []
    for r in (0.6, 5.0):
        for j in range(72):
            t = 2.0 * math.pi * (j + 0.5) / 72.0
            rings.append((r * math.cos(t), r * math.sin(t)))
    return Case(
        nx=n, ny=n, x0=-6.0, y0=-6.0, h=h, H=3, cfl=0.5, filter_sigma=0.0,
        wall=Wall("circle", 0.0, 0.0, rc=0.5),
        impedance=Impedance("msd", R=1.0, M=0.025, K=15.79),
        source=Monopole(4.0, 0.0, 1.0, 0.2, omega), steps=steps, probes=tuple(rings),
        dft_steps=int(round(2.0 / (0.5 * h))), radiation=True, rad_center=(0.0, 0.0),
        name="paper-monopole-601",
    )


def named(name: str) -> Case:
    table = {
        "flat-wall-201": flat_wall_201,
        "cylinder-pulse-1024": cylinder_pulse_1024,
        "monopole-4096": monopole_4096,
    }
    return table[name]()
