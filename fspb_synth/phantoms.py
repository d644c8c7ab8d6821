"""Seeded phantoms and plans for the five workload configurations.

C1  64^3 water cube at 0.25 cm with a lung slab (rho 0.25, depth 4-7 cm) and
    a bone slab (rho 1.8, depth 10-11 cm); one beam, 10x10 beamlets of 0.5 cm.
C2  128x128x96 head-and-neck-like phantom at 0.25 cm; 7 coplanar beams at
    51.4 degree steps, 20x20 beamlets each; fluence U[0,1] with 30% zeros.
C3  256x256x128 thorax-like phantom at 0.2 cm; 9 beams at 40 degree steps,
    30x30 beamlets each; fluence lognormal(0, 0.5).
C4  32 plans of uneven size (grids 96^3 to 256x256x160 at 2-3 mm, 5-9 beams,
    15^2 to 34^2 beamlets per beam), slab or head phantoms by parity.
C5  C2 geometry with per-seed random heads (surrogate training/held-out sets).

The sizes mirror the paper's clinical cases (Table 1: 128x128x72-103 voxels,
637-10,369 beamlets) and its 0.1-2.0 g/cm^3 commissioning range.  Every draw
comes from ``numpy.random.default_rng(seed)`` in a fixed order (structures
first, then per-voxel noise, then fluences).
"""
from __future__ import annotations

import math
from typing import Callable, List, Sequence, Tuple

import numpy as np

from .plan import Beam, Options, Plan, grid_origin_centered
from .tables import Tables, make_tables

AIR = 0.001


def _centers(n, spacing, origin):
    nx, ny, nz = n
    x = origin[0] + spacing[0] * np.arange(nx)
    y = origin[1] + spacing[1] * np.arange(ny)
    z = origin[2] + spacing[2] * np.arange(nz)
    return np.meshgrid(z, y, x, indexing="ij")  # each [nz, ny, nx]: Z, Y, X


def slab_density(n=(64, 64, 64), spacing=(0.25, 0.25, 0.25),
                 slabs=((-4.0, -1.0, 0.25), (2.0, 3.0, 1.8)), base=1.0,
                 origin=None) -> np.ndarray:
    """Water box with slabs perpendicular to y: voxels whose centre y lies in
    (y_lo, y_hi) get the slab density."""
    if origin is None:
        origin = grid_origin_centered(n, spacing)
    Z, Y, X = _centers(n, spacing, origin)
    rho = np.full(Y.shape, base, dtype=np.float64)
    for lo, hi, r in slabs:
        rho[(Y > lo) & (Y < hi)] = r
    return rho.astype(np.float32)


def _fluence_zeros(rng, n, zero_frac=0.3):
    f = rng.uniform(0.0, 1.0, size=n)
    zero = rng.uniform(0.0, 1.0, size=n) < zero_frac
    f[zero] = 0.0
    return f.astype(np.float32)


def plan_c1(tables: Tables | None = None) -> Plan:
    n, sp = (64, 64, 64), (0.25, 0.25, 0.25)
    origin = grid_origin_centered(n, sp)
    rho = slab_density(n, sp, origin=origin)
    beams = [Beam(gantry=0.0, nbx=10, nby=10, wx=0.5, wy=0.5)]
    f = np.ones(100, dtype=np.float32)
    return Plan("c1_slab64", rho, sp, origin, beams, f, tables or make_tables(0), Options())


def _random_unit_ball(rng) -> np.ndarray:
    while True:
        p = rng.uniform(-1.0, 1.0, size=3)
        if p @ p <= 1.0:
            return p


def c2_density(seed: int, n=(128, 128, 96), spacing=(0.25, 0.25, 0.25),
               semi=(8.0, 10.0, 10.5), center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Head-like phantom: soft-tissue ellipsoid N(1.03, 0.02), bone shell
    U(1.5, 1.9) at normalised radius 0.88-0.94, six air ellipsoids, air outside."""
    rng = np.random.default_rng(seed)
    origin = grid_origin_centered(n, spacing)
    cav = []
    for _ in range(6):
        ax = rng.uniform(0.5, 1.5, size=3)
        c = _random_unit_ball(rng) * 0.6 * np.asarray(semi) + np.asarray(center)
        cav.append((c, ax))
    Z, Y, X = _centers(n, spacing, origin)
    r = np.sqrt(((X - center[0]) / semi[0]) ** 2 + ((Y - center[1]) / semi[1]) ** 2
                + ((Z - center[2]) / semi[2]) ** 2)
    tissue = rng.normal(1.03, 0.02, size=X.shape)
    bone = rng.uniform(1.5, 1.9, size=X.shape)
    rho = np.full(X.shape, AIR)
    inside = r <= 1.0
    rho[inside] = tissue[inside]
    shell = (r >= 0.88) & (r <= 0.94)
    rho[shell] = bone[shell]
    for c, ax in cav:
        e = ((X - c[0]) / ax[0]) ** 2 + ((Y - c[1]) / ax[1]) ** 2 + ((Z - c[2]) / ax[2]) ** 2
        rho[(e <= 1.0) & inside] = AIR
    return rho.astype(np.float32)


def plan_c2(seed: int = 2, tables: Tables | None = None) -> Plan:
    n, sp = (128, 128, 96), (0.25, 0.25, 0.25)
    origin = grid_origin_centered(n, sp)
    rho = c2_density(seed, n, sp)
    rng = np.random.default_rng(seed + 10_000)
    beams = [Beam(gantry=math.radians(51.4 * k), nbx=20, nby=20) for k in range(7)]
    f = _fluence_zeros(rng, sum(b.n_beamlets for b in beams))
    return Plan("c2_head128", rho, sp, origin, beams, f, tables or make_tables(0), Options())


C3_ISO = (7.5, -1.0, 0.0)


def c3_density(seed: int = 3, n=(256, 256, 128), spacing=(0.2, 0.2, 0.2)) -> np.ndarray:
    """Thorax-like phantom (elliptic body along z, lungs, spine, tumour)."""
    rng = np.random.default_rng(seed)
    origin = grid_origin_centered(n, spacing)
    Z, Y, X = _centers(n, spacing, origin)
    lung_noise = rng.uniform(0.15, 0.35, size=X.shape)
    rho = np.full(X.shape, AIR)
    body = (X / 17.0) ** 2 + (Y / 12.0) ** 2 <= 1.0
    inner = (X / 15.5) ** 2 + (Y / 10.5) ** 2 <= 1.0
    rho[body] = 1.0                       # body, chest wall and mediastinum
    for cx in (-7.5, 7.5):
        lung = (((X - cx) / 6.0) ** 2 + ((Y + 0.5) / 8.5) ** 2 <= 1.0) & inner
        rho[lung] = lung_noise[lung]
    spine = (X ** 2 + (Y - 8.0) ** 2) <= 1.5 ** 2
    rho[spine] = 1.6
    tumour = ((X - C3_ISO[0]) ** 2 + (Y - C3_ISO[1]) ** 2 + (Z - C3_ISO[2]) ** 2) <= 1.5 ** 2
    rho[tumour] = 1.0
    return rho.astype(np.float32)


def plan_c3(seed: int = 3, tables: Tables | None = None) -> Plan:
    n, sp = (256, 256, 128), (0.2, 0.2, 0.2)
    origin = grid_origin_centered(n, sp)
    rho = c3_density(seed, n, sp)
    rng = np.random.default_rng(seed + 10_000)
    beams = [Beam(gantry=math.radians(40.0 * k), iso=C3_ISO, nbx=30, nby=30) for k in range(9)]
    nb = sum(b.n_beamlets for b in beams)
    f = rng.lognormal(0.0, 0.5, size=nb).astype(np.float32)
    return Plan("c3_lung256", rho, sp, origin, beams, f, tables or make_tables(0), Options())


def c3_objective(seed: int, n_vox: int):
    """Voxel weights w ~ U[0,1] and a unit-scale target u ~ U[0,1] (the
    target dose is u times the plan's maximum dose)."""
    rng = np.random.default_rng(seed + 20_000)
    w = rng.uniform(0.0, 1.0, size=n_vox).astype(np.float32)
    u = rng.uniform(0.0, 1.0, size=n_vox).astype(np.float32)
    return w, u


def plan_c4(p: int, tables: Tables | None = None) -> Plan:
    """Plan p (0..31) of the uneven batch."""
    rng = np.random.default_rng(4000 + p)
    nx, ny = (int(v) for v in rng.integers(96, 257, size=2))
    nz = int(rng.integers(96, 161))
    d = float(rng.uniform(0.2, 0.3))
    if p == 0:
        nx = ny = nz = 96
    if p == 31:
        nx, ny, nz = 256, 256, 160
    n, sp = (nx, ny, nz), (d, d, d)
    origin = grid_origin_centered(n, sp)
    n_b = int(rng.integers(5, 10))
    start = float(rng.uniform(0.0, 2.0 * math.pi))
    nbl = int(rng.integers(15, 35))
    beams = [Beam(gantry=(start + 2.0 * math.pi * k / n_b) % (2.0 * math.pi),
                  nbx=nbl, nby=nbl) for k in range(n_b)]
    seed = int(rng.integers(0, 2**31 - 1))
    if p % 2 == 0:
        ly = ny * d
        face = -ly / 2.0
        snap = lambda depth: face + round(depth * ly / 16.0 / d) * d
        slabs = ((snap(4.0), snap(7.0), 0.25), (snap(10.0), snap(11.0), 1.8))
        rho = slab_density(n, sp, slabs=slabs, origin=origin)
    else:
        semi = (0.8 * nx * d / 2.0 * 0.85, 0.8 * ny * d / 2.0, 0.8 * nz * d / 2.0)
        rho = c2_density(seed, n, sp, semi=semi)
    f = _fluence_zeros(np.random.default_rng(seed + 1), sum(b.n_beamlets for b in beams))
    return Plan(f"c4_plan{p:02d}", rho, sp, origin, beams, f, tables or make_tables(0), Options())


def plans_c4(indices: Sequence[int] | None = None, tables: Tables | None = None) -> List[Plan]:
    idx = range(32) if indices is None else indices
    t = tables or make_tables(0)
    return [plan_c4(p, t) for p in idx]


def c5_phantom(seed: int) -> np.ndarray:
    """Random head on the C2 grid (surrogate training seeds 1000-1199,
    held-out seeds 2000-2009)."""
    return c2_density(seed)


C5_TRAIN_SEEDS = range(1000, 1200)
C5_HELDOUT_SEEDS = range(2000, 2010)


def plan_c5(seed: int, tables: Tables | None = None) -> Plan:
    """C2 geometry (7 beams of 20 x 20 beamlets, 128 x 128 x 96 grid) on the
    random head of `seed`, fluences as for C2."""
    p = plan_c2(seed, tables)
    p.name = f"c5_head_{seed}"
    return p


def commissioning_plans(tables: Tables | None = None, scale: int = 1) -> List[Plan]:
    """Measurement set for fitting the commissioned tables: a water tank
    (depth doses, profiles and the off-axis horn of a 14 cm field of 1 cm
    beamlets) and a slab phantom (lung and bone slabs: the density factors
    and the weight drift).  scale = 2 halves the voxel size."""
    t = tables or make_tables(0)
    sp = (0.5 / scale,) * 3
    n_w = (40 * scale, 40 * scale, 30 * scale)
    water = Plan("tank", np.ones((n_w[2], n_w[1], n_w[0]), np.float32), sp,
                 grid_origin_centered(n_w, sp), [Beam(gantry=0.0, nbx=14, nby=14, wx=1.0, wy=1.0)],
                 np.ones(196, np.float32), t, Options())
    n_s = (32 * scale, 40 * scale, 32 * scale)
    o_s = grid_origin_centered(n_s, sp)
    slab = Plan("slabs", slab_density(n_s, sp, slabs=((-6.0, -3.0, 0.25), (1.0, 2.0, 1.8)),
                                      origin=o_s), sp, o_s,
                [Beam(gantry=0.0, nbx=8, nby=8, wx=0.5, wy=0.5)], np.ones(64, np.float32), t,
                Options())
    return [water, slab]


# Paper-shaped plans (Table 1 scales): CT down-sampled to 0.4 x 0.4 x 0.25 cm,
# beamlets of 0.2 x 0.5 cm (0.2 along the beam's x axis, the leaf motion).
PAPER_SPACING = (0.4, 0.4, 0.25)


def plan_paper_h5(seed: int = 5, tables: Tables | None = None) -> Plan:
    """Head-and-neck case shaped like H5: 128 x 128 x 72 voxels, 7
    non-coplanar beams (couch 0, +-20, +-30, +-15 degrees), 40 x 37 beamlets
    each (10,360 in all, H5 has 10,369), fluence U[0,1] with 30% zeros."""
    n = (128, 128, 72)
    origin = grid_origin_centered(n, PAPER_SPACING)
    rho = c2_density(seed, n, PAPER_SPACING, semi=(8.0, 10.0, 8.5))
    rng = np.random.default_rng(seed + 10_000)
    couch = (0.0, 20.0, -20.0, 30.0, -30.0, 15.0, -15.0)
    beams = [Beam(gantry=math.radians(51.4 * k), couch=math.radians(couch[k]), nbx=40, nby=37,
                  wx=0.2, wy=0.5) for k in range(7)]
    f = _fluence_zeros(rng, sum(b.n_beamlets for b in beams))
    return Plan("paper_h5_like", rho, PAPER_SPACING, origin, beams, f, tables or make_tables(0),
                Options())


def plan_paper_l2(seed: int = 6, tables: Tables | None = None) -> Plan:
    """Lung case shaped like L2: 128 x 128 x 103 voxels, 6 coplanar beams at
    60 degree steps on the right-lung target, 26 x 11 beamlets each (1,716 in
    all, L2 has 1,720), fluence U[0,1] with 30% zeros."""
    n = (128, 128, 103)
    origin = grid_origin_centered(n, PAPER_SPACING)
    rho = c3_density(seed, n, PAPER_SPACING)
    rng = np.random.default_rng(seed + 10_000)
    beams = [Beam(gantry=math.radians(60.0 * k), iso=C3_ISO, nbx=26, nby=11, wx=0.2, wy=0.5)
             for k in range(6)]
    f = _fluence_zeros(rng, sum(b.n_beamlets for b in beams))
    return Plan("paper_l2_like", rho, PAPER_SPACING, origin, beams, f, tables or make_tables(0),
                Options())


def plan_small(n=(24, 20, 16), spacing=(0.25, 0.25, 0.25), density=1.0,
               beams: Sequence[Beam] | None = None, fluence=None,
               tables: Tables | None = None, options: Options | None = None,
               origin=None, seed: int = 0, name: str = "small") -> Plan:
    """Small plan for tests.  ``density`` is a scalar, an array [nz, ny, nx]
    or a callable (Z, Y, X) -> array evaluated at voxel centres."""
    if origin is None:
        origin = grid_origin_centered(n, spacing)
    if callable(density):
        Z, Y, X = _centers(n, spacing, origin)
        rho = np.asarray(density(Z, Y, X), dtype=np.float32)
    elif np.isscalar(density):
        rho = np.full((n[2], n[1], n[0]), float(density), dtype=np.float32)
    else:
        rho = np.ascontiguousarray(density, dtype=np.float32)
    if beams is None:
        beams = [Beam(gantry=0.0, nbx=4, nby=4)]
    nb = sum(b.n_beamlets for b in beams)
    if fluence is None:
        fluence = np.random.default_rng(seed).uniform(0.2, 1.0, size=nb)
    fluence = np.ascontiguousarray(fluence, dtype=np.float32)
    return Plan(name, rho, tuple(spacing), tuple(origin), list(beams), fluence,
                tables or make_tables(0), options or Options())
