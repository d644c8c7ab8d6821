"""Plan containers: density grid, beams, fluences, tables and options."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

from .tables import Tables, make_tables


@dataclass
class Beam:
    """One treatment beam and its beamlet grid.

    Gantry 0 puts the source at ``iso - SAD * (0, 1, 0)`` so the beam travels
    +y; the couch angle rotates the beam about z (0 in all stock configs).
    The beamlet grid has ``nbx`` columns along the beam's x axis and ``nby``
    rows along its y axis (the patient z axis at couch 0); beamlet (n, m)
    has its centre at ``((m - (nbx-1)/2) * wx + cx, (n - (nby-1)/2) * wy + cy)``
    in the isocentre plane, and its full width at the isocentre is (wx, wy).
    """
    gantry: float
    couch: float = 0.0
    iso: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sad: float = 100.0
    nbx: int = 10
    nby: int = 10
    wx: float = 0.5
    wy: float = 0.5
    cx: float = 0.0
    cy: float = 0.0

    @property
    def n_beamlets(self) -> int:
        return self.nbx * self.nby


@dataclass
class Options:
    roi_radius: float = 5.0       # ROI cylinder radius around a beamlet axis (cm)
    rho_surface: float = 0.5      # body surface threshold on density
    smooth_sigma: float = 0.5     # Gaussian width of the smoothed density (cm)
    rho_min: float = 0.1          # commissioned density range
    rho_max: float = 2.0
    sample_step: float = 0.0      # 0 -> half the smallest voxel size
    dc_enabled: int = 1           # 1: 3D density correction, 0: plain FSPB
    siddon: int = 0               # 1: exact (Siddon) depth tables instead of uniform samples


@dataclass
class Plan:
    name: str
    density: np.ndarray                  # float32 [nz, ny, nx]
    spacing: Tuple[float, float, float]  # (dx, dy, dz)
    origin: Tuple[float, float, float]   # centre of voxel (0, 0, 0)
    beams: List[Beam]
    fluence: np.ndarray                  # float32 [n_beamlets], beam-major, row n, column m
    tables: Tables = field(default_factory=make_tables)
    options: Options = field(default_factory=Options)

    @property
    def shape(self):
        return self.density.shape

    @property
    def n_vox(self) -> int:
        return int(self.density.size)

    @property
    def n_beamlets(self) -> int:
        return int(sum(b.n_beamlets for b in self.beams))


def grid_origin_centered(n: Tuple[int, int, int], spacing: Tuple[float, float, float],
                         center=(0.0, 0.0, 0.0)) -> Tuple[float, float, float]:
    """Origin (centre of voxel 0) of an (nx, ny, nz) grid centred on ``center``."""
    return tuple(float(c - (ni - 1) * d / 2.0) for ni, d, c in zip(n, spacing, center))


def _f32(x) -> float:
    return float(np.float32(x))


def abi_rounded(plan: Plan) -> Plan:
    """The plan as the library's C interface receives it: every geometric,
    table-grid and option value that the interface passes as a 32-bit float
    (spacing, origin, beam angles, isocentre, SAD, beamlet widths and offsets,
    table starts and steps, the theta step, the option scalars) rounded to
    float32.  Arrays (density, fluence, table values) are float32 already.
    A reference that is given this plan computes on exactly the instance the
    library computes on."""
    import copy
    beams = [Beam(gantry=_f32(b.gantry), couch=_f32(b.couch), iso=tuple(_f32(v) for v in b.iso),
                  sad=_f32(b.sad), nbx=b.nbx, nby=b.nby, wx=_f32(b.wx), wy=_f32(b.wy),
                  cx=_f32(b.cx), cy=_f32(b.cy)) for b in plan.beams]
    tabs = copy.copy(plan.tables)
    for name, val in vars(plan.tables).items():
        if hasattr(val, "start") and hasattr(val, "step"):
            setattr(tabs, name, type(val)(_f32(val.start), _f32(val.step), val.values))
    tabs.theta_step = _f32(plan.tables.theta_step)
    o = copy.copy(plan.options)
    for name in ("roi_radius", "rho_surface", "smooth_sigma", "rho_min", "rho_max", "sample_step"):
        setattr(o, name, _f32(getattr(o, name)))
    return Plan(plan.name, plan.density, tuple(_f32(v) for v in plan.spacing),
                tuple(_f32(v) for v in plan.origin), beams, plan.fluence, tabs, o)
