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
