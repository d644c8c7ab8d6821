"""Synthetic commissioned kernel tables.

The paper fits its kernel coefficients (A, u, omega, the density factors f and
the weight-drift parameter b) to Monte Carlo doses of a slab phantom
(Section 2.1); those fitted tables are not published.  These tables are
smooth stand-ins with the same roles and index variables:

* ``A[theta][t_eq]``   longitudinal factor vs radiological depth and off-axis
                       angle (Eq. 2): build-up to 1.5 cm, then exp(-0.05 t),
                       times a mild horn term (1 + 0.5 theta^2).
* ``u1x,u1y,u2x,u2y``  water penumbra steepness vs geometric depth (Eq. 3-4):
                       u1 = 1/sigma(t), sigma(t) = 0.3 + 0.02 t, u2 = u1/3.
* ``w1, w2``           water component weights vs geometric depth.
* ``fu1, fu2``         penumbra widening factors vs density (u scales with rho).
* ``fw1, fw2``         weight factors vs smoothed density.
* ``b1, b2``           weight drift per cm vs density (b2 = -b1).

All density factors equal 1 at rho = 1 and b(1) = 0, so the density
corrections vanish in water.  Seed 0 gives the nominal coefficients; a seed
s > 0 scales each coefficient by an independent U(0.9, 1.1) draw.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Table1D:
    """Uniformly sampled 1-D table: value i sits at ``start + i*step``."""
    start: float
    step: float
    values: np.ndarray  # float32 [n]

    @property
    def n(self) -> int:
        return int(self.values.shape[-1])


@dataclass
class Tables:
    """The commissioned tables of one machine/energy.

    ``A`` is a 2-D table stored row-major as [n_theta][n_t]: row r holds
    A(t_eq, theta = theta_start + r*theta_step) sampled on the depth grid of
    ``A.start``/``A.step``.  ``theta_start`` is always 0.
    """
    A: Table1D                      # values shape [n_theta, n_t]
    theta_step: float
    u1x: Table1D
    u1y: Table1D
    u2x: Table1D
    u2y: Table1D
    w1: Table1D
    w2: Table1D
    fu1: Table1D
    fu2: Table1D
    fw1: Table1D
    fw2: Table1D
    b1: Table1D
    b2: Table1D

    @property
    def n_theta(self) -> int:
        return int(self.A.values.shape[0])

    def depth_tables(self):
        return [self.u1x, self.u1y, self.u2x, self.u2y, self.w1, self.w2]

    def density_tables(self):
        return [self.fu1, self.fu2, self.fw1, self.fw2, self.b1, self.b2]


T_START, T_STEP, T_N = 0.0, 0.1, 801          # depth grid 0..80 cm
TH_STEP, TH_N = 0.01, 26                      # theta grid 0..0.25 rad
R_START, R_STEP, R_N = 0.1, 0.01, 191         # density grid 0.1..2.0


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


TABLE_COEFFS = ("mu_a", "dmax", "s0", "s1", "w_slope", "f_slope", "b_slope", "horn")


def table_coeffs(seed: int = 0) -> np.ndarray:
    """Coefficient multipliers of a machine: ones (seed 0) or U(0.9, 1.1)."""
    if seed == 0:
        return np.ones(8)
    return np.random.default_rng(seed).uniform(0.9, 1.1, size=8)


def make_tables(seed: int = 0) -> Tables:
    """Tables for the nominal machine (seed 0) or a perturbed one (seed > 0)."""
    return make_tables_coeffs(table_coeffs(seed))


def make_tables_coeffs(c) -> Tables:
    """Tables from the 8 coefficient multipliers c (TABLE_COEFFS order) of
    the nominal machine's attenuation, build-up depth, lateral-width offset
    and slope, weight slope, weight-factor slope, drift slope and horn."""
    c = np.asarray(c, dtype=np.float64)
    mu_a, dmax, s0, s1, w_slope, f_slope, b_slope, horn = (
        0.05 * c[0], 1.5 * c[1], 0.3 * c[2], 0.02 * c[3],
        0.005 * c[4], 0.2 * c[5], 0.02 * c[6], 0.5 * c[7])

    t = T_START + T_STEP * np.arange(T_N, dtype=np.float64)
    th = TH_STEP * np.arange(TH_N, dtype=np.float64)
    rho = R_START + R_STEP * np.arange(R_N, dtype=np.float64)

    a0 = np.where(
        t >= dmax,
        np.exp(-mu_a * t),
        np.exp(-mu_a * dmax) * (0.5 + 0.5 * (1.0 - (1.0 - t / dmax) ** 2)),
    )
    A = a0[None, :] * (1.0 + horn * th[:, None] ** 2)
    sigma1 = s0 + s1 * t
    u1 = 1.0 / sigma1
    u2 = 1.0 / (3.0 * sigma1)
    w1 = np.maximum(0.5, 0.85 - w_slope * t)
    w2 = 1.0 - w1

    fu = 1.0 + (rho - 1.0)                 # u proportional to density
    fw1 = 1.0 + f_slope * (rho - 1.0)
    fw2 = 1.0 - f_slope * (rho - 1.0)
    b1 = b_slope * (rho - 1.0)
    b2 = -b1

    dt = lambda v: Table1D(T_START, T_STEP, _f32(v))
    dr = lambda v: Table1D(R_START, R_STEP, _f32(v))
    return Tables(
        A=Table1D(T_START, T_STEP, _f32(A)), theta_step=TH_STEP,
        u1x=dt(u1), u1y=dt(u1), u2x=dt(u2), u2y=dt(u2), w1=dt(w1), w2=dt(w2),
        fu1=dr(fu), fu2=dr(fu), fw1=dr(fw1), fw2=dr(fw2), b1=dr(b1), b2=dr(b2),
    )


def constant_tables(A: float = 1.0, u1: float = 3.0, u2: float = 1.0,
                    w1: float = 0.8, w2: float = 0.2,
                    n_t: int = 801, t_step: float = 0.1) -> Tables:
    """Depth- and angle-independent tables with unit density factors.

    Used by invariant tests (inverse square, lateral quadrature) where the
    longitudinal and lateral parts must be constants.
    """
    ones_t = np.ones(n_t)
    ones_r = np.ones(R_N)
    dt = lambda v: Table1D(0.0, t_step, _f32(v))
    dr = lambda v: Table1D(R_START, R_STEP, _f32(v))
    return Tables(
        A=Table1D(0.0, t_step, _f32(A * np.ones((TH_N, n_t)))), theta_step=TH_STEP,
        u1x=dt(u1 * ones_t), u1y=dt(u1 * ones_t), u2x=dt(u2 * ones_t),
        u2y=dt(u2 * ones_t), w1=dt(w1 * ones_t), w2=dt(w2 * ones_t),
        fu1=dr(ones_r), fu2=dr(ones_r), fw1=dr(ones_r), fw2=dr(ones_r),
        b1=dr(0 * ones_r), b2=dr(0 * ones_r),
    )
