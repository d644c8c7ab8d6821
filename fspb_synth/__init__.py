"""Seeded synthetic inputs for the finite-size pencil beam dose engine.

This package produces *data only*: CT-like density grids, beam setups,
fluence vectors and commissioned kernel tables.  It contains none of the
dose method's arithmetic (no ray tracing, no lateral kernel, no
superposition), so both the FP64 CPU oracle and the GPU library can be fed
from it without sharing any of the method's code.

Units: cm, radians, g/cm^3 relative to water.  Density grids are float32
arrays shaped [nz][ny][nx] (x fastest).  Voxel (i, j, k) has its centre at
``origin + (i*dx, j*dy, k*dz)``.

The paper's patient CTs, Eclipse plans and Monte Carlo commissioning data
are not available; the phantoms below are stand-ins with the voxel counts,
beam counts and beamlet counts of the paper's head-and-neck and lung cases
(Table 1) and the commissioning density range 0.1-2.0 g/cm^3 (Section 2.1).
"""
from .tables import (Tables, Table1D, make_tables, make_tables_coeffs, table_coeffs, TABLE_COEFFS,
                     constant_tables)
from .plan import Beam, Options, Plan, grid_origin_centered, abi_rounded
from .phantoms import (
    plan_c1, plan_c2, plan_c3, plans_c4, plan_c4, c5_phantom, plan_c5, plan_small,
    c2_density, c3_density, slab_density, c3_objective, C3_ISO, C5_TRAIN_SEEDS, C5_HELDOUT_SEEDS,
    plan_paper_h5, plan_paper_l2, PAPER_SPACING, commissioning_plans,
)

__all__ = [
    "Tables", "Table1D", "make_tables", "make_tables_coeffs", "table_coeffs", "TABLE_COEFFS",
    "constant_tables",
    "Beam", "Options", "Plan", "grid_origin_centered", "abi_rounded",
    "plan_c1", "plan_c2", "plan_c3", "plans_c4", "plan_c4", "c5_phantom", "plan_c5",
    "C5_TRAIN_SEEDS", "C5_HELDOUT_SEEDS", "plan_paper_h5", "plan_paper_l2", "PAPER_SPACING",
    "commissioning_plans",
    "plan_small", "c2_density", "c3_density", "slab_density", "c3_objective", "C3_ISO",
]
