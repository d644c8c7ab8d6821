"""FP64 reference of the 3D gamma index (the paper's evaluation, Section 2.3).

TEST INFRASTRUCTURE ONLY: the GPU library computes the gamma index with its
own kernel; this module recomputes it in float64 with NumPy, by brute force
over every offset of the search sphere, for the tests.

Definition (the readings are this build's; the paper gives the criteria
3% / 3 mm, global to the maximum reference dose, and the three statistics):
  for each voxel r of the reference grid,
    gamma(r)^2 = min( cap^2,
                      min over voxel offsets o with |o| <= cap * dd of
                          |o|^2 / dd^2 + (E(r + o) - R(r))^2 / dD^2 )
  where R is the reference dose, E the evaluated dose on the same grid,
  |o| the physical length of the offset (anisotropic voxels allowed),
  dd the distance criterion, dD = dose_frac * max(R) (or a given maximum),
  and offsets leaving the grid are skipped.  Statistics:
    gamma_max      max of gamma over the grid;
    gamma_avg_iso  mean of gamma over voxels with R >= iso_frac * max(R);
    pass_rate_iso  fraction of those voxels with gamma < 1.
"""
from __future__ import annotations

import numpy as np


def offsets(spacing, radius):
    """Integer voxel offsets (dz, dy, dx) within the sphere |o| <= radius
    (physical lengths), with their squared lengths."""
    dx, dy, dz = (float(v) for v in spacing)
    nx, ny, nz = (int(np.floor(radius / d)) for d in (dx, dy, dz))
    out = []
    for k in range(-nz, nz + 1):
        for j in range(-ny, ny + 1):
            for i in range(-nx, nx + 1):
                d2 = (i * dx) ** 2 + (j * dy) ** 2 + (k * dz) ** 2
                if d2 <= radius * radius:
                    out.append((k, j, i, d2))
    return out


def gamma(ref, ev, spacing, dist=0.3, dose_frac=0.03, cap=5.0, dose_max=None):
    """Gamma index of the evaluated dose ev against ref ([nz][ny][nx])."""
    R = np.asarray(ref, np.float64)
    E = np.asarray(ev, np.float64)
    assert R.shape == E.shape and R.ndim == 3
    dm = float(R.max()) if dose_max is None else float(dose_max)
    dD = dose_frac * dm
    best = np.full(R.shape, cap * cap)
    nz, ny, nx = R.shape
    for k, j, i, d2 in offsets(spacing, cap * dist):
        if abs(k) >= nz or abs(j) >= ny or abs(i) >= nx:
            continue                      # no voxel pair this far apart
        # r + o inside the grid: r in [max(0,-o), n - max(0,o))
        zs = slice(max(0, -k), nz - max(0, k))
        ys = slice(max(0, -j), ny - max(0, j))
        xs = slice(max(0, -i), nx - max(0, i))
        zt = slice(max(0, k), nz - max(0, -k))
        yt = slice(max(0, j), ny - max(0, -j))
        xt = slice(max(0, i), nx - max(0, -i))
        g2 = d2 / dist ** 2 + (E[zt, yt, xt] - R[zs, ys, xs]) ** 2 / dD ** 2
        np.minimum(best[zs, ys, xs], g2, out=best[zs, ys, xs])
    return np.sqrt(best)


def stats(g, ref, iso_frac=0.5, dose_max=None):
    R = np.asarray(ref, np.float64)
    dm = float(R.max()) if dose_max is None else float(dose_max)
    m = R >= iso_frac * dm
    n = int(m.sum())
    return dict(gamma_max=float(g.max()), gamma_avg_iso=float(g[m].mean()) if n else 0.0,
                pass_rate_iso=float((g[m] < 1.0).mean()) if n else 0.0, n_iso=n, dose_max=dm)
