"""Tile-configuration cache for the forward kernel.

The measurement itself is ``fspb_autotune`` in the library (it times every
schedule x brick shape x waves-per-workgroup configuration on the plan and
keeps the fastest).  This driver stores the winner in a JSON file keyed by the GPU
architecture and a shape bucket of the plan (grid size, beam count, beamlet
count, density-correction mode), so later plans of similar size reuse it
without timing.
"""
from __future__ import annotations

import json
import os
from pathlib import Path

import torch

DEFAULT_CACHE = Path(os.environ.get("FSPB_TUNE_CACHE",
                                    Path.home() / ".cache" / "fspb" / "autotune.json"))


def _bucket(n):
    """Power-of-two bucket (1.41x steps) of a size."""
    n = max(int(n), 1)
    b = 1
    while b * 1.41 < n:
        b = int(b * 1.41) + 1
    return b


def shape_key(geo, dc: int) -> str:
    arch = torch.cuda.get_device_properties(geo.device).gcnArchName.split(":")[0]
    nz, ny, nx = geo.shape
    info = geo.info()
    return (f"{arch}|vox{_bucket(nx * ny * nz)}|beams{info['n_beams']}"
            f"|bl{_bucket(info['n_beamlets'])}|dc{dc}")


def tune(geo, fluence, cache: Path | str | None = DEFAULT_CACHE, reps: int = 3,
         force: bool = False) -> dict:
    """Applies the cached configuration for geo's bucket, or measures one."""
    dc = int(geo.info()["dc_enabled"])
    key = shape_key(geo, dc)
    path = Path(cache) if cache else None
    table = {}
    if path and path.exists():
        try:
            table = json.loads(path.read_text())
        except (OSError, ValueError):
            table = {}
    if not force and key in table:
        e = table[key]
        geo.set_schedule(e.get("per_beam", 0))
        geo.set_tile(e["shape"], e["waves_per_block"])
        return dict(e, cached=True, key=key)
    results = geo.autotune(fluence, reps=reps)
    shape, wpb = geo.get_tile()
    pb = geo.get_schedule()
    best = next(r for r in results if r["shape"] == shape and r["waves_per_block"] == wpb
                and r["per_beam"] == pb)
    entry = dict(shape=shape, waves_per_block=wpb, per_beam=pb, dims=list(best["dims"]),
                 ms=best["ms"], all=[dict(r, dims=list(r["dims"])) for r in results])
    if path:
        table[key] = entry
        path.parent.mkdir(parents=True, exist_ok=True)
        tmp = path.with_suffix(".tmp")
        tmp.write_text(json.dumps(table, indent=1))
        os.replace(tmp, path)
    return dict(entry, cached=False, key=key)
