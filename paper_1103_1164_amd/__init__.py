"""MI355X (gfx950) finite-size pencil beam dose engine with 3D density
correction -- Python binding of libfspb.

    geo = Geometry.from_plan(plan)          # Algorithm A2 steps 1-5 on the GPU
    dose = geo.forward(fluence)             # Eq. 1 (kernel 5)
    grad = geo.adjoint(voxel_weight)        # transpose of Eq. 1
    dose = FspbDose.apply(fluence, geo)     # autograd: backward = adjoint

``plan`` is any object with the attributes density [nz,ny,nx], spacing,
origin, beams (gantry, couch, iso, sad, nbx, nby, wx, wy, cx, cy), tables and
options (see ``fspb_synth``).  Device memory and streams come from PyTorch;
all computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FspbError, check, load

__all__ = ["Geometry", "Batch", "Mlp", "FspbDose", "FspbError", "gamma_index", "load",
           "set_log_level"]


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f32(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    return t.contiguous()


_TABLE_NAMES = ("A", "u1x", "u1y", "u2x", "u2y", "w1", "w2", "fu1", "fu2", "fw1", "fw2", "b1", "b2")
_table_cache: dict = {}


def _marshal_tables(tables):
    """The ctypes view of a tables object.  Views are cached per identity of
    every table and value array (and the scalar fields), so a replaced table
    or array is marshalled afresh; the library compares table contents
    itself before reusing packed tables."""
    key = (int(tables.n_theta), float(tables.theta_step)) + tuple(
        (id(t), id(t.values), float(t.start), float(t.step))
        for t in (getattr(tables, n) for n in _TABLE_NAMES))
    hit = _table_cache.get(key)
    if hit is not None:
        return hit[0]
    keep = [tables]

    def tab(t):
        v = np.ascontiguousarray(t.values, dtype=np.float32)
        keep.append((t, t.values, v))
        return _lib.fspb_table1d(float(t.start), float(t.step), int(v.shape[-1]),
                                 v.ctypes.data_as(C.POINTER(C.c_float)))

    tabs = _lib.fspb_tables(tab(tables.A), int(tables.n_theta), float(tables.theta_step),
                            *[tab(getattr(tables, n)) for n in _TABLE_NAMES[1:]])
    if len(_table_cache) >= 16:
        _table_cache.pop(next(iter(_table_cache)))
    _table_cache[key] = (tabs, keep)      # keep: the objects whose ids form the key stay alive
    return tabs


def set_log_level(level: int) -> int:
    """Library diagnostics on stderr (0 none, 1 errors, 2 plan-level events,
    3 the forwards, adjoints, inferences and replays queued; see
    fspb_set_log_level); returns the previous level."""
    return int(load().fspb_set_log_level(int(level)))


def drift_tables(tables):
    """(1, ratio) when the commissioned b2 is ratio * b1 at every sample (the
    corrected pairs then read one weight-drift table), else (2, 0.0).  A host
    call of the library; no device needed."""
    r = C.c_float()
    n = load().fspb_drift_tables(C.byref(_marshal_tables(tables)), C.byref(r))
    check(n if n < 0 else 0, "fspb_drift_tables")
    return n, r.value


class Geometry:
    """A plan's geometry on the GPU (owning handle of libfspb)."""

    def __init__(self, density: torch.Tensor, spacing, origin, beams, tables, options=None,
                 stream=None, tile=None, schedule=None):
        L = load()
        if not (isinstance(density, torch.Tensor) and density.is_cuda):
            raise TypeError("density must be a CUDA (HIP) tensor")
        density = density.to(torch.float32).contiguous()
        self._density = density          # the CT the tables were traced through
        self.device = density.device
        nz, ny, nx = density.shape
        self.shape = (nz, ny, nx)
        ct = _lib.fspb_ct(nx, ny, nz, *map(float, spacing), *map(float, origin),
                          C.c_void_p(density.data_ptr()))
        bs = (_lib.fspb_beam * len(beams))()
        for k, b in enumerate(beams):
            bs[k] = _lib.fspb_beam(float(b.gantry), float(b.couch),
                                   (C.c_float * 3)(*map(float, b.iso)), float(b.sad),
                                   int(b.nbx), int(b.nby), float(b.wx), float(b.wy),
                                   float(b.cx), float(b.cy))
        tabs = _marshal_tables(tables)
        opt_p = None
        if options is not None or tile is not None or schedule is not None:
            # zero fields take the library's defaults; tile = (shape, waves
            # per workgroup) and schedule (0 bricks, 1 per-beam items) build
            # that forward schedule at creation
            opt = _lib.fspb_options()
            opt.dc_enabled = 1
            if options is not None:
                o = options
                opt.roi_radius, opt.rho_surface = float(o.roi_radius), float(o.rho_surface)
                opt.smooth_sigma, opt.rho_min = float(o.smooth_sigma), float(o.rho_min)
                opt.rho_max, opt.sample_step = float(o.rho_max), float(o.sample_step)
                opt.dc_enabled = int(o.dc_enabled)
                opt.flags = _lib.FSPB_FLAG_SIDDON if getattr(o, "siddon", 0) else 0
            if tile is not None:
                opt.tile_shape, opt.tile_waves = int(tile[0]), int(tile[1])
            if schedule is not None:
                opt.schedule = int(schedule)
            opt_p = C.byref(opt)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fspb_create_geometry(C.byref(ct), len(beams), bs, C.byref(tabs), opt_p,
                                         _stream(stream), C.byref(h)), "fspb_create_geometry")
        self._h = h
        self.n_beamlets = int(sum(int(b.nbx) * int(b.nby) for b in beams))
        self.n_vox = nx * ny * nz
        self.n_beams = len(beams)

    @classmethod
    def from_plan(cls, plan, device="cuda", dc_enabled: Optional[int] = None, stream=None,
                  tile=None, schedule=None):
        dens = torch.as_tensor(np.ascontiguousarray(plan.density, dtype=np.float32), device=device)
        opts = plan.options
        if dc_enabled is not None:
            import copy
            opts = copy.copy(opts)
            opts.dc_enabled = int(dc_enabled)
        return cls(dens, plan.spacing, plan.origin, plan.beams, plan.tables, opts, stream, tile,
                   schedule)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            load().fspb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if not self._h:
            raise FspbError(_lib.FSPB_E_STATE, "geometry is closed")
        return self._h

    # -- dose ---------------------------------------------------------------
    def forward(self, fluence: torch.Tensor, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
        f = _dev_f32(fluence, self.device)
        if f.numel() != self.n_beamlets:
            raise ValueError(f"fluence has {f.numel()} values, plan has {self.n_beamlets} beamlets")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        check(load().fspb_forward(self._handle(), C.c_void_p(f.data_ptr()),
                                  C.c_void_p(out.data_ptr()), _stream(stream)), "fspb_forward")
        return out

    def adjoint(self, voxel_weight: torch.Tensor, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
        w = _dev_f32(voxel_weight, self.device)
        if w.numel() != self.n_vox:
            raise ValueError(f"voxel weight has {w.numel()} values, grid has {self.n_vox}")
        if out is None:
            out = torch.empty(self.n_beamlets, dtype=torch.float32, device=self.device)
        check(load().fspb_adjoint(self._handle(), C.c_void_p(w.data_ptr()),
                                  C.c_void_p(out.data_ptr()), _stream(stream)), "fspb_adjoint")
        return out

    def beamlet_pair_counts(self, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Voxels paired with each beamlet (in ROI, t >= 0), device int32
        [n_beamlets], from the adjoint's beamlet-major traversal."""
        if out is None:
            out = torch.empty(self.n_beamlets, dtype=torch.int32, device=self.device)
        if out.dtype != torch.int32 or out.numel() != self.n_beamlets or not out.is_cuda:
            raise ValueError("out must be a device int32 tensor of n_beamlets values")
        check(load().fspb_beamlet_pair_counts(self._handle(), C.c_void_p(out.data_ptr()),
                                              _stream(stream)), "fspb_beamlet_pair_counts")
        return out

    def count_pairs(self, fluence: Optional[torch.Tensor] = None, per_voxel: bool = False,
                    stream=None):
        """Evaluated pairs (in ROI, t >= 0); with fluence, only f_i != 0."""
        fp = C.c_void_p(0)
        if fluence is not None:
            f = _dev_f32(fluence, self.device)
            fp = C.c_void_p(f.data_ptr())
        counts = None
        cp = C.c_void_p(0)
        if per_voxel:
            counts = torch.empty(self.shape, dtype=torch.int32, device=self.device)
            cp = C.c_void_p(counts.data_ptr())
        tot = C.c_ulonglong(0)
        check(load().fspb_count_pairs(self._handle(), fp, cp, C.byref(tot), _stream(stream)),
              "fspb_count_pairs")
        return (int(tot.value), counts) if per_voxel else int(tot.value)

    def count_pairs_noalloc(self, fluence: Optional[torch.Tensor] = None,
                            out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """The pair count of count_pairs into a device int64 word, with no
        allocation in the library and no host synchronisation."""
        fp = C.c_void_p(0)
        if fluence is not None:
            f = _dev_f32(fluence, self.device)
            fp = C.c_void_p(f.data_ptr())
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        if out.dtype != torch.int64 or out.numel() < 1 or not out.is_cuda:
            raise ValueError("out must be a device int64 tensor")
        check(load().fspb_count_pairs_noalloc(self._handle(), fp, C.c_void_p(out.data_ptr()),
                                              _stream(stream)), "fspb_count_pairs_noalloc")
        return out

    def wait_ready(self, stream=None) -> None:
        """Makes stream (default: the current one) wait on the device for this
        plan's creation work, e.g. before recording a timing event there."""
        check(load().fspb_wait_ready(self._handle(), _stream(stream)), "fspb_wait_ready")

    def update_density(self, density: torch.Tensor, stream=None) -> None:
        """Re-runs the density-dependent geometry (smoothing, entrances, depth
        tables) for a new CT of the same grid; asynchronous, graph-capturable.
        The tensor must stay alive until the work has run."""
        d = density
        if not (isinstance(d, torch.Tensor) and d.is_cuda and d.dtype == torch.float32
                and d.is_contiguous() and d.numel() == self.n_vox):
            raise ValueError("density must be a contiguous float32 CUDA tensor of the grid's size")
        check(load().fspb_update_density(self._handle(), C.c_void_p(d.data_ptr()), _stream(stream)),
              "fspb_update_density")
        self._density = d

    # -- learned surrogate ------------------------------------------------------
    def _ct(self, density):
        d = self._density if density is None else density
        if not (isinstance(d, torch.Tensor) and d.is_cuda and d.dtype == torch.float32
                and d.is_contiguous() and d.numel() == self.n_vox):
            raise ValueError("density must be a contiguous float32 CUDA tensor of the grid's size")
        return d

    def surrogate_samples(self, rows: torch.Tensor, density=None, stream=None):
        """Training rows for (voxel, beam) pairs rows [n, 2] (int32, device):
        returns (x BF16 [n, 224], targets FP32 [n, 6], valid int32 [n])."""
        r = rows
        if not (isinstance(r, torch.Tensor) and r.is_cuda and r.dtype == torch.int32
                and r.is_contiguous() and r.dim() == 2 and r.shape[1] == 2):
            raise ValueError("rows must be a contiguous int32 CUDA tensor [n, 2]")
        n = r.shape[0]
        x = torch.empty((n, _lib.FSPB_MLP_IN_PAD), dtype=torch.bfloat16, device=self.device)
        t = torch.empty((n, _lib.FSPB_MLP_OUT), dtype=torch.float32, device=self.device)
        v = torch.empty(n, dtype=torch.int32, device=self.device)
        check(load().fspb_surrogate_samples(self._handle(), C.c_void_p(self._ct(density).data_ptr()),
                                            C.c_void_p(r.data_ptr()), n, C.c_void_p(x.data_ptr()),
                                            C.c_void_p(t.data_ptr()), C.c_void_p(v.data_ptr()),
                                            _stream(stream)), "fspb_surrogate_samples")
        return x, t, v

    def surrogate_infer(self, mlp: "Mlp", density=None, out: Optional[torch.Tensor] = None,
                        stream=None) -> torch.Tensor:
        """Every (voxel, beam) row: [n_beams, n_vox, 8] = (u1x, u1y, u2x, u2y)
        log2 e, w1, w2, fallback flag, 0."""
        shape = (self.n_beams, self.n_vox, 8)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        elif tuple(out.shape) != shape or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 tensor {shape}")
        check(load().fspb_surrogate_infer(self._handle(), mlp._handle(),
                                          C.c_void_p(self._ct(density).data_ptr()),
                                          C.c_void_p(out.data_ptr()), _stream(stream)),
              "fspb_surrogate_infer")
        return out

    def forward_surrogate(self, fluence: torch.Tensor, prm: torch.Tensor,
                          out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        f = _dev_f32(fluence, self.device)
        if f.numel() != self.n_beamlets:
            raise ValueError(f"fluence has {f.numel()} values, plan has {self.n_beamlets} beamlets")
        if (tuple(prm.shape) != (self.n_beams, self.n_vox, 8) or prm.dtype != torch.float32
                or not prm.is_contiguous()):
            raise ValueError("prm must come from surrogate_infer")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        check(load().fspb_forward_surrogate(self._handle(), C.c_void_p(f.data_ptr()),
                                            C.c_void_p(prm.data_ptr()), C.c_void_p(out.data_ptr()),
                                            _stream(stream)), "fspb_forward_surrogate")
        return out

    @staticmethod
    def tile_shapes():
        L = load()
        n = L.fspb_tile_shapes(None, 0)
        dims = (C.c_int * (3 * n))()
        L.fspb_tile_shapes(dims, n)
        return [tuple(dims[3 * q:3 * q + 3]) for q in range(n)]

    def set_tile(self, shape: int, waves_per_block: int, stream=None) -> None:
        check(load().fspb_set_tile(self._handle(), int(shape), int(waves_per_block),
                                   _stream(stream)), "fspb_set_tile")

    def get_tile(self):
        s, w = C.c_int(), C.c_int()
        check(load().fspb_get_tile(self._handle(), C.byref(s), C.byref(w)), "fspb_get_tile")
        return s.value, w.value

    def set_schedule(self, per_beam: int, stream=None) -> None:
        """Forward work schedule: 0 = bricks longest-first, 1 = per-beam items
        (see fspb_set_schedule)."""
        check(load().fspb_set_schedule(self._handle(), int(per_beam), _stream(stream)),
              "fspb_set_schedule")

    def get_schedule(self) -> int:
        v = C.c_int()
        check(load().fspb_get_schedule(self._handle(), C.byref(v)), "fspb_get_schedule")
        return v.value

    def autotune(self, fluence: torch.Tensor, reps: int = 3, stream=None):
        """Times every tile configuration and keeps the fastest; returns the
        timings as a list of dicts."""
        f = _dev_f32(fluence, self.device)
        scratch = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        res = (_lib.fspb_tune_result * 64)()
        n = C.c_int(0)
        check(load().fspb_autotune(self._handle(), C.c_void_p(f.data_ptr()),
                                   C.c_void_p(scratch.data_ptr()), int(reps), _stream(stream),
                                   res, 64, C.byref(n)), "fspb_autotune")
        return [dict(shape=r.shape, dims=tuple(r.dims), waves_per_block=r.waves_per_block,
                     per_beam=r.per_beam, ms=r.ms) for r in res[:n.value]]

    def set_adjoint_slab(self, planes: int) -> None:
        """Grid planes per adjoint work unit (0: the default; see
        fspb_set_adjoint_slab)."""
        check(load().fspb_set_adjoint_slab(self._handle(), int(planes)), "fspb_set_adjoint_slab")

    def get_adjoint_slab(self) -> int:
        v = C.c_int()
        check(load().fspb_get_adjoint_slab(self._handle(), C.byref(v)), "fspb_get_adjoint_slab")
        return v.value

    def autotune_adjoint(self, voxel_weight: torch.Tensor, reps: int = 3, stream=None):
        """Times the adjoint at a few slab thicknesses and keeps the fastest;
        returns [dict(planes, ms)]."""
        w = _dev_f32(voxel_weight, self.device)
        if w.numel() != self.n_vox:
            raise ValueError(f"voxel weight has {w.numel()} values, grid has {self.n_vox}")
        scratch = torch.empty(self.n_beamlets, dtype=torch.float32, device=self.device)
        planes, ms, n = (C.c_int * 16)(), (C.c_float * 16)(), C.c_int(0)
        check(load().fspb_autotune_adjoint(self._handle(), C.c_void_p(w.data_ptr()),
                                           C.c_void_p(scratch.data_ptr()), int(reps),
                                           _stream(stream), planes, ms, 16, C.byref(n)),
              "fspb_autotune_adjoint")
        return [dict(planes=planes[i], ms=ms[i]) for i in range(n.value)]

    def set_dc(self, enabled: bool) -> None:
        check(load().fspb_set_dc(self._handle(), int(bool(enabled))), "fspb_set_dc")

    def info(self) -> dict:
        inf = _lib.fspb_info()
        check(load().fspb_geometry_info(self._handle(), C.byref(inf)), "fspb_geometry_info")
        d = {n: getattr(inf, n) for n, _ in _lib.fspb_info._fields_}
        d["smooth_radius"] = tuple(inf.smooth_radius)
        return d

    def smoothed_density(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        check(load().fspb_smoothed_density(self._handle(), C.c_void_p(out.data_ptr()),
                                           _stream(stream)), "fspb_smoothed_density")
        return out

    def beamlet(self, i: int, tables: bool = True) -> dict:
        inf = _lib.fspb_beamlet_info()
        check(load().fspb_beamlet(self._handle(), int(i), C.byref(inf), None, None, None, 0),
              "fspb_beamlet")
        out = dict(hit=bool(inf.hit), k_entry=inf.k_entry, n_samples=inf.n_samples, K=inf.K,
                   s_in=inf.s_in, s_entry=inf.s_entry, theta=inf.theta,
                   src=np.array(inf.src), d=np.array(inf.dir), ex=np.array(inf.ex),
                   ey=np.array(inf.ey), entry_margin=inf.entry_margin,
                   pair_consts=np.array([list(inf.pair_t), list(inf.pair_x), list(inf.pair_y)],
                                        dtype=np.float32))
        if tables and inf.K > 0:
            T, W1, W2 = (np.zeros(inf.K, np.float32) for _ in range(3))
            P = C.POINTER(C.c_float)
            check(load().fspb_beamlet(self._handle(), int(i), None, T.ctypes.data_as(P),
                                      W1.ctypes.data_as(P), W2.ctypes.data_as(P), inf.K),
                  "fspb_beamlet")
            out.update(T=T, W1=W1, W2=W2)
        return out


class Batch:
    """Many plans in one persistent launch (static longest-first schedule),
    with per-plan completion times and optional HIP-graph capture."""

    def __init__(self, geometries, shape: int = 0, waves_per_block: int = 8,
                 waves_per_cu: int = 32, policy: str = "latency", stream=None):
        self.geometries = list(geometries)
        n = len(self.geometries)
        pol = {"throughput": _lib.FSPB_SCHEDULE_THROUGHPUT,
               "latency": _lib.FSPB_SCHEDULE_LATENCY}[policy]
        hs = (C.c_void_p * n)(*[g._handle() for g in self.geometries])
        h = C.c_void_p()
        check(load().fspb_batch_create(n, hs, int(shape), int(waves_per_block), int(waves_per_cu),
                                       pol, _stream(stream), C.byref(h)), "fspb_batch_create")
        self._h = h
        self._keep = None

    def _ptrs(self, tensors, n_expect, what):
        if len(tensors) != len(self.geometries):
            raise ValueError(f"need one {what} tensor per plan")
        out = (C.c_void_p * len(tensors))()
        for k, (t, g) in enumerate(zip(tensors, self.geometries)):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                raise ValueError(f"{what} {k} must be a contiguous float32 CUDA tensor")
            if t.numel() != n_expect(g):
                raise ValueError(f"{what} {k} has {t.numel()} values, expected {n_expect(g)}")
            out[k] = t.data_ptr()
        return out

    def forward(self, fluences, doses, stream=None) -> None:
        fp = self._ptrs(fluences, lambda g: g.n_beamlets, "fluence")
        dp = self._ptrs(doses, lambda g: g.n_vox, "dose")
        check(load().fspb_batch_forward(self._h, fp, dp, _stream(stream)), "fspb_batch_forward")

    def capture(self, fluences, doses, densities=None, stream=None) -> None:
        """Captures (density updates +) the batch forward into a HIP graph.
        stream must not be the null stream; the tensors must outlive replays."""
        fp = self._ptrs(fluences, lambda g: g.n_beamlets, "fluence")
        dp = self._ptrs(doses, lambda g: g.n_vox, "dose")
        rp = None
        if densities is not None:
            rp = self._ptrs(densities, lambda g: g.n_vox, "density")
        self._keep = (list(fluences), list(doses), None if densities is None else list(densities))
        check(load().fspb_batch_capture(self._h, fp, dp, rp, _stream(stream)), "fspb_batch_capture")

    def replay(self, stream=None) -> None:
        check(load().fspb_batch_replay(self._h, _stream(stream)), "fspb_batch_replay")

    def latencies(self, stream=None):
        """(per-plan completion times in ms, whole launch in ms) of the last run."""
        n = len(self.geometries)
        ms = (C.c_double * n)()
        tot = C.c_double(0)
        check(load().fspb_batch_latencies(self._h, ms, C.byref(tot), _stream(stream)),
              "fspb_batch_latencies")
        return list(ms), tot.value

    def info(self):
        w, it = C.c_int(), C.c_longlong()
        check(load().fspb_batch_info(self._h, C.byref(w), C.byref(it)), "fspb_batch_info")
        return dict(n_waves=w.value, n_items=it.value)

    def close(self):
        if getattr(self, "_h", None):
            load().fspb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The learned surrogate's network (202 -> 64 -> 64 -> 6, GELU): BF16
    MFMA training and inference in libfspb, FP32 master weights, Adam.
    Parameters are flat FP32 in the layout W1 [202][64], b1, W2 [64][64], b2,
    W3 [64][6], b3."""

    N_IN, N_PAD, N_HID, N_OUT = (_lib.FSPB_MLP_IN, _lib.FSPB_MLP_IN_PAD, _lib.FSPB_MLP_HIDDEN,
                                 _lib.FSPB_MLP_OUT)
    N_PARAMS = _lib.FSPB_MLP_PARAMS

    def __init__(self, params, device="cuda"):
        L = load()
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size != self.N_PARAMS:
            raise ValueError(f"need {self.N_PARAMS} parameters, got {p.size}")
        self.device = torch.device(device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fspb_mlp_create(p.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)),
                  "fspb_mlp_create")
        self._h = h
        self.scaling = (np.zeros(6, np.float32), np.ones(6, np.float32))
        self.guard = None

    @classmethod
    def initial(cls, seed: int = 0, device="cuda") -> "Mlp":
        return cls(cls.init_params(seed), device)

    @staticmethod
    def init_params(seed: int = 0) -> np.ndarray:
        """Glorot-uniform weights, zero biases (seeded)."""
        rng = np.random.default_rng(seed)
        out = []
        for fi, fo in ((202, 64), (64, 64), (64, 6)):
            a = np.sqrt(6.0 / (fi + fo))
            out += [rng.uniform(-a, a, size=fi * fo), np.zeros(fo)]
        return np.concatenate(out).astype(np.float32)

    def close(self):
        if getattr(self, "_h", None):
            load().fspb_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if not self._h:
            raise FspbError(_lib.FSPB_E_STATE, "network is closed")
        return self._h

    @staticmethod
    def _rows(x, t=None):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.bfloat16
                and x.is_contiguous() and x.dim() == 2 and x.shape[1] == _lib.FSPB_MLP_IN_PAD):
            raise ValueError("x must be a contiguous bfloat16 CUDA tensor [n, 224]")
        if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda
                                  and t.dtype == torch.float32 and t.is_contiguous()
                                  and tuple(t.shape) == (x.shape[0], _lib.FSPB_MLP_OUT)):
            raise ValueError("targets must be a contiguous float32 CUDA tensor [n, 6]")
        return x.shape[0]

    def set_scaling(self, mean, stdev) -> None:
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(stdev, dtype=np.float32)
        check(load().fspb_mlp_set_scaling(self._handle(), m.ctypes.data_as(C.POINTER(C.c_float)),
                                          s.ctypes.data_as(C.POINTER(C.c_float))),
              "fspb_mlp_set_scaling")
        self.scaling = (m.copy(), s.copy())

    def set_guard(self, rho_lo=-np.inf, rho_hi=np.inf, het_max=np.inf, band_lo=None,
                  band_hi=None) -> None:
        big = float(np.finfo(np.float32).max)
        clip = lambda v: float(np.clip(v, -big, big))
        bl = [-big] * 6 if band_lo is None else [clip(v) for v in band_lo]
        bh = [big] * 6 if band_hi is None else [clip(v) for v in band_hi]
        g = _lib.fspb_surrogate_guard(clip(rho_lo), clip(rho_hi), clip(het_max),
                                      (C.c_float * 6)(*bl), (C.c_float * 6)(*bh))
        check(load().fspb_mlp_set_guard(self._handle(), C.byref(g)), "fspb_mlp_set_guard")
        self.guard = dict(rho_lo=rho_lo, rho_hi=rho_hi, het_max=het_max,
                          band_lo=list(bl), band_hi=list(bh))

    def loss_grad(self, x, t, stream=None):
        """(loss [1], gradient [N_PARAMS]) of the mean-square loss; FP32 device."""
        n = self._rows(x, t)
        g = torch.empty(self.N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        check(load().fspb_mlp_loss_grad(self._handle(), C.c_void_p(x.data_ptr()),
                                        C.c_void_p(t.data_ptr()), n, C.c_void_p(g.data_ptr()),
                                        C.c_void_p(loss.data_ptr()), _stream(stream)),
              "fspb_mlp_loss_grad")
        return loss, g

    def train_step(self, x, t, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, loss=None, stream=None):
        """One Adam step; returns the (device) loss before the step."""
        n = self._rows(x, t)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        opt = _lib.fspb_adam(float(lr), float(betas[0]), float(betas[1]), float(eps))
        check(load().fspb_mlp_train_step(self._handle(), C.c_void_p(x.data_ptr()),
                                         C.c_void_p(t.data_ptr()), n, C.byref(opt),
                                         C.c_void_p(loss.data_ptr()), _stream(stream)),
              "fspb_mlp_train_step")
        return loss

    def predict(self, x, stream=None) -> torch.Tensor:
        n = self._rows(x)
        y = torch.empty((n, _lib.FSPB_MLP_OUT), dtype=torch.float32, device=x.device)
        check(load().fspb_mlp_predict(self._handle(), C.c_void_p(x.data_ptr()), n,
                                      C.c_void_p(y.data_ptr()), _stream(stream)),
              "fspb_mlp_predict")
        return y

    def state(self) -> dict:
        """Checkpoint (host copies): params, Adam moments, step, scaling."""
        a = [np.empty(self.N_PARAMS, np.float32) for _ in range(3)]
        step = C.c_longlong(0)
        fp = lambda v: v.ctypes.data_as(C.POINTER(C.c_float))
        check(load().fspb_mlp_get_state(self._handle(), fp(a[0]), fp(a[1]), fp(a[2]),
                                        C.byref(step)), "fspb_mlp_get_state")
        return dict(params=a[0], adam_m=a[1], adam_v=a[2], step=np.int64(step.value),
                    mean=self.scaling[0].copy(), std=self.scaling[1].copy())

    def load_state(self, st: dict) -> None:
        a = [np.ascontiguousarray(st[k], dtype=np.float32) for k in ("params", "adam_m", "adam_v")]
        fp = lambda v: v.ctypes.data_as(C.POINTER(C.c_float))
        check(load().fspb_mlp_set_state(self._handle(), fp(a[0]), fp(a[1]), fp(a[2]),
                                        int(st["step"])), "fspb_mlp_set_state")
        if "mean" in st:
            self.set_scaling(st["mean"], st["std"])

    def save(self, path) -> None:
        np.savez(path, **self.state())

    def restore(self, path) -> None:
        with np.load(path, allow_pickle=False) as z:
            self.load_state({k: z[k] for k in z.files})


def gamma_index(ref: torch.Tensor, ev: torch.Tensor, spacing, dist: float = 0.3,
                dose_frac: float = 0.03, cap: float = 5.0, dose_max: float = 0.0,
                iso_frac: float = 0.5, out: Optional[torch.Tensor] = None, stream=None):
    """3D gamma index of ev against ref (same grid, [nz][ny][nx], spacing
    (dx, dy, dz) cm): returns (gamma grid, statistics dict)."""
    for t in (ref, ev):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                and t.is_contiguous() and t.dim() == 3):
            raise ValueError("ref and ev must be contiguous float32 CUDA tensors [nz][ny][nx]")
    if ref.shape != ev.shape:
        raise ValueError("ref and ev must have the same shape")
    nz, ny, nx = ref.shape
    if out is None:
        out = torch.empty_like(ref)
    p = _lib.fspb_gamma_params(float(dist), float(dose_frac), float(cap), float(dose_max),
                               float(iso_frac))
    st = _lib.fspb_gamma_stats()
    with torch.cuda.device(ref.device):
        check(load().fspb_gamma(C.c_void_p(ref.data_ptr()), C.c_void_p(ev.data_ptr()), nx, ny, nz,
                                *map(float, spacing), C.byref(p), C.c_void_p(out.data_ptr()),
                                C.byref(st), _stream(stream)), "fspb_gamma")
    return out, dict(gamma_max=st.gamma_max, gamma_avg_iso=st.gamma_avg_iso,
                     pass_rate_iso=st.pass_rate_iso, dose_max=st.dose_max, n_iso=st.n_iso)


class FspbDose(torch.autograd.Function):
    """D = forward(f); dL/df = adjoint(dL/dD)."""

    @staticmethod
    def forward(ctx, fluence: torch.Tensor, geometry: Geometry) -> torch.Tensor:
        ctx.geometry = geometry
        return geometry.forward(fluence.detach())

    @staticmethod
    def backward(ctx, grad_dose: torch.Tensor):
        g = ctx.geometry.adjoint(grad_dose.detach().contiguous())
        return g, None
