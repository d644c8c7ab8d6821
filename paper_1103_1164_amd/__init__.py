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

__all__ = ["Geometry", "Batch", "FspbDose", "FspbError", "load"]


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f32(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float32, device=device)
    return t.contiguous()


class Geometry:
    """A plan's geometry on the GPU (owning handle of libfspb)."""

    def __init__(self, density: torch.Tensor, spacing, origin, beams, tables, options=None,
                 stream=None):
        L = load()
        if not (isinstance(density, torch.Tensor) and density.is_cuda):
            raise TypeError("density must be a CUDA (HIP) tensor")
        density = density.to(torch.float32).contiguous()
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
        keep = []

        def tab(t):
            v = np.ascontiguousarray(t.values, dtype=np.float32)
            keep.append(v)
            return _lib.fspb_table1d(float(t.start), float(t.step), int(v.shape[-1]),
                                     v.ctypes.data_as(C.POINTER(C.c_float)))

        tabs = _lib.fspb_tables(tab(tables.A), int(tables.n_theta), float(tables.theta_step),
                                *[tab(getattr(tables, n)) for n in (
                                    "u1x", "u1y", "u2x", "u2y", "w1", "w2",
                                    "fu1", "fu2", "fw1", "fw2", "b1", "b2")])
        opt_p = None
        if options is not None:
            o = options
            opt = _lib.fspb_options(float(o.roi_radius), float(o.rho_surface),
                                    float(o.smooth_sigma), float(o.rho_min), float(o.rho_max),
                                    float(o.sample_step), int(o.dc_enabled), 0)
            opt_p = C.byref(opt)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(L.fspb_create_geometry(C.byref(ct), len(beams), bs, C.byref(tabs), opt_p,
                                         _stream(stream), C.byref(h)), "fspb_create_geometry")
        self._h = h
        self.n_beamlets = int(sum(int(b.nbx) * int(b.nby) for b in beams))
        self.n_vox = nx * ny * nz

    @classmethod
    def from_plan(cls, plan, device="cuda", dc_enabled: Optional[int] = None, stream=None):
        dens = torch.as_tensor(np.ascontiguousarray(plan.density, dtype=np.float32), device=device)
        opts = plan.options
        if dc_enabled is not None:
            import copy
            opts = copy.copy(opts)
            opts.dc_enabled = int(dc_enabled)
        return cls(dens, plan.spacing, plan.origin, plan.beams, plan.tables, opts, stream)

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
                     ms=r.ms) for r in res[:n.value]]

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
                   ey=np.array(inf.ey), entry_margin=inf.entry_margin)
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

    def __init__(self, geometries, shape: int = 0, waves_per_block: int = 4,
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
