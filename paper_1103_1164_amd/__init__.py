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

__all__ = ["Geometry", "FspbDose", "FspbError", "load"]


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
