"""FP64 CPU oracle of the DC-FSPB dose method (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It never imports the
GPU package and shares no code with it; both take their inputs from the
seeded generators in ``fspb_synth``.

The C source (``fspb_oracle.c``) follows the paper's definitions step by
step; see its header for the equation each function implements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
LIB_PATH = HERE / "liboracle.so"


def build(verbose: bool = False) -> Path:
    """Compile liboracle.so with gcc (OpenMP, -O2)."""
    # -ffp-contract=off: a * b + c is never fused behind the source's back
    # (the single-precision pair test fuses exactly where it calls fmaf)
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
           "-o", str(LIB_PATH), str(HERE / "fspb_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Table(C.Structure):
    _fields_ = [("start", C.c_double), ("step", C.c_double), ("n", C.c_int),
                ("v", C.POINTER(C.c_float))]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
                ("rho", C.POINTER(C.c_float))]


class _Beam(C.Structure):
    _fields_ = [("gantry", C.c_double), ("couch", C.c_double), ("iso", C.c_double * 3),
                ("sad", C.c_double), ("nbx", C.c_int), ("nby", C.c_int),
                ("wx", C.c_double), ("wy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class _Tables(C.Structure):
    _fields_ = [("A", _Table), ("n_theta", C.c_int), ("theta_step", C.c_double)] + [
        (n, _Table) for n in ("u1x", "u1y", "u2x", "u2y", "w1", "w2",
                              "fu1", "fu2", "fw1", "fw2", "b1", "b2")]


class _Options(C.Structure):
    _fields_ = [("roi_radius", C.c_double), ("rho_surface", C.c_double),
                ("smooth_sigma", C.c_double), ("rho_min", C.c_double),
                ("rho_max", C.c_double), ("sample_step", C.c_double),
                ("dc_enabled", C.c_int), ("siddon", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = HERE / "fspb_oracle.c"
        if not LIB_PATH.exists() or LIB_PATH.stat().st_mtime < src.stat().st_mtime:
            build()
        L = C.CDLL(str(LIB_PATH))
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Grid), C.c_int, C.POINTER(_Beam),
                                 C.POINTER(_Tables), C.POINTER(_Options)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_n_beamlets.argtypes = [C.c_void_p]
        L.orc_p.restype = C.c_double
        L.orc_p.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_frame.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)] + \
            [C.POINTER(C.c_double)] * 3 + [C.c_int]
        L.orc_smoothed_at.restype = C.c_double
        L.orc_smoothed_at.argtypes = [C.c_void_p, C.c_long]
        L.orc_smooth_all.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_smooth_radius.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.orc_pair_consts.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_float)]
        L.orc_pair.restype = C.c_double
        L.orc_pair.argtypes = [C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_int)]
        L.orc_dose.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_long, C.POINTER(C.c_long),
                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_longlong)]
        L.orc_adjoint.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_pair_counts.argtypes = [C.c_void_p, C.c_long, C.POINTER(C.c_long),
                                      C.POINTER(C.c_int)]
        L.orc_beamlet_pair_counts.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                              C.POINTER(C.c_longlong)]
        L.orc_trace_siddon.restype = C.c_int
        L.orc_trace_siddon.argtypes = [C.c_void_p, C.c_int] + [C.POINTER(C.c_double)] * 5 + [C.c_int]
        L.orc_density_at.restype = C.c_double
        L.orc_density_at.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_params.restype = C.c_int
        L.orc_params.argtypes = [C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_double)]
        L.orc_pair_given.restype = C.c_double
        L.orc_pair_given.argtypes = [C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int)]
        L.orc_nearest_beamlet.restype = C.c_int
        L.orc_nearest_beamlet.argtypes = [C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_double)]
        L.orc_surrogate_row.restype = C.c_int
        L.orc_surrogate_row.argtypes = [C.c_void_p, C.c_long, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int)]
        L.orc_dose_given.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_long,
                                     C.POINTER(C.c_long), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def p(x: float, u: float, x0: float) -> float:
    """Eq. 4 penumbra profile."""
    return lib().orc_p(float(x), float(u), float(x0))


class Oracle:
    """FP64 oracle for one plan (``fspb_synth.Plan``)."""

    def __init__(self, plan, dc_enabled: int | None = None, siddon: int | None = None):
        self.plan = plan
        self._keep = []
        g = plan.density
        nz, ny, nx = g.shape
        self._rho = np.ascontiguousarray(g, dtype=np.float32)
        grid = _Grid(nx, ny, nz, *map(float, plan.spacing), *map(float, plan.origin),
                     _ptr(self._rho, C.c_float))
        beams = (_Beam * len(plan.beams))()
        for k, b in enumerate(plan.beams):
            beams[k] = _Beam(float(b.gantry), float(b.couch), (C.c_double * 3)(*map(float, b.iso)),
                             float(b.sad), int(b.nbx), int(b.nby), float(b.wx), float(b.wy),
                             float(b.cx), float(b.cy))
        t = plan.tables

        def tab(tt):
            v = np.ascontiguousarray(tt.values, dtype=np.float32)
            self._keep.append(v)
            return _Table(float(tt.start), float(tt.step), int(v.shape[-1]), _ptr(v, C.c_float))

        tabs = _Tables(tab(t.A), int(t.n_theta), float(t.theta_step),
                       *[tab(getattr(t, n)) for n in ("u1x", "u1y", "u2x", "u2y", "w1", "w2",
                                                      "fu1", "fu2", "fw1", "fw2", "b1", "b2")])
        o = plan.options
        dc = o.dc_enabled if dc_enabled is None else dc_enabled
        sid = getattr(o, "siddon", 0) if siddon is None else siddon
        opts = _Options(float(o.roi_radius), float(o.rho_surface), float(o.smooth_sigma),
                        float(o.rho_min), float(o.rho_max), float(o.sample_step), int(dc), int(sid))
        self._structs = (grid, beams, tabs, opts)
        self.ctx = lib().orc_create(C.byref(grid), len(plan.beams), beams, C.byref(tabs),
                                    C.byref(opts))
        if not self.ctx:
            raise ValueError("oracle rejected the plan")
        self.n_beamlets = lib().orc_n_beamlets(self.ctx)
        self.shape = g.shape
        self.n_vox = int(g.size)

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().orc_destroy(self.ctx)
            self.ctx = None

    # -- per-beamlet geometry ---------------------------------------------
    def frame(self, i: int) -> dict:
        out = np.zeros(16)
        lib().orc_frame(self.ctx, int(i), _ptr(out, C.c_double))
        return dict(src=out[0:3].copy(), d=out[3:6].copy(), ex=out[6:9].copy(),
                    ey=out[9:12].copy(), theta=out[12], x0=out[13], y0=out[14], sad=out[15])

    def trace(self, i: int) -> dict:
        info = np.zeros(10)
        K = lib().orc_trace(self.ctx, int(i), _ptr(info, C.c_double), None, None, None, 0)
        T, W1, W2 = (np.zeros(max(K, 1)) for _ in range(3))
        lib().orc_trace(self.ctx, int(i), _ptr(info, C.c_double), _ptr(T, C.c_double),
                        _ptr(W1, C.c_double), _ptr(W2, C.c_double), K)
        return dict(hit=bool(info[0]), s_in=info[1], s_out=info[2], s_entry=info[3],
                    k_entry=int(info[4]), K=int(info[5]), s_exit=info[6], amb_rho=info[7],
                    step=info[8], n_samples=int(info[9]), T=T[:K], W1=W1[:K], W2=W2[:K])

    def trace_siddon(self, i: int) -> dict:
        """Siddon segment tables of beamlet i (context built with siddon=1)."""
        K = lib().orc_trace_siddon(self.ctx, int(i), None, None, None, None, None, 0)
        a = [np.zeros(max(K, 1)) for _ in range(5)]
        lib().orc_trace_siddon(self.ctx, int(i), *[_ptr(v, C.c_double) for v in a], K)
        return dict(K=K, t=a[0][:K], T=a[1][:K], W1=a[2][:K], W2=a[3][:K], rho=a[4][:K])

    def pair_consts(self, i: int) -> np.ndarray:
        """Single-precision constants of beamlet i's pair test, [3, 4]:
        rows (d, c_t), (ex, c_x), (ey, c_y)."""
        out = np.zeros(12, dtype=np.float32)
        lib().orc_pair_consts(self.ctx, int(i), _ptr(out, C.c_float))
        return out.reshape(3, 4)

    # -- smoothing --------------------------------------------------------
    def smoothed(self, vox=None) -> np.ndarray:
        if vox is None:
            out = np.zeros(self.n_vox)
            lib().orc_smooth_all(self.ctx, _ptr(out, C.c_double))
            return out.reshape(self.shape)
        vox = np.atleast_1d(np.asarray(vox, dtype=np.int64))
        return np.array([lib().orc_smoothed_at(self.ctx, int(v)) for v in vox])

    def smooth_radius(self):
        r = np.zeros(3, dtype=np.int32)
        lib().orc_smooth_radius(self.ctx, _ptr(r, C.c_int))
        return tuple(int(v) for v in r)

    # -- pair, dose, adjoint ----------------------------------------------
    def pair(self, vox: int, i: int):
        fl = C.c_int(0)
        v = lib().orc_pair(self.ctx, int(vox), int(i), C.byref(fl))
        return v, fl.value

    def dose(self, fluence=None, vox=None):
        """Returns (dose, amb, pairs) at the listed voxels (all when None)."""
        f = np.ascontiguousarray(self.plan.fluence if fluence is None else fluence,
                                 dtype=np.float32)
        assert f.shape == (self.n_beamlets,)
        if vox is None:
            n, vp = self.n_vox, None
        else:
            vox = np.ascontiguousarray(np.atleast_1d(vox), dtype=np.int64)
            n, vp = vox.size, _ptr(vox, C.c_long)
        d, a = np.zeros(n), np.zeros(n)
        pc = np.zeros(n, dtype=np.int64)
        lib().orc_dose(self.ctx, _ptr(f, C.c_float), n, vp, _ptr(d, C.c_double),
                       _ptr(a, C.c_double), _ptr(pc, C.c_longlong))
        if vox is None:
            return d.reshape(self.shape), a.reshape(self.shape), pc.reshape(self.shape)
        return d, a, pc

    def adjoint(self, w, beamlets=None):
        """Returns (g, amb) for the listed beamlets (all when None)."""
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        assert w.size == self.n_vox
        if beamlets is None:
            n, lp = self.n_beamlets, None
        else:
            beamlets = np.ascontiguousarray(np.atleast_1d(beamlets), dtype=np.int32)
            n, lp = beamlets.size, _ptr(beamlets, C.c_int)
        g, a = np.zeros(n), np.zeros(n)
        lib().orc_adjoint(self.ctx, _ptr(w, C.c_float), n, lp, _ptr(g, C.c_double),
                          _ptr(a, C.c_double))
        return g, a

    def beamlet_pair_counts(self, beamlets=None) -> np.ndarray:
        """Voxels paired with each listed beamlet (all when None)."""
        if beamlets is None:
            n, lp = self.n_beamlets, None
        else:
            beamlets = np.ascontiguousarray(np.atleast_1d(beamlets), dtype=np.int32)
            n, lp = beamlets.size, _ptr(beamlets, C.c_int)
        out = np.zeros(n, dtype=np.int64)
        lib().orc_beamlet_pair_counts(self.ctx, n, lp, _ptr(out, C.c_longlong))
        return out

    def pair_counts(self, vox=None) -> np.ndarray:
        if vox is None:
            n, vp = self.n_vox, None
        else:
            vox = np.ascontiguousarray(np.atleast_1d(vox), dtype=np.int64)
            n, vp = vox.size, _ptr(vox, C.c_long)
        out = np.zeros(n, dtype=np.int32)
        lib().orc_pair_counts(self.ctx, n, vp, _ptr(out, C.c_int))
        return out if vox is not None else out.reshape(self.shape)

    # -- learned-surrogate support (an extension beside the method) -------
    def density_at(self, points) -> np.ndarray:
        """Trilinear density (clamp-to-edge) at points [n, 3]."""
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        out = np.empty(len(pts))
        for k, q in enumerate(pts):
            out[k] = lib().orc_density_at(self.ctx, _ptr(q, C.c_double))
        return out

    def params(self, vox: int, i: int):
        """(six parameters (u1x, u1y, u2x, u2y, w1, w2), pair flags)."""
        out = np.zeros(6)
        fl = lib().orc_params(self.ctx, int(vox), int(i), _ptr(out, C.c_double))
        return out, fl

    def pair_given(self, vox: int, i: int, prm):
        prm = np.ascontiguousarray(prm, dtype=np.float64)
        fl = C.c_int(0)
        v = lib().orc_pair_given(self.ctx, int(vox), int(i), _ptr(prm, C.c_double), C.byref(fl))
        return v, fl.value

    def nearest_beamlet(self, vox: int, beam: int):
        """(beamlet index or -1, distance of the rounding from a tie)."""
        tie = C.c_double(0.0)
        i = lib().orc_nearest_beamlet(self.ctx, int(vox), int(beam), C.byref(tie))
        return i, tie.value

    def surrogate_rows(self, vox, beam):
        """Surrogate inputs of rows (vox[k], beam[k]): (features [n, 202],
        nearest beamlet or -1 [n], ambiguity flag [n], tie distance [n])."""
        vox = np.atleast_1d(np.asarray(vox, dtype=np.int64))
        beam = np.broadcast_to(np.asarray(beam, dtype=np.int64), vox.shape)
        feat = np.zeros((vox.size, 202))
        near = np.zeros(vox.size, dtype=np.int64)
        amb = np.zeros(vox.size, dtype=np.int32)
        tie = np.zeros(vox.size)
        f = np.zeros(202)
        a = C.c_int(0)
        for k, (v, b) in enumerate(zip(vox, beam)):
            near[k] = lib().orc_surrogate_row(self.ctx, int(v), int(b), _ptr(f, C.c_double),
                                              C.byref(a))
            amb[k] = a.value
            if near[k] >= 0:
                feat[k] = f
            tie[k] = self.nearest_beamlet(int(v), int(b))[1]
        return feat, near, amb, tie

    def dose_given(self, prm, fluence=None, vox=None):
        """Dose with per-(voxel, beam) parameters prm [n, n_beams, 7] (six
        parameters and a fallback flag).  Returns (dose, amb)."""
        f = np.ascontiguousarray(self.plan.fluence if fluence is None else fluence,
                                 dtype=np.float32)
        if vox is None:
            n, vp = self.n_vox, None
        else:
            vox = np.ascontiguousarray(np.atleast_1d(vox), dtype=np.int64)
            n, vp = vox.size, _ptr(vox, C.c_long)
        prm = np.ascontiguousarray(prm, dtype=np.float64)
        assert prm.shape == (n, len(self.plan.beams), 7)
        d, a = np.zeros(n), np.zeros(n)
        lib().orc_dose_given(self.ctx, _ptr(f, C.c_float), n, vp, _ptr(prm, C.c_double),
                             _ptr(d, C.c_double), _ptr(a, C.c_double))
        return d, a
