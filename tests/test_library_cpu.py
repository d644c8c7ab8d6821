"""Host-only checks of libfspb: it loads, exports every entry point the C
header declares, and rejects malformed input before touching a device."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

import fspb_synth as S

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib():
    from paper_1103_1164_amd import _lib
    return _lib


def _declared_functions():
    text = (ROOT / "include" / "fspb.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fspb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("fspb_create_geometry", "fspb_forward", "fspb_adjoint", "fspb_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    L = lib.load()
    names = _declared_functions()
    assert names
    for n in names:
        assert hasattr(L, n), n
        assert n in lib.SIGNATURES, n


def test_error_strings(lib):
    L = lib.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.fspb_error_string(code)
    assert L.fspb_error_string(-99) == b"unknown error"


def _args(lib, plan, density_ptr=0x1000):
    nz, ny, nx = plan.shape
    ct = lib.fspb_ct(nx, ny, nz, *plan.spacing, *plan.origin, C.c_void_p(density_ptr))
    bs = (lib.fspb_beam * len(plan.beams))()
    for k, b in enumerate(plan.beams):
        bs[k] = lib.fspb_beam(b.gantry, b.couch, (C.c_float * 3)(*b.iso), b.sad, b.nbx, b.nby,
                              b.wx, b.wy, b.cx, b.cy)
    keep = []

    def tab(t):
        v = np.ascontiguousarray(t.values, np.float32)
        keep.append(v)
        return lib.fspb_table1d(t.start, t.step, v.shape[-1], v.ctypes.data_as(C.POINTER(C.c_float)))

    t = plan.tables
    tabs = lib.fspb_tables(tab(t.A), t.n_theta, t.theta_step,
                           *[tab(getattr(t, n)) for n in ("u1x", "u1y", "u2x", "u2y", "w1", "w2",
                                                          "fu1", "fu2", "fw1", "fw2", "b1", "b2")])
    return ct, bs, tabs, keep


def _create(lib, ct, bs, tabs, opts=None, n_beams=None):
    h = C.c_void_p()
    rc = lib.load().fspb_create_geometry(C.byref(ct), len(bs) if n_beams is None else n_beams, bs,
                                         C.byref(tabs), C.byref(opts) if opts else None, None,
                                         C.byref(h))
    return rc, h


def test_validation_rejects_bad_input(lib):
    plan = S.plan_small(n=(8, 8, 8))
    ct, bs, tabs, keep = _args(lib, plan)
    ok_rc, h = _create(lib, ct, bs, tabs)
    # with valid input the call gets past validation: on a machine without a
    # gfx950 device it reports that, otherwise it succeeds
    assert ok_rc in (lib.FSPB_OK, lib.FSPB_E_UNSUPPORTED, lib.FSPB_E_HIP)
    if ok_rc == lib.FSPB_OK:
        lib.load().fspb_destroy(h)
    bad = []
    c2 = lib.fspb_ct.from_buffer_copy(ct); c2.nx = 0; bad.append((c2, bs, tabs, None, None))
    c2 = lib.fspb_ct.from_buffer_copy(ct); c2.dy = -1.0; bad.append((c2, bs, tabs, None, None))
    c2 = lib.fspb_ct.from_buffer_copy(ct); c2.density = None; bad.append((c2, bs, tabs, None, None))
    bad.append((ct, bs, tabs, None, 0))                       # no beams
    b2 = (lib.fspb_beam * 1).from_buffer_copy(bs); b2[0].nbx = 0; bad.append((ct, b2, tabs, None, None))
    b2 = (lib.fspb_beam * 1).from_buffer_copy(bs); b2[0].sad = 0.0; bad.append((ct, b2, tabs, None, None))
    b2 = (lib.fspb_beam * 1).from_buffer_copy(bs); b2[0].sad = 0.5; bad.append((ct, b2, tabs, None, None))  # source inside grid
    b2 = (lib.fspb_beam * 1).from_buffer_copy(bs); b2[0].gantry = float("nan"); bad.append((ct, b2, tabs, None, None))
    t2 = lib.fspb_tables.from_buffer_copy(tabs); t2.w2.n = 5; bad.append((ct, bs, t2, None, None))  # grid mismatch
    t2 = lib.fspb_tables.from_buffer_copy(tabs); t2.fu1.v = None; bad.append((ct, bs, t2, None, None))
    t2 = lib.fspb_tables.from_buffer_copy(tabs); t2.A.step = 0.0; bad.append((ct, bs, t2, None, None))
    o = lib.fspb_options(5, 0.5, 0.5, 0.1, 2.0, 0, 1, 7); bad.append((ct, bs, tabs, o, None))   # flags
    o = lib.fspb_options(5, 0.5, 0.5, 2.0, 0.1, 0, 1, 0); bad.append((ct, bs, tabs, o, None))   # rho range
    o = lib.fspb_options(5, 0.5, 0.5, 0.1, 2.0, 0, 3, 0); bad.append((ct, bs, tabs, o, None))   # dc flag
    o = lib.fspb_options(5, 0.5, 0.5, 0.1, 2.0, 0, 1, 0, 4, 8); bad.append((ct, bs, tabs, o, None))  # tile shape
    o = lib.fspb_options(5, 0.5, 0.5, 0.1, 2.0, 0, 1, 0, 0, 3); bad.append((ct, bs, tabs, o, None))  # tile waves
    for c, b, t, o, nb in bad:
        rc, h = _create(lib, c, b, t, o, nb)
        assert rc == lib.FSPB_E_ARG, lib.load().fspb_last_error()
        assert not h.value
        assert lib.load().fspb_last_error()


def test_null_handle_calls(lib):
    L = lib.load()
    assert L.fspb_forward(None, None, None, None) == lib.FSPB_E_ARG
    assert L.fspb_adjoint(None, None, None, None) == lib.FSPB_E_ARG
    assert L.fspb_set_dc(None, 1) == lib.FSPB_E_ARG
    info = lib.fspb_info()
    assert L.fspb_geometry_info(None, C.byref(info)) == lib.FSPB_E_ARG
    L.fspb_destroy(None)      # NULL-safe
    h = C.c_void_p(0x10)
    assert L.fspb_create_geometry(None, 1, None, None, None, None, C.byref(h)) == lib.FSPB_E_ARG
    assert h.value is None


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    """The binding refuses to run without the HIP library."""
    import importlib
    import paper_1103_1164_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.load()


def test_drift_table_mode_on_the_host(lib):
    """fspb_drift_tables: one weight-drift table when b2 is a multiple of b1
    at every sample of one grid (Section 2.1's single b has ratio 1), two
    otherwise; checked without a device on the table variants the GPU tests
    run."""
    import dataclasses
    from fspb_synth.tables import Table1D
    from paper_1103_1164_amd import drift_tables
    t = S.make_tables(0)
    b1 = t.b1
    rho = b1.start + b1.step * np.arange(b1.n)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    cases = [
        (t.b2, (1, -1.0)),                                                        # b2 = -b1
        (Table1D(b1.start, b1.step, b1.values.copy()), (1, 1.0)),                 # one b
        (Table1D(b1.start, b1.step, f32(0.5 * b1.values)), (1, 0.5)),
        (Table1D(b1.start, b1.step, f32(-0.6 * b1.values + 0.01 * (rho - 1) ** 2)), (2, 0.0)),
        (Table1D(b1.start, b1.step, f32(np.concatenate([-b1.values, -b1.values[-1:]]))), (2, 0.0)),
        (Table1D(b1.start + b1.step, b1.step, f32(-b1.values)), (2, 0.0)),        # shifted grid
    ]
    for b2, want in cases:
        assert drift_tables(dataclasses.replace(t, b2=b2)) == want
    z = Table1D(b1.start, b1.step, f32(0.0 * b1.values))
    assert drift_tables(dataclasses.replace(t, b1=z, b2=z)) == (1, 1.0)          # no drift at all
    assert drift_tables(dataclasses.replace(t, b1=z)) == (2, 0.0)                 # b1 = 0, b2 != 0
    L = lib.load()
    assert L.fspb_drift_tables(None, None) == lib.FSPB_E_ARG


def test_log_level_from_environment_and_setter(tmp_path):
    """FSPB_LOG_LEVEL sets the initial level (errors at 1 go to stderr with
    their code), fspb_set_log_level changes it and clamps, and the default
    is silent.  Runs in child processes so that the level is read fresh."""
    import subprocess
    import sys
    code = (
        "import ctypes as C\n"
        "from paper_1103_1164_amd import _lib, set_log_level\n"
        "L = _lib.load()\n"
        "print('initial', set_log_level(2))\n"
        "print('now', set_log_level(9))\n"
        "print('clamped', set_log_level(0))\n"
        "set_log_level(1)\n"
        "rc = L.fspb_create_geometry(None, 0, None, None, None, None, None)\n"
        "print('rc', rc)\n")
    env_base = {k: v for k, v in __import__('os').environ.items() if k != "FSPB_LOG_LEVEL"}
    for env_level, want_initial in ((None, 0), ("1", 1), ("3", 3), ("7", 3), ("x", 0)):
        env = dict(env_base)
        if env_level is not None:
            env["FSPB_LOG_LEVEL"] = env_level
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        lines = dict(l.split() for l in r.stdout.splitlines())
        assert int(lines["initial"]) == want_initial, (env_level, r.stdout)
        assert int(lines["now"]) == 2 and int(lines["clamped"]) == 3
        assert int(lines["rc"]) == -1
        errs = [l for l in r.stderr.splitlines() if l.startswith("[fspb] ")]
        assert len(errs) == 1 and "error -1" in errs[0] and "out is NULL" in errs[0], r.stderr
