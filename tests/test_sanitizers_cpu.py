"""CPU sanitizer runs (no GPU): the FP64 oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, driven through every entry point on small plans;
and the C ABI's host code (argument validation, error reporting, NULL
handles, host-only queries) built with the host-side sanitizers, driven
through its error paths.  Any sanitizer report makes the driver abort."""
import os
import shutil
import struct
import subprocess
from pathlib import Path

import numpy as np
import pytest

import fspb_synth as S

ROOT = Path(__file__).resolve().parent.parent
HERE = Path(__file__).resolve().parent / "sanitize"
TABLE_ORDER = ("A", "u1x", "u1y", "u2x", "u2y", "w1", "w2", "fu1", "fu2", "fw1", "fw2", "b1", "b2")
SAN_ENV = {"ASAN_OPTIONS": "abort_on_error=1:detect_leaks=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"}


def _dump(plan, path):
    """The plan in the driver's dump layout (see oracle_driver.c)."""
    nz, ny, nx = plan.density.shape
    b = bytearray(struct.pack("<3i6d", nx, ny, nz, *map(float, plan.spacing), *map(float, plan.origin)))
    b += np.ascontiguousarray(plan.density, dtype="<f4").tobytes()
    b += struct.pack("<i", len(plan.beams))
    for bm in plan.beams:
        b += struct.pack("<6d2i4d", bm.gantry, bm.couch, *map(float, bm.iso), bm.sad, bm.nbx, bm.nby,
                         bm.wx, bm.wy, bm.cx, bm.cy)
    t = plan.tables
    for name in TABLE_ORDER:
        tb = getattr(t, name)
        v = np.ascontiguousarray(tb.values, dtype="<f4").reshape(-1)
        b += struct.pack("<2d2i", float(tb.start), float(tb.step), int(np.shape(tb.values)[-1]), v.size)
        b += v.tobytes()
    b += struct.pack("<id", int(t.n_theta), float(t.theta_step))
    o = plan.options
    b += struct.pack("<6d2i", o.roi_radius, o.rho_surface, o.smooth_sigma, o.rho_min, o.rho_max,
                     o.sample_step, int(o.dc_enabled), 0)
    fl = np.ascontiguousarray(plan.fluence, dtype="<f4")
    b += struct.pack("<i", fl.size) + fl.tobytes()
    Path(path).write_bytes(bytes(b))


def _plans():
    rng = np.random.default_rng(17)
    n, sp = (17, 15, 11), (0.3, 0.25, 0.4)

    def body(Z, Y, X):
        r = (X / 2.0) ** 2 + (Y / 1.6) ** 2 + (Z / 1.8) ** 2
        return np.where(r <= 1.0, 1.0 + 0.4 * np.sin(3 * X), 0.001)
    out = [S.plan_small(n=n, spacing=sp, density=body, seed=3, name="body", beams=[
        S.Beam(gantry=1.0, couch=0.3, nbx=3, nby=4, wx=0.5, wy=0.4, cx=0.1),
        S.Beam(gantry=4.2, nbx=2, nby=2, wx=0.6, wy=0.6)])]
    rho = rng.uniform(0.05, 2.2, size=(9, 12, 14)).astype(np.float32)
    out.append(S.plan_small(n=(14, 12, 9), density=rho, seed=4, name="noise_plain",
                            options=S.Options(roi_radius=0.8, dc_enabled=0),
                            beams=[S.Beam(gantry=2.5, nbx=4, nby=2, wx=0.3, wy=0.5)]))
    return out


@pytest.fixture(scope="module")
def oracle_asan(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path_factory.mktemp("asan") / "oracle_driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-std=c99",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", str(exe), str(HERE / "oracle_driver.c"), str(ROOT / "oracle" / "fspb_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.parametrize("k", [0, 1])
def test_oracle_under_address_and_ub_sanitizers(oracle_asan, tmp_path, k):
    plan = _plans()[k]
    dump = tmp_path / "plan.bin"
    _dump(plan, dump)
    r = subprocess.run([str(oracle_asan), str(dump)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, **SAN_ENV})
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]


@pytest.fixture(scope="module")
def abi_asan(tmp_path_factory):
    """libfspb with its C ABI sources (fspb_api.hip, api_*.hip) compiled with
    the host-side sanitizers (device code as usual), the kernels' objects as
    built, and the driver linked against it."""
    from paper_1103_1164_amd import build as B
    hipcc = B.hipcc()
    clang = Path(hipcc).resolve().parent.parent / "llvm" / "bin" / "clang"
    if not clang.exists():
        pytest.skip("clang of the ROCm toolchain not found")
    api = [s for s in B.SOURCES if s == "fspb_api.hip" or s.startswith("api_")]
    others = [B.BUILD / (Path(s).stem + ".o") for s in B.SOURCES if s not in api]
    if not all(o.exists() for o in others):
        B.build()
    d = tmp_path_factory.mktemp("abi_asan")
    inc = ["-I", str(B.INCLUDE), "-I", str(B.CSRC)]
    objs = []
    for src in api:
        obj = d / (Path(src).stem + "_san.o")
        cmd = [hipcc, *B.HIPCC_FLAGS, "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *inc, "-c", str(B.CSRC / src), "-o", str(obj)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        objs.append(obj)
    lib = d / "libfspb_san.so"
    r = subprocess.run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *map(str, others),
                        *map(str, objs), "-o", str(lib)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    exe = d / "abi_driver"
    r = subprocess.run([str(clang), "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-I", str(B.INCLUDE), str(HERE / "abi_driver.c"),
                        "-L", str(d), "-lfspb_san", f"-Wl,-rpath,{d}", "-lm", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_abi_host_code_under_address_and_ub_sanitizers(abi_asan):
    # leaks inside the HIP runtime's own initialisation are not this code's:
    # the suppressions name only that runtime and the HSA runtime under it
    supp = abi_asan.parent / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler-register\n")
    env = {**os.environ, **SAN_ENV, "LSAN_OPTIONS": f"suppressions={supp}"}
    env.pop("HIP_VISIBLE_DEVICES", None)
    r = subprocess.run([str(abi_asan)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
