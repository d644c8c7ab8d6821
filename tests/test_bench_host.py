"""Host-side parts of bench.py that need no GPU: the refusal of more than
one GPU, the stage records (--jsonl), and the counter-record lookup that
keys traffic figures to the kernels' sources."""
import json
import subprocess
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_records(tmp_path):
    bench.StageLog(None).emit("nothing", x=1)          # no path: writes nothing
    assert not list(tmp_path.iterdir())
    path = tmp_path / "stages.jsonl"
    log = bench.StageLog(str(path))
    log.emit("first", workload="c2", seed=2, pairs=np.int64(7), ms=np.float32(1.5),
             nested={"a": np.float64(0.25), "b": [1, 2]})
    log.emit("second", value=None)
    lines = path.read_text().splitlines()
    assert len(lines) == 2
    a, b = (json.loads(x) for x in lines)
    assert a["stage"] == "first" and b["stage"] == "second"
    assert a["workload"] == "c2" and a["seed"] == 2 and a["pairs"] == 7 and a["ms"] == 1.5
    assert a["nested"] == {"a": 0.25, "b": [1, 2]} and b["value"] is None
    assert 0.0 <= a["t_s"] <= b["t_s"]
    bench.StageLog(str(path)).emit("third")             # appends
    assert len(path.read_text().splitlines()) == 3


def test_counter_records_follow_the_sources(tmp_path):
    rec = bench.pmc_record((3, 8))
    assert rec and rec["tile"] == "3,8"
    assert bench.pmc_record((0, 1)) == {}                # another tile: no record
    # a record taken on other sources is not used
    fake = tmp_path / "rec.md"
    text = bench.PMC_SUMMARY.read_text()
    sha = rec["source_sha256"]
    fake.write_text(text.replace(sha, "0" * len(sha)))
    assert bench.pmc_record((3, 8), fake) == {}
    # the hash covers code, not comments or layout
    a = "int f(int x) {  // twice\n  return 2 * x; /* the double */ }\n"
    b = "int f(int x)\n{\n    return 2 * x;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(a.replace("2 * x", "3 * x"))
