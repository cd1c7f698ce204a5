"""Host-side checks of the benchmark script (no GPU): it refuses more than one
GPU before touching the device, the committed counter summaries are read back
only for the kernel source and workload they were taken on, each summary's
bytes per launch are its scaled counters, and every profile command uses only
options the script accepts."""
import glob
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TRAFFIC = {
    bench.TRAFFIC_FILE: "slit-64x64x136-s8-eta0.25-f32",
    bench.TRAFFIC39_FILE: "slit-64x64x136-s8-eta0.25-f32",
    bench.TRAFFIC39T_FILE: "slit-64x64x136-s8-eta0.25-f32",
    bench.TRAFFIC_BULK_FILE: "bulk-256^3-s6-eta0.25-f32",
}


def _records(path):
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    return rec


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("path", sorted(TRAFFIC), ids=os.path.basename)
def test_traffic_summary_is_consistent(path):
    rec = _records(path)
    assert rec["workload"] == TRAFFIC[path]
    kib = 1024.0
    fetch = float(rec["fetch_kib_collide"]) * float(rec["fetch_scale"]) * kib
    write = float(rec["write_kib_collide"]) * float(rec["write_scale"]) * kib
    assert float(rec["fetch_bytes_per_launch"]) == pytest.approx(fetch, rel=1e-4)
    assert float(rec["write_bytes_per_launch"]) == pytest.approx(write, rel=1e-4)
    assert float(rec["bytes_per_launch"]) == pytest.approx(fetch + write, rel=1e-4)
    # the scales come from the 1 GiB copy kernel of the same run
    assert float(rec["fetch_scale"]) == pytest.approx(kib ** 2 / float(rec["fetch_kib_copy"]), rel=1e-4)
    assert float(rec["write_scale"]) == pytest.approx(kib ** 2 / float(rec["write_kib_copy"]), rel=1e-4)


@pytest.mark.parametrize("path", sorted(TRAFFIC), ids=os.path.basename)
def test_traffic_is_read_only_for_its_source_and_workload(path, monkeypatch):
    rec = _records(path)
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: rec["kernel_source_hash"])
    assert bench._traffic(TRAFFIC[path], path) == float(rec["bytes_per_launch"])
    assert bench._traffic("some-other-workload", path) is None
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0" * 16)
    assert bench._traffic(TRAFFIC[path], path) is None


def test_profile_commands_use_options_the_script_accepts():
    src = open(os.path.join(ROOT, "bench.py")).read()
    accepted = set(re.findall(r'add_argument\("(--[a-z0-9-]+)"', src))
    assert {"--gpus", "--steps", "--warmup", "--no-slit", "--surrogate-steps"} <= accepted
    files = glob.glob(os.path.join(ROOT, "profiles", "*"))
    assert files
    seen = 0
    for f in files:
        text = open(f).read().replace("\\\n", " ")
        for line in text.splitlines():
            if "bench.py" not in line or "rocprofv3" not in line:
                continue
            seen += 1
            opts = re.findall(r"(?<=\s)(--[a-z0-9-]+)", line.split("bench.py", 1)[1])
            assert set(opts) <= accepted, (os.path.basename(f), set(opts) - accepted)
    assert seen >= 8
