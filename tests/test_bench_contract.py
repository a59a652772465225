"""CPU checks of bench.py's contract: one GPU only (a request for more exits
with a message), and the stored counters feed the JSON line only for the
kernel revision they were taken at."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_valu_ceiling_follows_the_kernel_revision(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rev = bench.kernel_revision()
    (prof / "traffic.json").write_text(json.dumps({"valu": {"kernel_rev": rev, "mip_f32": 100.0}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_revision", lambda: rev)
    v = bench.valu_ceiling("mip_f32", 1e9, 10.0)
    # 100 lane slots x 1e9 samples in 10 ms = 1e13 slots/s against 256*4*16*2.4e9
    assert v["bound"] == "alu" and abs(v["frac"] - 1e13 / bench.VALU_PEAK) < 1e-4
    assert bench.valu_ceiling("bricked64_f32_mip", 1e9, 10.0) is None        # not measured
    (prof / "traffic.json").write_text(json.dumps({"valu": {"kernel_rev": "0" * 12, "mip_f32": 100.0}}))
    assert bench.valu_ceiling("mip_f32", 1e9, 10.0) is None                   # another revision


def test_committed_counters_match_the_sources():
    """The committed traffic counters were taken at the kernel sources in
    the tree (bench.py reports them only then)."""
    tj = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert tj["mip_f32"]["kernel_rev"] == bench.kernel_revision()
    assert tj["valu"]["kernel_rev"] == bench.kernel_revision()
