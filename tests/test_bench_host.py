"""Host-side checks of bench.py's contract (no GPU needed): the one-GPU
refusal, the counter summary being used only for the kernel source it was
taken on, and the JSON keys a benchmark line carries."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 123, "valu_busy": 0.5, "kernel_hash": bench.kernel_source_hash()}
    (prof / "traffic.json").write_text(json.dumps({"w/f32x2": entry, "w/f16x2": dict(entry, kernel_hash="0" * 16)}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash is of the real sources; only the summary's location moves
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: entry["kernel_hash"])
    assert bench.measured_traffic("w", "f32x2") == 123
    assert bench.measured_traffic("w", "f16x2") is None       # taken on another kernel source
    assert bench.measured_traffic("w", "bf16x2") is None      # never measured
    assert bench.measured_counters("w", "f32x2")["valu_busy"] == 0.5
    assert bench.measured_counters("w", "f16x2") is None


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    """A comment or layout edit keeps the hash (the counters stay valid for
    the same code); a change of code does not."""
    src = tmp_path / "paper_1004_5058_amd" / "csrc"
    src.mkdir(parents=True)
    real = os.path.join(ROOT, "paper_1004_5058_amd", "csrc")
    for name in ("lb_kernels.hip", "lb_device.hpp"):
        (src / name).write_text(open(os.path.join(real, name), encoding="utf-8").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    k = src / "lb_kernels.hip"
    text = k.read_text()
    k.write_text("// a new comment line\n" + text.replace("\n", "\n  ", 3) + "\n/* trailing\n block */\n")
    assert bench.kernel_source_hash() == h0
    old = "constexpr int pr_class(int cy) { return cy > 0 ? 0 :"
    assert old in text
    k.write_text(text.replace(old, old.replace("? 0 :", "? 1 :"), 1))
    assert bench.kernel_source_hash() != h0


def test_committed_counters_match_the_committed_kernels():
    """profiles/traffic.json is regenerated whenever the step kernel changes."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert d["couette_emulsion_4096x4096/f32x2"]["kernel_hash"] == bench.kernel_source_hash()
    assert bench.measured_traffic("couette_emulsion_4096x4096", "f32x2") > 0


@pytest.mark.parametrize("variant,b,floor", [("f32x2", 144, 72), ("f32", 144, 144), ("f16x2", 72, 36),
                                             ("bf16x2", 72, 36), ("f16dev", 72, 72), ("bf16dev", 72, 72),
                                             ("mom32", 48, 48)])
def test_bytes_per_update(variant, b, floor):
    """Per-update bytes of one step per pass in the variant's storage (18 loads
    + 18 stores, the moment form 6 + 6), and the bytes an update must move in
    the variant as run (half with two steps per pass)."""
    v = bench.VARIANTS[variant]
    assert v["bytes_per_lup"] == b and v["floor_per_lup"] == floor
    assert v["floor_per_lup"] * v["per_pass"] == v["bytes_per_lup"]


def test_unknown_variant_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--variants", "f32x3"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "unknown variant" in r.stderr
