"""Host-side logic of the benchmark and of the binding, on the CPU: the
one-GPU guard, the provenance rule of the recorded HBM traffic, and the loud
failure of the binding when the HIP library is absent (no fallback path)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_exits_with_a_message(args, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, env=e, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_recorded_traffic_follows_the_stencil_source(monkeypatch, tmp_path):
    t = bench.recorded_traffic(1)
    assert t is not None and t > 20 * 43_986_977      # taken on the current source: above the algorithmic bytes
    monkeypatch.setattr(bench, "stencil_hash", lambda: "0" * 16)
    assert bench.recorded_traffic(1) is None            # stale once the stencil source changes
    monkeypatch.undo()
    monkeypatch.setattr(bench, "COUNTER_FILE", str(tmp_path / "absent.txt"))
    assert bench.recorded_traffic(1) is None


def test_counter_file_names_the_current_source():
    vals = dict(l.strip().split("=", 1) for l in open(bench.COUNTER_FILE) if "=" in l and not l.startswith("#"))
    assert vals["stencil_sha"] == bench.stencil_hash()
    fetch, write = float(vals["fetch_bytes_per_apply"]), float(vals["write_bytes_per_apply"])
    assert abs(fetch + write - float(vals["traffic_bytes_per_apply"])) <= 1.0


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    from paper_2608_22946_amd import helm
    monkeypatch.setattr(helm, "_lib", None)
    monkeypatch.setattr(helm, "_LIB_PATH", str(tmp_path / "libhelm.so"))
    with pytest.raises(ImportError, match="missing"):
        helm.lib()
