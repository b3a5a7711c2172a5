"""Host logic of bench.py, without a GPU: the refusal of a multi-GPU run, the
lookup of committed counter summaries (reported only while the kernel source
they were taken on is unchanged), and the host description beside the CPU
baseline."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _tree(tmp_path, source_text, summary_sha, workload="3d-8-test", kind=0):
    csrc = tmp_path / "paper_2103_07537_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "solve_kernels.hip").write_text(source_text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_test.txt").write_text(
        "# counter summary\n\n"
        "  indented lines are prose, not keys = values\n"
        f"workload={workload}\nkind={kind}\nsource_sha256={summary_sha}\n"
        "traffic_bytes_per_launch=123456789\nvcycle_traffic_bytes=987654321\n")


def test_traffic_is_read_while_the_kernel_source_matches(tmp_path, monkeypatch):
    b = _bench()
    text = "// kernels\n"
    _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    traffic, src, vc = b.measured_traffic("3d-8-test", 0)
    assert traffic == 123456789.0 and vc == 987654321.0
    assert src == os.path.join("profiles", "traffic_test.txt")


@pytest.mark.parametrize("what", ["source changed", "other workload", "other kind"])
def test_traffic_is_dropped_otherwise(tmp_path, monkeypatch, what):
    b = _bench()
    text = "// kernels\n"
    sha = hashlib.sha256(text.encode()).hexdigest()
    if what == "source changed":
        _tree(tmp_path, text + "// edited\n", sha)
    elif what == "other workload":
        _tree(tmp_path, text, sha, workload="3d-16-test")
    else:
        _tree(tmp_path, text, sha, kind=1)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("3d-8-test", 0) == (None, None, None)


def test_host_description_names_the_cpu_and_its_cores():
    h = _bench().host_cpu()
    assert isinstance(h["model"], str) and h["model"]
    assert h["nproc"] >= 1 and 1 <= h["usable_cpus"] <= h["nproc"]
