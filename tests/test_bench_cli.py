"""bench.py's command line, checked on the CPU: the paths that must exit
before anything touches a GPU (a multi-GPU request, an unknown leg), and the
rule that a counter summary's traffic figure is used only while its recorded
kernel-source hash matches the source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_leg_is_refused():
    r = _run("--legs", "rgbd30k,nonsense", "--no-oracle")
    assert r.returncode == 2
    assert "nonsense" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_counted_kernel_source(tmp_path):
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    good = tmp_path / "good.md"
    good.write_text(f"# summary\n\n- kernel_source_sha256: `{sha}`\n- traffic_bytes_per_launch: `12345`\n")
    assert bench.measured_traffic(str(good)) == 12345.0
    stale = tmp_path / "stale.md"
    stale.write_text(f"# summary\n\n- kernel_source_sha256: `0{sha[1:]}`\n- traffic_bytes_per_launch: `12345`\n")
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None
