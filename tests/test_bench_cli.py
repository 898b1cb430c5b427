"""bench.py's host logic, checked on the CPU: the paths that must exit
before anything touches a GPU (a multi-GPU request, an unknown leg), the
rule that a counter summary's traffic figure is used only while its recorded
kernel-source hash matches the source, and the serving leg's served-rate
rule."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


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


def test_serving_window_rates():
    """The served-rate rule: completions over the second half of the arrival
    window against the arrivals there.  A server that keeps up completes
    about what arrives; a saturated one completes less there, even though
    everything completes in the end after the window (which completions
    over the whole span would blur)."""
    import numpy as np
    bench = _bench()
    rng = np.random.default_rng(0)
    window, rate = 10.0, 200.0
    arr = np.sort(rng.uniform(0, window, int(rate * window)))
    # kept up: every request takes 50 ms
    per_s, frac = bench.window_rates(arr, np.full(len(arr), 50.0), [True] * len(arr), window)
    assert abs(frac - 1.0) < 0.05 and abs(per_s - rate) < 0.1 * rate
    # saturated: the device finishes 100 per s in arrival order, the backlog
    # drains after the window
    done = np.arange(1, len(arr) + 1) / 100.0
    lat = (np.maximum(done, arr) - arr) * 1e3
    per_s, frac = bench.window_rates(arr, lat, [True] * len(arr), window)
    assert frac < 0.6 and abs(per_s - 100.0) < 10.0
    # failed requests do not count as served; no arrivals in the half: None
    _, frac = bench.window_rates(arr, np.full(len(arr), 50.0), [False] * len(arr), window)
    assert frac == 0.0
    assert bench.window_rates([0.1, 0.2], [1.0, 1.0], [True, True], window)[1] is None
