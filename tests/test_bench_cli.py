"""bench.py's command-line contract that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_figures_parse():
    """The committed counter summary carries the machine-readable lines
    bench.py looks for (whether they still match the sources is bench.py's
    own check at run time)."""
    sys.path.insert(0, ROOT)
    import bench
    text = open(os.path.join(ROOT, bench.PROFILE)).read()
    keys = [line.strip().split(": ", 1)[0] for line in text.splitlines()
            if line.strip().startswith(("traffic_bytes_per_launch_", "kernel_code_sha256:",
                                        "work_shape_"))]
    assert sorted(keys) == ["kernel_code_sha256", "traffic_bytes_per_launch_f32",
                            "traffic_bytes_per_launch_f64", "work_shape_f32", "work_shape_f64"]
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f
    json.dumps({"traffic": [bench.measured_traffic(4096, 200_000, precision=p)
                            for p in (32, 64)]})


def test_config_numbers_name_the_workloads():
    """--config 1..5 selects the five workloads; --gpus 2 is still refused
    first, so this runs without a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "--config" in r.stdout
    for c in ("1", "5"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", c,
                            "--gpus", "2"], capture_output=True, text=True, timeout=120)
        assert r.returncode == 2 and "one GPU" in r.stderr
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", "6"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr
