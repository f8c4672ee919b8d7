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


def test_onchip_and_batch_profile_figures_parse():
    """The on-chip loop's and the batch's committed counter summaries carry
    the lines bench.py reads for their vector-ALU rooflines."""
    sys.path.insert(0, ROOT)
    import bench
    for path, keys in ((bench.ONCHIP_PROFILE, ["onchip_code_sha256", "valu_insts_per_generation"]),
                       (bench.BATCH_PROFILE, ["batch_onchip_launches", "batch_valu_insts_per_call",
                                              "onchip_code_sha256"])):
        text = open(os.path.join(ROOT, path)).read()
        found = sorted(line.strip().split(": ", 1)[0] for line in text.splitlines()
                       if line.strip().startswith(tuple(k + ":" for k in keys)))
        assert found == sorted(keys), path
    for f in bench.ONCHIP_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f
    v = bench.onchip_valu_per_generation(1024, 10_000)
    b = bench.batch_valu_per_call(27)
    assert v is None or v > 0
    assert b is None or b > 0
    assert bench.batch_valu_per_call(-1) is None


def test_batch_and_serve_switches_are_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--batch-variants", "--no-onchip", "--autotune", "--skip-loop"):
        assert flag in r.stdout, flag


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
