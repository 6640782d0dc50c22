"""CPU checks of the benchmark's command line: one GPU only, and the workload list."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "single" in r.stderr


def test_unknown_workload_is_refused():
    r = _run("--workload", "no_such_surface")
    assert r.returncode == 2            # argparse: invalid choice
    assert "invalid choice" in r.stderr


def test_workloads_name_the_configs():
    sys.path.insert(0, ROOT)
    import bench
    import synth

    assert set(bench.WORKLOADS) == {"cap_2048", "sinusoid_4096", "sinusoid_128"}
    for name in bench.WORKLOADS:
        w = synth.config(name, side=16)
        assert w.name == name
