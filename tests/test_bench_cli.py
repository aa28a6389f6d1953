"""bench.py's command line on the CPU: more than one GPU is refused with a
message and exit status 2 before any GPU work; --help lists the modes."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_help_lists_the_modes():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--tuning", "--fft-only", "--dense-only",
                 "--copy-calibration"):
        assert flag in r.stdout


def test_algorithmic_model_matches_the_closed_form():
    """Per column of the Gaussian workload (N = 65537, s = 4096, L = 2^16):
    bytes w (s + N), flops (5 log2 L + 3) L + 2 s; over t = 4096 columns in
    FP32 that is 1.1409 GB and 22.31 GFLOP."""
    import bench
    cm = bench.col_model(65537, 4096, 4)
    assert cm["bytes"] == 4 * (4096 + 65537)
    assert cm["flops"] == (5 * 16 + 3) * 65536 + 2 * 4096
    assert abs(cm["bytes"] * 4096 - 1.1409e9) < 1e5
    assert abs(cm["flops"] * 4096 - 22.31e9) < 1e7


def test_roofline_credits_the_columns_of_one_launch():
    """Eight launches per step of 512 columns each, 57.8 us per launch: the
    dominant kernel is credited 512 columns' flops per launch."""
    import bench
    steps, t = 20, 4096
    prof = {"middle": (8 * steps * 0.0578, 8 * steps), "back": (8 * steps * 0.0445, 8 * steps),
            "collapse_T": (steps * 0.03, steps)}
    kern, roof = bench.leg_roofline(prof, steps, 65537, 4096, t, "f32")
    assert roof["kernel"] == "middle" and roof["columns_per_launch"] == 512
    fl = 512 * ((5 * 16 + 3) * 65536 + 2 * 4096) / 57.8e-6 / 1e12
    assert abs(roof["achieved"] - fl) < 1e-3
    assert abs(roof["frac"] - fl / 157.3) < 1e-4 and abs(roof["frac_nonpacked"] - fl / 78.6) < 1e-4
    assert kern["back"]["launches_per_step"] == 8
