"""Host-side checks of bench.py's contract (no GPU): one GPU only, a loud failure without a
device, the algorithmic byte counts per unit of work, and the dominant-kernel roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2", "--steps", "1")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    r = _run("--steps", "1")
    assert r.returncode != 0 and "HIP device" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_unit():
    # photon step: read x, k (6 doubles) and id, write x: 7 * 8 + 3 * 8
    assert bench.PHOTON_STEP_BYTES == 7 * 8 + 3 * 8
    # lepton step: read and write x, p (6 doubles each way) and n_events (4 B each way),
    # read id
    assert bench.LEPTON_STEP_BYTES == 2 * (6 * 8 + 4) + 8
    # child record: x, k, w (7 doubles), id and parent (8 B each), birth (4 B)
    assert bench.EMISSION_BYTES - 8 == 7 * 8 + 2 * 8 + 4
    assert bench.DEAD_SLOT_BYTES == 8
    assert bench.HBM_PEAK_GBS == 8000.0


def test_roofline_picks_the_dominant_kernel():
    r = dict(pho_ms=150.0, lep_ms=70.0, pho_bytes=6.6e11, lep_bytes=1e11)
    dom, kbytes, kms, achieved = bench.roofline_of(r)
    assert dom == "photon" and kbytes == 6.6e11 and kms == 150.0
    assert achieved == pytest.approx(6.6e11 / 0.150 / 1e9)
    r = dict(pho_ms=10.0, lep_ms=70.0, pho_bytes=1e10, lep_bytes=1e11)
    assert bench.roofline_of(r)[0] == "lepton"


def test_timed_steps_spread_over_the_job():
    s = bench.sampled_steps(600, 20)
    assert s == [15 + 30 * i for i in range(20)]
    assert bench.sampled_steps(600, None) == list(range(600))
    assert bench.sampled_steps(600, 600) == list(range(600))
    assert bench.sampled_steps(600, 1000) == list(range(600))
    assert bench.sampled_steps(7, 3) == [1, 3, 5]
    assert bench.sampled_steps(600, 0) == [300]


def test_kernel_names_match_the_profiler():
    assert bench.kernel_name("photon", "f64") == "photon_kernel<false, 1>"
    assert bench.kernel_name("lepton", "f64") == "lepton_kernel<false, 1, false>"
    assert bench.kernel_name("photon", "mixed") == "photon_kernel<true, 1>"
