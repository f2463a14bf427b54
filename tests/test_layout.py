"""Host-side bounds of the workspace arithmetic: tests/layout_check.cpp, built with
AddressSanitizer and UndefinedBehaviorSanitizer on its host code (hipcc, gfx950) and linked
against the library, checks for the benchmark's workspace shapes and edge cases that every
region of the qed_step, qed_thin and qed_sort_cells workspaces is aligned, inside and
disjoint, that the public size functions agree with the layouts, that the largest
candidate-list, arena and sort-tile index each kernel can form stays inside its region, and
that the sort's key geometry keeps every block key below the reserved keys.  It launches
nothing (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1412_6426_amd", "lib")


def test_workspace_layouts_hold_every_kernel_index(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not on PATH")
    if not os.path.exists(os.path.join(LIBDIR, "libqed.so")):
        from paper_1412_6426_amd import build
        build.build()
    exe = tmp_path / "layout_check"
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1412_6426_amd", "csrc"),
                    os.path.join(ROOT, "tests", "layout_check.cpp"), "-L", LIBDIR, "-lqed",
                    f"-Wl,-rpath,{LIBDIR}", "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1"))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ok: 0 failure(s)" in r.stdout
