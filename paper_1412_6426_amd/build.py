"""Build libqed.so for gfx950 in-tree (paper_1412_6426_amd/lib/libqed.so).

``python -m paper_1412_6426_amd.build`` runs one hipcc command over the HIP sources in
``csrc/``, one for the HBM counter-calibration program ``calib/hbm_copy.hip``
(``lib/hbm_copy``) and one for the access-pattern ceilings ``calib/hbm_patterns.hip``
(``lib/hbm_patterns``).  Packed-FP32 instructions are disabled for all device code.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC_DIR = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIB_DIR, "libqed.so")
COPY_PROBE = os.path.join(LIB_DIR, "hbm_copy")
PATTERN_PROBE = os.path.join(LIB_DIR, "hbm_patterns")
ARCH = os.environ.get("QED_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(SRC_DIR, "*.hip")))


def hipcc_command(out: str, extra=()):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-I", SRC_DIR,
            *extra, "-o", out, *sources()]


def copy_probe_command(out: str, src: str = "hbm_copy.hip"):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-o", out, os.path.join(HERE, "calib", src)]


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    for out, cmd in ((LIB, hipcc_command(LIB + ".tmp", extra)),
                     (COPY_PROBE, copy_probe_command(COPY_PROBE + ".tmp")),
                     (PATTERN_PROBE, copy_probe_command(PATTERN_PROBE + ".tmp",
                                                        "hbm_patterns.hip"))):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=tuple(a for a in sys.argv[1:] if a != "-v"))
