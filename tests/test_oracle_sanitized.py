"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer, every report fatal,
passes its pins: no out-of-bounds access, use after free, signed overflow, misaligned or
null dereference on the paths the pins exercise (the step with and without same-step
children, thinning, Schwinger pairs, the generators and their factors, the kinematics).
The sanitized copy is built from the oracle's own source into a temporary directory and
loaded in a child process; the oracle itself is untouched.  CPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_step.py", "tests/test_oracle_stats.py",
        "tests/test_oracle_same_step.py", "tests/test_oracle_thinning.py",
        "tests/test_oracle_thin_cells.py", "tests/test_oracle_thin_children.py",
        "tests/test_oracle_schwinger.py", "tests/test_oracle_kinematics.py",
        "tests/test_oracle_generator_factor.py", "tests/test_oracle_generator_forms.py"]


def _runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True, check=True).stdout.strip()


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_sanitized.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", str(lib), os.path.join(ORACLE, "qed_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, QED_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4",
               LD_PRELOAD=f"{_runtime('libasan.so')}:{_runtime('libubsan.so')}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=1200)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail
