"""Static checks of the separation between the product and its test oracle: the HIP library
and its binding never import, include or load the oracle; the oracle includes nothing of
the library; bench.py reaches the oracle only from its CPU-baseline leg."""
import ast
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1412_6426_amd")


def _imports(path):
    tree = ast.parse(open(path).read())
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [(a.name, node) for a in node.names]
        elif isinstance(node, ast.ImportFrom):
            out.append((node.module or "", node))
    return tree, out


def test_package_never_imports_the_oracle():
    for path in glob.glob(os.path.join(PKG, "**", "*.py"), recursive=True):
        _, imps = _imports(path)
        for name, _ in imps:
            assert not name.startswith("oracle") and "oracle" not in name.split("."), (path, name)
        assert "liboracle" not in open(path).read(), path


def test_hip_sources_and_oracle_share_no_headers():
    hip = glob.glob(os.path.join(PKG, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*"))
    for path in hip:
        txt = open(path).read()
        assert "qed_oracle" not in txt and "oracle/" not in txt, path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*.[ch]")):
        incs = re.findall(r'#include\s+[<"]([^>"]+)[>"]', open(path).read())
        for inc in incs:
            assert inc in ("qed_oracle.h", "math.h", "stdlib.h", "string.h", "omp.h",
                           "stdint.h", "stddef.h"), (path, inc)


def test_bench_reaches_the_oracle_only_from_its_cpu_baseline():
    tree, imps = _imports(os.path.join(ROOT, "bench.py"))
    owners = {}
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                owners.setdefault(id(node), fn.name)
    for name, node in imps:
        if name.startswith("oracle") or name == "tests.parity_util":
            assert owners.get(id(node)) == "cpu_baseline", (name, owners.get(id(node)))


def test_product_fails_loudly_without_its_library_or_device(tmp_path):
    """No CPU fallback: a missing libqed.so and a missing device are errors, not detours."""
    import subprocess
    import sys
    code = (
        "import sys\n"
        "from paper_1412_6426_amd import qed as Q\n"
        f"Q.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "Q._lib = None\n"
        "try:\n"
        "    Q.lib()\n"
        "except Q.QedError as e:\n"
        "    print('library:', e)\n"
        "else:\n"
        "    sys.exit(3)\n"
        "import torch\n"
        "if not torch.cuda.is_available():\n"
        "    from paper_1412_6426_amd.engine import Engine\n"
        "    try:\n"
        "        Engine([(10, 10, 10)], seeds=[0])\n"
        "    except Q.QedError as e:\n"
        "        print('device:', e)\n"
        "    else:\n"
        "        sys.exit(4)\n"
    )
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "library:" in r.stdout
