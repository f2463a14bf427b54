"""qed_step_noalloc (the step with the library's fixed scratch buffer as its workspace)
against qed_step with a caller-owned workspace, through the C ABI: two runs in a row on the
same GPU, the second smaller than the first, so the second starts from whatever the first
left in the shared buffer.  Stores are compared as multisets to the bar of the parity tests
(here bit-exact: the same kernels on the same inputs; only the child arenas differ in size,
which can change the order of the appended children), and every field of every step's
record except the lepton kernel's wavefront-iteration counts, which follow that order."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests.parity_util import compare_species

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import qed as Q  # noqa: E402
from paper_1412_6426_amd import runner as R  # noqa: E402
from paper_1412_6426_amd import workloads as W  # noqa: E402


def _note(msg):
    print(msg, flush=True)


def _run(e, w, noalloc):
    f, p = R.field_of(w), R.params_of(w)
    e.set_step(0)
    out = []
    for _ in range(w.n_steps):
        if noalloc:
            Q.qed_step_noalloc(e.tables.data_ptr(), e.stores, f, p, e.step_ctr.data_ptr(),
                               e.stats_buf.data_ptr(), e.stream)
        else:
            e.step(f, p)
        torch.cuda.synchronize()
        out.append(e.stats())
    return out


def _same(w, init, label):
    _note(f"{label}: qed_step")
    ref = R.engine_single(w, init, arena_records=0)
    rst = _run(ref, w, False)
    _note(f"{label}: qed_step_noalloc")
    e = R.engine_single(w, init, arena_records=0)
    st = _run(e, w, True)
    assert sum(s["emitted"] for s in st) > 1000 and sum(s["pairs"] for s in st) > 10
    for n, (a, b) in enumerate(zip(st, rst)):
        for k, v in a.items():
            if k in ("wave_iters", "low_occupancy_iters"):
                continue  # how the lepton kernel's wavefronts met the store's order
            if isinstance(v, float):  # workgroup partial sums add up in any order
                assert abs(v - b[k]) <= 1e-12 * abs(b[k]), (label, n, k)
            else:
                assert v == b[k], (label, n, k)
    assert int(e.step_ctr.item()) == w.n_steps
    for sp in range(3):
        compare_species(e.read(0, sp), ref.read(0, sp), sp, rtol=0.0, label=f"{label} {sp}")


def test_noalloc_step_matches_step_twice_in_a_row():
    big = W.rotating_e(n=800, periods=0.75, capacity=400_000, lepton_capacity=40_000)
    _same(big, W.rotating_e_initial(800, seed=13), "first, 800 seeds")
    small = W.rotating_e(n=150, periods=0.6, capacity=60_000, lepton_capacity=8_000)
    _same(small, W.rotating_e_initial(150, seed=14), "second, 150 seeds")


def test_noalloc_step_rejects_what_the_scratch_cannot_hold():
    w = W.rotating_e(n=10, periods=0.1, capacity=3_000_000, lepton_capacity=1000)
    e = R.engine_single(w, W.rotating_e_initial(10, seed=1), arena_records=0)
    need = Q.qed_work_bytes(1, 3_000_000, 0, False)
    assert need > Q.QED_STEP_SCRATCH_BYTES
    with pytest.raises(Q.QedError, match="scratch"):
        Q.qed_step_noalloc(e.tables.data_ptr(), e.stores, R.field_of(w), R.params_of(w),
                           e.step_ctr.data_ptr(), e.stats_buf.data_ptr(), e.stream)
    torch.cuda.synchronize()
    assert int(e.step_ctr.item()) == 0  # nothing was launched
