"""GPU emission generators as trials (qed_generator_trials, Sec. IV.G) against the oracle,
in the setting of the paper's comparison of the generators (gamma = 100, chi = 1).

Both sides draw the same Philox words per trial, so the modified and alternative generators
give bit-identical deltas (r1^3 and r1) and the same decisions, except where r2 lies within
1e-12 of P (the two sides' tables and formulas differ by a few ulps there): such trials are
counted and must be rare.  The standard generator's delta solves W(delta) = r2 W(1) on both
sides with different quadratures and root finders: W agrees to about 1e-14 W(1), so delta
agrees within 1e-12 W(1) / P(delta) (the slope of W there) plus 1e-13 delta.  At the full
size of the comparison (10^7 trials per generator) a sample of trials is checked one by
one."""
import ctypes as C

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():
    pytest.skip("needs a HIP device", allow_module_level=True)

import torch  # noqa: E402

from paper_1412_6426_amd import qed as Q  # noqa: E402

GAMMA, CHI = 100.0, 1.0
DTFAC = 0.5 * GAMMA / 1.6
DMIN = 1e-3
KEY = 0xE4E4


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def tables():
    t = torch.zeros(Q.qed_table_bytes() + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    view = t[off:off + Q.qed_table_bytes()]
    Q.qed_build_tables(view.data_ptr(), Q.qed_table_bytes(), 0)
    torch.cuda.synchronize()
    return t, view.data_ptr()


def _gpu(tables, gen, n, first=0, chi=CHI, gamma=GAMMA, dtfac=DTFAC, dmin=DMIN):
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    wb = Q.qed_generator_work_bytes(gen, chi, dmin)
    work = torch.empty(max(wb, 1) + 256, dtype=torch.uint8, device="cuda")
    wp = work.data_ptr() + ((-work.data_ptr()) % 256)
    Q.qed_generator_trials(tables[1], gen, chi, gamma, dtfac, dmin, KEY, first, n,
                           out.data_ptr(), wp if wb else None, wb, 0)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _draws(orc, trial):
    o = orc.philox([trial & 0xFFFFFFFF, trial >> 32, 0, 0], [KEY & 0xFFFFFFFF, KEY >> 32])
    return orc.uniform(o[0], o[1]), orc.uniform(o[2], o[3])


def _check_pointwise(orc, gen, g, o, first, chi=CHI, gamma=GAMMA, dtfac=DTFAC):
    """Same decisions except near the threshold; deltas bit-exact."""
    diff = np.nonzero((g > 0) != (o > 0))[0]
    for i in diff:
        r1, r2 = _draws(orc, first + int(i))
        if gen == orc.GEN_MODIFIED:
            p = orc.rate_modified(r1, chi, gamma, dtfac)
        else:
            p = orc.rate_emission(r1, chi, gamma, dtfac)
        assert abs(r2 - p) < 1e-12, (i, r2, p)
    assert len(diff) <= 2
    both = (g > 0) & (o > 0)
    assert np.array_equal(g[both], o[both])
    return int(both.sum())


@pytest.mark.parametrize("gen", [Q.QED_GEN_MODIFIED, Q.QED_GEN_ALTERNATIVE])
def test_short_generators_match_oracle(orc, tables, gen):
    for first, n in ((0, 300_000), (12_345_678_901, 70_001)):
        _note(f"generator {gen}: trials {first}..{first + n}")
        g = _gpu(tables, gen, n, first)
        o = orc.generator_trials(gen, CHI, GAMMA, DTFAC, KEY, n, first=first)
        assert _check_pointwise(orc, gen, g, o, first) > 0.15 * n


def _check_standard(orc, g, o, first, chi=CHI, gamma=GAMMA, dtfac=DTFAC, dmin=DMIN):
    w1 = orc.standard_w(1.0 - 1e-15, chi, gamma, dtfac, dmin)
    diff = np.nonzero((g > 0) != (o > 0))[0]
    for i in diff:
        r1, _ = _draws(orc, first + int(i))
        assert abs(r1 - w1) < 1e-12 * w1, i
    assert len(diff) <= 2
    both = np.nonzero((g > 0) & (o > 0))[0]
    dens = np.array([orc.rate_emission(float(d), chi, gamma, dtfac) for d in o[both]])
    tol = 1e-12 * w1 / np.maximum(dens, 1e-300) + 1e-13 * o[both]
    err = np.abs(g[both] - o[both])
    assert np.all(err <= tol), float((err / tol).max())
    assert np.all(g[both] >= dmin * (1 - 1e-12))
    return len(both)


def test_standard_generator_matches_oracle(orc, tables):
    n = 60_000
    _note(f"standard generator: {n} trials")
    g = _gpu(tables, Q.QED_GEN_STANDARD, n)
    o = orc.generator_trials(orc.GEN_STANDARD, CHI, GAMMA, DTFAC, KEY, n, delta_min=DMIN)
    assert _check_standard(orc, g, o, 0) > 0.2 * n


@pytest.mark.parametrize("chi,gamma,dmin,dtfac", [(0.05, 2000.0, 1e-6, 6000.0),
                                                   (20.0, 1e4, 1e-8, 500.0)])
def test_standard_generator_other_states(orc, tables, chi, gamma, dmin, dtfac):
    """A small and a large chi (W(1) about 0.2 and 0.3): cutoffs whose first interval starts
    off the table's nodes, for chi = 20 below the table (z from 3e-10, the small-z series),
    and for chi = 0.05 a rate that vanishes well before delta = 1."""
    n = 20_000
    _note(f"standard generator chi={chi}: {n} trials")
    g = _gpu(tables, Q.QED_GEN_STANDARD, n, chi=chi, gamma=gamma, dtfac=dtfac, dmin=dmin)
    o = orc.generator_trials(orc.GEN_STANDARD, chi, gamma, dtfac, KEY, n, delta_min=dmin)
    assert _check_standard(orc, g, o, 0, chi=chi, gamma=gamma, dtfac=dtfac, dmin=dmin) > 100


def test_full_size_comparison_sampled(orc, tables):
    """10^7 trials per generator, in the launch configuration the bench times; 1500 trials
    spread over the range are recomputed by the oracle one by one."""
    n = 10_000_000
    idx = np.unique(np.concatenate([np.arange(0, 500), np.arange(n - 500, n),
                                    np.random.default_rng(3).integers(0, n, 500)]))
    for gen in (Q.QED_GEN_MODIFIED, Q.QED_GEN_ALTERNATIVE, Q.QED_GEN_STANDARD):
        _note(f"full size, generator {gen}")
        g = _gpu(tables, gen, n)
        o = np.array([orc.generator_trials(gen, CHI, GAMMA, DTFAC, KEY, 1, first=int(i),
                                           delta_min=DMIN)[0] for i in idx])
        if gen == Q.QED_GEN_STANDARD:
            for k, i in enumerate(idx):
                assert _check_standard(orc, g[i:i + 1], o[k:k + 1], int(i)) >= 0
        else:
            for k, i in enumerate(idx):
                _check_pointwise(orc, gen, g[i:i + 1], o[k:k + 1], int(i))
        # whole-run properties: no NaN, deltas in range, the cutoff respected
        assert np.all(np.isfinite(g)) and np.all((g >= 0) & (g < 1))
        if gen == Q.QED_GEN_STANDARD:
            assert g[g > 0].min() >= DMIN * (1 - 1e-12)


def test_empty_and_missing_tables(orc, tables):
    assert _gpu(tables, Q.QED_GEN_STANDARD, 0).size == 0
    raw = torch.zeros(Q.qed_table_bytes() + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    out = _gpu((raw, raw.data_ptr() + off), Q.QED_GEN_MODIFIED, 1000)
    assert np.all(np.isnan(out))


@pytest.mark.parametrize("dmin", [1e-3, 1e-9])
def test_standard_w_table_matches_oracle(orc, tables, dmin):
    """gamma W(1) / dtfac over chi in [1e-3, 1e3] (41 values): the GPU sums its 8-point rule
    over the table intervals in a tree, the oracle its 5-point rule in order; both agree to
    a few thousand additions' rounding."""
    n, lo, hi = 41, 1e-3, 1e3
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    Q.qed_standard_w_table(tables[1], lo, hi, n, dmin, out.data_ptr(), 0)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    chis = [lo * 2.0 ** (np.log2(hi / lo) * i / (n - 1)) for i in range(n)]
    o = np.array([orc.standard_w(1.0 - 1e-15, c, 1.0, 1.0, dmin) for c in chis])
    np.testing.assert_allclose(g, o, rtol=1e-12, atol=0)
    assert np.all(np.diff(g) > 0)  # more emission at larger chi


def test_standard_w_table_without_tables(tables):
    raw = torch.zeros(Q.qed_table_bytes() + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    Q.qed_standard_w_table(raw.data_ptr() + off, 0.1, 10.0, 3, 1e-3, out.data_ptr(), 0)
    torch.cuda.synchronize()
    assert np.all(np.isnan(out.cpu().numpy()))
