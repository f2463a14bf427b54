"""Pins of the oracle's counter-based generator, uniform mapping and id rule."""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kats():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kats())
def test_philox_known_answers(orc, row):
    ctr, key, want = row[0:4], row[4:6], tuple(row[6:10])
    assert orc.philox(ctr, key) == want


def test_uniform_open_interval_endpoints(orc):
    assert orc.uniform(0, 0) == 2.0 ** -53
    assert orc.uniform(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert 0.0 < orc.uniform(0xFFFFFFFF, 0xFFFFFFFF) < 1.0
    # the top 52 bits of hi:lo decide the value
    assert orc.uniform(0x00000FFF, 0) == orc.uniform(0, 0)
    assert orc.uniform(0x00001000, 0) == 3.0 * 2.0 ** -53


def test_uniformity_ks(orc):
    # 20000 consecutive counters, one key: both uniforms pass a KS test
    r1, r2 = [], []
    for i in range(20000):
        o = orc.philox([i, 0, 7, 0], [12345, 678])
        r1.append(orc.uniform(o[0], o[1]))
        r2.append(orc.uniform(o[2], o[3]))
    assert stats.kstest(r1, "uniform").pvalue > 1e-3
    assert stats.kstest(r2, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(r1, r2)[0, 1]) < 0.03


def test_child_id_rule(orc):
    a = orc.child_id(5, 0, 3, 2, 1)
    assert a == orc.child_id(5, 0, 3, 2, 1)  # deterministic
    assert a >> 63 == 1  # children carry the top bit; seed ids are small
    ids = {orc.child_id(5, 0, 3, 2, p) for p in (1, 2, 3)}
    ids |= {orc.child_id(5, 0, 3, 3, 1), orc.child_id(5, 0, 4, 2, 1), orc.child_id(6, 0, 3, 2, 1),
            orc.child_id(5, 1, 3, 2, 1)}
    assert len(ids) == 7
    # the id is the first 64-bit word of Philox(key=parent, ctr=(step, substep|purpose<<16, seed))
    o = orc.philox([3, 2 | (1 << 16), 0, 0], [5, 0])
    assert a == ((o[1] << 32) | o[0]) | (1 << 63)
