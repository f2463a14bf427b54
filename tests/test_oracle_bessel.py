"""Pins of the oracle's Bessel-function integrals, series and tables.

The oracle evaluates K_{2/3}, int K_{5/3}, int K_{1/3} by DLMF 10.32.9 quadrature; here
they are checked against independent library routines (scipy.special.kv, adaptive
quadrature of kv, mpmath at 30 digits) and against the values the paper prints.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.txt")


def printed():
    out = {}
    with open(GOLD) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                out[line[0]] = (float(line[1]), float(line[2]))
    return out


@pytest.mark.parametrize("z", np.logspace(-7, math.log10(120.0), 23))
def test_k23_matches_scipy(orc, z):
    assert orc.B(z) == pytest.approx(special.kv(2.0 / 3.0, z), rel=2e-14)


@pytest.mark.parametrize("z", [1e-4, 1e-2, 0.3, 1.0, 3.0, 12.0, 60.0])
@pytest.mark.parametrize("nu", [5.0 / 3.0, 1.0 / 3.0])
def test_bessel_tail_integrals_match_quadrature(orc, nu, z):
    ref = integrate.quad(lambda t: special.kv(nu, t), z, np.inf, epsabs=0, epsrel=1e-13,
                         limit=500)[0]
    got = orc.A(z) if nu > 1 else orc.Cint(z)
    assert got == pytest.approx(ref, rel=2e-12)


@pytest.mark.parametrize("z", ["1e-9", "0.05", "1", "7.5", "40"])
def test_against_mpmath_30_digits(orc, z):
    mp.mp.dps = 30
    zz = mp.mpf(z)
    assert orc.B(float(z)) == pytest.approx(float(mp.besselk(mp.mpf(2) / 3, zz)), rel=2e-14)
    a = mp.quad(lambda t: mp.besselk(mp.mpf(5) / 3, t), [zz, zz + 1, mp.inf])
    c = mp.quad(lambda t: mp.besselk(mp.mpf(1) / 3, t), [zz, zz + 1, mp.inf])
    assert orc.A(float(z)) == pytest.approx(float(a), rel=2e-13)
    assert orc.Cint(float(z)) == pytest.approx(float(c), rel=2e-13)


def test_printed_synchrotron_values(orc):
    pv = printed()
    # Sec. IV.H: F1(x << 1) ~ 2.15 x^(1/3)
    coeff, tol = pv["F1_small_coeff"]
    assert orc.F1(1e-9) / 1e-3 == pytest.approx(coeff, rel=tol)
    # exact small-x coefficient 2^(2/3) Gamma(2/3) (DLMF 10.30.2 integrated)
    assert orc.F1(1e-12) / 1e-4 == pytest.approx(2 ** (2 / 3) * math.gamma(2 / 3), rel=1e-6)
    # Sec. IV.H: max F2 ~ 0.6
    xs = np.linspace(0.05, 2.0, 400)
    f2 = np.array([orc.F2(x) for x in xs])
    val, tol = pv["F2_max"]
    assert f2.max() == pytest.approx(val, rel=tol)
    # the maximum agrees with scipy's K_{2/3}
    assert f2.max() == pytest.approx(max(x * special.kv(2 / 3, x) for x in xs), rel=1e-12)


def test_series_region_matches_quadrature(orc):
    zlo = 2.0 ** orc.U_LO
    for z in np.logspace(-16, math.log10(zlo) - 1e-9, 12):
        a, b, c = orc.eval_abc(z, orc.TABLE)   # series branch
        A, B, Cc = orc.eval_abc(z, orc.EXACT)  # quadrature
        assert a == pytest.approx(A, rel=5e-13)
        assert b == pytest.approx(B, rel=5e-13)
        assert c == pytest.approx(Cc, rel=5e-13)


def test_series_constants_closed_forms(orc):
    t = orc.tables()
    g23, g13 = math.gamma(2 / 3), math.gamma(1 / 3)
    assert t.s_b0 == pytest.approx(0.5 * g23 * 2 ** (2 / 3), rel=1e-15)
    assert t.s_c0 == pytest.approx(math.pi / math.sqrt(3), rel=1e-15)
    # the z^(2/3) terms of int K_{5/3} = 2 K_{2/3} - int K_{1/3} cancel exactly
    assert 2 * t.s_b1 + t.s_c1 == pytest.approx(0.0, abs=1e-14)
    assert t.s_c1 == pytest.approx(0.75 * g13 * 2 ** (1 / 3), rel=1e-15)


def test_table_interpolation_error(orc):
    rng = np.random.default_rng(3)
    worst = 0.0
    for z in 2.0 ** rng.uniform(orc.U_LO, orc.U_HI, 4000):
        tab = orc.eval_abc(z, orc.TABLE)
        ex = orc.eval_abc(z, orc.EXACT)
        worst = max(worst, max(abs(a / b - 1.0) for a, b in zip(tab, ex)))
    assert worst < 3e-6
    # nodes are exact
    gA, gB, gC = orc.table_arrays()
    t = orc.tables()
    for i in (0, 1, 777, 2048, 4094):
        z = 2.0 ** (t.u_lo + i * t.du)
        assert gB[i] * math.exp(-z) == pytest.approx(special.kv(2 / 3, z), rel=2e-14)
    # beyond the last node the functions are taken as zero
    assert orc.eval_abc(2.0 ** orc.U_HI, orc.TABLE) == (0.0, 0.0, 0.0)


def test_table_layout(orc):
    t = orc.tables()
    assert t.n == orc.TABLE_N == 4096
    assert t.du == pytest.approx((orc.U_HI - orc.U_LO) / 4095, rel=1e-15)
