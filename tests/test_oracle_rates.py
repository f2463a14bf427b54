"""Pins of the oracle's emission and pair-creation rates (Eqs. (21), (24), (25), (30)).

Each rate is checked against closed forms that do not use the oracle's code: the
classical Larmor power (Eq. (7)), the quantum power of Eq. (15), the small-delta limit
printed after Eq. (24), the bounds of Eq. (27), photon-number and pair asymptotes
obtained analytically below (Mellin/Beta integrals of the small-z Bessel asymptotes and
Laplace's method), and the all-positive form of Eq. (30) evaluated with scipy.

Notation: dtfac = Delta t e^2 m c / hbar^2.  Integrals over delta are done in the
variable r1 with delta = r1^3 (the modified generator's change of variables), which
removes the delta^(-2/3) endpoint singularity.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from tests.test_oracle_bessel import printed

SQ3 = math.sqrt(3.0)
G23 = math.gamma(2.0 / 3.0)
B0 = 0.5 * G23 * 2.0 ** (2.0 / 3.0)  # K_{2/3}(z) ~ B0 z^(-2/3), DLMF 10.30.2


def _breaks(lo=1e-14, hi=1e-12):
    pts = [0.0] + [10.0 ** -k for k in range(12, 0, -1)] + [0.3, 0.5, 0.7]
    pts += [1.0 - 10.0 ** -k for k in range(1, 13)] + [1.0]
    return sorted(set(pts))


def integrate01(f):
    total = 0.0
    pts = _breaks()
    for a, b in zip(pts[:-1], pts[1:]):
        total += integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0]
    return total


def photon_number_rate(orc, chi, gamma=1e9):
    """W / (alpha/tau_C gamma^-1) = gamma/dtfac * int_0^1 P(delta) d delta."""
    return gamma * integrate01(lambda r: orc.rate_modified(r, chi, gamma, 1.0, orc.EXACT))


def radiated_power(orc, chi, gamma=1e9):
    """I / (e^2 m^2 c^3 / hbar^2) = gamma/dtfac * int_0^1 delta P(delta) d delta."""
    return gamma * integrate01(
        lambda r: r ** 3 * orc.rate_modified(r, chi, gamma, 1.0, orc.EXACT))


def pair_rate(orc, chi, kabs=1e9):
    """W_p / (alpha/tau_C (hbar w/m c^2)^-1) = kabs/dtfac * int_0^1 P_p d delta_e."""
    f = lambda d: orc.rate_pair(d, chi, kabs, 1.0, orc.EXACT)
    pts = [0.0, 1e-9, 1e-6, 1e-3, 0.05, 0.2, 0.4, 0.5, 0.6, 0.8, 0.95, 1 - 1e-3, 1 - 1e-6,
           1 - 1e-9, 1.0]
    return kabs * sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-11, limit=200)[0]
                      for a, b in zip(pts[:-1], pts[1:]))


# ---------------------------------------------------------------------------------------
def test_small_delta_limit_printed(orc):
    """Text after Eq. (24): P(delta<<1) ~ dtfac * 0.52 gamma^-1 chi^(2/3) delta^(-2/3).
    Exact constant: int_z^inf K_{5/3} ~ 2 B0 z^(-2/3) with z = 2 delta/(3 chi), so the
    coefficient is 2 B0 (3/2)^(2/3) / (sqrt(3) pi)."""
    val, tol = printed()["P_small_delta_coeff"]
    exact = 2 * B0 * 1.5 ** (2 / 3) / (SQ3 * math.pi)
    for chi in (0.1, 1.0, 10.0):
        gamma, delta = 50.0, 1e-15
        c = orc.rate_emission(delta, chi, gamma, 1.0, orc.EXACT) * gamma * delta ** (2 / 3) \
            / chi ** (2 / 3)
        assert c == pytest.approx(val, rel=tol)
        assert c == pytest.approx(exact, rel=1e-4)


def test_modified_generator_bounds_printed(orc):
    """Eq. (27): P_m(r1->0) ~ 1.5 chi^(2/3)/gamma (exact 3 x the constant above) and the
    high-energy branch max ~ 0.5 chi/gamma (= 4.5 max F2 / (sqrt(3) pi) chi/gamma)."""
    pv = printed()
    v1, t1 = pv["Pm_bound_first"]
    v2, t2 = pv["Pm_bound_second"]
    chi, gamma = 2.0, 300.0
    first = orc.rate_modified(1e-6, chi, gamma, 1.0, orc.EXACT) * gamma / chi ** (2 / 3)
    assert first == pytest.approx(v1, rel=t1)
    assert first == pytest.approx(6 * B0 * 1.5 ** (2 / 3) / (SQ3 * math.pi), rel=1e-3)
    # at very large chi the delta -> 1 branch dominates: max_r1 P_m ~ 0.5 chi / gamma
    chi = 1e6
    rs = 1.0 - np.logspace(-9, -1, 400)
    second = max(orc.rate_modified(r, chi, gamma, 1.0, orc.EXACT) for r in rs) * gamma / chi
    assert second == pytest.approx(v2, rel=t2)
    f2max = max(x * special.kv(2 / 3, x) for x in np.linspace(0.3, 0.55, 2001))
    assert second == pytest.approx(4.5 * f2max / (SQ3 * math.pi), rel=0.03)


def test_classical_limit_of_spectrum(orc):
    """Sec. IV.E: Eq. (21) reduces to the classical Eq. (20) for delta << 1, i.e.
    delta * P(delta) / F1(2 delta / (3 chi)) -> (sqrt(3)/(2 pi)) (chi/gamma) * dtfac."""
    chi, gamma = 0.7, 1e4
    for delta in (1e-9, 1e-7, 1e-5):
        ratio = delta * orc.rate_emission(delta, chi, gamma, 1.0, orc.EXACT) / \
            orc.F1(2 * delta / (3 * chi))
        assert ratio == pytest.approx(SQ3 / (2 * math.pi) * chi / gamma, rel=3 * delta / chi + 1e-12)


def test_classical_power_printed(orc):
    """Eq. (7): I^cl = (2/3) chi^2 in units e^2 m^2 c^3/hbar^2 (chi << 1)."""
    val, _ = printed()["I_classical_coeff"]
    chi = 1e-5
    assert radiated_power(orc, chi) / chi ** 2 == pytest.approx(val, rel=1e-4)


def test_power_first_quantum_correction(orc):
    """Known expansion of the quantum synchrotron power: (2/3) chi^2 (1 - (55 sqrt(3)/16) chi
    + O(chi^2)); pins the relative weight of the F2 term of Eq. (21) at small chi."""
    for chi in (1e-3, 3e-3):
        r = radiated_power(orc, chi) / ((2 / 3) * chi ** 2)
        assert (1 - r) / chi == pytest.approx(55 * SQ3 / 16, rel=0.02 + 60 * chi)


def test_quantum_power_printed(orc):
    """Eq. (15): I^q ~ 0.37 chi^(2/3) for chi >> 1.  With delta = y/(1+y) and the small-z
    asymptotes the limit is B0 (3/2)^(2/3) 64 / 243 ... = 32 * 3^(2/3) Gamma(2/3) / 243."""
    val, tol = printed()["I_quantum_coeff"]
    exact = 32 * 3 ** (2 / 3) * G23 / 243
    chi = 1e7
    c = radiated_power(orc, chi) / chi ** (2 / 3)
    assert c == pytest.approx(val, rel=tol)
    assert c == pytest.approx(exact, rel=2e-3)


def test_photon_number_rate_asymptotes(orc):
    """chi << 1: int_0^inf x K_{5/3}... gives W = (5/(2 sqrt 3)) chi (int_0^inf t K_{5/3} dt
    = 5 pi / 3, DLMF 10.43.19).  chi >> 1: W = 14 Gamma(2/3) / (9 * 3^(1/3)) chi^(2/3)
    (Beta integrals B(1/3,5/3) and B(7/3,2/3) of the small-z asymptotes)."""
    lo = 5 / (2 * SQ3)
    hi = 14 * G23 / (9 * 3 ** (1 / 3))
    chi = 1e-5
    assert photon_number_rate(orc, chi) / chi == pytest.approx(lo, rel=1e-4)
    chi = 1e7
    assert photon_number_rate(orc, chi) / chi ** (2 / 3) == pytest.approx(hi, rel=2e-3)


def test_pair_rate_asymptotes(orc):
    """chi_g << 1 (Laplace's method about delta_e = 1/2, z_p >= 8/(3 chi)):
    W_p -> (3 sqrt 3 / (16 sqrt 2)) chi e^(-8/(3 chi)), relative corrections O(chi).
    chi_g >> 1: W_p -> (15/28) 3^(2/3) Gamma(2/3)^4 / pi^2 chi^(2/3) (Beta(8/3, 2/3))."""
    lo = 3 * SQ3 / (16 * math.sqrt(2))
    ratios = {}
    for chi in (0.02, 0.01, 0.005):
        ratios[chi] = pair_rate(orc, chi) / (lo * chi * math.exp(-8 / (3 * chi)))
    assert abs(ratios[0.005] - 1) < abs(ratios[0.01] - 1) < abs(ratios[0.02] - 1)
    slope = (ratios[0.01] - ratios[0.005]) / 0.005
    assert ratios[0.005] - slope * 0.005 == pytest.approx(1.0, abs=2e-3)
    hi = (15 / 28) * 3 ** (2 / 3) * G23 ** 4 / math.pi ** 2
    chi = 1e7
    assert pair_rate(orc, chi) / chi ** (2 / 3) == pytest.approx(hi, rel=3e-3)


@pytest.mark.parametrize("chi", [0.05, 0.5, 3.0, 40.0])
def test_pair_rate_sign_reading(orc, chi):
    """Eq. (30) as printed has two negative factors, (delta_e - 1) delta_e and
    {F1 - 1.5 chi z F2}; their product must equal the positive Baier-Katkov form
    [(d/(1-d) + (1-d)/d) K_{2/3}(z) + int_z^inf K_{1/3}] / (sqrt(3) pi kabs) (scipy)."""
    kabs = 77.0
    for d in (1e-3, 0.1, 0.37, 0.5, 0.8, 0.999):
        z = 2.0 / (3.0 * chi * d * (1 - d))
        if z > 600:
            continue
        c13 = integrate.quad(lambda t: special.kv(1 / 3, t), z, np.inf, epsabs=0,
                             epsrel=1e-13)[0]
        ref = ((d / (1 - d) + (1 - d) / d) * special.kv(2 / 3, z) + c13) / (SQ3 * math.pi * kabs)
        got = orc.rate_pair(d, chi, kabs, 1.0, orc.EXACT)
        assert got > 0
        assert got == pytest.approx(ref, rel=1e-11)


def _tail_k53(z):
    """int_z^inf K_{5/3} by scipy quadrature on geometrically growing pieces."""
    edges = [z]
    while edges[-1] < 1.0:
        edges.append(edges[-1] * 4.0)
    total = sum(integrate.quad(lambda t: special.kv(5 / 3, t), a, b, epsabs=0, epsrel=1e-13)[0]
                for a, b in zip(edges[:-1], edges[1:]))
    return total + integrate.quad(lambda t: special.kv(5 / 3, t), edges[-1], np.inf, epsabs=0,
                                  epsrel=1e-13)[0]


@pytest.mark.parametrize("chi", [0.01, 0.3, 1.0, 20.0])
def test_emission_rate_against_scipy_form(orc, chi):
    """Eq. (24) equals dtfac [int_z^inf K_{5/3} + delta^2/(1-delta) K_{2/3}(z)]/(sqrt(3) pi gamma)
    (substituting z_q of Eq. (21)); right side from scipy."""
    gamma = 123.0
    for d in (1e-8, 1e-4, 0.05, 0.3, 0.7, 0.99):
        z = (2 / 3) * d / ((1 - d) * chi)
        if z > 600:
            continue
        a53 = _tail_k53(z)
        ref = (a53 + d * d / (1 - d) * special.kv(2 / 3, z)) / (SQ3 * math.pi * gamma)
        assert orc.rate_emission(d, chi, gamma, 1.0, orc.EXACT) == pytest.approx(ref, rel=1e-10)


def test_tabulated_rates_close_to_exact(orc):
    """Interpolated rates agree with the quadrature to the table's interpolation error; where
    the table returns zero (z >= 2^7) the exact rate is below 1e-40, far under the smallest
    uniform draw (2^-53), so no decision can differ."""
    rng = np.random.default_rng(11)
    worst_e = worst_p = 0.0
    for _ in range(2000):
        chi = 10 ** rng.uniform(-3, 3)
        r1 = rng.uniform(0, 1)
        for a, b in ((orc.rate_modified(r1, chi, 500.0, 1.0, orc.TABLE),
                      orc.rate_modified(r1, chi, 500.0, 1.0, orc.EXACT)),
                     (orc.rate_pair(r1, chi, 500.0, 1.0, orc.TABLE),
                      orc.rate_pair(r1, chi, 500.0, 1.0, orc.EXACT))):
            if a == 0.0:
                assert b < 1e-40
            else:
                worst_e = max(worst_e, abs(a / b - 1))
    assert worst_e < 3e-6


def test_zero_chi_and_edges(orc):
    assert orc.rate_modified(0.5, 0.0, 10.0, 1.0) == 0.0
    assert orc.rate_pair(0.5, 0.0, 10.0, 1.0) == 0.0
    assert orc.rate_emission(0.0, 1.0, 10.0, 1.0) == 0.0
    assert orc.rate_emission(1.0, 1.0, 10.0, 1.0) == 0.0
    # the r1 -> 0 limit of P_m is finite (the modified generator has no cutoff)
    p_small = orc.rate_modified(2.0 ** -53, 1.0, 10.0, 1.0)
    assert np.isfinite(p_small) and p_small > 0
