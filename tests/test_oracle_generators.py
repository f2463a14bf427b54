"""Statistical pins of the event generators (Sec. IV.G, Sec. V.A).

The modified generator draws r1, r2, takes delta = r1^3 and accepts when
r2 < 3 r1^2 P(r1^3); the accepted deltas must follow the density P(delta) of Eq. (24),
which is what the paper claims for it (no cutoff, no deficit).  Setup of the
paper's generator comparison: gamma = 100, chi = 1, 10^7 trials.  Expected counts per bin
come from the exact rate integrated with scipy; every bin must lie within 3 sigma.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from tests.test_oracle_bessel import printed


def _expected(orc, density, edges, n):
    exp = []
    for a, b in zip(edges[:-1], edges[1:]):
        exp.append(n * integrate.quad(density, a, b, epsabs=0, epsrel=1e-10, limit=200)[0])
    return np.array(exp)


def _check_bins(obs, exp, n, zmax=3.0):
    p = exp / n
    sig = np.sqrt(n * p * (1 - p))
    z = (obs - exp) / sig
    chi2 = float(np.sum(z ** 2))
    pval = stats.chi2.sf(chi2, len(obs))
    return np.abs(z).max(), pval


def test_modified_generator_reproduces_spectrum(orc):
    pv = printed()
    gamma, chi = pv["E4_gamma"][0], pv["E4_chi"][0]
    dtfac = 0.5 * gamma / 1.6  # keeps P_m <= ~0.5
    n = 10_000_000
    deltas = orc.emission_trials(chi, gamma, dtfac, key=0xE4, n=n, backend=orc.TABLE)
    # r1 in (0,1) => delta >= 2^-159; use log bins over [1e-9, 1) plus [0, 1e-9)
    edges = np.concatenate([[0.0], np.logspace(-9, -2, 15)[:-1], np.linspace(0.01, 1.0, 26)])
    obs, _ = np.histogram(deltas, bins=edges)
    dens = lambda d: orc.rate_emission(d, chi, gamma, dtfac, orc.EXACT)
    exp = _expected(orc, dens, edges, n)
    zmax, pval = _check_bins(obs, exp, n)
    assert zmax < 3.0, f"worst bin {zmax:.2f} sigma"
    assert pval > 1e-3
    # negative control: the reading delta = r1 (the generator's text in Sec. IV.G) would put the accepted r1
    # values, i.e. delta^(1/3), into the spectrum; that fails by a wide margin
    obs_bad, _ = np.histogram(np.cbrt(deltas), bins=edges)
    zbad, _ = _check_bins(obs_bad, exp, n)
    assert zbad > 50


def test_pair_generator_reproduces_spectrum(orc):
    chi, kabs = 2.0, 50.0
    dtfac = 20.0  # max P_p ~ 0.2
    n = 4_000_000
    de = orc.pair_trials(chi, kabs, dtfac, key=0xBEE, n=n, backend=orc.TABLE)
    edges = np.concatenate([[0.0], np.logspace(-6, -1.5, 8), np.linspace(0.05, 0.95, 19),
                            1 - np.logspace(-1.5, -6, 8), [1.0]])
    edges = np.unique(edges)
    obs, _ = np.histogram(de, bins=edges)
    dens = lambda d: orc.rate_pair(d, chi, kabs, dtfac, orc.EXACT)
    exp = _expected(orc, dens, edges, n)
    zmax, pval = _check_bins(obs[exp > 5], exp[exp > 5], n)
    assert zmax < 3.0, f"worst bin {zmax:.2f} sigma"
    assert pval > 1e-3
    # electron/positron symmetry of Eq. (30): P_p(d) = P_p(1-d)
    for d in (0.01, 0.2, 0.45):
        assert orc.rate_pair(d, chi, kabs, 1.0) == pytest.approx(orc.rate_pair(1 - d, chi, kabs, 1.0),
                                                                rel=1e-6)


def test_total_emission_probability(orc):
    """The acceptance fraction equals int_0^1 P(delta) d delta (no cutoff)."""
    gamma, chi, dtfac = 100.0, 1.0, 20.0
    n = 2_000_000
    k = len(orc.emission_trials(chi, gamma, dtfac, key=7, n=n))
    w = integrate.quad(lambda r: orc.rate_modified(r, chi, gamma, dtfac, orc.EXACT), 0, 1,
                       epsrel=1e-10, limit=200)[0]
    assert abs(k - n * w) < 4 * math.sqrt(n * w * (1 - w))
