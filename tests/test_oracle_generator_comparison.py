"""Pins of the oracle's three emission generators of Sec. IV.G, run as independent trials in
the setting of the paper's comparison of their spectra (gamma = 100, chi = 1).

With P(delta) the density of Eq. (24) over one interval (prefactor dtfac):
* standard (Eqs. (22)-(23)): a photon with probability W(1) = int_{delta_min}^1 P, its delta
  the root of W(delta) = r2 W(1); so the emitted deltas have density P on [delta_min, 1] and
  nothing below the cutoff;
* alternative (Eq. (24)): delta = r1 accepted iff r2 < P(r1); its spectrum is min(P, 1),
  short of P wherever P > 1 (low energies);
* modified (Eq. (25)): the same draws as the step's generator.

W is checked against scipy's quadrature of the exact (Bessel) density, the inversion against
Eq. (22) recomputed from the trial's own draws, and each spectrum bin by bin against its
closed form (3.5 sigma), with the alternative generator's low-energy deficit as a negative
control."""
import math

import numpy as np
import pytest
from scipy import integrate

from tests.test_oracle_generators import _check_bins, _expected

GAMMA, CHI = 100.0, 1.0
DTFAC = 0.5 * GAMMA / 1.6  # max P_m about 0.5 (the modified generator stays valid)
DMIN = 1e-3


def _w_scipy(orc, x, backend):
    # density in log(delta): smooth, with the delta^(-2/3) edge tamed
    f = lambda t: orc.rate_emission(math.exp(t), CHI, GAMMA, DTFAC, backend) * math.exp(t)
    return integrate.quad(f, math.log(DMIN), math.log(x), epsabs=0, epsrel=1e-12, limit=400)[0]


def test_standard_w_is_the_integral_of_the_density(orc):
    for x in (2e-3, 0.01, 0.1, 0.5, 0.9, 0.99):
        w = orc.standard_w(x, CHI, GAMMA, DTFAC, DMIN, backend=orc.EXACT)
        assert w == pytest.approx(_w_scipy(orc, x, orc.EXACT), rel=1e-10), x
        # the tabulated rates follow the exact ones to the table's interpolation error
        wt = orc.standard_w(x, CHI, GAMMA, DTFAC, DMIN, backend=orc.TABLE)
        assert wt == pytest.approx(w, rel=2e-6), x
    assert orc.standard_w(DMIN, CHI, GAMMA, DTFAC, DMIN) == 0.0


def _draws(orc, key, trial):
    o = orc.philox([trial & 0xFFFFFFFF, trial >> 32, 0, 0], [key & 0xFFFFFFFF, key >> 32])
    return orc.uniform(o[0], o[1]), orc.uniform(o[2], o[3])


def test_standard_inversion_solves_its_equation(orc):
    """The trial's delta satisfies W(delta) = r2 W(1) (Eq. (22)), with W recomputed by scipy
    from the exact density; trials that emit are exactly those with r1 < W(1)."""
    key = 0x5D
    d = orc.generator_trials(orc.GEN_STANDARD, CHI, GAMMA, DTFAC, key, 400, delta_min=DMIN,
                             backend=orc.EXACT)
    w1 = _w_scipy(orc, 1.0 - 1e-12, orc.EXACT)
    checked = 0
    for i, delta in enumerate(d):
        r1, r2 = _draws(orc, key, i)
        assert (delta > 0.0) == (r1 < w1), i
        if delta > 0.0:
            assert DMIN <= delta < 1.0
            assert _w_scipy(orc, delta, orc.EXACT) == pytest.approx(r2 * w1, rel=1e-9, abs=1e-13)
            checked += 1
    assert checked > 80


def test_standard_generator_spectrum(orc):
    n = 400_000
    d = orc.generator_trials(orc.GEN_STANDARD, CHI, GAMMA, DTFAC, 0x57D, n, delta_min=DMIN)
    e = d[d > 0.0]
    w1 = orc.standard_w(1.0 - 1e-15, CHI, GAMMA, DTFAC, DMIN)
    assert abs(len(e) - n * w1) < 4.0 * math.sqrt(n * w1 * (1 - w1))
    assert e.min() >= DMIN  # the cutoff: nothing below delta_min
    edges = np.concatenate([np.logspace(-3, -2, 5)[:-1], np.linspace(0.01, 1.0, 21)])
    obs, _ = np.histogram(e, bins=edges)
    exp = _expected(orc, lambda x: orc.rate_emission(x, CHI, GAMMA, DTFAC, orc.EXACT), edges, n)
    zmax, pval = _check_bins(obs, exp, n)
    assert zmax < 3.5 and pval > 1e-3, (zmax, pval)


def test_alternative_generator_spectrum_is_capped_at_one(orc):
    """Accepted deltas follow min(P, 1): below delta about 0.065, where P(delta) > 1 at this
    interval, the alternative generator falls short of the spectrum."""
    n = 1_000_000
    d = orc.generator_trials(orc.GEN_ALTERNATIVE, CHI, GAMMA, DTFAC, 0xA17, n)
    e = d[d > 0.0]
    edges = np.concatenate([[1e-6], np.logspace(-4, -2, 6)[:-1], np.linspace(0.01, 1.0, 21)])
    obs, _ = np.histogram(e, bins=edges)
    dens = lambda x: orc.rate_emission(x, CHI, GAMMA, DTFAC, orc.EXACT)
    capped = _expected(orc, lambda x: min(dens(x), 1.0), edges, n)
    zmax, pval = _check_bins(obs, capped, n)
    assert zmax < 3.5 and pval > 1e-3, (zmax, pval)
    # negative control: against the full density the low bins are far short
    full = _expected(orc, dens, edges, n)
    low = edges[1:] <= 0.01
    z = (obs[low] - full[low]) / np.sqrt(full[low])
    assert z.min() < -20.0


def test_modified_trials_are_the_emission_trials(orc):
    """The modified generator's trials are the step generator's (same draws, same test)."""
    d = orc.generator_trials(orc.GEN_MODIFIED, CHI, GAMMA, DTFAC, 0xE4, 200_000)
    ref = orc.emission_trials(CHI, GAMMA, DTFAC, key=0xE4, n=200_000)
    assert np.array_equal(d[d > 0.0], ref)
    # a later block of trials continues the same stream
    tail = orc.generator_trials(orc.GEN_MODIFIED, CHI, GAMMA, DTFAC, 0xE4, 1000, first=199_000)
    assert np.array_equal(tail, d[199_000:])


def test_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.generator_trials(7, CHI, GAMMA, DTFAC, 1, 10)
    with pytest.raises(ValueError):
        orc.generator_trials(orc.GEN_STANDARD, CHI, GAMMA, DTFAC, 1, 10, delta_min=0.0)


@pytest.mark.parametrize("chi", [1e-3, 0.1, 1.0, 10.0, 1e3])
def test_standard_w_over_chi_is_the_photon_number_rate(orc, chi):
    """gamma W(1) / dtfac with a cutoff of 1e-15 is the photon number rate int_0^1 P: what
    the cutoff leaves out is about 3 x 0.52 chi^(2/3) delta_min^(1/3) (the small-delta form
    printed after Eq. (24)), 1e-5 of it here."""
    from tests.test_oracle_rates import photon_number_rate
    w = orc.standard_w(1.0 - 1e-15, chi, 1.0, 1.0, 1e-15)
    missing = 3.0 * 0.52 * chi ** (2.0 / 3.0) * 1e-5
    assert w + missing == pytest.approx(photon_number_rate(orc, chi), rel=3e-5)
