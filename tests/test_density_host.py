"""The library's Fermi level (a pure host function, Alg. 5 step 1) against
the oracle's, and its argument checks; CPU only."""
import numpy as np
import pytest

import paper_1903_10959_amd as P
from oracle import density


@pytest.mark.parametrize("seed,n_fr,n_oc,frac,sigma", [(1, 30, 5, 0.01, 0.02), (2, 30, 5, 0.5, 0.02),
                                                        (3, 154, 870, 0.37, 1.58e-3), (4, 1, 0, 0.5, 1e-3),
                                                        (5, 77, 435, 0.99, 1.58e-3), (6, 12, 3, 0.2, 0.5)])
def test_fermi_level_matches_oracle(seed, n_fr, n_oc, frac, sigma):
    rng = np.random.default_rng(seed)
    e = np.sort(rng.uniform(-0.6, -0.1, n_fr))
    ne = 2 * (n_oc + frac * n_fr)
    mu = P.fermi_level(e, n_oc, ne, sigma)
    mu_o = density.fermi_level(e, n_oc, ne, sigma)
    # both solve the same equation: compare through the count, and mu itself
    # where the count is not flat
    assert abs(density.electron_count(e, n_oc, mu, sigma) - ne) < 1e-10 * ne
    assert abs(mu - mu_o) < 1e-9 * max(1.0, abs(mu_o)) or \
        abs(density.electron_count(e, n_oc, mu_o, sigma) - ne) < 1e-10 * ne


def test_fermi_level_closed_forms():
    e = np.array([-0.412, -0.377])
    assert abs(P.fermi_level(e, 7, 16, 3e-3) - e.mean()) < 1e-13
    d = np.array([0.003, 0.011, 0.04])
    e = np.concatenate([0.25 - d, 0.25 + d])
    assert abs(P.fermi_level(e, 2, 2 * (2 + 3), 0.01) - 0.25) < 1e-13


def test_fermi_level_rejects_bad_input():
    e = np.array([0.1, 0.2, 0.3])
    for args in [(e, 4, 8.0, 0.01), (e, 4, 14.0, 0.01), (e, 4, 11.0, 0.0), (e, 4, 11.0, -1.0),
                 (e, -1, 1.0, 0.01), (np.array([0.1, np.nan]), 0, 1.0, 0.01), (np.zeros(0), 0, 1.0, 0.01)]:
        with pytest.raises(P.ChfsiError):
            P.fermi_level(*args)
