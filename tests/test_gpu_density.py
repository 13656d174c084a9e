"""GPU parity of the spectrum-splitting Rayleigh-Ritz output and the nodal
electron density (Alg. 4, Alg. 5) against the oracle."""
import numpy as np
import pytest

import paper_1903_10959_amd as P
from oracle import chfsi as och
from oracle import density as ode
from oracle import fem
import workload
from gpu_util import make_ctx, oracle_apply, to_gpu, to_host

pytestmark = pytest.mark.gpu

SIGMA = 0.02


def _setup(ncols, seed):
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = och.cholgs(workload.start_block(c.n_dof, ncols, seed))
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    minv = 1.0 / np.sqrt(fem.mass_diag_kron(prob.L, prob.n_el, prob.p))
    return c, X, ap, minv


@pytest.mark.parametrize("ncols,n_fr", [(24, 4), (97, 15), (65, 1), (40, 40), (130, 20)])
def test_split_out_of_place_equals_in_place_and_keeps_X(ncols, n_fr):
    c, X, ap, _ = _setup(ncols, 700 + ncols)
    import torch
    Xg = to_gpu(X)
    Xfr = torch.full((X.shape[0], n_fr + 3), np.nan, dtype=torch.float64, device=Xg.device)[:, :n_fr]
    ev, rs = c.rayleigh_ritz_split(Xg, n_fr, mixed=False, Xfr=Xfr)
    assert np.array_equal(to_host(Xg), X)
    Xin = to_gpu(X)
    ev2, rs2 = c.rayleigh_ritz_split(Xin, n_fr, mixed=False)
    np.testing.assert_allclose(ev, ev2, rtol=0, atol=1e-14 * np.max(np.abs(ev2)))
    np.testing.assert_allclose(to_host(Xfr), to_host(Xin)[:, ncols - n_fr:], rtol=0, atol=1e-14)
    np.testing.assert_allclose(rs, rs2, rtol=1e-8, atol=1e-13)
    # against the oracle's Alg. 4 (vectors up to sign)
    Xo, Do, ro = ode.rayleigh_ritz_split(ap, X, n_fr)
    scale = max(1.0, np.max(np.abs(Do)))
    np.testing.assert_allclose(ev, Do, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(rs, ro, rtol=1e-6, atol=1e-11 * scale)
    G = to_host(Xfr)
    sgn = np.sign(np.sum(G * Xo, axis=0))
    assert np.max(np.abs(G * sgn - Xo)) < 1e-8
    c.close()


def test_split_rejects_overlapping_output():
    c, X, _, _ = _setup(24, 5)
    Xg = to_gpu(X)
    with pytest.raises(P.ChfsiError):
        c.rayleigh_ritz_split(Xg, 4, mixed=False, Xfr=Xg[:, 20:24])
    c.close()


@pytest.mark.parametrize("ncols,n_fr,frac", [(24, 4, 0.5), (97, 15, 0.37), (65, 1, 0.5), (40, 40, 0.8),
                                             (130, 20, 0.05), (200, 30, 0.95), (1100, 120, 0.4),
                                             (1030, 2, 0.5)])
def test_density_matches_oracle(ncols, n_fr, frac):
    """Element by element against the oracle's Alg. 4 + Alg. 5 on the same
    block; and the particle count sum_j M_jj rho_j = N_e."""
    import torch
    c, X, ap, minv = _setup(ncols, 800 + ncols)
    n_oc = ncols - n_fr
    ne = 2 * (n_oc + frac * n_fr)
    Xg = to_gpu(X)
    Xfr = torch.empty((X.shape[0], n_fr), dtype=torch.float64, device=Xg.device)
    ev, _ = c.rayleigh_ritz_split(Xg, n_fr, mixed=False, Xfr=Xfr)
    mu = P.fermi_level(ev, n_oc, ne, SIGMA)
    rho = to_host(c.density(Xg, Xfr, ev, mu, SIGMA))
    Xo, Do, _ = ode.rayleigh_ritz_split(ap, X, n_fr)
    mu_o = ode.fermi_level(Do, n_oc, ne, SIGMA)
    rho_o = ode.density_split(X, Xo, Do, mu_o, SIGMA, minv)
    np.testing.assert_allclose(rho, rho_o, rtol=0, atol=1e-11 * np.max(rho_o))
    M = 1.0 / minv ** 2
    assert abs(np.sum(M * rho) - ne) < 1e-11 * ne
    c.close()


def test_density_fully_occupied_and_ragged_ld():
    """n_fr = 0 (no fractional states) with a padded row stride and an odd
    column count (the scalar-load path)."""
    c, X, _, minv = _setup(33, 9)
    Xg = to_gpu(X, ld=40)
    rho = to_host(c.density(Xg))
    np.testing.assert_allclose(rho, 2 * minv ** 2 * np.sum(X * X, axis=1), rtol=1e-13, atol=0)
    c.close()


def test_density_from_mixed_split_keeps_the_particle_count():
    """The mixed projection perturbs Q_fr at FP32 level but Q_fr stays
    orthonormal, so the density still integrates to N_e; it differs from the
    FP64 density at FP32 level."""
    import torch
    c, X, _, minv = _setup(130, 31)
    n_fr, n_oc = 20, 110
    ne = 2 * (n_oc + 0.4 * n_fr)
    Xg = to_gpu(X)
    out = {}
    for mixed in (False, True):
        Xfr = torch.empty((X.shape[0], n_fr), dtype=torch.float64, device=Xg.device)
        ev, _ = c.rayleigh_ritz_split(Xg, n_fr, mixed=mixed, Xfr=Xfr)
        mu = P.fermi_level(ev, n_oc, ne, SIGMA)
        out[mixed] = to_host(c.density(Xg, Xfr, ev, mu, SIGMA))
    M = 1.0 / minv ** 2
    assert abs(np.sum(M * out[True]) - ne) < 1e-10 * ne
    d = np.max(np.abs(out[True] - out[False])) / np.max(out[False])
    assert d < 1e-4, d
    c.close()


def test_density_argument_checks():
    c, X, _, _ = _setup(24, 3)
    Xg = to_gpu(X)
    import torch
    Xfr = torch.zeros((X.shape[0], 4), dtype=torch.float64, device=Xg.device)
    with pytest.raises(P.ChfsiError):
        c.density(Xg, Xfr, np.zeros(4), 0.0, 0.0)        # sigma must be positive
    c.close()
