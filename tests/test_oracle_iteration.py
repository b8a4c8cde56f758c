"""Whole-iteration pins of the oracle (no GPU): weak-coupling order, exact
half-filling invariants and the self-energy tail."""
import math

import numpy as np
import pytest

from oracle import parquet as P
from workloads import config


def test_weak_coupling_deviation_from_second_order_is_third_order():
    """Lambda = U is exact through O(U^3), so the converged PA self-energy differs
    from the second-order diagram of G0 by O(U^3): log-log slope 3."""
    base = config("tiny_2x2")
    devs = []
    us = (0.05, 0.1, 0.2)
    for U in us:
        p = base.replace(U=U)
        g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
        st = P.solve(p, max_iter=150, tol=1e-13)
        z = np.zeros((g.Nve, g.Nk), complex)
        mu0 = P.find_mu(p, g, z)
        s2 = P.sigma_tilde1(p, g, P.dyson(p, g, z, mu0), mu0)
        devs.append(np.max(np.abs(st.sigma - s2)))
    slopes = np.diff(np.log(devs)) / np.diff(np.log(us))
    assert np.all(slopes > 2.85) and np.all(slopes < 3.2)


@pytest.fixture(scope="module")
def c1_solution():
    p = config("c1")
    st = P.solve(p, max_iter=100)
    return p, st


def test_c1_converges_and_is_particle_hole_symmetric(c1_solution):
    p, st = c1_solution
    assert st.last_dsigma < p.tol
    # half filling with a symmetric density of states: Sigma(i nu) purely imaginary
    assert np.max(np.abs(st.sigma.real)) < 1e-13
    # and odd in nu
    s = st.sigma[:, 0]
    assert np.max(np.abs(s + s[::-1])) < 1e-13


def test_c1_tail_matches_second_moment(c1_solution):
    """Sigma(i nu) -> U^2 n_s (1 - n_s) / (i nu) with n_s = 1/2 (tail claim of the
    results section); corrections are O(1/nu^3), so nu Im Sigma is within a few
    per cent of -U^2/4 for nu between 10 and 30 here."""
    p, st = c1_solution
    g = P.Grid(1, 1, p.Nv, p.f_ext)
    n = g.fext()
    nu = g.nu(n, p.beta)
    sel = (nu > 10) & (nu < 31)
    c1 = nu[sel] * st.sigma[sel, 0].imag
    assert np.all(np.abs(c1 + p.U**2 / 4) < 0.06 * p.U**2 / 4)
    # and it approaches the moment from above as nu grows
    assert abs(c1[-1] + 0.25) < abs(c1[0] + 0.25)


def test_iteration_is_deterministic_for_resume():
    p = config("tiny_2x2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    st = P.init_state(p, g)
    a = P.iterate(p, P.iterate(p, st, g), g)
    b = P.iterate(p, P.iterate(p, st, g), g)
    assert np.array_equal(a.sigma, b.sigma) and np.array_equal(a.phi, b.phi)
