"""Pins of the oracle's single-particle pieces against closed forms and
independent numerical routes (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import parquet as P
from workloads import config, random_sigma


def test_semicircle_g0_matches_quadrature():
    # G0(i nu) = int rho(e) / (i nu - e) de with rho(e) = 2/(pi D^2) sqrt(D^2 - e^2)
    D = 2.0
    for nu in (0.3, -0.7, 1.9, 12.0, -40.0):
        rho = lambda e: 2.0 / (math.pi * D**2) * math.sqrt(max(D * D - e * e, 0.0))
        re = integrate.quad(lambda e: rho(e) * (-e) / (nu * nu + e * e), -D, D, epsabs=1e-13)[0]
        im = integrate.quad(lambda e: rho(e) * (-nu) / (nu * nu + e * e), -D, D, epsabs=1e-13)[0]
        got = P.g0_semicircle(np.array([nu]), D)[0]
        assert abs(got - (re + 1j * im)) < 1e-10


def test_semicircle_tail():
    nu = np.array([1e3, -2e3])
    g = P.g0_semicircle(nu, 2.0)
    assert np.allclose(g * (1j * nu), 1.0, atol=1e-5)


def _fermi(x, beta):
    return 0.5 * (1.0 - np.tanh(0.5 * beta * x))


def test_density_at_u0_is_fermi_sum():
    p = config("c3", U=0.0)
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    zero = np.zeros((g.Nve, g.Nk), complex)
    eps = P.dispersion(g, p.t, p.tp)
    for mu in (-0.7, 0.0, 0.35):
        G = P.dyson(p, g, zero, mu)
        n = P.density_per_spin(p, g, G, mu)
        assert abs(n - np.mean(_fermi(eps - mu, p.beta))) < 1e-12


def test_density_with_sigma_matches_brute_force_frequency_sum():
    # Independent route: sum Re G over a very long frequency window directly.
    p = config("tiny_2x2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    sig = random_sigma(g.Nve, g.Nk, seed=3, scale=0.3)
    sig = 0.5 * (sig + np.conj(sig[::-1]))      # Sigma(-nu) = Sigma(nu)^*
    mu = 0.21
    G = P.dyson(p, g, sig, mu)
    n_or = P.density_per_spin(p, g, G, mu)
    eps = P.dispersion(g, p.t, p.tp)
    M = 400000
    nn = np.arange(-M, M)
    nu = (2 * nn + 1) * math.pi / p.beta
    tot = 0.0
    lo = -g.Nve // 2
    for K in range(g.Nk):
        s = np.zeros(2 * M, complex)
        s[M + lo:M + lo + g.Nve] = sig[:, K]
        gk = 1.0 / (1j * nu + mu - eps[K] - s)
        tot += np.sum(gk.real)
    n_bf = 0.5 + tot / p.beta / g.Nk
    # remaining tail beyond M: |xi| T sum 1/nu^2 ~ |xi| beta / (pi^2 M) ~ 1e-6
    assert abs(n_or - n_bf) < 5e-6


def test_find_mu_hits_filling_and_half_filling_symmetry():
    p = config("tiny_2x2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    zero = np.zeros((g.Nve, g.Nk), complex)
    mu = P.find_mu(p, g, zero)
    G = P.dyson(p, g, zero, mu)
    assert abs(2 * P.density_per_spin(p, g, G, mu) - p.filling) < 1e-10
    # particle-hole symmetric lattice (t' = 0) at half filling -> mu~ = 0
    q = config("tiny_2x2_hf", mu_mode=1)
    g2 = P.Grid(q.Lx, q.Ly, q.Nv, q.f_ext)
    z2 = np.zeros((g2.Nve, g2.Nk), complex)
    assert abs(P.find_mu(q, g2, z2)) < 1e-12


def _lindhard_static(eps, epsq, beta):
    fa, fb = _fermi(eps, beta), _fermi(epsq, beta)
    d = epsq - eps
    same = np.abs(d) < 1e-12
    fprime = -beta * fa * (1 - fa)
    return np.where(same, fprime, (fb - fa) / np.where(same, 1.0, d))


def test_ph_bubble_tends_to_lindhard():
    # (T/N) sum_{k in box} G G at omega = 0 -> (1/N) sum_K [f(e_K) - f(e_{K+Q})]/(e_K - e_{K+Q})
    p = config("tiny_2x2", Nv=400, U=0.0)
    g = P.Grid(p.Lx, p.Ly, p.Nv, 1)
    zero = np.zeros((g.Nve, g.Nk), complex)
    mu = 0.13
    G = P.dyson(p, g, zero, mu)
    xph, xpp = P.bubbles(p, g, G)
    eps = P.dispersion(g, p.t, p.tp) - mu
    for Q in range(g.Nk):
        s = xph[g.qidx(0, Q)].sum()
        epsq = eps[g.kadd(np.arange(g.Nk), Q)]
        ref = np.mean(_lindhard_static(eps, epsq, p.beta))
        # truncation: T sum_{|n|>Nv/2} 1/nu^2 = O(beta / (pi^2 Nv))
        assert abs(s - ref) < 3 * p.beta / (math.pi**2 * p.Nv)
        assert abs(s.imag) < 1e-12


def test_pp_bubble_tends_to_closed_form():
    # (T/2N) sum G(k) G(q-k) at q = (Q, 0) -> (1/2N) sum_K (1 - f(a) - f(b)) / (a + b)
    p = config("tiny_2x2", Nv=400, U=0.0)
    g = P.Grid(p.Lx, p.Ly, p.Nv, 1)
    zero = np.zeros((g.Nve, g.Nk), complex)
    mu = -0.4
    G = P.dyson(p, g, zero, mu)
    xph, xpp = P.bubbles(p, g, G)
    eps = P.dispersion(g, p.t, p.tp) - mu
    for Q in range(g.Nk):
        s = xpp[g.qidx(0, Q)].sum()
        a = eps
        b = eps[g.ksub(Q, np.arange(g.Nk))]
        fb = _fermi(b, p.beta)
        same = np.abs(a + b) < 1e-12
        ratio = np.where(same, p.beta * fb * (1 - fb),
                         (1 - _fermi(a, p.beta) - fb) / np.where(same, 1.0, a + b))
        ref = np.mean(ratio) / 2
        assert abs(s - ref) < 3 * p.beta / (math.pi**2 * p.Nv)


def test_pp_bubble_finite_transfer_matches_direct_pairs():
    # q = (Q, m != 0): the pp partner of nu_n is omega_m - nu_n, check against
    # an explicit (odd-integer) frequency bookkeeping.
    p = config("small_2x4", U=0.0)
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    sig = random_sigma(g.Nve, g.Nk, seed=11, scale=0.2)
    G = P.dyson(p, g, sig, 0.1)
    xph, xpp = P.bubbles(p, g, G)
    T = 1.0 / p.beta

    def Gof(odd, K):           # odd = 2n+1
        return G[(odd - 1) // 2 + g.NG // 2, K]

    for (m, Q) in [(1, 3), (-2, 5), (2, 0)]:
        for (n, K) in [(0, 1), (-3, 6), (2, 7)]:
            qi, ki = g.qidx(m, Q), g.kidx(n, K)
            odd_k = 2 * n + 1
            even_q = 2 * m
            ref_pp = T / (2 * g.Nk) * Gof(odd_k, K) * Gof(even_q - odd_k, g.ksub(Q, K))
            ref_ph = T / g.Nk * Gof(odd_k, K) * Gof(odd_k + even_q, g.kadd(K, Q))
            assert abs(xpp[qi, ki] - ref_pp) < 1e-15
            assert abs(xph[qi, ki] - ref_ph) < 1e-15


@pytest.mark.parametrize("t,tp", [(1.0, -0.2), (1.3, -0.37), (0.7, 0.25)])
def test_dispersion_at_high_symmetry_points(t, tp):
    """epsilon_K at the high-symmetry points of the square lattice, values that
    follow from cos 0 = 1, cos pi = -1, cos pi/2 = 0 alone:
    (0,0): -4t - 4t';  (pi,pi): 4t - 4t';  (pi,0) and (0,pi): 4t';
    (pi/2,0) and (0,pi/2): -2t;  (pi/2,pi/2): 0. A 4x4 grid (K = kx Ly + ky,
    k = 2 pi kx / Lx) and a 2x4 grid, which also fixes the orientation of the
    momentum index."""
    g = P.Grid(4, 4, 2, 1)
    eps = P.dispersion(g, t, tp)
    K = lambda kx, ky: kx * 4 + ky
    expect = {K(0, 0): -4 * t - 4 * tp, K(2, 2): 4 * t - 4 * tp, K(2, 0): 4 * tp, K(0, 2): 4 * tp,
              K(1, 0): -2 * t, K(0, 1): -2 * t, K(3, 0): -2 * t, K(1, 1): 0.0, K(1, 2): 2 * t}
    for k, v in expect.items():
        assert abs(eps[k] - v) < 1e-14, (k, eps[k], v)
    g2 = P.Grid(2, 4, 2, 1)
    e2 = P.dispersion(g2, t, tp)
    # kx in {0, pi}, ky in {0, pi/2, pi, 3pi/2}: K = kx_index * 4 + ky_index
    assert abs(e2[1] - (-2 * t)) < 1e-14          # (0, pi/2)
    assert abs(e2[4] - 4 * tp) < 1e-14            # (pi, 0)
    assert abs(e2[6] - (4 * t - 4 * tp)) < 1e-14  # (pi, pi)
    assert abs(e2[5] - 2 * t) < 1e-14             # (pi, pi/2)
