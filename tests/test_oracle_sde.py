"""Pins of the oracle's Schwinger-Dyson pieces (no GPU).

* Sigma~_1 (second-order diagram at all frequencies, imaginary-time route) is the
  limit of the direct double Matsubara sum over growing windows W (1/W^2 at
  particle-hole symmetry, 1/W otherwise), equals U^2/(4 i nu) in the atomic
  limit, and its quadrature is converged.
* The whole Bethe-Salpeter -> remap -> Schwinger-Dyson chain at O(U^3): with G
  held fixed, the second iteration from the bare vertex must reproduce the
  third-order ladder diagrams in closed form,
      Sigma3(k) = (U^3 T^2 / 2N^2) sum_{k',q} [ w_ph (chi_ph(k'-k) + chi_pp(k+k'+q))
                                              + w_pp (chi_pp(q) + chi_ph(k'-k)) ]
  restricted to the summation domain the kernel level implies
  (w_ph = G(k+q)G(k'+q)G(k'), w_pp = G(q-k')G(q-k)G(k'),
   chi_ph(p) = (T/N) sum_{k''} G(k'')G(k''+p), chi_pp(p) = (T/N) sum G(k'')G(p-k'')).
  At level 0 this exercises sigma_box, at level 1 sigma_tilde2.
* The textbook limit of that closed form: for the particle-hole symmetric
  impurity the particle-hole and particle-particle third-order terms cancel.
* Special cases: Phi = 0 gives Sigma = Sigma~_1; a Phi that the kernel
  functions reproduce exactly gives a zero box correction."""
import math

import numpy as np
import pytest

from oracle import parquet as P
from workloads import config, rand_complex


def _direct_second_order(p, g, G, pts):
    """-(U^2 T^2/2N^2) sum over the extended box of the two G G G products, written
    out with explicit frequency bookkeeping (independent of the oracle's tau route)."""
    T = 1.0 / p.beta
    Gf = lambda odd, K: G[(odd - 1) // 2 + g.NG // 2, K]
    out = []
    for (n, K) in pts:
        o = 2 * n + 1
        tot = 0.0
        for n2 in g.fext():
            o2 = 2 * n2 + 1
            for K2 in range(g.Nk):
                for m in g.bext():
                    e = 2 * m
                    for Q in range(g.Nk):
                        tot += Gf(o + e, g.kadd(K, Q)) * Gf(o2 + e, g.kadd(K2, Q)) * Gf(o2, K2)
                        tot += Gf(e - o2, g.ksub(Q, K2)) * Gf(e - o, g.ksub(Q, K)) * Gf(o2, K2)
        out.append(-p.U**2 * T**2 / (2 * g.Nk**2) * tot)
    return np.array(out)


def test_sigma_tilde1_local_is_the_limit_of_growing_matsubara_windows():
    """The all-frequency second-order diagram is the limit of the direct double
    Matsubara sum; at particle-hole symmetry the truncation falls like 1/W^2."""
    p = config("tiny_local", Nv=8)
    g = P.Grid(1, 1, 8, 2)
    G = P.dyson(p, g, np.zeros((g.Nve, 1), complex), 0.0)
    pts = [(0, 0), (1, 0), (-4, 0)]
    ref = P.sigma_tilde1(p, g, G, 0.0, k_list=pts)
    errs = []
    for f in (4, 8, 16):
        gw = P.Grid(1, 1, 8, f)
        Gw = P.dyson(p, gw, np.zeros((gw.Nve, 1), complex), 0.0)
        errs.append(np.abs(_direct_second_order(p, gw, Gw, pts) - ref))
    errs = np.array(errs)
    ratio = errs[:-1] / errs[1:]
    assert np.all(ratio > 3.5) and np.all(ratio < 4.5)
    assert np.max(errs[-1]) < 2e-3 * np.max(np.abs(ref))


def test_sigma_tilde1_lattice_is_the_limit_of_growing_matsubara_windows():
    p = config("tiny_2x2", U=1.3)
    mu = 0.17
    g = P.Grid(p.Lx, p.Ly, 4, 2)
    G = P.dyson(p, g, np.zeros((g.Nve, g.Nk), complex), mu)
    pts = [(0, 0), (1, 1), (-1, 3)]
    ref = P.sigma_tilde1(p, g, G, mu, k_list=pts)
    vals = []
    for f in (4, 8, 16):
        gw = P.Grid(p.Lx, p.Ly, 4, f)
        Gw = P.dyson(p, gw, np.zeros((gw.Nve, gw.Nk), complex), mu)
        vals.append(_direct_second_order(p, gw, Gw, pts))
    vals = np.array(vals)
    errs = np.abs(vals - ref)
    ratio = errs[:-1] / errs[1:]
    # away from particle-hole symmetry the real 1/nu^2 tails truncate as 1/W
    assert np.all(ratio > 1.8) and np.all(ratio < 2.3)
    assert np.max(np.abs(2 * vals[2] - vals[1] - ref)) < 0.15 * np.max(errs[-1])


def test_sigma_tilde1_atomic_limit():
    """D -> 0: G0 = 1/(i nu), G(tau) = -1/2, Sigma2 = U^2/(4 i nu) exactly."""
    p = config("tiny_local", Nv=8, D=1e-4, U=1.7)
    g = P.Grid(1, 1, 8, 2)
    G = P.dyson(p, g, np.zeros((g.Nve, 1), complex), 0.0)
    s = P.sigma_tilde1(p, g, G, 0.0)[:, 0]
    nu = g.nu(g.fext(), p.beta)
    assert np.max(np.abs(s - p.U**2 / (4j * nu))) < 1e-6


def test_sigma_tilde1_quadrature_is_converged():
    p = config("tiny_2x2", U=1.1)
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    sig = rand_complex((g.Nve, g.Nk), 12, 0.2)
    mu = -0.3
    G = P.dyson(p, g, sig, mu)
    a = P.sigma_tilde1(p, g, G, mu)
    tau, wt = P.tau_grid(p, g, mu)
    x, w = np.polynomial.legendre.leggauss(2 * len(tau))
    orig = P.tau_grid
    try:
        P.tau_grid = lambda *args: (0.5 * p.beta * (x + 1), 0.5 * p.beta * w)
        b = P.sigma_tilde1(p, g, G, mu)
    finally:
        P.tau_grid = orig
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


# ------------------------------------------------------------- third order
def _chi(g, G, p_m, p_Q, T, pp):
    """chi(p) = (T/N) sum_{k'' in box} G(k'') G(k''+p) (ph) or G(k'') G(p-k'') (pp),
    written with odd/even Matsubara integers (independent bookkeeping)."""
    s = 0.0
    for n in g.fbox():
        for K in range(g.Nk):
            odd = 2 * n + 1
            if pp:
                o2, K2 = 2 * p_m - odd, g.ksub(p_Q, K)
            else:
                o2, K2 = odd + 2 * p_m, g.kadd(K, p_Q)
            s += G[(odd - 1) // 2 + g.NG // 2, K] * G[(o2 - 1) // 2 + g.NG // 2, K2]
    return T / g.Nk * s


def _third_order_closed_form(p, g, G, pts, level):
    T = 1.0 / p.beta
    chi_ph = {(m, Q): _chi(g, G, m, Q, T, False) for m in g.bbox() for Q in range(g.Nk)}
    chi_pp = {(m, Q): _chi(g, G, m, Q, T, True) for m in g.bbox() for Q in range(g.Nk)}
    Gf = lambda odd, K: G[(odd - 1) // 2 + g.NG // 2, K]
    if level == 0:
        kp_range, q_range = g.fbox(), g.bbox()
    else:
        kp_range, q_range = g.fext(), g.bext()
    out = []
    for (n, K) in pts:
        tot = 0.0
        o = 2 * n + 1
        for n2 in kp_range:
            o2 = 2 * n2 + 1
            for K2 in range(g.Nk):
                for m in q_range:
                    e = 2 * m
                    for Q in range(g.Nk):
                        wph = Gf(o + e, g.kadd(K, Q)) * Gf(o2 + e, g.kadd(K2, Q)) * Gf(o2, K2)
                        wpp = Gf(e - o2, g.ksub(Q, K2)) * Gf(e - o, g.ksub(Q, K)) * Gf(o2, K2)
                        pm = (o2 - o) // 2                      # k' - k
                        pQ = g.ksub(K2, K)
                        Pm = (o + o2 + e) // 2                  # k + k' + q
                        PQ = g.kadd(g.kadd(K, K2), Q)
                        a = chi_ph.get((pm, pQ), 0.0)
                        b = chi_pp.get((Pm, PQ), 0.0)
                        c = chi_pp.get((m, Q), 0.0)
                        if level == 0:
                            # box domain: the stored reducible vertex needs every argument in the box
                            in_f = lambda x: -g.Nv // 2 <= x <= g.Nv // 2 - 1
                            a1 = a if in_f((o + e - 1) // 2) else 0.0       # k+q in box
                            a3 = a if in_f((e - o2 - 1) // 2) else 0.0      # q-k' in box
                        else:
                            a1 = a3 = a
                        tot += wph * (a1 + b) + wpp * (c + a3)
        out.append(p.U**3 * T**2 / (2 * g.Nk**2) * tot)
    return np.array(out)


def _oracle_delta(p, g, G, pts, level):
    """Sigma after the bare-vertex BSE and one remap/SDE pass, minus Sigma~_1, with G fixed."""
    xph, xpp = P.bubbles(p, g, G)
    lam = P.pa_lambda(p.U)
    gam0 = np.empty((4, g.Nq, g.n, g.n), complex)
    for r in range(4):
        gam0[r] = lam[r]
    phi1 = P.bse(g, gam0, xph, xpp)
    K1, K2 = P.kernel_functions(g, phi1, level)
    gam = P.remap(g, phi1, K1, K2, lam)
    F = gam + phi1
    s = P.sigma_tilde2(p, g, G, K1, K2, k_list=pts)
    box = [i for i, (n, K) in enumerate(pts) if g.in_fbox(n)]
    if box:
        sb = P.sigma_box(p, g, G, F, K1, K2, k_list=[pts[i] for i in box])
        s[box] += sb
    return s


@pytest.mark.parametrize("level", [0, 1])
def test_third_order_ladders_from_the_parquet_chain(level):
    base = config("tiny_2x2", Nv=4, f_ext=2, kernel_level=level)
    g = P.Grid(base.Lx, base.Ly, base.Nv, base.f_ext)
    sig = rand_complex((g.Nve, g.Nk), 4, 0.1)
    G = P.dyson(base, g, sig, 0.05)                 # any fixed G
    pts = [(0, 0), (-1, 2), (1, 3)] + ([(3, 1), (-4, 0)] if level else [])
    u = 1e-3
    d1 = _oracle_delta(base.replace(U=u), g, G, pts, level)
    d2 = _oracle_delta(base.replace(U=2 * u), g, G, pts, level)
    c3_oracle = 2 * d1 / u**3 - d2 / (8 * u**3)     # Richardson: removes the O(U^4) term
    c3_closed = _third_order_closed_form(base.replace(U=1.0), g, G, pts, level)
    assert np.max(np.abs(c3_oracle - c3_closed)) < 1e-5 * np.max(np.abs(c3_closed))


def test_third_order_cancels_at_particle_hole_symmetry():
    """Symmetric impurity (semicircle, half filling): the ph and pp third-order
    ladders cancel (the known vanishing of the third-order self-energy of the
    symmetric Anderson model); on a finite window the cancellation is up to
    truncation, which shrinks as the box grows."""
    rel = []
    for Nv in (8, 16):
        p = config("tiny_local", Nv=Nv, U=1.0)
        g = P.Grid(1, 1, Nv, 2)
        G = P.dyson(p, g, np.zeros((g.Nve, 1), complex), 0.0)
        T = 1.0 / p.beta
        full = _third_order_closed_form(p, g, G, [(0, 0)], 1)[0]
        # the ph half alone (w_ph * chi_ph(k'-k) + w_pp * chi_ph(k'-k)): reference scale
        chi = {m: _chi(g, G, m, 0, T, False) for m in g.bbox()}
        Gf = lambda odd: G[(odd - 1) // 2 + g.NG // 2, 0]
        ph = 0.0
        for n2 in g.fext():
            for m in g.bext():
                o, o2, e = 1, 2 * n2 + 1, 2 * m
                a = chi.get(n2, 0.0)
                ph += (Gf(o + e) * Gf(o2 + e) * Gf(o2) + Gf(e - o2) * Gf(e - o) * Gf(o2)) * a
        ph *= T**2 / 2
        rel.append(abs(full) / abs(ph))
    assert rel[1] < rel[0] and rel[1] < 0.1


# ---------------------------------------------------------- special cases
def test_zero_phi_gives_second_order_only():
    p = config("tiny_2x2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    G = P.dyson(p, g, rand_complex((g.Nve, g.Nk), 1, 0.1), 0.1)
    phi = np.zeros((4, g.Nq, g.n, g.n), complex)
    K1, K2 = P.kernel_functions(g, phi)
    F = P.remap(g, phi, K1, K2, P.pa_lambda(p.U)) + phi
    s = P.sigma_sde(p, g, G, F, K1, K2, 0.1)
    assert np.max(np.abs(s - P.sigma_tilde1(p, g, G, 0.1))) < 1e-15


def test_box_correction_vanishes_when_kernels_are_exact():
    p = config("tiny_2x2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    G = P.dyson(p, g, rand_complex((g.Nve, g.Nk), 2, 0.1), 0.1)
    c = rand_complex((4, g.Nq), 8, 0.3)
    u = rand_complex((4, g.Nq, g.n), 9, 0.3)
    phi = c[:, :, None, None] + u[:, :, :, None] + u[:, :, None, :]
    K1, K2 = P.kernel_functions(g, phi, 2)
    F = P.remap(g, phi, K1, K2, P.pa_lambda(p.U)) + phi
    sb = P.sigma_box(p, g, G, F, K1, K2)
    assert np.max(np.abs(sb)) < 1e-14
    assert np.max(np.abs(P.sigma_tilde2(p, g, G, K1, K2))) > 1e-4


def test_semicircle_pole_sum_is_converged():
    """The pole representation of the semicircle no longer changes with the
    number of poles: G0 at every box frequency and Sigma~_1 of the local
    problem agree for 200 and 320 poles (and the pole sum equals the closed
    form of G0)."""
    p = config("c1")
    g = P.Grid(1, 1, p.Nv, p.f_ext)
    nu = g.nu(g.fext(), p.beta)
    g0 = P.g0_semicircle(nu, p.D)
    for M in (200, 320):
        e, c = P.semicircle_poles(p.D, M)
        gp = (c[None, :] / (1j * nu[:, None] - e[None, :])).sum(axis=1)
        assert np.max(np.abs(gp - g0)) < 1e-14
    G = P.dyson(p, g, np.zeros((g.Nve, 1), complex), 0.0)
    a = P.sigma_tilde1(p, g, G, 0.0)
    orig = P.semicircle_poles
    try:
        P.semicircle_poles = lambda D, M=320: orig(D, 320)
        b = P.sigma_tilde1(p, g, G, 0.0)
    finally:
        P.semicircle_poles = orig
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(a))


# ------------------------------------------------- without the regulation
def test_plain_sde_of_the_bare_vertex_is_the_box_truncated_second_order():
    """Without the regulation, F = Lambda (Phi = 0) gives the second-order
    diagram with both sums truncated to the box; the explicit odd/even
    Matsubara loops of _direct_second_order on the f = 1 grid (the box) are the
    independent route. second_order_box (the bare-vertex start) is the same sum."""
    for name in ("tiny_2x2", "tiny_local"):
        p = config(name, f_ext=1, regulation=0)
        g = P.Grid(p.Lx, p.Ly, p.Nv, 1)
        G = P.dyson(p, g, rand_complex((g.Nve, g.Nk), 5, 0.1), 0.07)
        phi = np.zeros((4, g.Nq, g.n, g.n), complex)
        K1, K2 = P.kernel_functions(g, phi)
        F = P.remap(g, phi, K1, K2, P.pa_lambda(p.U)) + phi
        pts = [(int(n), K) for n in g.fbox() for K in range(g.Nk)]
        direct = _direct_second_order(p, g, G, pts).reshape(g.Nv, g.Nk)
        assert np.max(np.abs(P.sigma_plain(p, g, G, F) - direct)) < 1e-14 * np.max(np.abs(direct))
        assert np.max(np.abs(P.second_order_box(p, g, G) - direct)) < 1e-14 * np.max(np.abs(direct))


def test_plain_sde_third_order_is_the_box_ladder():
    """Through the BSE -> remap -> SDE chain at kernel level 0, the plain box sum
    minus its second-order part is the third-order ladder closed form on the box
    domain (Richardson in U removes O(U^4))."""
    base = config("tiny_2x2", Nv=4, f_ext=1, kernel_level=0, regulation=0)
    g = P.Grid(base.Lx, base.Ly, base.Nv, 1)
    G = P.dyson(base, g, rand_complex((g.Nve, g.Nk), 4, 0.1), 0.05)
    pts = [(0, 0), (-1, 2), (1, 3), (-2, 1)]
    idx = [(n + g.Nv // 2, K) for (n, K) in pts]

    def delta(u):
        p = base.replace(U=u)
        xph, xpp = P.bubbles(p, g, G)
        lam = P.pa_lambda(u)
        gam0 = np.empty((4, g.Nq, g.n, g.n), complex)
        for r in range(4):
            gam0[r] = lam[r]
        phi1 = P.bse(g, gam0, xph, xpp)
        K1, K2 = P.kernel_functions(g, phi1, 0)
        F = P.remap(g, phi1, K1, K2, lam) + phi1
        d = P.sigma_plain(p, g, G, F) - P.second_order_box(p, g, G)
        return np.array([d[i] for i in idx])

    u = 1e-3
    c3 = 2 * delta(u) / u**3 - delta(2 * u) / (8 * u**3)
    closed = _third_order_closed_form(base.replace(U=1.0), g, G, pts, 0)
    assert np.max(np.abs(c3 - closed)) < 1e-5 * np.max(np.abs(closed))


@pytest.mark.parametrize("level", [1, 2])
def test_plain_sde_splits_into_the_regulated_pieces_on_the_box(level):
    """With the regulation box equal to the box (f = 1), the plain box sum of F
    splits exactly into the pieces of the regulated equation, the all-frequency
    second order replaced by its box truncation:
    sigma_plain = second_order_box + Sigma~_2 + Sigma_box(F - F~), for a random
    reducible vertex at kernel levels 1 and 2 (out-of-box arguments read the
    kernels)."""
    p = config("tiny_2x2", f_ext=1, kernel_level=level)
    g = P.Grid(p.Lx, p.Ly, p.Nv, 1)
    G = P.dyson(p, g, rand_complex((g.Nve, g.Nk), 6, 0.1), 0.1)
    phi = rand_complex((4, g.Nq, g.n, g.n), 13, 0.2)
    K1, K2 = P.kernel_functions(g, phi, level)
    F = P.remap(g, phi, K1, K2, P.pa_lambda(p.U)) + phi
    plain = P.sigma_plain(p.replace(regulation=0), g, G, F)
    parts = P.second_order_box(p, g, G) + P.sigma_tilde2(p, g, G, K1, K2) + P.sigma_box(p, g, G, F, K1, K2)
    assert np.max(np.abs(plain - parts)) < 1e-13 * np.max(np.abs(plain))
