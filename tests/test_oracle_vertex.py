"""Pins of the oracle's two-particle pieces: kernel functions, the channel remap
(parquet equations), and the Bethe-Salpeter solve (no GPU)."""
import itertools

import numpy as np
import pytest

from oracle import parquet as P
from workloads import config, rand_complex, random_phi


def _grid(name, **kw):
    p = config(name, **kw)
    return p, P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)


def _separable_phi(g, seed):
    """Phi_r^{kk'}(q) = c_r(q) + u_r(k;q) + u_r(k';q): reproduced exactly by the
    second-level kernel value everywhere in the box."""
    c = rand_complex((4, g.Nq), seed)
    u = rand_complex((4, g.Nq, g.n), seed + 1)
    return c[:, :, None, None] + u[:, :, :, None] + u[:, :, None, :]


# ----------------------------------------------------------------- kernels
@pytest.mark.parametrize("edge_rule", [0, 1])
def test_second_level_kernel_reproduces_separable_phi(edge_rule):
    p, g = _grid("small_2x4")
    phi = _separable_phi(g, 5)
    K1, K2 = P.kernel_functions(g, phi, level=2, edge_rule=edge_rule)
    nk, Kk = g.kparts()
    mq, Qq = g.qparts()
    for r in range(4):
        kv = P.kernel_value(g, K1, K2, r, nk[None, :, None], Kk[None, :, None],
                            nk[None, None, :], Kk[None, None, :], mq[:, None, None], Qq[:, None, None])
        assert np.max(np.abs(kv - phi[r])) < 1e-13


def test_first_level_kernel_of_constant_phi_and_levels():
    p, g = _grid("tiny_2x2")
    c = rand_complex((4, g.Nq), 9)
    phi = np.broadcast_to(c[:, :, None, None], (4, g.Nq, g.n, g.n)).copy()
    K1, K2 = P.kernel_functions(g, phi, level=1)
    assert np.allclose(K1, c, atol=1e-14) and not np.any(K2)
    K1, K2 = P.kernel_functions(g, phi, level=2)
    assert np.allclose(K1, c, atol=1e-14) and np.max(np.abs(K2)) < 1e-14
    K1, K2 = P.kernel_functions(g, phi, level=0)
    assert not np.any(K1) and not np.any(K2)


def test_kernel_edges_follow_stripe_rule():
    g = P.Grid(2, 2, 8, 2)
    top, bot = 3, -4
    assert P.kernel_edges(g, P.CH_D, 2) == [top] and P.kernel_edges(g, P.CH_M, -1) == [bot]
    assert P.kernel_edges(g, P.CH_S, 2) == [bot] and P.kernel_edges(g, P.CH_T, -3) == [top]
    assert sorted(P.kernel_edges(g, P.CH_S, 0)) == [bot, top]
    assert P.kernel_edges(g, P.CH_D, 2, edge_rule=1) == [bot]


# ------------------------------------------------------------------- remap
def test_zero_phi_gives_lambda():
    p, g = _grid("tiny_2x2")
    phi = np.zeros((4, g.Nq, g.n, g.n), complex)
    K1, K2 = P.kernel_functions(g, phi)
    gam = P.remap(g, phi, K1, K2, P.pa_lambda(p.U))
    for r, lam in enumerate(P.pa_lambda(p.U)):
        assert np.all(gam[r] == lam)


@pytest.mark.parametrize("name,level", [("tiny_2x2", 2), ("small_2x4", 2), ("small_2x4", 1), ("tiny_local", 0)])
def test_crossing_symmetry_is_exact_for_random_phi(name, level):
    """F_d(q) = 1/2 F_s(k+k'+q) + 3/2 F_t(k+k'+q), F_m(q) = -1/2 F_s + 1/2 F_t,
    F_s(q) = 1/2 F_d(q-k-k') - 3/2 F_m(q-k-k'), F_t(q) = 1/2 F_d + 1/2 F_m
    (crossing-symmetry subsection): an algebraic identity of the parquet
    equations, so it must hold to rounding for any Phi whenever the partner
    transfer is in the box."""
    p, g = _grid(name)
    phi = random_phi(g.Nq, g.n, seed=77, scale=0.3)
    K1, K2 = P.kernel_functions(g, phi, level)
    gam = P.remap(g, phi, K1, K2, P.pa_lambda(p.U))
    F = gam + phi
    nk, Kk = g.kparts()
    mq, Qq = g.qparts()
    checked = 0
    for qi in range(g.Nq):
        for ki in range(g.n):
            for kpi in range(g.n):
                m, Q = mq[qi], Qq[qi]
                n, K = nk[ki], Kk[ki]
                n2, K2m = nk[kpi], Kk[kpi]
                mpp = n + n2 + m + 1
                if g.in_bbox(mpp):
                    qq = g.qidx(mpp, g.kadd(g.kadd(K, K2m), Q))
                    assert abs(F[0, qi, ki, kpi] - (0.5 * F[2, qq, ki, kpi] + 1.5 * F[3, qq, ki, kpi])) < 1e-12
                    assert abs(F[1, qi, ki, kpi] - (-0.5 * F[2, qq, ki, kpi] + 0.5 * F[3, qq, ki, kpi])) < 1e-12
                    checked += 1
                mst = m - n - n2 - 1
                if g.in_bbox(mst):
                    qq = g.qidx(mst, g.ksub(g.ksub(Q, K), K2m))
                    assert abs(F[2, qi, ki, kpi] - (0.5 * F[0, qq, ki, kpi] - 1.5 * F[1, qq, ki, kpi])) < 1e-12
                    assert abs(F[3, qi, ki, kpi] - (0.5 * F[0, qq, ki, kpi] + 0.5 * F[1, qq, ki, kpi])) < 1e-12
                    checked += 1
    assert checked > g.Nq * g.n


def test_remap_matches_dictionary_brute_force():
    """Independent bookkeeping: vertices keyed by physical Matsubara integers
    (odd 2n+1 for fermions, even 2m for bosons) and momentum tuples, the parquet
    equations evaluated with tuple arithmetic and explicit out-of-box rules."""
    p, g = _grid("tiny_2x2")
    phi = random_phi(g.Nq, g.n, seed=3, scale=0.4)
    K1, K2 = P.kernel_functions(g, phi, 2)
    gam = P.remap(g, phi, K1, K2, P.pa_lambda(p.U))
    L = (g.Lx, g.Ly)
    ferm = [2 * n + 1 for n in g.fbox()]
    bos = [2 * m for m in g.bbox()]
    moms = [(x, y) for x in range(g.Lx) for y in range(g.Ly)]
    kpts = [(w, k) for w in ferm for k in moms]
    qpts = [(w, k) for w in bos for k in moms]
    vert, k1d, k2d = {}, {}, {}
    for r in range(4):
        for a, q in enumerate(qpts):
            k1d[(r, q)] = K1[r, a]
            for b, k in enumerate(kpts):
                k2d[(r, k, q)] = K2[r, a, b]
                for c, kp in enumerate(kpts):
                    vert[(r, k, kp, q)] = phi[r, a, b, c]

    def add(x, y, s=1):
        return (x[0] + s * y[0], ((x[1][0] + s * y[1][0]) % L[0], (x[1][1] + s * y[1][1]) % L[1]))

    def P_(r, k1, k2, pp):
        key = (r, k1, k2, pp)
        if key in vert:
            return vert[key]
        if (r, pp) not in k1d:
            return 0.0
        v = k1d[(r, pp)]
        if (r, k1, pp) in k2d:
            v += k2d[(r, k1, pp)]
        if (r, k2, pp) in k2d:
            v += k2d[(r, k2, pp)]
        return v

    U = p.U
    for a, q in enumerate(qpts):
        for b, k in enumerate(kpts):
            for c, kp in enumerate(kpts):
                kq = add(k, q)
                kpmk = add(kp, k, -1)
                pp = add(add(k, kp), q)
                qmkp = add(q, kp, -1)
                qmkk = add(add(q, k, -1), kp, -1)
                gd = U - 0.5 * P_(0, k, kq, kpmk) - 1.5 * P_(1, k, kq, kpmk) + 0.5 * P_(2, k, kp, pp) + 1.5 * P_(3, k, kp, pp)
                gm = -U - 0.5 * P_(0, k, kq, kpmk) + 0.5 * P_(1, k, kq, kpmk) - 0.5 * P_(2, k, kp, pp) + 0.5 * P_(3, k, kp, pp)
                gs = 2 * U + 0.5 * P_(0, k, qmkp, kpmk) - 1.5 * P_(1, k, qmkp, kpmk) + 0.5 * P_(0, k, kp, qmkk) - 1.5 * P_(1, k, kp, qmkk)
                gt = -0.5 * P_(0, k, qmkp, kpmk) - 0.5 * P_(1, k, qmkp, kpmk) + 0.5 * P_(0, k, kp, qmkk) + 0.5 * P_(1, k, kp, qmkk)
                ref = np.array([gd, gm, gs, gt])
                assert np.max(np.abs(gam[:, a, b, c] - ref)) < 1e-13


# --------------------------------------------------------------------- BSE
def test_bse_first_iteration_is_rank_one_rpa():
    """From Gamma = F = Lambda the BSE is solved in closed form: with
    s(q) = sum_k X(k;q), Phi_d = U^2 s_ph/(1 - U s_ph), Phi_m = U^2 s_ph/(1 + U s_ph),
    Psi_s = -4U^2 s_pp/(1 + 2U s_pp), Psi_t = 0 (first-iteration discussion,
    which quotes the O(U^2) terms)."""
    p, g = _grid("small_2x4")
    st = P.init_state(p, g)
    mu = P.find_mu(p, g, st.sigma)
    G = P.dyson(p, g, st.sigma, mu)
    xph, xpp = P.bubbles(p, g, G)
    U = p.U
    gam = np.empty((4, g.Nq, g.n, g.n), complex)
    for r, lam in enumerate(P.pa_lambda(U)):
        gam[r] = lam
    phi = P.bse(g, gam, xph, xpp)
    sph = xph.sum(axis=1)[:, None, None]
    spp = xpp.sum(axis=1)[:, None, None]
    assert np.max(np.abs(phi[0] - U * U * sph / (1 - U * sph))) < 1e-12
    assert np.max(np.abs(phi[1] - U * U * sph / (1 + U * sph))) < 1e-12
    assert np.max(np.abs(phi[2] - (-4 * U * U * spp / (1 + 2 * U * spp)))) < 1e-12
    assert np.max(np.abs(phi[3])) < 1e-14


def test_bse_solution_satisfies_product_form():
    """Phi = s Gamma X F with F = Gamma + Phi, the BSE as printed (Eq. PA_F_Phi)."""
    p, g = _grid("tiny_2x2")
    gam = random_phi(g.Nq, g.n, seed=21, scale=1.0)
    xph = rand_complex((g.Nq, g.n), 22, 0.1)
    xpp = rand_complex((g.Nq, g.n), 23, 0.1)
    phi = P.bse(g, gam, xph, xpp)
    for r in range(4):
        X = xph if r < 2 else xpp
        F = gam[r] + phi[r]
        for qi in range(g.Nq):
            T = P.BSE_SIGN[r] * np.einsum("ab,b,bc->ac", gam[r, qi], X[qi], F[qi])
            assert np.max(np.abs(T - phi[r, qi])) < 1e-12


def test_bse_symmetric_gamma_gives_symmetric_f():
    """Push-through: Gamma^T = Gamma implies F = (1 - Gamma X)^{-1} Gamma = Gamma (1 - X Gamma)^{-1}
    is symmetric; catches a transposed operand in the solve."""
    n = 24
    A = rand_complex((n, n), 5)
    gam = A + A.T
    x = rand_complex((n,), 6, 0.05)
    phi = P.bse_block(gam, x, -1.0)
    F = gam + phi
    assert np.max(np.abs(F - F.T)) < 1e-12
