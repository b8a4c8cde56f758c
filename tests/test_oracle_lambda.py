"""Pins of the oracle's general (array-valued, local) fully irreducible vertex
Lambda_r(m; n, n') on the box (results section: full parquet and parquet DGA
take a local Lambda, extended by the parquet-approximation values):

* a box array equal to the parquet-approximation scalars reproduces the
  scalar path exactly, and a uniform array of the scalars of another U'
  reproduces the scalar path at U' (special cases that reduce);
* with a Lambda obeying the particle-hole / particle-particle crossing
  relations (built by crossing_lambda), the full vertex F = Gamma + Phi of a
  random Phi obeys the same crossing identities (the algebraic identity that
  pins the remap for the scalar Lambda): a Lambda entry added at the wrong
  transfer or in the wrong channel breaks it;
* crossing_lambda itself: the inverse relations hold at every partner pair."""
import numpy as np
import pytest

from oracle import parquet as P
from workloads import config, lambda_box_parts, random_phi


def _grid(name, **kw):
    p = config(name, **kw)
    return p, P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)


def _uniform(g, vals):
    out = np.empty((4, g.Nv - 1, g.Nv, g.Nv), dtype=np.complex128)
    for r in range(4):
        out[r] = vals[r]
    return out


@pytest.mark.parametrize("level", [0, 2])
def test_box_lambda_special_cases_reduce_to_scalar_path(level):
    p, g = _grid("tiny_2x2")
    phi = random_phi(g.Nq, g.n, seed=5, scale=0.3)
    K1, K2 = P.kernel_functions(g, phi, level)
    ref = P.remap(g, phi, K1, K2, P.pa_lambda(p.U))
    got = P.remap(g, phi, K1, K2, _uniform(g, P.pa_lambda(p.U)))
    assert np.max(np.abs(got - ref)) < 1e-14
    u2 = 0.7 * p.U
    ref2 = P.remap(g, phi, K1, K2, P.pa_lambda(u2))
    got2 = P.remap(g, phi, K1, K2, _uniform(g, P.pa_lambda(u2)))
    assert np.max(np.abs(got2 - ref2)) < 1e-14
    # a whole iteration with the box array equal to the scalars
    st = P.init_state(p, g)
    a = P.iterate(p, st, g)
    b = P.iterate(p, st, g, lam=_uniform(g, P.pa_lambda(p.U)))
    assert np.max(np.abs(a.sigma - b.sigma)) < 1e-14
    assert np.max(np.abs(a.phi - b.phi)) < 1e-14


def test_crossing_lambda_relations():
    p, g = _grid("tiny_2x2_hf")
    ld, lm = lambda_box_parts(g.Nv, seed=11, scale=0.5, symmetric=False)
    ld = ld + p.U
    lm = lm - p.U
    lam = P.crossing_lambda(g, p.U, ld, lm)
    checked = 0
    nv = g.Nv
    for jm in range(nv - 1):
        m = jm - (nv // 2 - 1)
        for i1 in range(nv):
            for i2 in range(nv):
                n, n2 = i1 - nv // 2, i2 - nv // 2
                mpp = n + n2 + m + 1                  # partner of a particle-hole transfer
                if g.in_bbox(mpp):
                    jp = mpp + nv // 2 - 1
                    assert abs(lam[0, jm, i1, i2] - (0.5 * lam[2, jp, i1, i2] + 1.5 * lam[3, jp, i1, i2])) < 1e-14
                    assert abs(lam[1, jm, i1, i2] - (-0.5 * lam[2, jp, i1, i2] + 0.5 * lam[3, jp, i1, i2])) < 1e-14
                    checked += 1
    assert checked > (nv - 1) * nv


@pytest.mark.parametrize("level", [0, 1, 2])
def test_full_vertex_with_crossing_lambda_obeys_crossing(level):
    p, g = _grid("tiny_2x2")
    ld, lm = lambda_box_parts(g.Nv, seed=12, scale=0.4, symmetric=False)
    lam = P.crossing_lambda(g, p.U, ld + p.U, lm - p.U)
    phi = random_phi(g.Nq, g.n, seed=78, scale=0.3)
    K1, K2 = P.kernel_functions(g, phi, level)
    F = P.remap(g, phi, K1, K2, lam) + phi
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


def test_misplaced_lambda_breaks_crossing():
    """The pin detects a plausible mistake: Lambda read at the wrong transfer
    (m shifted by one) violates the identity."""
    p, g = _grid("tiny_2x2")
    ld, lm = lambda_box_parts(g.Nv, seed=13, scale=0.4, symmetric=False)
    lam = P.crossing_lambda(g, p.U, ld + p.U, lm - p.U)
    bad = np.roll(lam, 1, axis=1)
    phi = np.zeros((4, g.Nq, g.n, g.n), dtype=np.complex128)
    K1, K2 = P.kernel_functions(g, phi, 0)
    F = P.remap(g, phi, K1, K2, bad)
    nk, Kk = g.kparts()
    mq, Qq = g.qparts()
    worst = 0.0
    for qi in range(g.Nq):
        for ki in range(g.n):
            for kpi in range(g.n):
                mpp = nk[ki] + nk[kpi] + mq[qi] + 1
                if g.in_bbox(mpp):
                    qq = g.qidx(mpp, g.kadd(g.kadd(Kk[ki], Kk[kpi]), Qq[qi]))
                    worst = max(worst, abs(F[0, qi, ki, kpi] - (0.5 * F[2, qq, ki, kpi] + 1.5 * F[3, qq, ki, kpi])))
    assert worst > 1e-3
