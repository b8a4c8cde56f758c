"""FP64 CPU oracle for one iteration of the parquet approximation (TEST INFRASTRUCTURE).

This module is the checker of the HIP path. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code with the GPU path and is written for legibility,
not speed: every function follows one equation of the paper (Li, Wentzell,
Pudleiner, Thunstroem, Held, "Efficient implementation of the parquet
equations -- role of the reducible vertex function and its kernel
approximation"), cited in its docstring.

Conventions (the GPU path documents the same layout in its C header; the index
arithmetic below is written independently):

* T = 1/beta, N = Nk = Lx*Ly momenta; K = (kx, ky) is stored as K = kx*Ly + ky,
  and k = 2 pi kx / Lx etc.  Momentum arithmetic is modulo the lattice.
* Fermionic Matsubara nu_n = (2n+1) pi T, bosonic omega_m = 2 m pi T.
  Box: n in [-Nv/2, Nv/2-1] (Nv values), m in [-(Nv/2-1), Nv/2-1] (Nv-1 values).
  Extended box (regulation sums): f*Nv fermionic, f*Nv-1 bosonic.
  Green's-function grid: NG = 2 f Nv fermionic frequencies.
* Compound indices are frequency-major: k = (n, K) -> (n + Nv/2)*Nk + K,
  q = (m, Q) -> (m + Nv/2 - 1)*Nk + Q.
* Vertex arrays are [channel][q][k][k'] with channels (d, m, s, t).
  G is [NG][Nk]; Sigma is [f*Nv][Nk]; bubbles are [Nq][n].
* Frequency sums of arguments:  k+q -> n+m (fermionic);  k'-k -> n'-n (bosonic);
  k+k'+q -> n+n'+m+1 (bosonic);  q-k' -> m-n'-1 (fermionic);
  q-k-k' -> m-n-n'-1 (bosonic).

Readings of the paper where it is silent or ambiguous are listed in the
repository's design notes; each is marked "reading" below.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against closed forms, exact algebraic identities, independent routes
(direct Matsubara sums, brute-force dictionaries, quadrature) or special cases:
single-particle pieces against quadrature, Fermi and Lindhard sums; the
kernels against vertices they reproduce exactly; the remap against the
crossing-symmetry identity and a dictionary brute force; the BSE against the
closed-form first iteration and the printed product form; Sigma~_1 against
growing direct Matsubara sums and the atomic limit; sigma_box and sigma_tilde2
(through the whole BSE -> remap -> SDE chain) against the closed-form
third-order ladder diagrams, whose particle-hole and particle-particle parts
cancel at particle-hole symmetry; a local box Lambda (full parquet / parquet
DGA input) against the scalar special cases and the crossing identities of F
for a crossing-symmetric Lambda.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

CH_D, CH_M, CH_S, CH_T = 0, 1, 2, 3
# Sign s_r of the Bethe-Salpeter kernel: Phi_{d/m} = +Gamma X F, Psi_t = +Gamma X F,
# Psi_s = -Gamma X F (Eq. PA_F_Phi, the "+-" of the pp line with t -> +, s -> -).
BSE_SIGN = (1.0, 1.0, -1.0, 1.0)


# ----------------------------------------------------------------------------
# grids and index arithmetic
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Grid:
    Lx: int
    Ly: int
    Nv: int
    f: int = 2

    def __post_init__(self):
        assert self.Nv % 2 == 0 and self.Nv >= 2
        self.Nk = self.Lx * self.Ly
        self.NW = self.Nv - 1
        self.Nve = self.f * self.Nv
        self.NWe = self.f * self.Nv - 1
        self.NG = 2 * self.f * self.Nv
        self.n = self.Nk * self.Nv
        self.Nq = self.Nk * self.NW
        kx, ky = np.divmod(np.arange(self.Nk), self.Ly)
        self.kx, self.ky = kx, ky

    # integer frequency ranges
    def fbox(self):
        return np.arange(-self.Nv // 2, self.Nv // 2)

    def bbox(self):
        return np.arange(-(self.Nv // 2 - 1), self.Nv // 2)

    def fext(self):
        return np.arange(-self.Nve // 2, self.Nve // 2)

    def bext(self):
        return np.arange(-(self.Nve // 2 - 1), self.Nve // 2)

    # membership
    def in_fbox(self, n):
        return (n >= -self.Nv // 2) & (n <= self.Nv // 2 - 1)

    def in_bbox(self, m):
        return (m >= -(self.Nv // 2 - 1)) & (m <= self.Nv // 2 - 1)

    def in_fext(self, n):
        return (n >= -self.Nve // 2) & (n <= self.Nve // 2 - 1)

    def in_bext(self, m):
        return (m >= -(self.Nve // 2 - 1)) & (m <= self.Nve // 2 - 1)

    # momentum arithmetic modulo the lattice
    def kadd(self, a, b):
        ax, ay = np.divmod(a, self.Ly)
        bx, by = np.divmod(b, self.Ly)
        return ((ax + bx) % self.Lx) * self.Ly + (ay + by) % self.Ly

    def kneg(self, a):
        ax, ay = np.divmod(a, self.Ly)
        return ((-ax) % self.Lx) * self.Ly + (-ay) % self.Ly

    def ksub(self, a, b):
        return self.kadd(a, self.kneg(b))

    # compound indices (caller guarantees the frequency is inside the range)
    def kidx(self, n, K):
        return (n + self.Nv // 2) * self.Nk + K

    def qidx(self, m, Q):
        return (m + self.Nv // 2 - 1) * self.Nk + Q

    def gidx(self, n):
        return n + self.NG // 2

    def eidx(self, n):
        return n + self.Nve // 2

    # decompositions of the box compound indices
    def kparts(self):
        idx = np.arange(self.n)
        i, K = np.divmod(idx, self.Nk)
        return i - self.Nv // 2, K

    def qparts(self):
        idx = np.arange(self.Nq)
        j, Q = np.divmod(idx, self.Nk)
        return j - (self.Nv // 2 - 1), Q

    def nu(self, n, beta):
        return (2 * np.asarray(n) + 1) * math.pi / beta


# ----------------------------------------------------------------------------
# single-particle part: model, Dyson equation, filling
# ----------------------------------------------------------------------------
def dispersion(grid: Grid, t: float, tp: float) -> np.ndarray:
    """epsilon_K of the square lattice (Eq. Hubbard); the t' term is the usual
    next-nearest-neighbour extension (reading: the paper has t only)."""
    ckx = np.cos(2 * math.pi * grid.kx / grid.Lx)
    cky = np.cos(2 * math.pi * grid.ky / grid.Ly)
    return -2.0 * t * (ckx + cky) - 4.0 * tp * ckx * cky


def g0_semicircle(nu: np.ndarray, D: float) -> np.ndarray:
    """Local non-interacting G for a semicircular density of states of
    half-bandwidth D, at z = i nu: (2/D^2) (z - i sgn(nu) sqrt(nu^2 + D^2)).
    Stand-in for the DMFT Weiss field that the results section feeds in."""
    nu = np.asarray(nu, dtype=float)
    return (2.0 / D**2) * (1j * nu - 1j * np.sign(nu) * np.sqrt(nu**2 + D**2))


def sigma_on_ggrid(grid: Grid, sigma_ext: np.ndarray) -> np.ndarray:
    """Sigma on the G grid: the stored values on the extended box, zero beyond
    (reading: Sigma is known on the extended box only)."""
    out = np.zeros((grid.NG, grid.Nk), dtype=np.complex128)
    lo = grid.gidx(-grid.Nve // 2)
    out[lo:lo + grid.Nve] = sigma_ext
    return out


def dyson(p, grid: Grid, sigma_ext: np.ndarray, mu: float) -> np.ndarray:
    """Dyson equation (Eq. PA_Dyson) on the G grid, fermionic frequencies.

    Lattice: G = 1/(i nu + mu~ - eps_K - Sigma), with the Hartree term absorbed
    into mu~ (the paper drops Hartree/Fock for the paramagnetic one-band model).
    Local (Nk = 1): G = 1/(1/G0 - Sigma) with the semicircle G0."""
    ng = np.arange(grid.NG) - grid.NG // 2
    nu = grid.nu(ng, p.beta)[:, None]
    sig = sigma_on_ggrid(grid, sigma_ext)
    if grid.Nk == 1:
        g0 = g0_semicircle(nu, p.D)
        return 1.0 / (1.0 / g0 - sig)
    eps = dispersion(grid, p.t, p.tp)[None, :]
    return 1.0 / (1j * nu + mu - eps - sig)


def density_per_spin(p, grid: Grid, G: np.ndarray, mu: float) -> float:
    """n_sigma = T/N sum_K sum_n G(K, i nu_n) e^{i nu 0+}.

    1/(i nu) contributes 1/2; the grid part is T/N sum Re G; beyond the G grid
    Sigma = 0, so G = 1/(i nu - xi_K) there and its real part -xi/(nu^2+xi^2)
    is summed in closed form using T sum_n 1/(nu_n^2 + xi^2) = tanh(beta xi/2)/(2 xi)."""
    T = 1.0 / p.beta
    N = grid.Nk
    total = 0.5 + (T / N) * float(np.sum(G.real))
    if grid.Nk == 1:
        return total  # local mode is only used at half filling; no tail needed
    eps = dispersion(grid, p.t, p.tp)
    xi = eps - mu
    npos = np.arange(grid.NG // 2)
    nu2 = grid.nu(npos, p.beta) ** 2
    tail = 0.0
    for x in xi:
        partial = float(np.sum(1.0 / (nu2 + x * x)))
        if abs(x) < 1e-300:
            full = p.beta**2 / 8.0
        else:
            full = p.beta * math.tanh(p.beta * x / 2.0) / (4.0 * x)
        tail += -x * (full - partial)
    return total + 2.0 * (T / N) * tail


def find_mu(p, grid: Grid, sigma_ext: np.ndarray) -> float:
    """mu~ such that 2 n_sigma = filling, by bisection (reading: the paper works at
    half filling and gives no rule; bisection is monotone in mu~ for fixed Sigma)."""
    if grid.Nk == 1 or p.mu_mode == 0:
        return float(p.mu_fixed)
    eps = dispersion(grid, p.t, p.tp)
    lo = float(eps.min()) - 10.0 - abs(p.U)
    hi = float(eps.max()) + 10.0 + abs(p.U)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        G = dyson(p, grid, sigma_ext, mid)
        n = 2.0 * density_per_spin(p, grid, G, mid)
        if n > p.filling:
            hi = mid
        else:
            lo = mid
        if hi - lo < 1e-14:
            break
    return 0.5 * (lo + hi)


# ----------------------------------------------------------------------------
# bubbles (the G G factors of the Bethe-Salpeter equations)
# ----------------------------------------------------------------------------
def g_at(grid: Grid, G: np.ndarray, n, K):
    """G(k) for fermionic index n (inside the G grid) and momentum index K."""
    return G[grid.gidx(np.asarray(n)), np.asarray(K)]


def bubbles(p, grid: Grid, G: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """X_ph(k;q) = (T/N) G(k) G(k+q) and X_pp(k;q) = (T/2N) G(k) G(q-k), k in the box
    (Eq. PA_F_Phi). Returned as [Nq][n]."""
    T = 1.0 / p.beta
    N = grid.Nk
    nk, Kk = grid.kparts()
    mq, Qq = grid.qparts()
    n_ = nk[None, :]
    K_ = Kk[None, :]
    m_ = mq[:, None]
    Q_ = Qq[:, None]
    gk = g_at(grid, G, np.broadcast_to(n_, (grid.Nq, grid.n)), np.broadcast_to(K_, (grid.Nq, grid.n)))
    g_kq = g_at(grid, G, n_ + m_, grid.kadd(K_, Q_))
    g_qmk = g_at(grid, G, m_ - n_ - 1, grid.ksub(Q_, K_))
    xph = (T / N) * gk * g_kq
    xpp = (T / (2 * N)) * gk * g_qmk
    return xph, xpp


# ----------------------------------------------------------------------------
# kernel functions (two-level parameter reduction of Phi)
# ----------------------------------------------------------------------------
def kernel_edges(grid: Grid, channel: int, m: int, edge_rule: int = 0):
    """Frequency index (or indices, averaged) of the box edge used to read the
    kernel of channel r at bosonic m. Reading of the first-level choice ("far
    away from the diagonal components and the stripes"): the ph channels have
    stripes near nu = 0 and nu = -omega, the pp channels near nu = 0 and nu = omega,
    so the edge on the other side is used; m = 0 averages both edges.
    edge_rule 1 takes the lowest edge always (the "k' = -30" example)."""
    top, bot = grid.Nv // 2 - 1, -grid.Nv // 2
    if edge_rule == 1:
        return [bot]
    if m == 0:
        return [top, bot]
    ph = channel in (CH_D, CH_M)
    if ph:
        return [top] if m > 0 else [bot]
    return [bot] if m > 0 else [top]


def kernel_functions(grid: Grid, phi: np.ndarray, level: int = 2, edge_rule: int = 0):
    """First-level K1_r(q) and second-level K2_r(k;q) kernels from the box-edge
    values of Phi_r (kernel-approximation subsection, first- and second-level
    paragraphs).

    K1_r(q)   = mean over K, K' of Phi_r^{(n_e,K),(n_e,K')}(q)
    K2_r(k;q) = mean over K'  of Phi_r^{k,(n_e,K')}(q) - K1_r(q)
    so that the second-level value K1 + K2(k) + K2(k') equals
    Phi~^k + Phi~^{k'} - Phi~ of the paper. Level 1: K2 = 0; level 0: both 0."""
    Nk = grid.Nk
    K1 = np.zeros((4, grid.Nq), dtype=np.complex128)
    K2 = np.zeros((4, grid.Nq, grid.n), dtype=np.complex128)
    if level == 0:
        return K1, K2
    mq, _ = grid.qparts()
    for r in range(4):
        for qi in range(grid.Nq):
            edges = kernel_edges(grid, r, int(mq[qi]), edge_rule)
            k1 = 0.0
            k2 = np.zeros(grid.n, dtype=np.complex128)
            for e in edges:
                cols = slice(grid.kidx(e, 0), grid.kidx(e, 0) + Nk)
                block = phi[r, qi][:, cols]            # [n][Nk]: all k, k' = (e, K')
                k2 = k2 + block.mean(axis=1)
                k1 = k1 + block[cols, :].mean()        # k = (e, K) rows
            K1[r, qi] = k1 / len(edges)
            K2[r, qi] = k2 / len(edges) - K1[r, qi]
    if level == 1:
        K2[:] = 0.0
    return K1, K2


def kernel_value(grid: Grid, K1, K2, r, n1, K1m, n2, K2m, mp, Qp):
    """Kernel approximation of Phi_r^{k1,k2}(p) for arbitrary arguments:
    K1_r(p) + [n1 in box] K2_r(k1;p) + [n2 in box] K2_r(k2;p) when p is inside
    the bosonic box, 0 otherwise (reading: transfers beyond the box are dropped,
    Phi decays like 1/omega^2 there)."""
    mp = np.asarray(mp)
    bp = grid.in_bbox(mp)
    b1 = grid.in_fbox(np.asarray(n1))
    b2 = grid.in_fbox(np.asarray(n2))
    mp_c = np.where(bp, mp, 0)
    qi = grid.qidx(mp_c, Qp)
    n1c = np.where(b1, n1, 0)
    n2c = np.where(b2, n2, 0)
    val = K1[r][qi] + np.where(b1, K2[r][qi, grid.kidx(n1c, K1m)], 0.0) \
        + np.where(b2, K2[r][qi, grid.kidx(n2c, K2m)], 0.0)
    return np.where(bp, val, 0.0)


def accessor(grid: Grid, phi, K1, K2, r, n1, K1m, n2, K2m, mp, Qp):
    """P_r(k1, k2; p): the stored Phi_r when every argument lies in the box,
    the kernel value otherwise (kernel approximation used only outside the box)."""
    n1 = np.asarray(n1)
    n2 = np.asarray(n2)
    mp = np.asarray(mp)
    inside = grid.in_fbox(n1) & grid.in_fbox(n2) & grid.in_bbox(mp)
    kv = kernel_value(grid, K1, K2, r, n1, K1m, n2, K2m, mp, Qp)
    qi = grid.qidx(np.where(inside, mp, 0), Qp)
    a = grid.kidx(np.where(inside, n1, 0), K1m)
    b = grid.kidx(np.where(inside, n2, 0), K2m)
    stored = phi[r][qi, a, b]
    return np.where(inside, stored, kv)


# ----------------------------------------------------------------------------
# the parquet equations: irreducible vertices from the reducible ones
# ----------------------------------------------------------------------------
def _remap_terms(grid: Grid, P, n, K, n2, K2, m, Q):
    """The eight reducible-vertex terms that enter Gamma_r at (q, k, k') with
    k = (n, K), k' = (n2, K2), q = (m, Q), for any accessor P(r, n1,K1, n2,K2, mp,Qp).

    ph-bar geometry:  P_{d,m}(k, k+q; k'-k)
    pp geometry:      P_{s,t}(k, k'; k+k'+q)
    s/t geometry 1:   P_{d,m}(k, q-k'; k'-k)
    s/t geometry 2:   P_{d,m}(k, k'; q-k-k')"""
    kpq_n, kpq_K = n + m, grid.kadd(K, Q)
    kpmk_m, kpmk_K = n2 - n, grid.ksub(K2, K)
    pp_m, pp_K = n + n2 + m + 1, grid.kadd(grid.kadd(K, K2), Q)
    qmkp_n, qmkp_K = m - n2 - 1, grid.ksub(Q, K2)
    qmkk_m, qmkk_K = m - n - n2 - 1, grid.ksub(grid.ksub(Q, K), K2)
    t = {}
    t["d_phbar"] = P(CH_D, n, K, kpq_n, kpq_K, kpmk_m, kpmk_K)
    t["m_phbar"] = P(CH_M, n, K, kpq_n, kpq_K, kpmk_m, kpmk_K)
    t["s_pp"] = P(CH_S, n, K, n2, K2, pp_m, pp_K)
    t["t_pp"] = P(CH_T, n, K, n2, K2, pp_m, pp_K)
    t["d_st1"] = P(CH_D, n, K, qmkp_n, qmkp_K, kpmk_m, kpmk_K)
    t["m_st1"] = P(CH_M, n, K, qmkp_n, qmkp_K, kpmk_m, kpmk_K)
    t["d_st2"] = P(CH_D, n, K, n2, K2, qmkk_m, qmkk_K)
    t["m_st2"] = P(CH_M, n, K, n2, K2, qmkk_m, qmkk_K)
    return t


def _combine_gamma(t, lam):
    """Coefficient tables of Eqs. PA_Gamma_dm and PA_Gamma_st."""
    gd = lam[0] - 0.5 * t["d_phbar"] - 1.5 * t["m_phbar"] + 0.5 * t["s_pp"] + 1.5 * t["t_pp"]
    gm = lam[1] - 0.5 * t["d_phbar"] + 0.5 * t["m_phbar"] - 0.5 * t["s_pp"] + 0.5 * t["t_pp"]
    gs = lam[2] + 0.5 * t["d_st1"] - 1.5 * t["m_st1"] + 0.5 * t["d_st2"] - 1.5 * t["m_st2"]
    gt = lam[3] - 0.5 * t["d_st1"] - 0.5 * t["m_st1"] + 0.5 * t["d_st2"] + 0.5 * t["m_st2"]
    return gd, gm, gs, gt


def pa_lambda(U: float):
    """Fully irreducible vertex of the parquet approximation: (U, -U, 2U, 0)."""
    return (U, -U, 2.0 * U, 0.0)


def lambda_at(grid: Grid, lam, r, m, n, n2):
    """Lambda_r(q; k, k') at transfer frequency m and fermionic frequencies n, n'
    (results section, full parquet / parquet DGA: the fully irreducible vertex
    is local, so the momenta do not enter). lam is either the four scalars of
    the parquet approximation or an array [4][Nv-1][Nv][Nv] on the box, index
    [r][m + Nv/2 - 1][n + Nv/2][n' + Nv/2]."""
    if np.ndim(lam) == 1:
        return lam[r]
    arr = np.asarray(lam)
    return arr[r][np.asarray(m) + grid.Nv // 2 - 1, np.asarray(n) + grid.Nv // 2, np.asarray(n2) + grid.Nv // 2]


def crossing_lambda(grid: Grid, U: float, lam_d, lam_m):
    """A local Lambda on the box that obeys the crossing relations between the
    particle-hole and particle-particle channels (crossing-symmetry subsection,
    which states that Lambda obeys the same relations as F), built from given
    d and m parts [Nv-1][Nv][Nv]: at (m; n, n') with partner transfer
    m' = m - n - n' - 1 in the box,
        Lambda_s(m) = 1/2 Lambda_d(m') - 3/2 Lambda_m(m'),
        Lambda_t(m) = 1/2 Lambda_d(m') + 1/2 Lambda_m(m'),
    which makes Lambda_d = 1/2 Lambda_s + 3/2 Lambda_t and
    Lambda_m = -1/2 Lambda_s + 1/2 Lambda_t hold at the inverse partner
    n + n' + m + 1; s and t keep their parquet-approximation values (2U, 0)
    where the partner lies outside the box."""
    nw, nv = grid.Nv - 1, grid.Nv
    out = np.empty((4, nw, nv, nv), dtype=np.complex128)
    out[0], out[1] = lam_d, lam_m
    out[2], out[3] = 2.0 * U, 0.0
    for jm in range(nw):
        m = jm - (nv // 2 - 1)
        for i1 in range(nv):
            for i2 in range(nv):
                n, n2 = i1 - nv // 2, i2 - nv // 2
                mp = m - n - n2 - 1
                if grid.in_bbox(mp):
                    jp = mp + nv // 2 - 1
                    out[2, jm, i1, i2] = 0.5 * lam_d[jp, i1, i2] - 1.5 * lam_m[jp, i1, i2]
                    out[3, jm, i1, i2] = 0.5 * lam_d[jp, i1, i2] + 0.5 * lam_m[jp, i1, i2]
    return out


def remap_points(grid: Grid, phi, K1, K2, lam, qi, ki, kpi):
    """Gamma_r (r = d, m, s, t) at the given box points (arrays of compound
    indices), Eqs. PA_Gamma_dm / PA_Gamma_st with the kernel fill."""
    qi, ki, kpi = np.asarray(qi), np.asarray(ki), np.asarray(kpi)
    jm, Q = np.divmod(qi, grid.Nk)
    m = jm - (grid.Nv // 2 - 1)
    i1, K = np.divmod(ki, grid.Nk)
    n = i1 - grid.Nv // 2
    i2, Kp = np.divmod(kpi, grid.Nk)
    n2 = i2 - grid.Nv // 2

    def P(r, a_n, a_K, b_n, b_K, p_m, p_Q):
        return accessor(grid, phi, K1, K2, r, a_n, a_K, b_n, b_K, p_m, p_Q)

    t = _remap_terms(grid, P, n, K, n2, Kp, m, Q)
    return np.stack(_combine_gamma(t, [lambda_at(grid, lam, r, m, n, n2) for r in range(4)]))


def remap(grid: Grid, phi, K1, K2, lam, chunk: int = 1 << 22):
    """Gamma_r on the whole box, [4][Nq][n][n]."""
    out = np.empty_like(phi)
    total = grid.Nq * grid.n * grid.n
    flat = out.reshape(4, -1)
    for s in range(0, total, chunk):
        idx = np.arange(s, min(total, s + chunk))
        qi, rest = np.divmod(idx, grid.n * grid.n)
        ki, kpi = np.divmod(rest, grid.n)
        flat[:, s:s + len(idx)] = remap_points(grid, phi, K1, K2, lam, qi, ki, kpi)
    return out


def full_vertex(gamma, phi):
    """F_r = Gamma_r + Phi_r (Eq. PA_F_G)."""
    return gamma + phi


# ----------------------------------------------------------------------------
# Bethe-Salpeter equations
# ----------------------------------------------------------------------------
def bse(grid: Grid, gamma, xph, xpp):
    """Phi_r^new = F_r - Gamma_r with F_r = [1 - s_r Gamma_r X_r]^{-1} Gamma_r for
    every transfer q (Eq. PA_F_Phi solved for F; the internal sum runs over the
    box, reading)."""
    out = np.empty_like(gamma)
    eye = np.eye(grid.n)
    for r in range(4):
        X = xph if r in (CH_D, CH_M) else xpp
        s = BSE_SIGN[r]
        for qi in range(grid.Nq):
            g = gamma[r, qi]
            A = eye - s * g * X[qi][None, :]
            F = np.linalg.solve(A, g)
            out[r, qi] = F - g
    return out


def bse_block(gamma_block, x_row, sign):
    """One block of the Bethe-Salpeter solve (used by the sampled large-size tests)."""
    n = gamma_block.shape[0]
    A = np.eye(n) - sign * gamma_block * x_row[None, :]
    F = np.linalg.solve(A, gamma_block)
    return F - gamma_block


# ----------------------------------------------------------------------------
# self-energy: regulated Schwinger-Dyson equation
# ----------------------------------------------------------------------------
def _g_ext(grid, G, n, K):
    return G[grid.gidx(n), K]


def _sde_weights(grid, G, n, K, n2, K2, m, Q):
    """G(k+q) G(k'+q) G(k') and G(q-k') G(q-k) G(k') of Eq. PA_Sigma."""
    g_kq = _g_ext(grid, G, n + m, grid.kadd(K, Q))
    g_kpq = _g_ext(grid, G, n2 + m, grid.kadd(K2, Q))
    g_kp = _g_ext(grid, G, n2, K2)
    g_qmkp = _g_ext(grid, G, m - n2 - 1, grid.ksub(Q, K2))
    g_qmk = _g_ext(grid, G, m - n - 1, grid.ksub(Q, K))
    return g_kq * g_kpq * g_kp, g_qmkp * g_qmk * g_kp


def _ext_pairs(grid):
    """All (k', q) with k' in the extended fermionic box and q in the extended bosonic box."""
    nf = grid.fext()
    mb = grid.bext()
    Nk = grid.Nk
    n2 = np.repeat(nf, Nk)
    K2 = np.tile(np.arange(Nk), len(nf))
    m = np.repeat(mb, Nk)
    Q = np.tile(np.arange(Nk), len(mb))
    return (n2[:, None], K2[:, None], m[None, :], Q[None, :])


def _box_pairs(grid):
    nf = grid.fbox()
    mb = grid.bbox()
    Nk = grid.Nk
    n2 = np.repeat(nf, Nk)
    K2 = np.tile(np.arange(Nk), len(nf))
    m = np.repeat(mb, Nk)
    Q = np.tile(np.arange(Nk), len(mb))
    return (n2[:, None], K2[:, None], m[None, :], Q[None, :])


def semicircle_poles(D: float, M: int = 200):
    """Pole representation of the semicircle: Gauss-Chebyshev (second kind)
    nodes e_j = D cos(j pi/(M+1)) with weights c_j = 2 sin^2(j pi/(M+1))/(M+1),
    so that G0(i nu) = sum_j c_j / (i nu - e_j) to machine precision for
    |nu| >= pi T with beta D <= 20 (convergence rate fixed by the distance
    nu/D of the pole of 1/(i nu - D x) from the real axis). M = 200 here; the
    pin tests show that the result no longer changes with M."""
    j = np.arange(1, M + 1)
    th = j * math.pi / (M + 1)
    return D * np.cos(th), 2.0 * np.sin(th) ** 2 / (M + 1)


def tau_grid(p, grid: Grid, mu: float):
    """Quadrature nodes and weights on [0, beta] for the imaginary-time route
    of Sigma~_1: composite Gauss-Legendre on the two halves [0, beta/2] and
    [beta/2, beta], each with 6 f Nv + 48 + 3 ceil(beta E) nodes, where
    E = max_K |eps_K - mu~| on the lattice and E = D locally: enough for the
    highest frequency of the integrand (about 4 nu_max) and its steepest
    exponential exp(-E tau). The pin tests check that doubling the nodes
    changes nothing."""
    if grid.Nk == 1:
        emax = p.D
    else:
        emax = float(np.max(np.abs(dispersion(grid, p.t, p.tp) - mu)))
    nh = 6 * grid.f * grid.Nv + 48 + 3 * int(math.ceil(p.beta * emax))
    x, w = np.polynomial.legendre.leggauss(nh)
    h = 0.5 * p.beta
    tau = np.concatenate([0.5 * h * (x + 1.0), h + 0.5 * h * (x + 1.0)])
    wt = np.concatenate([0.5 * h * w, 0.5 * h * w])
    return tau, wt


def _pole_tau(e, tau, beta):
    """Imaginary-time transform of 1/(i nu - e) on 0 < tau < beta,
    -exp(-e tau)/(1 + exp(-beta e)), written without overflow."""
    e = np.asarray(e, dtype=float)
    pos = e >= 0
    a = np.where(pos, -np.exp(-np.outer(tau, np.where(pos, e, 0.0))) / (1.0 + np.exp(-beta * np.where(pos, e, 0.0))), 0.0)
    b = np.where(~pos, -np.exp(np.outer(beta - tau, np.where(pos, 0.0, e))) / (np.exp(beta * np.where(pos, 0.0, e)) + 1.0), 0.0)
    return a + b


def g_tau(p, grid: Grid, G: np.ndarray, mu: float, tau: np.ndarray) -> np.ndarray:
    """G(K, tau) [Ntau][Nk] with every Matsubara frequency included: G equals the
    non-interacting pole part beyond the extended box (Sigma = 0 there), so
    G = G_pole + dG with dG supported on the extended box; the pole part is
    transformed analytically (anti-periodic), dG by its finite sum."""
    T = 1.0 / p.beta
    n_ext = grid.fext()
    nu = grid.nu(n_ext, p.beta)
    g_ext = G[grid.gidx(n_ext)]                                   # [Nve][Nk]
    if grid.Nk == 1:
        e, c = semicircle_poles(p.D)
        gpole_iw = (c[None, :] / (1j * nu[:, None] - e[None, :])).sum(axis=1)[:, None]
        gpole_tau = (_pole_tau(e, tau, p.beta) * c[None, :]).sum(axis=1)[:, None]
    else:
        xi = dispersion(grid, p.t, p.tp) - mu
        gpole_iw = 1.0 / (1j * nu[:, None] - xi[None, :])
        gpole_tau = _pole_tau(xi, tau, p.beta)
    dG = g_ext - gpole_iw
    return gpole_tau + T * np.exp(-1j * np.outer(tau, nu)) @ dG


def sigma_tilde1(p, grid: Grid, G, mu: float = 0.0, k_list=None):
    """Sigma~_1: the second-order diagram -U^2 G(r)^2 G(-r) with r = (R, tau),
    i.e. -(U^2 T^2 / 2N^2) sum_{k',q} [G(k+q)G(k'+q)G(k') + G(q-k')G(q-k)G(k')]
    over ALL Matsubara frequencies (high-frequency regulation subsection; the
    1/N of the printed sum is read as 1/N^2). The Fourier route of the paper is
    taken with exact anti-periodic transforms (g_tau) and Gauss-Legendre
    quadrature of the tau integral, which is analytic on [0, beta].
    Returns [f*Nv][Nk] (or the listed (n, K) points)."""
    tau, wt = tau_grid(p, grid, mu)
    gkt = g_tau(p, grid, G, mu, tau)                              # [Nt][Nk]
    R = np.arange(grid.Nk)
    rx, ry = np.divmod(R, grid.Ly)
    phase = np.exp(2j * math.pi * (np.outer(rx, grid.kx) / grid.Lx + np.outer(ry, grid.ky) / grid.Ly))  # [R][K]
    grt = gkt @ phase.T / grid.Nk                                 # G(R, tau)
    minus_r = grid.kneg(R)
    s_rt = p.U**2 * grt**2 * grt[::-1][:, minus_r]                # U^2 G(R,t)^2 G(-R, beta-t)
    n_ext = grid.fext()
    nu = grid.nu(n_ext, p.beta)
    s_rn = (np.exp(1j * np.outer(nu, tau)) * wt[None, :]) @ s_rt  # [Nve][R]
    s_kn = s_rn @ phase.conj()                                    # [Nve][K]
    if k_list is None:
        return s_kn
    return np.array([s_kn[grid.eidx(n), K] for (n, K) in k_list])


def _ext_points(grid):
    return [(int(n), int(K)) for n in grid.fext() for K in range(grid.Nk)]


def _kernel_vertex_combos(grid, K1, K2, lam, n, K, n2, K2m, m, Q):
    """F~_d - F~_m and F~_s + F~_t at (q, k, k') built from kernel values only
    (Eq. auxiliary_function generalised to every channel and to the kernel level
    in use, reading), i.e. the right-hand side of Eq. PA_F with each Phi replaced
    by its kernel approximation, the direct term included."""
    def P(r, a_n, a_K, b_n, b_K, p_m, p_Q):
        return kernel_value(grid, K1, K2, r, a_n, a_K, b_n, b_K, p_m, p_Q)

    t = _remap_terms(grid, P, n, K, n2, K2m, m, Q)
    gd, gm, gs, gt = _combine_gamma(t, lam)
    fd = gd + P(CH_D, n, K, n2, K2m, m, Q)
    fm = gm + P(CH_M, n, K, n2, K2m, m, Q)
    fs = gs + P(CH_S, n, K, n2, K2m, m, Q)
    ft = gt + P(CH_T, n, K, n2, K2m, m, Q)
    return fd - fm, fs + ft


def sigma_tilde2(p, grid: Grid, G, K1, K2, k_list=None):
    """Sigma~_2(k): the Schwinger-Dyson sum of (F~ - Lambda) over the extended box
    (k' in f*Nv fermionic, q in f*Nv-1 bosonic frequencies), high-frequency
    regulation subsection. Pinned by the third-order closed form at kernel
    level 1."""
    T = 1.0 / p.beta
    N = grid.Nk
    lam = pa_lambda(p.U)
    n2, K2m, m, Q = _ext_pairs(grid)
    pts = _ext_points(grid) if k_list is None else k_list
    out = np.empty(len(pts), dtype=np.complex128)
    for i, (n, K) in enumerate(pts):
        wph, wpp = _sde_weights(grid, G, n, K, n2, K2m, m, Q)
        dm, st = _kernel_vertex_combos(grid, K1, K2, lam, n, K, n2, K2m, m, Q)
        dm = dm - (lam[0] - lam[1])
        st = st - (lam[2] + lam[3])
        out[i] = -p.U * T**2 / (4 * N**2) * np.sum(wph * dm + wpp * st)
    return out if k_list is not None else out.reshape(grid.Nve, grid.Nk)


def sigma_box(p, grid: Grid, G, F, K1, K2, k_list=None):
    """Box part of the regulated Schwinger-Dyson equation:
    -(U T^2 / 4N^2) sum_{k',q in box} [G(k+q)G(k'+q)G(k') (dF_d - dF_m)
                                       + G(q-k')G(q-k)G(k') (dF_s + dF_t)],
    dF = F - F~ (Eq. PA_Sigma with the auxiliary vertex subtracted).
    Returns [Nv][Nk] for k in the box (or the listed (n, K) points).
    Pinned by the third-order closed form at kernel level 0 and by its vanishing
    when the kernel functions reproduce Phi exactly."""
    T = 1.0 / p.beta
    N = grid.Nk
    lam = pa_lambda(p.U)
    n2, K2m, m, Q = _box_pairs(grid)
    pts = [(int(n), int(K)) for n in grid.fbox() for K in range(grid.Nk)] if k_list is None else k_list
    out = np.empty(len(pts), dtype=np.complex128)
    # q-major / k'-minor index of the box pairs matches F[r][q][k][k']
    qi = grid.qidx(m, Q)            # [1, Nq]
    kpi = grid.kidx(n2, K2m)        # [n, 1]
    for i, (n, K) in enumerate(pts):
        ki = grid.kidx(n, K)
        wph, wpp = _sde_weights(grid, G, n, K, n2, K2m, m, Q)
        ftd_m, fts_t = _kernel_vertex_combos(grid, K1, K2, lam, n, K, n2, K2m, m, Q)
        fd_m = F[CH_D][qi, ki, kpi] - F[CH_M][qi, ki, kpi]
        fs_t = F[CH_S][qi, ki, kpi] + F[CH_T][qi, ki, kpi]
        out[i] = -p.U * T**2 / (4 * N**2) * np.sum(wph * (fd_m - ftd_m) + wpp * (fs_t - fts_t))
    return out if k_list is not None else out.reshape(grid.Nv, grid.Nk)


def second_order_box(p, grid: Grid, G):
    """The second-order diagram with both internal sums truncated to the box,
    -(U^2 T^2 / 2N^2) sum_{k' in box, q in box} [G(k+q)G(k'+q)G(k') + G(q-k')G(q-k)G(k')]
    (Eq. PA_Sigma at F = Lambda = (U, -U, 2U, 0) without regulation), for k in
    the box, [Nv][Nk]."""
    T = 1.0 / p.beta
    N = grid.Nk
    n2, K2m, m, Q = _box_pairs(grid)
    out = np.empty((grid.Nv, grid.Nk), dtype=np.complex128)
    for i, n in enumerate(grid.fbox()):
        for K in range(grid.Nk):
            wph, wpp = _sde_weights(grid, G, n, K, n2, K2m, m, Q)
            out[i, K] = -p.U**2 * T**2 / (2 * N**2) * np.sum(wph + wpp)
    return out


def sigma_plain(p, grid: Grid, G, F):
    """Eq. PA_Sigma evaluated plainly on the box, without the high-frequency
    regulation (the ablation the regulation subsection argues against):
    -(U T^2 / 4N^2) sum_{k', q in box} [G(k+q)G(k'+q)G(k') (F_d - F_m)
                                       + G(q-k')G(q-k)G(k') (F_s + F_t)]
    for k in the box, with the full vertex F = Gamma + Phi of the box. Nothing is
    known of Sigma outside the box, so the regulation box must be the box
    itself (f = 1). Returns [Nv][Nk]."""
    assert grid.f == 1, "without regulation Sigma lives on the box (f_ext = 1)"
    T = 1.0 / p.beta
    N = grid.Nk
    out = np.empty((grid.Nv, grid.Nk), dtype=np.complex128)
    for i, n in enumerate(grid.fbox()):
        for K in range(grid.Nk):
            ki = grid.kidx(n, K)
            acc = 0.0
            for qi in range(grid.Nq):
                jm, Qm = divmod(qi, grid.Nk)
                m = jm - (grid.Nv // 2 - 1)
                for kpi in range(grid.n):
                    i2, K2m = divmod(kpi, grid.Nk)
                    n2 = i2 - grid.Nv // 2
                    g_kq = G[grid.gidx(n + m), grid.kadd(K, Qm)]
                    g_kpq = G[grid.gidx(n2 + m), grid.kadd(K2m, Qm)]
                    g_kp = G[grid.gidx(n2), K2m]
                    g_qmkp = G[grid.gidx(m - n2 - 1), grid.ksub(Qm, K2m)]
                    g_qmk = G[grid.gidx(m - n - 1), grid.ksub(Qm, K)]
                    fdm = F[CH_D][qi, ki, kpi] - F[CH_M][qi, ki, kpi]
                    fst = F[CH_S][qi, ki, kpi] + F[CH_T][qi, ki, kpi]
                    acc += g_kq * g_kpq * g_kp * fdm + g_qmkp * g_qmk * g_kp * fst
            out[i, K] = -p.U * T**2 / (4 * N**2) * acc
    return out


def regulation_of(p) -> int:
    return int(getattr(p, "regulation", 1))


def sigma_sde(p, grid: Grid, G, F, K1, K2, mu: float = 0.0):
    """Sigma_new(k) = Sigma~_1 + Sigma~_2 + [k in box] Sigma_box on the extended
    box (high-frequency regulation); without regulation the plain box sum."""
    if regulation_of(p) == 0:
        return sigma_plain(p, grid, G, F)
    s = sigma_tilde1(p, grid, G, mu) + sigma_tilde2(p, grid, G, K1, K2)
    lo = grid.eidx(-grid.Nv // 2)
    s[lo:lo + grid.Nv] += sigma_box(p, grid, G, F, K1, K2)
    return s


# ----------------------------------------------------------------------------
# the self-consistent loop
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    sigma: np.ndarray           # [f*Nv][Nk]
    phi: np.ndarray             # [4][Nq][n][n]
    mu: float = 0.0
    iteration: int = 0
    last_dsigma: float = float("inf")


def init_state(p, grid: Optional[Grid] = None) -> State:
    """Bare-vertex start: Phi_r = 0 and Sigma_0 = Sigma~_1[G_0] (reading), where
    G_0 is the Dyson G with Sigma = 0 (mu~ from the filling); without the
    regulation the box-truncated second-order diagram of G_0."""
    grid = grid or Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    zero = np.zeros((grid.Nve, grid.Nk), dtype=np.complex128)
    mu0 = find_mu(p, grid, zero)
    G0 = dyson(p, grid, zero, mu0)
    sigma0 = second_order_box(p, grid, G0) if regulation_of(p) == 0 else sigma_tilde1(p, grid, G0, mu0)
    phi = np.zeros((4, grid.Nq, grid.n, grid.n), dtype=np.complex128)
    return State(sigma=sigma0, phi=phi, mu=mu0)


def iterate(p, st: State, grid: Optional[Grid] = None, return_parts: bool = False, lam=None):
    """One parquet iteration in the order Dyson -> bubbles -> kernels -> remap ->
    Schwinger-Dyson -> Bethe-Salpeter -> mixing (reading: the SDE and the BSE use
    the same G and Phi, so they are independent within an iteration). lam: the
    fully irreducible vertex, the parquet-approximation scalars by default or a
    local array on the box (lambda_at); the auxiliary vertex F~ of the
    regulation keeps the parquet-approximation values, so a box Lambda enters
    Sigma through F - F~ in the box part."""
    grid = grid or Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    mu = find_mu(p, grid, st.sigma)
    G = dyson(p, grid, st.sigma, mu)
    xph, xpp = bubbles(p, grid, G)
    K1, K2 = kernel_functions(grid, st.phi, p.kernel_level, p.edge_rule)
    lam = pa_lambda(p.U) if lam is None else lam
    gamma = remap(grid, st.phi, K1, K2, lam)
    F = full_vertex(gamma, st.phi)
    sigma_new = sigma_sde(p, grid, G, F, K1, K2, mu)
    phi_new = bse(grid, gamma, xph, xpp)
    dsig = float(np.max(np.abs(sigma_new - st.sigma)))
    a = p.alpha
    new = State(sigma=a * sigma_new + (1 - a) * st.sigma,
                phi=a * phi_new + (1 - a) * st.phi,
                mu=mu, iteration=st.iteration + 1, last_dsigma=dsig)
    if return_parts:
        parts = dict(G=G, xph=xph, xpp=xpp, K1=K1, K2=K2, gamma=gamma, F=F,
                     sigma_new=sigma_new, phi_new=phi_new, mu=mu)
        return new, parts
    return new


def solve(p, max_iter: int = 200, tol: Optional[float] = None, callback=None, lam=None) -> State:
    grid = Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    tol = p.tol if tol is None else tol
    st = init_state(p, grid)
    for _ in range(max_iter):
        st = iterate(p, st, grid, lam=lam)
        if callback is not None:
            callback(st)
        if st.last_dsigma < tol:
            break
    return st
