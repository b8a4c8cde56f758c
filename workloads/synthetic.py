"""Parameter sets and seeded draws for the parquet hot path.

Workloads (all synthetic; the paper's DMFT / CT-INT inputs are not available):

* ``c1``  momentum-independent parquet approximation: Nk = 1, Weiss field from a
  semicircular density of states (half-bandwidth D = 2), U = 1, beta = 5,
  half filling, fermionic box Nv = 32 (31 bosonic), mixing 0.5, tol 1e-8.
* ``c2``  4x4 square lattice, t = 1, t' = 0, U = 2, beta = 4, half filling,
  Nv = 16 (BSE dimension 256, 240 transfer blocks).
* ``c3``  8x8 square lattice, t = 1, t' = -0.2, U = 2, beta = 5, filling 0.9,
  Nv = 16 (BSE dimension 1024, 960 transfer blocks), kernel level 2.
* ``tiny*`` small boxes used by the unit and parity tests.

Random draws use ``numpy.random.Generator(PCG64(seed))`` so that every consumer
(the oracle, the HIP path, the tests) sees bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
from typing import Dict

import numpy as np


@dataclasses.dataclass(frozen=True)
class ModelParams:
    """Physical and numerical parameters of one parquet instance."""

    Lx: int
    Ly: int
    Nv: int                 # fermionic box size (even); bosonic box has Nv - 1
    U: float
    beta: float
    t: float = 1.0
    tp: float = 0.0         # next-nearest-neighbour hopping t'
    filling: float = 1.0    # total density n (both spins)
    D: float = 2.0          # semicircle half-bandwidth (local mode, Nk = 1)
    f_ext: int = 2          # extension factor of the regulation box
    kernel_level: int = 2   # 0: truncation, 1: K1 only, 2: K1 + K2
    regulation: int = 1     # 1: high-frequency regulation of the SDE; 0: plain box sum (needs f_ext = 1)
    edge_rule: int = 0      # 0: far edge per channel and sign of m; 1: lowest edge always
    mu_mode: int = 0        # 0: mu_tilde fixed to mu_fixed; 1: bisection on the filling
    mu_fixed: float = 0.0
    alpha: float = 0.5      # linear mixing of Sigma and Phi
    tol: float = 1e-8

    @property
    def Nk(self) -> int:
        return self.Lx * self.Ly

    @property
    def local(self) -> bool:
        return self.Nk == 1

    def replace(self, **kw) -> "ModelParams":
        return dataclasses.replace(self, **kw)


CONFIGS: Dict[str, ModelParams] = {
    "c1": ModelParams(Lx=1, Ly=1, Nv=32, U=1.0, beta=5.0, D=2.0, filling=1.0,
                      mu_mode=0, tol=1e-8),
    "c2": ModelParams(Lx=4, Ly=4, Nv=16, U=2.0, beta=4.0, t=1.0, tp=0.0,
                      filling=1.0, mu_mode=0, tol=1e-6),
    "c3": ModelParams(Lx=8, Ly=8, Nv=16, U=2.0, beta=5.0, t=1.0, tp=-0.2,
                      filling=0.9, mu_mode=1, tol=1e-6),
    # small boxes for tests
    "tiny_local": ModelParams(Lx=1, Ly=1, Nv=8, U=1.0, beta=5.0, D=2.0),
    "tiny_2x2": ModelParams(Lx=2, Ly=2, Nv=4, U=1.5, beta=3.0, tp=-0.1,
                            filling=0.95, mu_mode=1),
    "tiny_2x2_hf": ModelParams(Lx=2, Ly=2, Nv=8, U=2.0, beta=4.0),
    "small_4x4": ModelParams(Lx=4, Ly=4, Nv=4, U=2.0, beta=3.0, tp=-0.2,
                             filling=0.9, mu_mode=1),
    "small_2x4": ModelParams(Lx=2, Ly=4, Nv=6, U=1.5, beta=4.0, tp=0.1,
                             filling=1.05, mu_mode=1),
}


def config(name: str, **overrides) -> ModelParams:
    p = CONFIGS[name]
    return p.replace(**overrides) if overrides else p


def parameter_draws(base: ModelParams, box: Dict[str, tuple], seeds) -> list:
    """One parameter set per seed: every field named in box drawn uniformly
    from its (low, high) range by Generator(PCG64(seed)), in the order of box;
    a drawn filling is reached by bisection on the chemical potential
    (mu_mode = 1)."""
    out = []
    for s in seeds:
        rng = np.random.Generator(np.random.PCG64(int(s)))
        kw = {k: float(rng.uniform(lo, hi)) for k, (lo, hi) in box.items()}
        if "filling" in kw:
            kw["mu_mode"] = 1
        out.append(base.replace(**kw))
    return out


def batch_draws(count: int = 64, seed: int = 4, nvs=(8, 16, 24, 32)) -> list:
    """Independent 4x4-lattice instances (t = 1, t' = 0) drawn in sequence by
    one Generator(PCG64(seed)): U uniform in [0.5, 3], beta uniform in [2, 8],
    filling uniform in [0.8, 1] (bisection on the chemical potential), box
    size Nv uniform over nvs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        U = float(rng.uniform(0.5, 3.0))
        beta = float(rng.uniform(2.0, 8.0))
        n = float(rng.uniform(0.8, 1.0))
        nv = int(nvs[int(rng.integers(len(nvs)))])
        out.append(ModelParams(Lx=4, Ly=4, Nv=nv, U=U, beta=beta, t=1.0, tp=0.0, filling=n, mu_mode=1))
    return out


def rand_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Complex normal draws with Re, Im ~ N(0, scale^2 / 2) each (E|z|^2 = scale^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = scale / np.sqrt(2.0)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re * s + 1j * (im * s)).astype(np.complex128)


def bse_microbench_gamma(n: int, blocks, base_seed: int = 1510) -> np.ndarray:
    """Seeded i.i.d. complex N(0, 1/n) blocks, block b drawn from PCG64(base_seed + b)."""
    out = np.empty((len(blocks), n, n), dtype=np.complex128)
    for i, b in enumerate(blocks):
        out[i] = rand_complex((n, n), base_seed + int(b), scale=1.0 / np.sqrt(n))
    return out


def lambda_box_parts(nv: int, seed: int, scale: float = 0.3, n_inner=None, symmetric: bool = True):
    """Two seeded complex arrays [Nv-1][Nv][Nv] (bosonic index, two fermionic
    indices of a box of Nv fermionic frequencies) for the density and magnetic
    parts of a local fully irreducible vertex, nonzero only where all three
    frequency indices lie within n_inner of the box centre (None: the whole
    box); symmetric: equal under exchange of the two fermionic indices."""
    rng = np.random.default_rng(seed)
    nw = nv - 1
    out = []
    for _ in range(2):
        a = (rng.standard_normal((nw, nv, nv)) + 1j * rng.standard_normal((nw, nv, nv))) * (scale / np.sqrt(2.0))
        if symmetric:
            a = 0.5 * (a + a.transpose(0, 2, 1))
        if n_inner is not None:
            m = np.arange(nw) - (nv // 2 - 1)
            f = np.arange(nv) - nv // 2
            keep = ((np.abs(m) <= n_inner)[:, None, None] & (np.abs(f + 0.5) <= n_inner + 0.5)[None, :, None]
                    & (np.abs(f + 0.5) <= n_inner + 0.5)[None, None, :])
            a = np.where(keep, a, 0.0)
        out.append(a.astype(np.complex128))
    return out[0], out[1]


def random_phi(nq: int, n: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """Four seeded random reducible-vertex arrays, layout [channel][q][k][k']."""
    return rand_complex((4, nq, n, n), seed, scale)


def random_sigma(nfreq: int, nk: int, seed: int, scale: float = 0.2) -> np.ndarray:
    """Seeded random self-energy on [frequency][momentum]."""
    return rand_complex((nfreq, nk), seed, scale)


def lowrank_phi_factors(nq: int, n: int, nk: int, nv: int, seed: int, rank: int = 4,
                        scale: float = 0.1):
    """Seeded factors of a large reducible-vertex input that is cheap to evaluate
    point by point: Phi_r[q][k][k'] = sum_j u[r,q,k,j] v[r,q,k',j].

    Used where the full [4][Nq][n][n] array does not fit in host memory (the
    8x8, Nv = 16 case is 4e9 elements). Each factor row carries an envelope
    1 / (1 + |nu index| / 4) over the fermionic frequency of its compound
    index (frequency-major, k = (n + Nv/2) Nk + K), so entries are largest at
    the box centre and smaller at its edge, as for a vertex that decays with
    frequency. E|Phi|^2 is about scale^2 at the centre."""
    fac = np.sqrt(scale / np.sqrt(rank))
    u = rand_complex((4, nq, n, rank), seed, fac)
    v = rand_complex((4, nq, n, rank), seed + 1, fac)
    freq = np.arange(n) // nk - nv // 2 + 0.5
    env = 1.0 / (1.0 + np.abs(freq) / 4.0)
    u *= env[None, None, :, None]
    v *= env[None, None, :, None]
    return u, v
