"""Point-wise views of a low-rank reducible vertex for the FP64 oracle at sizes
whose full [4][Nq][n][n] array does not fit in host memory.

Phi_r[q][k][k'] = sum_j u[r,q,k,j] v[r,q,k',j] (factors from
``workloads.lowrank_phi_factors``). The views support exactly the indexing the
oracle performs:

* ``phi[r][qi, ki, kpi]`` with broadcastable index arrays (accessor, box SDE);
* ``phi[r, qi][:, cols]`` with a column slice (kernel-function edges).

``FullVertex`` gives F_r = Gamma_r + Phi_r at arbitrary points, Gamma_r from the
oracle's ``remap_points``; the four channels of one point set are computed once.
"""
from __future__ import annotations

import numpy as np

from oracle import parquet as P


class _Block:
    def __init__(self, u, v):
        self.u, self.v = u, v

    def __getitem__(self, key):
        rows, cols = key
        return self.u[rows] @ self.v[cols].T


class _Channel:
    def __init__(self, u, v):
        self.u, self.v = u, v

    def __getitem__(self, key):
        if isinstance(key, tuple) and len(key) == 3:
            q, a, b = np.broadcast_arrays(*(np.asarray(k, dtype=np.int64) for k in key))
            return np.einsum("...j,...j->...", self.u[q, a], self.v[q, b])
        raise TypeError("unsupported index")


class LowRankVertex:
    def __init__(self, u, v):
        self.u, self.v = u, v
        self.shape = (u.shape[0], u.shape[1], u.shape[2], v.shape[2])

    def __getitem__(self, key):
        if isinstance(key, tuple) and len(key) == 2:
            r, q = int(key[0]), int(key[1])
            return _Block(self.u[r, q], self.v[r, q])
        return _Channel(self.u[int(key)], self.v[int(key)])

    def block(self, r, q):
        return self.u[r, q] @ self.v[r, q].T


class FullVertex:
    """F_r = Gamma_r + Phi_r at arbitrary box points."""

    def __init__(self, grid, phi: LowRankVertex, K1, K2, lam):
        self.grid, self.phi, self.K1, self.K2, self.lam = grid, phi, K1, K2, lam
        self._key = None
        self._val = None

    def _all(self, q, a, b):
        key = (q.shape, a.shape, b.shape, q.tobytes(), a.tobytes(), b.tobytes())
        if key != self._key:
            gam = P.remap_points(self.grid, self.phi, self.K1, self.K2, self.lam, q, a, b)
            ph = np.stack([self.phi[r][q, a, b] for r in range(4)])
            self._key, self._val = key, gam + ph
        return self._val

    def __getitem__(self, r):
        outer = self

        class _F:
            def __getitem__(self, key):
                q, a, b = np.broadcast_arrays(*(np.asarray(k, dtype=np.int64) for k in key))
                return outer._all(q, a, b)[int(r)]

        return _F()
