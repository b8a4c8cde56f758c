"""Learned warm start: a small multilayer perceptron maps model parameters
(for instance U, beta, the filling n and t') to the converged kernel functions
K1_r(q), K2_r(k; q) and the self-energy of one box; the reducible vertex is
then rebuilt from the kernel values (phi_from_kernels, second-level kernel
form) and the iteration starts there instead of at the bare vertex.

The output layer is factorised: per field (K1, K2, Sigma) the library builds
an orthonormal basis of the centred training solutions (mlp_basis), the
network predicts the coordinates in those bases, and mlp_expand rebuilds the
fields. The head is then as wide as the training set, not as the box (K2 alone
has 3.9M complex values on the 8x8, Nv = 16 box). Training, inference, the
basis and the rebuild run in the library's kernels; this module moves tensors
and keeps the loop. The bare start remains the fallback when the
warm-started iteration fails."""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import native as N
from .ops import Solver, Stage, _ptr, _stream

FIELDS = ("k1", "k2", "sigma")


def _p(t, offset_elems: int = 0):
    return ctypes.c_void_p(t.data_ptr() + offset_elems * t.element_size())


class MLP:
    """Parameters on the device: FP32 master copy, bf16 copy, Adam moments."""

    def __init__(self, widths, device: str = "cuda:0", seed: int = 0):
        self.widths = [int(w) for w in widths]
        self.nl = len(widths) - 1
        self.w_arr = (ctypes.c_int32 * len(widths))(*self.widths)
        cnt = ctypes.c_size_t()
        N.check(N.load().mlp_param_count(self.w_arr, self.nl, ctypes.byref(cnt)))
        self.count = int(cnt.value)
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        parts = []
        for l in range(self.nl):
            fan_in, fan_out = self.widths[l], self.widths[l + 1]
            lim = np.sqrt(6.0 / (fan_in + fan_out))            # Glorot uniform
            parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
            parts.append(np.zeros(fan_out))
        self.p = torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(self.device)
        self.pb = torch.empty(self.count, dtype=torch.bfloat16, device=self.device)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.empty_like(self.p)
        self.loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self.step_count = 0
        N.check(N.load().mlp_to_bf16(_p(self.p), _p(self.pb), self.count, _stream()))

    def set_params(self, p: torch.Tensor):
        self.p.copy_(p.to(self.p.dtype))
        N.check(N.load().mlp_to_bf16(_p(self.p), _p(self.pb), self.count, _stream()))

    def forward(self, x: torch.Tensor):
        """x [B][w0] float32 -> (all activations, output view [B][wL])."""
        B = x.shape[0]
        acts = torch.empty(B * sum(self.widths[1:]), dtype=torch.float32, device=self.device)
        N.check(N.load().mlp_forward(self.w_arr, self.nl, _p(self.pb), _p(self.p), _p(x.contiguous()),
                                     _p(acts), B, _stream()))
        return acts, acts[-B * self.widths[-1]:].view(B, self.widths[-1])

    def backward(self, x, acts, target):
        B = x.shape[0]
        scratch = torch.empty(2 * B * max(self.widths), dtype=torch.float32, device=self.device)
        N.check(N.load().mlp_backward(self.w_arr, self.nl, _p(self.pb), _p(x), _p(acts), _p(target.contiguous()),
                                      _p(self.g), _p(self.loss), _p(scratch), B, _stream()))
        return self.loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step_count += 1
        N.check(N.load().mlp_adam(_p(self.p), _p(self.pb), _p(self.m), _p(self.v), _p(self.g), self.count,
                                  float(lr), float(beta1), float(beta2), float(eps), self.step_count, _stream()))

    def train(self, X: torch.Tensor, Y: torch.Tensor, steps: int, batch: int = 64, lr: float = 1e-3,
              seed: int = 0, lr_final: float = 1e-5, progress=None):
        """Minibatch Adam on (X, Y); cosine decay of the learning rate;
        progress(step, loss) is called every 500 steps if given."""
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        hist = []
        for it in range(steps):
            idx = torch.from_numpy(rng.choice(n, size=min(batch, n), replace=False)).to(self.device)
            xb, yb = X[idx].contiguous(), Y[idx].contiguous()
            acts, _ = self.forward(xb)
            self.backward(xb, acts, yb)
            a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * it / max(1, steps - 1)))
            self.adam(a)
            if it % 100 == 0 or it == steps - 1:
                hist.append((it, float(self.loss.item())))
                if progress is not None and it % 500 == 0:
                    progress(it, hist[-1][1])
        return hist


class KernelPredictor:
    """Model parameters -> K1 [4][Nq], K2 [4][Nq][n] and the self-energy
    [Nve][Nk] of one box (complex128).

    inputs: {name of a ModelParams field: (low, high)}, the sampling box of
    the parameters the network sees; each is mapped affinely to [-1, 1].
    Training solutions are added one at a time (add); fit builds the bases and
    trains the network on the coordinates."""

    def __init__(self, base, inputs, max_samples: int, hidden=(512, 512, 512), device: str = "cuda:0",
                 seed: int = 0):
        self.base = base
        self.inputs = dict(inputs)
        self.hidden = tuple(hidden)
        self.seed = seed
        self.device = torch.device(device)
        st = Stage(base, "fp64")
        self.shapes = {"k1": st.k1_shape, "k2": st.k2_shape, "sigma": st.sigma_shape}
        self.lens = {f: 2 * int(np.prod(self.shapes[f])) for f in FIELDS}
        self.cap = int(max_samples)
        self.Y = {f: torch.empty((self.cap, self.lens[f]), dtype=torch.float32, device=self.device) for f in FIELDS}
        self.params = []
        self.mlp = None

    def _x(self, params):
        rows = []
        for p in params:
            rows.append([2.0 * (getattr(p, k) - lo) / (hi - lo) - 1.0 for k, (lo, hi) in self.inputs.items()])
        return torch.tensor(rows, dtype=torch.float32, device=self.device)

    def add(self, p, k1, k2, sigma):
        """One converged solution (complex tensors on the device) as a training row."""
        i = len(self.params)
        if i >= self.cap:
            raise ValueError("training set is full")
        for f, v in zip(FIELDS, (k1, k2, sigma)):
            self.Y[f][i].copy_(torch.view_as_real(v.reshape(self.shapes[f]).to(torch.complex64)).reshape(-1))
        self.params.append(p)

    def fit(self, steps=3000, batch=64, lr=1e-3, progress=None):
        rows = len(self.params)
        if rows < 2:
            raise ValueError("need at least two training solutions")
        lib = N.load()
        wsb = ctypes.c_size_t()
        N.check(lib.mlp_basis_workspace(rows, ctypes.byref(wsb)))
        ws = torch.empty(int(wsb.value), dtype=torch.uint8, device=self.device)
        T = torch.empty((rows, 3 * rows), dtype=torch.float32, device=self.device)
        self.Q, self.mean, self.scale = {}, {}, {}
        for gi, f in enumerate(FIELDS):
            Y = self.Y[f][:rows].contiguous() if rows < self.cap else self.Y[f]
            self.mean[f] = torch.empty(self.lens[f], dtype=torch.float32, device=self.device)
            self.scale[f] = torch.empty(1, dtype=torch.float32, device=self.device)
            N.check(lib.mlp_basis(_p(Y), rows, self.lens[f], _p(self.mean[f]), _p(T, gi * rows), 3 * rows,
                                  _p(self.scale[f]), _p(ws), _stream()))
            self.Q[f] = Y
        self.Y = None                                     # the bases replace the raw rows
        self.rows = rows
        self.mlp = MLP([len(self.inputs), *self.hidden, 3 * rows], self.device, self.seed)
        X = self._x(self.params)
        return self.mlp.train(X, T, steps, min(batch, rows), lr, seed=self.seed, progress=progress)

    def predict(self, p):
        _, out = self.mlp.forward(self._x([p]))
        lib = N.load()
        res = []
        for gi, f in enumerate(FIELDS):
            y = torch.empty(self.lens[f], dtype=torch.float64, device=self.device)
            N.check(lib.mlp_expand(_p(self.Q[f]), self.rows, self.lens[f], _p(self.mean[f]),
                                   _p(out, gi * self.rows), _p(self.scale[f]), _p(y), _stream()))
            res.append(torch.view_as_complex(y.view(-1, 2)).reshape(self.shapes[f]))
        return tuple(res)


def phi_from_kernels(p, precision: str, k1: torch.Tensor, k2: torch.Tensor, phi_out: torch.Tensor):
    st = Stage(p, precision)
    N.check(N.load().phi_from_kernels(st._pp(), _ptr(k1, torch.complex128, st.k1_shape, "k1"),
                                      _ptr(k2, torch.complex128, st.k2_shape, "k2"),
                                      _ptr(phi_out, st.vdtype, st.vshape, "phi_out"), _stream()))


def converged_kernels(p, precision: str = "fp64", tol: float = 1e-8, max_iter: int = 400, solver=None):
    """Solve from the bare start; returns (converged, iterations, K1, K2, Sigma)
    of the last iteration (the kernel functions of the converged vertex).
    solver: a Solver of the same box and precision to reuse (re-initialised
    with p; its workspace is kept)."""
    s = solver if solver is not None else Solver(p, precision)
    if solver is not None:
        s.reinit(p)
    try:
        done, conv, _ = s.iterate(max_iter, tol)
    except N.ParquetError:
        s.close()
        return False, max_iter, None, None, None
    k1, k2, sig = s.get("k1"), s.get("k2"), s.get("sigma")
    s.close()
    return conv, done, k1, k2, sig


def solve_timed(p, precision, tol, max_iter, warm=None, keep=False):
    """Iterations and seconds to the convergence test of tol (see
    Solver.iterate) from the bare start, or from the vertex rebuilt from
    predicted kernels (warm = (k1, k2) or (k1, k2, sigma), the latter also
    starting the self-energy from the prediction); a warm start that does not
    converge is retried from the bare start (counted in both). keep: also
    return the final self-energy (key sigma) and kernel functions (key
    kernels: K1, K2, Sigma)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = Solver(p, precision)
    if warm is not None:
        s.warm_start(*warm)
    try:
        done, conv, _ = s.iterate(max_iter, tol)
    except N.ParquetError:
        done, conv = max_iter, False
    sigma = s.get("sigma") if keep and conv else None
    kernels = (s.get("k1"), s.get("k2"), sigma) if keep and conv else None
    s.close()
    fallback = False
    if warm is not None and not conv:
        fallback = True
        b = solve_timed(p, precision, tol, max_iter, keep=keep)
        done += b["iterations"]
        conv = b["converged"]
        sigma, kernels = b.get("sigma"), b.get("kernels")
    torch.cuda.synchronize()
    out = dict(iterations=done, converged=bool(conv), sec=time.perf_counter() - t0, fallback=fallback)
    if keep:
        out["sigma"] = sigma
        out["kernels"] = kernels
    return out
