"""Learned warm start: a small multilayer perceptron maps the model parameters
(U, beta) of the momentum-independent problem to its converged kernel
functions K1_r(q), K2_r(k; q); the reducible vertex is then rebuilt from them
(phi_from_kernels, second-level kernel form) and the iteration starts there
instead of at the bare vertex. Training, inference and the rebuild run in the
library's kernels (mlp_forward / mlp_backward / mlp_adam); this module only
moves tensors and keeps the loop. The bare start remains the fallback when
the warm-started iteration fails."""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import native as N
from .ops import Solver, Stage, _ptr, _stream


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


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
    """(U, beta) -> K1 [4][Nq], K2 [4][Nq][n] and the self-energy [Nve][Nk]
    for one box, with input scaling and per-output standardisation fitted on
    the training set."""

    def __init__(self, base, hidden=(512, 512, 512), device: str = "cuda:0", seed: int = 0):
        self.base = base
        self.stage = Stage(base, "fp64")
        d = self.stage.d
        self.nk1 = 4 * d.Nq
        self.nk2 = 4 * d.Nq * d.n
        self.nsig = d.Nve * d.Nk
        self.nout = 2 * (self.nk1 + self.nk2 + self.nsig)
        self.mlp = MLP([2, *hidden, self.nout], device, seed)
        self.device = torch.device(device)

    def _x(self, params):
        return torch.tensor([[p.U, p.beta] for p in params], dtype=torch.float32, device=self.device)

    def _scale_x(self, x):
        return (x - self.x_mean) / self.x_std

    @staticmethod
    def _flat(k1, k2, sig):
        return torch.cat([torch.view_as_real(k1).reshape(-1), torch.view_as_real(k2).reshape(-1),
                          torch.view_as_real(sig).reshape(-1)])

    def fit(self, params, k1s, k2s, sigs, steps=3000, batch=64, lr=1e-3, progress=None):
        x = self._x(params)
        y = torch.stack([self._flat(a, b, c) for a, b, c in zip(k1s, k2s, sigs)]).to(torch.float64)
        self.x_mean, self.x_std = x.mean(0), x.std(0).clamp_min(1e-6)
        self.y_mean, self.y_std = y.mean(0), y.std(0).clamp_min(1e-12)
        X = self._scale_x(x)
        Y = ((y - self.y_mean) / self.y_std).to(torch.float32)
        return self.mlp.train(X, Y, steps, batch, lr, progress=progress)

    def predict(self, p):
        X = self._scale_x(self._x([p]))
        _, out = self.mlp.forward(X)
        y = out[0].to(torch.float64) * self.y_std + self.y_mean
        d = self.stage.d
        a, b = 2 * self.nk1, 2 * (self.nk1 + self.nk2)
        k1 = torch.view_as_complex(y[:a].reshape(-1, 2).contiguous()).reshape(4, d.Nq)
        k2 = torch.view_as_complex(y[a:b].reshape(-1, 2).contiguous()).reshape(4, d.Nq, d.n)
        sig = torch.view_as_complex(y[b:].reshape(-1, 2).contiguous()).reshape(d.Nve, d.Nk)
        return k1.contiguous(), k2.contiguous(), sig.contiguous()


def phi_from_kernels(p, precision: str, k1: torch.Tensor, k2: torch.Tensor, phi_out: torch.Tensor):
    st = Stage(p, precision)
    N.check(N.load().phi_from_kernels(st._pp(), _ptr(k1, torch.complex128, st.k1_shape, "k1"),
                                      _ptr(k2, torch.complex128, st.k2_shape, "k2"),
                                      _ptr(phi_out, st.vdtype, st.vshape, "phi_out"), _stream()))


def converged_kernels(p, precision: str = "fp64", tol: float = 1e-8, max_iter: int = 400):
    """Solve from the bare start; returns (converged, iterations, K1, K2, Sigma)
    of the last iteration (the kernel functions of the converged vertex)."""
    s = Solver(p, precision)
    try:
        done, conv, _ = s.iterate(max_iter, tol)
    except N.ParquetError:
        s.close()
        return False, max_iter, None, None, None
    k1, k2, sig = s.get("k1"), s.get("k2"), s.get("sigma")
    s.close()
    return conv, done, k1, k2, sig


def solve_timed(p, precision, tol, max_iter, warm=None):
    """Iterations and seconds to max|dSigma| < tol from the bare start, or from
    the vertex rebuilt from predicted kernels (warm = (k1, k2) or (k1, k2,
    sigma), the latter also starting the self-energy from the prediction); a
    warm start that does not converge is retried from the bare start (counted
    in both)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = Solver(p, precision)
    if warm is not None:
        phi = torch.empty(s.stage.vshape, dtype=s.stage.vdtype, device=s.device)
        phi_from_kernels(p, precision, warm[0], warm[1], phi)
        s.set("phi", phi)
        del phi
        if len(warm) > 2:
            s.set("sigma", warm[2])
    try:
        done, conv, _ = s.iterate(max_iter, tol)
    except N.ParquetError:
        done, conv = max_iter, False
    s.close()
    fallback = False
    if warm is not None and not conv:
        fallback = True
        b = solve_timed(p, precision, tol, max_iter)
        done += b["iterations"]
        conv = b["converged"]
    torch.cuda.synchronize()
    return dict(iterations=done, converged=bool(conv), sec=time.perf_counter() - t0, fallback=fallback)
