"""Torch-facing wrappers of the stage entry points and the solver context.

Each wrapper validates tensor device, dtype, shape and contiguity, then hands
raw device pointers and the current HIP stream to libparquet. No arithmetic
of the method happens here.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import native as N


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, dtype, shape: Sequence[int], name: str) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Stage:
    """Shapes and dtypes of one parameter set, plus the stateless stage calls."""

    def __init__(self, p, precision: str = "fp64", resolve_slots: int = 0, bse_tol: float = 0.0,
                 bse_tile: int = 0):
        N.load()
        self.model = p
        self.precision = precision
        self.pp = N.make_params(p, precision, resolve_slots, bse_tol, bse_tile)
        self.d = N.dims(self.pp)
        self.vdtype = torch.complex128 if precision == "fp64" else torch.complex64
        d = self.d
        self.vshape = (4, d.Nq, d.n, d.n)
        self.sigma_shape = (d.Nve, d.Nk)
        self.g_shape = (d.NG, d.Nk)
        self.x_shape = (d.Nq, d.n)
        self.k1_shape = (4, d.Nq)
        self.k2_shape = (4, d.Nq, d.n)
        self.lam_shape = (4, d.NW, d.Nv, d.Nv)

    def _pp(self):
        return ctypes.byref(self.pp)

    # ---- stages
    def dyson_update(self, sigma, g_out, mu_out, stream=None):
        lib = N.load()
        N.check(lib.dyson_update(self._pp(), _ptr(sigma, torch.complex128, self.sigma_shape, "sigma"),
                                 _ptr(g_out, torch.complex128, self.g_shape, "g_out"),
                                 _ptr(mu_out, torch.float64, (1,), "mu_out"), _stream(stream)))

    def bubble_build(self, g, xph, xpp, stream=None):
        N.check(N.load().bubble_build(self._pp(), _ptr(g, torch.complex128, self.g_shape, "g"),
                                      _ptr(xph, torch.complex128, self.x_shape, "xph"),
                                      _ptr(xpp, torch.complex128, self.x_shape, "xpp"), _stream(stream)))

    def kernel_extract(self, phi, k1, k2, stream=None):
        N.check(N.load().kernel_extract(self._pp(), _ptr(phi, self.vdtype, self.vshape, "phi"),
                                        _ptr(k1, torch.complex128, self.k1_shape, "k1"),
                                        _ptr(k2, torch.complex128, self.k2_shape, "k2"), _stream(stream)))

    def channel_remap(self, lam, phi, k1, k2, gamma_out, lam_box=None, f_out=None, stream=None):
        """lam: 4 scalars; lam_box (optional): [4][Nv-1][Nv][Nv] complex128 local Lambda;
        f_out (optional): the full vertex Gamma + Phi."""
        arr = (ctypes.c_double * 4)(*[float(v) for v in lam])
        lb = ctypes.c_void_p(0) if lam_box is None else _ptr(lam_box, torch.complex128, self.lam_shape, "lam_box")
        fo = ctypes.c_void_p(0) if f_out is None else _ptr(f_out, self.vdtype, self.vshape, "f_out")
        N.check(N.load().channel_remap(self._pp(), arr, lb, _ptr(phi, self.vdtype, self.vshape, "phi"),
                                       _ptr(k1, torch.complex128, self.k1_shape, "k1"),
                                       _ptr(k2, torch.complex128, self.k2_shape, "k2"),
                                       _ptr(gamma_out, self.vdtype, self.vshape, "gamma_out"), fo,
                                       _stream(stream)))

    def sigma_workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        N.check(N.load().sigma_sde_workspace(self._pp(), ctypes.byref(b)))
        return int(b.value)

    def sigma_sde(self, phi, k1, k2, g, mu, sigma_out, ws=None, lam_box=None, stream=None):
        nb = self.sigma_workspace_bytes()
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=phi.device)
        lb = ctypes.c_void_p(0) if lam_box is None else _ptr(lam_box, torch.complex128, self.lam_shape, "lam_box")
        N.check(N.load().sigma_sde(self._pp(), _ptr(phi, self.vdtype, self.vshape, "phi"),
                                   _ptr(k1, torch.complex128, self.k1_shape, "k1"),
                                   _ptr(k2, torch.complex128, self.k2_shape, "k2"), lb,
                                   _ptr(g, torch.complex128, self.g_shape, "g"),
                                   _ptr(mu, torch.float64, (1,), "mu"),
                                   _ptr(sigma_out, torch.complex128, self.sigma_shape, "sigma_out"),
                                   _ptr(ws, torch.uint8, (ws.numel(),), "ws"), ctypes.c_size_t(ws.numel()),
                                   _stream(stream)))

    def sigma_sde_no_alloc(self, phi, k1, k2, g, mu, sigma_out, lam_box=None, stream=None):
        """sigma_sde with its scratch in the library's static device array (no workspace)."""
        lb = ctypes.c_void_p(0) if lam_box is None else _ptr(lam_box, torch.complex128, self.lam_shape, "lam_box")
        N.check(N.load().sigma_sde_no_alloc(self._pp(), _ptr(phi, self.vdtype, self.vshape, "phi"),
                                            _ptr(k1, torch.complex128, self.k1_shape, "k1"),
                                            _ptr(k2, torch.complex128, self.k2_shape, "k2"), lb,
                                            _ptr(g, torch.complex128, self.g_shape, "g"),
                                            _ptr(mu, torch.float64, (1,), "mu"),
                                            _ptr(sigma_out, torch.complex128, self.sigma_shape, "sigma_out"),
                                            _stream(stream)))

    def bse_workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        N.check(N.load().bse_workspace(self._pp(), ctypes.byref(b)))
        return int(b.value)

    def bse_solve(self, channel: int, gamma, chi0, phi_io, alpha: float = 1.0, stats=None, ws=None,
                  stream=None):
        """gamma, phi_io: [Nq][n][n] of one channel; chi0: [Nq][n] complex128."""
        d = self.d
        shp = (d.Nq, d.n, d.n)
        if ws is None:
            ws = torch.empty(self.bse_workspace_bytes(), dtype=torch.uint8, device=gamma.device)
        st = ctypes.c_void_p(0)
        if stats is not None:
            st = _ptr(stats, torch.int32, (d.Nq, 4), "stats")
        N.check(N.load().bse_solve(self._pp(), int(channel), int(self.pp.precision),
                                   _ptr(gamma, self.vdtype, shp, "gamma"),
                                   _ptr(chi0, torch.complex128, self.x_shape, "chi0"),
                                   _ptr(phi_io, self.vdtype, shp, "phi_io"), float(alpha), st,
                                   _ptr(ws, torch.uint8, (ws.numel(),), "ws"), ctypes.c_size_t(ws.numel()),
                                   _stream(stream)))

    def sigma_mix(self, sigma_new, sigma_io, alpha, dnorm, stream=None):
        N.check(N.load().sigma_mix(self._pp(), _ptr(sigma_new, torch.complex128, self.sigma_shape, "sigma_new"),
                                   _ptr(sigma_io, torch.complex128, self.sigma_shape, "sigma_io"), float(alpha),
                                   _ptr(dnorm, torch.float64, (1,), "dnorm"), _stream(stream)))


def workspace_bytes(p, precision: str = "fp64", resolve_slots: int = 0, bse_tol: float = 0.0) -> int:
    """Device workspace a context of these parameters needs (parquet_query_workspace)."""
    st = Stage(p, precision, resolve_slots, bse_tol)
    b = ctypes.c_size_t()
    N.check(N.load().parquet_query_workspace(st._pp(), ctypes.byref(b)))
    return int(b.value)


class Solver:
    """A parquet context on one device: workspace owned by a torch uint8 tensor
    (at least ws_bytes, so that reinit can take parameters of a larger need)."""

    def __init__(self, p, precision: str = "fp64", device: str = "cuda:0", stream=None, resolve_slots: int = 0,
                 bse_tol: float = 0.0, ws_bytes: int = 0, bse_tile: int = 0):
        self.stage = Stage(p, precision, resolve_slots, bse_tol, bse_tile)
        self._stage_args = (precision, resolve_slots, bse_tol, bse_tile)
        self.device = torch.device(device)
        self.stream = stream
        lib = N.load()
        b = ctypes.c_size_t()
        N.check(lib.parquet_query_workspace(self.stage._pp(), ctypes.byref(b)))
        self.ws = torch.empty(max(int(b.value), int(ws_bytes)), dtype=torch.uint8, device=self.device)
        if stream is not None:
            self.ws.record_stream(stream)      # the context's work runs on its own stream
        self.ctx = None
        self.reinit()

    def reinit(self, p=None):
        """Start again from the bare-vertex state (a new context on the same
        workspace: parquet_init, nothing allocated), with new model parameters
        p if given (any whose workspace fits the one held)."""
        if p is not None:
            st = Stage(p, *self._stage_args)
            b = ctypes.c_size_t()
            N.check(N.load().parquet_query_workspace(st._pp(), ctypes.byref(b)))
            if int(b.value) > self.ws.numel():
                raise ValueError(f"parameters need a {int(b.value)}-byte workspace, "
                                 f"this solver holds {self.ws.numel()}")
            self.stage = st
        self.close()
        ctx = ctypes.c_void_p()
        N.check(N.load().parquet_init(self.stage._pp(), ctypes.c_void_p(self.ws.data_ptr()),
                                      ctypes.c_size_t(self.ws.numel()), _stream(self.stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self.last_stats = None

    @property
    def dims(self):
        return self.stage.d

    def iterate(self, n: int = 1, tol: float = 0.0):
        """Up to n iterations, stopping on the convergence test of tol (tol > 0:
        the change of Sigma below tol; tol < 0: the estimated distance to the
        fixed point below |tol| max|Sigma|; tol = 0: never; see parquet_iterate).
        Returns (iterations done, converged, stats of the
        last iteration); not reaching tol is no error (converged is False).
        Raises ParquetError for a non-finite self-energy or an unresolved BSE
        block (the iterations done are kept in the context)."""
        st = N.PqIterStats()
        done = ctypes.c_int32()
        conv = ctypes.c_int32()
        status = N.load().parquet_iterate(self.ctx, int(n), float(tol), ctypes.byref(st),
                                          ctypes.byref(done), ctypes.byref(conv))
        self.last_stats = st
        self.last_status = status
        self.last_done = int(done.value)
        if status != N.PQ_ERR_NOT_CONVERGED:
            N.check(status)
        return int(done.value), bool(conv.value), st

    def _field_shape_dtype(self, name):
        s = self.stage
        return {
            "sigma": (s.sigma_shape, torch.complex128), "g": (s.g_shape, torch.complex128),
            "phi": (s.vshape, s.vdtype), "gamma": (s.vshape, s.vdtype),
            "k1": (s.k1_shape, torch.complex128), "k2": (s.k2_shape, torch.complex128),
            "mu": ((1,), torch.float64), "xph": (s.x_shape, torch.complex128),
            "xpp": (s.x_shape, torch.complex128), "lambda": (s.lam_shape, torch.complex128),
            "f": (s.vshape, s.vdtype),
        }[name]

    def get(self, name: str) -> torch.Tensor:
        shape, dtype = self._field_shape_dtype(name)
        out = torch.empty(shape, dtype=dtype, device=self.device)
        N.check(N.load().parquet_get(self.ctx, N.FIELDS[name], ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_size_t(out.numel() * out.element_size())))
        return out

    def set(self, name: str, value: torch.Tensor):
        shape, dtype = self._field_shape_dtype(name)
        v = value.to(device=self.device, dtype=dtype).contiguous()
        if tuple(v.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {shape}")
        N.check(N.load().parquet_set(self.ctx, N.FIELDS[name], ctypes.c_void_p(v.data_ptr()),
                                     ctypes.c_size_t(v.numel() * v.element_size())))

    def warm_start(self, k1: torch.Tensor, k2: torch.Tensor, sigma: torch.Tensor = None):
        """Rebuild Phi in place from kernel values (complex128, K1 [4][Nq] and
        K2 [4][Nq][n]) and, if given, take Sigma [Nve][Nk] (parquet_warm_start)."""
        st = self.stage
        sp = _ptr(sigma, torch.complex128, st.sigma_shape, "sigma") if sigma is not None else None
        N.check(N.load().parquet_warm_start(self.ctx, _ptr(k1, torch.complex128, st.k1_shape, "k1"),
                                            _ptr(k2, torch.complex128, st.k2_shape, "k2"), sp))

    def copy_state_from(self, other: "Solver"):
        """Take Sigma, mu~, Phi and the iteration count of another context of the
        same box (converting the vertex storage as needed)."""
        N.check(N.load().parquet_copy_state(self.ctx, other.ctx))

    def close(self):
        if self.ctx is not None:
            N.load().parquet_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None
_stream_pool = {}     # device -> streams not bound to a context


def new_stream(device: str = "cuda:0"):
    """A stream of its own for one context (hipStreamCreate, default priority),
    wrapped for torch; torch.cuda.Stream() draws from a small recycled pool, so
    two of those can be the same stream. Streams are never destroyed: a
    tensor recorded on a stream (the context workspace) makes torch's
    allocator record an event on that stream when the tensor is freed, which
    may happen after the context is gone. release_stream returns one for reuse."""
    global _hip
    pool = _stream_pool.setdefault(str(device), [])
    if pool:
        return pool.pop()
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipStreamCreate.restype = ctypes.c_int
    with torch.cuda.device(device):
        h = ctypes.c_void_p()
        if _hip.hipStreamCreate(ctypes.byref(h)) != 0:
            raise RuntimeError("hipStreamCreate failed")
        return torch.cuda.ExternalStream(h.value, device=torch.device(device))


def release_stream(stream):
    """Give a stream from new_stream back once no context uses it."""
    stream.synchronize()
    _stream_pool.setdefault(str(stream.device), []).append(stream)


def iterate_batch(solvers, n_iter: int, tol: float = 0.0):
    """Iterate several solvers concurrently (parquet_iterate_batch): each must
    own a stream of its own (Solver(..., stream=new_stream())). Returns the
    per-solver (iterations done, converged) lists."""
    n = len(solvers)
    arr = (ctypes.c_void_p * n)(*[s.ctx.value for s in solvers])
    done = (ctypes.c_int32 * n)()
    conv = (ctypes.c_int32 * n)()
    st = N.load().parquet_iterate_batch(arr, n, int(n_iter), float(tol), done, conv)
    if st not in (N.PQ_OK, N.PQ_ERR_NONFINITE, N.PQ_ERR_SINGULAR, N.PQ_ERR_NOT_CONVERGED):
        N.check(st)
    return [int(x) for x in done], [bool(x) for x in conv]


class Batch:
    """Instances of one box iterated together (parquet_batch_*): one vertex
    arena, one BSE launch sequence per channel over every active (instance, q)
    block, one HIP graph per round; autotune times the two complex64 update tiles
    on the batch's own block count at set-up."""

    def __init__(self, params, precision: str = "fp32", device: str = "cuda:0", autotune: bool = True):
        self.params = list(params)
        self.precision = precision
        self.device = torch.device(device)
        K = len(self.params)
        self.K = K
        self._pp = (N.PqParams * K)(*[N.make_params(p, precision) for p in self.params])
        lib = N.load()
        b = ctypes.c_size_t()
        N.check(lib.parquet_batch_query_workspace(self._pp, K, ctypes.byref(b)))
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.stream = new_stream(str(self.device))           # pooled: created once, reused
        self.ws.record_stream(self.stream)
        h = ctypes.c_void_p()
        N.check(lib.parquet_batch_init(self._pp, K, ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_size_t(b.value),
                                       ctypes.c_void_p(self.stream.cuda_stream), int(bool(autotune)),
                                       ctypes.byref(h)))
        self.h = h
        self.stage = Stage(self.params[0], precision)

    @staticmethod
    def workspace_bytes(params, precision: str = "fp32") -> int:
        K = len(params)
        pp = (N.PqParams * K)(*[N.make_params(p, precision) for p in params])
        b = ctypes.c_size_t()
        N.check(N.load().parquet_batch_query_workspace(pp, K, ctypes.byref(b)))
        return int(b.value)

    def iterate(self, n: int, tol: float = -1e-6, diverge: float = 0.0) -> int:
        """Up to n rounds; returns the number of instances still active."""
        left = ctypes.c_int32()
        N.check(N.load().parquet_batch_iterate(self.h, int(n), float(tol), float(diverge), ctypes.byref(left)))
        return int(left.value)

    def status(self):
        """Per instance: (iterations, state name, last change of Sigma)."""
        it = (ctypes.c_int32 * self.K)()
        st = (ctypes.c_int32 * self.K)()
        dn = (ctypes.c_double * self.K)()
        N.check(N.load().parquet_batch_status(self.h, it, st, dn))
        return [(int(it[i]), N.BATCH_STATES[int(st[i])], float(dn[i])) for i in range(self.K)]

    def tile(self):
        t = ctypes.c_int32()
        ms = (ctypes.c_float * 2)()
        N.check(N.load().parquet_batch_tile(self.h, ctypes.byref(t), ms))
        return int(t.value), float(ms[0]), float(ms[1])

    def get(self, i: int, name: str) -> torch.Tensor:
        st = self.stage
        shape, dtype = {"sigma": (st.sigma_shape, torch.complex128), "g": (st.g_shape, torch.complex128),
                        "mu": ((1,), torch.float64), "k1": (st.k1_shape, torch.complex128),
                        "k2": (st.k2_shape, torch.complex128), "phi": (st.vshape, st.vdtype)}[name]
        out = torch.empty(shape, dtype=dtype, device=self.device)
        N.check(N.load().parquet_batch_get(self.h, int(i), N.FIELDS[name], ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_size_t(out.numel() * out.element_size())))
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            N.load().parquet_batch_destroy(self.h)
            self.h = None
            release_stream(self.stream)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batched(params, precision: str = "fp32", device: str = "cuda:0", tol: float = -1e-6,
                max_iter: int = 150, diverge: float = 1e2, mem_budget: float = 200e9, autotune: bool = True,
                keep_sigma: bool = False, progress=None):
    """Solve many instances with the batched solver: grouped by box (lattice,
    Nv, f_ext), each group split into batches whose workspace fits
    mem_budget, the batches run one after another. Returns (per-instance
    records in the order of params, per-batch records)."""
    import time
    groups = {}
    for i, p in enumerate(params):
        groups.setdefault((p.Lx, p.Ly, p.Nv, p.f_ext), []).append(i)
    out = [None] * len(params)
    batches = []
    for key in sorted(groups):
        idx = groups[key]
        per = Batch.workspace_bytes([params[idx[0]]], precision)
        nd = N.dims(N.make_params(params[idx[0]], precision))
        cap = max(1, min(int(mem_budget // max(per, 1)), 16384 // nd.Nq))
        for c0 in range(0, len(idx), cap):
            chunk = idx[c0:c0 + cap]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b = Batch([params[i] for i in chunk], precision, device, autotune)
            t1 = time.perf_counter()
            rounds = 0
            while rounds < max_iter:
                left = b.iterate(min(10, max_iter - rounds), tol, diverge)
                rounds += min(10, max_iter - rounds)
                if progress is not None:
                    progress(key, rounds, left)
                if left == 0:
                    break
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tile = b.tile()
            for j, (it, state, dn) in zip(chunk, b.status()):
                rec = dict(iterations=it, state=state, converged=state == "converged", dsigma=dn)
                if keep_sigma:
                    rec["sigma"] = b.get(chunk.index(j), "sigma").cpu()
                out[j] = rec
            batches.append(dict(box=list(key), instances=len(chunk), setup_sec=round(t1 - t0, 3),
                                run_sec=round(t2 - t1, 3), tile=tile[0], tile_ms=[round(tile[1], 3), round(tile[2], 3)],
                                instance_iterations=sum(out[j]["iterations"] for j in chunk)))
            b.close()
            del b
            torch.cuda.empty_cache()
    return out, batches


class BatchRunner:
    """Solve many parquet instances to convergence on one device.

    Instances run concurrently, each in its own context and stream with its
    iteration captured in a graph (parquet_iterate_batch); at most `width` at a
    time and within `mem_budget` bytes of workspace, new instances starting as
    others finish. `autotune` picks the width from `widths` by timing a few
    batched iterations of copies of the median instance (instance-iterations
    per second) before the run."""

    def __init__(self, params, precision: str = "fp32", device: str = "cuda:0",
                 mem_budget: float = 200e9, widths=(1, 2, 4, 8, 16, 32)):
        self.params = list(params)
        self.precision = precision
        self.device = device
        self.mem_budget = float(mem_budget)
        self.widths = tuple(widths)
        self.width = None
        self.tuning = {}

    def _bytes(self, p):
        b = ctypes.c_size_t()
        N.check(N.load().parquet_query_workspace(ctypes.byref(N.make_params(p, self.precision)), ctypes.byref(b)))
        return int(b.value)

    def autotune(self, probe_iters: int = 3):
        import time
        sizes = sorted((self._bytes(p), i) for i, p in enumerate(self.params))
        p_med = self.params[sizes[len(sizes) // 2][1]]
        nb = self._bytes(p_med)
        best = None
        for w in self.widths:
            if w > len(self.params) or w * nb > self.mem_budget:
                break
            streams = [new_stream(self.device) for _ in range(w)]
            solvers = [Solver(p_med, self.precision, self.device, stream=st) for st in streams]
            iterate_batch(solvers, 1)                       # graph capture + first replay
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iterate_batch(solvers, probe_iters)
            torch.cuda.synchronize()
            rate = w * probe_iters / (time.perf_counter() - t0)
            self.tuning[w] = rate
            for sv in solvers:
                sv.close()
            del solvers, sv
            torch.cuda.empty_cache()
            for st in streams:
                release_stream(st)
            if best is None or rate > self.tuning[best]:
                best = w
        self.width = best or 1
        return self.width

    def run(self, tol: float = 1e-6, max_iter: int = 200, chunk: int = 5):
        """Returns one record per instance: iterations, converged, seconds from
        its start to its end (wall, shared with the instances beside it)."""
        import time
        width = self.width or self.autotune()
        pending = list(range(len(self.params)))
        active = []                 # (index, solver, start time, iterations)
        out = [None] * len(self.params)
        used = 0.0
        t_all = time.perf_counter()
        while pending or active:
            while pending and len(active) < width:
                i = pending[0]
                nb = self._bytes(self.params[i])
                if active and used + nb > self.mem_budget:
                    break
                pending.pop(0)
                st = new_stream(self.device)
                s = Solver(self.params[i], self.precision, self.device, stream=st)
                active.append([i, s, time.perf_counter(), 0, nb, st])
                used += nb
            done, conv = iterate_batch([a[1] for a in active], chunk, tol)
            keep = []
            for a, d, c in zip(active, done, conv):
                a[3] += d
                finished = c or a[3] >= max_iter or d < chunk
                if finished:
                    sig = a[1].get("sigma")
                    out[a[0]] = dict(iterations=a[3], converged=bool(c), sec=time.perf_counter() - a[2],
                                     finite=bool(torch.isfinite(torch.view_as_real(sig)).all()))
                    a[1].close()
                    a[1] = None
                    used -= a[4]
                    release_stream(a[5])
                else:
                    keep.append(a)
            active = keep
            torch.cuda.empty_cache()
        return out, time.perf_counter() - t_all


def converge_mixed(p, tol: float = -1e-6, switch_tol: float = -2e-5, max_iter: int = 200,
                   device: str = "cuda:0", low: str = "fp32", solvers=None, warm=None):
    """Iterate the complex64 path (precision ``low``: "fp32" or "bf16x3") from
    the bare-vertex start until the convergence test of switch_tol is met, then
    continue on the complex128/FP64 path from that state until the test of tol
    is met (tests as in parquet_iterate: negative values are relative distances
    to the fixed point). Returns the FP64 solver and a dict with the iteration
    counts of both phases (the first under the key iterations_fp32). ``solvers``:
    an already allocated (low, fp64) pair of the same box, re-initialised here
    (the low one is closed at the switch). warm: (K1, K2) or (K1, K2, Sigma)
    to start from (Solver.warm_start) instead of the bare vertex."""
    if low not in ("fp32", "bf16x3"):
        raise ValueError(f"low precision {low!r} must be fp32 or bf16x3")
    if solvers is not None:
        s32, s64 = solvers
        s32.reinit(p)
    else:
        s32 = Solver(p, low, device)
    if warm is not None:
        s32.warm_start(*warm)
    done32, conv32, st32 = s32.iterate(max_iter, switch_tol)
    torch.cuda.synchronize()
    if solvers is not None:
        s64.reinit(p)
    else:
        s64 = Solver(p, "fp64", device)
    s64.copy_state_from(s32)
    s32.close()
    del s32
    done64, conv64, st64 = s64.iterate(max(0, max_iter - done32), tol)
    info = dict(iterations_fp32=done32, iterations_fp64=done64, converged=bool(conv64),
                dsigma=st64.dsigma if done64 else st32.dsigma)
    return s64, info
