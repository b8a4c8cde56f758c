"""Learned warm start: the perceptron kernels against the CPU reference
(forward outputs, gradients at the bf16 weights, one Adam step), the vertex
rebuilt from kernel values against the oracle's kernel form, and the whole
pipeline on a small box (trained predictor, warm-started iteration converging
to the bare start's fixed point)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as M
from oracle import parquet as P
from workloads import config, rand_complex

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ws():
    from paper_1510_03330_amd import warmstart
    return warmstart


def _gemm_bound(p, widths, x, acts_ref, d_ref=None):
    """Elementwise error bounds of the matrix-core products against FP64 with
    the same bf16 weights: each FP32 operand split into hi + lo bf16 terms is
    off by at most 2^-16 of itself, the dropped lo x lo product of two split
    operands by 2^-16 of the product, and FP32 accumulation over K terms by K
    2^-24 of the sum of magnitudes; so |error| <= (3 2^-16 + K 2^-23) (|A| |B|)."""
    out = []
    h = np.abs(x)
    for (W, b), a in zip(M.unpack(p, widths), acts_ref):
        Wb = np.abs(M.bf16_round(W))
        K = W.shape[1]
        out.append((3 * 2.0 ** -16 + K * 2.0 ** -23) * (h @ Wb.T) + 2.0 ** -23 * np.abs(b))
        h = np.abs(a)
    return out


@pytest.mark.parametrize("widths,batch", [((2, 48, 40, 37), 9), ((3, 16, 16), 16), ((2, 512, 512, 130), 64),
                                          ((4, 96, 70, 200), 100)])
def test_mlp_forward_and_gradient_match_cpu(widths, batch):
    """Forward outputs and gradients of the bf16 matrix-core products against
    the FP64 reference at the same bf16 weights, within the error bound of the
    hi + lo operand split (shapes with ragged 64-tiles and 32-deep k rounds)."""
    print("CASE mlp", widths, batch, flush=True)
    ws = _ws()
    net = ws.MLP(widths, DEV, seed=1)
    rng = np.random.default_rng(2)
    p = (rng.standard_normal(net.count) * 0.3).astype(np.float32)
    net.set_params(torch.from_numpy(p))
    x = rng.standard_normal((batch, widths[0])).astype(np.float32)
    t = rng.standard_normal((batch, widths[-1])).astype(np.float32)
    X, Tt = torch.from_numpy(x).to(DEV), torch.from_numpy(t).to(DEV)
    acts, out = net.forward(X)
    p64 = p.astype(np.float64)
    ref = M.forward(p64, widths, x.astype(np.float64))
    # bound of the last layer, propagated from the hidden layers' own bounds
    # through the Lipschitz-1 tanh and the bf16 weights
    bounds = _gemm_bound(p64, widths, x.astype(np.float64), ref)
    prop = np.zeros((batch, widths[1]))
    for li, ((W, b), bd) in enumerate(zip(M.unpack(p64, widths), bounds)):
        e = bd + (prop @ np.abs(M.bf16_round(W)).T if li > 0 else 0.0)
        prop = e
    y = out.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(y - ref[-1]) <= 1.01 * prop + 1e-30)
    loss = net.backward(X, acts, Tt)
    lref, gref = M.loss_and_grad(p64, widths, x.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss.item()) - lref) < 1e-5 * max(1.0, lref)
    g = net.g.cpu().numpy()
    # the gradient products are split on both sides; with the propagated
    # forward error the relative error stays near 1e-4 of the largest entry
    assert np.max(np.abs(g - gref)) < 2e-4 * max(1e-3, np.max(np.abs(gref)))


def test_mlp_products_are_exact_on_bf16_representable_inputs():
    """With weights, inputs and upstream gradients that are small integers
    times powers of two (exact in bf16, products and sums exact in FP32), the
    matrix-core forward pass of a linear network and its weight gradient are
    exact: pins the operand layout and the k/m/n tiling (a transposed or
    shifted operand gives a different integer)."""
    ws = _ws()
    # one linear layer: the forward product is ragged in m (batch 32 of a
    # 64-tile) and k (70 of 32-deep rounds), the weight gradient in n (70);
    # batch x outputs = 2^13 makes d = 2 (y - t) / count exact
    widths, batch = (70, 256), 32
    net = ws.MLP(widths, DEV, seed=0)
    rng = np.random.default_rng(7)
    W = rng.integers(-8, 9, size=(256, 70)).astype(np.float32) / 8.0
    b = rng.integers(-4, 5, size=256).astype(np.float32)
    net.set_params(torch.from_numpy(np.concatenate([W.ravel(), b])))
    x = rng.integers(-16, 17, size=(batch, 70)).astype(np.float32) / 4.0
    X = torch.from_numpy(x).to(DEV)
    acts, out = net.forward(X)
    ref = x.astype(np.float64) @ W.T.astype(np.float64) + b
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    e = rng.integers(-3, 4, size=(batch, 256)).astype(np.float64)
    Tt = torch.from_numpy((ref - e).astype(np.float32)).to(DEV)
    net.backward(X, acts, Tt)
    d = 2.0 * e / (batch * 256)
    g = net.g.cpu().numpy().astype(np.float64)
    assert np.array_equal(g[:256 * 70], (d.T @ x.astype(np.float64)).ravel())
    assert np.array_equal(g[256 * 70:], d.sum(axis=0))


def test_mlp_basis_and_expand():
    """The factorised head: the basis rows are orthonormal, the mean is the
    row mean, the coordinates are lower triangular and rebuild every training
    row, a duplicated row adds no direction and neither does the last row (the
    centred rows sum to zero), and mlp_expand of a coordinate row gives back
    that training row."""
    import ctypes
    from paper_1510_03330_amd import native as Nn
    rows, L = 9, 5000
    rng = np.random.default_rng(11)
    Y0 = rng.standard_normal((rows, L)).astype(np.float32)
    Y0[5] = Y0[2]                                            # no new direction
    Y = torch.from_numpy(Y0.copy()).to(DEV)
    mean = torch.empty(L, dtype=torch.float32, device=DEV)
    coef = torch.empty((rows, rows + 3), dtype=torch.float32, device=DEV)
    scale = torch.empty(1, dtype=torch.float32, device=DEV)
    lib = Nn.load()
    wsb = ctypes.c_size_t()
    Nn.check(lib.mlp_basis_workspace(rows, ctypes.byref(wsb)))
    ws = torch.empty(int(wsb.value), dtype=torch.uint8, device=DEV)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    Nn.check(lib.mlp_basis(p(Y), rows, L, p(mean), p(coef), rows + 3, p(scale), p(ws), None))
    Q = Y.cpu().numpy().astype(np.float64)
    mu = Y0.astype(np.float64).mean(axis=0)
    assert np.max(np.abs(mean.cpu().numpy() - mu)) < 1e-6
    kept = [i for i in range(rows) if i not in (5, rows - 1)]
    assert np.max(np.abs(Q[5])) == 0.0 and np.max(np.abs(Q[rows - 1])) == 0.0
    G = Q[kept] @ Q[kept].T
    assert np.max(np.abs(G - np.eye(len(kept)))) < 1e-5
    C = coef.cpu().numpy().astype(np.float64)[:, :rows] * float(scale.item())
    assert np.all(C[np.triu_indices(rows, 1)] == 0.0)
    rebuilt = mu + C @ Q
    assert np.max(np.abs(rebuilt - Y0)) < 1e-5 * np.max(np.abs(Y0))
    out = torch.empty(L, dtype=torch.float64, device=DEV)
    c3 = coef[3, :rows].contiguous()
    Nn.check(lib.mlp_expand(p(Y), rows, L, p(mean), p(c3), p(scale), p(out), None))
    assert np.max(np.abs(out.cpu().numpy() - Y0[3])) < 1e-5 * np.max(np.abs(Y0))


def test_mlp_adam_step_matches_cpu():
    ws = _ws()
    net = ws.MLP((2, 8, 5), DEV, seed=3)
    p0 = net.p.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(net.count).astype(np.float32)
    m, v = np.zeros(net.count), np.zeros(net.count)
    p = p0
    for step in (1, 2, 3):
        net.g.copy_(torch.from_numpy(g))
        net.adam(1e-2)
        p, m, v = M.adam(p, m, v, g.astype(np.float64), step, 1e-2)
    assert np.max(np.abs(net.p.cpu().numpy() - p)) < 1e-6
    assert torch.equal(net.pb, net.p.to(torch.bfloat16))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phi_from_kernels_matches_oracle_kernel_form(prec):
    ws = _ws()
    p = config("small_2x4")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    K1 = rand_complex((4, g.Nq), 5, 0.3)
    K2 = rand_complex((4, g.Nq, g.n), 6, 0.3)
    st_dtype = torch.complex128 if prec == "fp64" else torch.complex64
    phi = torch.empty((4, g.Nq, g.n, g.n), dtype=st_dtype, device=DEV)
    ws.phi_from_kernels(p, prec, torch.from_numpy(K1).to(DEV), torch.from_numpy(K2).to(DEV), phi)
    got = phi.cpu().numpy().astype(np.complex128)
    nk, Kk = g.kparts()
    mq, Qq = g.qparts()
    tol = 1e-15 if prec == "fp64" else 1e-6
    for r in range(4):
        for qi in range(0, g.Nq, 3):
            ref = P.kernel_value(g, K1, K2, r, nk[:, None], Kk[:, None], nk[None, :], Kk[None, :], mq[qi], Qq[qi])
            assert np.max(np.abs(got[r, qi] - ref)) < tol * 4


WS_BOX = {"U": (0.8, 1.6), "beta": (2.0, 4.0), "filling": (0.85, 1.0), "tp": (-0.2, 0.0)}


@pytest.fixture(scope="module")
def small_predictor():
    """A 4 -> 3 x 64 -> coordinates network trained on the converged solutions
    of 32 seeded draws (seeds 0..31) of a 2x2 lattice, Nv = 8."""
    from workloads import parameter_draws
    ws = _ws()
    base = config("tiny_2x2_hf", Nv=8, alpha=0.5)
    train = parameter_draws(base, WS_BOX, range(32))
    pred = ws.KernelPredictor(base, WS_BOX, max_samples=len(train), hidden=(64, 64, 64), seed=0)
    for p in train:
        conv, it, k1, k2, sig = ws.converged_kernels(p, "fp64", tol=1e-9, max_iter=400)
        if conv:
            pred.add(p, k1, k2, sig)
    assert len(pred.params) >= 24
    hist = pred.fit(steps=1500, batch=32, lr=3e-3)
    assert hist[-1][1] < 0.1 * hist[0][1]
    return base, pred


def test_warm_start_pipeline_small(small_predictor):
    """Train on seeded (U, beta, n, t') draws of a 2x2 lattice and start a
    held-out one from the predicted kernels: it reaches the bare start's fixed
    point."""
    print("CASE warm start pipeline", flush=True)
    ws = _ws()
    base, pred = small_predictor
    from workloads import parameter_draws
    held = parameter_draws(base, WS_BOX, [10000])[0]
    k1, k2, sig = pred.predict(held)
    from paper_1510_03330_amd.ops import Solver
    a, b = Solver(held, "fp64"), Solver(held, "fp64")
    phi = torch.empty(a.stage.vshape, dtype=a.stage.vdtype, device=DEV)
    ws.phi_from_kernels(held, "fp64", k1, k2, phi)
    a.set("phi", phi)
    a.set("sigma", sig)
    a.iterate(400, 1e-11)
    b.iterate(400, 1e-11)
    assert torch.max(torch.abs(a.get("sigma") - b.get("sigma"))).item() < 1e-9
    a.close()
    b.close()


def test_warm_start_gain_on_held_out_seeds(small_predictor):
    """The gain of the trained network: on held-out seeds (10000 on) the
    warm-started iteration needs fewer iterations than the bare-vertex start,
    on average, to the same stopping rule (Sigma within 1e-6 relative of the
    fixed point), none falls back, and both reach the same fixed point."""
    print("CASE warm start gain", flush=True)
    ws = _ws()
    base, pred = small_predictor
    from workloads import parameter_draws
    held = parameter_draws(base, WS_BOX, range(10000, 10008))
    it_b, it_w = [], []
    for p in held:
        k1, k2, sig = pred.predict(p)
        w = ws.solve_timed(p, "fp64", -1e-6, 400, warm=(k1, k2, sig), keep=True)
        b = ws.solve_timed(p, "fp64", -1e-6, 400, keep=True)
        assert w["converged"] and b["converged"] and not w["fallback"], p
        smax = torch.max(torch.abs(b["sigma"])).item()
        assert torch.max(torch.abs(w["sigma"] - b["sigma"])).item() < 2e-6 * smax
        it_b.append(b["iterations"])
        it_w.append(w["iterations"])
    print("iterations bare", it_b, "warm", it_w, flush=True)
    assert np.mean(it_w) < np.mean(it_b)
