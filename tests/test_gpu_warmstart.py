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


@pytest.mark.parametrize("widths,batch", [((2, 48, 40, 37), 9), ((3, 16, 16), 16), ((2, 512, 512, 130), 64)])
def test_mlp_forward_and_gradient_match_cpu(widths, batch):
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
    ref = M.forward(p.astype(np.float64), widths, x.astype(np.float64))
    y = out.cpu().numpy()
    assert np.max(np.abs(y - ref[-1])) < 2e-5 * max(1.0, np.max(np.abs(ref[-1])))
    loss = net.backward(X, acts, Tt)
    lref, gref = M.loss_and_grad(p.astype(np.float64), widths, x.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss.item()) - lref) < 1e-5 * max(1.0, lref)
    g = net.g.cpu().numpy()
    assert np.max(np.abs(g - gref)) < 1e-4 * max(1e-3, np.max(np.abs(gref)))


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


def test_warm_start_pipeline_small():
    """Train on a handful of converged local-model solves and start a held-out
    one from the predicted kernels: it reaches the same fixed point."""
    print("CASE warm start pipeline", flush=True)
    ws = _ws()
    base = config("tiny_local", Nv=8, alpha=0.5)
    train = [base.replace(U=u, beta=b) for u in (0.6, 0.8, 1.0, 1.2) for b in (2.0, 3.0, 4.0)]
    k1s, k2s, sigs, ps = [], [], [], []
    for p in train:
        conv, it, k1, k2, sig = ws.converged_kernels(p, "fp64", tol=1e-9)
        assert conv
        ps.append(p), k1s.append(k1), k2s.append(k2), sigs.append(sig)
    pred = ws.KernelPredictor(base, hidden=(64, 64), seed=0)
    hist = pred.fit(ps, k1s, k2s, sigs, steps=400, batch=12, lr=3e-3)
    assert hist[-1][1] < hist[0][1]
    held = base.replace(U=0.9, beta=2.5)
    k1, k2, sig = pred.predict(held)
    warm = ws.solve_timed(held, "fp64", 1e-9, 300, warm=(k1, k2, sig))
    bare = ws.solve_timed(held, "fp64", 1e-9, 300)
    assert warm["converged"] and bare["converged"] and not warm["fallback"]
    from paper_1510_03330_amd.ops import Solver
    a, b = Solver(held, "fp64"), Solver(held, "fp64")
    phi = torch.empty(a.stage.vshape, dtype=a.stage.vdtype, device=DEV)
    ws.phi_from_kernels(held, "fp64", k1, k2, phi)
    a.set("phi", phi)
    a.iterate(300, 1e-11)
    b.iterate(300, 1e-11)
    assert torch.max(torch.abs(a.get("sigma") - b.get("sigma"))).item() < 1e-9
    a.close()
    b.close()
