"""The batched solver (parquet_batch_*): instances of one box in one vertex
arena, the BSE of every active (instance, q) block in one launch sequence per
channel, one HIP graph per round. Checked against the oracle instance by
instance, against independent contexts bit for bit (including the retirement
of instances that converge at different rounds), and the two FP32 update
tiles the set-up timing chooses between against each other."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import parquet as P
from workloads import config, parameter_draws, rand_complex, bse_microbench_gamma

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _ops():
    from paper_1510_03330_amd import ops
    return ops


INSTANCES = [dict(), dict(U=1.2, beta=2.5, filling=0.9, tp=-0.2), dict(U=0.7, beta=4.0, filling=1.0, tp=0.0,
                                                                        kernel_level=1)]


def test_batch_instances_match_oracle():
    """Three instances of the 2x2, Nv = 4 box (different U, beta, filling, t'
    and kernel level) in one batch: two rounds give each instance's Sigma, Phi
    and mu of two oracle iterations."""
    ops = _ops()
    ps = [config("tiny_2x2", **o) for o in INSTANCES]
    print("CASE batch vs oracle", flush=True)
    b = ops.Batch(ps, "fp64", DEV, autotune=False)
    g = P.Grid(ps[0].Lx, ps[0].Ly, ps[0].Nv, ps[0].f_ext)
    states = [P.init_state(p, g) for p in ps]
    for i in range(len(ps)):
        assert relerr(H(b.get(i, "sigma")), states[i].sigma) < 1e-12
    for rnd in range(2):
        assert b.iterate(1, 0.0) == len(ps)
        states = [P.iterate(p, st, g) for p, st in zip(ps, states)]
        for i, st in enumerate(states):
            assert relerr(H(b.get(i, "sigma")), st.sigma) < 1e-11, (rnd, i)
            assert relerr(H(b.get(i, "phi")), st.phi) < 1e-11, (rnd, i)
            assert abs(H(b.get(i, "mu"))[0] - st.mu) < 1e-12
        for (it, state, dn), st in zip(b.status(), states):
            assert it == rnd + 1 and state == "running"
            assert abs(dn - st.last_dsigma) < 1e-10 * max(1.0, st.last_dsigma)
    b.close()


@pytest.mark.parametrize("prec,tol", [("fp64", -1e-7), ("fp32", -1e-5), ("bf16x3", -1e-5)])
def test_batch_equals_independent_contexts_with_retirement(prec, tol):
    """Six seeded 2x4, Nv = 6 instances run to the relative stopping rule in
    one batch and each in its own context: every instance stops at the same
    iteration with a bit-identical Sigma, also after other instances retired
    and its vertex moved to another arena slot (complex64: to 1e-5, above
    the FP32 rounding floor of the fixed point)."""
    ops = _ops()
    base = config("small_2x4", alpha=0.5)
    ps = parameter_draws(base, {"U": (0.8, 1.6), "beta": (2.0, 4.0), "filling": (0.9, 1.05), "tp": (-0.2, 0.2)},
                         range(100, 106))
    print("CASE batch vs contexts", prec, flush=True)
    b = ops.Batch(ps, prec, DEV, autotune=False)
    rounds = 0
    while b.iterate(5, tol, 1e2) > 0 and rounds < 300:
        rounds += 5
    stat = b.status()
    assert all(s == "converged" for _, s, _ in stat), stat
    assert len(set(it for it, _, _ in stat)) > 1           # retired at different rounds
    for i, p in enumerate(ps):
        s = ops.Solver(p, prec, DEV)
        done, conv, st = s.iterate(300, tol)
        assert conv and done == stat[i][0], (i, done, stat[i])
        assert torch.equal(s.get("sigma"), b.get(i, "sigma")), i
        assert torch.equal(s.get("k2"), b.get(i, "k2")), i
        s.close()
    b.close()


@pytest.mark.parametrize("prec,tile,rel", [("fp32", 1, 1e-6), ("bf16x3", 1, 5e-5)])
def test_update_tiles_agree(prec, tile, rel):
    """The complex64 update tiles (bse_tile 0: 64 x 64 per wave, 1: 64 x 32)
    run the same products in the same order. The FP32 tiles both start their
    accumulators from C and agree to FP32 rounding (the compiler contracts the
    epilogue arithmetic of the two instantiations differently); the BF16x3
    narrow tile loads its C tile across the steps and adds it after the
    products, a different FP32 summation order whose rounding the solve
    carries (about 1e-5 of max|F| here). On the 4x4, Nv = 16 box (n = 256: two
    panels, the forward and the back-substitution update both take the
    tile)."""
    ops = _ops()
    p = config("c2")
    out = []
    for t in (0, tile):
        st = ops.Stage(p, prec, bse_tile=t)
        d = st.d
        gam = torch.from_numpy(bse_microbench_gamma(d.n, range(d.Nq)).astype(np.complex64)).to(DEV)
        x = torch.from_numpy(rand_complex((d.Nq, d.n), 77, 0.3)).to(DEV)
        phi = torch.from_numpy(rand_complex((d.Nq, d.n, d.n), 78, 0.1).astype(np.complex64)).to(DEV)
        st.bse_solve(1, gam, x, phi, alpha=0.5)
        out.append(phi)
    assert not torch.equal(out[0], torch.zeros_like(out[0]))
    diff = (out[0] - out[1]).abs().max().item()
    assert diff <= rel * out[0].abs().max().item(), (tile, diff)


@pytest.mark.parametrize("prec,nv", [("fp32", 64), ("bf16x3", 64), ("fp64", 48)])
def test_lookahead_iteration_equals_captured_batch(prec, nv):
    """parquet_iterate runs the next panel's diagonal-block inversion and
    pivot-row step on a second stream beside the update of the rows below it
    (look-ahead); the batched solver captures the same kernels on one stream
    without it. On boxes with several panels (2x4 lattice, Nv = 64: n = 512,
    four panels of 128; Nv = 48 for complex128: six panels of 64), where
    every look-ahead point is reached, two iterations of both agree bit for
    bit: the steps that run beside the update touch nothing it reads or
    writes."""
    ops = _ops()
    p = config("small_2x4", Nv=nv)
    print("CASE look-ahead vs captured", prec, nv, flush=True)
    s = ops.Solver(p, prec, DEV)
    s.iterate(2, 0.0)
    sig, k2 = s.get("sigma"), s.get("k2")
    s.close()
    del s
    torch.cuda.empty_cache()
    b = ops.Batch([p], prec, DEV, autotune=False)
    b.iterate(2, 0.0, 0.0)
    assert torch.equal(sig, b.get(0, "sigma"))
    assert torch.equal(k2, b.get(0, "k2"))
    b.close()
    torch.cuda.empty_cache()
