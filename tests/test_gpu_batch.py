"""Many instances on one device: one whole iteration captured in a HIP graph per
context and replayed concurrently (parquet_iterate_batch), and the wave
scheduler with its width autotuner (BatchRunner).

Graph replays are checked against eager iterations of an identical context
after every replay, with the program's own eager work and synchronisations
between replays; a box Lambda set between replays makes the context capture
its iteration again."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import parquet as P
from workloads import config, lambda_box_parts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ops():
    from paper_1510_03330_amd import ops
    return ops


def _pair(p, prec):
    ops = _ops()
    a = ops.Solver(p, prec, DEV, stream=ops.new_stream(DEV))
    b = ops.Solver(p, prec, DEV, stream=ops.new_stream(DEV))
    return a, b


@pytest.mark.parametrize("prec,name", [("fp64", "tiny_2x2"), ("fp32", "small_4x4"), ("bf16x3", "small_2x4")])
def test_graph_replay_matches_eager(prec, name):
    print("CASE graph replay", prec, name, flush=True)
    ops = _ops()
    p = config(name)
    eager, graphed = _pair(p, prec)
    scratch = torch.randn(1 << 20, device=DEV)
    for it in range(5):
        if it == 3:                 # a box Lambda from here on: the graph is captured again
            g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
            ld, lm = lambda_box_parts(g.Nv, seed=5, scale=0.2)
            lam = P.crossing_lambda(g, p.U, ld + p.U, lm - p.U)
            for s in (eager, graphed):
                s.set("lambda", torch.from_numpy(lam))
        eager.iterate(1)
        done, conv = ops.iterate_batch([graphed], 1)
        assert done == [1]
        scratch.mul_(1.0001).add_(0.5)          # eager work of the program between replays
        torch.cuda.synchronize()
        for f in ("sigma", "phi", "gamma", "k2", "xph"):
            assert torch.equal(eager.get(f), graphed.get(f)), (it, f)
    eager.close()
    graphed.close()


def test_concurrent_batch_of_different_boxes_matches_one_by_one():
    print("CASE batch of boxes", flush=True)
    ops = _ops()
    ps = [config("tiny_2x2"), config("small_2x4", U=1.2), config("tiny_local"), config("small_4x4", Nv=6)]
    batch = [ops.Solver(p, "fp64", DEV, stream=ops.new_stream(DEV)) for p in ps]
    single = [ops.Solver(p, "fp64", DEV, stream=ops.new_stream(DEV)) for p in ps]
    done, conv = ops.iterate_batch(batch, 4)
    assert done == [4] * len(ps)
    for s in single:
        s.iterate(4)
    for a, b in zip(batch, single):
        assert torch.equal(a.get("sigma"), b.get("sigma"))
        assert torch.equal(a.get("phi"), b.get("phi"))
    # convergence retires instances one by one
    done, conv = ops.iterate_batch(batch, 300, 1e-9)
    for s, d, c in zip(batch, done, conv):
        assert c and d < 300
    for s in batch + single:
        s.close()


def test_batch_runner_matches_individual_convergence():
    print("CASE batch runner", flush=True)
    ops = _ops()
    ps = [config("tiny_2x2", U=u, beta=b) for u in (1.0, 1.5) for b in (2.0, 3.0)] + \
         [config("tiny_local", U=1.0), config("small_2x4")]
    runner = ops.BatchRunner(ps, precision="fp64", widths=(1, 2, 4))
    w = runner.autotune(probe_iters=2)
    assert w in (1, 2, 4) and set(runner.tuning) <= {1, 2, 4}
    recs, total = runner.run(tol=1e-9, max_iter=300, chunk=7)
    for p, r in zip(ps, recs):
        s = ops.Solver(p, "fp64", DEV)
        done, conv, _ = s.iterate(300, 1e-9)
        s.close()
        assert r["converged"] == conv and r["iterations"] == done, (p, r, done)
