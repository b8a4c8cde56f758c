"""Whole-iteration parity of the HIP solver context (parquet_init / parquet_iterate)
with the FP64 oracle: a few iterations on small lattices, and the converged
self-energy of the momentum-independent parquet approximation (Nk = 1,
semicircle, U = 1, beta = 5, Nv = 32) to the 1e-6 relative bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import parquet as P
from workloads import config

pytestmark = pytest.mark.gpu


def _solver(p, prec):
    from paper_1510_03330_amd.ops import Solver
    return Solver(p, prec)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("name", ["tiny_2x2", "small_2x4", "tiny_local"])
def test_first_iterations_match_oracle(name):
    print("CASE iterations", name, flush=True)
    p = config(name)
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    st = P.init_state(p, g)
    s = _solver(p, "fp64")
    assert relerr(H(s.get("sigma")), st.sigma) < 1e-12
    for it in range(3):
        st = P.iterate(p, st, g)
        done, conv, stats = s.iterate(1)
        assert done == 1
        assert abs(stats.dsigma - st.last_dsigma) < 1e-10 * max(1.0, st.last_dsigma)
        assert relerr(H(s.get("sigma")), st.sigma) < 1e-11
        assert relerr(H(s.get("phi")), st.phi) < 1e-11
        if g.Nk > 1:
            assert abs(H(s.get("mu"))[0] - st.mu) < 1e-12
    s.close()


@pytest.fixture(scope="module")
def c1_oracle():
    p = config("c1")
    return p, P.solve(p, max_iter=100)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-6)])
def test_c1_converged_sigma(c1_oracle, prec, tol):
    print("CASE c1 converged", prec, flush=True)
    p, ref = c1_oracle
    s = _solver(p, prec)
    done, conv, stats = s.iterate(200, p.tol)
    assert conv, stats.dsigma
    sig = H(s.get("sigma"))
    assert relerr(sig, ref.sigma) < tol
    phi = H(s.get("phi")).astype(np.complex128)
    assert relerr(phi, ref.phi) < 10 * tol
    s.close()


def test_resume_reproduces_next_iterate():
    """Checkpoint/resume: set the state of a second context from the first and
    the next iterates agree bitwise (FP64 path)."""
    p = config("tiny_2x2")
    a = _solver(p, "fp64")
    a.iterate(2)
    b = _solver(p, "fp64")
    b.set("sigma", a.get("sigma"))
    b.set("phi", a.get("phi"))
    a.iterate(1)
    b.iterate(1)
    assert torch.equal(a.get("sigma"), b.get("sigma"))
    assert torch.equal(a.get("phi"), b.get("phi"))
