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


@pytest.mark.parametrize("name,over", [("tiny_2x2", {}), ("small_2x4", {}), ("tiny_local", {}),
                                       ("tiny_2x2", dict(kernel_level=0, f_ext=1)),
                                       ("tiny_2x2", dict(kernel_level=1, f_ext=3)),
                                       ("tiny_local", dict(kernel_level=0, f_ext=1)),
                                       ("tiny_local", dict(kernel_level=1, f_ext=2, U=3.0, beta=2.0)),
                                       ("tiny_2x2", dict(regulation=0, f_ext=1, kernel_level=0)),
                                       ("tiny_2x2", dict(regulation=0, f_ext=1)),
                                       ("small_2x4", dict(regulation=0, f_ext=1, kernel_level=1)),
                                       ("tiny_local", dict(regulation=0, f_ext=1, kernel_level=2))])
def test_first_iterations_match_oracle(name, over):
    """Three whole iterations against the oracle, also at the kernel levels,
    regulation boxes and regulation settings the ablation study runs (level 0
    truncation, level 1, f_ext 1..3, the plain unregulated box sum)."""
    print("CASE iterations", name, over, flush=True)
    p = config(name, **over)
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


@pytest.mark.parametrize("name,crossing", [("tiny_2x2", False), ("tiny_local", True), ("small_2x4", True)])
def test_iterations_with_box_lambda(name, crossing):
    """Full parquet / parquet DGA input: a local Lambda on the box set on the
    context (PQ_FIELD_LAMBDA); three iterations against the oracle. crossing:
    a crossing-symmetric Lambda (crossing_lambda) perturbed within an inner
    box of two frequencies, else a general perturbation in every channel."""
    from workloads import lambda_box_parts
    print("CASE iterations box lambda", name, crossing, flush=True)
    p = config(name)
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    if crossing:
        ld, lm = lambda_box_parts(g.Nv, seed=91, scale=0.3, n_inner=1, symmetric=True)
        lam = P.crossing_lambda(g, p.U, ld + p.U, lm - p.U)
    else:
        pa = P.pa_lambda(p.U)
        a, b = lambda_box_parts(g.Nv, seed=92, scale=0.3, symmetric=False)
        c, e = lambda_box_parts(g.Nv, seed=93, scale=0.3, symmetric=False)
        lam = np.stack([pa[r] + part for r, part in enumerate((a, b, c, e))])
    st = P.init_state(p, g)
    s = _solver(p, "fp64")
    s.set("lambda", torch.from_numpy(lam))
    assert np.max(np.abs(H(s.get("lambda")) - lam)) == 0.0
    for it in range(3):
        st = P.iterate(p, st, g, lam=lam)
        done, conv, stats = s.iterate(1)
        assert done == 1
        assert relerr(H(s.get("sigma")), st.sigma) < 1e-11
        assert relerr(H(s.get("phi")), st.phi) < 1e-11
    s.close()


def test_lambda_field_defaults_to_parquet_approximation():
    p = config("tiny_2x2")
    s = _solver(p, "fp32")
    lam = H(s.get("lambda"))
    for r, v in enumerate((p.U, -p.U, 2 * p.U, 0.0)):
        assert np.all(lam[r] == v)
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


def test_copy_state_between_contexts():
    """parquet_copy_state: same storage -> the next iterates agree bitwise;
    complex64 -> complex128 -> the vertex is widened exactly; different boxes
    are rejected before anything runs."""
    from paper_1510_03330_amd.native import ParquetError, PQ_ERR_ARG
    print("CASE copy_state", flush=True)
    p = config("tiny_2x2")
    a = _solver(p, "fp64")
    a.iterate(2)
    b = _solver(p, "fp64")
    b.copy_state_from(a)
    a.iterate(1)
    b.iterate(1)
    assert torch.equal(a.get("sigma"), b.get("sigma"))
    assert torch.equal(a.get("phi"), b.get("phi"))
    c32 = _solver(p, "fp32")
    c32.iterate(2)
    c64 = _solver(p, "fp64")
    c64.copy_state_from(c32)
    assert torch.equal(c64.get("phi"), c32.get("phi").to(torch.complex128))
    assert torch.equal(c64.get("sigma"), c32.get("sigma"))
    other = _solver(config("small_2x4"), "fp64")
    with pytest.raises(ParquetError) as e:
        other.copy_state_from(a)
    assert e.value.status == PQ_ERR_ARG
    for s in (a, b, c32, c64, other):
        s.close()


def test_c1_mixed_precision_converges_to_fp64_solution(c1_oracle):
    """FP32 iterations to 1e-5, then FP64 iterations from that state to the
    1e-8 tolerance: the converged Sigma and Phi carry FP64 accuracy (the FP32
    rounding of the hand-over state is iterated away)."""
    from paper_1510_03330_amd.ops import converge_mixed
    print("CASE c1 mixed precision", flush=True)
    p, ref = c1_oracle
    s, info = converge_mixed(p, tol=p.tol, switch_tol=1e-5, max_iter=200)     # absolute changes
    assert info["converged"] and info["iterations_fp32"] > 0 and info["iterations_fp64"] > 0
    assert relerr(H(s.get("sigma")), ref.sigma) < 1e-8
    assert relerr(H(s.get("phi")), ref.phi) < 1e-7
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reinit_restarts_from_the_bare_vertex(prec):
    """Solver.reinit() (a new context on the same workspace) restarts from the
    bare-vertex state: the iterations after it are bitwise those of a fresh
    solver, although the workspace still holds the previous run's vertex."""
    print("CASE reinit", prec, flush=True)
    p = config("small_2x4")
    a = _solver(p, prec)
    a.iterate(4)
    a.reinit()
    a.iterate(2)
    b = _solver(p, prec)
    b.iterate(2)
    for f in ("sigma", "phi", "k2"):
        assert np.array_equal(H(a.get(f)), H(b.get(f))), f
    a.close()
    b.close()


# ----------------------------------------------------------- failure statuses
def _status_of(fn):
    from paper_1510_03330_amd.native import ParquetError
    try:
        fn()
    except ParquetError as e:
        return e.status
    return 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nan_sigma_set_through_the_context_is_reported(prec):
    """A NaN put into Sigma through parquet_set reaches G, the bubbles and the
    new self-energy; parquet_iterate stops after that one iteration with
    PQ_ERR_NONFINITE (the iteration is counted), and the context stays usable:
    setting a finite state again iterates normally."""
    from paper_1510_03330_amd.native import PQ_ERR_NONFINITE
    print("CASE nan sigma", prec, flush=True)
    p = config("tiny_2x2")
    s = _solver(p, prec)
    good = s.get("sigma")
    bad = good.clone()
    bad[3, 1] = complex(float("nan"), 0.0)
    s.set("sigma", bad)
    assert _status_of(lambda: s.iterate(5, 1e-8)) == PQ_ERR_NONFINITE
    assert s.last_done == 1 and s.last_stats.iteration == 1
    assert not np.isfinite(H(s.get("sigma"))).all()
    s.set("sigma", good)
    s.set("phi", torch.zeros_like(s.get("phi")))
    done, conv, st = s.iterate(2)
    assert done == 2 and np.isfinite(st.dsigma)
    s.close()


def test_single_iteration_with_zero_tolerance_and_not_converged():
    """n_iter = 1 with tol = 0: one iteration, PQ_OK, not converged. With a
    tolerance that one iteration cannot reach: PQ_ERR_NOT_CONVERGED from the C
    ABI (the Python wrapper returns converged = False and keeps the status)."""
    import ctypes
    from paper_1510_03330_amd import native as N
    p = config("tiny_2x2")
    s = _solver(p, "fp64")
    done, conv, st = s.iterate(1, 0.0)
    assert (done, conv, s.last_status) == (1, False, N.PQ_OK)
    done, conv, st = s.iterate(1, 1e-14)
    assert (done, conv, s.last_status) == (1, False, N.PQ_ERR_NOT_CONVERGED)
    d, c = ctypes.c_int32(), ctypes.c_int32()
    assert N.load().parquet_iterate(s.ctx, 2, 1e-14, None, ctypes.byref(d), ctypes.byref(c)) == N.PQ_ERR_NOT_CONVERGED
    assert (d.value, c.value) == (2, 0)
    assert N.load().parquet_iterate(s.ctx, 0, 1e-14, None, ctypes.byref(d), ctypes.byref(c)) == N.PQ_OK
    assert d.value == 0
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_unresolved_blocks_make_the_iteration_singular(prec):
    """An error tolerance no complex64 solution can meet (1e-12) flags every
    block with a nonzero vertex; with two FP64 re-solve slots per channel the
    others stay unresolved and parquet_iterate returns PQ_ERR_SINGULAR after
    the iteration, with the counts in the iteration stats. With the default
    slots every flagged block is re-solved and the iteration is OK, and its
    results match the FP64 path to complex64 storage accuracy."""
    from paper_1510_03330_amd.native import PQ_ERR_SINGULAR
    from paper_1510_03330_amd.ops import Solver
    print("CASE singular", prec, flush=True)
    p = config("tiny_2x2")
    s = Solver(p, prec, resolve_slots=2, bse_tol=1e-12)
    assert _status_of(lambda: s.iterate(3)) == PQ_ERR_SINGULAR
    st = s.last_stats
    # (the first iteration's rank-one blocks can be solved exactly in complex64)
    assert 1 <= s.last_done <= 3 and st.unresolved_blocks > 0 and st.flagged_blocks > 8
    assert st.resolved_blocks <= 8                       # two slots per channel
    s.close()
    s = Solver(p, prec, bse_tol=1e-12)
    ref = _solver(p, "fp64")
    for _ in range(2):
        done, conv, st = s.iterate(1)
        ref.iterate(1)
        assert done == 1 and st.unresolved_blocks == 0 and st.resolved_blocks == st.flagged_blocks
    assert relerr(H(s.get("phi")).astype(np.complex128), H(ref.get("phi"))) < 1e-6
    s.close()
    ref.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_vertex_field(prec):
    """PQ_FIELD_F: F = Gamma[Phi] + Phi of the current state (Eq. PA_F_G) after
    two iterations, against the oracle's remap of that Phi plus Phi; the
    stateless channel_remap gives the same F through its f_out argument."""
    print("CASE full vertex", prec, flush=True)
    p = config("small_2x4")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    s = _solver(p, prec)
    s.iterate(2)
    phi = H(s.get("phi")).astype(np.complex128)
    K1, K2 = P.kernel_functions(g, phi, p.kernel_level, p.edge_rule)
    ref = P.full_vertex(P.remap(g, phi, K1, K2, P.pa_lambda(p.U)), phi)
    tol = 1e-12 if prec == "fp64" else 2e-6
    F = s.get("f")
    assert relerr(H(F).astype(np.complex128), ref) < tol
    st = s.stage
    gam = torch.empty_like(F)
    f2 = torch.empty_like(F)
    st.channel_remap(P.pa_lambda(p.U), s.get("phi"), s.get("k1"), s.get("k2"), gam, f_out=f2)
    assert torch.equal(f2, F)
    s.close()


# ------------------------------------------------------ 4x4 lattice, Nv = 16
@pytest.fixture(scope="module")
def c2_two_iterations():
    """The oracle's first two iterations on the 4x4 lattice (U = 2, beta = 4,
    Nv = 16: 240 blocks of n = 256 per channel) from the bare-vertex start."""
    print("CASE c2 oracle", flush=True)
    p = config("c2")
    g = P.Grid(p.Lx, p.Ly, p.Nv, p.f_ext)
    st = P.init_state(p, g)
    out = [st]
    for _ in range(2):
        st = P.iterate(p, st, g)
        out.append(st)
    return p, g, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-5), ("bf16x3", 2e-4)])
def test_c2_two_iterations_match_oracle(c2_two_iterations, prec, tol):
    """Whole-iteration parity at the 4x4, Nv = 16 size (n = 256, 240 blocks):
    Sigma and Phi after each of two iterations from the bare-vertex start.
    FP64: rounding order only. Complex64 paths: complex64 storage of Phi and
    Gamma (6e-8), the BSE error below its estimate tolerance (1e-5) times the
    blocks' amplification into Sigma."""
    print("CASE c2 two iterations", prec, flush=True)
    p, g, states = c2_two_iterations
    s = _solver(p, prec)
    assert relerr(H(s.get("sigma")), states[0].sigma) < 1e-12
    for it in (1, 2):
        done, conv, stats = s.iterate(1)
        assert done == 1 and stats.unresolved_blocks == 0
        es = relerr(H(s.get("sigma")), states[it].sigma)
        ep = relerr(H(s.get("phi")).astype(np.complex128), states[it].phi)
        print(f"   iteration {it}: sigma {es:.3g}, phi {ep:.3g}, flagged {stats.flagged_blocks}, "
              f"max estimate {stats.max_err_est:.3g}", flush=True)
        assert es < tol and ep < 10 * tol, (it, es, ep)
    s.close()


@pytest.mark.parametrize("rel", [1e-6, 1e-8])
def test_relative_stopping_rule_reaches_the_fixed_point(rel):
    """parquet_iterate with tol = -rel stops once alpha dsigma / (1 - rho) is
    below rel max|Sigma| (rho the measured contraction): the result is within
    rel of the fixed point (the oracle's solution of the local problem
    converged to a change below 1e-13), and it stops earlier for the looser
    target. The contraction estimate needs seven iterations of the same state,
    so a call with n_iter = 6 cannot converge."""
    print("CASE relative stop", rel, flush=True)
    p = config("c1")
    ref = P.solve(p, max_iter=300, tol=1e-13)
    s = _solver(p, "fp64")
    done, conv, _ = s.iterate(6, -1.0)
    assert done == 6 and not conv
    s.reinit()
    done, conv, st = s.iterate(300, -rel)
    assert conv, st.dsigma
    err = relerr(H(s.get("sigma")), ref.sigma)
    print(f"   {done} iterations, distance {err:.3g}", flush=True)
    assert err < rel
    assert err > 1e-3 * rel          # it stopped near the target, not far beyond
    s.close()
