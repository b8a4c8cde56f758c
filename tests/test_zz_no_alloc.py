"""sigma_sde_no_alloc (the Schwinger-Dyson stage with its scratch in the
library's static device array) against sigma_sde with a caller workspace, on
the same inputs, through the C ABI: two calls in a row, the second on a
smaller box, so that the second call runs on the scratch the first one left
behind. Both run the same kernels, so the outputs agree bitwise."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import config, lambda_box_parts, random_phi, random_sigma

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(name, prec, seed):
    from paper_1510_03330_amd.ops import Stage
    p = config(name)
    st = Stage(p, prec)
    d = st.d
    sig = random_sigma(d.Nve, d.Nk, seed=seed, scale=0.1)
    sig = 0.5 * (sig + np.conj(sig[::-1]))
    g = torch.empty(st.g_shape, dtype=torch.complex128, device=DEV)
    mu = torch.empty(1, dtype=torch.float64, device=DEV)
    st.dyson_update(torch.from_numpy(sig).to(DEV), g, mu)
    phi = torch.from_numpy(random_phi(d.Nq, d.n, seed=seed + 1, scale=0.2)).to(device=DEV, dtype=st.vdtype)
    k1 = torch.empty(st.k1_shape, dtype=torch.complex128, device=DEV)
    k2 = torch.empty(st.k2_shape, dtype=torch.complex128, device=DEV)
    st.kernel_extract(phi, k1, k2)
    return st, phi, k1, k2, g, mu


def _call_no_alloc(st, phi, k1, k2, g, mu, out, lam_box=None):
    from paper_1510_03330_amd import native as N
    lb = ctypes.c_void_p(0) if lam_box is None else ctypes.c_void_p(lam_box.data_ptr())
    status = N.load().sigma_sde_no_alloc(ctypes.byref(st.pp), ctypes.c_void_p(phi.data_ptr()),
                                         ctypes.c_void_p(k1.data_ptr()), ctypes.c_void_p(k2.data_ptr()), lb,
                                         ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    N.check(status)


@pytest.mark.parametrize("cases", [(("c2", "fp32", 11, False), ("tiny_2x2", "fp64", 21, True)),
                                   (("small_2x4", "fp64", 31, True), ("tiny_local", "fp32", 41, False))])
def test_no_alloc_sigma_matches_workspace_entry_point(cases):
    print("CASE no-alloc", cases, flush=True)
    for name, prec, seed, with_lam in cases:
        st, phi, k1, k2, g, mu = _inputs(name, prec, seed)
        lam = None
        if with_lam:
            a, b = lambda_box_parts(st.d.Nv, seed=seed + 2, scale=0.3)
            U = st.model.U
            lam = torch.from_numpy(np.stack([U + a, -U + b, np.full_like(a, 2 * U), np.zeros_like(a)])).to(DEV)
        ref = torch.empty(st.sigma_shape, dtype=torch.complex128, device=DEV)
        st.sigma_sde(phi, k1, k2, g, mu, ref, lam_box=lam)
        got = torch.full(st.sigma_shape, complex(float("nan"), 0.0), dtype=torch.complex128, device=DEV)
        _call_no_alloc(st, phi, k1, k2, g, mu, got, lam)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(got)).all()
        assert torch.equal(got, ref), (name, float((got - ref).abs().max()))
        del phi
        torch.cuda.empty_cache()
