"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, its struct layouts agree with the ctypes binding, and host-side
validation rejects bad arguments before anything reaches a device."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1510_03330_amd import native as N
from workloads import config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parquet.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\*?\s+\*?([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = N.load()
    declared = _declared_functions()
    assert len(declared) >= 18
    assert sorted(declared) == sorted(N.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "parquet.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pq_params), sizeof(pq_dims), sizeof(pq_iter_stats),
         sizeof(pq_bse_block_stats), offsetof(pq_params, U), offsetof(pq_dims, vertex_elems));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(N.PqParams)
    assert vals[1] == ctypes.sizeof(N.PqDims)
    assert vals[2] == ctypes.sizeof(N.PqIterStats)
    assert vals[3] == ctypes.sizeof(N.PqBseBlockStats)
    assert vals[4] == N.PqParams.U.offset
    assert vals[5] == N.PqDims.vertex_elems.offset


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "tiny_2x2", "small_2x4"])
def test_dims_from_params(name):
    p = config(name)
    d = N.dims(N.make_params(p, "fp64"))
    Nk = p.Lx * p.Ly
    assert (d.Nk, d.Nv, d.NW, d.n, d.Nq) == (Nk, p.Nv, p.Nv - 1, Nk * p.Nv, Nk * (p.Nv - 1))
    assert d.Nve == p.f_ext * p.Nv and d.NG == 2 * p.f_ext * p.Nv
    assert d.vertex_elems == d.Nq * d.n * d.n


@pytest.mark.parametrize("bad", [dict(Nv=7), dict(Nv=0), dict(f_ext=0), dict(kernel_level=3),
                                 dict(alpha=0.0), dict(alpha=1.5), dict(beta=-1.0), dict(Lx=9, Ly=9),
                                 dict(edge_rule=2), dict(mu_mode=4), dict(regulation=0), dict(regulation=2),
                                 dict(regulation=0, f_ext=2)])
def test_invalid_params_are_rejected_on_the_host(bad):
    p = config("tiny_2x2", **bad)
    pp = N.make_params(p, "fp64")
    d = N.PqDims()
    st = N.load().pq_dims_from_params(ctypes.byref(pp), ctypes.byref(d))
    assert st == N.PQ_ERR_ARG
    assert N.load().parquet_last_error()


def test_precision_storage_mismatch_is_rejected():
    pp = N.make_params(config("tiny_2x2"), "fp64")
    pp.storage = N.PQ_STORE_C64
    d = N.PqDims()
    assert N.load().pq_dims_from_params(ctypes.byref(pp), ctypes.byref(d)) == N.PQ_ERR_ARG


def test_null_pointers_are_rejected_before_enqueue():
    pp = N.make_params(config("tiny_2x2"), "fp64")
    lib = N.load()
    assert lib.bubble_build(ctypes.byref(pp), None, None, None, None) == N.PQ_ERR_ARG
    assert lib.channel_remap(ctypes.byref(pp), None, None, None, None, None, None, None, None) == N.PQ_ERR_ARG
    assert lib.parquet_iterate(None, 1, 0.0, None, None, None) == N.PQ_ERR_ARG
    # workspace too small is reported, not enqueued
    fake = ctypes.c_void_p(0x1000)
    st = lib.bse_solve(ctypes.byref(pp), 0, 0, fake, fake, ctypes.c_void_p(0x2000), 1.0, None, fake,
                       ctypes.c_size_t(16), None)
    assert st == N.PQ_ERR_NOMEM
    # aliasing input/output is rejected
    st = lib.bse_solve(ctypes.byref(pp), 0, 0, fake, fake, fake, 1.0, None, fake, ctypes.c_size_t(16), None)
    assert st == N.PQ_ERR_ARG


def test_workspace_queries_scale_with_storage():
    p = config("c3")
    b64 = ctypes.c_size_t()
    b32 = ctypes.c_size_t()
    lib = N.load()
    N.check(lib.parquet_query_workspace(ctypes.byref(N.make_params(p, "fp64")), ctypes.byref(b64)))
    N.check(lib.parquet_query_workspace(ctypes.byref(N.make_params(p, "fp32")), ctypes.byref(b32)))
    # vertex arrays dominate: complex128 needs about twice complex64, and both fit 288 GB
    assert 1.8 < b64.value / b32.value < 2.2
    assert b64.value < 250e9


def test_precision_storage_pairs():
    """BF16x3 and FP32 eliminate complex64 storage, FP64 complex128; other
    pairs and unknown precisions are rejected on the host."""
    p = config("c3")
    lib = N.load()
    d = N.PqDims()
    for prec in ("fp64", "fp32", "bf16x3"):
        pp = N.make_params(p, prec)
        assert pp.precision == N.PRECISIONS[prec]
        N.check(lib.pq_dims_from_params(ctypes.byref(pp), ctypes.byref(d)))
    b32, b3 = ctypes.c_size_t(), ctypes.c_size_t()
    N.check(lib.parquet_query_workspace(ctypes.byref(N.make_params(p, "fp32")), ctypes.byref(b32)))
    N.check(lib.parquet_query_workspace(ctypes.byref(N.make_params(p, "bf16x3")), ctypes.byref(b3)))
    assert b32.value == b3.value
    bad = N.make_params(p, "bf16x3")
    bad.storage = N.PQ_STORE_C128
    assert lib.pq_dims_from_params(ctypes.byref(bad), ctypes.byref(d)) == N.PQ_ERR_ARG
    bad = N.make_params(p, "fp32")
    bad.precision = 3
    assert lib.pq_dims_from_params(ctypes.byref(bad), ctypes.byref(d)) == N.PQ_ERR_ARG
    with pytest.raises(ValueError):
        N.make_params(p, "fp16")


def test_mlp_widths_are_checked_on_the_host():
    """mlp_param_count accepts 1..16 layers of widths 1..4194240 (65535 GEMM
    tiles of 64) and counts W and b of every layer; anything else is ERR_ARG."""
    lib = N.load()
    cnt = ctypes.c_size_t()

    def count(widths):
        arr = (ctypes.c_int32 * len(widths))(*widths)
        return lib.mlp_param_count(arr, len(widths) - 1, ctypes.byref(cnt))

    assert count([2, 512, 512, 512, 494464]) == N.PQ_OK
    assert cnt.value == (2 * 512 + 512) + 2 * (512 * 512 + 512) + (512 * 494464 + 494464)
    assert count([3, 4194240]) == N.PQ_OK and cnt.value == 3 * 4194240 + 4194240
    assert count([3, 4194241]) == N.PQ_ERR_ARG
    assert count([0, 4]) == N.PQ_ERR_ARG
    assert count([4]) == N.PQ_ERR_ARG                       # no layer
    assert count([1] * 18) == N.PQ_ERR_ARG                  # 17 layers


def test_mlp_basis_arguments_are_checked_on_the_host():
    """The factorised head's calls check their sizes and pointers before
    touching the device: rows in 1..4096, a coordinate stride of at least
    rows, non-null buffers; the workspace grows with the row count."""
    lib = N.load()
    b1, b2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.mlp_basis_workspace(8, ctypes.byref(b1)) == N.PQ_OK
    assert lib.mlp_basis_workspace(64, ctypes.byref(b2)) == N.PQ_OK and b2.value > b1.value
    assert lib.mlp_basis_workspace(0, ctypes.byref(b1)) == N.PQ_ERR_ARG
    assert lib.mlp_basis_workspace(4097, ctypes.byref(b1)) == N.PQ_ERR_ARG
    f = ctypes.c_void_p(0x1000)
    assert lib.mlp_basis(f, 8, 100, f, f, 7, f, f, None) == N.PQ_ERR_ARG          # ld < rows
    assert lib.mlp_basis(f, 8, 0, f, f, 8, f, f, None) == N.PQ_ERR_ARG            # empty rows
    assert lib.mlp_basis(None, 8, 100, f, f, 8, f, f, None) == N.PQ_ERR_ARG
    assert lib.mlp_expand(f, 0, 100, f, f, f, f, None) == N.PQ_ERR_ARG
    assert lib.mlp_expand(f, 8, 100, f, None, f, f, None) == N.PQ_ERR_ARG
    assert lib.parquet_warm_start(None, f, f, None) == N.PQ_ERR_ARG


def test_no_alloc_entry_point_rejects_boxes_beyond_its_scratch():
    """sigma_sde_no_alloc checks the scratch its parameters need against the
    64 MiB static array before touching the device: an 8x8 lattice with
    Nv = 64 and f = 4 needs more and gets PQ_ERR_NOMEM; null pointers give
    PQ_ERR_ARG."""
    lib = N.load()
    big = N.make_params(config("c3", Nv=64, f_ext=4), "fp32")
    ws = ctypes.c_size_t()
    N.check(lib.sigma_sde_workspace(ctypes.byref(big), ctypes.byref(ws)))
    assert ws.value > 64 << 20
    fake = ctypes.c_void_p(0x1000)
    assert lib.sigma_sde_no_alloc(ctypes.byref(big), fake, fake, fake, None, fake, fake, fake, None) == N.PQ_ERR_NOMEM
    assert b"static scratch" in lib.parquet_last_error()
    small = N.make_params(config("c3"), "fp32")
    N.check(lib.sigma_sde_workspace(ctypes.byref(small), ctypes.byref(ws)))
    assert ws.value < 64 << 20
    assert lib.sigma_sde_no_alloc(ctypes.byref(small), None, fake, fake, None, fake, fake, fake, None) == N.PQ_ERR_ARG


def test_batch_arguments_are_checked_on_the_host():
    """The batched solver's sizes are validated before anything touches the
    device: instances of different boxes, precisions or mixing are refused,
    as are batches above 16384 BSE blocks per channel; the workspace grows
    with the instance count; bse_tile is 0 or 1."""
    lib = N.load()

    def query(ps, prec="fp32"):
        arr = (N.PqParams * len(ps))(*[N.make_params(p, prec) for p in ps])
        b = ctypes.c_size_t()
        return lib.parquet_batch_query_workspace(arr, len(ps), ctypes.byref(b)), b.value

    p = config("small_2x4")
    st1, b1 = query([p])
    st3, b3 = query([p, p.replace(U=2.0, beta=3.0, filling=0.95), p.replace(tp=-0.1, kernel_level=1)])
    assert st1 == N.PQ_OK and st3 == N.PQ_OK and b3 > 2 * b1
    assert query([p, p.replace(Nv=8)])[0] == N.PQ_ERR_ARG
    assert query([p, p.replace(alpha=0.3)])[0] == N.PQ_ERR_ARG
    big = config("c2", Nv=32)                           # Nq = 496: 34 instances exceed 16384 blocks
    assert query([big] * 33)[0] == N.PQ_OK
    assert query([big] * 34)[0] == N.PQ_ERR_ARG
    assert b"16384" in lib.parquet_last_error()
    assert lib.parquet_batch_query_workspace(None, 1, ctypes.byref(ctypes.c_size_t())) == N.PQ_ERR_ARG
    bad = N.make_params(p, "fp32", bse_tile=2)
    assert lib.pq_dims_from_params(ctypes.byref(bad), ctypes.byref(N.PqDims())) == N.PQ_ERR_ARG
    assert lib.parquet_batch_iterate(None, 1, 0.0, 0.0, None) == N.PQ_ERR_ARG
    assert lib.parquet_batch_destroy(None) == N.PQ_OK
