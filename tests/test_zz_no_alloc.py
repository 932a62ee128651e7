"""The allocation-free entry point solve_tri_tensor_noalloc, called through
the C ABI, against solve_tri_tensor on the same inputs: two calls in a row,
the second with a smaller problem (the scratch array keeps the first call's
contents, which must not leak into the second), plus the pair form and the
size limit."""
import ctypes

import numpy as np
import pytest

import tt_inputs as ti

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def tt():
    import paper_1905_09539_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    torch.cuda.synchronize()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def solve_noalloc_abi(T, B, X, C=None):
    m = tt()
    L = m.lib()
    tp = m._ptr_array([t.data_ptr() for t in T])
    cp = m._ptr_array([c.data_ptr() for c in C]) if C is not None else None
    o = m._opts()
    rc = L.solve_tri_tensor_noalloc(B.dim(), m._shape(B.shape), tp, cp, ctypes.c_void_p(B.data_ptr()),
                                    ctypes.c_void_p(X.data_ptr()), ctypes.byref(o))
    return rc


@pytest.mark.parametrize("first,second", [((96, 80, 112), (33, 17, 40)), ((64, 64, 64), (16, 16, 16)),
                                          ((24, 20, 18, 22), (9, 7, 8, 6))])
def test_noalloc_matches_allocating_entry_point(first, second):
    for k, shape in enumerate((first, second)):
        p = ti.laplace_tri(shape, seed=40 + k, bumps="every8" if k == 0 else "random")
        T = [dev(t) for t in p["T"]]
        B = dev(p["B"])
        print(f"case noalloc call {k}: shape {shape}", flush=True)
        Xref = tt().solve_tri(T, B)
        X = torch.full_like(B, float("nan"))
        rc = solve_noalloc_abi(T, B, X)
        assert rc == 0, tt().lib().tt_last_error()
        e = rel(X, Xref)
        print(f"noalloc {shape}: relative difference to solve_tri_tensor {e:.3e}", flush=True)
        assert e <= 1e-12


def test_noalloc_pair_form_and_in_place():
    shape = (30, 26, 34)
    p = ti.pair_tri(shape, seed=44)
    A = [dev(a) for a in p["A"]]
    C = [dev(c) for c in p["C"]]
    B = dev(p["B"])
    print("case noalloc pair", flush=True)
    Xref = tt().solve_tri(A, B, C=C)
    X = torch.empty_like(B)
    assert solve_noalloc_abi(A, B, X, C=C) == 0, tt().lib().tt_last_error()
    assert rel(X, Xref) <= 1e-12
    q = ti.laplace_tri(shape, seed=45, bumps="every8")
    T = [dev(t) for t in q["T"]]
    Bq = dev(q["B"])
    Xq = tt().solve_tri(T, Bq)
    print("case noalloc in place", flush=True)
    assert solve_noalloc_abi(T, Bq, Bq) == 0, tt().lib().tt_last_error()
    assert rel(Bq, Xq) <= 1e-12


def test_noalloc_rejects_too_large():
    shape = (200, 200, 200)  # two accumulators alone need 128 MB
    T = [torch.eye(n, dtype=torch.float64, device="cuda") for n in shape]
    B = torch.ones(shape, dtype=torch.float64, device="cuda")
    X = torch.empty_like(B)
    print("case noalloc too large", flush=True)
    rc = solve_noalloc_abi(T, B, X)
    assert rc == tt().TT_EINVAL
    assert b"allocation-free" in tt().lib().tt_last_error()
