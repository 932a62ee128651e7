"""Second operator class (Sec. 3, eq. (3.1)) on the GPU against the oracle:
X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d = B.

Triangular coefficients (orders 1 to 4, every 2x2-block pattern, ragged
shapes, thin modes) against the oracle's direct element-wise solve (no C^{-1}
reduction, no partial products); dense coefficients (Algorithm 4) against the
oracle through the generator's exact QZ and Schur factors; a 128^3 residual
of the operator evaluated with torch; the shifted Kronecker case (eq. (1.6))
and a singular pencil."""
import numpy as np
import pytest

import oracle
import tt_inputs as ti

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def tt():
    import paper_1905_09539_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape,bumps,seed", [
    ((20, 18, 22), "every8", 1), ((33, 17, 40), "random", 2), ((9, 7, 8), "aligned", 3),
    ((16, 16, 16), "every8", 4), ((5, 1, 30), "random", 5), ((41, 9, 3), "none", 6),
    ((10, 9, 8, 7), "every8", 7), ((12, 12, 12, 12), "aligned", 8), ((7, 13, 5, 9), "random", 9),
    ((40, 30), "every8", 10), ((25,), "random", 11),
])
def test_gsylv_tri_matches_oracle(shape, bumps, seed):
    p = ti.gsylv_tri(shape, seed=seed, bumps=bumps)
    print(f"case gsylv tri {shape} {bumps}", flush=True)
    X = tt().solve_gsylv([dev(a) for a in p["A"]], dev(p["C"]), dev(p["B"]))
    torch.cuda.synchronize()
    Xo = oracle.gsylv_solve(p["A"], p["C"], p["B"])
    e = rel(X.cpu().numpy(), Xo)
    print(f"gsylv {shape}: {e:.3e}", flush=True)
    assert e <= TOL


@pytest.mark.parametrize("nmin", [2, 3, 5, 8])
def test_gsylv_leaf_sizes(nmin):
    shape = (26, 23, 19)
    p = ti.gsylv_tri(shape, seed=12, bumps="random")
    print(f"case gsylv nmin {nmin}", flush=True)
    X = tt().solve_gsylv([dev(a) for a in p["A"]], dev(p["C"]), dev(p["B"]), nmin=nmin)
    torch.cuda.synchronize()
    assert rel(X.cpu().numpy(), oracle.gsylv_solve(p["A"], p["C"], p["B"])) <= TOL


@pytest.mark.parametrize("shape", [(24, 20, 18), (10, 9, 8, 7), (30, 26)])
def test_gsylv_dense_matches_oracle(shape):
    p = ti.gsylv_dense(shape, seed=13, bumps="every8")
    print(f"case gsylv dense {shape}", flush=True)
    X = tt().solve_gsylv_general(p["A"], p["C"], dev(p["B"]))
    torch.cuda.synchronize()
    Xo = oracle.gsylv_dense_solve_with_factors(p["Q"], p["S"], p["T"], p["Z"], p["U"], p["Tq"], p["B"])
    e = rel(X.cpu().numpy(), Xo)
    print(f"gsylv dense {shape}: {e:.3e}", flush=True)
    assert e <= TOL


def test_gsylv_in_place_and_plan_reuse():
    shape = (21, 19, 17)
    p = ti.gsylv_tri(shape, seed=14, bumps="every8")
    A = [dev(a) for a in p["A"]]
    C = dev(p["C"])
    plan = tt().Plan(A, shape, C=C, gsylv=True)
    Xo = oracle.gsylv_solve(p["A"], p["C"], p["B"])
    print("case gsylv plan reuse / in place", flush=True)
    for _ in range(2):
        B = dev(p["B"])
        plan.solve(B, B)  # in place
        plan.status()
        assert rel(B.cpu().numpy(), Xo) <= TOL
    plan.close()


def test_gsylv_128_residual_and_corner():
    shape = (128, 128, 128)
    p = ti.gsylv_tri(shape, seed=15, bumps="every8")
    A = [dev(a) for a in p["A"]]
    C = dev(p["C"])
    B = dev(p["B"])
    print("case gsylv 128^3", flush=True)
    X = tt().solve_gsylv(A, C, B)
    torch.cuda.synchronize()
    Y = torch.movedim(torch.tensordot(A[0], X, dims=([1], [0])), 0, 0)
    Z = torch.tensordot(C, X, dims=([1], [0]))
    Z = torch.movedim(torch.tensordot(A[1], Z, dims=([1], [1])), 0, 1)
    Z = torch.movedim(torch.tensordot(A[2], Z, dims=([1], [2])), 0, 2)
    r = float(torch.linalg.vector_norm(Y + Z - B) / torch.linalg.vector_norm(B))
    print(f"gsylv 128^3 residual {r:.3e}", flush=True)
    assert r <= 1e-13
    # the far corner box depends only on itself when no box edge cuts a
    # 2x2 block (C is upper triangular, the A_mu quasi-triangular)
    lo = [96] * 3
    for mu in range(3):
        while lo[mu] > 0 and p["A"][mu][lo[mu], lo[mu] - 1] != 0.0:
            lo[mu] -= 1
    sl = tuple(slice(l, None) for l in lo)
    Xo = oracle.gsylv_solve([np.ascontiguousarray(a[l:, l:]) for a, l in zip(p["A"], lo)],
                            np.ascontiguousarray(p["C"][lo[0]:, lo[0]:]), np.ascontiguousarray(p["B"][sl]))
    e = rel(X.cpu().numpy()[sl], Xo)
    print(f"gsylv 128^3 corner: {e:.3e}", flush=True)
    assert e <= TOL


def test_gsylv_96x4_residual_and_corner():
    """The d = 4 benchmark workload (96^4, leaf edge 5): residual of the whole
    solve (torch) and the self-contained far corner [76, 96)^4 against the
    oracle's direct solve."""
    shape = (96, 96, 96, 96)
    p = ti.gsylv_tri(shape, seed=17, bumps="every8")
    A = [dev(a) for a in p["A"]]
    C = dev(p["C"])
    B = dev(p["B"])
    print("case gsylv 96^4", flush=True)
    X = tt().solve_gsylv(A, C, B)
    torch.cuda.synchronize()
    R = B - torch.tensordot(A[0], X, dims=([1], [0]))
    Z = X
    for nu in range(4):
        Z = torch.movedim(torch.tensordot(C if nu == 0 else A[nu], Z, dims=([1], [nu])), 0, nu)
    R -= Z
    r = float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))
    print(f"gsylv 96^4 residual {r:.3e}", flush=True)
    assert r <= 1e-13
    lo = [76] * 4
    for mu in range(4):
        while lo[mu] > 0 and p["A"][mu][lo[mu], lo[mu] - 1] != 0.0:
            lo[mu] -= 1
    sl = tuple(slice(l, None) for l in lo)
    Xo = oracle.gsylv_solve([np.ascontiguousarray(a[l:, l:]) for a, l in zip(p["A"], lo)],
                            np.ascontiguousarray(p["C"][lo[0]:, lo[0]:]), np.ascontiguousarray(p["B"][sl]))
    e = rel(X.cpu().numpy()[sl], Xo)
    print(f"gsylv 96^4 corner: {e:.3e}", flush=True)
    assert e <= TOL


def test_gsylv_shifted_kronecker():
    """Eq. (1.6): A_1 = -lambda I, operator A_d (x) .. (x) A_2 (x) C - lambda I."""
    shape = (18, 15, 12)
    p = ti.gsylv_tri(shape, seed=16, bumps="every8")
    A = [-0.3 * np.eye(shape[0])] + p["A"][1:]
    print("case gsylv shifted", flush=True)
    X = tt().solve_gsylv([dev(a) for a in A], dev(p["C"]), dev(p["B"]))
    torch.cuda.synchronize()
    assert rel(X.cpu().numpy(), oracle.gsylv_solve(A, p["C"], p["B"])) <= TOL


def test_gsylv_singular_reported():
    n = 6
    C = np.triu(np.ones((n, n)))
    A = [-C, np.eye(5), np.eye(4)]
    print("case gsylv singular", flush=True)
    with pytest.raises(tt().TTError) as e:
        tt().solve_gsylv([dev(a) for a in A], dev(C), dev(np.ones((n, 5, 4))))
    assert e.value.code == tt().TT_ESINGULAR
