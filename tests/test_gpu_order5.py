"""Order d = 5 on the GPU (Sec. 2.4 experiments' highest order): the two
adjacent modes with the smallest product of sizes are merged (Algorithm 3,
perfect shuffle + 4x4 real Schur forms, tests/test_merge.py) and the merged
4-mode equation runs the order-4 path.  Compared with the oracle's direct
order-5 block back-substitution (which never merges)."""
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
    ((6, 5, 7, 4, 6), "every8", 1), ((8, 8, 8, 8, 8), "aligned", 2), ((5, 6, 4, 7, 3), "random", 3),
    ((16, 16, 16, 16, 16), "every8", 4), ((9, 1, 10, 3, 12), "aligned", 5), ((20, 12, 4, 4, 9), "random", 6),
])
def test_order5_laplace_matches_oracle(shape, bumps, seed):
    p = ti.laplace_tri(shape, seed=seed, bumps=bumps)
    print(f"case order5 {shape} {bumps}", flush=True)
    X = tt().solve_tri([dev(t) for t in p["T"]], dev(p["B"]))
    torch.cuda.synchronize()
    Xo = oracle.lap_solve(p["T"], p["B"])
    e = rel(X.cpu().numpy(), Xo)
    print(f"order5 {shape}: {e:.3e}", flush=True)
    assert e <= TOL


def test_order5_pair_matches_oracle():
    shape = (5, 4, 6, 5, 4)
    p = ti.pair_tri(shape, seed=7, bumps="aligned")
    print("case order5 pair", flush=True)
    X = tt().solve_tri([dev(a) for a in p["A"]], dev(p["B"]), C=[dev(c) for c in p["C"]])
    torch.cuda.synchronize()
    e = rel(X.cpu().numpy(), oracle.pair_solve(p["A"], p["C"], p["B"], method="direct"))
    print(f"order5 pair: {e:.3e}", flush=True)
    assert e <= TOL


def test_order5_dense_matches_oracle():
    shape = (7, 6, 5, 6, 4)
    p = ti.laplace_dense(shape, seed=8, bumps="aligned")
    print("case order5 dense", flush=True)
    X = tt().solve_general(p["A"], dev(p["B"]))
    torch.cuda.synchronize()
    e = rel(X.cpu().numpy(), oracle.dense_solve_with_factors(p["Q"], p["T"], p["B"]))
    print(f"order5 dense: {e:.3e}", flush=True)
    assert e <= TOL


def test_order5_plan_reuse_in_place_and_empty():
    shape = (6, 7, 5, 6, 5)
    p = ti.laplace_tri(shape, seed=9, bumps="every8")
    T = [dev(t) for t in p["T"]]
    plan = tt().Plan(T, shape)
    Xo = oracle.lap_solve(p["T"], p["B"])
    print("case order5 plan reuse", flush=True)
    for _ in range(2):
        B = dev(p["B"])
        plan.solve(B, B)
        plan.status()
        assert rel(B.cpu().numpy(), Xo) <= TOL
    plan.close()
    z = (4, 0, 3, 2, 2)
    q = ti.laplace_tri(z, seed=10, bumps="none")
    X = tt().solve_tri([dev(t) for t in q["T"]], dev(q["B"]))
    assert X.numel() == 0


def test_order5_40_residual_and_corner():
    """The order-5 benchmark workload (40^5, modes 3 and 4 merged into 1600):
    residual of the whole solve (torch) and the self-contained far corner
    [30, 40)^5 against the oracle's order-5 substitution."""
    shape = (40, 40, 40, 40, 40)
    p = ti.laplace_tri(shape, seed=8, bumps="every8")
    T = [dev(t) for t in p["T"]]
    B = dev(p["B"])
    print("case order5 40^5", flush=True)
    X = tt().solve_tri(T, B)
    torch.cuda.synchronize()
    R = B.clone()
    for mu in range(5):
        R -= torch.movedim(torch.tensordot(T[mu], X, dims=([1], [mu])), 0, mu)
    r = float(torch.linalg.vector_norm(R) / torch.linalg.vector_norm(B))
    print(f"order5 40^5 residual {r:.3e}", flush=True)
    assert r <= 1e-13
    lo = [30] * 5
    for mu in range(5):
        while lo[mu] > 0 and p["T"][mu][lo[mu], lo[mu] - 1] != 0.0:
            lo[mu] -= 1
    sl = tuple(slice(l, None) for l in lo)
    Xo = oracle.lap_solve([np.ascontiguousarray(t[l:, l:]) for t, l in zip(p["T"], lo)],
                          np.ascontiguousarray(p["B"][sl]))
    e = rel(X.cpu().numpy()[sl], Xo)
    print(f"order5 40^5 corner: {e:.3e}", flush=True)
    assert e <= TOL
