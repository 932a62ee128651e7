"""The ill-conditioned (hard) variant: eigenvalue sums down to 0.05.

Per-mode real parts are drawn from U[0.05/3, 2] with one 1x1 diagonal entry
per mode pinned to 0.05/3, so the smallest eigenvalue sum is exactly 0.05 and
the operator's condition number reaches ~1e5..1e6.  Any FP64 solver then has a
forward error of order kappa * u, above 1e-12, so the reference is the oracle
in x87 long double (u ~ 5.4e-20) and the bound is stated in terms of a
condition estimate (Hager/Higham, tests/condest.py, pinned to the exact
condition number of the assembled operator in test_condest.py).  The FP64
oracle itself, which solves every coupled 2x2 / 4x4 / 8x8 tuple by Gaussian
elimination with partial pivoting, gives the yardstick an FP64 solver reaches
on the same data.  The benign variant (sums in [3, 6]) meets 1e-12.
"""
import numpy as np
import pytest

import oracle
import tt_inputs as ti
from condest import cond1_estimate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def tt():
    import paper_1905_09539_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n", [24, 48, 96])
def test_hard_variant_vs_long_double(n):
    shape = (n, n, n)
    p = ti.laplace_tri(shape, seed=3, bumps="every8", hard_sum=0.05)
    print(f"case hard n={n}", flush=True)
    X = tt().solve_tri([dev(t) for t in p["T"]], dev(p["B"]))
    torch.cuda.synchronize()
    Xg = X.cpu().numpy()
    Xld = oracle.lap_solve(p["T"], p["B"], precision="ld")
    X64 = oracle.lap_solve(p["T"], p["B"])
    kappa = cond1_estimate(p["T"], shape)
    e_gpu, e_o64 = rel(Xg, Xld), rel(X64, Xld)
    print(f"hard n={n}: kappa_1 ~ {kappa:.3e}, kappa*u {kappa * U64:.3e}, GPU error {e_gpu:.3e}, "
          f"FP64 oracle error {e_o64:.3e}", flush=True)
    assert kappa > 1e4  # the variant really is ill-conditioned
    assert e_gpu <= 8 * kappa * U64
    # within a small factor of what GEPP-based FP64 substitution reaches
    assert e_gpu <= 10 * e_o64 + 1e-15


@pytest.mark.parametrize("n", [24, 48])
def test_hard_coupled_tuples_vs_long_double(n):
    """The smallest eigenvalue sum (0.05) reached by coupled tuples too: the
    8-unknown tuple of the first 2x2 blocks of the three modes (eigenvalue
    0.05 + i (0.2 + 0.3 - 0.5)) and 4-unknown tuples of two such blocks with
    a pinned 1x1 entry.  Same bounds as the 1x1 case: kappa-based against the
    long-double oracle, and within a small factor of the FP64 oracle, which
    solves every tuple by Gaussian elimination with partial pivoting."""
    shape = (n, n, n)
    p = ti.laplace_tri(shape, seed=3, bumps="every8", hard_sum=0.05, hard_coupled=True)
    print(f"case hard coupled n={n}", flush=True)
    X = tt().solve_tri([dev(t) for t in p["T"]], dev(p["B"]))
    torch.cuda.synchronize()
    Xg = X.cpu().numpy()
    Xld = oracle.lap_solve(p["T"], p["B"], precision="ld")
    X64 = oracle.lap_solve(p["T"], p["B"])
    kappa = cond1_estimate(p["T"], shape)
    e_gpu, e_o64 = rel(Xg, Xld), rel(X64, Xld)
    print(f"hard coupled n={n}: kappa_1 ~ {kappa:.3e}, GPU error {e_gpu:.3e}, FP64 oracle error {e_o64:.3e}",
          flush=True)
    assert kappa > 1e5
    assert e_gpu <= 8 * kappa * U64
    assert e_gpu <= 10 * e_o64 + 1e-15


@pytest.mark.parametrize("n", [24, 96])
def test_benign_variant_vs_long_double(n):
    p = ti.laplace_tri((n, n, n), seed=3, bumps="every8")
    print(f"case benign n={n}", flush=True)
    X = tt().solve_tri([dev(t) for t in p["T"]], dev(p["B"]))
    torch.cuda.synchronize()
    e = rel(X.cpu().numpy(), oracle.lap_solve(p["T"], p["B"], precision="ld"))
    print(f"benign n={n}: GPU error vs long double {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hard_variant_mixed_precision(prec):
    """FP32-MFMA (and three-term BF16) refinement on the hard variant:
    kappa * u_fp32 ~ 0.06 < 1, so refinement still contracts (slowly); the
    refined X is compared with the long-double oracle against the same
    kappa-based bound as FP64."""
    n = 48
    p = ti.laplace_tri((n, n, n), seed=3, bumps="every8", hard_sum=0.05)
    info = {}
    X = torch.empty_like(dev(p["B"]))
    print("case hard mp", prec, flush=True)
    code = {"fp32": tt().TT_MP_FP32, "bf16": tt().TT_MP_BF16}[prec]
    try:
        tt().solve_tri([dev(t) for t in p["T"]], dev(p["B"]), X=X, prec=code, tol=1e-13,
                       max_iter=30, info=info)
    except tt().TTError as e:  # refinement may stall at the FP64 accuracy level
        assert e.code == tt().TT_ENOTCONV
    torch.cuda.synchronize()
    Xld = oracle.lap_solve(p["T"], p["B"], precision="ld")
    kappa = cond1_estimate(p["T"], (n, n, n))
    e = rel(X.cpu().numpy(), Xld)
    print(f"hard mp {prec}: {info.get('iterations')} iterations, ratio {info.get('ratio'):.3e}, "
          f"error {e:.3e}, kappa*u {kappa * U64:.3e}", flush=True)
    assert e <= 8 * kappa * U64
