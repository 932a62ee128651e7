"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each check uses a dense
Kronecker solve, a closed form, a textbook routine (SciPy's Bartels-Stewart
Sylvester solver), an identity, or a brute-force count.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import tt_inputs as ti
from kron import laplace_dense, pair_dense, unvecF, vecF

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------- fixtures --

def test_golden_merged_pattern_eq2_9():
    """The dense-operator convention used below reproduces the sparsity pattern
    the paper prints for I (x) A_1 + A_2 (x) I (Sec. 2.3, eq. (2.9))."""
    rows = {"A1": [], "A2": [], "M": []}
    with open(os.path.join(HERE, "golden", "merged_pattern_eq2_9.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tag, *vals = line.split()
            rows[tag].append([v == "x" for v in vals])
    P1, P2, PM = (np.array(rows[k]) for k in ("A1", "A2", "M"))
    g = np.random.default_rng(5)
    A1 = np.where(P1, g.uniform(1, 2, P1.shape), 0.0)
    A2 = np.where(P2, g.uniform(1, 2, P2.shape), 0.0)
    # d = 2 operator of eq. (1.4) in the paper's vec order: A_2 (x) I + I (x) A_1
    M = laplace_dense([A1, A2])
    assert M.shape == PM.shape == (12, 12)
    assert np.array_equal(M != 0, PM)


# ------------------------------------------------------- Laplace-like solve --

@pytest.mark.parametrize("shape,bumps", [
    ((8, 8, 8), "every8"), ((8, 8, 8), "aligned"), ((7, 5, 6), "random"),
    ((8, 3, 8), "aligned"), ((5, 5, 5, 5), "aligned"), ((4, 5, 3, 5), "random"),
    ((9, 7), "random"), ((6,), "aligned"), ((1, 1, 1), "none"), ((2, 2, 2), "aligned"),
])
def test_lap_solve_vs_dense_kronecker(shape, bumps):
    p = ti.laplace_tri(shape, seed=11, bumps=bumps)
    T, B = p["T"], p["B"]
    X = oracle.lap_solve(T, B)
    A = laplace_dense(T)
    Xd = unvecF(np.linalg.solve(A, vecF(B)), B.shape)
    assert rel(X, Xd) < 1e-13
    # the long double instantiation agrees too
    assert rel(oracle.lap_solve(T, B, precision="ld"), Xd) < 1e-13


def test_lap_solve_random_bumps_many_seeds():
    for seed in range(12):
        shape = tuple(np.random.default_rng(seed).integers(1, 8, 3))
        p = ti.laplace_tri(shape, seed=seed, bumps="random")
        X = oracle.lap_solve(p["T"], p["B"])
        Xd = unvecF(np.linalg.solve(laplace_dense(p["T"]), vecF(p["B"])), p["B"].shape)
        assert rel(X, Xd) < 1e-13, seed


def test_lap_solve_transposed_vs_dense():
    p = ti.laplace_tri((6, 7, 5), seed=3, bumps="random")
    L = oracle.lap_solve(p["T"], p["B"], trans=True)
    Ld = unvecF(np.linalg.solve(laplace_dense(p["T"]).T, vecF(p["B"])), p["B"].shape)
    assert rel(L, Ld) < 1e-13


def test_closed_form_diagonal():
    """Diagonal T_mu: X_ijk = B_ijk / (a1_i + a2_j + a3_k)."""
    g = np.random.default_rng(1)
    shape = (64, 48, 40)
    a = [g.uniform(1, 2, n) for n in shape]
    T = [np.diag(x) for x in a]
    B = g.standard_normal(shape)
    X = oracle.lap_solve(T, B)
    Xc = B / (a[0][:, None, None] + a[1][None, :, None] + a[2][None, None, :])
    assert rel(X, Xc) < 1e-15


def _real_eigvec(T, k):
    """Eigenvector of upper quasi-triangular T for the 1x1 eigenvalue T[k,k]:
    v[k] = 1, v[j] = 0 for j > k, rows above by back-substitution with
    (T - lam I); only valid when no bump touches row k."""
    n = T.shape[0]
    lam = T[k, k]
    v = np.zeros(n)
    v[k] = 1.0
    i = k - 1
    while i >= 0:
        if i > 0 and T[i, i - 1] != 0.0:  # 2x2 bump rows i-1, i
            rhs = -np.array([T[i - 1, i + 1:k + 1] @ v[i + 1:k + 1], T[i, i + 1:k + 1] @ v[i + 1:k + 1]])
            M = T[i - 1:i + 1, i - 1:i + 1] - lam * np.eye(2)
            v[i - 1:i + 1] = np.linalg.solve(M, rhs)
            i -= 2
        else:
            v[i] = -(T[i, i + 1:k + 1] @ v[i + 1:k + 1]) / (T[i, i] - lam)
            i -= 1
    return lam, v


def test_eigenvector_rank1_rhs():
    """B = v1 o v2 o v3 with T_mu v_mu = lam_mu v_mu  =>  X = B / (lam1+lam2+lam3)."""
    shape = (40, 33, 24)
    p = ti.laplace_tri(shape, seed=4, bumps="every8")
    lams, vs = [], []
    for t, k in zip(p["T"], (20, 30, 5)):
        assert t[k, k - 1] == 0 and (k + 1 >= t.shape[0] or t[k + 1, k] == 0)
        lam, v = _real_eigvec(t, k)
        assert np.linalg.norm(t @ v - lam * v) < 1e-12 * np.linalg.norm(v)
        lams.append(lam)
        vs.append(v)
    B = np.einsum("i,j,k->ijk", *vs)
    X = oracle.lap_solve(p["T"], B)
    assert rel(X, B / sum(lams)) < 1e-13


def test_d2_is_sylvester():
    """d = 2: X x_1 T_1 + X x_2 T_2 = T_1 X + X T_2^T = B (Sec. 1, eq. (1.1))."""
    p = ti.laplace_tri((120, 90), seed=7, bumps="every8")
    X = oracle.lap_solve(p["T"], p["B"])
    Xs = sla.solve_sylvester(p["T"][0], p["T"][1].T, p["B"])
    assert rel(X, Xs) < 1e-12


def test_d3_merged_sylvester():
    """d = 3 with modes 1 and 2 merged: (T1 (x) I + I (x) T2) X' + X' T3^T = B'
    with X' the (n1 n2) x n3 row-major reshape (Sec. 2.2, Algorithm 3)."""
    shape = (12, 10, 16)
    p = ti.laplace_tri(shape, seed=8, bumps="every8")
    T1, T2, T3 = p["T"]
    Am = np.kron(T1, np.eye(shape[1])) + np.kron(np.eye(shape[0]), T2)
    Bp = p["B"].reshape(shape[0] * shape[1], shape[2])
    Xs = sla.solve_sylvester(Am, T3.T, Bp).reshape(shape)
    X = oracle.lap_solve(p["T"], p["B"])
    assert rel(X, Xs) < 1e-12


def test_residual_and_adjoint_identity():
    p = ti.laplace_tri((30, 26, 22), seed=9, bumps="every8")
    T, B = p["T"], p["B"]
    G = ti.gaussian_tensor(B.shape, ti.rng(9, ti.ROLE_G))
    X = oracle.lap_solve(T, B)
    # residual: applying the operator by the dense mode-product definition
    Y = sum(np.moveaxis(np.tensordot(t, X, axes=(1, mu)), 0, mu) for mu, t in enumerate(T))
    eps = np.finfo(float).eps
    scale = sum(np.linalg.norm(t, 2) for t in T) * np.linalg.norm(X) + np.linalg.norm(B)
    assert np.linalg.norm(Y - B) / scale < 20 * eps
    # <L^{-1} B, G> = <B, L^{-T} G>
    Lam = oracle.lap_solve(T, G, trans=True)
    lhs, rhs = np.vdot(X, G), np.vdot(B, Lam)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_lap_apply_vs_dense():
    p = ti.laplace_tri((5, 6, 4), seed=2, bumps="random")
    Y = oracle.lap_apply(p["T"], p["B"])
    Yd = unvecF(laplace_dense(p["T"]) @ vecF(p["B"]), p["B"].shape)
    assert rel(Y, Yd) < 1e-14
    Yt = oracle.lap_apply(p["T"], p["B"], trans=True)
    Ytd = unvecF(laplace_dense(p["T"]).T @ vecF(p["B"]), p["B"].shape)
    assert rel(Yt, Ytd) < 1e-14


def test_mode_product_vs_tensordot():
    g = np.random.default_rng(3)
    X = g.standard_normal((5, 7, 6, 4))
    for mu in range(4):
        M = g.standard_normal((3, X.shape[mu]))
        Y = oracle.mode_product(X, M, mu)
        Yr = np.moveaxis(np.tensordot(M, X, axes=(1, mu)), 0, mu)
        assert rel(Y, Yr) < 1e-14


def test_singular_detected():
    """Uniqueness fails when an eigenvalue sum vanishes (Sec. 2)."""
    T1 = np.diag([1.0, 2.0, 3.0])
    T2 = np.diag([0.5, -2.0, 4.0])  # 2.0 + (-2.0) = 0
    T3 = np.zeros((1, 1))
    B = np.ones((3, 3, 1))
    with pytest.raises(oracle.OracleError, match="singular"):
        oracle.lap_solve([T1, T2, T3], B)


def test_invalid_structure_detected():
    T = np.triu(np.ones((4, 4)))
    T[2, 0] = 1.0  # below the first subdiagonal
    with pytest.raises(oracle.OracleError, match="invalid"):
        oracle.lap_solve([T, np.eye(2)], np.ones((4, 2)))
    T = np.triu(np.ones((4, 4)))
    T[1, 0] = T[2, 1] = 1.0  # two adjacent subdiagonal entries
    with pytest.raises(oracle.OracleError, match="invalid"):
        oracle.lap_solve([T, np.eye(2)], np.ones((4, 2)))


def test_long_double_hard_variant_close_to_f64():
    """Eigenvalue sums down to 0.05: both precisions solve the same system;
    the difference is bounded by the conditioning, not by a bug."""
    p = ti.laplace_tri((16, 16, 16), seed=3, hard_sum=0.05)
    Xd = oracle.lap_solve(p["T"], p["B"])
    Xl = oracle.lap_solve(p["T"], p["B"], precision="ld")
    A = laplace_dense(p["T"])
    Xref = unvecF(np.linalg.solve(A, vecF(p["B"])), p["B"].shape)
    kappa = np.linalg.cond(A)
    eps = np.finfo(float).eps
    assert rel(Xl, Xref) < 10 * kappa * eps
    assert rel(Xd, Xl) < 10 * kappa * eps


# ------------------------------------------------------------- pair form --

@pytest.mark.parametrize("shape", [(4, 4, 4, 4), (3, 5, 4, 2), (6, 5, 7), (5, 6)])
def test_pair_direct_vs_dense(shape):
    p = ti.pair_tri(shape, seed=13, bumps="random")
    X = oracle.pair_solve(p["A"], p["C"], p["B"], method="direct")
    M = pair_dense(p["A"], p["C"])
    Xd = unvecF(np.linalg.solve(M, vecF(p["B"])), p["B"].shape)
    assert rel(X, Xd) < 1e-13
    Y = oracle.pair_apply(p["A"], p["C"], X)
    assert rel(Y, p["B"]) < 1e-13


@pytest.mark.parametrize("shape", [(5, 5, 5, 5), (8, 6, 4, 3), (9, 10, 8)])
def test_pair_reduced_vs_direct(shape):
    p = ti.pair_tri(shape, seed=17, bumps="every8")
    Xr = oracle.pair_solve(p["A"], p["C"], p["B"], method="reduced")
    Xd = oracle.pair_solve(p["A"], p["C"], p["B"], method="direct")
    assert rel(Xr, Xd) < 1e-13


def test_pair_identity_C_is_laplace():
    p = ti.pair_tri((7, 6, 5, 4), seed=19)
    I = [np.eye(a.shape[0]) for a in p["A"]]
    Xr = oracle.pair_solve(p["A"], I, p["B"], method="reduced")
    Xl = unvecF(np.linalg.solve(laplace_dense(p["A"]), vecF(p["B"])), p["B"].shape)
    assert rel(Xr, Xl) < 1e-13


def test_pair_diagonal_closed_form():
    """Diagonal pairs: X = B / sum_mu a_mu prod_{nu != mu} c_nu."""
    g = np.random.default_rng(23)
    shape = (10, 9, 8, 7)
    a = [g.uniform(1, 2, n) for n in shape]
    c = [g.uniform(1, 2, n) for n in shape]
    B = g.standard_normal(shape)
    X = oracle.pair_solve([np.diag(x) for x in a], [np.diag(x) for x in c], B)
    grids = lambda v: np.ix_(*v)
    den = np.zeros(shape)
    for mu in range(4):
        fac = [a[nu] if nu == mu else c[nu] for nu in range(4)]
        den += np.einsum("i,j,k,l->ijkl", *fac)
    assert rel(X, B / den) < 1e-15


# -------------------------------------------------------------- gradient --

def test_grad_vs_dense_kronecker():
    """dL/dT_mu[a,b] for L = <G, X>, X = L(T)^{-1} B: the dense gradient of
    <g, A^{-1} b> w.r.t. A is -lam x^T with A^T lam = g; projected onto the
    Kronecker positions of T_mu[a, b]."""
    shape = (4, 3, 5)
    p = ti.laplace_tri(shape, seed=29, bumps="aligned")
    T, B = p["T"], p["B"]
    G = ti.gaussian_tensor(shape, ti.rng(29, ti.ROLE_G))
    A = laplace_dense(T)
    x = np.linalg.solve(A, vecF(B))
    lam = np.linalg.solve(A.T, vecF(G))
    dA = -np.outer(lam, x)
    X = unvecF(x, shape)
    Lam = oracle.lap_solve(T, G, trans=True)
    d = len(shape)
    for mu in range(d):
        n = shape[mu]
        ref = np.zeros((n, n))
        for a in range(n):
            for b in range(n):
                E = np.zeros((n, n))
                E[a, b] = 1.0
                facs = [E if nu == mu else np.eye(shape[nu]) for nu in reversed(range(d))]
                K = np.ones((1, 1))
                for f in facs:
                    K = np.kron(K, f)
                ref[a, b] = np.sum(dA * K)
        dT = oracle.grad_T(T, Lam, X, mu, mask=False)
        assert rel(dT, ref) < 1e-12
        dTm = oracle.grad_T(T, Lam, X, mu, mask=True)
        mask = ti.pattern_mask(T[mu])
        assert np.array_equal(dTm[~mask], np.zeros((~mask).sum()))
        assert rel(dTm[mask], ref[mask]) < 1e-12


def test_grad_finite_differences():
    shape = (6, 5, 7)
    p = ti.laplace_tri(shape, seed=31, bumps="every8")
    T, B = p["T"], p["B"]
    G = ti.gaussian_tensor(shape, ti.rng(31, ti.ROLE_G))
    X = oracle.lap_solve(T, B)
    Lam = oracle.lap_solve(T, G, trans=True)
    h = 1e-6
    for mu in range(3):
        D = ti.direction((shape[mu], shape[mu]), 31, mu) * ti.pattern_mask(T[mu])
        Tp = [t + h * D if nu == mu else t for nu, t in enumerate(T)]
        Tm = [t - h * D if nu == mu else t for nu, t in enumerate(T)]
        fd = (np.vdot(G, oracle.lap_solve(Tp, B)) - np.vdot(G, oracle.lap_solve(Tm, B))) / (2 * h)
        an = np.sum(oracle.grad_T(T, Lam, X, mu) * D)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # dL/dB = Lam
    Dir = ti.direction(shape, 31, 9)
    fd = (np.vdot(G, oracle.lap_solve(T, B + h * Dir)) - np.vdot(G, oracle.lap_solve(T, B - h * Dir))) / (2 * h)
    assert abs(fd - np.vdot(Lam, Dir)) <= 1e-6 * max(1.0, abs(fd))


# ------------------------------------------------------------ flop count --

def _brute_force_fma(T, shape):
    """Count multiply-adds of element-wise back-substitution by literally
    walking every element and every coefficient it meets (tiny sizes)."""
    d = len(shape)
    cnt = 0
    for idx in np.ndindex(*shape):
        for mu in range(d):
            t = T[mu]
            i = idx[mu]
            # partner entries: strictly upper row entries and the bump subdiagonal
            cnt += shape[mu] - 1 - i
            if i > 0 and t[i, i - 1] != 0.0:
                cnt += 1
    return cnt


@pytest.mark.parametrize("shape,bumps", [((6, 5, 7), "every8"), ((9, 9, 9), "every8"), ((5, 4, 3, 6), "aligned")])
def test_flops_brute_force(shape, bumps):
    p = ti.laplace_tri(shape, seed=1, bumps=bumps)
    assert oracle.flops_tri(p["T"], shape) == 2 * _brute_force_fma(p["T"], shape)


def test_flops_closed_form_cube():
    n = 512
    T = [np.triu(np.ones((n, n)))] * 3
    assert oracle.flops_tri(T, (n, n, n)) == 3 * (n - 1) * n ** 3


def test_dense_with_factors_vs_dense():
    p = ti.laplace_dense((6, 5, 7), seed=37)
    X = oracle.dense_solve_with_factors(p["Q"], p["T"], p["B"])
    Xd = unvecF(np.linalg.solve(laplace_dense(p["A"]), vecF(p["B"])), p["B"].shape)
    assert rel(X, Xd) < 1e-12


@pytest.mark.parametrize("shape", [(6, 5, 7), (3, 5, 4, 2), (9, 8)])
def test_pair_dense_with_factors_vs_dense(shape):
    """Dense pair form (Sec. 3) through known generalized Schur factors
    against the assembled Kronecker operator (eq. 1.4 for pairs)."""
    p = ti.pair_dense(shape, seed=41, bumps="random")
    X = oracle.pair_dense_solve_with_factors(p["Q"], p["S"], p["T"], p["Z"], p["B"])
    Xd = unvecF(np.linalg.solve(pair_dense(p["A"], p["C"]), vecF(p["B"])), p["B"].shape)
    assert rel(X, Xd) < 1e-12
    assert rel(oracle.pair_apply(p["A"], p["C"], X), p["B"]) < 1e-13


# ---------------------------------------------------------------------------
# Second operator class, eq. (1.5) / (3.1): X x_1 A_1 + X x_1 C x_2 A_2 .. = B
# ---------------------------------------------------------------------------
from kron import gsylv_dense  # noqa: E402


@pytest.mark.parametrize("shape,bumps", [((7, 6), "every8"), ((5, 4, 6), "aligned"), ((6, 5, 4), "random"),
                                         ((4, 3, 4, 3), "aligned"), ((9, 9, 2), "every8"),
                                         ((3, 4, 5, 4), "none")])
def test_gsylv_solve_vs_dense_kronecker(shape, bumps):
    p = ti.gsylv_tri(shape, seed=51, bumps=bumps)
    X = oracle.gsylv_solve(p["A"], p["C"], p["B"])
    Xd = unvecF(np.linalg.solve(gsylv_dense(p["A"], p["C"]), vecF(p["B"])), p["B"].shape)
    assert rel(X, Xd) < 1e-12
    Y = oracle.gsylv_apply(p["A"], p["C"], X)
    assert rel(unvecF(gsylv_dense(p["A"], p["C"]) @ vecF(X), X.shape), Y) < 1e-14
    assert rel(Y, p["B"]) < 1e-13


def test_gsylv_d2_is_generalized_sylvester():
    """d = 2: A_1 X + C X A_2^T = B (Sec. 1), i.e. the Sylvester equation
    (C^{-1} A_1) X + X A_2^T = C^{-1} B, solved by SciPy (Bartels-Stewart)."""
    p = ti.gsylv_tri((60, 45), seed=52, bumps="every8")
    X = oracle.gsylv_solve(p["A"], p["C"], p["B"])
    Ci = np.linalg.inv(p["C"])
    Xs = sla.solve_sylvester(Ci @ p["A"][0], p["A"][1].T, Ci @ p["B"])
    assert rel(X, Xs) < 1e-11


def test_gsylv_diagonal_closed_form():
    """Diagonal A_mu, C: X = B / (a_1 + c prod_{mu >= 2} a_mu)."""
    g = np.random.default_rng(53)
    shape = (7, 6, 5, 4)
    a = [1.0 + g.random(n) for n in shape]
    c = 1.0 + g.random(shape[0])
    B = g.standard_normal(shape)
    X = oracle.gsylv_solve([np.diag(v) for v in a], np.diag(c), B)
    den = a[0][:, None, None, None] + c[:, None, None, None] * (
        a[1][None, :, None, None] * a[2][None, None, :, None] * a[3][None, None, None, :])
    assert rel(X, B / den) < 1e-15


def test_gsylv_shifted_kronecker_eigenvector_rhs():
    """Eq. (1.6), A_1 = -lambda I: the operator is A_d (x) .. (x) A_2 (x) C -
    lambda I.  With B = e_1 o v_2 o v_3 (C e_1 = c_11 e_1 for upper
    triangular C, A_mu v_mu = alpha_mu v_mu): X = B / (c_11 alpha_2 alpha_3 -
    lambda).  The same right-hand side with a general A_1 whose first row is
    a 1x1 block gives B / (a_11 + c_11 alpha_2 alpha_3)."""
    shape = (12, 17, 13)
    p = ti.gsylv_tri(shape, seed=54, bumps="every8")
    alphas, vs = [], []
    for t, k in zip(p["A"][1:], (9, 3)):
        assert t[k, k - 1] == 0 and t[k + 1, k] == 0
        alpha, v = _real_eigvec(t, k)
        alphas.append(alpha)
        vs.append(v)
    e1 = np.zeros(shape[0])
    e1[0] = 1.0
    B = np.einsum("i,j,k->ijk", e1, *vs)
    lam = 0.37
    Ash = [-lam * np.eye(shape[0])] + p["A"][1:]
    X = oracle.gsylv_solve(Ash, p["C"], B)
    assert rel(X, B / (p["C"][0, 0] * alphas[0] * alphas[1] - lam)) < 1e-13
    assert p["A"][0][1, 0] == 0.0
    X2 = oracle.gsylv_solve(p["A"], p["C"], B)
    assert rel(X2, B / (p["A"][0][0, 0] + p["C"][0, 0] * alphas[0] * alphas[1])) < 1e-13


def test_gsylv_long_double_agrees():
    p = ti.gsylv_tri((7, 8, 6), seed=55, bumps="every8")
    X = oracle.gsylv_solve(p["A"], p["C"], p["B"])
    Xl = oracle.gsylv_solve(p["A"], p["C"], p["B"], precision="ld")
    assert rel(X, Xl) < 1e-14


def test_gsylv_singular_detected():
    """A_1 = -C and A_2 = I: the pencil eigenvalue 1 meets -A_2's eigenvalue."""
    n = 4
    C = np.triu(np.ones((n, n)))
    with pytest.raises(oracle.OracleError):
        oracle.gsylv_solve([-C, np.eye(3), np.eye(2)], C, np.ones((n, 3, 2)))


@pytest.mark.parametrize("shape", [(6, 5, 4), (4, 3, 4, 3), (8, 7)])
def test_gsylv_dense_with_factors_vs_dense(shape):
    """Algorithm 4 with known factors against the assembled dense operator."""
    p = ti.gsylv_dense(shape, seed=56, bumps="random")
    X = oracle.gsylv_dense_solve_with_factors(p["Q"], p["S"], p["T"], p["Z"], p["U"], p["Tq"], p["B"])
    Xd = unvecF(np.linalg.solve(gsylv_dense(p["A"], p["C"]), vecF(p["B"])), p["B"].shape)
    assert rel(X, Xd) < 1e-12
    assert rel(oracle.gsylv_apply(p["A"], p["C"], X), p["B"]) < 1e-13
