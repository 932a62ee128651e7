"""Host real Schur decomposition (the host step of Algorithm 1): A = U T U^T
with U orthogonal and T upper quasi-triangular in standard form.  CPU only."""
import numpy as np
import scipy.linalg as sla
import pytest

import tt_inputs as ti

U64 = np.finfo(np.float64).eps


def tt():
    import paper_1905_09539_amd as m
    return m


def check_schur(A, T, U, c=50.0):
    n = A.shape[0]
    an = max(np.linalg.norm(A), 1e-300)
    assert np.linalg.norm(A - U @ T @ U.T) <= c * max(n, 1) * U64 * an
    assert np.linalg.norm(U.T @ U - np.eye(n)) <= c * max(n, 1) * U64
    # quasi-triangular: nothing below the first subdiagonal, isolated bumps
    assert np.all(np.tril(T, -2) == 0.0)
    sub = np.diag(T, -1)
    nz = np.nonzero(sub)[0]
    assert np.all(np.diff(nz) >= 2), "two consecutive nonzero subdiagonal entries"
    # standardised 2x2 blocks: equal diagonal, off-diagonals of opposite sign
    for k in nz:
        assert T[k, k] == T[k + 1, k + 1]
        assert T[k, k + 1] * T[k + 1, k] < 0.0
    return nz


def eig_of_T(T):
    """Eigenvalues of a standardised quasi-triangular T (block by block)."""
    n = T.shape[0]
    ev, k = [], 0
    while k < n:
        if k + 1 < n and T[k + 1, k] != 0.0:
            a, b, c = T[k, k], T[k, k + 1], T[k + 1, k]
            w = np.sqrt(-b * c)
            ev += [a + 1j * w, a - 1j * w]
            k += 2
        else:
            ev.append(T[k, k] + 0j)
            k += 1
    return np.array(ev)


def match_sets(a, b):
    """Greedy nearest matching distance between two eigenvalue multisets."""
    b = list(b)
    worst = 0.0
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[j]))
        b.pop(j)
    return worst


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (12, 4), (50, 5), (151, 6)])
def test_gaussian_matrices(n, seed):
    A = np.random.default_rng(seed).standard_normal((n, n))
    T, U = tt().schur_host(A)
    check_schur(A, T, U)
    # Gaussian matrices have well-conditioned eigenvalues: compare with the
    # eigenvalues LAPACK computes for A
    assert match_sets(eig_of_T(T), np.linalg.eigvals(A)) <= 1e-8 * max(1.0, np.linalg.norm(A))


@pytest.mark.parametrize("n,bumps", [(8, "every8"), (40, "every8"), (97, "random"), (200, "aligned")])
def test_generator_matrices(n, bumps):
    """A = Q T Q^T from the input generator (the dense-coefficient workload)."""
    g = ti.rng(7, ti.ROLE_T, 0, n)
    T0 = ti.quasi_triangular(n, g, bumps=bumps)
    Q = ti.random_orthogonal(n, ti.rng(7, ti.ROLE_Q, 0, n))
    A = Q @ T0 @ Q.T
    T, U = tt().schur_host(A)
    check_schur(A, T, U)
    # similarity invariants: trace and sum of squares of the eigenvalues
    assert abs(np.trace(T) - np.trace(T0)) <= 100 * n * U64 * np.linalg.norm(A)
    assert abs(np.trace(T @ T) - np.trace(T0 @ T0)) <= 1e3 * n * U64 * np.linalg.norm(A) ** 2


def test_well_separated_eigenvalues_match_generator():
    """Nearly normal T (tiny strict upper part): eigenvalues are well
    conditioned, so those of the computed T match the generator's."""
    n = 60
    g = np.random.default_rng(11)
    T0 = np.diag(np.linspace(1.0, 2.0, n)) + 1e-3 * np.triu(g.standard_normal((n, n)), 1)
    for k in (7, 23, 41):  # complex pairs a +- i b
        a, b = T0[k, k], 0.3
        T0[k, k + 1], T0[k + 1, k], T0[k + 1, k + 1] = b, -b, a
    Q = ti.random_orthogonal(n, np.random.default_rng(12))
    A = Q @ T0 @ Q.T
    T, U = tt().schur_host(A)
    nz = check_schur(A, T, U)
    assert len(nz) == 3
    assert match_sets(eig_of_T(T), eig_of_T(T0)) <= 1e-10


@pytest.mark.parametrize("case", ["zero", "identity", "upper", "rotation", "real2x2", "jordan", "blockrep"])
def test_special_matrices(case):
    n = 6
    if case == "zero":
        A = np.zeros((n, n))
    elif case == "identity":
        A = np.eye(n)
    elif case == "upper":
        A = np.triu(np.random.default_rng(1).standard_normal((n, n)))
    elif case == "rotation":
        A = np.array([[0.0, 1.0], [-1.0, 0.0]])
    elif case == "real2x2":
        A = np.array([[1.0, 2.0], [3.0, 4.0]])
    elif case == "jordan":
        A = np.eye(n) * 2.0 + np.diag(np.ones(n - 1), 1)
    else:  # repeated complex pair, block diagonal
        R = np.array([[1.0, 2.0], [-2.0, 1.0]])
        A = np.kron(np.eye(3), R)
    T, U = tt().schur_host(A)
    nz = check_schur(A, T, U)
    if case == "rotation":
        assert len(nz) == 1 and abs(T[0, 0]) < 1e-15 and abs(T[0, 1] * T[1, 0] + 1.0) < 1e-14
    if case == "real2x2":
        assert len(nz) == 0
        assert match_sets(np.diag(T), [(5 - np.sqrt(33)) / 2, (5 + np.sqrt(33)) / 2]) < 1e-13
    if case == "blockrep":
        assert len(nz) == 3


def test_non_finite_rejected():
    A = np.eye(4)
    A[1, 2] = np.nan
    with pytest.raises(tt().TTError):
        tt().schur_host(A)


# ---------------------------------------------------------------- QZ (Sec. 3)
def check_qz(A, C, S, T, Q, Z, c=50.0):
    n = A.shape[0]
    assert np.linalg.norm(A - Q @ S @ Z.T) <= c * max(n, 1) * U64 * max(np.linalg.norm(A), 1e-300)
    assert np.linalg.norm(C - Q @ T @ Z.T) <= c * max(n, 1) * U64 * max(np.linalg.norm(C), 1e-300)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= c * max(n, 1) * U64
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= c * max(n, 1) * U64
    assert np.all(np.tril(T, -1) == 0.0)
    assert np.all(np.tril(S, -2) == 0.0)
    nz = np.nonzero(np.diag(S, -1))[0]
    assert np.all(np.diff(nz) >= 2), "two consecutive nonzero subdiagonal entries"
    # a 2x2 block is kept only for a complex pair
    for k in nz:
        ev = sla.eigvals(S[k:k + 2, k:k + 2], T[k:k + 2, k:k + 2])
        assert abs(ev[0].imag) > 0.0
    return nz


def pencil_eigs(S, T):
    n, ev, k = S.shape[0], [], 0
    while k < n:
        if k + 1 < n and S[k + 1, k] != 0.0:
            ev += list(sla.eigvals(S[k:k + 2, k:k + 2], T[k:k + 2, k:k + 2]))
            k += 2
        else:
            ev.append(S[k, k] / T[k, k])
            k += 1
    return np.array(ev, dtype=complex)


def match_eigs(ev, ref):
    ev, worst = list(ev), 0.0
    for r in ref:
        d = [abs(r - e) for e in ev]
        j = int(np.argmin(d))
        worst = max(worst, d[j] / max(1.0, abs(r)))
        ev.pop(j)
    return worst


def _pencils():
    g = np.random.default_rng(5)
    out = []
    for n in (1, 2, 3, 5, 17, 64):
        out.append(("random", g.normal(size=(n, n)), g.normal(size=(n, n)) + 2.0 * np.eye(n)))
    n = 40
    M = g.normal(size=(n, n))
    out.append(("symmetric A, C = I", M + M.T, np.eye(n)))
    out.append(("upper triangular C", g.normal(size=(n, n)), np.triu(g.normal(size=(n, n))) + 3.0 * np.eye(n)))
    k = 12
    Ar = np.zeros((2 * k, 2 * k))
    for i in range(k):
        Ar[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[1.0 + 0.1 * i, 2.0], [-2.0, 1.0 + 0.1 * i]]
    Qr = ti.random_orthogonal(2 * k, g)
    out.append(("complex pairs only", Qr @ Ar @ Qr.T, np.eye(2 * k) + 0.05 * g.normal(size=(2 * k, 2 * k))))
    p = ti.pair_dense((30, 24), seed=3)
    out.append(("generated dense pair", p["A"][0], p["C"][0]))
    return out


@pytest.mark.parametrize("case", _pencils(), ids=lambda c: f"{c[0]}-{c[1].shape[0]}")
def test_qz_properties_and_eigenvalues(case):
    """A = Q S Z^T, C = Q T Z^T, orthogonal factors, the patterns of the
    generalized real Schur form, and the pencil's eigenvalues against
    scipy.linalg.eigvals(A, C)."""
    _, A, C = case
    S, T, Q, Z = tt().qz_host(A, C)
    nz = check_qz(A, C, S, T, Q, Z)
    # the generated pencil has clustered non-normal eigenvalues (condition
    # ~1e8): its eigenvalues agree only to what that allows; QZ's guarantee
    # is the backward error checked above
    tol = 1e-6 if case[0] == "generated dense pair" else 1e-10
    assert match_eigs(pencil_eigs(S, T), sla.eigvals(A, C)) < tol
    if case[0] == "symmetric A, C = I":
        assert len(nz) == 0
    if case[0] == "complex pairs only":
        assert len(nz) == A.shape[0] // 2


def test_qz_identity_C_gives_real_schur_spectrum():
    A = ti.laplace_dense((20, 3, 3), seed=8)["A"][0]
    S, T, Q, Z = tt().qz_host(A, np.eye(20))
    check_qz(A, np.eye(20), S, T, Q, Z)
    assert match_eigs(pencil_eigs(S, T), np.linalg.eigvals(A)) < 1e-10


def test_qz_errors():
    g = np.random.default_rng(2)
    C = g.normal(size=(9, 9))
    C[:, 4] = 0.0
    with pytest.raises(tt().TTError, match="singular"):
        tt().qz_host(g.normal(size=(9, 9)), C)
    A = g.normal(size=(5, 5))
    A[1, 2] = np.inf
    with pytest.raises(tt().TTError):
        tt().qz_host(A, np.eye(5))


def test_general_pair_plan_rejects_singular_C():
    """The dense-pair plan fails on the host (before any device work) when
    some C_mu is singular."""
    import ctypes
    m = tt()
    p = ti.pair_dense((6, 5, 4), seed=4)
    C = [c.copy() for c in p["C"]]
    C[1][:, 0] = 0.0
    _, ap = m._host_mats(p["A"])
    _, cp = m._host_mats(C)
    o = m.Opts()
    m.lib().tt_opts_default(ctypes.byref(o))
    h = ctypes.c_void_p()
    rc = m.lib().tt_plan_create_general_pair(ctypes.byref(h), 3, m._shape((6, 5, 4)), ap, cp, ctypes.byref(o))
    assert rc == m.TT_ESINGULAR
    assert not h.value
    assert b"singular" in m.lib().tt_last_error()
