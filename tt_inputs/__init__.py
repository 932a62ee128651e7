"""Seeded synthetic inputs for Kronecker-structured tensor equations.

This module only draws random inputs; it holds none of the solver's
arithmetic.  Both the CPU oracle tests and the GPU path take their inputs
from here, so the two sides always see bit-identical data.

Conventions
-----------
* Tensors are float64 numpy arrays in C order with shape ``(n_1, ..., n_d)``:
  the last mode varies fastest in memory.
* A coefficient ``T[mu]`` is a row-major ``n_mu x n_mu`` float64 array.
* Upper quasi-triangular coefficients (real Schur form, Sec. 2 of the paper)
  carry 2x2 diagonal blocks ("bumps") ``[[a, b], [-b, a]]`` whose eigenvalues
  are the complex pair ``a +/- i b``.
* Every random stream is ``default_rng(SeedSequence([seed, role, mu, item]))``
  so any single coefficient or right-hand side can be regenerated alone.
"""
from __future__ import annotations

import numpy as np

ROLE_T, ROLE_Q, ROLE_C, ROLE_B, ROLE_G, ROLE_DIR, ROLE_SHAPE, ROLE_Z = 0, 1, 2, 3, 4, 5, 6, 7


def rng(seed: int, role: int, mu: int = 0, item: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), role, mu, item]))


def bump_starts(n: int, kind: str = "every8", g: np.random.Generator | None = None):
    """0-based first rows of the 2x2 bumps of an n x n coefficient.

    kind:
      "every8"  - starts i = 7, 15, 23, ... (1-based rows 8,9; 16,17; ...).
                  Every power-of-two split point falls inside a bump.
      "aligned" - starts i = 0, 8, 16, ...
      "random"  - non-overlapping random starts, about one per 8 rows.
      "none"    - upper triangular, no bumps.
    """
    if kind == "none" or n < 2:
        return []
    if kind == "every8":
        return [i for i in range(7, n - 1, 8)]
    if kind == "aligned":
        return [i for i in range(0, n - 1, 8)]
    if kind == "random":
        assert g is not None
        out, i = [], 0
        while i < n - 1:
            if g.random() < 0.125:
                out.append(i)
                i += 2
            else:
                i += 1
        return out
    raise ValueError(kind)


def quasi_triangular(n: int, g: np.random.Generator, bumps="every8",
                     diag_lo: float = 1.0, diag_hi: float = 2.0,
                     imag_lo: float = 0.1, imag_hi: float = 0.5,
                     offdiag_scale: float | None = None) -> np.ndarray:
    """Upper quasi-triangular T: diagonal (real parts) ~ U[diag_lo, diag_hi],
    strict upper part ~ N(0,1)/sqrt(n), bumps [[a, b], [-b, a]] with
    b ~ U[imag_lo, imag_hi]."""
    T = np.zeros((n, n))
    if n == 0:
        return T
    scale = (1.0 / np.sqrt(n)) if offdiag_scale is None else offdiag_scale
    up = g.standard_normal((n, n)) * scale
    T[np.triu_indices(n, 1)] = up[np.triu_indices(n, 1)]
    T[np.diag_indices(n)] = g.uniform(diag_lo, diag_hi, n)
    starts = bump_starts(n, bumps, g) if isinstance(bumps, str) else list(bumps)
    for i in starts:
        a = T[i, i]
        b = g.uniform(imag_lo, imag_hi)
        T[i + 1, i + 1] = a
        T[i, i + 1] = b
        T[i + 1, i] = -b
    return T


def upper_triangular(n: int, g: np.random.Generator, diag_lo=1.0, diag_hi=2.0) -> np.ndarray:
    C = np.triu(g.standard_normal((n, n)) / np.sqrt(max(n, 1)), 1)
    C[np.diag_indices(n)] = g.uniform(diag_lo, diag_hi, n)
    return C


def random_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Q from the QR factorisation of an N(0,1) matrix, signs fixed so that
    diag(R) > 0 (Haar distributed)."""
    Z = g.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def gaussian_tensor(shape, g: np.random.Generator) -> np.ndarray:
    return np.ascontiguousarray(g.standard_normal(tuple(int(x) for x in shape)))


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns a dict of numpy arrays.
# ---------------------------------------------------------------------------

def laplace_tri(shape, seed=0, bumps="every8", diag=(1.0, 2.0), hard_sum=None, hard_coupled=False):
    """Triangular Laplace-like problem  sum_mu X x_mu T_mu = B.

    hard_sum: if given, real parts are drawn from U[hard_sum/d, 2] and one 1x1
    diagonal entry per mode is pinned to hard_sum/d, so that the smallest
    eigenvalue sum is exactly hard_sum.
    hard_coupled (with hard_sum): also the first 2x2 block of every mode gets
    real part hard_sum/d and imaginary parts 0.2, 0.3, 0.5, 0.7 (modes 0..3),
    so that coupled tuples reach the same smallest sum: the tuple of the
    first blocks of modes 0, 1, 2 has the eigenvalue
    hard_sum + i (0.2 + 0.3 - 0.5) = hard_sum, and the tuples of two such
    blocks with the pinned 1x1 entries have hard_sum + i (b_mu - b_nu).
    """
    shape = tuple(int(x) for x in shape)
    d = len(shape)
    T = []
    for mu, n in enumerate(shape):
        g = rng(seed, ROLE_T, mu)
        lo, hi = diag
        if hard_sum is not None:
            lo, hi = hard_sum / d, 2.0
        t = quasi_triangular(n, g, bumps, lo, hi)
        if hard_sum is not None and n > 0:
            in_bump = np.zeros(n, bool)
            for i in range(n - 1):
                if t[i + 1, i] != 0.0:
                    in_bump[i] = in_bump[i + 1] = True
            free = np.flatnonzero(~in_bump)
            if len(free):
                t[free[-1], free[-1]] = hard_sum / d
            if hard_coupled:
                first = [i for i in range(n - 1) if t[i + 1, i] != 0.0]
                if first:
                    i, b = first[0], (0.2, 0.3, 0.5, 0.7)[mu]
                    t[i, i] = t[i + 1, i + 1] = hard_sum / d
                    t[i, i + 1], t[i + 1, i] = b, -b
        T.append(t)
    B = gaussian_tensor(shape, rng(seed, ROLE_B))
    return {"T": T, "B": B}


def laplace_dense(shape, seed=0, bumps="every8", hard_sum=None):
    """Dense coefficients A_mu = Q_mu T_mu Q_mu^T with T_mu as laplace_tri."""
    p = laplace_tri(shape, seed, bumps, hard_sum=hard_sum)
    Q = [random_orthogonal(t.shape[0], rng(seed, ROLE_Q, mu)) for mu, t in enumerate(p["T"])]
    A = [np.ascontiguousarray(q @ t @ q.T) for q, t in zip(Q, p["T"])]
    p.update({"Q": Q, "A": A})
    return p


def pair_tri(shape, seed=0, bumps="every8", c_lo=None):
    """Pair form  sum_mu X x_1 C_1 ... x_mu A_mu ... x_d C_d = B.
    c_lo: if given, the diagonal of each C_mu is log-uniform in [c_lo, 1]
    (strict upper part N(0,1)/sqrt(n) scaled by c_lo) instead of U[1, 2]:
    ill-conditioned C_mu."""
    shape = tuple(int(x) for x in shape)
    A = [quasi_triangular(n, rng(seed, ROLE_T, mu), bumps) for mu, n in enumerate(shape)]
    if c_lo is None:
        C = [upper_triangular(n, rng(seed, ROLE_C, mu)) for mu, n in enumerate(shape)]
    else:
        C = []
        for mu, n in enumerate(shape):
            g = rng(seed, ROLE_C, mu)
            c = np.triu(g.standard_normal((n, n)) * (c_lo / np.sqrt(max(n, 1))), 1)
            c[np.diag_indices(n)] = np.exp(g.uniform(np.log(c_lo), 0.0, n))
            C.append(c)
    B = gaussian_tensor(shape, rng(seed, ROLE_B))
    return {"A": A, "C": C, "B": B}


def gsylv_tri(shape, seed=0, bumps="every8"):
    """Second operator class (eq. (3.1)) with triangular coefficients:
    X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d = B, A_mu upper quasi-triangular
    as laplace_tri, C upper triangular with diagonal U[1,2]."""
    shape = tuple(int(x) for x in shape)
    A = [quasi_triangular(n, rng(seed, ROLE_T, mu), bumps) for mu, n in enumerate(shape)]
    C = upper_triangular(shape[0], rng(seed, ROLE_C, 0))
    B = gaussian_tensor(shape, rng(seed, ROLE_B))
    return {"A": A, "C": C, "B": B}


def gsylv_dense(shape, seed=0, bumps="every8"):
    """Dense second class (Algorithm 4): A_1 = Q S Z^T, C = Q T Z^T with
    (S, T) the triangular pair of gsylv_tri and A_mu = U_mu Tq_mu U_mu^T
    (mu >= 2), all orthogonal factors random (so the reductions are known)."""
    p = gsylv_tri(shape, seed, bumps)
    Q = random_orthogonal(shape[0], rng(seed, ROLE_Q, 0))
    Z = random_orthogonal(shape[0], rng(seed, ROLE_Z, 0))
    U = [random_orthogonal(n, rng(seed, ROLE_Q, mu)) for mu, n in enumerate(shape) if mu >= 1]
    A = [np.ascontiguousarray(Q @ p["A"][0] @ Z.T)]
    A += [np.ascontiguousarray(u @ t @ u.T) for u, t in zip(U, p["A"][1:])]
    Cd = np.ascontiguousarray(Q @ p["C"] @ Z.T)
    return {"A": A, "C": Cd, "B": p["B"], "S": p["A"][0], "T": p["C"], "Q": Q, "Z": Z, "U": U,
            "Tq": p["A"][1:]}


def pair_dense(shape, seed=0, bumps="every8"):
    """Dense pair form: A_mu = Q_mu S_mu Z_mu^T, C_mu = Q_mu T_mu Z_mu^T with
    (S_mu, T_mu) the triangular pair of pair_tri and Q_mu, Z_mu random
    orthogonal (so the generalized Schur factors are known)."""
    p = pair_tri(shape, seed, bumps)
    Q = [random_orthogonal(a.shape[0], rng(seed, ROLE_Q, mu)) for mu, a in enumerate(p["A"])]
    Z = [random_orthogonal(a.shape[0], rng(seed, ROLE_Z, mu)) for mu, a in enumerate(p["A"])]
    Ad = [np.ascontiguousarray(q @ a @ z.T) for q, a, z in zip(Q, p["A"], Z)]
    Cd = [np.ascontiguousarray(q @ c @ z.T) for q, c, z in zip(Q, p["C"], Z)]
    return {"A": Ad, "C": Cd, "B": p["B"], "S": p["A"], "T": p["C"], "Q": Q, "Z": Z}


def uneven_batch(count=64, lo=32, hi=192, seed=0, d=3, bumps="every8"):
    """Batch of independent triangular Laplace problems with mode sizes drawn
    independently and uniformly from {lo, ..., hi}."""
    gs = rng(seed, ROLE_SHAPE)
    shapes = [tuple(int(x) for x in gs.integers(lo, hi + 1, d)) for _ in range(count)]
    probs = []
    for b, shp in enumerate(shapes):
        T = [quasi_triangular(n, rng(seed, ROLE_T, mu, b), bumps) for mu, n in enumerate(shp)]
        B = gaussian_tensor(shp, rng(seed, ROLE_B, 0, b))
        G = gaussian_tensor(shp, rng(seed, ROLE_G, 0, b))
        probs.append({"T": T, "B": B, "G": G})
    return probs


def direction(shape, seed, item):
    """Unit-Frobenius random direction for directional finite differences."""
    v = gaussian_tensor(shape, rng(seed, ROLE_DIR, 0, item))
    return v / np.linalg.norm(v)


def pattern_mask(T: np.ndarray) -> np.ndarray:
    """Entries of a quasi-triangular coefficient that the solver reads: the
    upper triangle plus the nonzero subdiagonal entries of the bumps."""
    n = T.shape[0]
    m = np.triu(np.ones((n, n), bool))
    for i in range(n - 1):
        if T[i + 1, i] != 0.0:
            m[i + 1, i] = True
    return m
