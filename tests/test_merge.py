"""Merge of two modes (Algorithm 3, Sec. 2.2, real quasi-triangular case):
A' = A_a (x) I + I (x) A_b, perfect shuffle of the block rows of A_a's 2x2
blocks, real Schur forms of the resulting 4x4 diagonal blocks.  Host only.

Pins: the permuted sparsity pattern the paper prints for its eq. (2.9)
example (golden fixture), A' = V Tm V^T with V orthogonal, Tm upper
quasi-triangular (the solver's own structure check accepts it), and the
eigenvalues of Tm are the pairwise sums of those of A_a and A_b."""
import os

import numpy as np
import pytest

import tt_inputs as ti

tt = pytest.importorskip("paper_1905_09539_amd")
HERE = os.path.dirname(os.path.abspath(__file__))


def _pattern(name, tag):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, *vals = line.split()
            if t == tag:
                rows.append([v == "x" for v in vals])
    return np.array(rows)


def test_golden_shuffled_pattern():
    P1 = _pattern("merged_pattern_eq2_9.txt", "A1")  # inner, 4x4
    P2 = _pattern("merged_pattern_eq2_9.txt", "A2")  # outer, 3x3
    PP = _pattern("shuffled_merged_pattern_sec2_2.txt", "P")
    g = np.random.default_rng(7)
    A1 = np.where(P1, g.uniform(1, 2, P1.shape), 0.0)
    A2 = np.where(P2, g.uniform(1, 2, P2.shape), 0.0)
    Tm, V, perm = tt.merge_modes_host(A2, A1)
    Ap = np.kron(A2, np.eye(4)) + np.kron(np.eye(3), A1)
    Ps = Ap[np.ix_(perm, perm)]
    assert np.array_equal(Ps != 0, PP)


def _quasi_ok(T):
    n = T.shape[0]
    below = np.tril(T, -2)
    sub = np.diag(T, -1)
    return not below.any() and not np.any((sub[:-1] != 0) & (sub[1:] != 0)) if n > 2 else not below.any()


@pytest.mark.parametrize("na,nb,ba,bb", [(8, 12, "every8", "every8"), (5, 7, "aligned", "aligned"),
                                         (16, 3, "random", "aligned"), (6, 6, "none", "aligned"),
                                         (9, 4, "aligned", "none"), (1, 5, "none", "aligned")])
def test_merge_factors(na, nb, ba, bb):
    g = np.random.default_rng(na * 31 + nb)
    Ta = ti.quasi_triangular(na, g, ba)
    Tb = ti.quasi_triangular(nb, g, bb)
    Tm, V, perm = tt.merge_modes_host(Ta, Tb)
    A = np.kron(Ta, np.eye(nb)) + np.kron(np.eye(na), Tb)
    m = na * nb
    assert np.linalg.norm(V.T @ V - np.eye(m)) < 1e-13 * m
    assert np.linalg.norm(V @ Tm @ V.T - A) < 1e-13 * np.linalg.norm(A)
    assert _quasi_ok(Tm)
    assert sorted(perm.tolist()) == list(range(m))
    # the solver's planner accepts Tm as upper quasi-triangular
    tt.schedule_info([Tm, np.eye(2), np.eye(2)], (m, 2, 2), nmin=8)
    ea = np.linalg.eigvals(Ta)
    eb = np.linalg.eigvals(Tb)
    sums = list((ea[:, None] + eb[None, :]).ravel())
    em = np.linalg.eigvals(Tm)
    # greedy matching (eigenvalues of these non-normal matrices are computed
    # to about sqrt(u) where sums coincide)
    for z in em:
        k = int(np.argmin([abs(z - w) for w in sums]))
        assert abs(z - sums[k]) < 1e-6
        sums.pop(k)
