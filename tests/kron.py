"""Dense Kronecker reference operators for tests (tiny sizes only).

The paper's vectorisation (Sec. 2, eq. (2.1)) runs i_1 fastest, i.e. numpy
order='F'.  In that ordering the Laplace-like operator of eq. (1.4) is
  A = A_d (x) I (x) .. (x) I + .. + I (x) .. (x) I (x) A_1.
"""
import numpy as np


def kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def laplace_dense(T):
    """Dense matrix of sum_mu X x_mu T_mu acting on vec_F(X), eq. (1.4)."""
    d = len(T)
    n = [t.shape[0] for t in T]
    N = int(np.prod(n))
    A = np.zeros((N, N))
    for mu in range(d):
        # factors from mode d (slowest in F order) down to mode 1 (fastest)
        facs = [T[nu] if nu == mu else np.eye(n[nu]) for nu in reversed(range(d))]
        A += kron_all(facs)
    return A


def pair_dense(A, C):
    """Dense matrix of sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d on vec_F(X)."""
    d = len(A)
    n = [a.shape[0] for a in A]
    N = int(np.prod(n))
    M = np.zeros((N, N))
    for mu in range(d):
        facs = [A[nu] if nu == mu else C[nu] for nu in reversed(range(d))]
        M += kron_all(facs)
    return M


def vecF(X):
    return X.flatten(order="F")


def unvecF(v, shape):
    return v.reshape(shape, order="F")


def gsylv_dense(A, C):
    """Dense matrix of X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d on vec_F(X),
    eq. (1.5): I (x) .. (x) I (x) A_1 + A_d (x) .. (x) A_2 (x) C."""
    d = len(A)
    n = [a.shape[0] for a in A]
    first = kron_all([np.eye(n[nu]) for nu in reversed(range(1, d))] + [A[0]])
    second = kron_all([A[nu] for nu in reversed(range(1, d))] + [C])
    return first + second
