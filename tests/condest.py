"""1-norm condition number of the Laplace-like operator (test helper).

L = sum_mu I (x) .. (x) T_mu (x) .. (x) I (eq. (1.4)) acting on tensors.
||L||_1 is exact: column j = (j_1..j_d) of L holds T_mu[:, j_mu] along each
mode and the diagonal entry sum_mu T_mu[j_mu, j_mu], so
  colsum(j) = sum_mu sum_{i != j_mu} |T_mu[i, j_mu]| + |sum_mu T_mu[j_mu, j_mu]|.
||L^{-1}||_1 is estimated with Hager's method as refined by Higham
(N. J. Higham, "FORTRAN codes for estimating the one-norm of a real or complex
matrix", ACM TOMS 14, 1988): power-type steps with solves by L and L^T, plus
the alternating-sign test vector.  The solves are the oracle's (long double
by default), so the estimate does not depend on the GPU path.
"""
import numpy as np

import oracle


def laplace_norm1(T):
    d = len(T)
    cols, diag = [], []
    for t in T:
        a = np.abs(t)
        dg = np.diag(t).copy()
        cols.append(a.sum(axis=0) - np.abs(dg))
        diag.append(dg)
    tot_off = np.zeros([1] * d)
    tot_dg = np.zeros([1] * d)
    for mu in range(d):
        shp = [1] * d
        shp[mu] = -1
        tot_off = tot_off + cols[mu].reshape(shp)
        tot_dg = tot_dg + diag[mu].reshape(shp)
    return float(np.max(tot_off + np.abs(tot_dg)))


def inverse_norm1_estimate(T, shape, precision="ld", itmax=5):
    shape = tuple(int(x) for x in shape)
    N = int(np.prod(shape))
    x = np.full(shape, 1.0 / N)
    est = 0.0
    xi_old = None
    for k in range(itmax):
        y = oracle.lap_solve(T, x, precision=precision)
        est_new = float(np.abs(y).sum())
        xi = np.where(y >= 0, 1.0, -1.0)
        if k > 0 and (est_new <= est or (xi_old is not None and np.array_equal(xi, xi_old))):
            est = max(est, est_new)
            break
        est = est_new
        xi_old = xi
        z = oracle.lap_solve(T, xi, trans=True, precision=precision)
        j = int(np.argmax(np.abs(z)))
        if k > 0 and np.abs(z).max() <= float((z * x).sum()):
            break
        x = np.zeros(shape)
        x.flat[j] = 1.0
    # alternating test vector b_i = (-1)^i (1 + i / (N - 1))
    idx = np.arange(N)
    b = ((-1.0) ** idx * (1.0 + idx / max(N - 1, 1))).reshape(shape)
    y = oracle.lap_solve(T, b, precision=precision)
    alt = 2.0 * float(np.abs(y).sum()) / (3.0 * N)
    return max(est, alt)


def cond1_estimate(T, shape, precision="ld"):
    return laplace_norm1(T) * inverse_norm1_estimate(T, shape, precision)
