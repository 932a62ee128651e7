"""CPU oracle (test infrastructure only).

Plain, slow, obviously correct FP64 (and x87 long double) implementations of
what the solver computes, written from the paper's definitions.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may use
this package; the solver library never links, imports or calls it, and this
package never imports the solver.

Paper references (Chen & Kressner, arXiv 1905.09539):
  * mu-mode product and matricization: Sec. 2, eq. (2.1);
  * Laplace-like equation sum_mu X x_mu A_mu = B: eq. (1.4) / (2.2);
    uniqueness iff no eigenvalue sum vanishes (Sec. 2);
  * real Schur (upper quasi-triangular) coefficients: Sec. 2, Algorithm 1;
  * the two-matrices-per-mode family: Conclusions;
  * the second operator class X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d:
    eq. (1.5) / (3.1), Sec. 3 (Algorithms 4-6).

Parity status per function (pins live in tests/test_oracle_pins.py):
  lap_solve ........ pinned (dense Kronecker LU, closed forms, Sylvester,
                     eigenvector right-hand sides, residual)
  lap_solve (trans)  pinned (adjoint identity, dense Kronecker LU of A^T)
  lap_apply ........ pinned (dense Kronecker matrix-vector product)
  mode_product ..... pinned (numpy tensordot)
  pair_solve_direct  pinned (dense Kronecker LU)
  pair_solve_reduced pinned (direct solve, dense Kronecker LU, C = I case)
  grad_T ........... pinned (dense-Kronecker gradient, finite differences)
  flops_tri ........ pinned (closed form d (n-1) N for triangular cubes,
                     brute-force count of multiply-adds)
  dense_solve_with_factors  pinned (dense Kronecker LU of the dense A_mu)
  gsylv_apply ...... pinned (dense Kronecker matrix of eq. (1.5))
  gsylv_solve ...... pinned (dense Kronecker LU, SciPy Sylvester at d = 2,
                     closed form for diagonal coefficients, eigenvector
                     right-hand sides, the shifted Kronecker case eq. (1.6))
  gsylv_dense_solve_with_factors  pinned (dense Kronecker LU of the dense
                     second-class operator)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_impl.h")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO) or any(
            os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC[0], "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        i64p = P(ctypes.c_int64)
        dpp = P(ctypes.c_void_p)
        vp = ctypes.c_void_p
        for sfx in ("_f64", "_ld"):
            getattr(L, "oracle_lap_solve" + sfx).argtypes = [ctypes.c_int, i64p, dpp, vp, vp, ctypes.c_int]
            getattr(L, "oracle_lap_solve" + sfx).restype = ctypes.c_int
            getattr(L, "oracle_lap_apply" + sfx).argtypes = [ctypes.c_int, i64p, dpp, vp, vp, ctypes.c_int]
            getattr(L, "oracle_mode_product" + sfx).argtypes = [ctypes.c_int, i64p, ctypes.c_int, vp, ctypes.c_int64, vp, vp]
            getattr(L, "oracle_pair_apply" + sfx).argtypes = [ctypes.c_int, i64p, dpp, dpp, vp, vp]
            getattr(L, "oracle_pair_solve_direct" + sfx).argtypes = [ctypes.c_int, i64p, dpp, dpp, vp, vp]
            getattr(L, "oracle_pair_solve_direct" + sfx).restype = ctypes.c_int
            getattr(L, "oracle_pair_solve_reduced" + sfx).argtypes = [ctypes.c_int, i64p, dpp, dpp, vp, vp]
            getattr(L, "oracle_pair_solve_reduced" + sfx).restype = ctypes.c_int
            getattr(L, "oracle_gsylv_apply" + sfx).argtypes = [ctypes.c_int, i64p, dpp, vp, vp, vp]
            getattr(L, "oracle_gsylv_solve_direct" + sfx).argtypes = [ctypes.c_int, i64p, dpp, vp, vp, vp]
            getattr(L, "oracle_gsylv_solve_direct" + sfx).restype = ctypes.c_int
            getattr(L, "oracle_grad_T" + sfx).argtypes = [ctypes.c_int, i64p, ctypes.c_int, vp, vp, vp, vp, ctypes.c_int]
        L.oracle_flops_tri.argtypes = [ctypes.c_int, i64p, dpp]
        L.oracle_flops_tri.restype = ctypes.c_double
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


_STATUS = {1: "invalid (coefficient not upper quasi-triangular)", 2: "singular (eigenvalue sum zero)"}


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _shape(x):
    return (ctypes.c_int64 * len(x))(*[int(v) for v in x])


def _ptrs(mats):
    arr = (ctypes.c_void_p * len(mats))(*[m.ctypes.data for m in mats])
    return arr


def _sfx(precision):
    return {"f64": "_f64", "ld": "_ld"}[precision]


def lap_solve(T, B, trans=False, precision="f64"):
    """Unique X with sum_mu X x_mu T_mu = B (trans: T_mu^T), eq. (2.2)."""
    B = _f64(B)
    T = [_f64(t) for t in T]
    X = np.empty_like(B)
    rc = getattr(lib(), "oracle_lap_solve" + _sfx(precision))(
        B.ndim, _shape(B.shape), _ptrs(T), B.ctypes.data, X.ctypes.data, int(bool(trans)))
    if rc:
        raise OracleError(_STATUS.get(rc, str(rc)))
    return X


def lap_apply(T, X, trans=False, precision="f64"):
    """sum_mu X x_mu T_mu (trans: T_mu^T), eq. (2.2)."""
    X = _f64(X)
    T = [_f64(t) for t in T]
    Y = np.empty_like(X)
    getattr(lib(), "oracle_lap_apply" + _sfx(precision))(
        X.ndim, _shape(X.shape), _ptrs(T), X.ctypes.data, Y.ctypes.data, int(bool(trans)))
    return Y


def mode_product(X, M, mu, precision="f64"):
    """X x_mu M with M of shape (m, n_mu): Y_(mu) = M X_(mu) (Sec. 2)."""
    X = _f64(X)
    M = _f64(M)
    shp = list(X.shape)
    assert M.shape[1] == shp[mu]
    out = shp.copy()
    out[mu] = M.shape[0]
    Y = np.empty(out)
    getattr(lib(), "oracle_mode_product" + _sfx(precision))(
        X.ndim, _shape(shp), mu, M.ctypes.data, M.shape[0], X.ctypes.data, Y.ctypes.data)
    return Y


def pair_apply(A, C, X, precision="f64"):
    X = _f64(X)
    A = [_f64(a) for a in A]
    C = [_f64(c) for c in C]
    Y = np.empty_like(X)
    getattr(lib(), "oracle_pair_apply" + _sfx(precision))(
        X.ndim, _shape(X.shape), _ptrs(A), _ptrs(C), X.ctypes.data, Y.ctypes.data)
    return Y


def pair_solve(A, C, B, method="reduced", precision="f64"):
    B = _f64(B)
    A = [_f64(a) for a in A]
    C = [_f64(c) for c in C]
    X = np.empty_like(B)
    fn = getattr(lib(), f"oracle_pair_solve_{method}" + _sfx(precision))
    rc = fn(B.ndim, _shape(B.shape), _ptrs(A), _ptrs(C), B.ctypes.data, X.ctypes.data)
    if rc:
        raise OracleError(_STATUS.get(rc, str(rc)))
    return X


def gsylv_apply(A, C, X, precision="f64"):
    """X x_1 A_1 + X x_1 C x_2 A_2 .. x_d A_d (second class, eq. (3.1));
    A[0], C act on the first mode."""
    X = _f64(X)
    A = [_f64(a) for a in A]
    C = _f64(C)
    Y = np.empty_like(X)
    getattr(lib(), "oracle_gsylv_apply" + _sfx(precision))(
        X.ndim, _shape(X.shape), _ptrs(A), C.ctypes.data, X.ctypes.data, Y.ctypes.data)
    return Y


def gsylv_solve(A, C, B, precision="f64"):
    """Unique X of the second class (eq. (3.1)) with upper quasi-triangular
    A_mu and upper triangular C, by direct element-wise back-substitution
    (O(N^2): small sizes)."""
    B = _f64(B)
    A = [_f64(a) for a in A]
    C = _f64(C)
    X = np.empty_like(B)
    rc = getattr(lib(), "oracle_gsylv_solve_direct" + _sfx(precision))(
        B.ndim, _shape(B.shape), _ptrs(A), C.ctypes.data, B.ctypes.data, X.ctypes.data)
    if rc:
        raise OracleError(_STATUS.get(rc, str(rc)))
    return X


def gsylv_dense_solve_with_factors(Q, S, T, Z, U, Tq, B, precision="f64"):
    """X for the dense second class with known factors (Algorithm 4):
    A_1 = Q S Z^T, C = Q T Z^T, A_mu = U_mu Tq_mu U_mu^T (mu >= 2):
    B~ = B x_1 Q^T x_mu U_mu^T, X~ = gsylv_solve([S, Tq..], T, B~),
    X = X~ x_1 Z x_mu U_mu."""
    W = _f64(B)
    W = mode_product(W, _f64(Q).T.copy(), 0, precision)
    for mu, u in enumerate(U, start=1):
        W = mode_product(W, _f64(u).T.copy(), mu, precision)
    Xt = gsylv_solve([S] + list(Tq), T, W, precision=precision)
    Xt = mode_product(Xt, _f64(Z), 0, precision)
    for mu, u in enumerate(U, start=1):
        Xt = mode_product(Xt, _f64(u), mu, precision)
    return Xt


def grad_T(T, Lam, X, mu, mask=True, precision="f64"):
    """-Lam_(mu) X_(mu)^T, optionally masked to the pattern of T[mu]."""
    Lam = _f64(Lam)
    X = _f64(X)
    t = _f64(T[mu])
    n = t.shape[0]
    dT = np.empty((n, n))
    getattr(lib(), "oracle_grad_T" + _sfx(precision))(
        X.ndim, _shape(X.shape), mu, t.ctypes.data, Lam.ctypes.data, X.ctypes.data,
        dT.ctypes.data, int(bool(mask)))
    return dT


def flops_tri(T, shape):
    T = [_f64(t) for t in T]
    return lib().oracle_flops_tri(len(shape), _shape(shape), _ptrs(T))


def dense_solve_with_factors(Q, T, B, precision="f64"):
    """X for dense A_mu = Q_mu T_mu Q_mu^T (Algorithm 1 with known factors):
    B~ = B x_mu Q_mu^T, X~ = lap_solve(T, B~), X = X~ x_mu Q_mu."""
    W = _f64(B)
    for mu, q in enumerate(Q):
        W = mode_product(W, _f64(q).T.copy(), mu, precision)
    Xt = lap_solve(T, W, precision=precision)
    for mu, q in enumerate(Q):
        Xt = mode_product(Xt, _f64(q), mu, precision)
    return Xt


def pair_dense_solve_with_factors(Q, S, T, Z, B, precision="f64"):
    """X for the dense pair form with known generalized Schur factors
    A_mu = Q_mu S_mu Z_mu^T, C_mu = Q_mu T_mu Z_mu^T (Sec. 3):
    B~ = B x_mu Q_mu^T, X~ = pair_solve(S, T, B~), X = X~ x_mu Z_mu."""
    W = _f64(B)
    for mu, q in enumerate(Q):
        W = mode_product(W, _f64(q).T.copy(), mu, precision)
    Xt = pair_solve(S, T, W, method="reduced", precision=precision)
    for mu, z in enumerate(Z):
        Xt = mode_product(Xt, _f64(z), mu, precision)
    return Xt


def num_threads():
    return lib().oracle_num_threads()


def set_threads(t):
    lib().oracle_set_threads(int(t))
