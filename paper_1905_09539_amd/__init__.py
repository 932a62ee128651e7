"""Python binding of libtt.so, the MI355X (gfx950) solver for linear systems
with Kronecker product structure (Chen & Kressner, arXiv 1905.09539).

This module only marshals arguments: every step of the solve runs in the HIP
kernels of libtt.so (see include/tt.h).  PyTorch provides device memory and
streams.  There is no CPU fallback: if libtt.so is missing, importing the
solver functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libtt.so")

TT_OK, TT_EINVAL, TT_ESINGULAR, TT_ENOMEM, TT_EHIP, TT_ENOTCONV = range(6)
TT_FP64, TT_MP_FP32, TT_MP_BF16 = 0, 1, 2


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


_STATUS = {0: "TT_OK", 1: "TT_EINVAL", 2: "TT_ESINGULAR", 3: "TT_ENOMEM", 4: "TT_EHIP", 5: "TT_ENOTCONV"}


class Opts(ctypes.Structure):
    _fields_ = [("nmin", ctypes.c_int), ("prec", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("deterministic", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("info", ctypes.c_double * 4)]


_lib = None

# exported C symbols declared in include/tt.h
SYMBOLS = [
    "tt_opts_default", "tt_status_str", "tt_last_error", "solve_tri_tensor",
    "solve_general_tensor", "solve_backward", "solve_tri_tensor_batched",
    "solve_backward_batched", "tt_plan_create", "tt_plan_create_batched", "tt_plan_solve",
    "tt_plan_solve_batched", "tt_plan_status", "tt_plan_flops", "tt_plan_destroy",
    "tt_schedule_info", "tt_schedule_info_class", "tt_plan_profile", "tt_plan_profile_waves", "tt_plan_create_general", "tt_plan_info", "tt_schur_host", "tt_qz_host",
    "tt_plan_create_general_pair", "tt_plan_coefficient_grads", "tt_plan_solve_graph",
    "tt_copy_device", "tt_workspace_bytes", "solve_tri_tensor_noalloc",
    "solve_gsylv_tensor", "solve_gsylv_general_tensor", "tt_plan_create_gsylv", "tt_plan_create_gsylv_general",
    "tt_merge_modes_host",
]


def lib():
    """Load libtt.so (built by build.py / __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise ImportError(f"{_SO} is missing: build it with python -m paper_1905_09539_amd.build")
        L = ctypes.CDLL(_SO)
        vp, i64p, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)
        L.tt_last_error.restype = ctypes.c_char_p
        L.tt_status_str.restype = ctypes.c_char_p
        L.tt_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.tt_workspace_bytes.argtypes = [ctypes.c_int, i64p, ctypes.c_int]
        L.tt_workspace_bytes.restype = ctypes.c_size_t
        L.solve_tri_tensor.argtypes = [ctypes.c_int, i64p, vp, vp, vp, vp, ctypes.POINTER(Opts)]
        L.solve_tri_tensor_noalloc.argtypes = [ctypes.c_int, i64p, vp, vp, vp, vp, ctypes.POINTER(Opts)]
        L.solve_gsylv_tensor.argtypes = [ctypes.c_int, i64p, vp, vp, vp, vp, ctypes.POINTER(Opts)]
        L.solve_gsylv_general_tensor.argtypes = [ctypes.c_int, i64p, vp, vp, vp, vp, ctypes.POINTER(Opts)]
        L.tt_plan_create_gsylv.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, vp, vp, ctypes.POINTER(Opts)]
        L.tt_plan_create_gsylv_general.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, vp, vp,
                                                   ctypes.POINTER(Opts)]
        L.solve_general_tensor.argtypes = [ctypes.c_int, i64p, vp, vp, vp, ctypes.POINTER(Opts)]
        L.solve_backward.argtypes = [ctypes.c_int, i64p, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(Opts)]
        L.solve_tri_tensor_batched.argtypes = [ctypes.c_int, ip, vp, vp, vp, vp, ctypes.POINTER(Opts)]
        L.solve_backward_batched.argtypes = [ctypes.c_int, ip, vp, vp, vp, vp, vp, vp, ctypes.c_int,
                                             ctypes.POINTER(Opts)]
        L.tt_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, vp, vp, ctypes.c_int,
                                     ctypes.POINTER(Opts)]
        L.tt_plan_create_batched.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ip, vp, vp, ctypes.c_int,
                                             ctypes.POINTER(Opts)]
        L.tt_plan_solve.argtypes = [vp, vp, vp, vp]
        L.tt_plan_solve_graph.argtypes = [vp, vp, vp, vp]
        L.tt_copy_device.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.tt_plan_solve_batched.argtypes = [vp, vp, vp, vp]
        L.tt_plan_status.argtypes = [vp]
        L.tt_plan_flops.argtypes = [vp]
        L.tt_plan_flops.restype = ctypes.c_double
        L.tt_plan_destroy.argtypes = [vp]
        L.tt_plan_profile.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.tt_schedule_info.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.tt_schedule_info_class.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_double)]
        L.tt_plan_create_general.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, vp, ctypes.POINTER(Opts)]
        L.tt_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.tt_schur_host.argtypes = [ctypes.c_int, vp, vp, vp]
        L.tt_merge_modes_host.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, vp]
        L.tt_qz_host.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.tt_plan_coefficient_grads.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp]
        L.tt_plan_create_general_pair.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64p, vp, vp,
                                                  ctypes.POINTER(Opts)]
        L.tt_plan_profile_waves.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                            ctypes.c_int64]
        _lib = L
    return _lib


def _check(rc):
    if rc != TT_OK:
        raise TTError(rc, lib().tt_last_error().decode())


def _shape(shape):
    return (ctypes.c_int64 * len(shape))(*[int(x) for x in shape])


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


def _dev(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _opts(nmin=0, prec=TT_FP64, tol=1e-13, max_iter=10, stream=None, workspace=None):
    o = Opts()
    lib().tt_opts_default(ctypes.byref(o))
    o.nmin, o.prec, o.tol, o.max_iter = int(nmin), int(prec), float(tol), int(max_iter)
    o.stream = _stream(stream).value
    if workspace is not None:
        import torch
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.is_contiguous()):
            raise TypeError("workspace must be a contiguous CUDA tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def workspace_bytes(shape, prec=TT_FP64):
    """Device bytes that one single-problem solve_tri / solve_general /
    solve_backward call of this shape and precision needs at most
    (tt_workspace_bytes); pass a CUDA tensor of at least this size as
    workspace= and the call allocates no device memory."""
    return int(lib().tt_workspace_bytes(len(shape), _shape(shape), int(prec)))


def solve_tri(T, B, C=None, X=None, nmin=0, prec=TT_FP64, tol=1e-13, max_iter=10, stream=None, info=None,
              workspace=None):
    """Solve sum_mu X x_mu T_mu = B (Laplace-like form, eq. (2.2)) or, with
    C given, the pair form sum_mu X x_1 C_1 .. x_mu T_mu .. x_d C_d = B.
    T, C: lists of n_mu x n_mu float64 CUDA tensors (T upper quasi-triangular,
    C upper triangular); B: float64 CUDA tensor of shape (n_1, ..., n_d).
    prec=TT_MP_FP32 (TT_MP_BF16): FP32-MFMA (split-BF16 MFMA) updates with
    FP64 leaves and FP64 refinement (info, if a dict,
    receives iterations and the last correction ratio).  workspace: an
    optional CUDA tensor of at least workspace_bytes(B.shape, prec) bytes
    from which every device buffer of the call is carved."""
    import torch
    if X is None:
        X = torch.empty_like(B)
    tp = _ptr_array([_dev(t) for t in T])
    cp = _ptr_array([_dev(c) for c in C]) if C is not None else None
    o = _opts(nmin=nmin, prec=prec, tol=tol, max_iter=max_iter, stream=stream, workspace=workspace)
    rc = lib().solve_tri_tensor(B.dim(), _shape(B.shape), tp, cp, _dev(B), _dev(X), ctypes.byref(o))
    if info is not None:
        info.update(iterations=int(o.info[0]), ratio=o.info[1], host_seconds=o.info[2])
    _check(rc)
    return X


def solve_tri_noalloc(T, B, X, C=None, nmin=0, stream=None):
    """solve_tri through solve_tri_tensor_noalloc: no device allocation in
    the library (its buffers live in a fixed 64 MiB scratch array per GPU);
    X must be given (float64 CUDA tensor shaped like B)."""
    tp = _ptr_array([_dev(t) for t in T])
    cp = _ptr_array([_dev(c) for c in C]) if C is not None else None
    o = _opts(nmin=nmin, stream=stream)
    _check(lib().solve_tri_tensor_noalloc(B.dim(), _shape(B.shape), tp, cp, _dev(B), _dev(X), ctypes.byref(o)))
    return X


def solve_gsylv(A, C, B, X=None, nmin=0, stream=None, workspace=None):
    """Second operator class (eq. (3.1)): X x_1 A_1 + X x_1 C x_2 A_2 .. x_d
    A_d = B with upper quasi-triangular A_mu and upper triangular C, all
    float64 CUDA tensors (C acts on the first mode)."""
    import torch
    if X is None:
        X = torch.empty_like(B)
    ap = _ptr_array([_dev(a) for a in A])
    o = _opts(nmin=nmin, stream=stream, workspace=workspace)
    _check(lib().solve_gsylv_tensor(B.dim(), _shape(B.shape), ap, ctypes.c_void_p(_dev(C)), _dev(B), _dev(X),
                                    ctypes.byref(o)))
    return X


def solve_gsylv_general(A, C, B, X=None, nmin=0, stream=None, workspace=None):
    """Second operator class with dense HOST coefficients (Algorithm 4: host
    QZ of (A_1, C) and real Schur of A_2 .. A_d, GPU transforms and solve)."""
    import torch
    if X is None:
        X = torch.empty_like(B)
    mats, ap = _host_mats(A)
    Cm = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    o = _opts(nmin=nmin, stream=stream, workspace=workspace)
    _check(lib().solve_gsylv_general_tensor(B.dim(), _shape(B.shape), ap, ctypes.c_void_p(Cm.ctypes.data), _dev(B),
                                            _dev(X), ctypes.byref(o)))
    return X


def _host_mats(A):
    mats = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in A]
    return mats, _ptr_array([m.ctypes.data for m in mats])


def solve_general(A, B, X=None, nmin=0, prec=TT_FP64, tol=1e-13, max_iter=10, stream=None, info=None,
                  workspace=None):
    """Algorithm 1: solve sum_mu X x_mu A_mu = B for dense A_mu given as HOST
    (numpy) n_mu x n_mu arrays; B: float64 CUDA tensor.  Host Schur, then
    transforms and the triangular solve on the GPU."""
    import torch
    if X is None:
        X = torch.empty_like(B)
    mats, ap = _host_mats(A)
    o = _opts(nmin=nmin, prec=prec, tol=tol, max_iter=max_iter, stream=stream, workspace=workspace)
    rc = lib().solve_general_tensor(B.dim(), _shape(B.shape), ap, _dev(B), _dev(X), ctypes.byref(o))
    if info is not None:
        info.update(iterations=int(o.info[0]), ratio=o.info[1], host_seconds=o.info[2])
    _check(rc)
    return X


# the dense-coefficient solve under its short name
solve = solve_general


def refine(A, B, X=None, prec=TT_MP_FP32, tol=1e-13, max_iter=10, dense=True, stream=None):
    """Mixed-precision solve with FP64 iterative refinement (solve_general, or
    solve_tri with dense=False and device triangular A); returns X and a dict
    with the refinement iterations and the last correction ratio."""
    info = {}
    if dense:
        X = solve_general(A, B, X=X, prec=prec, tol=tol, max_iter=max_iter, stream=stream, info=info)
    else:
        X = solve_tri(A, B, X=X, prec=prec, tol=tol, max_iter=max_iter, stream=stream, info=info)
    return X, info


def solve_backward(T, X, G, dB=None, grads=True, dense_grad=False, nmin=0, stream=None, workspace=None):
    """Adjoint of solve_tri for L with dL/dX = G: returns (dB, dT) with
    dB = Lam solving sum_mu Lam x_mu T_mu^T = G and dT[mu] = -Lam_(mu) X_(mu)^T
    (masked to the pattern of T[mu] unless dense_grad); dT is None if not grads."""
    import torch
    if dB is None:
        dB = torch.empty_like(G)
    tp = _ptr_array([_dev(t) for t in T])
    dT = [torch.empty_like(t) for t in T] if grads else None
    dtp = _ptr_array([_dev(t) for t in dT]) if grads else None
    o = _opts(nmin=nmin, stream=stream, workspace=workspace)
    _check(lib().solve_backward(G.dim(), _shape(G.shape), tp, ctypes.c_void_p(_dev(X)) if grads else None,
                                _dev(G), _dev(dB), dtp, int(bool(dense_grad)), ctypes.byref(o)))
    return dB, dT


def solve_backward_batched(T, X, G, grads=True, dense_grad=False, nmin=0, stream=None):
    """Batched solve_backward over independent problems (lists of per-problem
    coefficient lists and tensors).  Returns (list of dB, list of dT lists)."""
    import torch
    count = len(G)
    ds = (ctypes.c_int * count)(*[g.dim() for g in G])
    shp = [_shape(g.shape) for g in G]
    shp_arr = (ctypes.c_void_p * count)(*[ctypes.cast(x, ctypes.c_void_p).value for x in shp])
    tarrs = [_ptr_array([_dev(t) for t in Tb]) for Tb in T]
    t_arr = (ctypes.c_void_p * count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in tarrs])
    dB = [torch.empty_like(g) for g in G]
    dT = [[torch.empty_like(t) for t in Tb] for Tb in T] if grads else None
    dtarrs = [_ptr_array([_dev(t) for t in l]) for l in dT] if grads else None
    dt_arr = (ctypes.c_void_p * count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in dtarrs]) if grads else None
    o = _opts(nmin=nmin, stream=stream)
    _check(lib().solve_backward_batched(count, ds, shp_arr, t_arr, _ptr_array([_dev(x) for x in X]),
                                        _ptr_array([_dev(g) for g in G]), _ptr_array([_dev(b) for b in dB]),
                                        dt_arr, int(bool(dense_grad)), ctypes.byref(o)))
    return dB, dT


def schur_host(A):
    """Host real Schur decomposition A = U T U^T (numpy in, numpy out)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n = A.shape[0]
    T = np.zeros_like(A)
    U = np.zeros_like(A)
    _check(lib().tt_schur_host(n, A.ctypes.data, T.ctypes.data, U.ctypes.data))
    return T, U


def merge_modes_host(Ta, Tb):
    """Host merge of two adjacent modes (Algorithm 3, real quasi-triangular
    case): returns (Tm, V, perm) with Ta (x) I + I (x) Tb = V Tm V^T, Tm upper
    quasi-triangular, perm the perfect-shuffle order (numpy in, numpy out)."""
    Ta = np.ascontiguousarray(np.asarray(Ta, dtype=np.float64))
    Tb = np.ascontiguousarray(np.asarray(Tb, dtype=np.float64))
    na, nb = Ta.shape[0], Tb.shape[0]
    Tm = np.zeros((na * nb, na * nb))
    V = np.zeros_like(Tm)
    perm = np.zeros(na * nb, dtype=np.int32)
    _check(lib().tt_merge_modes_host(na, Ta.ctypes.data, nb, Tb.ctypes.data, Tm.ctypes.data, V.ctypes.data,
                                     perm.ctypes.data))
    return Tm, V, perm


def qz_host(A, C):
    """Host real generalized Schur decomposition A = Q S Z^T, C = Q T Z^T
    (numpy in, numpy out: S, T, Q, Z)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    n = A.shape[0]
    S, T, Q, Z = (np.zeros_like(A) for _ in range(4))
    _check(lib().tt_qz_host(n, A.ctypes.data, C.ctypes.data, S.ctypes.data, T.ctypes.data, Q.ctypes.data,
                            Z.ctypes.data))
    return S, T, Q, Z


class Plan:
    """A reusable schedule for solving with fixed coefficients (tt_plan_*).
    T: device coefficient list (C: optional device list for the pair form);
    general=True takes T (and C, for the pair form) as HOST dense matrices
    (Algorithm 1 pipeline; with C: host QZ, Sec. 3)."""

    def __init__(self, T, shape=None, nmin=0, trans=False, batch_T=None, batch_shapes=None, C=None,
                 general=False, prec=TT_FP64, tol=1e-13, max_iter=10, gsylv=False):
        self._h = ctypes.c_void_p()
        o = _opts(nmin=nmin, prec=prec, tol=tol, max_iter=max_iter)
        if gsylv:
            # second operator class (eq. (3.1)): T = A_1 .. A_d, C acts on mode 1
            self.count = 1
            self.shapes = [tuple(int(x) for x in shape)]
            if general:
                mats, ap = _host_mats(T)
                Cm = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
                self._keep = [mats, ap, Cm]
                _check(lib().tt_plan_create_gsylv_general(ctypes.byref(self._h), len(shape), _shape(shape), ap,
                                                          ctypes.c_void_p(Cm.ctypes.data), ctypes.byref(o)))
            else:
                self._keep = [_ptr_array([_dev(t) for t in T])]
                _check(lib().tt_plan_create_gsylv(ctypes.byref(self._h), len(shape), _shape(shape), self._keep[0],
                                                  ctypes.c_void_p(_dev(C)), ctypes.byref(o)))
        elif general and C is not None:
            mats, ap = _host_mats(T)
            cmats, cp = _host_mats(C)
            self._keep = [mats, ap, cmats, cp]
            self.count = 1
            self.shapes = [tuple(int(x) for x in shape)]
            _check(lib().tt_plan_create_general_pair(ctypes.byref(self._h), len(shape), _shape(shape), ap, cp,
                                                     ctypes.byref(o)))
        elif general:
            mats, ap = _host_mats(T)
            self._keep = [mats, ap]
            self.count = 1
            self.shapes = [tuple(int(x) for x in shape)]
            _check(lib().tt_plan_create_general(ctypes.byref(self._h), len(shape), _shape(shape), ap,
                                                ctypes.byref(o)))
        elif batch_T is None:
            self._keep = [_ptr_array([_dev(t) for t in T])]
            cp = None
            if C is not None:
                cp = _ptr_array([_dev(c) for c in C])
                self._keep.append(cp)
            self.count = 1
            self.shapes = [tuple(int(x) for x in shape)]
            _check(lib().tt_plan_create(ctypes.byref(self._h), len(shape), _shape(shape), self._keep[0], cp,
                                        int(bool(trans)), ctypes.byref(o)))
        else:
            self.count = len(batch_T)
            self.shapes = [tuple(int(x) for x in s) for s in batch_shapes]
            ds = (ctypes.c_int * self.count)(*[len(s) for s in self.shapes])
            shp = [_shape(s) for s in self.shapes]
            shp_arr = (ctypes.c_void_p * self.count)(*[ctypes.cast(s, ctypes.c_void_p).value for s in shp])
            tarrs = [_ptr_array([_dev(t) for t in Tb]) for Tb in batch_T]
            t_arr = (ctypes.c_void_p * self.count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in tarrs])
            self._keep = [shp, tarrs]
            _check(lib().tt_plan_create_batched(ctypes.byref(self._h), self.count, ds, shp_arr, t_arr,
                                                int(bool(trans)), ctypes.byref(o)))

    @property
    def flops(self):
        return lib().tt_plan_flops(self._h)

    def solve(self, B, X=None, stream=None, graph=False):
        """Enqueue the solve (no host synchronisation).  graph=True replays
        the launch sequence from a HIP graph recorded on the first call for
        the same (B, X, stream) (single-problem FP64 plans, on a created,
        non-default stream)."""
        import torch
        if self.count == 1:
            if X is None:
                X = torch.empty_like(B)
            fn = lib().tt_plan_solve_graph if graph else lib().tt_plan_solve
            _check(fn(self._h, ctypes.c_void_p(_dev(B)), ctypes.c_void_p(_dev(X)), _stream(stream)))
            return X
        if X is None:
            X = [torch.empty_like(b) for b in B]
        bp = _ptr_array([_dev(b) for b in B])
        xp = _ptr_array([_dev(x) for x in X])
        _check(lib().tt_plan_solve_batched(self._h, bp, xp, _stream(stream)))
        return X

    def coefficient_grads(self, T, X, Lam, dT=None, dense_grad=False, stream=None):
        """dT[mu] = -Lam_(mu) X_(mu)^T (masked to the pattern of T[mu] unless
        dense_grad) for every problem of this triangular plan.  Single plans:
        T a coefficient list, X and Lam tensors; batched plans: lists of
        those.  Returns dT (lists of n_mu x n_mu tensors)."""
        import torch
        single = self.count == 1 and torch.is_tensor(X)
        Tb, Xb, Lb = ([T], [X], [Lam]) if single else (T, X, Lam)
        if dT is None:
            dT = [[torch.empty_like(t) for t in Ti] for Ti in Tb]
        elif single:
            dT = [dT]
        tarrs = [_ptr_array([_dev(t) for t in Ti]) for Ti in Tb]
        darrs = [_ptr_array([_dev(t) for t in Di]) for Di in dT]
        t_arr = (ctypes.c_void_p * len(tarrs))(*[ctypes.cast(a, ctypes.c_void_p).value for a in tarrs])
        d_arr = (ctypes.c_void_p * len(darrs))(*[ctypes.cast(a, ctypes.c_void_p).value for a in darrs])
        _check(lib().tt_plan_coefficient_grads(self._h, t_arr, _ptr_array([_dev(x) for x in Xb]),
                                               _ptr_array([_dev(l) for l in Lb]), d_arr, int(bool(dense_grad)),
                                               _stream(stream)))
        return dT[0] if single else dT

    def profile(self, B, X, stream=None, serial=False):
        """Run one solve with timing events around every launch (on the
        launch's own stream; serial=True puts every launch on one stream, so
        each kernel runs alone); returns per kernel class ("leaf", "update")
        the summed launch milliseconds, algorithmic flops, algorithmic HBM
        bytes and launch count, and "solve_ms" (first leaf launch to the end
        of the last update)."""
        out = (ctypes.c_double * 12)()
        _check(lib().tt_plan_profile(self._h, ctypes.c_void_p(_dev(B)), ctypes.c_void_p(_dev(X)),
                                     _stream(stream), int(bool(serial)), out))
        res = {}
        for k, name in enumerate(["leaf", "update"]):
            res[name] = {"ms": out[4 * k], "flops": out[4 * k + 1], "bytes": out[4 * k + 2],
                         "launches": int(out[4 * k + 3])}
        res["solve_ms"] = out[8]
        return res

    def profile_waves(self, B, X, waves, stream=None, serial=False):
        """Per-wave timeline of one profiled solve: a list with, for each of
        the plan's `waves` hyperplane waves, a dict of the leaf launch's and
        the update launch's start/end (ms from the first leaf launch, None
        for an empty launch), its leaf blocks and its update tiles."""
        out = (ctypes.c_double * (6 * waves))()
        _check(lib().tt_plan_profile_waves(self._h, ctypes.c_void_p(_dev(B)), ctypes.c_void_p(_dev(X)),
                                           _stream(stream), int(bool(serial)), out, ctypes.c_int64(waves)))
        res = []
        for k in range(waves):
            o = out[6 * k:6 * k + 6]
            res.append({"leaf": None if o[0] < 0 else (o[0], o[1]),
                        "update": None if o[2] < 0 else (o[2], o[3]),
                        "leaves": int(o[4]), "tiles": int(o[5])})
        return res

    def status(self):
        _check(lib().tt_plan_status(self._h))

    def info(self):
        out = (ctypes.c_double * 4)()
        _check(lib().tt_plan_info(self._h, out))
        return {"iterations": int(out[0]), "ratio": out[1], "build_seconds": out[2], "schur_seconds": out[3]}

    def close(self):
        if self._h:
            lib().tt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_device(src, dst, stream=None):
    """dst <- src (same-size contiguous float64 device tensors) with the
    library's copy kernel (the benchmark's byte-counter reference)."""
    if src.numel() != dst.numel():
        raise ValueError("copy_device: sizes differ")
    _check(lib().tt_copy_device(ctypes.c_void_p(_dev(src)), ctypes.c_void_p(_dev(dst)), src.numel(),
                                _stream(stream)))


def schedule_info(T_host, shape, nmin=0, cls=0):
    """Host-only: statistics and dependency check of the solve schedule for
    coefficients given as numpy arrays (no GPU needed); cls 1: the schedule
    of the second operator class (tt_schedule_info_class)."""
    Th = [np.ascontiguousarray(t, dtype=np.float64) for t in T_host]
    out = (ctypes.c_double * 14)()
    _check(lib().tt_schedule_info_class(len(shape), _shape(shape), _ptr_array([t.ctypes.data for t in Th]),
                                        int(nmin), int(cls), out))
    keys = ["flops", "flops_leaf", "flops_update", "waves", "leaves", "tasks", "items", "launches",
            "bmax0", "bmax1", "bmax2", "bmax3", "dependency_violation", "plan_bytes"]
    return dict(zip(keys, list(out)))


class _PlanCache:
    """Reusable plans keyed by the coefficient tensors themselves: an entry
    holds weak references to its T tensors and their in-place versions, so
    it is used only while the same tensors, unmodified, are passed again
    (a freed tensor whose memory is reused never matches)."""

    def __init__(self, cap=8):
        self.cap = cap
        self.entries = []  # (refs, versions, shape, trans, plan), newest last
        self.misses = 0    # plans built so far

    def get(self, T, shape, trans):
        import weakref
        shape = tuple(int(x) for x in shape)
        vers = tuple(t._version for t in T)
        for i, (refs, v, shp, tr, plan) in enumerate(self.entries):
            if tr == trans and shp == shape and v == vers and len(refs) == len(T) and \
                    all(r() is t for r, t in zip(refs, T)):
                self.entries.append(self.entries.pop(i))
                return plan
        plan = Plan(list(T), shape, trans=trans)
        self.misses += 1
        self.entries.append(([weakref.ref(t) for t in T], vers, shape, trans, plan))
        while len(self.entries) > self.cap:
            self.entries.pop(0)[4].close()
        return plan


_plans = None


def _plan_cache():
    global _plans
    if _plans is None:
        _plans = _PlanCache()
    return _plans


def _autograd_class():
    import torch

    class TriTensorSolve(torch.autograd.Function):
        """X = solve_tri(T, B) with gradients: dL/dB = Lam (adjoint solve)
        and dL/dT_mu = -Lam_(mu) X_(mu)^T masked to the pattern of T_mu.
        Usage: X = TriTensorSolve.apply(B, T_1, ..., T_d).  The forward plan
        and the adjoint plan (T_mu^T, reversed order) are built once per set
        of coefficient tensors and reused while those tensors are unchanged."""

        @staticmethod
        def forward(ctx, B, *T):
            T = [t.contiguous() for t in T]
            plan = _plan_cache().get(T, B.shape, False)
            X = plan.solve(B.contiguous())
            plan.status()
            ctx.save_for_backward(X, *T)
            return X

        @staticmethod
        def backward(ctx, G):
            X, *T = ctx.saved_tensors
            need_T = any(ctx.needs_input_grad[1:])
            planb = _plan_cache().get(T, X.shape, True)
            dB = planb.solve(G.contiguous())
            dT = planb.coefficient_grads(T, X, dB) if need_T else [None] * len(T)
            planb.status()
            return (dB,) + tuple(dT)

    return TriTensorSolve


def __getattr__(name):
    if name == "TriTensorSolve":
        cls = _autograd_class()
        globals()["TriTensorSolve"] = cls
        return cls
    raise AttributeError(name)
