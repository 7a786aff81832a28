"""FP64 CPU oracle for the t-product toolbox (Lu, 2018).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU product path never does.
It shares no code with the GPU library: the C sources here are compiled with
gcc into ``liboracle.so`` and follow the paper's definitions and algorithms in
double precision (see the header of ``tp_oracle.c`` for the readings taken).

Arrays are numpy, C-contiguous, with the tube index last: a real tensor of
size n1 x n2 x n3 is ``np.ndarray((n1, n2, n3), float64)``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "or_set_threads": (None, [_I]),
        "or_get_threads": (_I, []),
        "or_dft3": (None, [_D, _I, _I, _I, _I, _D]),
        "or_bcirc": (None, [_D, _I, _I, _I, _D]),
        "or_unfold": (None, [_D, _I, _I, _I, _D]),
        "or_fold": (None, [_D, _I, _I, _I, _D]),
        "or_tprod_def": (None, [_D, _D, _I, _I, _I, _I, _D]),
        "or_tprod_def_entries": (None, [_D, _D, _I, _I, _I, _I,
                                        ctypes.POINTER(ctypes.c_longlong), ctypes.c_longlong, _D]),
        "or_tprod_fft": (None, [_D, _D, _I, _I, _I, _I, _D]),
        "or_tran": (None, [_D, _I, _I, _I, _D]),
        "or_teye": (None, [_I, _I, _D]),
        "or_svd": (_I, [_D, _I, _I, _I, _D, _D, _D]),
        "or_tsvd": (_I, [_D, _I, _I, _I, _D, _D, _D, _D]),
        "or_slice_sigma": (_I, [_D, _I, _I, _I, _D]),
        "or_tnn": (ctypes.c_double, [_D, _I, _I, _I]),
        "or_tsn": (ctypes.c_double, [_D, _I, _I, _I]),
        "or_tubalrank": (_I, [_D, _I, _I, _I, ctypes.c_double, ctypes.c_double]),
        "or_prox_tnn": (_I, [_D, _I, _I, _I, ctypes.c_double, _D]),
        "or_svt_real": (_I, [_D, _I, _I, ctypes.c_double, _D]),
        "or_tqr": (_I, [_D, _I, _I, _I, _D, _D]),
        "or_tinv": (_I, [_D, _I, _I, _D]),
        "or_trpca": (_I, [_D, _I, _I, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, _I, _D, _D, _D, ctypes.POINTER(ctypes.c_int)]),
    }
    U32 = ctypes.POINTER(ctypes.c_uint)
    IP = ctypes.POINTER(ctypes.c_int)
    sig.update({
        "or_philox4x32_10": (None, [U32, U32, U32]),
        "or_sketch_matrix": (None, [_I, _I, _I, _I, ctypes.c_ulonglong, _D]),
        "or_cholqr2": (_I, [_D, _I, _I, _I, _D]),
        "or_prox_tnn_rsvd": (_I, [_D, _I, _I, _I, ctypes.c_double, IP, _I, _I, _I, ctypes.c_ulonglong, _D, IP, IP]),
        "or_slice_features": (None, [_D, _I, _I, _I, ctypes.c_double, IP, _D, _D]),
        "or_mlp_param_count": (_I, [_I, _I]),
        "or_mlp_forward": (None, [_D, _I, _I, _D, _I, _D]),
        "or_mlp_loss_grad": (ctypes.c_double, [_D, _I, _I, _D, _D, _I, ctypes.c_double, _D]),
    })
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _real(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cplx(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def get_threads() -> int:
    return int(_load().or_get_threads())


def dft3(X, inverse=False):
    """eq (2) along mode 3 (or F^*/n3 of eq (1) when inverse)."""
    X = _cplx(X)
    n1, n2, n3 = X.shape
    Y = np.empty_like(X)
    _load().or_dft3(_dp(X), n1, n2, n3, int(bool(inverse)), _dp(Y))
    return Y


def bcirc(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    M = np.empty((n1 * n3, n2 * n3))
    _load().or_bcirc(_dp(A), n1, n2, n3, _dp(M))
    return M


def unfold(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    M = np.empty((n1 * n3, n2))
    _load().or_unfold(_dp(A), n1, n2, n3, _dp(M))
    return M


def fold(M, n1, n2, n3):
    M = _real(M)
    assert M.shape == (n1 * n3, n2)
    A = np.empty((n1, n2, n3))
    _load().or_fold(_dp(M), n1, n2, n3, _dp(A))
    return A


def tprod(A, B):
    """Definition 2.1 (eq (9)) evaluated block row by block row."""
    A, B = _real(A), _real(B)
    n1, n2, n3 = A.shape
    assert B.shape[0] == n2 and B.shape[2] == n3
    l = B.shape[1]
    C = np.empty((n1, l, n3))
    _load().or_tprod_def(_dp(A), _dp(B), n1, n2, l, n3, _dp(C))
    return C


def tprod_entries(A, B, flat_idx):
    """eq (9) at flat indices (i*l + j)*n3 + t of C."""
    A, B = _real(A), _real(B)
    n1, n2, n3 = A.shape
    l = B.shape[1]
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.shape[0])
    _load().or_tprod_def_entries(_dp(A), _dp(B), n1, n2, l, n3,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                                 idx.shape[0], _dp(out))
    return out


def tprod_fft(A, B):
    """Algorithm 1 in FP64 (plain DFT, no FFT)."""
    A, B = _real(A), _real(B)
    n1, n2, n3 = A.shape
    l = B.shape[1]
    C = np.empty((n1, l, n3))
    _load().or_tprod_fft(_dp(A), _dp(B), n1, n2, l, n3, _dp(C))
    return C


def tran(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    At = np.empty((n2, n1, n3))
    _load().or_tran(_dp(A), n1, n2, n3, _dp(At))
    return At


def teye(n, n3):
    Ie = np.empty((n, n, n3))
    _load().or_teye(n, n3, _dp(Ie))
    return Ie


def svd(M, full=False):
    """One-sided Jacobi SVD of a complex (or real) matrix: (U, sigma, V, sweeps)."""
    M = _cplx(M)
    m, n = M.shape
    p = min(m, n)
    sig = np.empty(p)
    U = np.empty((m, m if full else p), dtype=np.complex128)
    V = np.empty((n, n if full else p), dtype=np.complex128)
    rc = _load().or_svd(_dp(M), m, n, int(bool(full)), _dp(sig), _dp(U), _dp(V))
    return U, sig, V, rc


def tsvd(A):
    """Algorithm 2: returns (U, S, V, max_imag, status)."""
    A = _real(A)
    n1, n2, n3 = A.shape
    U = np.empty((n1, n1, n3))
    S = np.empty((n1, n2, n3))
    V = np.empty((n2, n2, n3))
    mi = ctypes.c_double(0.0)
    rc = _load().or_tsvd(_dp(A), n1, n2, n3, _dp(U), _dp(S), _dp(V), ctypes.byref(mi))
    return U, S, V, mi.value, rc


def slice_sigma(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    sig = np.empty((n3, min(n1, n2)))
    _load().or_slice_sigma(_dp(A), n1, n2, n3, _dp(sig))
    return sig


def tnn(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    return float(_load().or_tnn(_dp(A), n1, n2, n3))


def tsn(A):
    A = _real(A)
    n1, n2, n3 = A.shape
    return float(_load().or_tsn(_dp(A), n1, n2, n3))


def tubalrank(A, tol=-1.0, eps=2.0 ** -23):
    """Definition 2.7 with the tolerance of tp_tubalrank (tol < 0: max(n1,n2) eps S(1,1,1))."""
    A = _real(A)
    n1, n2, n3 = A.shape
    return int(_load().or_tubalrank(_dp(A), n1, n2, n3, float(tol), float(eps)))


def prox_tnn(Y, tau):
    """Algorithm 3 (t-SVT) in FP64."""
    Y = _real(Y)
    n1, n2, n3 = Y.shape
    X = np.empty_like(Y)
    rc = _load().or_prox_tnn(_dp(Y), n1, n2, n3, float(tau), _dp(X))
    if rc < 0:
        raise ValueError("tau must be >= 0")
    return X


def prox_tnn_lapack(Y, tau, slices=None):
    """Theorem 2.3 (eq (20)-(21)) written out with library primitives, for
    sizes where the Jacobi oracle above takes too long (1024 x 1024 slices):
    numpy's FFT along mode 3, numpy's (LAPACK) SVD of each of the
    floor(n3/2)+1 leading Fourier slices, W = U (S - tau)_+ V^*, the trailing
    slices as the conjugates (eq (8)), inverse FFT.  FP64 throughout.
    With `slices` (a list of slice indices k < floor(n3/2)+1) only those
    slices are computed and returned as {k: W^(k)} (Fourier domain), for
    sampled checks of a full-size result."""
    Y = _real(Y)
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    F = np.fft.fft(Y, axis=2)

    def svt(k):
        A = F[:, :, k]
        if k == 0 or (n3 % 2 == 0 and k == n3 // 2):
            A = A.real  # the real slices (eq (4)); a real SVD
        U, s, Vh = np.linalg.svd(A, full_matrices=False)
        d = np.maximum(s - tau, 0.0)
        keep = d > 0
        return (U[:, keep] * d[keep]) @ Vh[keep, :]

    if slices is not None:
        return {int(k): svt(int(k)) for k in slices}
    W = np.empty((n1, n2, n3), dtype=np.complex128)
    for k in range(h):
        W[:, :, k] = svt(k)
    for k in range(h, n3):
        W[:, :, k] = np.conj(W[:, :, n3 - k])
    return np.ascontiguousarray(np.fft.ifft(W, axis=2).real)


def tqr(A):
    """Theorem 2.4: A = Q * R (FP64), Q orthogonal, R f-upper triangular with
    real non-negative diagonals of its Fourier slices.  Returns (Q, R)."""
    A = _real(A)
    n1, n2, n3 = A.shape
    Q = np.empty((n1, n1, n3))
    R = np.empty((n1, n2, n3))
    _load().or_tqr(_dp(A), n1, n2, n3, _dp(Q), _dp(R))
    return Q, R


def tinv(A):
    """Definition 2.4: the inverse of a square tensor (FP64).  Returns (B,
    status) with status 0, or 1 + the first singular Fourier slice."""
    A = _real(A)
    n, n2, n3 = A.shape
    if n != n2:
        raise ValueError("tinv needs n x n x n3")
    B = np.empty_like(A)
    rc = _load().or_tinv(_dp(A), n, n3, _dp(B))
    return B, int(rc)


def trpca(X, lam=None, mu=1e-3, rho=1.1, mu_max=1e10, tol=1e-5, max_iter=500):
    """Tensor robust PCA by the inexact ALM around prox_tnn, in FP64.
    lam defaults to 1/sqrt(max(n1, n2) n3).  Returns dict(L, S, Lam, iters,
    converged)."""
    X = _real(X)
    n1, n2, n3 = X.shape
    if lam is None:
        lam = 1.0 / np.sqrt(max(n1, n2) * n3)
    L, S, Lam = np.empty_like(X), np.empty_like(X), np.empty_like(X)
    it = ctypes.c_int(0)
    rc = _load().or_trpca(_dp(X), n1, n2, n3, float(lam), float(mu), float(rho), float(mu_max), float(tol),
                          int(max_iter), _dp(L), _dp(S), _dp(Lam), ctypes.byref(it))
    if rc < 0:
        raise ValueError("bad TRPCA argument")
    return dict(L=L, S=S, Lam=Lam, iters=it.value, converged=bool(rc))


def svt_real(M, tau):
    M = _real(M)
    m, n = M.shape
    out = np.empty_like(M)
    _load().or_svt_real(_dp(M), m, n, float(tau), _dp(out))
    return out


# ---------------------------------------------------------- learned rank --
def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11): 4 counter words, 2 key words -> 4 words."""
    c = (ctypes.c_uint * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint * 4)()
    _load().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def sketch_matrix(n, l, slice_index, real, seed):
    Om = np.empty((n, l), dtype=np.complex128)
    _load().or_sketch_matrix(n, l, slice_index, int(bool(real)), int(seed), _dp(Om))
    return Om


def cholqr2(Y, lact=None):
    """CholeskyQR2 of Y (m x l): returns (Q, R, status)."""
    Q = _cplx(Y).copy()
    m, l = Q.shape
    R = np.empty((l, l), dtype=np.complex128)
    st = _load().or_cholqr2(_dp(Q), m, l, l if lact is None else int(lact), _dp(R))
    return Q, R, st


def prox_tnn_rsvd(Y, tau, kpred, oversample=10, power=2, lfull=None, seed=0):
    """Randomized-SVD prox (see tp_oracle.h): returns (X, fallback, rank)."""
    Y = _real(Y)
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    kp = np.ascontiguousarray(kpred, dtype=np.int32)
    assert kp.shape == (h,)
    X = np.empty_like(Y)
    fb = np.zeros(h, dtype=np.int32)
    rk = np.zeros(h, dtype=np.int32)
    IP = ctypes.POINTER(ctypes.c_int)
    if lfull is None:
        lfull = min(n1, n2) + 1
    st = _load().or_prox_tnn_rsvd(_dp(Y), n1, n2, n3, float(tau), kp.ctypes.data_as(IP), int(oversample),
                                  int(power), int(lfull), int(seed), _dp(X), fb.ctypes.data_as(IP),
                                  rk.ctypes.data_as(IP))
    if st < 0:
        raise ValueError("tau must be >= 0")
    return X, fb, rk


def mlp_param_count(d, h):
    return int(_load().or_mlp_param_count(d, h))


def mlp_forward(params, X, d, h):
    X = _real(X)
    y = np.empty(X.shape[0])
    _load().or_mlp_forward(_dp(_real(params)), d, h, _dp(X), X.shape[0], _dp(y))
    return y


def mlp_loss_grad(params, X, t, d, h, under=4.0):
    params = _real(params)
    X, t = _real(X), _real(t)
    g = np.empty_like(params)
    loss = _load().or_mlp_loss_grad(_dp(params), d, h, _dp(X), _dp(t), X.shape[0], float(under), _dp(g))
    return float(loss), g


def slice_features(Y, tau, prev=None, prev_sigma=None):
    Y = _real(Y)
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    f = np.empty((h, 12))
    IP = ctypes.POINTER(ctypes.c_int)
    pv = None if prev is None else np.ascontiguousarray(prev, dtype=np.int32)
    ps = None if prev_sigma is None else _real(prev_sigma)
    _load().or_slice_features(_dp(Y), n1, n2, n3, float(tau), None if pv is None else pv.ctypes.data_as(IP),
                              None if ps is None else _dp(ps), _dp(f))
    return f


# order-p tensors (numpy; see nd.py)
from .nd import prox_tnn_nd, teye_nd, tnn_nd, tprod_nd, tprod_nd_conv, tprod_nd_fft, tran_nd  # noqa: E402,F401
