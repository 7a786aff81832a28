"""FP64 oracle for order-p tensors (p >= 3): the t-product extended to p
modes by recursion on the last mode, the tensor nuclear norm over all
Fourier slices and its proximal operator.

TEST INFRASTRUCTURE ONLY (as the rest of the oracle package).

The order-p t-product (the extension the paper's introduction defers to its
reference [6]) is defined recursively: for p = 3 it is the t-product of
Definition 2.1; for p > 3 the frontal "slices" along the last mode are
order-(p-1) tensors and

    C(..., k) = sum_j A(..., j) * B(..., (k - j) mod n_p),

the block-circulant product along mode p (bcirc of order-(p-1) blocks times
the unfolded B), with * the order-(p-1) product.  Unrolling the recursion,
C(:, :, i3, ..., ip) = sum over (j3, ..., jp) of the matrix products
A(:, :, j) B(:, :, (i - j) mod (n3, ..., np)): a multi-dimensional circular
convolution over modes 3..p of frontal-slice matrix products.  A DFT along
each of modes 3..p diagonalises it (the order-p form of eq (10)), which the
second route below uses; the two routes share nothing but numpy.

The nuclear norm and its prox follow Definition 2.9 / eq (14) and
Theorem 2.3 with the DFT over modes 3..p in place of the mode-3 DFT:
||A||_* = (1/rho) sum over all rho = n3 ... np Fourier slices of the matrix
nuclear norms, and Prox_tau applies the matrix SVT with threshold tau to
every Fourier slice (Parseval over modes 3..p makes the proof of
Theorem 2.3 carry over unchanged).
"""
import itertools

import numpy as np


def _tprod3(A, B):
    from . import tprod
    return tprod(A, B)


def tprod_nd(A, B):
    """C = A * B by the recursive definition (block circulant along the last
    mode, the 3-way t-product of the package at the bottom)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.ndim != B.ndim or A.ndim < 3 or A.shape[1] != B.shape[0] or A.shape[2:] != B.shape[2:]:
        raise ValueError(f"shape mismatch {A.shape} {B.shape}")
    if A.ndim == 3:
        return _tprod3(A, B)
    n = A.shape[-1]
    C = np.zeros((A.shape[0], B.shape[1]) + A.shape[2:], dtype=np.float64)
    for k in range(n):
        for j in range(n):
            C[..., k] += tprod_nd(A[..., j], B[..., (k - j) % n])
    return C


def tprod_nd_conv(A, B):
    """The unrolled definition: explicit multi-index circular convolution of
    frontal-slice matrix products (tiny sizes only)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    dims = A.shape[2:]
    C = np.zeros((A.shape[0], B.shape[1]) + dims, dtype=np.float64)
    idx = list(itertools.product(*[range(d) for d in dims]))
    for i in idx:
        acc = np.zeros((A.shape[0], B.shape[1]))
        for j in idx:
            d = tuple((a - b) % n for a, b, n in zip(i, j, dims))
            acc += A[(slice(None), slice(None)) + j] @ B[(slice(None), slice(None)) + d]
        C[(slice(None), slice(None)) + i] = acc
    return C


def _axes(X):
    return tuple(range(2, X.ndim))


def tprod_nd_fft(A, B):
    """C = A * B through the DFT over modes 3..p: Cbar = Abar Bbar per slice."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Ab = np.fft.fftn(A, axes=_axes(A))
    Bb = np.fft.fftn(B, axes=_axes(B))
    Cb = np.einsum("ij...,jl...->il...", Ab, Bb)
    return np.ascontiguousarray(np.fft.ifftn(Cb, axes=_axes(A)).real)


def teye_nd(n, dims):
    """Identity tensor: I(:, :, 1, ..., 1) = I_n, all other frontal slices 0."""
    I = np.zeros((n, n) + tuple(dims), dtype=np.float64)
    I[(slice(None), slice(None)) + (0,) * len(dims)] = np.eye(n)
    return I


def tran_nd(A):
    """Transpose of an order-p real tensor (recursive Definition 2.2): every
    frontal matrix transposed, the frontal indices of modes 3..p negated
    modulo their sizes."""
    A = np.asarray(A, dtype=np.float64)
    At = np.swapaxes(A, 0, 1)
    for ax in range(2, A.ndim):
        n = A.shape[ax]
        At = np.take(At, [(-i) % n for i in range(n)], axis=ax)
    return np.ascontiguousarray(At)


def _slices(Xb):
    """Fourier slices as an array (rho, n1, n2)."""
    n1, n2 = Xb.shape[:2]
    return np.moveaxis(Xb.reshape(n1, n2, -1), 2, 0)


def tnn_nd(A):
    """||A||_* = (1/rho) sum over all rho Fourier slices of sum_i sigma_i."""
    A = np.asarray(A, dtype=np.float64)
    rho = int(np.prod(A.shape[2:]))
    Ab = np.fft.fftn(A, axes=_axes(A))
    return float(sum(np.linalg.svd(S, compute_uv=False).sum() for S in _slices(Ab)) / rho)


def prox_tnn_nd(Y, tau):
    """Prox_tau(Y): the matrix SVT with threshold tau on every Fourier slice."""
    Y = np.asarray(Y, dtype=np.float64)
    Yb = np.fft.fftn(Y, axes=_axes(Y))
    n1, n2 = Y.shape[:2]
    S = _slices(Yb)
    W = np.empty_like(S)
    for k in range(S.shape[0]):
        U, sig, Vh = np.linalg.svd(S[k], full_matrices=False)
        W[k] = (U * np.maximum(sig - tau, 0.0)) @ Vh
    Wb = np.moveaxis(W, 0, 2).reshape(Yb.shape)
    return np.ascontiguousarray(np.fft.ifftn(Wb, axes=_axes(Y)).real)
