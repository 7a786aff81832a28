"""Pins of the FP64 oracle's tensor inverse (Definition 2.4) and T-QR
(Theorem 2.4).  The checks go through the t-product definition (bcirc, no
DFT), numpy's matrix routines for n3 = 1, and closed forms."""
import numpy as np
import pytest

import oracle


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("n,n3", [(5, 4), (6, 7), (3, 1), (8, 2)])
def test_tinv_definition(n, n3):
    A = _rand((n, n, n3), n * 10 + n3)
    B, st = oracle.tinv(A)
    assert st == 0
    I = oracle.teye(n, n3)
    assert np.abs(oracle.tprod(A, B) - I).max() < 1e-10   # eq (11), by the definition of *
    assert np.abs(oracle.tprod(B, A) - I).max() < 1e-10
    if n3 == 1:
        assert np.allclose(B[:, :, 0], np.linalg.inv(A[:, :, 0]), atol=1e-10)


def test_tinv_identity_involution_and_singular():
    I = oracle.teye(4, 5)
    B, st = oracle.tinv(I)
    assert st == 0 and np.abs(B - I).max() < 1e-14
    A = _rand((4, 4, 6), 3)
    B, _ = oracle.tinv(A)
    A2, _ = oracle.tinv(B)
    assert np.abs(A2 - A).max() < 1e-9
    # f-diagonal tensor: its inverse is entrywise on the Fourier diagonals; a
    # tube of zeros on the diagonal makes every Fourier slice singular
    Z = np.zeros((3, 3, 4))
    Z[0, 0, :] = 1.0
    Z[2, 2, :] = 2.0
    _, st = oracle.tinv(Z)
    assert st == 1


@pytest.mark.parametrize("n1,n2,n3", [(6, 4, 5), (4, 6, 4), (5, 5, 3), (7, 3, 1), (3, 7, 2)])
def test_tqr_factorisation(n1, n2, n3):
    A = _rand((n1, n2, n3), n1 * 100 + n2 * 10 + n3)
    Q, R = oracle.tqr(A)
    I = oracle.teye(n1, n3)
    Qh = oracle.tran(Q)
    assert np.abs(oracle.tprod(Qh, Q) - I).max() < 1e-10  # Definition 2.5
    assert np.abs(oracle.tprod(Q, Qh) - I).max() < 1e-10
    assert np.abs(oracle.tprod(Q, R) - A).max() < 1e-10   # eq (22)
    for t in range(n3):                                   # f-upper triangular
        assert np.abs(np.tril(R[:, :, t], -1)).max() < 1e-12
    Rb = np.fft.fft(R, axis=2)                           # diag of each Fourier slice real, >= 0
    for k in range(n3):
        d = np.diagonal(Rb[:, :, k])
        assert np.abs(d.imag).max() < 1e-10 and d.real.min() > -1e-10
    if n3 == 1:  # the matrix case against numpy, rephased to a non-negative diagonal
        q, r = np.linalg.qr(A[:, :, 0], mode="complete")
        sg = np.sign(np.diagonal(r))
        sg[sg == 0] = 1
        D = np.ones(n1)
        D[:len(sg)] = sg
        q, r = q * D, (r.T * D).T
        p = min(n1, n2)
        assert np.allclose(R[:, :, 0], r, atol=1e-10)
        assert np.allclose(Q[:, :p, 0], q[:, :p], atol=1e-10)


def test_tqr_of_orthogonal_and_upper():
    # Q * R with given orthogonal Q and f-upper R of positive Fourier diagonals is returned as is
    A = _rand((4, 4, 3), 11)
    Q0, R0 = oracle.tqr(A)
    Q, R = oracle.tqr(oracle.tprod(Q0, R0))
    assert np.abs(R - R0).max() < 1e-10 and np.abs(Q - Q0).max() < 1e-10
