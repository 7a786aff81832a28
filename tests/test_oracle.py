"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an identity stated in the paper, a worked example of the paper, a
special case that reduces to a textbook or library routine (numpy's FFT and
LAPACK SVD serve only as third opinions here), or brute force on tiny inputs.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def rel(a, b):
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    n = max(np.linalg.norm(np.asarray(b)), 1e-300)
    return d / n


def rand(*shape):
    return RNG.standard_normal(shape)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def dft_matrix(n):
    """F_n of Section 2.2 built from numpy's FFT of the identity (library route)."""
    return np.fft.fft(np.eye(n), axis=0)


# ------------------------------------------------------------------ DFT ----
@pytest.mark.parametrize("n3", [1, 2, 3, 4, 5, 7, 8, 16, 50])
def test_dft_matches_library_fft(orc, n3):
    """eq (2) against numpy's FFT; the inverse against numpy's IFFT (F^*/n, eq (1))."""
    X = crand(3, 4, n3)
    assert rel(orc.dft3(X), np.fft.fft(X, axis=2)) < 1e-13
    assert rel(orc.dft3(X, inverse=True), np.fft.ifft(X, axis=2)) < 1e-13


@pytest.mark.parametrize("n3", [1, 2, 5, 6, 9, 32])
def test_dft_parseval_and_real_symmetry(orc, n3):
    """eq (1) gives ||Abar||_F^2 = n3 ||A||_F^2; eq (8) the conjugate symmetry of
    a real tensor's slices with slice 1 (and the middle slice for even n3) real."""
    A = rand(4, 3, n3)
    Ab = orc.dft3(A)
    assert abs(np.linalg.norm(Ab) ** 2 - n3 * np.linalg.norm(A) ** 2) < 1e-12 * n3 * np.linalg.norm(A) ** 2
    assert np.all(Ab[:, :, 0].imag == 0.0)
    if n3 % 2 == 0:
        assert np.all(Ab[:, :, n3 // 2].imag == 0.0)
    for k in range(1, n3):
        assert np.allclose(Ab[:, :, k], np.conj(Ab[:, :, n3 - k]), atol=1e-12, rtol=0)


def test_dft_roundtrip(orc):
    X = crand(2, 3, 12)
    assert rel(orc.dft3(orc.dft3(X), inverse=True), X) < 1e-14


# --------------------------------------------------------- bcirc, unfold ----
def test_bcirc_block_pattern(orc):
    """eq (6) written out for n3 = 3: block rows [A1 A3 A2], [A2 A1 A3], [A3 A2 A1]."""
    n1, n2, n3 = 2, 2, 3
    A = np.zeros((n1, n2, n3))
    for t in range(n3):
        A[:, :, t] = (t + 1) * 10 + np.arange(n1 * n2).reshape(n1, n2)
    M = orc.bcirc(A)
    S = [A[:, :, t] for t in range(n3)]
    expect = np.block([[S[0], S[2], S[1]], [S[1], S[0], S[2]], [S[2], S[1], S[0]]])
    assert np.array_equal(M, expect)


def test_unfold_fold(orc):
    A = rand(3, 4, 5)
    U = orc.unfold(A)
    assert np.array_equal(U, np.concatenate([A[:, :, t] for t in range(5)], axis=0))
    assert np.array_equal(orc.fold(U, 3, 4, 5), A)


@pytest.mark.parametrize("n3", [1, 2, 3, 4, 7])
def test_block_diagonalisation_eq7(orc, n3):
    """(F (x) I_n1) bcirc(A) (F^{-1} (x) I_n2) is block diagonal with the DFT slices."""
    n1, n2 = 3, 2
    A = rand(n1, n2, n3)
    F = dft_matrix(n3)
    lhs = np.kron(F, np.eye(n1)) @ orc.bcirc(A) @ np.kron(np.linalg.inv(F), np.eye(n2))
    Ab = orc.dft3(A)
    expect = np.zeros((n1 * n3, n2 * n3), dtype=complex)
    for k in range(n3):
        expect[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = Ab[:, :, k]
    assert np.abs(lhs - expect).max() < 1e-12 * max(1.0, np.abs(expect).max())


# --------------------------------------------------------------- tprod -----
def test_tprod_equals_fold_bcirc_unfold(orc):
    """Definition 2.1 (eq (9)) with the product formed by numpy's matmul."""
    A, B = rand(4, 3, 5), rand(3, 6, 5)
    C = orc.fold(orc.bcirc(A) @ orc.unfold(B), 4, 6, 5)
    assert rel(orc.tprod(A, B), C) < 1e-14


@pytest.mark.parametrize("n3", [1, 2, 3, 8, 11])
def test_tprod_is_circular_convolution(orc, n3):
    """n1 = n2 = l = 1: the t-product of two tubes is their circular convolution
    (eq (3)), computed here with numpy's FFT."""
    a, b = rand(1, 1, n3), rand(1, 1, n3)
    conv = np.real(np.fft.ifft(np.fft.fft(a[0, 0]) * np.fft.fft(b[0, 0])))
    assert rel(orc.tprod(a, b)[0, 0], conv) < 1e-13
    assert rel(orc.tprod_fft(a, b)[0, 0], conv) < 1e-13


def test_tprod_algorithm1_equals_definition_exhaustive(orc):
    """Algorithm 1 (FFT route, eq (10)) equals Definition 2.1 on every tiny shape."""
    for n1, n2, l in itertools.product([1, 2, 3], repeat=3):
        for n3 in range(1, 9):
            A, B = rand(n1, n2, n3), rand(n2, l, n3)
            ref = orc.tprod(A, B)
            assert rel(orc.tprod_fft(A, B), ref) < 1e-12, (n1, n2, l, n3)


def test_tprod_entries(orc):
    A, B = rand(5, 4, 6), rand(4, 3, 6)
    C = orc.tprod(A, B)
    idx = RNG.choice(C.size, 40, replace=False)
    assert rel(orc.tprod_entries(A, B, idx), C.reshape(-1)[idx]) < 1e-14


@pytest.mark.parametrize("n3", [1, 4, 5])
def test_identity_tensor(orc, n3):
    """Definition 2.3: A*I = A, I*A = A, and every DFT slice of I is the identity."""
    A = rand(3, 4, n3)
    assert rel(orc.tprod(A, orc.teye(4, n3)), A) < 1e-15
    assert rel(orc.tprod(orc.teye(3, n3), A), A) < 1e-15
    Ib = orc.dft3(orc.teye(3, n3))
    for k in range(n3):
        assert np.allclose(Ib[:, :, k], np.eye(3), atol=1e-15)


def test_tran_worked_example(orc):
    """Definition 2.2, the worked example for n3 = 4 (golden fixture)."""
    n1, n2, n3 = 2, 3, 4
    A = np.zeros((n1, n2, n3))
    for s in range(n3):
        A[:, :, s] = 10 * (s + 1) + np.arange(n1 * n2).reshape(n1, n2)
    blocks, cur = [], []
    with open(os.path.join(GOLDEN, "tran_n3_4.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("slice"):
                if cur:
                    blocks.append(np.array(cur, dtype=float))
                cur = []
            else:
                cur.append([float(v) for v in line.split()])
    blocks.append(np.array(cur, dtype=float))
    At = orc.tran(A)
    assert At.shape == (n2, n1, n3)
    for s in range(n3):
        assert np.array_equal(At[:, :, s], blocks[s])


@pytest.mark.parametrize("n3", [1, 2, 5, 6])
def test_transpose_reverses_product(orc, n3):
    """(A*B)^* = B^* * A^*: tran maps each DFT slice to its conjugate transpose
    (Definition 2.2 with eq (10)), so the order of the product reverses."""
    A, B = rand(3, 4, n3), rand(4, 2, n3)
    lhs = orc.tran(orc.tprod(A, B))
    rhs = orc.tprod(orc.tran(B), orc.tran(A))
    assert rel(lhs, rhs) < 1e-13
    assert np.array_equal(orc.tran(orc.tran(A)), A)
    Ab, Atb = orc.dft3(A), orc.dft3(orc.tran(A))
    for k in range(n3):
        assert np.allclose(Atb[:, :, k], Ab[:, :, k].conj().T, atol=1e-12)


def test_tprod_associative(orc):
    A, B, C = rand(3, 4, 5), rand(4, 2, 5), rand(2, 3, 5)
    assert rel(orc.tprod(orc.tprod(A, B), C), orc.tprod(A, orc.tprod(B, C))) < 1e-13


# ----------------------------------------------------------------- SVD -----
def test_svd_textbook_2x2(orc):
    """[[3,0],[4,5]]: A^T A = [[25,20],[20,25]] has eigenvalues 45 and 5."""
    U, s, V, rc = orc.svd(np.array([[3.0, 0.0], [4.0, 5.0]]))
    assert rc >= 1
    assert np.allclose(s, [np.sqrt(45.0), np.sqrt(5.0)], rtol=1e-15, atol=0)


def test_svd_diagonal_and_zero(orc):
    D = np.diag([0.5, -3.0, 2.0]).astype(complex)
    U, s, V, _ = orc.svd(D)
    assert np.allclose(s, [3.0, 2.0, 0.5], rtol=1e-15)
    U, s, V, _ = orc.svd(np.zeros((4, 3)), full=True)
    assert np.all(s == 0)
    assert np.allclose(U.conj().T @ U, np.eye(4), atol=1e-15)
    assert np.allclose(V.conj().T @ V, np.eye(3), atol=1e-15)


@pytest.mark.parametrize("m,n,cplx", [(6, 4, True), (4, 6, True), (5, 5, True), (7, 3, False),
                                      (3, 7, False), (1, 5, True), (5, 1, True), (30, 20, True)])
def test_svd_against_lapack(orc, m, n, cplx):
    M = crand(m, n) if cplx else rand(m, n)
    for full in (False, True):
        U, s, V, rc = orc.svd(M, full=full)
        assert rc >= 0
        assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-13, atol=1e-14)
        p = min(m, n)
        assert rel((U[:, :p] * s) @ V[:, :p].conj().T, M) < 1e-13
        assert np.abs(U.conj().T @ U - np.eye(U.shape[1])).max() < 1e-13
        assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-13
        if not cplx:
            assert np.all(U.imag == 0) and np.all(V.imag == 0)


def test_svd_rank_deficient(orc):
    X = crand(8, 3) @ crand(3, 6)
    U, s, V, rc = orc.svd(X, full=True)
    assert np.allclose(s, np.linalg.svd(X, compute_uv=False), rtol=1e-12, atol=1e-12)
    assert np.abs(U.conj().T @ U - np.eye(8)).max() < 1e-12
    assert np.abs(V.conj().T @ V - np.eye(6)).max() < 1e-12
    assert rel((U[:, :6] * s) @ V.conj().T, X) < 1e-13


# ---------------------------------------------------------------- t-SVD ----
@pytest.mark.parametrize("n1,n2,n3", [(4, 3, 5), (3, 4, 4), (4, 4, 1), (5, 2, 6), (2, 5, 3)])
def test_tsvd_invariants(orc, n1, n2, n3):
    """Theorem 2.2 / Algorithm 2: A = U*S*V^*, U and V orthogonal (Definition 2.5),
    S f-diagonal (Definition 2.6), eq (13) ordering and eq (14) averaging."""
    A = rand(n1, n2, n3)
    U, S, V, mi, rc = orc.tsvd(A)
    assert rc == 0 and mi < 1e-13
    assert rel(orc.tprod(orc.tprod(U, S), orc.tran(V)), A) < 1e-12
    for Q, n in ((U, n1), (V, n2)):
        assert rel(orc.tprod(orc.tran(Q), Q), orc.teye(n, n3)) < 1e-12
        assert rel(orc.tprod(Q, orc.tran(Q)), orc.teye(n, n3)) < 1e-12
    off = S.copy()
    p = min(n1, n2)
    for i in range(p):
        off[i, i, :] = 0
    assert np.abs(off).max() < 1e-13
    d = np.array([S[i, i, 0] for i in range(p)])
    assert np.all(np.diff(d) <= 1e-13) and np.all(d >= -1e-13)
    sig = orc.slice_sigma(A)
    assert np.allclose(d, sig.mean(axis=0), rtol=1e-12, atol=1e-13)
    assert np.allclose(sig, np.stack([np.linalg.svd(orc.dft3(A)[:, :, k], compute_uv=False)
                                      for k in range(n3)]), rtol=1e-12, atol=1e-13)


def test_tsvd_low_tubal_rank(orc):
    P, Q = rand(6, 2, 4), rand(2, 5, 4)
    A = orc.tprod(P, Q)
    U, S, V, mi, rc = orc.tsvd(A)
    assert rel(orc.tprod(orc.tprod(U, S), orc.tran(V)), A) < 1e-12
    assert rel(orc.tprod(orc.tran(U), U), orc.teye(6, 4)) < 1e-12
    # Definition 2.7 / eq (16): tubal rank 2
    d = np.array([S[i, i, 0] for i in range(5)])
    assert np.all(d[:2] > 1e-3) and np.all(np.abs(d[2:]) < 1e-12 * d[0])


# ---------------------------------------------------------- tnn and tsn ----
@pytest.mark.parametrize("n1,n2,n3", [(3, 4, 5), (4, 4, 1), (2, 3, 6), (5, 2, 2)])
def test_tnn_brute_force_bcirc(orc, n1, n2, n3):
    """Definition 2.9 with eq (14): tnn = (1/n3) ||bcirc(A)||_* (the 1/n3 reading
    of eq (18)); brute force by LAPACK on bcirc(A) with no DFT at all."""
    A = rand(n1, n2, n3)
    nuc = np.linalg.svd(orc.bcirc(A), compute_uv=False).sum()
    assert abs(orc.tnn(A) - nuc / n3) < 1e-12 * nuc
    U, S, V, _, _ = orc.tsvd(A)
    assert abs(orc.tnn(A) - sum(S[i, i, 0] for i in range(min(n1, n2)))) < 1e-12 * nuc


@pytest.mark.parametrize("n,n3", [(1, 1), (3, 4), (5, 7)])
def test_tnn_tsn_identity(orc, n, n3):
    Ie = orc.teye(n, n3)
    assert abs(orc.tnn(Ie) - n) < 1e-13
    assert abs(orc.tsn(Ie) - 1.0) < 1e-14


def test_tnn_matrix_case(orc):
    M = rand(5, 3)
    assert abs(orc.tnn(M[:, :, None]) - np.linalg.svd(M, compute_uv=False).sum()) < 1e-13


@pytest.mark.parametrize("n1,n2,n3", [(3, 4, 5), (2, 2, 6)])
def test_tsn_brute_force_bcirc(orc, n1, n2, n3):
    """Definition 2.8 with eq (17): ||bcirc(A)||."""
    A = rand(n1, n2, n3)
    assert abs(orc.tsn(A) - np.linalg.norm(orc.bcirc(A), 2)) < 1e-12 * orc.tsn(A)


# ----------------------------------------------------------------- prox ----
def _bcirc_svt(orc, Y, tau):
    """SVT of the real matrix bcirc(Y) by LAPACK, read back as a tensor through
    its first block column; also returns how far the result is from block
    circulant.  No DFT is involved."""
    n1, n2, n3 = Y.shape
    M = orc.bcirc(Y)
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    Xb = (U * np.maximum(s - tau, 0.0)) @ Vh
    X = np.zeros_like(Y)
    for t in range(n3):
        X[:, :, t] = Xb[t * n1:(t + 1) * n1, 0:n2]
    return X, np.abs(Xb - orc.bcirc(X)).max()


@pytest.mark.parametrize("n1,n2,n3,tau", [(3, 4, 5, 0.7), (4, 3, 4, 1.5), (3, 3, 1, 0.5),
                                          (2, 5, 6, 0.3), (4, 4, 3, 0.0)])
def test_prox_brute_force_bcirc(orc, n1, n2, n3, tau):
    """bcirc(Prox_tau(Y)) = SVT_tau(bcirc(Y)): eq (19) scaled by n3 through eq (7)
    and Parseval, so the matrix SVT of bcirc(Y) is the brute-force answer."""
    Y = rand(n1, n2, n3)
    Xb, circ_err = _bcirc_svt(orc, Y, tau)
    assert circ_err < 1e-12
    assert rel(orc.prox_tnn(Y, tau), Xb) < 1e-12


def test_prox_identity_closed_form(orc):
    Ie = orc.teye(4, 6)
    for tau in (0.0, 0.25, 1.0, 3.0):
        assert np.abs(orc.prox_tnn(Ie, tau) - max(1 - tau, 0) * Ie).max() < 1e-14


def test_prox_zero_above_spectral_norm(orc):
    Y = rand(3, 5, 4)
    X = orc.prox_tnn(Y, orc.tsn(Y) * 1.0001)
    assert np.abs(X).max() < 1e-13


def test_prox_matrix_case(orc):
    M = rand(5, 4)
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    expect = (U * np.maximum(s - 0.8, 0)) @ Vh
    assert rel(orc.prox_tnn(M[:, :, None], 0.8)[:, :, 0], expect) < 1e-13
    assert rel(orc.svt_real(M, 0.8), expect) < 1e-13


@pytest.mark.parametrize("n3", [1, 4, 7])
def test_prox_tube_soft_threshold(orc, n3):
    """n1 = n2 = 1: each DFT bin is a 1x1 slice, so the prox soft-thresholds the
    modulus of every bin, z (1 - tau/|z|)_+ (numpy FFT as the library route)."""
    y = rand(1, 1, n3)
    z = np.fft.fft(y[0, 0])
    tau = 0.6 * np.median(np.abs(z))
    w = z * np.maximum(0.0, 1.0 - tau / np.maximum(np.abs(z), 1e-300))
    assert rel(orc.prox_tnn(y, tau)[0, 0], np.real(np.fft.ifft(w))) < 1e-13


def test_prox_optimality(orc):
    """eq (19): the prox minimises tau*tnn(X) + 0.5 ||X - Y||_F^2."""
    Y, tau = rand(4, 3, 5), 0.9
    X = orc.prox_tnn(Y, tau)

    def f(Z):
        return tau * orc.tnn(Z) + 0.5 * np.linalg.norm(Z - Y) ** 2

    f0 = f(X)
    for _ in range(20):
        D = rand(4, 3, 5)
        for eps in (1e-2, 1e-4):
            assert f(X + eps * D) >= f0 - 1e-12


def test_prox_nonexpansive(orc):
    Y1, Y2 = rand(3, 4, 6), rand(3, 4, 6)
    d = np.linalg.norm(orc.prox_tnn(Y1, 0.8) - orc.prox_tnn(Y2, 0.8))
    assert d <= np.linalg.norm(Y1 - Y2) * (1 + 1e-12)


def test_prox_rejects_negative_tau(orc):
    with pytest.raises(ValueError):
        orc.prox_tnn(rand(2, 2, 2), -1.0)


@pytest.mark.parametrize("n1,n2,n3,r", [(7, 6, 5, 3), (5, 9, 4, 2), (6, 6, 1, 4), (8, 5, 6, 5)])
def test_tubalrank_of_product(orc, n1, n2, n3, r):
    """Definition 2.7: P * Q with P n1 x r x n3, Q r x n2 x n3 generic has tubal
    rank r (every Fourier slice has rank r)."""
    rng = np.random.default_rng(n1 * 10 + r)
    A = orc.tprod(rng.standard_normal((n1, r, n3)), rng.standard_normal((r, n2, n3)))
    assert orc.tubalrank(A) == r


def test_tubalrank_special_cases(orc):
    """teye(n, n3) has tubal rank n, the zero tensor 0, and for n3 = 1 the
    tubal rank is the matrix rank (numpy)."""
    assert orc.tubalrank(orc.teye(4, 3)) == 4
    assert orc.tubalrank(np.zeros((3, 4, 2))) == 0
    rng = np.random.default_rng(2)
    M = rng.standard_normal((6, 2)) @ rng.standard_normal((2, 5))
    assert orc.tubalrank(M[:, :, None]) == np.linalg.matrix_rank(M) == 2
    # singular tubes are formed per rank position across the Fourier slices
    # (each slice's values sorted), so the tubal rank is the largest slice
    # rank, not the number of nonzero tubes of A: here the DC slice holds one
    # tube and the Nyquist slice the other, each slice has rank 1
    A = np.zeros((3, 3, 4))
    A[0, 0, :] = [1.0, -1.0, 1.0, -1.0]  # energy only at the Nyquist bin
    A[1, 1, :] = 1.0                     # only at DC
    assert orc.tubalrank(A) == 1
    A[1, 1, :] = [1.0, 1.0, -1.0, -1.0]  # now bins 1 and 3: a second slice with rank 1
    A[2, 2, :] = 1.0                     # and DC again: DC rank 1, Nyquist rank 1
    assert orc.tubalrank(A) == 1
    A[2, 2, :] = [1.0, -1.0, 1.0, -1.0]  # the Nyquist slice now has rank 2
    assert orc.tubalrank(A) == 2


# ---------------------------------------------------------------------------
# The library-primitive form of the exact prox (numpy FFT + LAPACK SVD per
# slice), used for full-size checks, against the Jacobi oracle and against
# the SVT of bcirc(Y) (no DFT at all: the prox of eq (19) is the matrix SVT
# of the block circulant matrix, eq (18) and Theorem 2.3).
@pytest.mark.parametrize("n1,n2,n3", [(9, 7, 5), (6, 11, 4), (8, 8, 1), (5, 5, 2)])
def test_prox_lapack_matches_jacobi_and_bcirc(orc, n1, n2, n3):
    rng = np.random.default_rng(n1 + 10 * n2 + 100 * n3)
    Y = rng.standard_normal((n1, n2, n3))
    tau = 0.3 * orc.tsn(Y)
    X = orc.prox_tnn_lapack(Y, tau)
    ref = orc.prox_tnn(Y, tau)
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)
    U, s, Vh = np.linalg.svd(orc.bcirc(Y))
    Wb = (U[:, :len(s)] * np.maximum(s - tau, 0)) @ Vh[:len(s)]
    # first block column of the circulant result = unfold(X)
    assert np.linalg.norm(Wb[:, :n2] - orc.unfold(X)) <= 1e-12 * np.linalg.norm(ref)
    k = n3 // 2
    part = orc.prox_tnn_lapack(Y, tau, slices=[k])
    assert np.allclose(part[k], np.fft.fft(ref, axis=2)[:, :, k], atol=1e-12 * np.linalg.norm(ref))
