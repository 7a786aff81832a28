"""Pins of the learned-rank part of the oracle: the counter-based generator,
CholeskyQR2, the randomized prox against the exact prox of Theorem 2.3 where
the two must agree, and the MLP gradient against central differences."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(777)


def test_philox_known_answers(orc):
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_sketch_matrix_statistics(orc):
    Om = orc.sketch_matrix(2000, 40, 3, False, 12345)
    assert abs(Om.real.mean()) < 0.01 and abs(Om.imag.mean()) < 0.01
    assert abs((np.abs(Om) ** 2).mean() - 1.0) < 0.02   # E|z|^2 = 1 for (z0 + i z1)/sqrt(2)
    R = orc.sketch_matrix(2000, 40, 3, True, 12345)
    assert np.all(R.imag == 0) and abs((R.real ** 2).mean() - 1.0) < 0.02
    # counter based: a sub-block is the same whatever the matrix size
    assert np.array_equal(orc.sketch_matrix(10, 5, 3, False, 12345), Om[:10, :5])
    assert not np.array_equal(orc.sketch_matrix(10, 5, 4, False, 12345), Om[:10, :5])


@pytest.mark.parametrize("m,l", [(50, 7), (300, 40), (64, 64)])
def test_cholqr2(orc, m, l):
    Y = RNG.standard_normal((m, l)) + 1j * RNG.standard_normal((m, l))
    Q, R, st = orc.cholqr2(Y)
    assert st == 0
    assert np.abs(Q.conj().T @ Q - np.eye(l)).max() < 1e-13
    assert np.abs(Q @ R - Y).max() < 1e-11 * np.abs(Y).max()
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R).real > 0) and np.allclose(np.diag(R).imag, 0)
    # same R as Householder QR up to column phases (textbook uniqueness)
    _, Rh = np.linalg.qr(Y)
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rh)), rtol=1e-10)


def test_cholqr2_inactive_columns(orc):
    Y = np.zeros((30, 8), dtype=complex)
    Y[:, :5] = RNG.standard_normal((30, 5))
    Q, R, st = orc.cholqr2(Y, lact=5)
    assert st == 0 and np.all(Q[:, 5:] == 0)
    assert np.abs(Q[:, :5].conj().T @ Q[:, :5] - np.eye(5)).max() < 1e-13


def lowrank(orc, n1, n2, n3, r, seed):
    rng = np.random.default_rng(seed)
    return orc.tprod(rng.standard_normal((n1, r, n3)), rng.standard_normal((r, n2, n3)))


@pytest.mark.parametrize("n1,n2,n3,r", [(40, 30, 6, 3), (25, 40, 5, 4), (32, 32, 4, 6)])
def test_rsvd_prox_exact_on_low_rank(orc, n1, n2, n3, r):
    """Every Fourier slice has rank r <= l: the range finder captures the whole
    range, so the randomized prox equals the exact prox (Theorem 2.3)."""
    Y = lowrank(orc, n1, n2, n3, r, seed=n1 + r)
    h = n3 // 2 + 1
    tau = 0.3 * orc.tsn(Y)
    kpred = np.full(h, r, dtype=np.int32)
    X, fb, rk = orc.prox_tnn_rsvd(Y, tau, kpred, oversample=5, power=2, seed=9)
    assert np.all(fb == 0)
    ref = orc.prox_tnn(Y, tau)
    assert np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)
    sig = orc.slice_sigma(Y)[:h]
    assert np.array_equal(rk, (sig > tau).sum(axis=1))


def test_rsvd_prox_check_forces_fallback(orc):
    """k = 0 predicted on full-rank slices with small tau: the check
    sigma_(k+1) < tau fails on every slice and the full SVD is used."""
    Y = RNG.standard_normal((20, 16, 5))
    h = 3
    tau = 0.05 * orc.tsn(Y)
    X, fb, rk = orc.prox_tnn_rsvd(Y, tau, np.zeros(h, dtype=np.int32), oversample=3, power=2, seed=1)
    assert np.all(fb == 1)
    assert np.linalg.norm(X - orc.prox_tnn(Y, tau)) <= 1e-12 * np.linalg.norm(Y)


def test_rsvd_prox_full_width_and_cap(orc):
    Y = RNG.standard_normal((12, 10, 4))
    h = 3
    tau = 0.2 * orc.tsn(Y)
    ref = orc.prox_tnn(Y, tau)
    X, fb, _ = orc.prox_tnn_rsvd(Y, tau, np.full(h, 10, dtype=np.int32), oversample=2, power=1, seed=3)
    assert np.all(fb == 0) and np.linalg.norm(X - ref) <= 1e-9 * np.linalg.norm(ref)   # l = min(n1,n2)
    X, fb, _ = orc.prox_tnn_rsvd(Y, tau, np.full(h, 4, dtype=np.int32), oversample=2, power=1, lfull=6, seed=3)
    assert np.all(fb == 1) and np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)  # l >= lfull


def test_mlp_closed_forms(orc):
    d, h = 3, 4
    npar = orc.mlp_param_count(d, h)
    assert npar == h * d + h + 2 * (h * h + h) + h + 1
    p = np.zeros(npar)
    p[-1] = 0.75                       # b4 only: y = b4
    X = RNG.standard_normal((5, d))
    assert np.allclose(orc.mlp_forward(p, X, d, h), 0.75)
    # single path x0 -> relu -> relu -> relu -> y
    p = np.zeros(npar)
    W1 = 0
    b1 = h * d
    W2 = b1 + h
    b2 = W2 + h * h
    W3 = b2 + h
    b3 = W3 + h * h
    w4 = b3 + h
    p[W1 + 0] = 1.0
    p[W2 + 0] = 1.0
    p[W3 + 0] = 1.0
    p[w4 + 0] = 2.0
    X = np.array([[1.5, 3, 3], [-2.0, 1, 1]])
    assert np.allclose(orc.mlp_forward(p, X, d, h), [3.0, 0.0])


def test_mlp_gradient_central_differences(orc):
    d, h, N = 5, 6, 17
    npar = orc.mlp_param_count(d, h)
    p = RNG.standard_normal(npar) * 0.5
    X = RNG.standard_normal((N, d))
    t = RNG.standard_normal(N)
    loss, g = orc.mlp_loss_grad(p, X, t, d, h, under=4.0)
    eps = 1e-6
    num = np.empty(npar)
    for i in range(npar):
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        num[i] = (orc.mlp_loss_grad(pp, X, t, d, h, 4.0)[0] - orc.mlp_loss_grad(pm, X, t, d, h, 4.0)[0]) / (2 * eps)
    assert np.abs(num - g).max() <= 1e-6 * max(1.0, np.abs(g).max())
    # the loss weighs under-prediction `under` times more
    y = orc.mlp_forward(p, X, d, h)
    e = y - t
    assert abs(loss - np.mean(np.where(e >= 0, 1.0, 4.0) * e * e)) < 1e-12 * max(1.0, loss)


# ---------------------------------------------------------------------------
# Power iterations of the randomized prox outside the exact regime: a
# Gaussian tensor has a slowly decaying spectrum in every Fourier slice, so
# with l well below the rank the result depends on the number of subspace
# iterations q.  The oracle must agree with an independent numpy subspace
# iteration started from the same sketch Om (Householder QR instead of
# CholeskyQR2: the projector Q Q^* does not depend on how the basis is
# orthonormalised), and the q = 0, 1, 2 results must differ from each other
# and approach the exact prox as q grows.
def numpy_rsvd_prox(orc, Y, tau, l, q, seed):
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    F = np.fft.fft(Y, axis=2)
    W = np.zeros_like(F)
    for k in range(h):
        real = k == 0 or (n3 % 2 == 0 and k == n3 // 2)
        A = F[:, :, k].real.astype(complex) if real else F[:, :, k]
        Om = orc.sketch_matrix(n2, l, k, real, seed)
        Q = np.linalg.qr(A @ Om)[0]
        for _ in range(q):
            Z = np.linalg.qr(A.conj().T @ Q)[0]
            Q = np.linalg.qr(A @ Z)[0]
        U, s, Vh = np.linalg.svd(Q.conj().T @ A, full_matrices=False)
        W[:, :, k] = Q @ (U * np.maximum(s - tau, 0.0)) @ Vh
    for k in range(h, n3):
        W[:, :, k] = W[:, :, n3 - k].conj()
    return np.fft.ifft(W, axis=2).real


@pytest.mark.parametrize("n1,n2,n3", [(60, 50, 5), (48, 64, 6)])
def test_rsvd_prox_power_iterations_vs_numpy(orc, n1, n2, n3):
    rng = np.random.default_rng(n1 * n2 + n3)
    Y = rng.standard_normal((n1, n2, n3))
    h = n3 // 2 + 1
    tau = 0.45 * orc.tsn(Y)
    l = 8                       # l < rank = min(n1, n2): not exact
    kpred = np.full(h, l, dtype=np.int32)
    exact = orc.prox_tnn(Y, tau)
    res = {}
    for q in (0, 1, 2):
        # oversample 0: l = kpred, so the count check never sends a slice to the full SVD
        X, fb, _ = orc.prox_tnn_rsvd(Y, tau, kpred, oversample=0, power=q, seed=21)
        assert np.all(fb == 0)
        ref = numpy_rsvd_prox(orc, Y, tau, l, q, seed=21)
        assert np.linalg.norm(X - ref) <= 1e-10 * np.linalg.norm(ref), q
        res[q] = X
    # the iterations matter here (far above the agreement tolerance), and help
    assert np.linalg.norm(res[0] - res[1]) > 1e-3 * np.linalg.norm(exact)
    assert np.linalg.norm(res[1] - res[2]) > 1e-4 * np.linalg.norm(exact)
    e = [np.linalg.norm(res[q] - exact) for q in (0, 1, 2)]
    assert e[2] < e[1] < e[0]


# ---------------------------------------------------------------------------
# Slice features (the rank model's inputs, a definition of this build) on
# inputs whose Fourier slices are known in closed form.
def test_slice_features_identity_tensor(orc):
    n, n3 = 7, 6
    tau = 0.3
    f = orc.slice_features(orc.teye(n, n3), tau)
    h = n3 // 2 + 1
    # every Fourier slice of the identity tensor is I_n: ||.||_F = sqrt(n), column norms 1
    assert np.allclose(f[:, 0], np.log(tau))            # log(tau / (sqrt(n) / sqrt(n)))
    assert np.allclose(f[:, 1], np.log(1.0 / tau))
    assert np.all(f[:, 2:4] == 0) and np.all(f[:, 8:] == 0)
    assert np.allclose(f[:, 4], np.arange(h) / (n3 // 2))
    assert np.array_equal(f[:, 5], [1.0, 0, 0, 1.0])
    assert np.allclose(f[:, 6], np.log(n) / 8) and np.allclose(f[:, 7], 0.0)


def test_slice_features_rank_one_tensor(orc):
    # A(i,j,t) = u_i v_j w_t with w_t = 1 + cos(2 pi t / n3): the DFT of the
    # tube is w^_0 = n3, w^_1 = n3 / 2, w^_k = 0 for 2 <= k <= n3/2, so slice
    # k is w^_k u v^T, ||.||_F = |w^_k| ||u|| ||v||, largest column norm
    # |w^_k| ||u|| max|v_j|
    n1, n2, n3 = 9, 5, 8
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(n1), rng.standard_normal(n2)
    w = 1.0 + np.cos(2 * np.pi * np.arange(n3) / n3)
    A = u[:, None, None] * v[None, :, None] * w[None, None, :]
    tau, p = 0.7, min(n1, n2)
    f = orc.slice_features(A, tau)
    what = [n3, n3 / 2]
    for k in range(2):
        fro = what[k] * np.linalg.norm(u) * np.linalg.norm(v)
        assert np.isclose(f[k, 0], np.log(tau * np.sqrt(p) / fro), rtol=1e-12)
        assert np.isclose(f[k, 1], np.log(what[k] * np.linalg.norm(u) * np.abs(v).max() / tau), rtol=1e-12)
    # (numerically) zero slices: tau / rms sigma and the column norm / tau at
    # their clamped limits
    assert np.all(f[2:, 0] == 30.0) and np.all(f[2:, 1] == -30.0)
    Z = orc.slice_features(np.zeros((4, 3, 2)), tau)
    assert np.all(Z[:, 0] == 30.0) and np.all(Z[:, 1] == -30.0)
    assert np.allclose(f[:, 7], np.log(n1 / p))


def test_slice_features_previous_call(orc):
    n1, n2, n3 = 10, 12, 4
    h = n3 // 2 + 1
    Y = np.random.default_rng(5).standard_normal((n1, n2, n3))
    tau, p = 0.8, 10
    prev = np.array([3, 0, 7], dtype=np.int32)
    ps = np.zeros((h, 64))
    ps[0, :4] = [5.0, 3.0, 0.7, 0.5]    # 2 above tau, 3 above tau / 1.25 = 0.64, smallest kept <= tau
    ps[1, :3] = [2.0, 1.5, 1.0]         # every kept value above tau
    f = orc.slice_features(Y, tau, prev, ps)
    assert np.allclose(f[:, 2], prev / p) and np.all(f[:, 3] == 1.0)
    assert np.allclose(f[:, 8], [2 / p, 3 / p, 0.0])
    assert np.allclose(f[:, 9], [3 / p, 3 / p, 0.0])
    assert np.allclose(f[:2, 10], [np.log(5.0 / 0.8), np.log(2.0 / 0.8)]) and f[2, 10] == -30.0
    assert np.array_equal(f[:, 11], [0.0, 1.0, 0.0])
