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
