"""Pins of the FP64 oracle's tensor robust PCA (inexact ALM around prox_tnn).

The paper names TRPCA as the use of the prox of Theorem 2.3 but gives no
algorithm, so the oracle is pinned to the optimality conditions of the convex
problem  min ||L||_* + lam ||S||_1  s.t.  L + S = X, which hold whatever the
implementation:
  - after every S step the multiplier satisfies -Lam in lam d||S||_1 exactly:
    |Lam| <= lam entrywise and -Lam = lam sign(S) on the support of S;
  - at convergence -Lam is also a subgradient of the TNN at L: its dual norm,
    the tensor spectral norm (Definition 2.8), is 1, and <-Lam, L> = ||L||_*
    (Definition 2.9);
  - a planted low-tubal-rank plus sparse instance is recovered.
"""
import numpy as np
import pytest

import oracle


def _instance(n=30, n3=6, r=2, frac=0.05, seed=0):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((n, r, n3)) / np.sqrt(n)
    Q = rng.standard_normal((r, n, n3)) / np.sqrt(n)
    L0 = oracle.tprod(P, Q)
    S0 = np.zeros_like(L0)
    m = rng.random(L0.shape) < frac
    S0[m] = rng.choice([-1.0, 1.0], int(m.sum()))
    return L0, S0


@pytest.mark.parametrize("n,n3,r", [(30, 6, 2), (24, 5, 1)])
def test_trpca_optimality_and_recovery(n, n3, r):
    L0, S0 = _instance(n, n3, r)
    X = L0 + S0
    res = oracle.trpca(X)
    assert res["converged"]
    L, S, Lam = res["L"], res["S"], res["Lam"]
    lam = 1.0 / np.sqrt(n * n3)
    # exact conditions of the S step
    assert np.abs(Lam).max() <= lam * (1 + 1e-12)
    supp = S != 0
    assert supp.any()
    assert np.abs(-Lam[supp] - lam * np.sign(S[supp])).max() <= 1e-12 * lam
    # TNN subgradient at convergence
    assert abs(oracle.tsn(Lam) - 1.0) <= 1e-3
    tnn = oracle.tnn(L)
    assert abs(-(Lam * L).sum() - tnn) <= 1e-4 * tnn
    # feasibility within the stopping tolerance, and recovery
    assert np.abs(L + S - X).max() <= 1e-5 * max(1.0, np.abs(X).max())
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) < 1e-3
    assert np.linalg.norm(S - S0) / np.linalg.norm(S0) < 1e-3


def test_trpca_zero_input():
    X = np.zeros((8, 7, 4))
    res = oracle.trpca(X)
    assert res["converged"] and res["iters"] == 1
    assert not res["L"].any() and not res["S"].any() and not res["Lam"].any()


def test_trpca_iteration_cap():
    L0, S0 = _instance(20, 4, 2, seed=3)
    res = oracle.trpca(L0 + S0, max_iter=3)
    assert res["iters"] == 3 and not res["converged"]
    # the S-step conditions hold after any iteration
    lam = 1.0 / np.sqrt(20 * 4)
    assert np.abs(res["Lam"]).max() <= lam * (1 + 1e-12)


def test_trpca_bad_arguments():
    with pytest.raises(ValueError):
        oracle.trpca(np.ones((3, 3, 2)), lam=-1.0)
    with pytest.raises(ValueError):
        oracle.trpca(np.ones((3, 3, 2)), max_iter=0)
