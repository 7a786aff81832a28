"""Native tensor robust PCA (tp_trpca) against the FP64 oracle's inexact ALM,
the Python driver and the optimality conditions of the problem
min ||L||_* + lam ||S||_1 s.t. L + S = X (see tests/test_oracle_trpca.py)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import paper_1806_07247_amd as m
    return m


def _instance(n, n3, r, frac=0.05, seed=0):
    import oracle
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((n, r, n3)) / np.sqrt(n)
    Q = rng.standard_normal((r, n, n3)) / np.sqrt(n)
    L0 = oracle.tprod(P, Q)
    S0 = np.zeros_like(L0)
    m = rng.random(L0.shape) < frac
    S0[m] = rng.choice([-1.0, 1.0], int(m.sum()))
    return (L0 + S0).astype(np.float32), L0, S0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n,n3,r", [(30, 6, 2), (33, 7, 3)])
def test_trpca_matches_oracle_and_kkt(tp, n, n3, r):
    import oracle
    X, L0, S0 = _instance(n, n3, r)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Lam = torch.empty_like(Xd)
    res = tp.tp_trpca(Xd, Lam=Lam)
    assert res["converged"]
    L, S, Lm = res["L"].cpu().numpy(), res["S"].cpu().numpy(), Lam.cpu().numpy()
    ref = oracle.trpca(X.astype(np.float64))
    assert ref["converged"]
    assert abs(res["iters"] - ref["iters"]) <= 3
    assert _rel(L, ref["L"]) < 1e-3 and _rel(S, ref["S"]) < 1e-3
    assert _rel(L, L0) < 1e-3
    # optimality conditions on the GPU result
    lam = 1.0 / np.sqrt(n * n3)
    assert np.abs(Lm).max() <= lam * (1 + 1e-4)
    supp = S != 0
    assert np.abs(-Lm[supp] - lam * np.sign(S[supp])).max() <= 1e-4 * lam
    assert abs(oracle.tsn(Lm.astype(np.float64)) - 1.0) <= 2e-3
    tnn = oracle.tnn(L.astype(np.float64))
    assert abs(-(Lm.astype(np.float64) * L).sum() - tnn) <= 2e-3 * tnn


def test_trpca_matches_python_driver(tp):
    from paper_1806_07247_amd import trpca
    X, _, _ = _instance(40, 8, 3, seed=4)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    res = tp.tp_trpca(Xd)
    py = trpca.trpca(Xd, trpca.ProxFull(Xd.shape, dev))
    assert res["converged"] and py["converged"]
    assert abs(res["iters"] - py["iters"]) <= 2
    assert _rel(res["L"].cpu().numpy(), py["L"].cpu().numpy()) < 1e-4
    assert _rel(res["S"].cpu().numpy(), py["S"].cpu().numpy()) < 1e-4


def test_trpca_learned_prox(tp):
    from paper_1806_07247_amd import rank_model
    X, L0, _ = _instance(96, 8, 4, seed=5)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    full = tp.tp_trpca(Xd)
    mlp = rank_model.load(device=dev)
    lr = tp.tp_trpca(Xd, learned=dict(mlp=mlp, max_rank=32))
    assert full["converged"] and lr["converged"]
    assert abs(lr["iters"] - full["iters"]) <= 3
    Lf, Ll = full["L"].cpu().numpy(), lr["L"].cpu().numpy()
    assert _rel(Ll, Lf) < 1e-3
    assert _rel(Ll, L0) < 1e-3


def test_trpca_edges(tp):
    dev = torch.device("cuda:0")
    # zero input: converged after one iteration with L = S = 0
    Z = torch.zeros((8, 7, 4), device=dev)
    res = tp.tp_trpca(Z)
    assert res["converged"] and res["iters"] == 1
    assert not res["L"].any() and not res["S"].any()
    # iteration cap
    X, _, _ = _instance(20, 5, 2, seed=6)
    res = tp.tp_trpca(torch.from_numpy(X).to(dev), max_iter=2)
    assert res["iters"] == 2 and not res["converged"]
    # n1 n2 n3 not a multiple of 4, input at an offset of one float (scalar path)
    import oracle
    X, _, _ = _instance(7, 3, 1, seed=7)  # 7 x 7 x 3 = 147 entries
    buf = torch.zeros(X.size + 1, device=dev)
    buf[1:] = torch.from_numpy(X.ravel()).to(dev)
    Xv = buf[1:].view(X.shape)
    assert Xv.data_ptr() % 16 != 0
    res = tp.tp_trpca(Xv)
    ref = oracle.trpca(X.astype(np.float64))
    assert res["converged"] == ref["converged"]
    assert _rel(res["L"].cpu().numpy(), ref["L"]) < 1e-3
    # non-finite input is rejected
    Xn = torch.from_numpy(X).to(dev)
    Xn[0, 0, 0] = float("nan")
    with pytest.raises(Exception):
        tp.tp_trpca(Xn)
