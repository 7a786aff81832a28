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


def test_trpca_learned_prox_host_driven_same_bits(tp):
    """tp_trpca around the learned prox in its host-driven form
    (TP_PARAM_LEARNED_HOST = 1) takes the same iterations and gives the same
    bits as with the default, device-gated form."""
    from paper_1806_07247_amd import rank_model
    X, _, _ = _instance(96, 8, 4, seed=5)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    mlp = rank_model.load(device=dev)
    lib = tp._lib.load()
    out = {}
    try:
        for mode in (0, 1):
            assert lib.tp_set_param(12, mode) == 0  # TP_PARAM_LEARNED_HOST
            out[mode] = tp.tp_trpca(Xd, learned=dict(mlp=mlp, max_rank=32))
            torch.cuda.synchronize()
    finally:
        lib.tp_set_param(12, 0)
    assert out[0]["iters"] == out[1]["iters"] and out[0]["converged"] == out[1]["converged"]
    assert torch.equal(out[0]["L"], out[1]["L"]) and torch.equal(out[0]["S"], out[1]["S"])


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


def test_trpca_record_replays_bitwise(tp):
    """The per-call record of the native TRPCA driver: call 0's input is X, and
    every recorded call replays bitwise through tp_slice_features and
    tp_prox_tnn_learned from the recorded inputs, the tau sequence of
    tp_trpca_taus, seed + i, and call i-1's counts, singular values and basis."""
    import numpy as np
    from paper_1806_07247_amd import rank_model, trpca
    dev = torch.device("cuda:0")
    n, n3, mr = 48, 6, 16
    X, _, _ = trpca.make_problem(n, n3, 3, 0.05, 5, dev)
    h = n3 // 2 + 1
    K = 6
    rec = dict(max_calls=K,
               inputs=torch.zeros((K, n, n, n3), device=dev),
               features=torch.zeros((K, h, tp.TP_MLP_INPUTS), device=dev),
               counts=torch.zeros((K, h), dtype=torch.int32, device=dev),
               sigmas=torch.zeros((K, h, tp.TP_SIGMA_KEEP), device=dev),
               bases=torch.zeros((K,) + tp.basis_shape(n, n3, mr), device=dev),
               basis_cols=torch.zeros((K, h), dtype=torch.int32, device=dev))
    mlp = rank_model.load(device=dev)
    lo = dict(mlp=mlp, max_rank=mr, seed=77, accuracy=2e-5)
    res = tp.tp_trpca(X, learned=lo, record=rec, max_iter=200)
    assert res["iters"] > K
    assert torch.equal(rec["inputs"][0], X)
    taus = tp.tp_trpca_taus(K)
    ws = torch.empty(tp.tp_prox_tnn_learned_workspace_size(n, n, n3, mr), dtype=torch.uint8, device=dev)
    out = torch.empty_like(X)
    rk = torch.zeros(h, dtype=torch.int32, device=dev)
    so = torch.zeros((h, tp.TP_SIGMA_KEEP), device=dev)
    bo = torch.zeros(tp.basis_shape(n, n3, mr), device=dev)
    bc = torch.zeros(h, dtype=torch.int32, device=dev)
    for i in range(K):
        Y = rec["inputs"][i].contiguous()
        pr = rec["counts"][i - 1].contiguous() if i else None
        ps = rec["sigmas"][i - 1].contiguous() if i else None
        f = tp.tp_slice_features(Y, taus[i], pr, ps)
        assert torch.equal(f, rec["features"][i]), i
        tp.tp_prox_tnn_learned(Y, taus[i], mlp=mlp, max_rank=mr, seed=77 + i, accuracy=2e-5, prev_rank=pr,
                               prev_sigma=ps, warm_basis=rec["bases"][i - 1].contiguous() if i else None,
                               warm_cols=rec["basis_cols"][i - 1].contiguous() if i else None, basis_out=bo,
                               basis_cols_out=bc, out=out, rank=rk, sigma_out=so, workspace=ws)
        assert torch.equal(rk, rec["counts"][i]), i
        assert torch.equal(so, rec["sigmas"][i]), i
        assert torch.equal(bc, rec["basis_cols"][i]), i
    # the full-SVD driver records inputs and unchained features
    rec2 = dict(max_calls=2, inputs=torch.zeros((2, n, n, n3), device=dev),
                features=torch.zeros((2, h, tp.TP_MLP_INPUTS), device=dev))
    tp.tp_trpca(X, record=rec2, max_iter=200)
    assert torch.equal(rec2["inputs"][0], X)
    f1 = tp.tp_slice_features(rec2["inputs"][1].contiguous(), taus[1])
    assert torch.equal(f1, rec2["features"][1])
    assert np.isfinite(rec2["features"].cpu().numpy()).all()
