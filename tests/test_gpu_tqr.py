"""GPU tensor inverse (Definition 2.4) and T-QR (Theorem 2.4) against the FP64
oracle and the defining identities."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import paper_1806_07247_amd as m
    return m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _well_conditioned(n, n3, seed):
    import oracle
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n, n3)) / np.sqrt(n)
    return (G + 2.0 * oracle.teye(n, n3)).astype(np.float32)


@pytest.mark.parametrize("n,n3", [(5, 4), (16, 7), (33, 8), (64, 2), (1, 5), (100, 3), (7, 1)])
def test_tinv_matches_oracle(tp, n, n3):
    import oracle
    dev = torch.device("cuda:0")
    A = _well_conditioned(n, n3, n * 7 + n3)
    h = n3 // 2 + 1
    info = torch.full((h,), -1, dtype=torch.int32, device=dev)
    Ad = torch.from_numpy(A).to(dev)
    B = tp.tp_tinv(Ad, info=info).cpu().numpy()
    ref, st = oracle.tinv(A.astype(np.float64))
    assert st == 0 and int(info.abs().sum()) == 0
    assert _rel(B, ref) < 1e-5
    # Definition 2.4 on the GPU result: A * B = B * A = I
    I = torch.from_numpy(oracle.teye(n, n3).astype(np.float32)).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    assert float((tp.tp_tprod(Ad, Bd) - I).abs().max()) < 1e-4
    assert float((tp.tp_tprod(Bd, Ad) - I).abs().max()) < 1e-4


def test_tinv_singular_slice_reported(tp):
    dev = torch.device("cuda:0")
    A = np.zeros((4, 4, 6), np.float32)
    A[0, 0, :] = 1.0
    A[1, 1, :] = 2.0
    A[3, 3, :] = 3.0
    info = torch.zeros(4, dtype=torch.int32, device=dev)
    tp.tp_tinv(torch.from_numpy(A).to(dev), info=info)
    # constant tubes: Fourier slice 0 is diag(6, 12, 0, 18), singular at step 2;
    # the other slices are zero, singular at step 0
    assert info.cpu().numpy().tolist() == [3, 1, 1, 1]


@pytest.mark.parametrize("n1,n2,n3", [(6, 4, 5), (4, 6, 4), (20, 20, 8), (33, 17, 6), (17, 33, 7), (1, 5, 3),
                                      (5, 1, 3), (64, 48, 16), (9, 9, 1)])
def test_tqr_matches_oracle(tp, n1, n2, n3):
    import oracle
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(n1 * 100 + n2 * 10 + n3)
    A = rng.standard_normal((n1, n2, n3)).astype(np.float32)
    Ad = torch.from_numpy(A).to(dev)
    Q, R = tp.tp_tqr(Ad)
    Qn, Rn = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = oracle.tqr(A.astype(np.float64))
    p = min(n1, n2)
    assert _rel(Rn, Ro) < 1e-4                       # unique R
    assert _rel(Qn[:, :p, :], Qo[:, :p, :]) < 1e-4   # and the leading columns of Q
    # Theorem 2.4 on the GPU result: Q orthogonal, Q * R = A, R f-upper triangular
    I = torch.from_numpy(oracle.teye(n1, n3).astype(np.float32)).to(dev)
    Qh = tp.tp_tran(Q)
    assert float((tp.tp_tprod(Qh, Q) - I).abs().max()) < 1e-4
    assert float((tp.tp_tprod(Q, Qh) - I).abs().max()) < 1e-4
    assert _rel(tp.tp_tprod(Q, R).cpu().numpy(), A) < 1e-5
    for t in range(n3):
        assert np.abs(np.tril(Rn[:, :, t], -1)).max() < 1e-5 * max(1.0, np.abs(Rn).max())


def test_tqr_tinv_argument_errors(tp):
    from paper_1806_07247_amd import _lib
    lib = _lib.load()
    assert lib.tp_tinv(None, None, 4, 3, None, None, 0, None) == -1
    assert lib.tp_tinv_workspace_size(0, 3) == 0
    assert lib.tp_tqr_workspace_size(3, 4, 0) == 0
    with pytest.raises(ValueError):
        tp.tp_tinv(torch.zeros((3, 4, 2), device="cuda:0"))
