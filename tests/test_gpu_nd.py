"""GPU parity of the order-p calls (tp_tprod_nd, tp_prox_tnn_nd, tp_tnn_nd)
against the FP64 order-p oracle (oracle/nd.py, which routes through numpy's
fftn over all modes 3..p, not the half spectrum the library keeps).

Tolerances: relative Frobenius error <= 1e-5 for the product, <= 1e-4 for
the prox (the 3-way prox bar) and 1e-5 relative for the nuclear norm."""
import numpy as np
import pytest

from helpers import rel_fro, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07247_amd as tp
    tp._lib.load()
    return tp


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


TPROD_SHAPES = [
    (4, 3, 2, (3, 4)), (5, 6, 7, (2, 3, 2)), (17, 13, 11, (5, 6)), (33, 31, 29, (3, 5)),
    (20, 16, 12, (4, 1, 3)), (9, 7, 5, (1, 8)), (6, 5, 4, (2, 2, 2, 2)), (64, 48, 40, (3, 7)),
    (3, 2, 4, (7,)), (40, 36, 33, (2, 64)), (12, 10, 9, (16, 9)),
]


@pytest.mark.parametrize("shape", TPROD_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}x{s[2]}_{'x'.join(map(str, s[3]))}")
def test_tprod_nd_matches_oracle(tp, orc, shape):
    from paper_1806_07247_amd import inputs
    n1, n2, l, dims = shape
    A = inputs.tensor_nd((n1, n2) + dims, seed=1)
    B = inputs.tensor_nd((n2, l) + dims, seed=2)
    say(f"tprod_nd {shape}")
    C = tp.tp_tprod_nd(gpu(A), gpu(B)).cpu().numpy()
    ref = orc.tprod_nd_fft(A, B)
    err = rel_fro(C, ref)
    say(f"  rel.err {err:.2e}")
    assert C.shape == ref.shape
    assert err <= 1e-5


def test_tprod_nd_three_way_is_tprod(tp):
    """nd = 1 runs the 3-way kernels: bitwise equal to tp_tprod (FP32)."""
    from paper_1806_07247_amd import inputs
    A, B = inputs.tprod_pair(33, 31, 29, 8, seed=3)
    a, b = gpu(A), gpu(B)
    assert torch.equal(tp.tp_tprod_nd(a, b), tp.tp_tprod(a, b))


def test_tprod_nd_identity(tp, orc):
    from paper_1806_07247_amd import inputs
    dims = (3, 4, 2)
    A = inputs.tensor_nd((7, 5) + dims, seed=4)
    I = orc.teye_nd(5, dims).astype(np.float32)
    C = tp.tp_tprod_nd(gpu(A), gpu(I)).cpu().numpy()
    assert rel_fro(C, A) <= 1e-6


def test_tprod_nd_larger_sampled(tp, orc):
    """648 kept slices of 64 x 48 x 40 products (modes 8 x 9 x 16)."""
    from paper_1806_07247_amd import inputs
    dims = (8, 9, 16)
    A = inputs.tensor_nd((64, 48) + dims, seed=5)
    B = inputs.tensor_nd((48, 40) + dims, seed=6)
    C = tp.tp_tprod_nd(gpu(A), gpu(B)).cpu().numpy()
    err = rel_fro(C, orc.tprod_nd_fft(A, B))
    say(f"  648 slices: rel.err {err:.2e}")
    assert err <= 1e-5


PROX_SHAPES = [(12, 9, (3, 4)), (20, 30, (2, 3, 2)), (7, 5, (5,)), (16, 16, (4, 6)), (33, 20, (1, 3, 4))]


@pytest.mark.parametrize("shape", PROX_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}_{'x'.join(map(str, s[2]))}")
def test_prox_tnn_nd_matches_oracle(tp, orc, shape):
    from paper_1806_07247_amd import inputs
    n1, n2, dims = shape
    P, Q = inputs.lowrank_nd(n1, n2, dims, 3, seed=7)
    Y = (orc.tprod_nd_fft(P, Q) + 0.05 * inputs.tensor_nd((n1, n2) + dims, seed=8)).astype(np.float32)
    tau = 0.3 * float(np.sqrt(n1 * n2 * 1e-3 * np.prod(dims)))
    h = tp.tp_half_slices_nd(dims)
    info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    rank = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_nd(gpu(Y), tau, info=info, rank=rank).cpu().numpy()
    ref = orc.prox_tnn_nd(Y.astype(np.float64), tau)
    err = rel_fro(X, ref)
    say(f"prox_nd {shape} tau {tau:.3f}: rel.err {err:.2e}, ranks {rank.cpu().numpy()[:6]}")
    assert err <= 1e-4
    assert bool((info.cpu() > 0).all())
    r = rank.cpu().numpy()
    assert r.min() >= 0 and r.max() <= min(n1, n2)


def test_prox_tnn_nd_zero_tau(tp):
    from paper_1806_07247_amd import inputs
    Y = inputs.tensor_nd((9, 6, 3, 4), seed=9)
    X = tp.tp_prox_tnn_nd(gpu(Y), 0.0).cpu().numpy()
    assert rel_fro(X, Y) <= 1e-5


def test_prox_tnn_nd_three_way_is_prox(tp):
    from paper_1806_07247_amd import inputs
    Y = gpu(inputs.tensor_nd((20, 15, 6), seed=10))
    assert torch.equal(tp.tp_prox_tnn_nd(Y, 0.8), tp.tp_prox_tnn(Y, 0.8))


@pytest.mark.parametrize("shape", [(8, 6, (3, 4)), (5, 9, (2, 5, 2)), (12, 12, (7,)), (10, 4, (4, 1, 6))],
                         ids=lambda s: f"{s[0]}x{s[1]}_{'x'.join(map(str, s[2]))}")
def test_tnn_nd_matches_oracle(tp, orc, shape):
    from paper_1806_07247_amd import inputs
    n1, n2, dims = shape
    A = inputs.tensor_nd((n1, n2) + dims, seed=11)
    v = float(tp.tp_tnn_nd(gpu(A)).cpu())
    ref = orc.tnn_nd(A.astype(np.float64))
    say(f"tnn_nd {shape}: {v:.6f} vs {ref:.6f}")
    assert v == pytest.approx(ref, rel=1e-5)


def test_tnn_nd_identity(tp, orc):
    I = orc.teye_nd(6, (3, 4, 2)).astype(np.float32)
    assert float(tp.tp_tnn_nd(gpu(I)).cpu()) == pytest.approx(6.0, rel=1e-6)
