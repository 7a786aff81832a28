"""GPU tsn (Definition 2.8), tubal rank (Definition 2.7), conjugate transpose
(Definition 2.2) and identity tensor (Definition 2.3) against the FP64
oracle.  tran and teye move values only: compared bit for bit.  tsn: 1e-5
relative.  Tubal rank: exact on inputs whose rank is unambiguous."""
import numpy as np
import pytest

from helpers import say

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
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 1), (4, 3, 2), (7, 9, 5), (33, 17, 8), (64, 100, 50)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tran_bit_exact(tp, orc, shape):
    A = np.random.default_rng(sum(shape)).standard_normal(shape).astype(np.float32)
    At = tp.tp_tran(gpu(A)).cpu().numpy()
    assert np.array_equal(At, orc.tran(A).astype(np.float32))
    # transposing twice gives A back
    assert np.array_equal(tp.tp_tran(tp.tp_tran(gpu(A))).cpu().numpy(), A)


@pytest.mark.parametrize("n,n3", [(1, 1), (4, 3), (17, 8)])
def test_teye_bit_exact(tp, orc, n, n3):
    assert np.array_equal(tp.tp_teye(n, n3).cpu().numpy(), orc.teye(n, n3).astype(np.float32))


@pytest.mark.parametrize("shape", [(6, 5, 4), (40, 30, 7), (120, 90, 16), (33, 70, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tsn(tp, orc, shape):
    A = np.random.default_rng(len(shape) + shape[0]).standard_normal(shape).astype(np.float32)
    v = float(tp.tp_tsn(gpu(A)))
    ref = orc.tsn(A)
    say(f"  tsn {shape}: {v:.6f} vs {ref:.6f}")
    assert abs(v - ref) <= 1e-5 * ref
    assert abs(float(tp.tp_tsn(tp.tp_teye(5, 4))) - 1.0) <= 1e-6


@pytest.mark.parametrize("n1,n2,n3,r", [(30, 20, 6, 3), (25, 40, 5, 7), (64, 64, 8, 1), (90, 70, 4, 12),
                                        (50, 50, 1, 9)])
def test_tubalrank(tp, orc, n1, n2, n3, r):
    rng = np.random.default_rng(n1 + r)
    A = orc.tprod(rng.standard_normal((n1, r, n3)), rng.standard_normal((r, n2, n3))).astype(np.float32)
    k = int(tp.tp_tubalrank(gpu(A)))
    say(f"  tubal rank {n1}x{n2}x{n3}: {k} (oracle {orc.tubalrank(A)}, built with {r})")
    assert k == r == orc.tubalrank(A)
    assert int(tp.tp_tubalrank(tp.tp_teye(6, n3))) == 6
    assert int(tp.tp_tubalrank(torch.zeros((5, 4, n3), device="cuda:0"))) == 0
    # an explicit tolerance above every tube gives 0
    assert int(tp.tp_tubalrank(gpu(A), tol=1e30)) == 0
