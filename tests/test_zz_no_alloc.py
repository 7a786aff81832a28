"""tp_tprod_noalloc: the t-product of tp_tprod with its workspace in the
library's device-resident array (for callers that cannot allocate),
compared with tp_tprod through the C ABI on two calls in a row, the second
smaller, and the size limit."""
import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_07247_amd import _lib
    return _lib.load()


def run_pair(lib, n1, n2, l, n3, prec, seed):
    from paper_1806_07247_amd import inputs
    import paper_1806_07247_amd as tp
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=seed)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = tp.tp_tprod(dA, dB, prec=prec)
    C = torch.full((n1, l, n3), float("nan"), device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.tp_tprod_noalloc(dA.data_ptr(), dB.data_ptr(), C.data_ptr(), n1, n2, l, n3,
                              {"fp32": 0, "bf16x3": 1, "bf16": 2}[prec], stream)
    assert st == 0
    torch.cuda.synchronize()
    return C, ref


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_noalloc_matches_tprod_twice(lib, prec):
    # the same kernels on the same inputs: the results agree bitwise
    for shape in [(64, 48, 40, 32), (12, 10, 9, 7)]:   # second call smaller
        C, ref = run_pair(lib, *shape, prec, seed=sum(shape))
        say(f"noalloc {prec} {shape}: max diff {float((C - ref).abs().max()):.3e}")
        assert torch.equal(C, ref)


def test_noalloc_size_limit(lib):
    import paper_1806_07247_amd as tp
    cap = lib.tp_tprod_noalloc_max_bytes()
    assert cap >= 1 << 20
    n1 = n2 = l = 512
    n3 = 64
    assert tp.tp_tprod_workspace_size(n1, n2, l, n3) > cap
    x = torch.zeros(1, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    # rejected on the host before anything is enqueued (the pointers are never used)
    assert lib.tp_tprod_noalloc(x.data_ptr(), x.data_ptr(), x.data_ptr(), n1, n2, l, n3, 0, stream) == -3
