"""GPU parity of the batched pipeline (many tensors of uneven n1, n2, l, n3
in one plan) against the FP64 oracle, and HIP-graph capture and replay of a
bound plan.  Tolerances: tprod 1e-5 and prox 1e-4 relative Frobenius per
tensor (the per-tensor entry points' bars)."""
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
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


# uneven shapes: wide and tall, odd and even n3 (n3 = 1 and non-powers of two),
# sizes around the 32 / 64 tile edges
SHAPES = [(5, 7, 3, 4), (33, 16, 40, 8), (64, 64, 64, 16), (17, 90, 20, 1), (70, 31, 65, 12), (128, 100, 24, 7),
          (1, 9, 2, 5), (48, 48, 48, 32), (96, 20, 110, 3), (12, 128, 9, 64)]


@pytest.mark.parametrize("tile", [1, 2])
def test_batch_tprod(tp, orc, tile):
    rng = np.random.default_rng(5)
    As = [rng.standard_normal((a, b, n3)).astype(np.float32) for a, b, l, n3 in SHAPES]
    Bs = [rng.standard_normal((b, l, n3)).astype(np.float32) for a, b, l, n3 in SHAPES]
    outs = tp.tp_batch_tprod([gpu(a) for a in As], [gpu(b) for b in Bs], tile=tile)
    errs = [rel_fro(c.cpu().numpy(), orc.tprod_fft(a, b)) for a, b, c in zip(As, Bs, outs)]
    say(f"  batch tprod tile {tile}: max rel.err {max(errs):.2e}")
    assert max(errs) <= 1e-5


PROX_SHAPES = [(20, 30, 5), (64, 40, 8), (37, 37, 1), (128, 96, 16), (9, 70, 12), (100, 128, 3), (3, 2, 4)]


def lowrank_plus(rng, n1, n2, n3, r):
    P = rng.standard_normal((n1, r, n3)) / np.sqrt(n1)
    Q = rng.standard_normal((r, n2, n3)) / np.sqrt(n2)
    return P, Q


def test_batch_prox_absolute_tau(tp, orc):
    rng = np.random.default_rng(6)
    Ys, taus = [], []
    for n1, n2, n3 in PROX_SHAPES:
        P, Q = lowrank_plus(rng, n1, n2, n3, 3)
        Y = (orc.tprod_fft(P, Q) + 0.1 * rng.standard_normal((n1, n2, n3))).astype(np.float32)
        Ys.append(Y)
        taus.append(float(0.3 * orc.tsn(Y)))
    b = tp.TPBatch("prox", [gpu(y) for y in Ys], taus=taus, ranks=True)
    outs = b.run()
    for Y, tau, X, rk in zip(Ys, taus, outs, b.ranks):
        ref = orc.prox_tnn(Y, np.float32(tau))
        err = rel_fro(X.cpu().numpy(), ref)
        assert err <= 1e-4, (Y.shape, err)
        h = Y.shape[2] // 2 + 1
        assert np.array_equal(rk.cpu().numpy(), (orc.slice_sigma(Y)[:h] > np.float32(tau)).sum(axis=1))
    assert np.allclose(b.tau_used.cpu().numpy(), np.float32(taus))


def test_batch_prox_relative_tau(tp, orc):
    """tau_i = 0.1 tsn(A_i), computed on the device between the SVD and the
    shrinkage, on N(0,1) tensors (the batching workload's recipe)."""
    rng = np.random.default_rng(7)
    As = [rng.standard_normal(s).astype(np.float32) for s in PROX_SHAPES]
    b = tp.TPBatch("prox", [gpu(a) for a in As], taus=[0.1] * len(As), tau_rel=True)
    outs = b.run()
    used = b.tau_used.cpu().numpy()
    for A, X, t in zip(As, outs, used):
        tau = 0.1 * orc.tsn(A)
        assert abs(t - tau) <= 1e-5 * tau
        err = rel_fro(X.cpu().numpy(), orc.prox_tnn(A, np.float32(t)))
        assert err <= 1e-4, (A.shape, err)


def test_batch_graph_replay(tp, orc):
    """A bound plan captured in a HIP graph and replayed gives the eager
    result at every replay, with other work on the stream in between."""
    from paper_1806_07247_amd import inputs
    shapes = inputs.batch_shapes(count=24, seed=3)
    pairs = inputs.batch_tensors(shapes, seed=3)
    As = [gpu(a) for a, _ in pairs]
    Bs = [gpu(b) for _, b in pairs]
    bt = tp.TPBatch("tprod", As, Bs)
    bp = tp.TPBatch("prox", As, taus=[0.1] * len(As), tau_rel=True)
    eager_t = [c.clone() for c in bt.run()]
    eager_p = [c.clone() for c in bp.run()]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            bt.run()
            bp.run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for c in bt.outs + bp.outs:
            c.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda:0").sum()  # other work between replays
        torch.cuda.synchronize()
        for c, e in zip(bt.outs, eager_t):
            assert torch.equal(c, e), rep
        for c, e in zip(bp.outs, eager_p):
            assert torch.equal(c, e), rep
    del junk
    # and the eager results are the oracle's
    for (a, b), c in zip(pairs[:6], eager_t[:6]):
        assert rel_fro(c.cpu().numpy(), orc.tprod_fft(a, b)) <= 1e-5


def test_batch_config_sampled(tp, orc):
    """The 256-tensor batching workload: every tprod and prox output, on a
    sample of tensors against the oracle."""
    from paper_1806_07247_amd import inputs
    shapes = inputs.batch_shapes(seed=0)
    pairs = inputs.batch_tensors(shapes, seed=0)
    As = [gpu(a) for a, _ in pairs]
    Bs = [gpu(b) for _, b in pairs]
    bt = tp.TPBatch("tprod", As, Bs)
    bp = tp.TPBatch("prox", As, taus=[0.1] * len(As), tau_rel=True)
    ct = bt.run()
    cp = bp.run()
    torch.cuda.synchronize()
    say(f"  batch stats tprod {bt.stats()} prox {bp.stats()}")
    rng = np.random.default_rng(11)
    for i in rng.choice(len(pairs), size=6, replace=False):
        a, b = pairs[i]
        assert rel_fro(ct[i].cpu().numpy(), orc.tprod_fft(a, b)) <= 1e-5
        t = float(bp.tau_used[i])
        assert abs(t - 0.1 * orc.tsn(a)) <= 1e-5 * t
        assert rel_fro(cp[i].cpu().numpy(), orc.prox_tnn(a, np.float32(t))) <= 1e-4
