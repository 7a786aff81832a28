"""GPU parity of the learned-rank path against the FP64 oracle: MLP forward
and gradient, Adam, slice features, and the randomized-SVD prox (exact on
low-rank slices, forced fallback, agreement with the oracle's randomized prox
on the same Philox sketch).  Tolerances: MLP 1e-5 relative (FP32 vs FP64),
prox 1e-4 relative Frobenius."""
import numpy as np
import pytest

from helpers import rel_fro, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

D, H = 12, 64


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07247_amd as tp
    tp._lib.load()
    return tp


def gpu(x, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to("cuda:0")


def rand_params(orc, seed):
    rng = np.random.default_rng(seed)
    n = orc.mlp_param_count(D, H)
    return (rng.standard_normal(n) * 0.3).astype(np.float32)


def test_mlp_param_count(tp, orc):
    assert tp.tp_mlp_param_count() == orc.mlp_param_count(D, H)


def test_mlp_forward_and_grad(tp, orc):
    rng = np.random.default_rng(5)
    p = rand_params(orc, 1)
    X = rng.standard_normal((1000, D)).astype(np.float32)
    t = rng.standard_normal(1000).astype(np.float32)
    y = tp.tp_mlp_forward(gpu(p), gpu(X)).cpu().numpy()
    yref = orc.mlp_forward(p, X, D, H)
    assert np.abs(y - yref).max() <= 1e-5 * max(1.0, np.abs(yref).max())
    g, l = tp.tp_mlp_loss_grad(gpu(p), gpu(X), gpu(t), under=4.0)
    lref, gref = orc.mlp_loss_grad(p, X, t, D, H, under=4.0)
    say(f"loss {float(l):.6f} vs {lref:.6f}; grad max diff {np.abs(g.cpu().numpy() - gref).max():.2e}")
    assert abs(float(l) - lref) <= 1e-5 * max(1.0, abs(lref))
    assert np.abs(g.cpu().numpy() - gref).max() <= 1e-5 * max(1.0, np.abs(gref).max())
    g2, _ = tp.tp_mlp_loss_grad(gpu(p), gpu(X), gpu(t), under=4.0)
    assert torch.equal(g, g2)  # deterministic reduction order


def test_adam_step(tp):
    rng = np.random.default_rng(8)
    n = tp.tp_mlp_param_count()
    p, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    m, v = rng.standard_normal(n).astype(np.float32) * 0.1, np.abs(rng.standard_normal(n)).astype(np.float32) * 0.1
    P, G, M, V = gpu(p), gpu(g), gpu(m), gpu(v)
    tp.tp_mlp_adam(P, G, M, V, step=3, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8)
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    p2 = p - 1e-2 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    assert np.allclose(P.cpu().numpy(), p2, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("shape", [(20, 30, 8), (33, 17, 5), (64, 64, 1)])
def test_features(tp, orc, shape):
    from paper_1806_07247_amd import inputs
    Y = inputs.random_tensor(shape, seed=3)
    h = shape[2] // 2 + 1
    prev = np.arange(h, dtype=np.int32) % 5
    rng = np.random.default_rng(2)
    ps = np.zeros((h, 64), dtype=np.float32)
    for k in range(h):
        c = int(rng.integers(0, 65))
        ps[k, :c] = np.sort(rng.uniform(0.1, 3.0, size=c))[::-1]
    for pv, sv in ((None, None), (prev, None), (prev, ps)):
        f = tp.tp_slice_features(gpu(Y), 0.7, None if pv is None else gpu(pv, np.int32),
                                 None if sv is None else gpu(sv)).cpu().numpy()
        ref = orc.slice_features(Y, np.float32(0.7), pv, sv)
        assert np.abs(f - ref).max() < 1e-5


def lowrank(orc, n1, n2, n3, r, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    A = orc.tprod(rng.standard_normal((n1, r, n3)), rng.standard_normal((r, n2, n3)))
    if noise:
        A = A + noise * rng.standard_normal(A.shape)
    return A.astype(np.float32)


# (512, 300, 4, 6): inner dimensions >= 256 with few output tiles, so the
# range-finder products are split along k (split-K partial sums)
@pytest.mark.parametrize("n1,n2,n3,r", [(64, 48, 6, 3), (40, 70, 5, 4), (128, 128, 8, 6), (200, 160, 4, 10),
                                        (512, 300, 4, 6)])
def test_learned_prox_exact_on_low_rank(tp, orc, n1, n2, n3, r):
    Y = lowrank(orc, n1, n2, n3, r, seed=n1 + r)
    tau = 0.2 * orc.tsn(Y)
    h = n3 // 2 + 1
    say(f"learned prox low-rank {n1}x{n2}x{n3} r={r}")
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    rk = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=r, oversample=6, power_iters=2, max_rank=32, seed=4,
                               rank=rk, fallback=fb).cpu().numpy()
    ref = orc.prox_tnn(Y, np.float32(tau))
    err = rel_fro(X, ref)
    say(f"  rel.err {err:.2e} fallback {fb.cpu().numpy().tolist()} rank {rk.cpu().numpy().tolist()}")
    assert err <= 1e-4
    assert int(fb.sum()) == 0
    sig = orc.slice_sigma(Y)[:h]
    assert np.array_equal(rk.cpu().numpy(), (sig > np.float32(tau)).sum(axis=1))


def test_learned_prox_split_parts_with_gram(tp, orc):
    """Range-finder products split along k leave their parts, summed together
    with the first CholeskyQR pass's Gram (k_reduce_gram); the same call with
    the split turned off (TP_PARAM_GEMM_KSPLIT = 1: one part, plain Gram)
    agrees to FP32 rounding, and both match the full-SVD prox."""
    from paper_1806_07247_amd import _lib
    lib = _lib.load()
    n1, n2, n3, r = 768, 320, 4, 6
    Y = gpu(lowrank(orc, n1, n2, n3, r, seed=77))
    tau = 0.2 * orc.tsn(Y.cpu().numpy())
    kw = dict(fixed_rank=r, oversample=6, power_iters=2, max_rank=32, seed=9)
    X_split = tp.tp_prox_tnn_learned(Y, tau, **kw).cpu().numpy()
    try:
        assert lib.tp_set_param(8, 1) == 0
        X_one = tp.tp_prox_tnn_learned(Y, tau, **kw).cpu().numpy()
    finally:
        lib.tp_set_param(8, 0)
    X_full = tp.tp_prox_tnn(Y, tau).cpu().numpy()
    d = rel_fro(X_split, X_one)
    e1, e2 = rel_fro(X_split, X_full), rel_fro(X_one, X_full)
    say(f"  split vs one part {d:.2e}; vs full SVD {e1:.2e} / {e2:.2e}")
    assert d <= 1e-5
    assert e1 <= 1e-4 and e2 <= 1e-4


def test_learned_prox_matches_oracle_rsvd(tp, orc):
    """Same Philox sketch, same predicted counts: GPU (FP32 data, FP64
    CholeskyQR and rotations) against the FP64 oracle of the randomized prox."""
    Y = lowrank(orc, 96, 80, 6, 5, seed=11, noise=0.05)
    tau = 0.15 * orc.tsn(Y)
    h = 4
    # k = 5, oversample 4: l = 9, rounded up to the call's common width 16,
    # which every slice uses, so the count check allows 16 - 4 = 12
    kp = np.full(h, 12, dtype=np.int32)
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=5, oversample=4, power_iters=2, max_rank=16, seed=99,
                               accuracy=0.0, fallback=fb).cpu().numpy()
    ref, fbr, _ = orc.prox_tnn_rsvd(Y, np.float32(tau), kp, oversample=4, power=2, lfull=17, seed=99)
    err = rel_fro(X, ref)
    say(f"  vs oracle rsvd: rel.err {err:.2e}, fallback gpu {fb.cpu().numpy().tolist()} oracle {fbr.tolist()}")
    assert np.array_equal(fb.cpu().numpy(), fbr)
    assert err <= 1e-4
    exact = orc.prox_tnn(Y, np.float32(tau))
    say(f"  vs exact prox: rel.err {rel_fro(X, exact):.2e}")


def test_learned_prox_forced_fallback(tp, orc):
    """k = 0 predicted on full-rank slices: every check fails, every slice goes
    through the full SVD, and the result is the exact prox."""
    from paper_1806_07247_amd import inputs
    Y = inputs.random_tensor((48, 40, 6), seed=21)
    tau = 0.05 * orc.tsn(Y)
    h = 4
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=0, oversample=3, max_rank=16, fallback=fb,
                               info=info).cpu().numpy()
    assert int(fb.sum()) == h and int(info.min()) > 0
    assert rel_fro(X, orc.prox_tnn(Y, np.float32(tau))) <= 1e-4
    # l > max_rank also goes to the full SVD
    fb.zero_()
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=30, oversample=10, max_rank=16, fallback=fb).cpu().numpy()
    assert int(fb.sum()) == h
    assert rel_fro(X, orc.prox_tnn(Y, np.float32(tau))) <= 1e-4


def test_learned_prox_wide_retry(tp, orc):
    """Under-predicted counts (k = 2 on tubal rank 6): without the retry every
    slice fails the count check and takes the full SVD; with it the slices are
    redone once at the widest sketch (k = max_rank - oversample) and pass."""
    Y = lowrank(orc, 90, 70, 6, 6, seed=17)
    tau = 0.1 * orc.tsn(Y)
    h = 4
    sig = orc.slice_sigma(Y)[:h]
    exact = orc.prox_tnn(Y, np.float32(tau))
    assert (sig > np.float32(tau)).sum(axis=1).min() > 2
    for retry in (False, True):
        fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        rk = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=2, oversample=4, max_rank=24, retry_wide=retry,
                                   rank=rk, fallback=fb).cpu().numpy()
        err = rel_fro(X, exact)
        say(f"  retry={retry}: rel.err {err:.2e} fallback {fb.cpu().numpy().tolist()}")
        assert int(fb.sum()) == (0 if retry else h)
        assert err <= 1e-4
        assert np.array_equal(rk.cpu().numpy(), (sig > np.float32(tau)).sum(axis=1))


def test_learned_prox_with_mlp_runs(tp, orc):
    """An MLP whose output is the constant log1p(4)/log1p(p) predicts k = 4."""
    Y = lowrank(orc, 50, 50, 4, 4, seed=2)
    n = tp.tp_mlp_param_count()
    p = np.zeros(n, dtype=np.float32)
    p[-1] = np.log1p(4) / np.log1p(50)
    h = 3
    rk = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    tau = 0.1 * orc.tsn(Y)
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, mlp=gpu(p), oversample=5, max_rank=16, rank=rk, fallback=fb).cpu().numpy()
    assert int(fb.sum()) == 0
    assert rel_fro(X, orc.prox_tnn(Y, np.float32(tau))) <= 1e-4


def test_learned_prox_sigma_out(tp, orc):
    """sigma_out holds each slice's leading singular values (decreasing), from
    the randomized SVD or, for fallback slices, the full SVD."""
    Y = lowrank(orc, 60, 50, 6, 4, seed=8, noise=0.01)
    h = 4
    so = torch.zeros((h, 64), dtype=torch.float32, device="cuda:0")
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    kp = torch.tensor([4, 0, 4, 4], dtype=torch.int32)
    tau = 0.05 * orc.tsn(Y)
    tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=4, oversample=6, max_rank=16, fallback=fb, sigma_out=so)
    sig = orc.slice_sigma(Y)[:h]
    out = so.cpu().numpy()
    assert int(fb.sum()) == 0
    for k in range(h):
        c = int((out[k] > 0).sum())
        assert c >= 4 and np.all(np.diff(out[k, :c]) <= 0)
        assert np.allclose(out[k, :4], sig[k, :4], rtol=1e-4)
    # every slice through the full SVD: sigma_out = leading 64 exact values
    so.zero_()
    tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=20, oversample=2, max_rank=16, fallback=fb, sigma_out=so)
    assert int(fb.sum()) == h
    assert np.allclose(so.cpu().numpy()[:, :50], sig[:, :50], rtol=1e-4, atol=1e-6)


def test_learned_prox_deterministic(tp, orc):
    Y = gpu(lowrank(orc, 70, 60, 6, 5, seed=3, noise=0.01))
    a = tp.tp_prox_tnn_learned(Y, 1.0, fixed_rank=5, max_rank=24, seed=1)
    b = tp.tp_prox_tnn_learned(Y, 1.0, fixed_rank=5, max_rank=24, seed=1)
    assert torch.equal(a, b)


def test_learned_prox_accuracy_check(tp, orc):
    """Kept singular values close above a noise bulk: two power iterations do
    not resolve the kept subspace to 1e-4; the a posteriori residual check
    adds iterations (or falls back) until the result is within 1e-4 of the
    exact prox."""
    rng = np.random.default_rng(31)
    n, n3, r = 120, 4, 5
    P = rng.standard_normal((n, r, n3)) / np.sqrt(n)
    Q = rng.standard_normal((r, n, n3)) / np.sqrt(n)
    L = orc.tprod(P, Q) * 0.7
    Y = (L + 0.35 * rng.standard_normal((n, n, n3)) / np.sqrt(n)).astype(np.float32)
    sig = orc.slice_sigma(Y)[:3]
    tau = float(np.sort(sig[:, r - 1])[0]) * 0.8
    say(f"  sigma_r {sig[:, r - 1].round(3).tolist()} sigma_r+1 {sig[:, r].round(3).tolist()} tau {tau:.3f}")
    exact = orc.prox_tnn(Y, np.float32(tau))
    kw = dict(fixed_rank=r, oversample=3, power_iters=2, max_rank=16, seed=5)
    loose = tp.tp_prox_tnn_learned(gpu(Y), tau, accuracy=0.0, **kw).cpu().numpy()
    fb = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    tight = tp.tp_prox_tnn_learned(gpu(Y), tau, accuracy=2e-5, max_power_iters=60, accuracy_ref=1, fallback=fb,
                                   **kw).cpu().numpy()
    e0, e1 = rel_fro(loose, exact), rel_fro(tight, exact)
    say(f"  without check {e0:.2e}, with check {e1:.2e}, fallback {fb.cpu().numpy().tolist()}")
    assert e1 <= 1e-4
    assert e0 > e1
    # the default check: relative to the larger of the result and the input
    dflt = tp.tp_prox_tnn_learned(gpu(Y), tau, accuracy=2e-5, max_power_iters=60, **kw).cpu().numpy()
    e2 = float(np.linalg.norm(dflt - exact) / max(np.linalg.norm(exact), np.linalg.norm(Y)))
    say(f"  default check: {e2:.2e} relative to max(|X*|, |Y|)")
    assert e2 <= 1e-4


def test_learned_prox_warm_start(tp, orc):
    """A sequence of prox calls on slowly changing inputs: with the previous
    call's range basis as the sketch, every result stays within 1e-4 of the
    exact prox and the a posteriori check needs fewer power iterations.
    Measured as fallbacks under a budget: for iteration budgets q = 2, 3, ...
    slices still inaccurate after q iterations take the full SVD; the warm
    start never needs more fallbacks than the cold start (a Gaussian sketch
    every call), and fewer for some budget."""
    rng = np.random.default_rng(41)
    n1, n2, n3, r = 120, 110, 6, 5
    # kept values close above a noise bulk (slow subspace convergence from a
    # random start, as in test_learned_prox_accuracy_check)
    P = rng.standard_normal((n1, r, n3)) / np.sqrt(n1)
    Q = rng.standard_normal((r, n2, n3)) / np.sqrt(n2)
    base = orc.tprod(P, Q) * 0.7 + 0.35 * rng.standard_normal((n1, n2, n3)) / np.sqrt(n1)
    h = n3 // 2 + 1
    seq = [(base + 1e-3 * t * rng.standard_normal(base.shape) / np.sqrt(n1)).astype(np.float32) for t in range(5)]
    tau = float(np.sort(orc.slice_sigma(seq[0])[:h, r - 1])[0]) * 0.8
    exact = [orc.prox_tnn(Y, np.float32(tau)) for Y in seq]

    def run(warm, q):
        bs = [torch.zeros(tp.basis_shape(n2, n3, 16), dtype=torch.float32, device="cuda:0") for _ in range(2)]
        bc = [torch.zeros(h, dtype=torch.int32, device="cuda:0") for _ in range(2)]
        fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        errs, nfb = [], 0
        for t, Y in enumerate(seq):
            kw = dict(fixed_rank=5, oversample=3, power_iters=1, max_rank=16, seed=t, accuracy=2e-5,
                      max_power_iters=q, accuracy_ref=1, retry_wide=False, fallback=fb)
            if warm:
                kw.update(basis_out=bs[t % 2], basis_cols_out=bc[t % 2])
                if t > 0:
                    kw.update(warm_basis=bs[(t - 1) % 2], warm_cols=bc[(t - 1) % 2])
            X = tp.tp_prox_tnn_learned(gpu(Y), tau, **kw).cpu().numpy()
            errs.append(rel_fro(X, exact[t]))
            if t > 0:
                nfb += int(fb.sum())
        return max(errs), nfb

    gain = False
    for q in range(2, 13):
        (ec, fc), (ew, fw) = run(False, q), run(True, q)
        say(f"  budget {q}: fallback slices after the first call cold {fc}, warm {fw}; max rel.err {ec:.1e} / {ew:.1e}")
        assert ec <= 1e-4 and ew <= 1e-4
        assert fw <= fc
        gain = gain or fw < fc
        if fc == 0:
            break
    assert gain


def test_rsvd_breakdown_falls_back(tp, orc):
    """Every tube alternates in sign, so only the middle slice k = n3/2 is
    nonzero in exact arithmetic; the DC slice (a sum of +x and -x) comes out
    exactly zero.  There the sketch Y = Ybar Om is zero, its Gram matrix has
    no positive pivot, and the CholeskyQR breakdown must send the slice to
    the full SVD rather than pass a broken basis on.  (The other slices hold
    rounding noise of the transform and may stay on the randomized path.)
    The output stays finite and equal to the exact prox."""
    rng = np.random.default_rng(41)
    n1, n2, n3 = 90, 70, 6
    U = rng.standard_normal((n1, n2))
    Y = (U[:, :, None] * ((-1.0) ** np.arange(n3))[None, None, :]).astype(np.float32)
    tau = 0.2 * orc.tsn(Y)
    h = n3 // 2 + 1
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=6, max_rank=32, fallback=fb, accuracy=0.0).cpu().numpy()
    ref = orc.prox_tnn(Y, np.float32(tau))
    f = fb.cpu().numpy()
    say(f"fallback {f.tolist()} err {rel_fro(X, ref):.2e}")
    assert np.all(np.isfinite(X))
    assert f[0] == 1                     # the exactly zero slice
    assert rel_fro(X, ref) <= 1e-4


@pytest.mark.parametrize("accuracy", [0.0, 2e-5])
def test_rsvd_rank_deficient_narrower_than_sketch(tp, orc, accuracy):
    """Slices of exact rank 3 with a sketch of 32 columns (kpred 20 + 10,
    rounded up): the sketch's Gram matrix is singular.  Either the basis
    passes the checks (its span then contains the whole range and the result
    is exact) or the slice falls back; the output must be finite and equal
    to the exact prox either way."""
    rng = np.random.default_rng(43)
    n1, n2, n3, r = 100, 40, 5, 3
    Y = orc.tprod(rng.standard_normal((n1, r, n3)), rng.standard_normal((r, n2, n3))).astype(np.float32)
    tau = 0.1 * orc.tsn(Y)
    h = n3 // 2 + 1
    fb = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    X = tp.tp_prox_tnn_learned(gpu(Y), tau, fixed_rank=20, max_rank=64, fallback=fb,
                               accuracy=accuracy).cpu().numpy()
    ref = orc.prox_tnn(Y, np.float32(tau))
    say(f"fallback {fb.cpu().numpy().tolist()} err {rel_fro(X, ref):.2e}")
    assert np.all(np.isfinite(X))
    assert rel_fro(X, ref) <= 1e-4


def _graph_case(orc, case):
    """Input and settings of one graph-replay case."""
    from paper_1806_07247_amd import inputs
    if case == "randomized":
        Y = lowrank(orc, 90, 70, 6, 6, seed=17, noise=0.01)
        return Y, 0.1 * orc.tsn(Y), dict(fixed_rank=8, oversample=4, max_rank=24, seed=3)
    if case == "fallback":  # k = 0 on full-rank slices: every slice through the full SVD
        Y = inputs.random_tensor((48, 40, 6), seed=21)
        return Y, 0.05 * orc.tsn(Y), dict(fixed_rank=0, oversample=3, max_rank=16, retry_wide=False)
    if case == "retry":  # under-predicted counts: the wide retry runs
        Y = lowrank(orc, 90, 70, 6, 6, seed=17)
        return Y, 0.1 * orc.tsn(Y), dict(fixed_rank=2, oversample=4, max_rank=24, retry_wide=True)
    # accuracy rounds: kept values close above a noise bulk
    rng = np.random.default_rng(31)
    n, n3, r = 120, 4, 5
    Lt = orc.tprod(rng.standard_normal((n, r, n3)) / np.sqrt(n), rng.standard_normal((r, n, n3)) / np.sqrt(n)) * 0.7
    Y = (Lt + 0.35 * rng.standard_normal((n, n, n3)) / np.sqrt(n)).astype(np.float32)
    sig = orc.slice_sigma(Y)[:3]
    tau = float(np.sort(sig[:, r - 1])[0]) * 0.8
    return Y, tau, dict(fixed_rank=r, oversample=3, power_iters=2, max_rank=16, seed=5, accuracy=2e-5,
                        max_power_iters=6, accuracy_ref=1)


@pytest.mark.parametrize("case", ["randomized", "fallback", "retry", "accuracy"])
def test_learned_prox_graph_replay(tp, orc, case):
    """Every decision of the learned prox (sketch width, accuracy rounds, wide
    retry, fallback to the full SVD) is taken on the device, so the call can
    be captured in a HIP graph: three replays, with eager work and host
    synchronisation between them, give the eager call's bits in the result,
    the counts, the fallback flags, the sweeps and the singular values."""
    Y, tau, kw = _graph_case(orc, case)
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    dev = "cuda:0"
    Yd = gpu(Y)
    ws = torch.empty(tp.tp_prox_tnn_learned_workspace_size(n1, n2, n3, kw["max_rank"]), dtype=torch.uint8,
                     device=dev)
    out = torch.empty_like(Yd)
    bufs = dict(rank=torch.zeros(h, dtype=torch.int32, device=dev), fallback=torch.zeros(h, dtype=torch.int32, device=dev),
                info=torch.zeros(h, dtype=torch.int32, device=dev),
                sigma_out=torch.zeros((h, tp.TP_SIGMA_KEEP), dtype=torch.float32, device=dev))

    def call():
        tp.tp_prox_tnn_learned(Yd, tau, out=out, workspace=ws, **bufs, **kw)

    call()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in bufs.items()}
    ref["X"] = out.clone()
    fb = int(ref["fallback"].sum())
    say(f"{case}: fallback slices {fb} of {h}, rank {ref['rank'].cpu().tolist()}")
    if case == "fallback":
        assert fb == h
    if case in ("randomized", "retry"):
        assert fb == 0
    exact = orc.prox_tnn(Y, np.float32(tau))
    assert rel_fro(ref["X"].cpu().numpy(), exact) <= 1e-4

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()  # warm-up on the capturing stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        call()
    for rep in range(3):
        out.fill_(float("nan"))
        for v in bufs.values():
            v.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref["X"]), f"replay {rep}: result differs"
        for k, v in bufs.items():
            assert torch.equal(v, ref[k]), f"replay {rep}: {k} differs"


LEARNED_HOST = 12  # TP_PARAM_LEARNED_HOST


@pytest.mark.parametrize("case", ["randomized", "fallback", "retry", "accuracy"])
def test_learned_prox_host_driven(tp, orc, case):
    """The host-driven form (the host reads the round, retry and fallback
    decisions and enqueues only the launches that run) gives the bits of the
    device-gated form in the result, the counts, the fallback flags, the
    sweeps, the singular values and the stored basis; on a capturing stream
    it keeps the device-gated form, so a captured call replays to the same
    bits."""
    Y, tau, kw = _graph_case(orc, case)
    n1, n2, n3 = Y.shape
    h = n3 // 2 + 1
    dev = "cuda:0"
    lib = tp._lib.load()
    Yd = gpu(Y)
    ws = torch.empty(tp.tp_prox_tnn_learned_workspace_size(n1, n2, n3, kw["max_rank"]), dtype=torch.uint8,
                     device=dev)
    bshape = tp.basis_shape(n2, n3, kw["max_rank"])

    def fresh():
        return dict(rank=torch.full((h,), -7, dtype=torch.int32, device=dev),
                    fallback=torch.full((h,), -7, dtype=torch.int32, device=dev),
                    info=torch.full((h,), -7, dtype=torch.int32, device=dev),
                    sigma_out=torch.full((h, tp.TP_SIGMA_KEEP), -7.0, dtype=torch.float32, device=dev),
                    basis_out=torch.full(bshape, -7.0, dtype=torch.float32, device=dev),
                    basis_cols_out=torch.full((h,), -7, dtype=torch.int32, device=dev))

    def call(bufs, out):
        tp.tp_prox_tnn_learned(Yd, tau, out=out, workspace=ws, **bufs, **kw)

    results = {}
    try:
        for mode in (0, 1):
            assert lib.tp_set_param(LEARNED_HOST, mode) == 0
            bufs, out = fresh(), torch.full_like(Yd, float("nan"))
            call(bufs, out)
            torch.cuda.synchronize()
            results[mode] = dict(bufs, X=out)
        say(f"{case}: fallback {int(results[0]['fallback'].sum())} of {h}, rank "
            f"{results[0]['rank'].cpu().tolist()}")
        for k, v in results[0].items():
            assert torch.equal(results[1][k], v), f"host-driven {k} differs"
        # captured with the host-driven form requested: the device-gated form runs
        bufs, out = fresh(), torch.full_like(Yd, float("nan"))
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            call(bufs, out)  # warm-up on the capturing stream (host-driven, not capturing)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            call(bufs, out)
        for v in list(bufs.values()) + [out]:
            v.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in results[0].items():
            got = out if k == "X" else bufs[k]
            assert torch.equal(got, v), f"captured replay: {k} differs"
    finally:
        lib.tp_set_param(LEARNED_HOST, 0)
