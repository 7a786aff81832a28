"""GPU parity of the per-slice Jacobi SVD on tall slices (more than 256
rows, the instantiations with 64-lane pair groups) through tp_prox_tnn
(Algorithm 3), tp_tnn (Definition 2.9) and tp_tsvd (Algorithm 2), against
the FP64 oracle, in every form of the kernel: one workgroup per slice with
the slice in LDS (TP_PARAM_JACOBI_MODE 1, where it fits) and the
multi-workgroup block forms (mode 2; always taken when the slice does not fit
in LDS): block pairs through MFMA Gram matrices (the default without V), and
the column-rotation forms, one launch per sweep or per block step.

Tolerances as in the other prox / tnn / tsvd tests: prox 1e-4, tnn 1e-5,
tsvd 1e-5 (relative Frobenius).
"""
import numpy as np
import pytest

from helpers import rel_fro, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

JACOBI_MODE = 1  # TP_PARAM_JACOBI_MODE


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07247_amd as tp
    tp._lib.load()
    return tp


JACOBI_BLOCK = 0     # TP_PARAM_JACOBI_BLOCK
JACOBI_STEPWISE = 9  # TP_PARAM_JACOBI_STEPWISE
JACOBI_GRAM = 11     # TP_PARAM_JACOBI_GRAM: 1 off, 2 / 3 block pairs of 16 / 32 columns


# (mode, stepwise, gram): the Gram form applies to the blocked form without V
# (prox, tnn); tsvd (with V) takes the column-rotation block kernel in all
@pytest.fixture(params=[(1, 0, 0), (2, 0, 2), (2, 0, 3), (2, 2, 1), (2, 1, 1)],
                ids=["one_wg", "blocked_gram16", "blocked_gram32", "blocked_sweep", "blocked_stepwise"])
def mode(request, tp):
    lib = tp._lib.load()
    m, stepwise, gram = request.param
    assert lib.tp_set_param(JACOBI_MODE, m) == 0
    assert lib.tp_set_param(JACOBI_STEPWISE, stepwise) == 0
    assert lib.tp_set_param(JACOBI_GRAM, gram) == 0
    yield request.param
    lib.tp_set_param(JACOBI_MODE, 0)
    lib.tp_set_param(JACOBI_STEPWISE, 0)
    lib.tp_set_param(JACOBI_GRAM, 0)


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


# R = max(n1, n2) > 256: 300 and 520 (64-lane groups, 8 / 16 rows per lane),
# 1024 (16 rows per lane), 1100 (32 rows per lane); narrow ones fit in LDS
PROX_SHAPES = [(300, 60, 4), (60, 300, 5), (520, 36, 3), (1024, 18, 3), (1100, 12, 2), (300, 260, 4),
               (520, 300, 3), (1024, 256, 3), (256, 1024, 2)]


@pytest.mark.parametrize("shape", PROX_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_prox_tall_slices(tp, orc, mode, shape):
    from paper_1806_07247_amd import inputs
    Y = inputs.random_tensor(shape, seed=sum(shape) + 7)
    tau = 0.3 * orc.tsn(Y)
    h = shape[2] // 2 + 1
    info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    rank = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    say(f"prox {shape} mode {mode} tau={tau:.4g}")
    X = tp.tp_prox_tnn(gpu(Y), tau, info=info, rank=rank).cpu().numpy()
    ref = orc.prox_tnn(Y, np.float32(tau))
    err = rel_fro(X, ref)
    say(f"  rel.err {err:.3e} sweeps {info.cpu().numpy().tolist()} rank {rank.cpu().numpy().tolist()}")
    assert err <= 1e-4
    assert int(info.min()) > 0
    sig = orc.slice_sigma(Y)[:h]
    assert np.array_equal(rank.cpu().numpy(), (sig > np.float32(tau)).sum(axis=1))


@pytest.mark.parametrize("shape", [(300, 60, 4), (1024, 18, 3), (520, 300, 3), (256, 1024, 2)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tnn_tall_slices(tp, orc, mode, shape):
    from paper_1806_07247_amd import inputs
    A = inputs.random_tensor(shape, seed=3 * sum(shape))
    say(f"tnn {shape} mode {mode}")
    v = float(tp.tp_tnn(gpu(A)).cpu())
    ref = orc.tnn(A)
    say(f"  {v} vs {ref}")
    assert abs(v - ref) <= 1e-5 * abs(ref)


@pytest.mark.parametrize("shape", [(300, 48, 3), (48, 300, 4), (520, 40, 2), (300, 260, 2)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tsvd_tall_slices(tp, orc, mode, shape):
    from paper_1806_07247_amd import inputs
    A = inputs.random_tensor(shape, seed=11 * sum(shape))
    n1, n2, n3 = shape
    h = n3 // 2 + 1
    info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
    say(f"tsvd {shape} mode {mode}")
    U, S, V = (t.cpu().numpy().astype(np.float64) for t in tp.tp_tsvd(gpu(A), info=info))
    assert int(info.min()) > 0
    rec = orc.tprod(orc.tprod(U, S), orc.tran(V))
    e_rec = rel_fro(rec, A)
    e_u = np.abs(orc.tprod(orc.tran(U), U) - orc.teye(n1, n3)).max()
    e_v = np.abs(orc.tprod(orc.tran(V), V) - orc.teye(n2, n3)).max()
    _, Sref, _, _, _ = orc.tsvd(A)
    e_s = rel_fro(S, Sref)
    say(f"  rec {e_rec:.2e} U^*U {e_u:.2e} V^*V {e_v:.2e} S {e_s:.2e} sweeps {info.cpu().numpy().tolist()}")
    assert e_rec <= 1e-5 and e_s <= 1e-5
    assert e_u <= 1e-4 and e_v <= 1e-4


# The one-launch-per-sweep block kernel (forced) at forced block widths: ragged last
# blocks, an empty padding block (odd block counts), fewer columns than one
# block, tall and wide slices, 16- and 64-lane groups.
@pytest.mark.parametrize("width", [4, 8, 16, 64])
@pytest.mark.parametrize("shape", [(200, 37, 3), (300, 130, 4), (130, 200, 2), (96, 3, 2), (600, 70, 3)],
                         ids=lambda s: "x".join(map(str, s)))
def test_prox_block_widths(tp, orc, shape, width):
    from paper_1806_07247_amd import inputs
    lib = tp._lib.load()
    assert lib.tp_set_param(JACOBI_MODE, 2) == 0
    assert lib.tp_set_param(JACOBI_BLOCK, width) == 0
    assert lib.tp_set_param(JACOBI_STEPWISE, 2) == 0
    assert lib.tp_set_param(JACOBI_GRAM, 1) == 0
    try:
        Y = inputs.random_tensor(shape, seed=5 * sum(shape) + width)
        tau = 0.2 * orc.tsn(Y)
        h = shape[2] // 2 + 1
        info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        rank = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        say(f"prox {shape} block width {width}")
        X = tp.tp_prox_tnn(gpu(Y), tau, info=info, rank=rank).cpu().numpy()
        ref = orc.prox_tnn(Y, np.float32(tau))
        err = rel_fro(X, ref)
        say(f"  rel.err {err:.3e} sweeps {info.cpu().numpy().tolist()}")
        assert err <= 1e-4
        assert int(info.min()) > 0
        sig = orc.slice_sigma(Y)[:h]
        assert np.array_equal(rank.cpu().numpy(), (sig > np.float32(tau)).sum(axis=1))
        v = float(tp.tp_tnn(gpu(Y)).cpu())
        assert abs(v - orc.tnn(Y)) <= 1e-5 * orc.tnn(Y)
    finally:
        lib.tp_set_param(JACOBI_MODE, 0)
        lib.tp_set_param(JACOBI_BLOCK, 0)
        lib.tp_set_param(JACOBI_STEPWISE, 0)
        lib.tp_set_param(JACOBI_GRAM, 0)


# The Gram block sweep (forced, both block-pair widths): ragged last blocks, an
# empty padding block, odd heights (a last row without its pair), heights below
# one MFMA row group, conjugate-transposed wide slices, real DC / Nyquist
# slices (even n3), slices a little above one block pair.
@pytest.mark.parametrize("gram", [2, 3], ids=["gram16", "gram32"])
@pytest.mark.parametrize("shape", [(200, 37, 3), (201, 45, 4), (300, 130, 4), (130, 200, 2), (96, 17, 2),
                                   (600, 70, 3), (200, 200, 5), (7, 40, 3), (1030, 33, 2), (64, 64, 6)],
                         ids=lambda s: "x".join(map(str, s)))
def test_prox_gram_sweep(tp, orc, shape, gram):
    from paper_1806_07247_amd import inputs
    lib = tp._lib.load()
    assert lib.tp_set_param(JACOBI_MODE, 2) == 0
    assert lib.tp_set_param(JACOBI_GRAM, gram) == 0
    try:
        Y = inputs.random_tensor(shape, seed=7 * sum(shape) + gram)
        tau = 0.2 * orc.tsn(Y)
        h = shape[2] // 2 + 1
        info = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        rank = torch.zeros(h, dtype=torch.int32, device="cuda:0")
        say(f"prox {shape} gram {gram}")
        X = tp.tp_prox_tnn(gpu(Y), tau, info=info, rank=rank).cpu().numpy()
        ref = orc.prox_tnn(Y, np.float32(tau))
        err = rel_fro(X, ref)
        say(f"  rel.err {err:.3e} sweeps {info.cpu().numpy().tolist()}")
        assert err <= 1e-4
        assert int(info.min()) > 0
        sig = orc.slice_sigma(Y)[:h]
        assert np.array_equal(rank.cpu().numpy(), (sig > np.float32(tau)).sum(axis=1))
        v = float(tp.tp_tnn(gpu(Y)).cpu())
        assert abs(v - orc.tnn(Y)) <= 1e-5 * orc.tnn(Y)
    finally:
        lib.tp_set_param(JACOBI_MODE, 0)
        lib.tp_set_param(JACOBI_GRAM, 0)


def test_prox_full_size_slices(tp, orc):
    """1024 x 1024 slices (the learned-rank workload's slice shape, 16 rows per
    lane, blocked) against the FP64 prox of Theorem 2.3 written with LAPACK."""
    from paper_1806_07247_amd import inputs
    parts = inputs.lowrank_sparse_parts(1024, 1024, 4, 12, 1.0 / 1024, 0.05, 0.0, seed=21)
    Y = (orc.tprod(parts["P"], parts["Q"]) + parts["S"]).astype(np.float32)
    # tau at a tenth of the spectral norm of the DC slice (numpy's SVD: the
    # threshold only has to fall inside the spectrum)
    tau = 0.1 * float(np.linalg.svd(Y.astype(np.float64).sum(axis=2), compute_uv=False)[0])
    info = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    say("prox 1024x1024x4 (blocked, one launch per sweep)")
    X = tp.tp_prox_tnn(gpu(Y), tau, info=info).cpu().numpy()
    ref = orc.prox_tnn_lapack(Y, float(np.float32(tau)))
    err = rel_fro(X, ref)
    say(f"  rel.err {err:.3e} sweeps {info.cpu().numpy().tolist()}")
    assert err <= 1e-4
    assert int(info.min()) > 0
