"""GPU parity of tp_tprod (Algorithm 1) against the FP64 oracle.

Tolerance: relative Frobenius error <= 1e-5 for FP32 and split-BF16 (BF16X3)
slice products; plain BF16 is only bounded loosely (its error is reported by
the benchmark).  The oracle is the definition (eq (9)) on the same float32
inputs, upcast to float64.
"""
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


TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 2e-2}

SHAPES = [
    (1, 1, 1, 1), (1, 1, 1, 5), (3, 2, 4, 1), (5, 3, 7, 2), (5, 3, 7, 3), (7, 9, 4, 4),
    (6, 5, 4, 7), (17, 13, 11, 8), (33, 31, 29, 16), (64, 48, 40, 32), (130, 70, 129, 5),
    (65, 17, 66, 50), (70, 65, 80, 64), (40, 36, 33, 128), (20, 30, 10, 100),
]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_tprod_matches_definition(tp, orc, shape, prec):
    from paper_1806_07247_amd import inputs
    n1, n2, l, n3 = shape
    say(f"tprod {shape} {prec}")
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=sum(shape))
    C = tp.tp_tprod(gpu(A), gpu(B), prec=prec).cpu().numpy()
    ref = orc.tprod(A, B)
    err = rel_fro(C, ref)
    say(f"  rel.err {err:.3e}")
    assert err <= TOL[prec]


def test_tprod_parity_config(tp, orc):
    """A 64x48x32, B 48x40x32, N(0,1), seed 0: 17 slice products."""
    from paper_1806_07247_amd import inputs
    A, B = inputs.tprod_parity(seed=0)
    ref = orc.tprod(A, B)
    for prec in ("fp32", "bf16x3"):
        C = tp.tp_tprod(gpu(A), gpu(B), prec=prec).cpu().numpy()
        err = rel_fro(C, ref)
        say(f"parity config {prec}: rel.err {err:.3e}")
        assert err <= 1e-5


def test_tprod_identity_and_transpose(tp, orc):
    from paper_1806_07247_amd import inputs
    A = inputs.random_tensor((37, 29, 12), seed=3)
    Ie = orc.teye(29, 12).astype(np.float32)
    C = tp.tp_tprod(gpu(A), gpu(Ie)).cpu().numpy()
    assert rel_fro(C, A) < 1e-6
    B = inputs.random_tensor((29, 21, 12), seed=4)
    lhs = orc.tran(tp.tp_tprod(gpu(A), gpu(B)).cpu().numpy())
    rhs = tp.tp_tprod(gpu(orc.tran(B).astype(np.float32)), gpu(orc.tran(A).astype(np.float32))).cpu().numpy()
    assert rel_fro(lhs, rhs) < 1e-5


def test_tprod_deterministic(tp):
    from paper_1806_07247_amd import inputs
    A, B = inputs.tprod_pair(100, 90, 80, 16, seed=9)
    a, b = gpu(A), gpu(B)
    for prec in ("fp32", "bf16x3"):
        c1 = tp.tp_tprod(a, b, prec=prec)
        c2 = tp.tp_tprod(a, b, prec=prec)
        assert torch.equal(c1, c2)


def test_tprod_precision_config_sampled(tp, orc):
    """A 512x512x128, B 512x256x128 (the precision workload): 4000 entries
    checked against the definition, in the launch configuration the
    benchmark times."""
    from paper_1806_07247_amd import inputs
    A, B = inputs.tprod_precision(seed=0)
    rng = np.random.default_rng(1)
    idx = rng.choice(512 * 256 * 128, size=4000, replace=False)
    ref = orc.tprod_entries(A, B, idx)
    for prec in ("fp32", "bf16x3", "bf16"):
        say(f"precision config {prec}")
        C = tp.tp_tprod(gpu(A), gpu(B), prec=prec).cpu().numpy().reshape(-1)
        err = rel_fro(C[idx], ref)
        say(f"  sampled rel.err {err:.3e}")
        assert err <= TOL[prec]


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
def test_tprod_every_tile_variant(tp, orc, variant, prec):
    """Each slice-product tile shape (forced through TP_PARAM_GEMM_VARIANT) on
    a shape with ragged edges in every dimension (75 output columns: FP32
    variants 7 and 8 fall back to the 64 x 64 tile; bf16 variants 1-5 are
    its five tiles, 6-8 the 64 x 64 one)."""
    from paper_1806_07247_amd import _lib, inputs
    lib = _lib.load()
    A, B = inputs.tprod_pair(131, 67, 75, 6, seed=variant)
    ref = orc.tprod(A, B)
    try:
        assert lib.tp_set_param(4, variant) == 0
        C = tp.tp_tprod(gpu(A), gpu(B), prec=prec).cpu().numpy()
    finally:
        lib.tp_set_param(4, 0)
    err = rel_fro(C, ref)
    say(f"  variant {variant} {prec}: rel.err {err:.2e}")
    assert err <= TOL[prec]


NARROW = [(131, 67, 40, 6), (200, 333, 8, 5), (64, 64, 64, 4), (257, 1024, 16, 3), (70, 96, 4, 7),
          (128, 256, 48, 4), (1, 64, 12, 2), (96, 100, 20, 9)]


@pytest.mark.parametrize("shape", NARROW, ids=lambda s: "x".join(map(str, s)))
def test_tprod_narrow_output_kernel(tp, orc, shape):
    """FP32 slice products with at most 64 output columns (a multiple of 4)
    and an inner dimension >= 64 take the narrow-output kernel: full 64-row
    tiles with whole 32-deep stages (the unmasked loop) and ragged rows, inner
    dimensions and widths (the masked loop); real first and last slices."""
    from paper_1806_07247_amd import inputs
    n1, n2, l, n3 = shape
    say(f"tprod narrow {shape}")
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=7 * sum(shape))
    C = tp.tp_tprod(gpu(A), gpu(B), prec="fp32").cpu().numpy()
    err = rel_fro(C, orc.tprod(A, B))
    say(f"  rel.err {err:.3e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("shape", [(100, 40, 24, 5), (64, 16, 8, 4), (70, 3, 4, 2)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tprod_narrow_output_kernel_short_inner(tp, orc, shape):
    """The narrow-output kernel forced (variant 7) on inner dimensions below
    its by-shape threshold: a single partial stage, masked."""
    from paper_1806_07247_amd import _lib, inputs
    lib = _lib.load()
    n1, n2, l, n3 = shape
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=3 * sum(shape))
    try:
        assert lib.tp_set_param(4, 7) == 0
        C = tp.tp_tprod(gpu(A), gpu(B), prec="fp32").cpu().numpy()
    finally:
        lib.tp_set_param(4, 0)
    err = rel_fro(C, orc.tprod(A, B))
    say(f"  narrow forced {shape}: rel.err {err:.2e}")
    assert err <= TOL["fp32"]


WIDE = [(64, 17, 256, 5), (128, 48, 512, 4), (192, 1, 256, 3), (64, 40, 768, 6), (128, 32, 256, 2),
        (64, 8, 512, 9), (130, 40, 40, 5), (64, 48, 64, 3), (1000, 8, 16, 4), (33, 12, 4, 6), (5, 3, 60, 2)]


@pytest.mark.parametrize("shape", WIDE, ids=lambda s: "x".join(map(str, s)))
def test_tprod_wide_output_kernel(tp, orc, shape):
    """FP32 slice products with an inner dimension of at most 48 take the
    wide-output kernel (A in registers, the output streamed): whole 64 x 256
    output tiles, and (masked) outputs at most 64 columns wide with ragged
    rows; inner dimensions 1 .. 48 (ragged against its 16-deep stages), real
    first and last slices."""
    from paper_1806_07247_amd import inputs
    n1, n2, l, n3 = shape
    say(f"tprod wide {shape}")
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=11 * sum(shape))
    C = tp.tp_tprod(gpu(A), gpu(B), prec="fp32").cpu().numpy()
    err = rel_fro(C, orc.tprod(A, B))
    say(f"  rel.err {err:.3e}")
    assert err <= TOL["fp32"]


def _sweep_shapes(count=40, seed=2024):
    """Seeded random shapes biased to the slice-product kernels' boundaries:
    output widths multiples of 4 up to 64 (narrow / masked wide), inner
    dimensions around 48 and 64, 64-row and 256-column multiples, and ragged
    sizes that fall back to the tiles."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n1 = int(rng.choice([int(rng.integers(1, 200)), 64 * int(rng.integers(1, 4))]))
        n2 = int(rng.choice([int(rng.integers(1, 130)), 48, 64, 65, 47, 256, 300]))
        l = int(rng.choice([4 * int(rng.integers(1, 17)), int(rng.integers(1, 70)), 256]))
        n3 = int(rng.integers(1, 9))
        out.append((n1, n2, l, n3))
    return out


@pytest.mark.parametrize("shape", _sweep_shapes(), ids=lambda s: "x".join(map(str, s)))
def test_tprod_shape_sweep(tp, orc, shape):
    """FP32 tprod on seeded random shapes against the FP64 oracle (whichever
    slice-product kernel each shape selects)."""
    from paper_1806_07247_amd import inputs
    n1, n2, l, n3 = shape
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=n1 * 7 + n2 * 3 + l + n3)
    C = tp.tp_tprod(gpu(A), gpu(B), prec="fp32").cpu().numpy()
    err = rel_fro(C, orc.tprod(A, B))
    say(f"  sweep {shape}: rel.err {err:.2e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("direct", [1, 2])
@pytest.mark.parametrize("shape", [(33, 31, 29, 8), (70, 65, 80, 64), (40, 36, 33, 128), (17, 13, 11, 16)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tprod_fft_load_variants(tp, orc, direct, shape):
    """Forward transform with direct per-lane tube loads (1) and LDS-staged
    loads (2), forced through TP_PARAM_FFT_DIRECT."""
    from paper_1806_07247_amd import _lib, inputs
    lib = _lib.load()
    n1, n2, l, n3 = shape
    A, B = inputs.tprod_pair(n1, n2, l, n3, seed=n3 + direct)
    try:
        assert lib.tp_set_param(6, direct) == 0
        C = tp.tp_tprod(gpu(A), gpu(B)).cpu().numpy()
    finally:
        lib.tp_set_param(6, 0)
    assert rel_fro(C, orc.tprod(A, B)) <= TOL["fp32"]
