"""Pins of the order-p oracle (oracle/nd.py) against what the definitions
fix, independent of its own formulas: the 3-way product of the package, the
unrolled circular convolution by brute force, reductions when a mode has
size 1, the identity, associativity, the transpose identity, TNN of the
identity, and optimality of the prox."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng


def rand(*shape, seed=0):
    return RNG(seed).standard_normal(shape)


def test_p3_fft_route_is_the_three_way_product():
    A, B = rand(4, 3, 5, seed=1), rand(3, 2, 5, seed=2)
    C = oracle.tprod(A, B)
    assert np.allclose(oracle.tprod_nd(A, B), C, atol=1e-12)
    assert np.allclose(oracle.tprod_nd_fft(A, B), C, atol=1e-12)


@pytest.mark.parametrize("dims", [(2, 3), (3, 1, 2), (1, 2, 2)])
def test_definition_is_the_circular_convolution(dims):
    A, B = rand(3, 2, *dims, seed=3), rand(2, 4, *dims, seed=4)
    conv = oracle.tprod_nd_conv(A, B)
    assert np.allclose(oracle.tprod_nd(A, B), conv, atol=1e-12)
    assert np.allclose(oracle.tprod_nd_fft(A, B), conv, atol=1e-12)


def test_brute_force_conv_by_hand():
    # 1 x 1 frontal slices: the product is the plain 2-D circular convolution
    a, b = rand(1, 1, 3, 4, seed=5), rand(1, 1, 3, 4, seed=6)
    ref = np.zeros((3, 4))
    for i in range(3):
        for j in range(4):
            for p in range(3):
                for q in range(4):
                    ref[i, j] += a[0, 0, p, q] * b[0, 0, (i - p) % 3, (j - q) % 4]
    assert np.allclose(oracle.tprod_nd(a, b)[0, 0], ref, atol=1e-12)


def test_unit_last_mode_reduces_to_lower_order():
    A, B = rand(3, 4, 5, seed=7), rand(4, 2, 5, seed=8)
    C = oracle.tprod(A, B)
    assert np.allclose(oracle.tprod_nd(A[..., None], B[..., None])[..., 0], C, atol=1e-12)
    assert np.allclose(oracle.tprod_nd_fft(A[..., None, None], B[..., None, None])[..., 0, 0], C, atol=1e-12)


def test_identity_both_sides():
    dims = (3, 2)
    A = rand(4, 3, *dims, seed=9)
    assert np.allclose(oracle.tprod_nd(oracle.teye_nd(4, dims), A), A, atol=1e-12)
    assert np.allclose(oracle.tprod_nd(A, oracle.teye_nd(3, dims)), A, atol=1e-12)


def test_associative():
    dims = (2, 3)
    A, B, C = rand(2, 3, *dims, seed=10), rand(3, 2, *dims, seed=11), rand(2, 2, *dims, seed=12)
    lhs = oracle.tprod_nd(oracle.tprod_nd(A, B), C)
    rhs = oracle.tprod_nd(A, oracle.tprod_nd(B, C))
    assert np.allclose(lhs, rhs, atol=1e-10)


def test_transpose_of_product():
    dims = (3, 2, 2)
    A, B = rand(2, 3, *dims, seed=13), rand(3, 4, *dims, seed=14)
    lhs = oracle.tran_nd(oracle.tprod_nd_fft(A, B))
    rhs = oracle.tprod_nd_fft(oracle.tran_nd(B), oracle.tran_nd(A))
    assert np.allclose(lhs, rhs, atol=1e-12)
    # for p = 3 the transpose is Definition 2.2 of the package
    A3 = rand(3, 4, 5, seed=15)
    assert np.allclose(oracle.tran_nd(A3), oracle.tran(A3), atol=0)


def test_tnn_identity_and_three_way():
    assert oracle.tnn_nd(oracle.teye_nd(5, (3, 4))) == pytest.approx(5.0, rel=1e-12)
    A = rand(4, 3, 6, seed=16)
    assert oracle.tnn_nd(A) == pytest.approx(oracle.tnn(A), rel=1e-10)
    # a mode of size 1 changes nothing
    assert oracle.tnn_nd(A[..., None]) == pytest.approx(oracle.tnn(A), rel=1e-10)


def test_prox_reductions():
    Y = rand(4, 3, 5, seed=17)
    assert np.allclose(oracle.prox_tnn_nd(Y, 0.0), Y, atol=1e-12)
    ref = oracle.prox_tnn(Y, 0.7)
    assert np.allclose(oracle.prox_tnn_nd(Y, 0.7), ref, atol=1e-10)
    assert np.allclose(oracle.prox_tnn_nd(Y[..., None], 0.7)[..., 0], ref, atol=1e-10)


def test_prox_is_the_minimiser():
    """X = Prox_tau(Y) minimises tau ||X||_* + ||X - Y||^2 / 2: no random
    perturbation lowers the objective (independent of the SVT formula)."""
    Y = rand(3, 4, 2, 3, seed=18)
    tau = 0.9
    X = oracle.prox_tnn_nd(Y, tau)

    def f(Z):
        return tau * oracle.tnn_nd(Z) + 0.5 * np.sum((Z - Y) ** 2)

    f0 = f(X)
    rng = RNG(19)
    for _ in range(20):
        D = rng.standard_normal(Y.shape)
        for eps in (1e-2, 1e-3):
            assert f(X + eps * D) >= f0 - 1e-12
    # and it shrinks: some slice rank drops at this tau
    assert oracle.tnn_nd(X) < oracle.tnn_nd(Y)
