"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the t-product
arithmetic.  A low-tubal-rank tensor L = P * Q is returned as its factors P
and Q: whoever needs L composes it (the tests with the CPU oracle, the
benchmark with the library's own t-product).

Every generator uses numpy's PCG64 with independent child streams spawned from
one SeedSequence per (workload, seed), drawn in float64 and rounded once to
float32, which is the precision every consumer receives.

Workloads (all sizes n1 x n2 x n3, tube index last, C-contiguous):
  * tprod parity     A 64x48x32, B 48x40x32, i.i.d. N(0,1)
  * prox full SVD    Y = P*Q + S + E, 200x200x50: P 200x10x50, Q 10x200x50
                     i.i.d. N(0, 1/200); S has exactly 10% of its entries set to
                     a random sign (+-1) at uniformly drawn distinct positions;
                     E i.i.d. N(0, 1e-3) (1e-3 is the variance);
                     tau = 1/sqrt(200*50)
  * tprod precision  A 512x512x128, B 512x256x128, i.i.d. N(0,1)
  * batching         256 tensors, n1, n2, l ~ U{16..128}, n3 ~ U{8,16,32,64},
                     i.i.d. N(0,1)
  * learned rank     1024x1024x64, r ~ U{5..40}, P 1024xrx64 and Q rx1024x64
                     i.i.d. N(0, 1/1024), 5% sparse +-1 outliers
"""
import numpy as np

_STREAMS = 8


def _streams(seed: int, tag: int):
    ss = np.random.SeedSequence([int(seed), int(tag)])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(_STREAMS)]


def gaussian(rng, shape, var=1.0):
    """i.i.d. N(0, var) in float64, rounded to float32."""
    return (rng.standard_normal(shape) * np.sqrt(var)).astype(np.float32)


def sparse_signs(rng, shape, frac):
    """exactly round(frac*N) entries set to +-1 (Rademacher) at distinct uniform positions."""
    n = int(np.prod(shape))
    k = int(round(frac * n))
    out = np.zeros(n, dtype=np.float32)
    pos = rng.choice(n, size=k, replace=False)
    out[pos] = np.where(rng.integers(0, 2, size=k) == 0, -1.0, 1.0).astype(np.float32)
    return out.reshape(shape)


# ---------------------------------------------------------------- workloads --
def tprod_pair(n1, n2, l, n3, seed=0):
    """A (n1 x n2 x n3) and B (n2 x l x n3), i.i.d. N(0,1)."""
    ra, rb = _streams(seed, 1)[:2]
    return gaussian(ra, (n1, n2, n3)), gaussian(rb, (n2, l, n3))


def tprod_parity(seed=0):
    return tprod_pair(64, 48, 40, 32, seed)


def tprod_precision(seed=0):
    return tprod_pair(512, 512, 256, 128, seed)


def lowrank_sparse_parts(n1, n2, n3, r, var_pq, sparse_frac, noise_var, seed=0):
    """Factors and additive parts of Y = P*Q + S + E.

    Returns dict(P, Q, S, E) (E is None when noise_var == 0)."""
    rp, rq, rs, re_ = _streams(seed, 2)[:4]
    P = gaussian(rp, (n1, r, n3), var_pq)
    Q = gaussian(rq, (r, n2, n3), var_pq)
    S = sparse_signs(rs, (n1, n2, n3), sparse_frac)
    E = gaussian(re_, (n1, n2, n3), noise_var) if noise_var > 0 else None
    return dict(P=P, Q=Q, S=S, E=E)


def prox_full_parts(seed=0, n=200, n3=50, r=10):
    """Parts of the full-SVD prox workload; tau = 1/sqrt(n*n3)."""
    parts = lowrank_sparse_parts(n, n, n3, r, 1.0 / n, 0.10, 1e-3, seed)
    parts["tau"] = 1.0 / np.sqrt(n * n3)
    return parts


def learned_rank_parts(seed=0, n=1024, n3=64):
    rr = _streams(seed, 3)[0]
    r = int(rr.integers(5, 41))
    parts = lowrank_sparse_parts(n, n, n3, r, 1.0 / n, 0.05, 0.0, seed)
    parts["r"] = r
    return parts


def batch_shapes(count=256, seed=0):
    """(n1, n2, l, n3) for each tensor of the batching workload."""
    rng = _streams(seed, 4)[0]
    n1 = rng.integers(16, 129, size=count)
    n2 = rng.integers(16, 129, size=count)
    l = rng.integers(16, 129, size=count)
    n3 = rng.choice(np.array([8, 16, 32, 64]), size=count)
    return [(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(n1, n2, l, n3)]


def batch_tensors(shapes, seed=0):
    """A_i (n1 x n2 x n3) and B_i (n2 x l x n3) for every shape, i.i.d. N(0,1)."""
    rng = _streams(seed, 5)[0]
    out = []
    for (n1, n2, l, n3) in shapes:
        out.append((gaussian(rng, (n1, n2, n3)), gaussian(rng, (n2, l, n3))))
    return out


def random_tensor(shape, seed=0, var=1.0):
    return gaussian(_streams(seed, 6)[0], shape, var)


def tensor_nd(shape, seed=0, var=1.0):
    """An order-p tensor of the given shape, i.i.d. N(0, var), float32."""
    return gaussian(_streams(seed, 7)[0], tuple(shape), var)


def lowrank_nd(n1, n2, dims, r, seed=0):
    """P * Q of order p (P n1 x r x dims, Q r x n2 x dims, i.i.d. N(0, 1/n1)),
    returned as the two factors; the product is formed by the caller."""
    rp, rq = _streams(seed, 8)[:2]
    return gaussian(rp, (n1, r) + tuple(dims), 1.0 / n1), gaussian(rq, (r, n2) + tuple(dims), 1.0 / n1)

