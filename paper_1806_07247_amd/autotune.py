"""Autotuner for the launch schedules of libtp.so.

Candidates are equivalent schedules selected through tp_set_param (Jacobi
block width and mode, slice GEMM tile variant).  Each candidate is timed with
HIP events on the current GPU and its result is checked against the default
schedule (same operation, same input) before it can be chosen.  The winners
are written to a JSON cache keyed by operation and shape bucket; the Python
binding applies the cached parameters before each call whose shape falls in
a tuned bucket.

    python -m paper_1806_07247_amd.autotune [--out FILE] [--quick]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_gfx950.json")

PARAM = {"jacobi_block": 0, "jacobi_mode": 1, "jacobi_blocked_below": 2, "jacobi_sweeps": 3,
         "gemm_variant": 4}


def _bucket(v):
    b = 1
    while b < v:
        b *= 2
    return b


def svd_key(n1, n2, n3):
    """Bucket of an SVD-based call: (rows, cols) of the work matrix rounded up
    to powers of two and the number of half-spectrum slices."""
    R, P = max(n1, n2), min(n1, n2)
    return f"svd:{_bucket(R)}x{_bucket(P)}:h{_bucket(n3 // 2 + 1)}"


def gemm_key(n1, n2, l, n3):
    return f"gemm:{_bucket(n1)}x{_bucket(n2)}x{_bucket(l)}:h{_bucket(n3 // 2 + 1)}"


_cache = None


def load_cache(path=CACHE):
    global _cache
    if _cache is None:
        _cache = {}
        if os.path.exists(path):
            with open(path) as f:
                _cache = json.load(f)
    return _cache


def apply(lib, key):
    """Set the cached parameters of bucket `key` (defaults for the rest)."""
    entry = load_cache().get(key, {})
    for name, k in PARAM.items():
        lib.tp_set_param(k, int(entry.get(name, 0)))


def _time(fn, reps=10, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_svd(lib, shape, seed=0, widths=(8, 10, 13, 17, 21, 25, 32, 40), tol=1e-5):
    import torch

    import paper_1806_07247_amd as tp
    from paper_1806_07247_amd import inputs
    n1, n2, n3 = shape
    Y = torch.from_numpy(inputs.random_tensor(shape, seed=seed)).cuda()
    tau = 0.05 * float(Y.abs().max())
    for k in PARAM.values():
        lib.tp_set_param(k, 0)
    ref = tp.tp_prox_tnn(Y, tau)
    results = []
    cands = [{"jacobi_mode": 1}] + [{"jacobi_mode": 2, "jacobi_block": w} for w in widths]
    for c in cands:
        for k in PARAM.values():
            lib.tp_set_param(k, 0)
        for name, v in c.items():
            lib.tp_set_param(PARAM[name], v)
        try:
            X = tp.tp_prox_tnn(Y, tau)
        except Exception as e:  # a schedule that cannot run this shape
            results.append((float("inf"), c, str(e)))
            continue
        d = float(torch.linalg.norm(X - ref) / torch.linalg.norm(ref))
        if not d <= tol:
            results.append((float("inf"), c, f"mismatch {d:.2e}"))
            continue
        ms = _time(lambda: tp.tp_prox_tnn(Y, tau))
        results.append((ms, c, ""))
        print(f"  {shape} {c}: {ms:.3f} ms", file=sys.stderr, flush=True)
    for k in PARAM.values():
        lib.tp_set_param(k, 0)
    best = min(results, key=lambda r: r[0])
    return best, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--shapes", default="200x200x50,128x128x16,64x64x64,1024x1024x8")
    args = ap.parse_args()
    import torch  # noqa: F401

    from paper_1806_07247_amd import _lib
    lib = _lib.load()
    cache = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            cache = json.load(f)
    for s in args.shapes.split(","):
        shape = tuple(int(v) for v in s.split("x"))
        (ms, c, _), res = tune_svd(lib, shape)
        key = svd_key(*shape)
        cache[key] = dict(c, ms=round(ms, 4), shape=s)
        print(f"{key}: {c} {ms:.3f} ms", flush=True)
    with open(args.out, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
