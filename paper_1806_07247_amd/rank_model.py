"""Training and evaluation of the per-slice rank predictor.

Training samples come from the method's own prox calls inside TRPCA-ADMM
runs (trpca.py): for every call and every leading Fourier slice, the
features of tp_slice_features (with the previous call's count and leading
singular values of that slice) and the exact count k* of singular values
above tau (from the widest randomized sketch with the a posteriori check, or
the full SVD where that falls back).
The target is t = log1p(k*) / log1p(min(n1, n2)); the network is trained on
the GPU with the library's own kernels (tp_mlp_loss_grad, tp_mlp_adam) on the
asymmetric squared loss (under-prediction weighted `under` times, since it
costs a fallback to the full SVD).

    python -m paper_1806_07247_amd.rank_model train [--out FILE] [--runs N] ...
    python -m paper_1806_07247_amd.rank_model train --native --shapes 1024x1024x64 --runs 2000
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

import paper_1806_07247_amd as tp
from paper_1806_07247_amd import trpca

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "rank_mlp_gfx950.npy")


def init_params(seed=0):
    """He-uniform weights, zero biases, packed as in include/tp.h."""
    rng = np.random.default_rng(seed)
    D, H = tp.TP_MLP_INPUTS, 64
    parts = []
    for fan_in, fan_out in ((D, H), (H, H), (H, H), (H, 1)):
        b = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-b, b, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == tp.tp_mlp_param_count()
    return p


def save(params, path=WEIGHTS, meta=None):
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)
    if meta is not None:
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1, sort_keys=True)


def load(path=WEIGHTS, device="cuda:0"):
    p = np.load(path, allow_pickle=False)
    return torch.from_numpy(p.astype(np.float32)).to(device)


def label_prox(shape, device, max_rank=64, oversample=10):
    """Exact per-slice counts at a fraction of the full-SVD cost: the learned
    path with the widest sketch (kpred = max_rank - oversample) and the
    a posteriori check; slices with more singular values above tau fall back
    to the full SVD, whose count is exact as well."""
    return trpca.ProxLearned(shape, device, mlp=None, fixed_rank=max_rank - oversample, oversample=oversample,
                             max_rank=max_rank, use_prev=False)


def rank_for(n, rng):
    """Tubal rank of the learned-rank workload, r ~ U{5..40} at n = 1024,
    scaled to smaller n."""
    r = int(rng.integers(5, 41))
    return max(2, int(round(r * n / 1024.0)))


def collect(shapes, runs, seed0, device, max_iter=200, log=print):
    """Features and targets from TRPCA runs on n x n x n3 problems (tubal rank
    r, 5% +-1 outliers); the previous call's count of each slice is a feature."""
    feats, targets = [], []
    run = 0
    for shape in shapes:
        n, _, n3 = shape
        for _ in range(runs):
            seed = seed0 + run
            run += 1
            rng = np.random.default_rng(seed)
            r = rank_for(n, rng)
            X, _, _ = trpca.make_problem(n, n3, r, 0.05, seed, device)
            prox = label_prox(shape, device)
            prev = {"rank": None, "sigma": None}

            def record(Yin, tau, rank, sigma):
                f = tp.tp_slice_features(Yin, tau, prev["rank"], prev["sigma"])
                feats.append(f.cpu().numpy())
                t = np.log1p(rank.cpu().numpy().astype(np.float64)) / np.log1p(min(shape[0], shape[1]))
                targets.append(t)
                prev["rank"] = rank.clone()
                prev["sigma"] = sigma.clone()

            t0 = time.perf_counter()
            res = trpca.trpca(X, prox, max_iter=max_iter, record=record)
            log(f"  {shape} seed {seed} r {r}: {res['iters']} iterations, {prox.fallbacks} fallback slices, "
                f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return np.concatenate(feats).astype(np.float32), np.concatenate(targets).astype(np.float32)


def problem_gpu(n, n3, seed, device, frac=0.05):
    """A training problem of the learned-rank workload's recipe, drawn on the
    device from torch's seeded generator (host generation of 1024^2 x 64
    problems costs seconds each): tubal rank r ~ U{5..40} scaled to n as in
    rank_for, P (n x r x n3) and Q (r x n x n3) entries N(0, 1/n), X = P*Q + S
    with +-1 outliers at Bernoulli(frac) positions.  Returns (X, r)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = int(torch.randint(5, 41, (1,), generator=g, device=device).item())
    r = max(2, int(round(r * n / 1024.0)))
    P = torch.randn((n, r, n3), generator=g, device=device) / math.sqrt(n)
    Q = torch.randn((r, n, n3), generator=g, device=device) / math.sqrt(n)
    pos = torch.rand((n, n, n3), generator=g, device=device) < frac
    sgn = torch.rand((n, n, n3), generator=g, device=device) < 0.5
    S = torch.where(pos, torch.where(sgn, -1.0, 1.0), 0.0).to(torch.float32)
    X = tp.tp_tprod(P.contiguous(), Q.contiguous())
    X.add_(S)
    return X, r


def collect_native(shape, runs, seed0, device, labeller=None, max_iter=100, log=print):
    """Training samples from native TRPCA runs (tp_trpca with its per-call
    record): the features of every prox input (with the previous call's count
    and singular values) and the exact count of every slice, from the
    learned prox with the count check, the accuracy rounds, the wide retry and
    the full-SVD fallback (so the count is exact whatever the labeller's
    network predicts; labeller None uses the widest sketch).  Samples stay on
    the device.  Returns (F, T) torch tensors."""
    n1, n2, n3 = shape
    h = n3 // 2 + 1
    p = min(n1, n2)
    rec = dict(max_calls=max_iter,
               features=torch.zeros((max_iter, h, tp.TP_MLP_INPUTS), dtype=torch.float32, device=device),
               counts=torch.zeros((max_iter, h), dtype=torch.int32, device=device))
    lo = dict(mlp=labeller, fixed_rank=0 if labeller is not None else 54, accuracy=2e-5)
    feats, targets = [], []
    t0 = time.perf_counter()
    for i in range(runs):
        seed = seed0 + i
        X, r = problem_gpu(n1, n3, seed, device)
        lo["seed"] = seed * 1000
        res = tp.tp_trpca(X, learned=lo, max_iter=max_iter, record=rec)
        k = min(res["iters"], max_iter)
        feats.append(rec["features"][:k].reshape(-1, tp.TP_MLP_INPUTS).clone())
        c = rec["counts"][:k].reshape(-1).to(torch.float64)
        targets.append((torch.log1p(c) / math.log1p(p)).to(torch.float32))
        if i % 100 == 0 or i == runs - 1:
            log(f"  run {i + 1}/{runs} seed {seed} r {r}: {res['iters']} iterations, converged {res['converged']}, "
                f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return torch.cat(feats), torch.cat(targets)


def train(F, T, device, steps=3000, batch=4096, lr=2e-3, under=4.0, seed=0, log=print):
    params = torch.from_numpy(init_params(seed)).to(device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    Fd = F.to(device) if isinstance(F, torch.Tensor) else torch.from_numpy(F).to(device)
    Td = T.to(device) if isinstance(T, torch.Tensor) else torch.from_numpy(T).to(device)
    n = F.shape[0]
    rng = np.random.default_rng(seed + 1)
    ws = torch.empty(tp._lib.load().tp_mlp_train_workspace_size(min(batch, n)), dtype=torch.uint8, device=device)
    grad = torch.empty_like(params)
    loss = torch.empty((), dtype=torch.float32, device=device)
    hist = []
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.integers(0, n, size=min(batch, n))).to(device)
        tp.tp_mlp_loss_grad(params, Fd[idx].contiguous(), Td[idx].contiguous(), under=under, grad=grad, loss=loss,
                            workspace=ws)
        lr_t = lr * (0.5 * (1 + math.cos(math.pi * step / steps)) * 0.9 + 0.1)
        tp.tp_mlp_adam(params, grad, m, v, step, lr=lr_t)
        if step % 250 == 0 or step == 1:
            hist.append((step, float(loss)))
            log(f"  step {step}: loss {float(loss):.5f}", file=sys.stderr, flush=True)
    return params, hist


def evaluate(params, F, T, device):
    """Under-prediction rate and mean absolute error of the predicted counts;
    p is recovered from the feature log(p)/8."""
    if isinstance(F, torch.Tensor):
        F, T = F.cpu().numpy(), T.cpu().numpy()
    y = tp.tp_mlp_forward(params, torch.from_numpy(F).to(device)).cpu().numpy()
    p = np.rint(np.exp(F[:, 6].astype(np.float64) * 8.0))
    kpred = np.clip(np.rint(np.expm1(y * np.log1p(p))), 0, p)
    ktrue = np.rint(np.expm1(T * np.log1p(p)))
    under = float(np.mean(kpred < ktrue))
    mae = float(np.mean(np.abs(kpred - ktrue)))
    return dict(under_rate=under, mae=mae)


class PrevRank(trpca.ProxLearned):
    """No network: each slice's predicted count is the largest count of the
    previous call (0 at the first call)."""

    name = "prev"

    def __call__(self, Y, tau, out):
        self.fixed_rank = int(self.prev.max()) if self.have_prev else 0
        return super().__call__(Y, tau, out)


def gain(mlp, seeds, device, shape=(1024, 1024, 64), full_runs=1, log=print, extra=None):
    """TRPCA on held-out problems of the learned-rank workload, driven by the
    prox with the trained network, without it (previous count; a constant
    count), and with the full SVD (the paper's method).  Reports total prox
    time, fallback slices, recovery error, and the error of sampled learned
    prox calls against the full-SVD prox on the same inputs."""
    n, _, n3 = shape
    out = {"shape": list(shape), "runs": []}
    for si, seed in enumerate(seeds):
        X, L0, r = trpca.learned_workload(seed, device, n, n3)
        row = {"seed": seed, "r": r}
        caps = []
        mlp_prox = trpca.ProxLearned(shape, device, mlp=mlp)

        def cap(k, Y, tau):  # inputs and the previous call's outputs of some mlp-driven calls
            if k % 6 == 3 and mlp_prox.have_prev:
                caps.append((k, Y.clone(), tau, mlp_prox.prev.clone(), mlp_prox.prev_sigma.clone()))

        variants = [("mlp", mlp_prox),
                    ("mlp_noretry", trpca.ProxLearned(shape, device, mlp=mlp, retry_wide=False)),
                    ("prev", PrevRank(shape, device)),
                    ("const30", trpca.ProxLearned(shape, device, fixed_rank=30, use_prev=False)),
                    ("const54", trpca.ProxLearned(shape, device, fixed_rank=54, use_prev=False))]
        for name, params in (extra or {}).items():
            variants.append((name, trpca.ProxLearned(shape, device, mlp=params)))
        if si < full_runs:
            variants.append(("full", trpca.ProxFull(shape, device)))
        for name, prox in variants:
            res = trpca.trpca(X, prox, capture=cap if name == "mlp" else None, time_prox=True)
            row[name] = dict(prox_ms=round(res["prox_ms"], 1), iters=res["iters"],
                             fallback_slices=getattr(prox, "fallbacks", None),
                             L_err=float((res["L"] - L0).norm() / L0.norm()))
            log(f"  seed {seed} r {r} {name}: {row[name]}", file=sys.stderr, flush=True)
        errs = []
        for k, Y, tau, pr, ps in caps:
            Xl = tp.tp_prox_tnn_learned(Y, tau, mlp=mlp, prev_rank=pr, prev_sigma=ps)
            Xf = tp.tp_prox_tnn(Y, tau)
            errs.append((k, float((Xl - Xf).norm() / max(float(Xf.norm()), 1e-30))))
        row["sampled_call_rel_err"] = errs
        out["runs"].append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--under", type=float, default=32.0, help="weight of under-prediction in the loss")
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--eval-seeds", default="10000,10001")
    ap.add_argument("--full-runs", type=int, default=1)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--shapes", default="1024x1024x64,512x512x32,256x256x32")
    ap.add_argument("--runs", type=int, default=12, help="ADMM runs per shape")
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0, help="first ADMM seed (the evaluation uses 10000 and up)")
    ap.add_argument("--native", action="store_true",
                    help="collect from native TRPCA runs at the first shape on device-drawn problems")
    ap.add_argument("--labeller", default=None, help="weights of the network that drives the labelling prox")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    if args.cmd == "evaluate":
        seeds = [int(v) for v in args.eval_seeds.split(",")]
        print(json.dumps(gain(load(args.weights, dev), seeds, dev, full_runs=args.full_runs)), flush=True)
        return
    t0 = time.perf_counter()
    shapes = [tuple(int(v) for v in sh.split("x")) for sh in args.shapes.split(",")]
    if args.native:
        lab = load(args.labeller, dev) if args.labeller else None
        F, T = collect_native(shapes[0], args.runs, args.seed, dev, labeller=lab,
                              max_iter=min(args.max_iter, 100))
        val = torch.zeros(F.shape[0], dtype=torch.bool, device=F.device)
    else:
        F, T = collect(shapes, args.runs, args.seed, dev, max_iter=args.max_iter)
        val = np.zeros(F.shape[0], dtype=bool)
    t1 = time.perf_counter()
    # hold out 10% of the samples (every tenth)
    val[::10] = True
    params, hist = train(F[~val], T[~val], dev, steps=args.steps, seed=args.seed, under=args.under)
    ev = evaluate(params, F[val], T[val], dev)
    meta = dict(samples=int(F.shape[0]), shapes=args.shapes if not args.native else args.shapes.split(",")[0],
                runs_per_shape=args.runs, seed0=args.seed, native=bool(args.native),
                labeller=os.path.basename(args.labeller) if args.labeller else None,
                under=args.under, steps=args.steps,
                collect_s=round(t1 - t0, 1), train_s=round(time.perf_counter() - t1, 1), loss=hist,
                heldout=ev)
    save(params.cpu().numpy(), args.out, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
