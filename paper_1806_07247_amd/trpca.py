"""Tensor robust PCA by the inexact augmented Lagrangian method, the setting
in which the paper places the proximal operator of the TNN as the key
subproblem.  It drives the library's prox (full or learned-rank) and records
per-slice training samples for the rank predictor.

    min ||L||_* + lam ||S||_1  s.t.  L + S = X,   lam = 1/sqrt(max(n1,n2) n3)
    L <- Prox_{1/mu}(X - S - Lam/mu)          (tp_prox_tnn / tp_prox_tnn_learned)
    S <- soft(X - L - Lam/mu, lam/mu)
    Lam <- Lam + mu (L + S - X);  mu <- min(rho mu, mu_max)
stopping when the largest entry change of L, S and of L + S - X is at most
tol * max(1, max |X|) (a relative tolerance: FP32 data cannot reach the 1e-8
absolute tolerance customary in double precision).

The elementwise updates of S and Lam are torch tensor operations on the GPU
(they are the loop around the prox, not the slice pipeline).
"""
import math
import time

import torch

import paper_1806_07247_amd as tp


class ProxFull:
    """The paper's prox (Algorithm 3, full SVD per slice)."""

    name = "full"

    def __init__(self, shape, device):
        n1, n2, n3 = shape
        self.h = tp.half_slices(n3)
        self.ws = torch.empty(tp.tp_prox_tnn_workspace_size(n1, n2, n3), dtype=torch.uint8, device=device)
        self.rank = torch.zeros(self.h, dtype=torch.int32, device=device)

    def __call__(self, Y, tau, out):
        tp.tp_prox_tnn(Y, tau, out=out, rank=self.rank, workspace=self.ws)
        return out


class ProxLearned:
    """Learned-rank prox: the MLP (or a fixed count) sizes a randomized SVD;
    the previous call's per-slice count is fed back as a feature."""

    name = "learned"

    def __init__(self, shape, device, mlp=None, fixed_rank=0, oversample=10, power_iters=2, max_rank=64, seed=0,
                 use_prev=True, accuracy=2e-5, max_power_iters=8, retry_wide=True, accuracy_ref=0, warm=True):
        n1, n2, n3 = shape
        self.h = tp.half_slices(n3)
        self.mlp, self.fixed_rank = mlp, fixed_rank
        self.oversample, self.power_iters, self.max_rank, self.seed = oversample, power_iters, max_rank, seed
        self.accuracy, self.max_power_iters, self.retry_wide = accuracy, max_power_iters, retry_wide
        self.accuracy_ref = accuracy_ref
        self.ws = torch.empty(tp.tp_prox_tnn_learned_workspace_size(n1, n2, n3, max_rank), dtype=torch.uint8,
                              device=device)
        self.rank = torch.zeros(self.h, dtype=torch.int32, device=device)
        self.fallback = torch.zeros(self.h, dtype=torch.int32, device=device)
        self.prev = torch.zeros(self.h, dtype=torch.int32, device=device)
        self.sigma = torch.zeros((self.h, tp.TP_SIGMA_KEEP), dtype=torch.float32, device=device)
        self.prev_sigma = torch.zeros_like(self.sigma)
        self.have_prev = False
        self.use_prev = use_prev
        # warm start: the previous call's range basis (two buffers, swapped per call)
        self.warm = warm
        if warm:
            bs = tp.basis_shape(n2, n3, max_rank)
            self.basis = [torch.zeros(bs, dtype=torch.float32, device=device) for _ in range(2)]
            self.bcols = [torch.zeros(self.h, dtype=torch.int32, device=device) for _ in range(2)]
        self.calls = 0
        self.fallbacks = 0

    def warm_inputs(self):
        """(warm_basis, warm_cols) the next call takes (None without a previous call)."""
        if not (self.warm and self.have_prev):
            return None, None
        return self.basis[self.calls % 2 ^ 1], self.bcols[self.calls % 2 ^ 1]

    def __call__(self, Y, tau, out):
        use = self.use_prev and self.have_prev
        wb, wc = self.warm_inputs()
        tp.tp_prox_tnn_learned(Y, tau, mlp=self.mlp, fixed_rank=self.fixed_rank,
                               warm_basis=wb, warm_cols=wc,
                               basis_out=self.basis[self.calls % 2] if self.warm else None,
                               basis_cols_out=self.bcols[self.calls % 2] if self.warm else None,
                               prev_rank=self.prev if use else None, prev_sigma=self.prev_sigma if use else None,
                               oversample=self.oversample, power_iters=self.power_iters, max_rank=self.max_rank,
                               seed=self.seed + self.calls, accuracy=self.accuracy,
                               max_power_iters=self.max_power_iters, retry_wide=self.retry_wide,
                               accuracy_ref=self.accuracy_ref, out=out,
                               rank=self.rank,
                               fallback=self.fallback, sigma_out=self.sigma, workspace=self.ws)
        self.prev.copy_(self.rank)
        self.prev_sigma.copy_(self.sigma)
        self.have_prev = True
        self.calls += 1
        self.fallbacks += int(self.fallback.sum())
        return out


def trpca(X, prox, lam=None, mu=1e-3, rho=1.1, mu_max=1e10, tol=1e-5, max_iter=500, record=None, capture=None,
          time_prox=False):
    """Inexact ALM for TRPCA on the GPU tensor X.

    record(Yin, tau, rank_tensor, sigma_tensor) is called after every prox
    call (for training samples); capture(k, Yin, tau) lets a caller keep prox inputs.
    Returns dict(L, S, iters, prox_ms (if timed), converged)."""
    n1, n2, n3 = X.shape
    if lam is None:
        lam = 1.0 / math.sqrt(max(n1, n2) * n3)
    L = torch.zeros_like(X)
    S = torch.zeros_like(X)
    Lam = torch.zeros_like(X)
    Lnew = torch.empty_like(X)
    Yin = torch.empty_like(X)
    prox_ms = 0.0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    it = 0
    converged = False
    scale = max(1.0, float(X.abs().max()))
    for it in range(1, max_iter + 1):
        torch.sub(X, S, out=Yin)
        Yin.sub_(Lam, alpha=1.0 / mu)
        tau = 1.0 / mu
        if capture is not None:
            capture(it, Yin, tau)
        if time_prox:
            ev0.record()
        prox(Yin, tau, Lnew)
        if time_prox:
            ev1.record()
            torch.cuda.synchronize()
            prox_ms += ev0.elapsed_time(ev1)
        if record is not None:
            record(Yin, tau, getattr(prox, "rank", None), getattr(prox, "sigma", None))
        R = X - Lnew - Lam / mu
        Snew = torch.sign(R) * torch.clamp(R.abs() - lam / mu, min=0.0)
        resid = Lnew + Snew - X
        dL = float((Lnew - L).abs().max())
        dS = float((Snew - S).abs().max())
        dr = float(resid.abs().max())
        Lam.add_(resid, alpha=mu)
        L.copy_(Lnew)
        S = Snew
        mu = min(rho * mu, mu_max)
        if max(dL, dS, dr) <= tol * scale:
            converged = True
            break
    return dict(L=L, S=S, iters=it, prox_ms=prox_ms, converged=converged)


def make_problem(n, n3, r, sparse_frac, seed, device):
    """X = P*Q + S (low tubal rank r plus sparse +-1 outliers), the learned-rank
    workload's recipe at any size n x n x n3 (P, Q entries N(0, 1/n))."""
    from paper_1806_07247_amd import inputs
    parts = inputs.lowrank_sparse_parts(n, n, n3, r, 1.0 / n, sparse_frac, 0.0, seed)
    P = torch.from_numpy(parts["P"]).to(device)
    Q = torch.from_numpy(parts["Q"]).to(device)
    L0 = tp.tp_tprod(P, Q)
    S0 = torch.from_numpy(parts["S"]).to(device)
    return (L0 + S0).contiguous(), L0, S0


def learned_workload(seed, device, n=1024, n3=64):
    """The learned-rank workload: X = P*Q + S, n x n x n3, tubal rank
    r ~ U{5..40} drawn from the seed's own stream, P, Q entries N(0, 1/n),
    5% +-1 outliers.  Returns (X, L0, r)."""
    from paper_1806_07247_amd import inputs
    parts = inputs.learned_rank_parts(seed, n, n3)
    P = torch.from_numpy(parts["P"]).to(device)
    Q = torch.from_numpy(parts["Q"]).to(device)
    L0 = tp.tp_tprod(P, Q)
    X = (L0 + torch.from_numpy(parts["S"]).to(device)).contiguous()
    return X, L0, parts["r"]


def timed_run(X, prox, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = trpca(X, prox, **kw)
    torch.cuda.synchronize()
    res["wall_s"] = time.perf_counter() - t0
    return res
