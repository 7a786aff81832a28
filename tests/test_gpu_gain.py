"""What the trained rank network gains over the method without it.

On a held-out problem of the learned-rank workload at the size the network
was trained for (1024 x 1024 x 64; the seed is not among the training
seeds), a TRPCA-ADMM run is driven by the learned prox; every prox call's
input is kept and run through the learned prox and through the paper's
full-SVD prox (Algorithm 3) on the same GPU.  The test requires the learned
calls to be at least 3x faster in total and each within 1e-4 of the
full-SVD result, relative to the larger of that result and the input.  It
also reports the error relative to the result alone.

Against the method without the network, whole ADMM runs are timed with the
network, with the previous call's largest count and with a constant count of
30: the network must not be slower than the constant count.  Over the
previous-count setting its gain is nil on this workload (measured on the 16
held-out seeds 10000..10015 at 1024x1024x64: 1557 ms against 1554 ms of
prox time): the counts settle within a few ADMM calls, and the wide retry
makes the few under-predicted calls cheap, so the test only reports it.
"""
import json

import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1806_07247_amd as tp
    tp._lib.load()
    return tp


def _timed(fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    out = fn()
    b.record()
    torch.cuda.synchronize()
    return out, a.elapsed_time(b)


@pytest.mark.parametrize("n,n3,seed", [(1024, 64, 10002)])
def test_trained_network_gain(tp, n, n3, seed):
    from paper_1806_07247_amd import rank_model, trpca
    dev = torch.device("cuda:0")
    X, L0, r = trpca.learned_workload(seed, dev, n, n3)
    shape = (n, n, n3)
    h = n3 // 2 + 1
    mlp = rank_model.load(device=dev)
    prox = trpca.ProxLearned(shape, dev, mlp=mlp)
    calls = []

    def cap(k, Y, tau):
        wb, wc = prox.warm_inputs()
        calls.append((Y.clone(), tau, prox.calls, prox.prev.clone() if prox.have_prev else None,
                      prox.prev_sigma.clone() if prox.have_prev else None,
                      wb.clone() if wb is not None else None, wc.clone() if wc is not None else None))

    res = trpca.trpca(X, prox, capture=cap)
    assert res["converged"]
    rec = float((res["L"] - L0).norm() / L0.norm())
    say(f"gain test {n}x{n}x{n3} seed {seed} r {r}: {res['iters']} ADMM iterations, L rel.err {rec:.2e}")
    assert rec < 1e-3

    full = trpca.ProxFull(shape, dev)
    out_l = torch.empty_like(X)
    out_f = torch.empty_like(X)
    rk = torch.zeros(h, dtype=torch.int32, device=dev)
    fb = torch.zeros(h, dtype=torch.int32, device=dev)
    ws = torch.empty(tp.tp_prox_tnn_learned_workspace_size(n, n, n3, 64), dtype=torch.uint8, device=dev)
    # warm both paths once
    full(calls[-1][0], calls[-1][1], out_f)
    tp.tp_prox_tnn_learned(calls[-1][0], calls[-1][1], mlp=mlp, out=out_l, workspace=ws)
    torch.cuda.synchronize()
    t_l, t_f, errs, errs_in, fbs = 0.0, 0.0, [], [], 0
    bout = torch.empty(tp.basis_shape(n, n3), dtype=torch.float32, device=dev)
    bcols = torch.zeros(h, dtype=torch.int32, device=dev)
    for Y, tau, sd, pr, ps, wb, wc in calls:
        _, ms_f = _timed(lambda: full(Y, tau, out_f))
        _, ms_l = _timed(lambda: tp.tp_prox_tnn_learned(Y, tau, mlp=mlp, prev_rank=pr, prev_sigma=ps, seed=sd,
                                                         warm_basis=wb, warm_cols=wc, basis_out=bout,
                                                         basis_cols_out=bcols, out=out_l, rank=rk, fallback=fb,
                                                         workspace=ws))
        t_f += ms_f
        t_l += ms_l
        fbs += int(fb.sum())
        d = float((out_l - out_f).norm())
        ref = float(out_f.norm())
        errs.append(0.0 if d == 0.0 else d / ref if ref > 0 else float("inf"))
        errs_in.append(0.0 if d == 0.0 else d / max(ref, float(Y.norm())))

    # the method without the network: ADMM driven by heuristic counts
    others = {}
    for name, p in (("network", trpca.ProxLearned(shape, dev, mlp=mlp)),
                    ("previous_count", rank_model.PrevRank(shape, dev)),
                    ("constant_30", trpca.ProxLearned(shape, dev, fixed_rank=30, use_prev=False))):
        rr = trpca.trpca(X, p, time_prox=True)
        others[name] = {"prox_ms": round(rr["prox_ms"], 1), "iters": rr["iters"], "fallback_slices": p.fallbacks}
    report = {"calls": len(calls), "full_svd_ms": round(t_f, 1), "learned_ms": round(t_l, 1),
              "speedup": round(t_f / t_l, 2), "max_rel_err": max(errs), "median_rel_err": float(np.median(errs)),
              "max_err_rel_to_max_of_result_and_input": max(errs_in),
              "fallback_slices": fbs, "admm_runs": others}
    say("  " + json.dumps(report))
    assert t_f / t_l >= 3.0
    assert others["network"]["prox_ms"] <= 1.05 * others["constant_30"]["prox_ms"]
    # error relative to the larger of the result and the input (the learned
    # prox checks its Ritz residuals at that scale)
    assert max(errs_in) <= 1e-4
