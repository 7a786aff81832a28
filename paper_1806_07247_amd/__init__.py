"""MI355X (gfx950) t-product library: Python binding of libtp.so.

The functions here have the names of the C entry points in include/tp.h and
only marshal arguments: tensors are torch CUDA (HIP) float32 tensors, the
outputs and the workspace are allocated with torch on the tensors' device,
and the kernels are enqueued on torch's current stream.  Every step of the
computation runs in the library's HIP kernels.
"""
import ctypes

import torch

from . import _lib
from ._lib import TPError

TP_PREC_FP32 = 0
TP_PREC_BF16X3 = 1
TP_PREC_BF16 = 2
TP_MLP_INPUTS = 12
TP_SIGMA_KEEP = 64
_PREC = {"fp32": TP_PREC_FP32, "bf16x3": TP_PREC_BF16X3, "bf16": TP_PREC_BF16}

__all__ = ["tp_tprod", "tp_tprod_workspace_size", "tp_tsvd", "tp_tsvd_workspace_size", "tp_prox_tnn", "tp_prox_tnn_workspace_size",
           "tp_tnn", "tp_tnn_workspace_size", "tp_prox_tnn_learned", "tp_prox_tnn_learned_workspace_size",
           "tp_slice_features", "tp_mlp_param_count", "tp_mlp_forward", "tp_mlp_loss_grad", "tp_mlp_adam",
           "tp_trace_enable", "tp_trace_collect_work", "tp_kernel_name", "TPBatch", "tp_batch_tprod",
           "tp_tprod_nd", "tp_tprod_nd_workspace_size", "tp_prox_tnn_nd", "tp_prox_tnn_nd_workspace_size",
           "tp_tnn_nd", "tp_tnn_nd_workspace_size", "tp_half_slices_nd", "tp_trpca_taus",
           "tp_tsn", "tp_tubalrank", "tp_tran", "tp_teye",
           "tp_batch_prox",
           "half_slices", "TPError", "TP_PREC_FP32",
           "TP_PREC_BF16X3", "TP_PREC_BF16", "library_path"]


def library_path():
    return _lib.LIB_PATH


def _prec(p):
    return _PREC[p] if isinstance(p, str) else int(p)


def _dev_tensor(x, name, ndim=3):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU device")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if x.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return x.contiguous()


def _stream(dev):
    return ctypes_void(torch.cuda.current_stream(dev).cuda_stream)


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(int(v))


def _workspace(nbytes, dev):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)


def tp_tprod_workspace_size(n1, n2, l, n3, prec="fp32"):
    return int(_lib.load().tp_tprod_workspace_size(n1, n2, l, n3, _prec(prec)))


def tp_tprod(A, B, prec="fp32", out=None, workspace=None):
    """C = A * B (Definition 2.1) through Algorithm 1 on the GPU."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    B = _dev_tensor(B, "B")
    n1, n2, n3 = A.shape
    if B.shape[0] != n2 or B.shape[2] != n3:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    l = B.shape[1]
    C = out if out is not None else torch.empty((n1, l, n3), dtype=torch.float32, device=A.device)
    ws_bytes = lib.tp_tprod_workspace_size(n1, n2, l, n3, _prec(prec))
    ws = workspace if workspace is not None else _workspace(ws_bytes, A.device)
    st = lib.tp_tprod(A.data_ptr(), B.data_ptr(), C.data_ptr(), n1, n2, l, n3, _prec(prec),
                      ws.data_ptr(), ws.numel(), _stream(A.device))
    _lib.check("tp_tprod", st)
    return C


def half_slices(n3):
    """ceil((n3+1)/2) = floor(n3/2)+1: Fourier slices that get a dense operation."""
    return n3 // 2 + 1


def _ptr(t):
    return None if t is None else t.data_ptr()


def tp_prox_tnn_workspace_size(n1, n2, n3):
    return int(_lib.load().tp_prox_tnn_workspace_size(n1, n2, n3))


def tp_prox_tnn(Y, tau, out=None, info=None, rank=None, workspace=None):
    """X = Prox_tau(Y) (eq (19)) by Algorithm 3 on the GPU.

    info / rank: optional int32 device tensors of half_slices(n3) entries."""
    lib = _lib.load()
    Y = _dev_tensor(Y, "Y")
    n1, n2, n3 = Y.shape
    X = out if out is not None else torch.empty_like(Y)
    ws_bytes = lib.tp_prox_tnn_workspace_size(n1, n2, n3)
    ws = workspace if workspace is not None else _workspace(ws_bytes, Y.device)
    st = lib.tp_prox_tnn(Y.data_ptr(), X.data_ptr(), n1, n2, n3, float(tau), _ptr(info), _ptr(rank),
                         ws.data_ptr(), ws.numel(), _stream(Y.device))
    _lib.check("tp_prox_tnn", st)
    return X


def tp_tnn_workspace_size(n1, n2, n3):
    return int(_lib.load().tp_tnn_workspace_size(n1, n2, n3))


def tp_tnn(A, out=None, info=None, workspace=None):
    """Tensor nuclear norm (Definition 2.9); returns a 0-d float64 device tensor."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    res = out if out is not None else torch.empty((), dtype=torch.float64, device=A.device)
    ws_bytes = lib.tp_tnn_workspace_size(n1, n2, n3)
    ws = workspace if workspace is not None else _workspace(ws_bytes, A.device)
    st = lib.tp_tnn(A.data_ptr(), n1, n2, n3, res.data_ptr(), _ptr(info), ws.data_ptr(), ws.numel(),
                    _stream(A.device))
    _lib.check("tp_tnn", st)
    return res


# ------------------------------------------------------------ order-p --
def _dims(shape):
    """Host int array of modes 3..p for the *_nd calls."""
    d = (ctypes.c_int * len(shape))(*[int(v) for v in shape])
    return len(shape), d


def _nd_tensor(x, name):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU device")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if x.dim() < 3:
        raise ValueError(f"{name} must have at least 3 dimensions")
    return x.contiguous()


def tp_half_slices_nd(dims):
    """Fourier slices kept for modes 3..p of sizes dims: n3 ... n_(p-1) * (floor(np/2)+1)."""
    r = 1
    for v in dims[:-1]:
        r *= int(v)
    return r * (int(dims[-1]) // 2 + 1)


def tp_tprod_nd_workspace_size(n1, n2, l, dims):
    nd, d = _dims(dims)
    return int(_lib.load().tp_tprod_nd_workspace_size(n1, n2, l, nd, d))


def tp_tprod_nd(A, B, out=None, workspace=None):
    """C = A * B for order-p tensors (A n1 x n2 x dims, B n2 x l x dims)."""
    lib = _lib.load()
    A = _nd_tensor(A, "A")
    B = _nd_tensor(B, "B")
    if B.dim() != A.dim() or B.shape[0] != A.shape[1] or B.shape[2:] != A.shape[2:]:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    n1, n2 = A.shape[:2]
    l = B.shape[1]
    nd, d = _dims(A.shape[2:])
    C = out if out is not None else torch.empty((n1, l) + tuple(A.shape[2:]), dtype=torch.float32, device=A.device)
    ws_bytes = lib.tp_tprod_nd_workspace_size(n1, n2, l, nd, d)
    ws = workspace if workspace is not None else _workspace(ws_bytes, A.device)
    st = lib.tp_tprod_nd(A.data_ptr(), B.data_ptr(), C.data_ptr(), n1, n2, l, nd, d, ws.data_ptr(), ws.numel(),
                         _stream(A.device))
    _lib.check("tp_tprod_nd", st)
    return C


def tp_prox_tnn_nd(Y, tau, out=None, info=None, rank=None, workspace=None):
    """X = Prox_tau(Y) for an order-p tensor (SVT of every Fourier slice).

    info / rank: optional int32 device tensors of tp_half_slices_nd(Y.shape[2:]) entries."""
    lib = _lib.load()
    Y = _nd_tensor(Y, "Y")
    n1, n2 = Y.shape[:2]
    nd, d = _dims(Y.shape[2:])
    X = out if out is not None else torch.empty_like(Y)
    ws_bytes = lib.tp_prox_tnn_nd_workspace_size(n1, n2, nd, d)
    ws = workspace if workspace is not None else _workspace(ws_bytes, Y.device)
    st = lib.tp_prox_tnn_nd(Y.data_ptr(), X.data_ptr(), n1, n2, nd, d, float(tau), _ptr(info), _ptr(rank),
                            ws.data_ptr(), ws.numel(), _stream(Y.device))
    _lib.check("tp_prox_tnn_nd", st)
    return X


def tp_tnn_nd(A, out=None, info=None, workspace=None):
    """Nuclear norm of an order-p tensor; returns a 0-d float64 device tensor."""
    lib = _lib.load()
    A = _nd_tensor(A, "A")
    n1, n2 = A.shape[:2]
    nd, d = _dims(A.shape[2:])
    res = out if out is not None else torch.empty((), dtype=torch.float64, device=A.device)
    ws_bytes = lib.tp_tnn_nd_workspace_size(n1, n2, nd, d)
    ws = workspace if workspace is not None else _workspace(ws_bytes, A.device)
    st = lib.tp_tnn_nd(A.data_ptr(), n1, n2, nd, d, res.data_ptr(), _ptr(info), ws.data_ptr(), ws.numel(),
                       _stream(A.device))
    _lib.check("tp_tnn_nd", st)
    return res


def tp_tsvd_workspace_size(n1, n2, n3):
    return int(_lib.load().tp_tsvd_workspace_size(n1, n2, n3))


def tp_tsvd(A, info=None, workspace=None):
    """t-SVD A = U * S * V^* (Theorem 2.2) by Algorithm 2; returns (U, S, V)."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    U = torch.empty((n1, n1, n3), dtype=torch.float32, device=A.device)
    S = torch.empty((n1, n2, n3), dtype=torch.float32, device=A.device)
    V = torch.empty((n2, n2, n3), dtype=torch.float32, device=A.device)
    ws_bytes = lib.tp_tsvd_workspace_size(n1, n2, n3)
    ws = workspace if workspace is not None else _workspace(ws_bytes, A.device)
    st = lib.tp_tsvd(A.data_ptr(), U.data_ptr(), S.data_ptr(), V.data_ptr(), n1, n2, n3, _ptr(info),
                     ws.data_ptr(), ws.numel(), _stream(A.device))
    _lib.check("tp_tsvd", st)
    return U, S, V


def tp_prox_tnn_learned_workspace_size(n1, n2, n3, max_rank=64):
    return int(_lib.load().tp_prox_tnn_learned_workspace_size(n1, n2, n3, max_rank))


def tp_prox_tnn_learned(Y, tau, mlp=None, fixed_rank=0, prev_rank=None, prev_sigma=None, oversample=10,
                        power_iters=2, max_rank=64, seed=0, accuracy=2e-5, max_power_iters=8, retry_wide=True,
                        accuracy_ref=0, warm_basis=None, warm_cols=None, basis_out=None, basis_cols_out=None,
                        out=None, rank=None, fallback=None, info=None, sigma_out=None, workspace=None):
    """Learned-rank prox (see include/tp.h); mlp is a float32 device tensor of
    tp_mlp_param_count() parameters or None (then every slice uses fixed_rank).
    rank / fallback / info: optional int32 device tensors of half_slices(n3).
    basis_out (float32, basis_shape(n2, n3, max_rank)) and basis_cols_out
    (int32, half_slices(n3)) receive the range basis that warm_basis /
    warm_cols of the next call take."""
    lib = _lib.load()
    Y = _dev_tensor(Y, "Y")
    n1, n2, n3 = Y.shape
    X = out if out is not None else torch.empty_like(Y)
    for t, shape in ((warm_basis, basis_shape(n2, n3, max_rank)), (basis_out, basis_shape(n2, n3, max_rank))):
        if t is not None and (tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous()):
            raise ValueError(f"basis tensors must be contiguous float32 of shape {shape}")
    for t in (warm_cols, basis_cols_out):
        if t is not None and (t.numel() != half_slices(n3) or t.dtype != torch.int32):
            raise ValueError("basis column counts must be int32 of half_slices(n3)")
    opts = _lib.LearnedOpts(_ptr(mlp), int(fixed_rank), _ptr(prev_rank), _ptr(prev_sigma), int(oversample),
                            int(power_iters),
                            int(max_rank), int(seed) & 0xFFFFFFFFFFFFFFFF, float(accuracy), int(max_power_iters),
                            int(bool(retry_wide)), int(accuracy_ref), _ptr(warm_basis), _ptr(warm_cols),
                            _ptr(basis_out), _ptr(basis_cols_out))
    ws_bytes = lib.tp_prox_tnn_learned_workspace_size(n1, n2, n3, int(max_rank))
    ws = workspace if workspace is not None else _workspace(ws_bytes, Y.device)
    st = lib.tp_prox_tnn_learned(Y.data_ptr(), X.data_ptr(), n1, n2, n3, float(tau), ctypes.byref(opts),
                                 _ptr(rank), _ptr(fallback), _ptr(info), _ptr(sigma_out), ws.data_ptr(),
                                 ws.numel(), _stream(Y.device))
    _lib.check("tp_prox_tnn_learned", st)
    return X


def tp_tinv(A, out=None, info=None, workspace=None):
    """Tensor inverse (Definition 2.4) of a square n x n x n3 tensor; info:
    optional int32 device tensor of half_slices(n3) (0, or j+1 for a singular
    slice)."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n, n2, n3 = A.shape
    if n != n2:
        raise ValueError("tp_tinv needs an n x n x n3 tensor")
    B = out if out is not None else torch.empty_like(A)
    ws = workspace if workspace is not None else _workspace(lib.tp_tinv_workspace_size(n, n3), A.device)
    st = lib.tp_tinv(A.data_ptr(), B.data_ptr(), n, n3, _ptr(info), ws.data_ptr(), ws.numel(), _stream(A.device))
    _lib.check("tp_tinv", st)
    return B


def tp_tqr(A, workspace=None):
    """T-QR (Theorem 2.4): returns (Q, R) with A = Q * R."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    Q = torch.empty((n1, n1, n3), dtype=torch.float32, device=A.device)
    R = torch.empty_like(A)
    ws = workspace if workspace is not None else _workspace(lib.tp_tqr_workspace_size(n1, n2, n3), A.device)
    st = lib.tp_tqr(A.data_ptr(), Q.data_ptr(), R.data_ptr(), n1, n2, n3, ws.data_ptr(), ws.numel(),
                    _stream(A.device))
    _lib.check("tp_tqr", st)
    return Q, R


def tp_trpca_workspace_size_for(shape, learned=None, **kw):
    """Workspace bytes of tp_trpca for an X of this shape and these settings."""
    n1, n2, n3 = (int(v) for v in shape)
    lo = None
    if learned is not None:
        lo = _lib.LearnedOpts(None, 0, None, None, 10, 2, int(learned.get("max_rank", 64)), 0, 0.0, 8, 1, 0,
                              None, None, None, None)
    opts = _lib.TrpcaOpts(0.0, float(kw.get("mu", 1e-3)), float(kw.get("rho", 1.1)), float(kw.get("mu_max", 1e10)),
                          float(kw.get("tol", 1e-5)), int(kw.get("max_iter", 500)),
                          ctypes.pointer(lo) if lo is not None else None)
    return int(_lib.load().tp_trpca_workspace_size(n1, n2, n3, ctypes.byref(opts)))


def tp_trpca_taus(count, mu=1e-3, rho=1.1, mu_max=1e10):
    """tau of the first `count` prox calls of tp_trpca (tau_i = 1/mu_i, the
    penalty updated in double precision from the float32 settings)."""
    f = ctypes.c_float
    m, r, mx = float(f(mu).value), float(f(rho).value), float(f(mu_max).value)
    out = []
    for _ in range(count):
        out.append(float(f(1.0 / m).value))
        m = min(r * m, mx)
    return out


def tp_trpca(X, lam=None, mu=1e-3, rho=1.1, mu_max=1e10, tol=1e-5, max_iter=500, learned=None, L=None, S=None,
             Lam=None, workspace=None, record=None):
    """Tensor robust PCA (include/tp.h): min ||L||_* + lam ||S||_1 s.t. L + S = X
    by the inexact ALM, natively.  learned: None for the full-SVD prox, else a
    dict of tp_prox_tnn_learned settings (mlp, fixed_rank, oversample,
    power_iters, max_rank, seed, accuracy, max_power_iters, retry_wide,
    accuracy_ref).  record: None or a dict with max_calls and any of the
    device tensors inputs, features, counts, sigmas, bases, basis_cols
    (tp_trpca_record).  Returns dict(L, S, Lam (if given), iters, converged)."""
    lib = _lib.load()
    X = _dev_tensor(X, "X")
    n1, n2, n3 = X.shape
    for t, name in ((L, "L"), (S, "S"), (Lam, "Lam")):
        if t is not None and (tuple(t.shape) != tuple(X.shape) or t.dtype != torch.float32 or not t.is_contiguous()
                              or not t.is_cuda):
            raise ValueError(f"{name} must be a contiguous float32 device tensor shaped like X")
    Lo = L if L is not None else torch.empty_like(X)
    So = S if S is not None else torch.empty_like(X)
    lo = None
    if learned is not None:
        d = dict(mlp=None, fixed_rank=0, oversample=10, power_iters=2, max_rank=64, seed=0, accuracy=2e-5,
                 max_power_iters=8, retry_wide=True, accuracy_ref=0)
        d.update(learned)
        lo = _lib.LearnedOpts(_ptr(d["mlp"]), int(d["fixed_rank"]), None, None, int(d["oversample"]),
                              int(d["power_iters"]), int(d["max_rank"]), int(d["seed"]) & 0xFFFFFFFFFFFFFFFF,
                              float(d["accuracy"]), int(d["max_power_iters"]), int(bool(d["retry_wide"])),
                              int(d["accuracy_ref"]), None, None, None, None)
    rec = None
    if record is not None:
        rec = _lib.TrpcaRecord(int(record["max_calls"]), *[_ptr(record.get(k)) for k in
                                                           ("inputs", "features", "counts", "sigmas", "bases",
                                                            "basis_cols")])
    opts = _lib.TrpcaOpts(float(lam) if lam is not None else 0.0, float(mu), float(rho), float(mu_max), float(tol),
                          int(max_iter), ctypes.pointer(lo) if lo is not None else None,
                          ctypes.pointer(rec) if rec is not None else None)
    ws_bytes = lib.tp_trpca_workspace_size(n1, n2, n3, ctypes.byref(opts))
    if ws_bytes == 0:
        raise ValueError("bad TRPCA settings")
    ws = workspace if workspace is not None else _workspace(ws_bytes, X.device)
    it, conv = ctypes.c_int(0), ctypes.c_int(0)
    st = lib.tp_trpca(X.data_ptr(), Lo.data_ptr(), So.data_ptr(), n1, n2, n3, ctypes.byref(opts), _ptr(Lam),
                      ctypes.byref(it), ctypes.byref(conv), ws.data_ptr(), ws.numel(), _stream(X.device))
    _lib.check("tp_trpca", st)
    return dict(L=Lo, S=So, Lam=Lam, iters=it.value, converged=bool(conv.value))


def basis_shape(n2, n3, max_rank=64):
    """Shape of a warm-start basis buffer: (2, half_slices(n3), n2, max_rank)."""
    return (2, half_slices(n3), int(n2), int(max_rank))


def tp_slice_features(Y, tau, prev_rank=None, prev_sigma=None, workspace=None):
    """Per-slice features of the rank predictor: (half_slices(n3), TP_MLP_INPUTS) float32 device tensor."""
    lib = _lib.load()
    Y = _dev_tensor(Y, "Y")
    n1, n2, n3 = Y.shape
    f = torch.empty((half_slices(n3), TP_MLP_INPUTS), dtype=torch.float32, device=Y.device)
    ws_bytes = lib.tp_slice_features_workspace_size(n1, n2, n3)
    ws = workspace if workspace is not None else _workspace(ws_bytes, Y.device)
    st = lib.tp_slice_features(Y.data_ptr(), n1, n2, n3, float(tau), _ptr(prev_rank), _ptr(prev_sigma),
                               f.data_ptr(), ws.data_ptr(), ws.numel(), _stream(Y.device))
    _lib.check("tp_slice_features", st)
    return f


def tp_mlp_param_count():
    return int(_lib.load().tp_mlp_param_count())


def tp_mlp_forward(params, x):
    lib = _lib.load()
    x = x.contiguous()
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _lib.check("tp_mlp_forward", lib.tp_mlp_forward(params.data_ptr(), x.data_ptr(), y.data_ptr(), x.shape[0],
                                                    _stream(x.device)))
    return y


def tp_mlp_loss_grad(params, x, t, under=4.0, grad=None, loss=None, workspace=None):
    """Returns (grad, loss) device tensors of the asymmetric squared loss."""
    lib = _lib.load()
    x, t = x.contiguous(), t.contiguous()
    b = x.shape[0]
    g = grad if grad is not None else torch.empty_like(params)
    l = loss if loss is not None else torch.empty((), dtype=torch.float32, device=x.device)
    ws = workspace if workspace is not None else _workspace(lib.tp_mlp_train_workspace_size(b), x.device)
    _lib.check("tp_mlp_loss_grad", lib.tp_mlp_loss_grad(params.data_ptr(), x.data_ptr(), t.data_ptr(), b,
                                                        float(under), g.data_ptr(), l.data_ptr(), ws.data_ptr(),
                                                        ws.numel(), _stream(x.device)))
    return g, l


def tp_mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    lib = _lib.load()
    _lib.check("tp_mlp_adam", lib.tp_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                              int(step), float(lr), float(beta1), float(beta2), float(eps),
                                              _stream(params.device)))


def tp_trace_enable(enable=True):
    _lib.check("tp_trace_enable", _lib.load().tp_trace_enable(int(bool(enable))))


def tp_kernel_name(kid):
    return _lib.load().tp_kernel_name(int(kid)).decode()


def tp_trace_collect_work(capacity=1 << 16):
    """Launches recorded since the last collect: list of (kernel name, ms,
    algorithmic flops, algorithmic bytes), in launch order."""
    lib = _lib.load()
    ids = (ctypes.c_int * capacity)()
    ms = (ctypes.c_float * capacity)()
    fl = (ctypes.c_double * capacity)()
    by = (ctypes.c_double * capacity)()
    n = lib.tp_trace_collect_work(ids, ms, fl, by, capacity)
    _lib.check("tp_trace_collect_work", n if n < 0 else 0)
    return [(tp_kernel_name(ids[i]), float(ms[i]), float(fl[i]), float(by[i])) for i in range(min(n, capacity))]


TP_BATCH_TPROD = 0
TP_BATCH_PROX = 1
TP_BATCH_TAU_REL = 1


class TPBatch:
    """A bound batch plan (tp_batch_create + tp_batch_bind): run() enqueues
    the whole batch on the current stream (capturable in a HIP graph).

    op "tprod": outputs C_i = A_i * B_i.  op "prox": outputs the prox of
    tau_i ||.||_* at A_i, with tau_i = taus[i], or taus[i] * tsn(A_i) when
    tau_rel.  The tensors (inputs and outputs) and the workspace are kept
    alive by the plan."""

    def __init__(self, op, As, Bs=None, taus=None, tau_rel=False, outs=None, ranks=False, tile=0, grid_fft=0,
                 grid_gemm=0, grid_jacobi=0, max_sweeps=0, tuned=True):
        lib = _lib.load()
        if tuned and not (tile or grid_fft or grid_gemm or grid_jacobi):
            from . import autotune
            o = autotune.batch_opts(op, autotune.batch_shapes_of(As, Bs if op == "tprod" else None))
            tile, grid_fft = o.get("tile", 0), o.get("grid_fft", 0)
            grid_gemm, grid_jacobi = o.get("grid_gemm", 0), o.get("grid_jacobi", 0)
        self._lib = lib
        self.op = {"tprod": TP_BATCH_TPROD, "prox": TP_BATCH_PROX}[op]
        self.As = [_dev_tensor(a, "A") for a in As]
        dev = self.As[0].device
        n = len(self.As)
        if self.op == TP_BATCH_TPROD:
            if Bs is None or len(Bs) != n:
                raise ValueError("tprod needs one B per A")
            self.Bs = [_dev_tensor(b, "B") for b in Bs]
            shapes = [(a.shape[0], a.shape[1], b.shape[1], a.shape[2]) for a, b in zip(self.As, self.Bs)]
            for a, b in zip(self.As, self.Bs):
                if b.shape[0] != a.shape[1] or b.shape[2] != a.shape[2]:
                    raise ValueError("B must be n2 x l x n3")
            self.outs = outs or [torch.empty((s[0], s[2], s[3]), dtype=torch.float32, device=dev) for s in shapes]
        else:
            self.Bs = [None] * n
            if taus is None or len(taus) != n:
                raise ValueError("prox needs one tau per tensor")
            shapes = [(a.shape[0], a.shape[1], 0, a.shape[2]) for a in self.As]
            self.outs = outs or [torch.empty_like(a) for a in self.As]
        self.ranks = ([torch.zeros(half_slices(s[3]), dtype=torch.int32, device=dev) for s in shapes]
                      if (ranks and self.op == TP_BATCH_PROX) else [None] * n)
        self.tau_used = (torch.zeros(n, dtype=torch.float32, device=dev) if self.op == TP_BATCH_PROX else None)
        items = (_lib.BatchItem * n)()
        for i, (sh, a, b, c) in enumerate(zip(shapes, self.As, self.Bs, self.outs)):
            it = items[i]
            it.n1, it.n2, it.l, it.n3 = int(sh[0]), int(sh[1]), int(sh[2]), int(sh[3])
            it.A = a.data_ptr()
            it.B = b.data_ptr() if b is not None else None
            it.C = c.data_ptr()
            it.tau = float(taus[i]) if taus is not None else 0.0
            it.rank = self.ranks[i].data_ptr() if self.ranks[i] is not None else None
            it.tau_used = (self.tau_used.data_ptr() + 4 * i) if self.tau_used is not None else None
        opts = _lib.BatchOpts(int(tile), int(grid_fft), int(grid_gemm), int(grid_jacobi), int(max_sweeps))
        plan = ctypes.c_void_p()
        flags = TP_BATCH_TAU_REL if tau_rel else 0
        _lib.check("tp_batch_create", lib.tp_batch_create(ctypes.byref(plan), self.op, items, n, flags,
                                                           ctypes.byref(opts)))
        self._plan = plan
        self.workspace = _workspace(lib.tp_batch_workspace_size(plan), dev)
        _lib.check("tp_batch_bind", lib.tp_batch_bind(plan, _ptr(self.workspace), self.workspace.numel(),
                                                       _stream(dev)))

    def run(self):
        _lib.check("tp_batch_run", self._lib.tp_batch_run(self._plan, _stream(self.As[0].device)))
        return self.outs

    def stats(self):
        st = _lib.BatchStats()
        _lib.check("tp_batch_stats", self._lib.tp_batch_stats(self._plan, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _lib.BatchStats._fields_}

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            self._lib.tp_batch_destroy(plan)
            self._plan = None


def tp_batch_tprod(As, Bs, **kw):
    """C_i = A_i * B_i for every pair, as one batch."""
    b = TPBatch("tprod", As, Bs, **kw)
    return b.run()


def tp_batch_prox(As, taus, tau_rel=False, **kw):
    """prox of tau_i ||.||_* at every A_i, as one batch."""
    b = TPBatch("prox", As, taus=taus, tau_rel=tau_rel, **kw)
    return b.run()


def tp_tsn(A, info=None, workspace=None):
    """Tensor spectral norm (Definition 2.8) as a float64 device scalar tensor."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    out = torch.empty((), dtype=torch.float64, device=A.device)
    ws = workspace if workspace is not None else _workspace(lib.tp_tsn_workspace_size(n1, n2, n3), A.device)
    _lib.check("tp_tsn", lib.tp_tsn(A.data_ptr(), n1, n2, n3, out.data_ptr(), _ptr(info), ws.data_ptr(),
                                    ws.numel(), _stream(A.device)))
    return out


def tp_tubalrank(A, tol=-1.0, info=None, workspace=None):
    """Tensor tubal rank (Definition 2.7) as an int32 device scalar tensor
    (tol < 0: max(n1, n2) 2^-23 S(1,1,1))."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    out = torch.empty((), dtype=torch.int32, device=A.device)
    ws = workspace if workspace is not None else _workspace(lib.tp_tubalrank_workspace_size(n1, n2, n3), A.device)
    _lib.check("tp_tubalrank", lib.tp_tubalrank(A.data_ptr(), n1, n2, n3, float(tol), out.data_ptr(), _ptr(info),
                                                ws.data_ptr(), ws.numel(), _stream(A.device)))
    return out


def tp_tran(A, out=None):
    """Conjugate transpose (Definition 2.2) of a real tensor: n2 x n1 x n3."""
    lib = _lib.load()
    A = _dev_tensor(A, "A")
    n1, n2, n3 = A.shape
    out = out if out is not None else torch.empty((n2, n1, n3), dtype=torch.float32, device=A.device)
    _lib.check("tp_tran", lib.tp_tran(A.data_ptr(), out.data_ptr(), n1, n2, n3, _stream(A.device)))
    return out


def tp_teye(n, n3, device="cuda:0"):
    """Identity tensor (Definition 2.3), n x n x n3."""
    lib = _lib.load()
    out = torch.empty((n, n, n3), dtype=torch.float32, device=device)
    _lib.check("tp_teye", lib.tp_teye(out.data_ptr(), int(n), int(n3), _stream(out.device)))
    return out
