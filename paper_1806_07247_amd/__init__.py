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
           "tp_trace_enable", "tp_trace_collect_work", "tp_kernel_name",
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
                        accuracy_ref=0,
                        out=None, rank=None, fallback=None, info=None, sigma_out=None, workspace=None):
    """Learned-rank prox (see include/tp.h); mlp is a float32 device tensor of
    tp_mlp_param_count() parameters or None (then every slice uses fixed_rank).
    rank / fallback / info: optional int32 device tensors of half_slices(n3)."""
    lib = _lib.load()
    Y = _dev_tensor(Y, "Y")
    n1, n2, n3 = Y.shape
    X = out if out is not None else torch.empty_like(Y)
    opts = _lib.LearnedOpts(_ptr(mlp), int(fixed_rank), _ptr(prev_rank), _ptr(prev_sigma), int(oversample),
                            int(power_iters),
                            int(max_rank), int(seed) & 0xFFFFFFFFFFFFFFFF, float(accuracy), int(max_power_iters),
                            int(bool(retry_wide)), int(accuracy_ref))
    ws_bytes = lib.tp_prox_tnn_learned_workspace_size(n1, n2, n3, int(max_rank))
    ws = workspace if workspace is not None else _workspace(ws_bytes, Y.device)
    st = lib.tp_prox_tnn_learned(Y.data_ptr(), X.data_ptr(), n1, n2, n3, float(tau), ctypes.byref(opts),
                                 _ptr(rank), _ptr(fallback), _ptr(info), _ptr(sigma_out), ws.data_ptr(),
                                 ws.numel(), _stream(Y.device))
    _lib.check("tp_prox_tnn_learned", st)
    return X


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
