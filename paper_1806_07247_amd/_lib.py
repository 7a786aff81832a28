"""ctypes binding of libtp.so (argument marshalling only).

Every computation runs in the HIP kernels of libtp.so.  torch supplies device
memory (outputs and the workspace) and the current stream; nothing here
computes on the host, and there is no fallback: if libtp.so is missing or the
device is not a GPU, calls raise.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtp.so")

_VP = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
_F = ctypes.c_float

# name -> (restype, argtypes); must match include/tp.h
SIGNATURES = {
    "tp_status_string": (ctypes.c_char_p, [_I]),
    "tp_version": (_I, []),
    "tp_tprod_workspace_size": (_SZ, [_I, _I, _I, _I, _I]),
    "tp_tprod": (_I, [_VP, _VP, _VP, _I, _I, _I, _I, _I, _VP, _SZ, _VP]),
    "tp_tprod_noalloc": (_I, [_VP, _VP, _VP, _I, _I, _I, _I, _I, _VP]),
    "tp_tprod_noalloc_max_bytes": (_SZ, []),
    "tp_tsvd_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_tsvd": (_I, [_VP, _VP, _VP, _VP, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "tp_prox_tnn_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_prox_tnn": (_I, [_VP, _VP, _I, _I, _I, _F, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tnn_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_tnn": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tprod_nd_workspace_size": (_SZ, [_I, _I, _I, _I, _VP]),
    "tp_tprod_nd": (_I, [_VP, _VP, _VP, _I, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "tp_prox_tnn_nd_workspace_size": (_SZ, [_I, _I, _I, _VP]),
    "tp_prox_tnn_nd": (_I, [_VP, _VP, _I, _I, _I, _VP, _F, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tnn_nd_workspace_size": (_SZ, [_I, _I, _I, _VP]),
    "tp_tnn_nd": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tsn_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_tsn": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tubalrank_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_tubalrank": (_I, [_VP, _I, _I, _I, ctypes.c_double, _VP, _VP, _VP, _SZ, _VP]),
    "tp_tran": (_I, [_VP, _VP, _I, _I, _I, _VP]),
    "tp_teye": (_I, [_VP, _I, _I, _VP]),
    "tp_set_param": (_I, [_I, _I]),
    "tp_get_param": (_I, [_I]),
    "tp_trace_enable": (_I, [_I]),
    "tp_trace_collect": (_I, [ctypes.POINTER(_I), ctypes.POINTER(_F), _I]),
    "tp_trace_collect_work": (_I, [ctypes.POINTER(_I), ctypes.POINTER(_F), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), _I]),
    "tp_kernel_name": (ctypes.c_char_p, [_I]),
}

_U64 = ctypes.c_ulonglong


class LearnedOpts(ctypes.Structure):
    """tp_learned_opts of include/tp.h"""
    _fields_ = [("mlp", _VP), ("fixed_rank", _I), ("prev_rank", _VP), ("prev_sigma", _VP), ("oversample", _I),
                ("power_iters", _I), ("max_rank", _I), ("seed", _U64), ("accuracy", _F), ("max_power_iters", _I),
                ("retry_wide", _I), ("accuracy_ref", _I), ("warm_basis", _VP), ("warm_cols", _VP),
                ("basis_out", _VP), ("basis_cols_out", _VP)]


SIGNATURES.update({
    "tp_tinv_workspace_size": (_SZ, [_I, _I]),
    "tp_tinv": (_I, [_VP, _VP, _I, _I, _VP, _VP, _SZ, _VP]),
    "tp_tqr_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_tqr": (_I, [_VP, _VP, _VP, _I, _I, _I, _VP, _SZ, _VP]),
})


class TrpcaRecord(ctypes.Structure):
    """tp_trpca_record of include/tp.h"""
    _fields_ = [("max_calls", _I), ("inputs", _VP), ("features", _VP), ("counts", _VP), ("sigmas", _VP),
                ("bases", _VP), ("basis_cols", _VP)]


class TrpcaOpts(ctypes.Structure):
    """tp_trpca_opts of include/tp.h"""
    _fields_ = [("lam", _F), ("mu", _F), ("rho", _F), ("mu_max", _F), ("tol", _F), ("max_iter", _I),
                ("learned", ctypes.POINTER(LearnedOpts)), ("record", ctypes.POINTER(TrpcaRecord))]


SIGNATURES.update({
    "tp_trpca_workspace_size": (_SZ, [_I, _I, _I, ctypes.POINTER(TrpcaOpts)]),
    "tp_trpca": (_I, [_VP, _VP, _VP, _I, _I, _I, ctypes.POINTER(TrpcaOpts), _VP, ctypes.POINTER(_I),
                      ctypes.POINTER(_I), _VP, _SZ, _VP]),
})


SIGNATURES.update({
    "tp_prox_tnn_learned_workspace_size": (_SZ, [_I, _I, _I, _I]),
    "tp_prox_tnn_learned": (_I, [_VP, _VP, _I, _I, _I, _F, ctypes.POINTER(LearnedOpts), _VP, _VP, _VP, _VP, _VP,
                                 _SZ, _VP]),
    "tp_slice_features_workspace_size": (_SZ, [_I, _I, _I]),
    "tp_slice_features": (_I, [_VP, _I, _I, _I, _F, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "tp_mlp_param_count": (_I, []),
    "tp_mlp_forward": (_I, [_VP, _VP, _VP, _I, _VP]),
    "tp_mlp_train_workspace_size": (_SZ, [_I]),
    "tp_mlp_loss_grad": (_I, [_VP, _VP, _VP, _I, _F, _VP, _VP, _VP, _SZ, _VP]),
    "tp_mlp_adam": (_I, [_VP, _VP, _VP, _VP, _I, _F, _F, _F, _F, _VP]),
})



class BatchItem(ctypes.Structure):
    """tp_batch_item of include/tp.h"""
    _fields_ = [("n1", _I), ("n2", _I), ("l", _I), ("n3", _I), ("A", _VP), ("B", _VP), ("C", _VP), ("tau", _F),
                ("rank", _VP), ("tau_used", _VP)]


class BatchOpts(ctypes.Structure):
    """tp_batch_opts of include/tp.h"""
    _fields_ = [("tile", _I), ("grid_fft", _I), ("grid_gemm", _I), ("grid_jacobi", _I), ("max_sweeps", _I)]


class BatchStats(ctypes.Structure):
    """tp_batch_stats_t of include/tp.h"""
    _fields_ = [("fft_units", _I), ("gemm_units", _I), ("slice_units", _I), ("tile", _I), ("grid_fft", _I),
                ("grid_gemm", _I), ("grid_jacobi", _I), ("gemm_flops", ctypes.c_double),
                ("fft_bytes", ctypes.c_double)]


SIGNATURES.update({
    "tp_batch_create": (_I, [ctypes.POINTER(_VP), _I, ctypes.POINTER(BatchItem), _I, _I, ctypes.POINTER(BatchOpts)]),
    "tp_batch_workspace_size": (_SZ, [_VP]),
    "tp_batch_bind": (_I, [_VP, _VP, _SZ, _VP]),
    "tp_batch_run": (_I, [_VP, _VP]),
    "tp_batch_stats": (_I, [_VP, ctypes.POINTER(BatchStats)]),
    "tp_batch_destroy": (_I, [_VP]),
})

_lib = None


class TPError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = load().tp_status_string(status).decode()
        super().__init__(f"{fn} failed with status {status} ({msg})")


def load():
    """Load libtp.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libtp.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_1806_07247_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(fn, status):
    if status != 0:
        raise TPError(fn, status)
