"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/tp.h is exported by libtp.so, and argument errors are reported before
anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(tp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1806_07247_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtp.so not built")
    return _lib.load()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("tp_tprod",):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_1806_07247_amd", "libtp.so"))
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(lib):
    from paper_1806_07247_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def test_tprod_argument_errors(lib):
    ws = lib.tp_tprod_workspace_size(4, 3, 2, 5, 0)
    assert ws > 0
    assert lib.tp_tprod(None, FAKE, FAKE, 4, 3, 2, 5, 0, FAKE, ws, None) == -1
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 7, FAKE, ws, None) == -1
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 0, 3, 2, 5, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 0, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 2000, 0, FAKE, ws, None) == -2
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 0, FAKE, ws - 1, None) == -3
    assert lib.tp_tprod(FAKE, FAKE, FAKE, 4, 3, 2, 5, 0, None, ws, None) == -3
    assert lib.tp_status_string(-3) == b"workspace missing or too small"


def test_workspace_query(lib):
    # half spectra of A, B, C: 2 planes * (n3/2+1) slices each, 256-byte aligned
    h = 5 // 2 + 1
    need = sum(((2 * h * e * 4 + 255) // 256) * 256 for e in (4 * 3, 3 * 2, 4 * 2))
    assert lib.tp_tprod_workspace_size(4, 3, 2, 5, 0) >= need
    assert lib.tp_tprod_workspace_size(0, 3, 2, 5, 0) == 0


def test_batch_plan_validation(lib):
    """tp_batch_create validates items on the host; a valid plan is sized
    without touching the (fake) device pointers."""
    from paper_1806_07247_amd import _lib
    items = (_lib.BatchItem * 2)()
    for it, (n1, n2, l, n3) in zip(items, [(5, 7, 3, 4), (20, 9, 11, 6)]):
        it.n1, it.n2, it.l, it.n3 = n1, n2, l, n3
        it.A, it.B, it.C = 0x1000, 0x2000, 0x3000
        it.tau = 0.5
    plan = ctypes.c_void_p()
    assert lib.tp_batch_create(ctypes.byref(plan), 0, items, 2, 0, None) == 0
    ws = lib.tp_batch_workspace_size(plan)
    assert ws > 0
    st = _lib.BatchStats()
    assert lib.tp_batch_stats(plan, ctypes.byref(st)) == 0
    # units: 64 tubes per transform unit (A, B forward; C inverse), one tile per slice product
    fft = sum(-(-n1 * n2 // 64) + -(-n2 * l // 64) + -(-n1 * l // 64)
              for n1, n2, l, n3 in [(5, 7, 3, 4), (20, 9, 11, 6)])
    assert st.fft_units == fft
    assert st.gemm_units == 3 + 4  # one 32x32 tile per slice, h = 3 and 4
    assert lib.tp_batch_bind(plan, ctypes.c_void_p(0x4000), ws - 1, None) == -3
    assert lib.tp_batch_run(plan, None) == -1  # not bound
    assert lib.tp_batch_destroy(plan) == 0
    # errors: op, count, flags, shapes, prox limits, tau
    assert lib.tp_batch_create(ctypes.byref(plan), 2, items, 2, 0, None) == -1
    assert lib.tp_batch_create(ctypes.byref(plan), 0, items, 0, 0, None) == -1
    assert lib.tp_batch_create(ctypes.byref(plan), 0, items, 2, 1, None) == -1  # relative tau is prox only
    items[1].n3 = 129
    assert lib.tp_batch_create(ctypes.byref(plan), 0, items, 2, 0, None) == -2
    items[1].n3 = 6
    items[1].n1 = 129
    assert lib.tp_batch_create(ctypes.byref(plan), 1, items, 2, 0, None) == -2
    items[1].n1 = 20
    items[0].tau = -1.0
    assert lib.tp_batch_create(ctypes.byref(plan), 1, items, 2, 0, None) == -1
    items[0].tau = 0.5
    items[0].B = None
    assert lib.tp_batch_create(ctypes.byref(plan), 0, items, 2, 0, None) == -1
    assert lib.tp_batch_create(ctypes.byref(plan), 1, items, 2, 1, None) == 0  # prox needs no B
    assert lib.tp_batch_destroy(plan) == 0


def test_trpca_argument_errors(lib):
    from paper_1806_07247_amd import _lib
    ok = _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e10, 1e-5, 500, None)
    ws = lib.tp_trpca_workspace_size(6, 5, 4, ctypes.byref(ok))
    assert ws >= 3 * 6 * 5 * 4 * 4
    it, conv = ctypes.c_int(0), ctypes.c_int(0)

    def call(opts, n1=6, ws_bytes=ws, x=FAKE):
        return lib.tp_trpca(x, FAKE, FAKE, n1, 5, 4, opts, None, ctypes.byref(it), ctypes.byref(conv), FAKE,
                            ws_bytes, None)

    assert call(None) == -1
    assert call(ctypes.byref(ok), x=None) == -1
    for bad in (_lib.TrpcaOpts(0.0, 0.0, 1.1, 1e10, 1e-5, 500, None),       # mu <= 0
                _lib.TrpcaOpts(0.0, 1e-3, 0.9, 1e10, 1e-5, 500, None),      # rho < 1
                _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e-4, 1e-5, 500, None),      # mu_max < mu
                _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e10, -1.0, 500, None),      # tol < 0
                _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e10, 1e-5, 0, None)):       # max_iter < 1
        assert call(ctypes.byref(bad)) == -1
        assert lib.tp_trpca_workspace_size(6, 5, 4, ctypes.byref(bad)) == 0
    lo = _lib.LearnedOpts(None, 5, None, None, 10, 2, 65, 0, 0.0, 8, 1, 0, None, None, None, None)
    bad_l = _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e10, 1e-5, 500, ctypes.pointer(lo))  # max_rank > 64
    assert call(ctypes.byref(bad_l)) == -1
    assert call(ctypes.byref(ok), n1=0) == -2
    assert call(ctypes.byref(ok), ws_bytes=ws - 1) == -3
    lo.max_rank = 16
    good_l = _lib.TrpcaOpts(0.0, 1e-3, 1.1, 1e10, 1e-5, 500, ctypes.pointer(lo))
    assert lib.tp_trpca_workspace_size(6, 5, 4, ctypes.byref(good_l)) > ws


def test_nd_argument_errors(lib):
    """Order-p calls: shapes and the host dims array are checked before
    anything is enqueued (the fake device pointers are never touched)."""
    D = ctypes.c_int * 4
    dims = D(3, 4, 5, 6)
    ws = lib.tp_tprod_nd_workspace_size(4, 3, 2, 3, dims)
    assert ws > 0
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 0, dims, FAKE, ws, None) == -2
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 9, dims, FAKE, ws, None) == -2
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 2, None, FAKE, ws, None) == -1
    assert lib.tp_tprod_nd(None, FAKE, FAKE, 4, 3, 2, 2, dims, FAKE, ws, None) == -1
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 2, D(3, 0), FAKE, ws, None) == -2
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 2, D(3, 1025), FAKE, ws, None) == -2
    # more than 65535 kept slices: 300 * 300 * (2/2 + 1)
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 3, D(300, 300, 2), FAKE, ws, None) == -2
    assert lib.tp_tprod_nd_workspace_size(4, 3, 2, 3, D(300, 300, 2)) == 0
    assert lib.tp_tprod_nd(FAKE, FAKE, FAKE, 4, 3, 2, 3, dims, FAKE, ws - 1, None) == -3
    # the workspace holds three slice stacks and a scratch stack; nd = 3 reads
    # dims 3, 4, 5: 3 * 4 * (5/2 + 1) = 36 slices
    need = sum(2 * 36 * e * 4 for e in (4 * 3, 3 * 2, 4 * 2, 4 * 3))
    assert ws >= need
    pw = lib.tp_prox_tnn_nd_workspace_size(6, 5, 2, dims)
    assert pw > 0
    assert lib.tp_prox_tnn_nd(FAKE, FAKE, 6, 5, 2, dims, ctypes.c_float(-1.0), None, None, FAKE, pw, None) == -1
    assert lib.tp_prox_tnn_nd(FAKE, FAKE, 6, 5, 2, dims, ctypes.c_float(0.5), None, None, FAKE, pw - 1, None) == -3
    assert lib.tp_prox_tnn_nd(FAKE, FAKE, 6, 3000, 2, dims, ctypes.c_float(0.5), None, None, FAKE, pw, None) == -5
    tw = lib.tp_tnn_nd_workspace_size(6, 5, 2, dims)
    assert tw > 0
    assert lib.tp_tnn_nd(FAKE, 6, 5, 2, dims, None, None, FAKE, tw, None) == -1
    assert lib.tp_tnn_nd(FAKE, 6, 5, 2, dims, FAKE, None, FAKE, tw - 1, None) == -3
