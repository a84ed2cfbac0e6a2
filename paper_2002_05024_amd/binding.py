"""ctypes binding of ``libneig.so`` (the C ABI in ``include/neig.h``).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Matrices are torch float64 CUDA (HIP) tensors in column-major layout
(``stride(0) == 1``, leading dimension ``stride(1)``); the calls run on
``torch.cuda.current_stream()`` unless a stream is given.  There is no CPU
fallback: if the library is missing or the tensors are not on the GPU, the
call raises :class:`NeigError`.
"""
from __future__ import annotations

import ctypes
import os
from collections import namedtuple

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libneig.so")
_lib = None

_i = ctypes.c_int
_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)


class NeigError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [
        ("ns", _i),
        ("nw", _i),
        ("nmin", _i),
        ("chain", _i),
        ("chase_w", _i),
        ("deflation", _i),
        ("maxit", _i),
        ("nibble", _i),
        ("exc", _i),
        ("timing", _i),
        ("policy", _i),
        ("seed", _i),
        ("rec_nw", _i),
        ("rec_ns", _i),
        ("aed_ends", _i),
        ("overlap", _i),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_longlong),
        ("aeds", ctypes.c_longlong),
        ("aed_deflated", ctypes.c_longlong),
        ("shifts_used", ctypes.c_longlong),
        ("exceptional", ctypes.c_longlong),
        ("small_solves", ctypes.c_longlong),
        ("swap_failures", ctypes.c_longlong),
        ("iterations", ctypes.c_longlong),
        ("gemm_flops", ctypes.c_double),
        ("chase_flops", ctypes.c_double),
        ("small_flops", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("t_aed_ms", ctypes.c_double),
        ("t_sweep_ms", ctypes.c_double),
        ("t_small_ms", ctypes.c_double),
        ("alg_flops", ctypes.c_double),
        ("gpu_update_ms", ctypes.c_double),
        ("gpu_chase_ms", ctypes.c_double),
        ("gpu_aed_ms", ctypes.c_double),
        ("gpu_small_ms", ctypes.c_double),
        ("gpu_other_ms", ctypes.c_double),
        ("n_update", ctypes.c_double),
        ("n_chase", ctypes.c_double),
        ("aed_qr_iters", ctypes.c_double),
        ("aed_swaps", ctypes.c_double),
        ("aed_cyc_qr", ctypes.c_double),
        ("aed_cyc_defl", ctypes.c_double),
        ("aed_cyc_hess", ctypes.c_double),
        ("aed_late", ctypes.c_double),
        ("policy_used", ctypes.c_double),
        ("policy_fallback", ctypes.c_double),
        ("aed_flops", ctypes.c_double),
        ("rec_aeds", ctypes.c_double),
        ("rec_inner_aeds", ctypes.c_double),
        ("rec_inner_sweeps", ctypes.c_double),
        ("gpu_rec_defl_ms", ctypes.c_double),
        ("chase_bytes", ctypes.c_double),
        ("aeds_top", ctypes.c_double),
        ("aed_top_deflated", ctypes.c_double),
        ("aed_launches", ctypes.c_double),
        ("gpu_update_far_ms", ctypes.c_double),
        ("n_update_far", ctypes.c_double),
        ("gemm_flops_far", ctypes.c_double),
    ]


SchurResult = namedtuple("SchurResult", "wr wi Z info")


def library_path() -> str:
    return _LIB_PATH


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise NeigError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so both share one runtime (devices, streams, memory) in this process
    _torch()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.neig_schur.argtypes = [_i, _vp, _i, _vp, _i, _vp, _vp, _vp]
    lib.neig_schur.restype = _i
    lib.neig_schur_batched.argtypes = [_i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.neig_schur_batched.restype = _i
    lib.neig_schur_batched_noalloc.argtypes = [_i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.neig_schur_batched_noalloc.restype = _i
    _fp = ctypes.POINTER(ctypes.c_float)
    sigs = {
        "neig_policy_bins": [_ip, _ip],
        "neig_policy_set": [_fp, _i, ctypes.c_float],
        "neig_policy_log": [_i, _fp, _ip, _fp],
        "neig_policy_features": [_i, _vp, _i, _i, _i, ctypes.c_double, _fp, _fp, _ip, _fp, _vp],
        "neig_mlp_grad": [_i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "neig_mlp_adam": [_vp, _vp, _vp, _vp, _i, ctypes.c_float, _vp],
        "neig_mlp_infer": [_i, _vp, _vp, _vp, _vp, _vp, _vp],
        "neig_reorder": [_i, _vp, _i, _vp, _i, _ip, _vp, _vp, _ip, _vp],
        "neig_hessenberg": [_i, _vp, _i, _vp, _i, _vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _i
    lib.neig_batched_flops.argtypes = [_dp]
    lib.neig_batched_flops.restype = _i
    lib.neig_set_batched_tune.argtypes = [_i, _ip, _ip, _ip, _ip, _ip]
    lib.neig_set_batched_tune.restype = _i
    lib.neig_get_batched_tune.argtypes = [_ip, _ip, _ip, _ip, _ip, _ip]
    lib.neig_get_batched_tune.restype = _i
    lib.neig_sweep.argtypes = [_i, _vp, _i, _vp, _i, _i, _i, _i, _dp, _dp, _vp]
    lib.neig_sweep.restype = _i
    lib.neig_aed.argtypes = [_i, _vp, _i, _vp, _i, _i, _i, _i, _ip, _ip, _dp, _dp, _vp]
    lib.neig_aed.restype = _i
    lib.neig_aed_top.argtypes = [_i, _vp, _i, _vp, _i, _i, _i, _i, _ip, _ip, _dp, _dp, _vp]
    lib.neig_aed_top.restype = _i
    lib.neig_small_schur.argtypes = [_i, _vp, _i, _vp, _i, _vp, _vp, _vp]
    lib.neig_small_schur.restype = _i
    lib.neig_set_params.argtypes = [ctypes.POINTER(Params)]
    lib.neig_set_params.restype = _i
    lib.neig_get_params.argtypes = [ctypes.POINTER(Params)]
    lib.neig_get_params.restype = _i
    lib.neig_get_stats.argtypes = [ctypes.POINTER(Stats)]
    lib.neig_get_stats.restype = _i
    lib.neig_finalize.argtypes = []
    lib.neig_finalize.restype = None
    lib.neig_version.argtypes = []
    lib.neig_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _torch():
    import torch

    return torch


def _check_matrix(name, t, n):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise NeigError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise NeigError(f"{name} must be float64")
    if not t.is_cuda:
        raise NeigError(f"{name} must be a GPU tensor (no CPU path)")
    if t.dim() != 2 or t.shape[0] != n or t.shape[1] != n:
        raise NeigError(f"{name} must be {n}x{n}")
    if n > 0 and (t.stride(0) != 1 or t.stride(1) < n):
        raise NeigError(f"{name} must be column-major (stride(0) == 1, stride(1) >= n)")
    return max(1, t.stride(1)) if n > 0 else 1


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def colmajor(a, device="cuda"):
    """A column-major float64 device copy of a numpy array or tensor."""
    torch = _torch()
    import numpy as np

    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    a = np.asarray(a, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).t()


def _raise(name, info):
    if info < 0:
        if info <= -100:
            raise NeigError(f"{name}: HIP runtime error {-100 - info}")
        raise NeigError(f"{name}: argument {-info} is invalid")


def schur(H, Z=None, stream=None) -> SchurResult:
    """Real Schur form in place: on return H holds S and Z holds Z_in Q, with
    H_in = Z_out S Z_out^T when Z_in = I (eq. 4).  Z=None starts from I.
    info > 0 counts unconverged eigenvalues (the call can be repeated)."""
    torch = _torch()
    lib = load_library()
    n = H.shape[0]
    ldh = _check_matrix("H", H, n)
    if Z is None:
        Z = torch.eye(n, dtype=torch.float64, device=H.device).t().contiguous().t()
    ldz = _check_matrix("Z", Z, n)
    wr = torch.empty(n, dtype=torch.float64, device=H.device)
    wi = torch.empty(n, dtype=torch.float64, device=H.device)
    info = lib.neig_schur(n, ctypes.c_void_p(H.data_ptr()), ldh, ctypes.c_void_p(Z.data_ptr()), ldz,
                          ctypes.c_void_p(wr.data_ptr()), ctypes.c_void_p(wi.data_ptr()), _stream_ptr(stream))
    _raise("neig_schur", info)
    return SchurResult(wr, wi, Z, info)


def small_schur(H, Z=None, stream=None) -> SchurResult:
    """Real Schur form of a matrix small enough for one workgroup's LDS (the
    double-shift QR used for small blocks and for AED windows), in place."""
    torch = _torch()
    lib = load_library()
    n = H.shape[0]
    ldh = _check_matrix("H", H, n)
    if Z is None:
        Z = torch.eye(n, dtype=torch.float64, device=H.device).t().contiguous().t()
    ldz = _check_matrix("Z", Z, n)
    wr = torch.empty(n, dtype=torch.float64, device=H.device)
    wi = torch.empty(n, dtype=torch.float64, device=H.device)
    info = lib.neig_small_schur(n, ctypes.c_void_p(H.data_ptr()), ldh, ctypes.c_void_p(Z.data_ptr()), ldz,
                                ctypes.c_void_p(wr.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                                _stream_ptr(stream))
    _raise("neig_small_schur", info)
    return SchurResult(wr, wi, Z, info)


def sweep(H, Z, ktop, kbot, shifts_re, shifts_im, stream=None) -> int:
    """One multishift QR sweep over the active block [ktop, kbot] with the given
    shifts (complex pairs adjacent), H and Z updated in place."""
    import numpy as np

    lib = load_library()
    n = H.shape[0]
    ldh = _check_matrix("H", H, n)
    ldz = _check_matrix("Z", Z, n)
    sr = np.ascontiguousarray(shifts_re, dtype=np.float64)
    si = np.ascontiguousarray(shifts_im, dtype=np.float64)
    ns = int(sr.size)
    info = lib.neig_sweep(n, ctypes.c_void_p(H.data_ptr()), ldh, ctypes.c_void_p(Z.data_ptr()), ldz,
                          int(ktop), int(kbot), ns, sr.ctypes.data_as(_dp), si.ctypes.data_as(_dp),
                          _stream_ptr(stream))
    _raise("neig_sweep", info)
    return info


def aed(H, Z, ktop, kbot, nw, stream=None, leading=False):
    """One aggressive-early-deflation step on the trailing window of [ktop, kbot]
    (or, with ``leading``, on its leading window).  Returns (nd, shifts_re,
    shifts_im): deflated count and the undeflated Ritz values (shift
    candidates, bottom-most last)."""
    import numpy as np

    lib = load_library()
    fn = lib.neig_aed_top if leading else lib.neig_aed
    n = H.shape[0]
    ldh = _check_matrix("H", H, n)
    ldz = _check_matrix("Z", Z, n)
    nd = ctypes.c_int(0)
    nsh = ctypes.c_int(0)
    sr = np.zeros(max(nw, 1))
    si = np.zeros(max(nw, 1))
    info = fn(n, ctypes.c_void_p(H.data_ptr()), ldh, ctypes.c_void_p(Z.data_ptr()), ldz, int(ktop), int(kbot),
              int(nw), ctypes.byref(nd), ctypes.byref(nsh), sr.ctypes.data_as(_dp), si.ctypes.data_as(_dp),
              _stream_ptr(stream))
    _raise("neig_aed_top" if leading else "neig_aed", info)
    k = nsh.value
    return nd.value, sr[:k].copy(), si[:k].copy()


class BatchedCall:
    """Device-side argument tables of one neig_schur_batched call.  Keeping this
    object alive keeps the tables alive, which a captured graph needs."""

    def __init__(self, Hs, Zs, wrs, wis, info, meta, ptrs):
        self.Hs, self.Zs, self.wrs, self.wis, self.info = Hs, Zs, wrs, wis, info
        self.meta, self.ptrs = meta, ptrs


def batched_tables(Hs, Zs=None):
    """Output buffers and the device argument tables for a list of problems."""
    torch = _torch()
    b = len(Hs)
    dev = Hs[0].device if b else torch.device("cuda")
    if Zs is None:
        Zs = [torch.eye(h.shape[0], dtype=torch.float64, device=dev).t().contiguous().t() for h in Hs]
    if len(Zs) != b:
        raise NeigError("schur_batched: Hs and Zs differ in length")
    ns = [int(h.shape[0]) for h in Hs]
    ldh = [_check_matrix("H", h, k) for h, k in zip(Hs, ns)]
    ldz = [_check_matrix("Z", z, k) for z, k in zip(Zs, ns)]
    wrs = [torch.empty(k, dtype=torch.float64, device=dev) for k in ns]
    wis = [torch.empty(k, dtype=torch.float64, device=dev) for k in ns]
    meta = torch.tensor(ns + ldh + ldz, dtype=torch.int32, device=dev)
    ptrs = torch.tensor([h.data_ptr() for h in Hs] + [z.data_ptr() for z in Zs]
                        + [w.data_ptr() for w in wrs] + [w.data_ptr() for w in wis],
                        dtype=torch.int64, device=dev)
    info = torch.zeros(b, dtype=torch.int32, device=dev)
    return BatchedCall(Hs, Zs, wrs, wis, info, meta, ptrs)


def launch_batched(call, stream=None, noalloc: bool = False) -> None:
    """Enqueue neig_schur_batched (or, with ``noalloc``, the entry point that
    allocates nothing, neig_schur_batched_noalloc) for the tables of ``call``
    (asynchronous)."""
    lib = load_library()
    b = len(call.Hs)
    m, p = call.meta.data_ptr(), call.ptrs.data_ptr()
    vp = ctypes.c_void_p
    name = "neig_schur_batched_noalloc" if noalloc else "neig_schur_batched"
    rc = getattr(lib, name)(b, vp(m), vp(p), vp(m + 4 * b), vp(p + 8 * b), vp(m + 8 * b), vp(p + 16 * b),
                            vp(p + 24 * b), vp(call.info.data_ptr()), _stream_ptr(stream))
    _raise(name, rc)


def schur_batched(Hs, Zs=None, stream=None):
    """Real Schur forms of a list of independent problems of uneven size in one
    asynchronous call on ``stream`` (default: torch's current stream).  Returns a
    :class:`BatchedCall` holding Hs (overwritten by S), Zs, wrs, wis and the
    per-problem info tensor."""
    call = batched_tables(Hs, Zs)
    launch_batched(call, stream)
    return call


def batched_flops() -> float:
    """neig_batched_flops: the method's operation count of the last
    neig_schur_batched call on the current device (waits for the device)."""
    out = ctypes.c_double(0.0)
    _raise("neig_batched_flops", load_library().neig_batched_flops(ctypes.byref(out)))
    return out.value


def schur_batched_noalloc(Hs, Zs=None, stream=None):
    """As :func:`schur_batched`, through neig_schur_batched_noalloc (at most
    NEIG_BATCH_NOALLOC_MAX problems; the library allocates nothing)."""
    call = batched_tables(Hs, Zs)
    launch_batched(call, stream, noalloc=True)
    return call


def set_batched_tune(n_hi, nw, ns, nmin, chase_w) -> None:
    """Per-size-class parameters of the batched solver (lists of equal length)."""
    lib = load_library()
    k = len(nw)
    arrs = [(ctypes.c_int * k)(*[int(x) for x in a]) for a in (list(n_hi) + [0] * (k - len(n_hi)), nw, ns, nmin,
                                                                chase_w)]
    rc = lib.neig_set_batched_tune(k, *arrs)
    if rc != 0:
        raise NeigError(f"neig_set_batched_tune: invalid argument {-rc}")


def get_batched_tune() -> dict:
    lib = load_library()
    k = 16
    cnt = ctypes.c_int()
    arrs = [(ctypes.c_int * k)() for _ in range(5)]
    lib.neig_get_batched_tune(ctypes.byref(cnt), *arrs)
    names = ("n_hi", "nw", "ns", "nmin", "chase_w")
    return {nm: list(a)[: cnt.value] for nm, a in zip(names, arrs)}


MLP_NPARAM = 6848
MLP_NIN = 24


def policy_bins():
    """(shift-count bins, window-size bins) of the proposal network's heads."""
    lib = load_library()
    a, b = (ctypes.c_int * 8)(), (ctypes.c_int * 8)()
    lib.neig_policy_bins(a, b)
    return list(a), list(b)


def policy_set(theta=None, min_conf: float = 0.0) -> None:
    """Install (host array of MLP_NPARAM floats) or remove (None) the network."""
    import numpy as np

    lib = load_library()
    if theta is None:
        rc = lib.neig_policy_set(None, 0, float(min_conf))
    else:
        th = np.ascontiguousarray(theta, dtype=np.float32)
        rc = lib.neig_policy_set(th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(th.size), float(min_conf))
    if rc != 0:
        raise NeigError(f"neig_policy_set: invalid argument {-rc}")


def policy_log():
    """Decisions of the last neig_schur call: (features [k,24], bins [k,2],
    stats [k,4] = deflations, ms, m, applied)."""
    import numpy as np

    lib = load_library()
    k = lib.neig_policy_log(0, None, None, None)
    feat = np.zeros((max(k, 1), MLP_NIN), dtype=np.float32)
    bins = np.zeros((max(k, 1), 2), dtype=np.int32)
    st = np.zeros((max(k, 1), 4), dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.neig_policy_log(k, feat.ctypes.data_as(fp), bins.ctypes.data_as(_ip), st.ctypes.data_as(fp))
    return feat[:k], bins[:k], st[:k]


def policy_features(H, ktop: int, kbot: int, hnorm: float, extra, stream=None):
    """Features of the active block [ktop, kbot] of the device matrix H and the
    installed network's (bins, probabilities) for them."""
    import numpy as np

    lib = load_library()
    n = int(H.shape[0])
    ldh = _check_matrix("H", H, n)
    ex = np.ascontiguousarray(extra, dtype=np.float32)
    feat = np.zeros(MLP_NIN, dtype=np.float32)
    bins = np.zeros(2, dtype=np.int32)
    conf = np.zeros(2, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    rc = lib.neig_policy_features(n, ctypes.c_void_p(H.data_ptr()), ldh, int(ktop), int(kbot), float(hnorm),
                                  ex.ctypes.data_as(fp), feat.ctypes.data_as(fp), bins.ctypes.data_as(_ip),
                                  conf.ctypes.data_as(fp), _stream_ptr(stream))
    _raise("neig_policy_features", rc)
    return feat, bins, conf


def _dev(t, dtype, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise NeigError(f"{name}: expected a contiguous {dtype} GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def mlp_grad(X, a, c, w, theta, stream=None):
    """(loss, grad) of the reward-weighted cross-entropy on the GPU (FP32)."""
    torch = _torch()
    lib = load_library()
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    rc = lib.neig_mlp_grad(int(X.shape[0]), _dev(X, torch.float32, "X"), _dev(a, torch.int32, "a"),
                           _dev(c, torch.int32, "c"), _dev(w, torch.float32, "w"),
                           _dev(theta, torch.float32, "theta"), ctypes.c_void_p(grad.data_ptr()),
                           ctypes.c_void_p(loss.data_ptr()), _stream_ptr(stream))
    _raise("neig_mlp_grad", rc)
    return loss, grad


def mlp_adam(theta, grad, m, v, step: int, lr: float, stream=None) -> None:
    torch = _torch()
    lib = load_library()
    rc = lib.neig_mlp_adam(_dev(theta, torch.float32, "theta"), _dev(grad, torch.float32, "grad"),
                           _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"), int(step), float(lr),
                           _stream_ptr(stream))
    _raise("neig_mlp_adam", rc)


def mlp_infer(X, theta, stream=None):
    """(logits [B,16], bins [B,2], conf [B,2]) with BF16 operands on the GPU."""
    torch = _torch()
    lib = load_library()
    B = int(X.shape[0])
    logits = torch.empty((B, 16), dtype=torch.float32, device=X.device)
    bins = torch.empty((B, 2), dtype=torch.int32, device=X.device)
    conf = torch.empty((B, 2), dtype=torch.float32, device=X.device)
    rc = lib.neig_mlp_infer(B, _dev(X, torch.float32, "X"), _dev(theta, torch.float32, "theta"),
                            ctypes.c_void_p(logits.data_ptr()), ctypes.c_void_p(bins.data_ptr()),
                            ctypes.c_void_p(conf.data_ptr()), _stream_ptr(stream))
    _raise("neig_mlp_infer", rc)
    return logits, bins, conf


def hessenberg(A, Q=None, accumulate=True, stream=None):
    """Reduce A (device FP64, column-major, in place) to upper Hessenberg form.
    With ``accumulate`` the orthogonal factor is applied to Q (identity when Q
    is None) and returned: A_in = Q H Q^T for Q_in = I.  Returns Q or None."""
    torch = _torch()
    lib = load_library()
    n = int(A.shape[0])
    lda = _check_matrix("A", A, n)
    qp, ldq = None, 1
    if accumulate:
        if Q is None:
            Q = torch.eye(n, dtype=torch.float64, device=A.device).t().contiguous().t()
        ldq = _check_matrix("Q", Q, n)
        qp = ctypes.c_void_p(Q.data_ptr())
    info = lib.neig_hessenberg(n, ctypes.c_void_p(A.data_ptr()), lda, qp, ldq, _stream_ptr(stream))
    _raise("neig_hessenberg", info)
    return Q if accumulate else None


def reorder(S, Z, select, stream=None):
    """Move the selected eigenvalues (host sequence of 0/1 per diagonal position)
    of the Schur form S (device, in place) to the leading block; Z updated in
    place.  Returns (wr, wi, m, info)."""
    import numpy as np

    torch = _torch()
    lib = load_library()
    n = int(S.shape[0])
    lds = _check_matrix("S", S, n)
    ldz = _check_matrix("Z", Z, n)
    sel = np.ascontiguousarray(select, dtype=np.int32)
    if sel.size != n:
        raise NeigError("reorder: select needs one entry per diagonal position")
    wr = torch.empty(n, dtype=torch.float64, device=S.device)
    wi = torch.empty(n, dtype=torch.float64, device=S.device)
    m = ctypes.c_int()
    info = lib.neig_reorder(n, ctypes.c_void_p(S.data_ptr()), lds, ctypes.c_void_p(Z.data_ptr()), ldz,
                            sel.ctypes.data_as(_ip), ctypes.c_void_p(wr.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                            ctypes.byref(m), _stream_ptr(stream))
    _raise("neig_reorder", info)
    return wr, wi, m.value, info


def set_params(**kw) -> None:
    lib = load_library()
    p = Params()
    lib.neig_get_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise NeigError(f"unknown parameter {k}")
        setattr(p, k, int(v))
    rc = lib.neig_set_params(ctypes.byref(p))
    if rc != 0:
        raise NeigError(f"neig_set_params: invalid field {-rc}")


def get_params() -> dict:
    lib = load_library()
    p = Params()
    lib.neig_get_params(ctypes.byref(p))
    return {f: getattr(p, f) for f, _ in Params._fields_}


def get_stats() -> dict:
    lib = load_library()
    s = Stats()
    lib.neig_get_stats(ctypes.byref(s))
    return {f: getattr(s, f) for f, _ in Stats._fields_ if f != "reserved"}


def finalize() -> None:
    if _lib is not None:
        _lib.neig_finalize()
