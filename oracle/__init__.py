"""CPU oracle for the Schur reduction (test infrastructure only).

Plain, slow, single-threaded FP64 reference written from the textbook
definitions the paper relies on (Section 2, eq. 3 and eq. 4; Section 3.2 for the
double-shift bulge chase).  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library and never calls it; the two sides implement the same readings
of the paper (deflation criteria, exceptional shift, reflector sign
convention), each in code of its own.

The numerical work lives in ``neig_oracle.c`` (compiled with gcc into
``liboracle.so`` next to this file by :func:`build`); this module only marshals
numpy arrays (column-major copies) through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "neig_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build() -> str:
    """Compile the oracle with gcc (-O2, no BLAS, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i = ctypes.c_int
    lib.neig_oracle_hessenberg.argtypes = [i, _dp, i, _dp, i]
    lib.neig_oracle_schur.argtypes = [i, _dp, i, _dp, i, _dp, _dp, i]
    lib.neig_oracle_francis_step.argtypes = [i, _dp, i, _dp, i, i, i, ctypes.c_double, ctypes.c_double]
    lib.neig_oracle_std2x2.argtypes = [_dp] * 10
    lib.neig_oracle_std2x2.restype = None
    lib.neig_oracle_cond.argtypes = [i, _dp, i, _dp]
    lib.neig_oracle_cond_subset.argtypes = [i, _dp, i, ctypes.POINTER(ctypes.c_int), i, _dp]
    lib.neig_oracle_last_iterations.argtypes = []
    lib.neig_oracle_swap.argtypes = [i, _dp, i, _dp, i, i, i, i]
    lib.neig_oracle_reorder.argtypes = [i, _dp, i, _dp, i, ctypes.POINTER(ctypes.c_int), _dp, _dp,
                                        ctypes.POINTER(ctypes.c_int)]
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def hessenberg(A):
    """Householder reduction: returns (H, Q1) with A = Q1 H Q1^T (eq. 3)."""
    lib = _load()
    H = _f64(A)
    n = H.shape[0]
    Q = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib.neig_oracle_hessenberg(n, _ptr(H), max(1, n), _ptr(Q), max(1, n))
    if info != 0:
        raise ValueError(f"neig_oracle_hessenberg: info={info}")
    return H, Q


def schur(H, Z=None, maxit: int = 0):
    """Double-shift Francis QR: returns (S, Z, wr, wi, info) with H = Z S Z^T
    (eq. 4) and Z_out = Z_in Q.  info > 0: rows/cols 0..info-1 unreduced."""
    lib = _load()
    S = _f64(H)
    n = S.shape[0]
    Zo = np.eye(n, dtype=np.float64, order="F") if Z is None else _f64(Z)
    wr = np.zeros(n)
    wi = np.zeros(n)
    info = lib.neig_oracle_schur(n, _ptr(S), max(1, n), _ptr(Zo), max(1, n), _ptr(wr), _ptr(wi), int(maxit))
    return S, Zo, wr, wi, info


def last_iterations() -> int:
    """Double-shift iterations used by the most recent :func:`schur` call."""
    return int(_load().neig_oracle_last_iterations())


def francis_step(H, Z, tr: float, det: float, ilo: int = 0, ihi: int | None = None):
    """One implicit double-shift step on rows/cols ilo..ihi with the shift
    polynomial x^2 - tr x + det (full-width updates of H and Z)."""
    lib = _load()
    Hc = _f64(H)
    Zc = _f64(Z)
    n = Hc.shape[0]
    ihi = n - 1 if ihi is None else ihi
    info = lib.neig_oracle_francis_step(n, _ptr(Hc), n, _ptr(Zc), n, ilo, ihi, float(tr), float(det))
    if info != 0:
        raise ValueError("francis_step needs a block of at least 3 rows")
    return Hc, Zc


def std2x2(a: float, b: float, c: float, d: float):
    """Standardise [[a b][c d]]; returns (block 2x2, cs, sn, (rt1r, rt1i, rt2r, rt2i))
    with [[a b][c d]] = G block G^T, G = [[cs -sn][sn cs]]."""
    lib = _load()
    vals = [ctypes.c_double(float(x)) for x in (a, b, c, d)] + [ctypes.c_double() for _ in range(6)]
    lib.neig_oracle_std2x2(*[ctypes.byref(v) for v in vals])
    a2, b2, c2, d2, cs, sn, r1, i1, r2, i2 = (v.value for v in vals)
    return np.array([[a2, b2], [c2, d2]]), cs, sn, (r1, i1, r2, i2)


def cond(S):
    """Eigenvalue condition numbers (capped at 1/eps) for each diagonal position of
    a quasi-triangular S."""
    lib = _load()
    Sc = _f64(S)
    n = Sc.shape[0]
    out = np.zeros(n)
    info = lib.neig_oracle_cond(n, _ptr(Sc), max(1, n), _ptr(out))
    if info != 0:
        raise ValueError(f"neig_oracle_cond: info={info}")
    return out


def cond_subset(S, idx):
    """Condition numbers of the eigenvalues at the listed diagonal positions of a
    quasi-triangular S (each O(n^2))."""
    lib = _load()
    Sc = _f64(S)
    n = Sc.shape[0]
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.zeros(ix.size)
    info = lib.neig_oracle_cond_subset(n, _ptr(Sc), max(1, n), ix.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                       int(ix.size), _ptr(out))
    if info != 0:
        raise ValueError(f"neig_oracle_cond_subset: info={info}")
    return out


def swap(S, Z, st: int, p: int, q: int):
    """Exchange the adjacent diagonal blocks at st (sizes p then q).  Returns
    (S, Z, info); info 1 = swap rejected."""
    lib = _load()
    Sc = _f64(S)
    Zc = _f64(Z)
    n = Sc.shape[0]
    info = lib.neig_oracle_swap(n, _ptr(Sc), max(1, n), _ptr(Zc), max(1, n), int(st), int(p), int(q))
    return Sc, Zc, info


def reorder(S, Z, select):
    """Move the selected eigenvalues to the leading block (relative order kept).
    Returns (S, Z, wr, wi, m, info)."""
    lib = _load()
    Sc = _f64(S)
    Zc = _f64(Z)
    n = Sc.shape[0]
    sel = np.ascontiguousarray(select, dtype=np.int32)
    wr = np.zeros(n)
    wi = np.zeros(n)
    m = ctypes.c_int()
    info = lib.neig_oracle_reorder(n, _ptr(Sc), max(1, n), _ptr(Zc), max(1, n),
                                   sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(wr), _ptr(wi),
                                   ctypes.byref(m))
    return Sc, Zc, wr, wi, m.value, info
