"""Result checks for a real Schur decomposition H = Z S Z^T (test code).

P1 backward error, P2 orthogonality, P3 structure of S and of (wr, wi),
P4 spectral invariants of the input, P5 eigenvalue matching.  numpy only; the
large-n variants in the GPU tests do the same products with torch on the GPU.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps  # 2^-52


def backward_error(H, S, Z) -> float:
    H = np.asarray(H)
    nh = np.linalg.norm(H)
    if nh == 0:
        return float(np.linalg.norm(Z @ S @ Z.T))
    return float(np.linalg.norm(H - Z @ S @ Z.T) / nh)


def orthogonality(Z) -> float:
    n = Z.shape[0]
    return float(np.linalg.norm(Z.T @ Z - np.eye(n)))


def structure_violations(S, wr, wi) -> list:
    """Standardised real Schur form: exact zeros below the subdiagonal, no two
    consecutive nonzero subdiagonal entries, 2x2 blocks with equal diagonal
    entries and off-diagonal entries of opposite sign, and wr/wi equal to the
    block eigenvalues bit for bit."""
    S = np.asarray(S)
    n = S.shape[0]
    bad = []
    if n == 0:
        return bad
    low = np.tril(S, -2)
    if np.any(low != 0):
        bad.append("nonzero below subdiagonal")
    sub = np.diag(S, -1)
    j = 0
    while j < n:
        if j + 1 < n and sub[j] != 0:
            if j + 2 < n and sub[j + 1] != 0:
                bad.append(f"consecutive nonzero subdiagonal at {j}")
            a, b, c, d = S[j, j], S[j, j + 1], S[j + 1, j], S[j + 1, j + 1]
            if a != d:
                bad.append(f"2x2 at {j}: unequal diagonal")
            if not (b * c < 0):
                bad.append(f"2x2 at {j}: off-diagonal signs")
            im = np.sqrt(abs(b)) * np.sqrt(abs(c))
            if not (wr[j] == a and wr[j + 1] == d and wi[j] == im and wi[j + 1] == -im):
                bad.append(f"2x2 at {j}: wr/wi mismatch")
            j += 2
        else:
            if wr[j] != S[j, j] or wi[j] != 0:
                bad.append(f"1x1 at {j}: wr/wi mismatch")
            j += 1
    return bad


def invariant_errors(H, wr, wi) -> dict:
    """|sum lambda - tr H| and |sum lambda^2 - tr H^2| (relative to ||H||_F and
    ||H||_F^2).  tr H^2 of a Hessenberg matrix is sum h_ii^2 + 2 sum h_{i,i+1} h_{i+1,i}."""
    H = np.asarray(H)
    nh = np.linalg.norm(H)
    tr = np.trace(H)
    tr2 = np.sum(np.diag(H) ** 2) + 2.0 * np.sum(np.diag(H, 1) * np.diag(H, -1))
    lam = np.asarray(wr) + 1j * np.asarray(wi)
    s1 = np.sum(lam)
    s2 = np.sum(lam * lam)
    scale = nh if nh > 0 else 1.0
    return {
        "trace": float(abs(s1 - tr) / scale),
        "trace_sq": float(abs(s2 - tr2) / scale**2),
        "imag_sum": float(abs(s1.imag) / scale),
    }


def eigs(wr, wi) -> np.ndarray:
    return np.asarray(wr) + 1j * np.asarray(wi)


def match_eigenvalues(a, b):
    """Pair two eigenvalue lists: sort both by (real, |imag|, sign imag); if a pair
    is far apart, fall back to the optimal assignment on |a_i - b_j|.
    Returns (a_sorted, b_matched, perm) with b_matched[k] paired to a_sorted[k]."""
    a = np.asarray(a, dtype=complex)
    b = np.asarray(b, dtype=complex)

    def key(z):
        return np.lexsort((np.sign(z.imag), np.abs(z.imag), z.real))

    ia, ib = key(a), key(b)
    A, B = a[ia], b[ib]
    scale = max(np.max(np.abs(a)) if a.size else 1.0, 1.0)
    if a.size and np.max(np.abs(A - B)) > 1e-8 * scale:
        from scipy.optimize import linear_sum_assignment

        cost = np.abs(A[:, None] - B[None, :])
        r, c = linear_sum_assignment(cost)
        B = B[c[np.argsort(r)]]
    return A, B


def std2x2_cases():
    """2x2 blocks for the standardisation pins: hand-picked special cases (already
    triangular, zero upper entry, equal diagonal, tiny coupling, near underflow,
    strongly graded) and 400 seeded random blocks, half of them with entries
    spread over 16 orders of magnitude."""
    g = np.random.default_rng(12)
    cases = [(1, 2, 3, 4), (1, -2, 3, 1), (0, 1, -1, 0), (2, 0, 3, 5), (2, 3, 0, 5), (1, 1e-20, 1e-20, 1),
             (1, 1, -1e-18, 1), (3, 4, 4, 3), (0, 0, 1, 0), (1e-300, 1e-300, -1e-300, 1e-300), (5, -1, 1, 5),
             (1, 4, 1, 1), (-2, 1e8, -1e-8, 3)]
    cases += [tuple(g.standard_normal(4)) for _ in range(200)]
    cases += [tuple(g.standard_normal(4) * 10.0 ** g.integers(-8, 8, 4)) for _ in range(200)]
    return cases


def t_eigs_in_order(T):
    """Eigenvalues of a standardised quasi-triangular T in diagonal order."""
    n = T.shape[0]
    out = np.zeros(n, dtype=complex)
    j = 0
    while j < n:
        if j + 1 < n and T[j + 1, j] != 0:
            b = np.sqrt(abs(T[j, j + 1] * T[j + 1, j]))
            out[j], out[j + 1] = T[j, j] + 1j * b, T[j, j] - 1j * b
            j += 2
        else:
            out[j] = T[j, j]
            j += 1
    return out
