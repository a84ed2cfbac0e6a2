"""Pins of the CPU oracle against what mathematics fixes (no GPU).

Each test targets a different way the oracle could be wrong: closed forms for
the 2x2 standardisation, the implicit-Q theorem for the bulge chase (a dropped
term or a wrong index changes the iterate), exactly known spectra (companion
matrices, cyclic shift, normal and prescribed-spectrum matrices), library
routines on special cases (eigvalsh, LAPACK Hessenberg and eigenvectors), and
the invariants of the result.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from checks import (EPS, backward_error, eigs, invariant_errors, match_eigenvalues, orthogonality, std2x2_cases,
                    structure_violations)
from paper_2002_05024_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- 2x2 blocks

@pytest.mark.parametrize("blk", std2x2_cases())
def test_std2x2_closed_form(blk):
    a, b, c, d = blk
    B = np.array([[a, b], [c, d]])
    S, cs, sn, (r1, i1, r2, i2) = oracle.std2x2(a, b, c, d)
    G = np.array([[cs, -sn], [sn, cs]])
    nb = np.linalg.norm(B)
    assert abs(cs * cs + sn * sn - 1) <= 4 * EPS
    # similarity: B = G S G^T
    assert np.linalg.norm(G @ S @ G.T - B) <= 8 * EPS * nb
    if S[1, 0] == 0:
        assert i1 == 0 and i2 == 0 and r1 == S[0, 0] and r2 == S[1, 1]
    else:
        assert S[0, 0] == S[1, 1] and S[0, 1] * S[1, 0] < 0
        assert r1 == r2 == S[0, 0] and i1 > 0 and i2 == -i1
        assert i1 == np.sqrt(abs(S[0, 1])) * np.sqrt(abs(S[1, 0]))
    # eigenvalues: trace and determinant of B are fixed
    l1, l2 = complex(r1, i1), complex(r2, i2)
    assert abs((l1 + l2) - (a + d)) <= 8 * EPS * nb
    assert abs(l1 * l2 - (a * d - b * c)) <= 16 * EPS * nb * nb
    # against the roots of the characteristic polynomial when well separated
    disc = (a - d) ** 2 + 4 * b * c
    if abs(disc) > 1e-6 * nb * nb and nb > 1e-100:
        roots = np.roots([1.0, -(a + d), a * d - b * c])
        got = np.array([l1, l2])
        A, R = match_eigenvalues(got, roots)
        assert np.max(np.abs(A - R)) <= 1e-9 * nb


# ---------------------------------------------------------------- Hessenberg reduction

@pytest.mark.parametrize("n", [1, 2, 3, 7, 40])
def test_hessenberg_reduction(n):
    A = inputs.rng(99, n).standard_normal((n, n))
    H, Q = oracle.hessenberg(A)
    assert np.all(np.tril(H, -2) == 0)
    assert backward_error(A, H, Q) <= 10 * n * EPS
    assert orthogonality(Q) <= 10 * n * EPS
    assert np.allclose(Q[:, 0], np.eye(n)[:, 0], atol=0)
    # implicit-Q theorem: with Q e1 = e1 the Hessenberg form is unique up to a
    # diagonal sign matrix D (LAPACK's reduction is a library run, not read)
    H2, _ = inputs.to_hessenberg(A)
    if n >= 2:
        d = np.ones(n)
        for k in range(1, n):
            d[k] = d[k - 1] * np.sign(H[k, k - 1]) * np.sign(H2[k, k - 1])
        assert np.linalg.norm(d[:, None] * H * d[None, :] - H2) <= 1e-10 * np.linalg.norm(A)


# ---------------------------------------------------------------- bulge chase (implicit-Q theorem)

def _implicit_q_reference(H, tr, det, ilo, ihi):
    """H' = Q^T H Q with p(Hb) = Hb^2 - tr Hb + det I = Q_b R on the block (library QR)."""
    n = H.shape[0]
    Hb = H[ilo:ihi + 1, ilo:ihi + 1]
    P = Hb @ Hb - tr * Hb + det * np.eye(Hb.shape[0])
    Qb, _ = np.linalg.qr(P)
    Q = np.eye(n)
    Q[ilo:ihi + 1, ilo:ihi + 1] = Qb
    return Q.T @ H @ Q, Q


@pytest.mark.parametrize("n,ilo,ihi,tr,det", [
    (12, 0, 11, 20.0, 109.0),       # complex pair 10 +- 3i, far from the spectrum
    (12, 0, 11, -11.0, 30.0),       # real pair -5, -6
    (15, 3, 11, 14.0, 53.0),        # block step: full-width updates outside the block
    (5, 1, 3, 9.0, 25.0),           # smallest block (three rows)
])
def test_francis_step_implicit_q(n, ilo, ihi, tr, det):
    H = inputs.random_hessenberg(n, inputs.rng(98, n + ilo))
    if ilo > 0:
        H[ilo, ilo - 1] = 0.0
    if ihi + 1 < n:
        H[ihi + 1, ihi] = 0.0
    Ho, Zo = oracle.francis_step(H, np.eye(n), tr, det, ilo, ihi)
    Href, Qref = _implicit_q_reference(H, tr, det, ilo, ihi)
    # fix the column signs: D chosen so that D Q^T Zo is closest to I
    d = np.sign(np.sum(Qref * Zo, axis=0))
    d[d == 0] = 1
    nh = np.linalg.norm(H)
    assert np.linalg.norm(Zo - Qref * d[None, :]) <= 1e-11
    assert np.linalg.norm(Ho - d[:, None] * Href * d[None, :]) <= 1e-11 * nh
    assert np.all(np.tril(Ho, -2) == 0)
    assert backward_error(H, Ho, Zo) <= 20 * n * EPS


# ---------------------------------------------------------------- full Schur reduction

def _check_schur(H, S, Z, wr, wi, info, bound=50):
    n = H.shape[0]
    assert info == 0
    assert backward_error(H, S, Z) <= bound * max(n, 1) * EPS
    assert orthogonality(Z) <= bound * max(n, 1) * EPS
    assert structure_violations(S, wr, wi) == []
    inv = invariant_errors(H, wr, wi)
    assert inv["trace"] <= 10 * np.sqrt(n) * n * EPS
    assert inv["trace_sq"] <= 10 * n * n * EPS
    assert inv["imag_sum"] <= 10 * n * EPS


def test_schur_trivial_sizes():
    S, Z, wr, wi, info = oracle.schur(np.zeros((0, 0)))
    assert info == 0 and S.shape == (0, 0)
    S, Z, wr, wi, info = oracle.schur(np.array([[3.5]]))
    assert info == 0 and wr[0] == 3.5 and wi[0] == 0 and Z[0, 0] == 1
    # 2x2 complex and real
    for blk in ([[1.0, 2.0], [-3.0, 4.0]], [[1.0, 2.0], [3.0, 4.0]]):
        H = np.array(blk)
        S, Z, wr, wi, info = oracle.schur(H)
        _check_schur(H, S, Z, wr, wi, info)


def test_schur_triangular_input_is_untouched():
    g = inputs.rng(97, 0)
    H = np.asfortranarray(np.triu(g.standard_normal((30, 30))))
    S, Z, wr, wi, info = oracle.schur(H)
    assert info == 0
    assert oracle.last_iterations() == 0
    assert np.array_equal(S, H) and np.array_equal(Z, np.eye(30))
    assert np.array_equal(wr, np.diag(H)) and np.all(wi == 0)


@pytest.mark.parametrize("n", [3, 5, 20, 64, 150])
def test_schur_random_hessenberg_invariants(n):
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 1000 + n))
    S, Z, wr, wi, info = oracle.schur(H)
    _check_schur(H, S, Z, wr, wi, info)
    # LAPACK eigenvalues as an independent backward-stable reference where the
    # oracle's own condition estimate makes the comparison meaningful
    cnd = oracle.cond(S)
    ref = scipy.linalg.eigvals(H)
    A, B = match_eigenvalues(eigs(wr, wi), ref)
    ca = cnd[np.lexsort((np.sign(wi), np.abs(wi), wr))]
    nh = np.linalg.norm(H)
    pinned = ca * 1e-10 < 1
    assert np.all(np.abs(A - B)[pinned] <= 1e-10 * nh * ca[pinned])


@pytest.mark.parametrize("name", [c["name"] for c in json.load(open(os.path.join(GOLDEN, "companion.json")))["cases"]])
def test_schur_companion_golden(name):
    case = [c for c in json.load(open(os.path.join(GOLDEN, "companion.json")))["cases"] if c["name"] == name][0]
    c = np.array(case["coeffs"], dtype=np.float64)
    n = c.size
    C = np.zeros((n, n), order="F")
    C[0, :] = -c
    for i in range(1, n):
        C[i, i - 1] = 1.0
    S, Z, wr, wi, info = oracle.schur(C)
    _check_schur(C, S, Z, wr, wi, info)
    roots = np.array([complex(r, i) for r, i in case["roots"]])
    A, B = match_eigenvalues(eigs(wr, wi), roots)
    assert np.max(np.abs(A - B)) <= case["tol"] * max(1.0, np.max(np.abs(roots)))


@pytest.mark.parametrize("n", [4, 8, 16, 31])
def test_schur_cyclic_shift_roots_of_unity(n):
    """Standard shifts make no progress on the cyclic shift matrix; only the
    exceptional shifts get it to converge.  Eigenvalues: the n-th roots of unity."""
    C = inputs.cyclic_shift(n)
    S, Z, wr, wi, info = oracle.schur(C)
    _check_schur(C, S, Z, wr, wi, info)
    roots = np.exp(2j * np.pi * np.arange(n) / n)
    A, B = match_eigenvalues(eigs(wr, wi), roots)
    assert np.max(np.abs(A - B)) <= 1e-12
    assert oracle.last_iterations() >= 10


@pytest.mark.parametrize("n", [10, 60])
def test_schur_normal_matrix_eigenvalues(n):
    A, lam = inputs.normal_matrix(n, inputs.rng(inputs.NORMAL, n))
    H, _ = oracle.hessenberg(A)
    S, Z, wr, wi, info = oracle.schur(H)
    _check_schur(H, S, Z, wr, wi, info)
    cnd = oracle.cond(S)
    assert np.max(np.abs(cnd - 1)) <= 1e-8
    X, Y = match_eigenvalues(eigs(wr, wi), lam)
    assert np.max(np.abs(X - Y)) <= 10 * n * EPS * np.linalg.norm(H)


@pytest.mark.parametrize("n", [40, 120])
def test_schur_prescribed_spectrum(n):
    """U T U^T with a well-conditioned T (strictly-upper std 0.1/sqrt(n)): the
    computed eigenvalues agree with the prescribed ones to 1e-10 ||H|| cond."""
    A, lam = inputs.prescribed_matrix(n, inputs.rng(inputs.PRESCRIBED, n), 0.1 / np.sqrt(n))
    H, Q1 = oracle.hessenberg(A)
    S, Z, wr, wi, info = oracle.schur(H, Q1)
    assert info == 0
    assert backward_error(A, S, Z) <= 50 * n * EPS
    assert orthogonality(Z) <= 50 * n * EPS
    cnd = oracle.cond(S)
    order = np.lexsort((np.sign(wi), np.abs(wi), wr))
    X, Y = match_eigenvalues(eigs(wr, wi), lam)
    assert np.all(np.abs(X - Y) <= 1e-10 * np.linalg.norm(H) * cnd[order])


@pytest.mark.parametrize("n", [9, 50])
def test_schur_symmetric_tridiagonal(n):
    T = inputs.symmetric_tridiagonal(n, inputs.rng(inputs.TRIDIAG, n))
    S, Z, wr, wi, info = oracle.schur(T)
    _check_schur(T, S, Z, wr, wi, info)
    assert np.all(wi == 0)
    assert np.linalg.norm(np.triu(S, 1)) <= 50 * n * EPS * np.linalg.norm(T)
    assert np.max(np.abs(np.sort(wr) - np.linalg.eigvalsh(T))) <= 50 * n * EPS * np.linalg.norm(T)


def test_schur_reducible_matches_blocks():
    n, k = 40, 17
    H = inputs.random_hessenberg(n, inputs.rng(96, 0))
    H[k, k - 1] = 0.0
    S, Z, wr, wi, info = oracle.schur(H)
    _check_schur(H, S, Z, wr, wi, info)
    top = oracle.schur(H[:k, :k])
    bot = oracle.schur(H[k:, k:])
    both = np.concatenate([eigs(top[2], top[3]), eigs(bot[2], bot[3])])
    A, B = match_eigenvalues(eigs(wr, wi), both)
    assert np.max(np.abs(A - B)) <= 1e-13 * np.linalg.norm(H)
    # the zero subdiagonal decouples: Z is block diagonal
    assert np.all(Z[k:, :k] == 0) and np.all(Z[:k, k:] == 0)


def test_schur_graded():
    n = 60
    H = inputs.graded_hessenberg(n, inputs.rng(inputs.GRADED, n))
    S, Z, wr, wi, info = oracle.schur(H)
    _check_schur(H, S, Z, wr, wi, info)


def test_schur_iteration_limit_then_resume():
    n = 40
    H = inputs.random_hessenberg(n, inputs.rng(95, 0))
    S, Z, wr, wi, info = oracle.schur(H, maxit=3)
    assert info > 0
    # still a valid similarity: H = Z S Z^T
    assert backward_error(H, S, Z) <= 50 * n * EPS
    S2, Z2, wr2, wi2, info2 = oracle.schur(S, Z)
    _check_schur(H, S2, Z2, wr2, wi2, info2)


def test_schur_rejects_nonfinite():
    H = inputs.random_hessenberg(6, inputs.rng(94, 0))
    H[2, 3] = np.nan
    assert oracle.schur(H)[4] == -2


def test_schur_z_in_composes():
    """Z_out = Z_in Q (eq. 3 then eq. 4): with Z_in = Q1 the result is a Schur
    decomposition of the original A."""
    n = 30
    A = inputs.rng(93, 0).standard_normal((n, n))
    H, Q1 = oracle.hessenberg(A)
    S, Z, wr, wi, info = oracle.schur(H, Q1)
    assert info == 0
    assert backward_error(A, S, Z) <= 50 * n * EPS
    S2, Z2, _, _, _ = oracle.schur(H)
    assert np.linalg.norm(Z - Q1 @ Z2) <= 1e-12 * n


# ---------------------------------------------------------------- condition numbers

def test_cond_matches_lapack_eigenvectors():
    n = 12
    A = inputs.rng(92, 0).standard_normal((n, n))
    H, _ = oracle.hessenberg(A)
    S, Z, wr, wi, info = oracle.schur(H)
    c = oracle.cond(S)
    w, vl, vr = scipy.linalg.eig(A, left=True, right=True)
    cref = np.array([np.linalg.norm(vl[:, i]) * np.linalg.norm(vr[:, i]) / abs(np.vdot(vl[:, i], vr[:, i]))
                     for i in range(n)])
    X, Y = match_eigenvalues(eigs(wr, wi), w)
    order = np.lexsort((np.sign(wi), np.abs(wi), wr))
    # pair the LAPACK cond values through the same matching
    idx = [int(np.argmin(np.abs(w - y))) for y in Y]
    assert np.allclose(c[order], cref[idx], rtol=1e-6)


def test_cond_subset_matches_full():
    T, _ = inputs.prescribed_quasi_triangular(70, inputs.rng(inputs.PRESCRIBED, 770), 0.1)
    full = oracle.cond(T)
    idx = [0, 3, 10, 11, 40, 69]
    assert np.allclose(oracle.cond_subset(T, idx), full[idx], rtol=1e-12)


def test_cond_of_prescribed_matrix_is_cond_of_t():
    """Eigenvalue condition numbers are invariant under orthogonal similarity:
    cond computed on the prescribed T equals cond computed on the oracle's Schur
    form of U T U^T (same eigenvalue, matched)."""
    n = 40
    g = inputs.rng(inputs.PRESCRIBED, 771)
    T, lam = inputs.prescribed_quasi_triangular(n, g, 0.1 / np.sqrt(n))
    U = inputs.haar_orthogonal(n, g)
    A = U @ T @ U.T
    H, _ = oracle.hessenberg(A)
    S, Z, wr, wi, info = oracle.schur(H)
    cs = oracle.cond(S)
    ct = oracle.cond(T)
    lt = np.diag(T) + 1j * np.zeros(n)
    # read T's eigenvalues in its diagonal order
    j = 0
    lt = np.zeros(n, dtype=complex)
    while j < n:
        if j + 1 < n and T[j + 1, j] != 0:
            b = np.sqrt(abs(T[j, j + 1] * T[j + 1, j]))
            lt[j], lt[j + 1] = T[j, j] + 1j * b, T[j, j] - 1j * b
            j += 2
        else:
            lt[j] = T[j, j]
            j += 1
    ls = eigs(wr, wi)
    for k in range(n):
        m = int(np.argmin(np.abs(ls - lt[k])))
        assert abs(cs[m] - ct[k]) <= 1e-6 * ct[k]
