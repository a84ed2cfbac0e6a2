"""Seeded synthetic inputs for the Schur reduction (shared by the tests, the
smoke check and the benchmark).

This module holds none of the method's arithmetic: it only draws random
numbers and assembles matrices of the shapes, distributions and structure the
paper's experiments use (Hessenberg forms of random matrices, Section 5) and of
the well-conditioned families used to pin eigenvalues.  Every generator takes
an explicit ``numpy.random.Generator``; :func:`rng` derives one from
``(family, index)`` so a case is named by two integers.

All matrices are returned as float64 Fortran-ordered (column-major) arrays,
the layout the library and the oracle both use.
"""
from __future__ import annotations

import numpy as np

# family ids used with rng(); fixed so a (family, index) pair names one input
PLAIN = 1        # random N(0,1) upper Hessenberg
PRESCRIBED = 2   # U T U^T with a prescribed quasi-triangular T
FULL = 3         # the large random Hessenberg case
BATCHED = 4      # batch of uneven sizes
LEARNED = 5      # three-family mix
NORMAL = 6       # normal matrices (all eigenvalue condition numbers 1)
TRIDIAG = 7      # symmetric tridiagonal
GRADED = 8       # row-graded random Hessenberg


def rng(family: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(family), int(index)])))


def random_hessenberg(n: int, g: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Entries on and above the subdiagonal i.i.d. N(0, scale^2), zeros below."""
    G = g.standard_normal((n, n)) * scale
    return np.asfortranarray(np.triu(G, -1))


def graded_hessenberg(n: int, g: np.random.Generator) -> np.ndarray:
    """Row grading D G, D = diag(10^(-8 i / n)), G random N(0,1) Hessenberg."""
    G = random_hessenberg(n, g)
    d = 10.0 ** (-8.0 * np.arange(n) / max(n, 1))
    return np.asfortranarray(d[:, None] * G)


def cyclic_shift(n: int) -> np.ndarray:
    """Ones on the subdiagonal and in the top-right corner: the eigenvalues are the
    n-th roots of unity and the matrix is orthogonal."""
    C = np.zeros((n, n), order="F")
    for i in range(1, n):
        C[i, i - 1] = 1.0
    if n > 0:
        C[0, n - 1] = 1.0
    return C


def symmetric_tridiagonal(n: int, g: np.random.Generator) -> np.ndarray:
    d = g.standard_normal(n)
    e = g.standard_normal(max(n - 1, 0))
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    return np.asfortranarray(T)


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of an N(0,1) matrix with the column
    signs fixed by the diagonal of R (library QR, used only to make inputs)."""
    X = g.standard_normal((n, n))
    Q, R = np.linalg.qr(X)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return np.asfortranarray(Q * s[None, :])


def prescribed_quasi_triangular(n: int, g: np.random.Generator, upper_std: float):
    """T with n - 2*floor(n/4) real eigenvalues U[-1,1] and floor(n/4) complex pairs
    uniform in the unit disk (z = sqrt(u) e^{i theta}, theta ~ U[0, pi)) held as
    blocks [[Re z, Im z], [-Im z, Re z]] in shuffled order; entries strictly above
    the diagonal blocks are N(0, upper_std^2).  Returns (T, eigenvalues)."""
    npair = n // 4
    nreal = n - 2 * npair
    reals = g.uniform(-1.0, 1.0, nreal)
    u = g.uniform(0.0, 1.0, npair)
    th = g.uniform(0.0, np.pi, npair)
    z = np.sqrt(u) * np.exp(1j * th)
    kinds = np.array([0] * nreal + [1] * npair)
    g.shuffle(kinds)
    T = np.triu(g.standard_normal((n, n)) * upper_std, 1)
    eig = []
    pos, ir, ic = 0, 0, 0
    for k in kinds:
        if k == 0:
            T[pos, pos] = reals[ir]
            eig.append(complex(reals[ir], 0.0))
            ir += 1
            pos += 1
        else:
            a, b = z[ic].real, z[ic].imag
            T[pos, pos] = a
            T[pos + 1, pos + 1] = a
            T[pos, pos + 1] = b
            T[pos + 1, pos] = -b
            eig.extend([complex(a, b), complex(a, -b)])
            ic += 1
            pos += 2
    return np.asfortranarray(T), np.array(eig)


def prescribed_matrix(n: int, g: np.random.Generator, upper_std: float):
    """A = U T U^T with U Haar and T from :func:`prescribed_quasi_triangular`.
    Returns (A, eigenvalues)."""
    T, eig = prescribed_quasi_triangular(n, g, upper_std)
    U = haar_orthogonal(n, g)
    A = U @ T @ U.T
    return np.asfortranarray(A), eig


def normal_matrix(n: int, g: np.random.Generator):
    """U D U^T with D block diagonal of 1x1 reals and 2x2 rotations-times-radius:
    a normal matrix, so every eigenvalue has condition number 1."""
    T, eig = prescribed_quasi_triangular(n, g, 0.0)
    U = haar_orthogonal(n, g)
    return np.asfortranarray(U @ T @ U.T), eig


def to_hessenberg(A: np.ndarray):
    """Upper Hessenberg form (H, Q1) with A = Q1 H Q1^T via LAPACK (scipy) -- a
    library routine used only to make inputs quickly at large n; the tests pin it
    against the oracle's own Householder reduction at small n."""
    import scipy.linalg

    H, Q = scipy.linalg.hessenberg(np.asarray(A, dtype=np.float64), calc_q=True)
    H = np.triu(H, -1)
    return np.asfortranarray(H), np.asfortranarray(Q)


def batch_sizes(count: int, g: np.random.Generator, lo: int = 32, hi: int = 1024) -> np.ndarray:
    """Problem sizes drawn uniformly from [lo, hi]."""
    return g.integers(lo, hi + 1, size=count)


def prescribed_hessenberg(n: int, g: np.random.Generator, upper_std: float):
    """Hessenberg form of U T U^T (U Haar, T prescribed) without forming U.

    The Hessenberg form of an orthogonal similarity V^T T V is fixed, up to a
    diagonal sign similarity, by the first column of V (implicit-Q uniqueness);
    for Haar U that column is uniform on the unit sphere.  So a Householder
    reflector P with P e1 = w, w uniform, followed by the Hessenberg reduction of
    P T P gives the same distribution as reducing U T U^T, at a third of the
    cost.  Returns (H, eigenvalues)."""
    import scipy.linalg

    T, eig = prescribed_quasi_triangular(n, g, upper_std)
    w = g.standard_normal(n)
    w /= np.linalg.norm(w)
    v = w.copy()
    v[0] -= 1.0  # P = I - 2 v v^T / v^T v maps e1 to w
    vv = float(v @ v)
    if vv > 0.0:
        f = 2.0 / vv
        T = T - f * np.outer(v, v @ T)
        T = T - f * np.outer(T @ v, v)
    H = scipy.linalg.hessenberg(np.asfortranarray(T), calc_q=False, overwrite_a=True)
    return np.asfortranarray(np.triu(H, -1)), eig


def batched_problem(seed: int, i: int, n: int, upper_std: float = 0.1):
    """Problem i of a batch: even i random N(0,1) Hessenberg, odd i a Hessenberg
    matrix with a prescribed spectrum (:func:`prescribed_hessenberg`).  Returns
    (H, eigenvalues or None)."""
    g = rng(BATCHED, 1_000_000 + 10_000 * int(seed) + int(i))
    if i % 2 == 0:
        return random_hessenberg(n, g), None
    return prescribed_hessenberg(n, g, upper_std)


def batched_workload(count: int = 512, seed: int = 0, lo: int = 32, hi: int = 1024, upper_std: float = 0.1,
                     threads: int = 8):
    """The batched workload: ``count`` problems with n uniform in [lo, hi], half
    random and half prescribed-spectrum, made by ``threads`` single-threaded
    workers.  Returns (list of H, list of spectra)."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    sizes = batch_sizes(count, rng(BATCHED, 999_999 - int(seed)), lo, hi)
    with threadpool_limits(limits=1):
        with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            out = list(ex.map(lambda a: batched_problem(seed, a[0], int(a[1]), upper_std), enumerate(sizes)))
    return [h for h, _ in out], [lam for _, lam in out]
