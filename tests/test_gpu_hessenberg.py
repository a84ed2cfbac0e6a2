"""Hessenberg reduction through the C ABI against the oracle's unblocked
Householder reduction: the same reflector convention makes H and Q1 unique
(implicit-Q theorem with Q1 e1 = e1), so they are compared element by element
at sizes that span several panels, row blocks and GEMV chunks with ragged
tails; degenerate inputs (already Hessenberg, zero columns, n <= 2); a given
Q_in; and the full-size prescribed-spectrum matrix through the whole pipeline
A -> H -> S checked by backward error and orthogonality.

Tolerances: both sides are backward stable (backward error and orthogonality
within 50 n eps, checked first); for these Gaussian inputs the subdiagonal
entries are far from zero, so H and Q1 move by a modest multiple of n eps under
that backward error: elementwise H within 10 n eps ||A||_F, Q1 within 50 n eps.
A reordered-summation model of the blocked algorithm in numpy differs from the
oracle by up to 1.0 and 2.7 of those units."""
import numpy as np
import pytest

import oracle
from checks import EPS, backward_error, eigs, match_eigenvalues, orthogonality, structure_violations, t_eigs_in_order
from gpu_util import gpu_backward_error, gpu_orthogonality, say, to_dev, to_host
from paper_2002_05024_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def neig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_05024_amd import binding

    binding.load_library()
    return binding


def gpu_reduce(neig, A, Q=None):
    Ad = to_dev(A)
    Qd = neig.hessenberg(Ad, None if Q is None else to_dev(Q))
    return to_host(Ad), to_host(Qd)


@pytest.mark.parametrize("n", [3, 4, 5, 17, 64, 65, 66, 67, 129, 200, 333, 600])
def test_hessenberg_matches_oracle(neig, n):
    A = inputs.rng(97, n).standard_normal((n, n))
    say(f"hessenberg n={n}")
    H1, Q1 = gpu_reduce(neig, A)
    H0, Q0 = oracle.hessenberg(A)
    assert np.all(np.tril(H1, -2) == 0.0)
    be, oe = backward_error(A, H1, Q1), orthogonality(Q1)
    na = np.linalg.norm(A)
    dh = np.abs(H1 - H0).max() / (n * EPS * na)
    dq = np.abs(Q1 - Q0).max() / (n * EPS)
    say(f"  backward {be / (n * EPS):.3f} n eps, orth {oe / (n * EPS):.3f} n eps, "
        f"|dH| {dh:.3f} n eps ||A||, |dQ| {dq:.3f} n eps")
    assert be <= 50 * n * EPS and oe <= 50 * n * EPS
    assert dh <= 10.0 and dq <= 50.0


def test_hessenberg_ragged_large_matches_oracle(neig):
    """n = 1100: several 256-row workgroups in the column kernels, several
    512-row GEMV blocks, 17 panels with a ragged last one."""
    n = 1100
    A = inputs.rng(97, n).standard_normal((n, n))
    H1, Q1 = gpu_reduce(neig, A)
    H0, Q0 = oracle.hessenberg(A)
    dh = np.abs(H1 - H0).max() / (n * EPS * np.linalg.norm(A))
    dq = np.abs(Q1 - Q0).max() / (n * EPS)
    say(f"  n={n} |dH| {dh:.3f} n eps ||A||, |dQ| {dq:.3f} n eps")
    assert dh <= 10.0 and dq <= 50.0


def test_hessenberg_wide_chunk_path(neig):
    """n = 8704: trailing blocks of more than 8192 rows take the wide-chunk
    matrix-vector path (the one the n = 20000 benchmark runs); checked by
    backward error, orthogonality and exact zeros, with FP64 products on the
    GPU (the oracle would take minutes here)."""
    import torch

    n = 8704
    g = inputs.rng(95, n)
    A0 = torch.from_numpy(g.standard_normal((n, n))).cuda().t()  # column-major view
    A = A0.clone(memory_format=torch.preserve_format)
    Q = torch.eye(n, dtype=torch.float64, device="cuda").t()
    say(f"hessenberg n={n} (wide chunks)")
    neig.hessenberg(A, Q)
    torch.cuda.synchronize()
    assert float(torch.tril(A, -2).abs().max()) == 0.0
    # A0 = Q H Q^T: the backward error of the similarity with S := H
    be = gpu_backward_error(A0, A, Q)
    oe = gpu_orthogonality(Q)
    say(f"  backward {be:.2e} orth {oe:.2e}")
    assert be <= 50 * n * EPS and oe <= 50 * n * EPS


@pytest.mark.parametrize("n", [0, 1, 2])
def test_hessenberg_trivial_sizes(neig, n):
    A = inputs.rng(96, n).standard_normal((n, n))
    H1, Q1 = gpu_reduce(neig, A)
    assert np.array_equal(H1, A) and np.array_equal(Q1, np.eye(n))


def test_hessenberg_input_already_hessenberg_is_untouched(neig):
    """Every reflector is the identity (tau = 0): H = A and Q1 = I exactly."""
    n = 150
    A = np.triu(inputs.rng(95, n).standard_normal((n, n)), -1)
    H1, Q1 = gpu_reduce(neig, A)
    assert np.array_equal(H1, A) and np.array_equal(Q1, np.eye(n))


def test_hessenberg_zero_columns(neig):
    """Columns whose part below the subdiagonal is zero (tau = 0 in the middle
    of a panel) next to ordinary ones."""
    n = 140
    A = inputs.rng(94, n).standard_normal((n, n))
    for j in (0, 5, 6, 63, 64, 100):
        A[j + 2:, j] = 0.0
    H1, Q1 = gpu_reduce(neig, A)
    H0, Q0 = oracle.hessenberg(A)
    assert np.abs(H1 - H0).max() <= 10 * n * EPS * np.linalg.norm(A)
    assert np.abs(Q1 - Q0).max() <= 50 * n * EPS


def test_hessenberg_without_q_and_with_q_in(neig):
    n = 230
    A = inputs.rng(93, n).standard_normal((n, n))
    H1, Q1 = gpu_reduce(neig, A)
    Ad = to_dev(A)
    assert neig.hessenberg(Ad, accumulate=False) is None
    assert np.array_equal(to_host(Ad), H1)  # the same kernels, the same H
    Qin, _ = np.linalg.qr(inputs.rng(92, n).standard_normal((n, n)))
    H2, Q2 = gpu_reduce(neig, A, Qin)
    assert np.array_equal(H2, H1)
    assert np.abs(Q2 - Qin @ Q1).max() <= 50 * n * EPS


def test_pipeline_prescribed_n4000(neig):
    """The prescribed-spectrum workload from its dense form: GPU Hessenberg
    reduction, then the Schur reduction with Z = Q1; ||A - Z S Z^T|| and the
    orthogonality of Z within 50 n eps; the eigenvalues are the prescribed ones
    (well-conditioned variant, strictly upper part 0.1/sqrt(n))."""
    import torch

    n = 4000
    g = inputs.rng(inputs.PRESCRIBED, 4200)
    T, lam = inputs.prescribed_quasi_triangular(n, g, 0.1 / np.sqrt(n))
    U = inputs.haar_orthogonal(n, g)
    A = np.asfortranarray(U @ T @ U.T)  # the construction of inputs.prescribed_matrix, T kept
    Ad = to_dev(A)
    A0 = Ad.clone()
    say(f"pipeline n={n}")
    Qd = neig.hessenberg(Ad)
    be, oe = gpu_backward_error(A0, Ad, Qd), gpu_orthogonality(Qd)
    say(f"  hessenberg backward {be / (n * EPS):.3f} n eps, orth {oe / (n * EPS):.3f} n eps")
    assert be <= 50 * n * EPS and oe <= 50 * n * EPS
    assert float(torch.tril(Ad, -2).abs().max()) == 0.0
    r = neig.schur(Ad, Qd)
    assert r.info == 0
    be, oe = gpu_backward_error(A0, Ad, r.Z), gpu_orthogonality(r.Z)
    say(f"  A -> S backward {be / (n * EPS):.3f} n eps, orth {oe / (n * EPS):.3f} n eps")
    assert be <= 50 * n * EPS and oe <= 50 * n * EPS
    S = to_host(Ad)
    assert structure_violations(S, r.wr.cpu().numpy(), r.wi.cpu().numpy()) == []
    # eigenvalues against the prescribed ones within 1e-10 ||A||_F cond(lambda);
    # the condition numbers come from the prescribed T (an input), computed one
    # by one for the eigenvalues that are not already within 1e-12 ||A||_F
    lt = t_eigs_in_order(T)
    X, Y = match_eigenvalues(lt, eigs(r.wr.cpu().numpy(), r.wi.cpu().numpy()))
    na = np.linalg.norm(A)
    err = np.abs(X - Y)
    loose = np.nonzero(err > 1e-12 * na)[0]
    if loose.size:
        pos = np.array([int(np.argmin(np.abs(lt - X[k]))) for k in loose])
        cond = oracle.cond_subset(T, pos)
        say(f"  {loose.size} eigenvalues beyond 1e-12 ||A||: worst err/(||A|| cond) "
            f"{np.max(err[loose] / (na * cond)):.2e}")
        assert np.all(err[loose] <= 1e-10 * na * cond)


def test_hessenberg_padded_leading_dimensions(neig):
    """lda, ldq > n: the padding rows are neither read into the result nor written."""
    import torch

    n, pad = 150, 7
    A = inputs.rng(91, n).standard_normal((n, n))
    H1, Q1 = gpu_reduce(neig, A)
    Ab = torch.full((n, n + pad), 7.5, dtype=torch.float64, device="cuda")
    Qb = torch.full((n, n + pad), -3.25, dtype=torch.float64, device="cuda")
    Ad = Ab.t()[:n, :]  # column-major n x n view, leading dimension n + pad
    Qd = Qb.t()[:n, :]
    Ad.copy_(torch.from_numpy(A).cuda())
    Qd.copy_(torch.eye(n, dtype=torch.float64, device="cuda"))
    assert Ad.stride() == (1, n + pad)
    neig.hessenberg(Ad, Qd)
    assert np.array_equal(to_host(Ad), H1) and np.array_equal(to_host(Qd), Q1)
    assert bool((Ab.t()[n:, :] == 7.5).all()) and bool((Qb.t()[n:, :] == -3.25).all())
