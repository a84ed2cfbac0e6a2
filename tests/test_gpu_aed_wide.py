"""AED windows larger than one workgroup's LDS (Section 3.2: the window's Schur
form by a recursive application of the QR algorithm), through the C ABI:
one AED step on windows of 128..384 rows with the off-diagonal updates
checked by the similarity they must preserve; windows whose deflation count is
fixed by construction; and whole reductions run with wide windows."""
import numpy as np
import pytest

from checks import EPS, backward_error, eigs, invariant_errors, match_eigenvalues, orthogonality, structure_violations
from gpu_util import say, to_dev, to_host
from paper_2002_05024_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def neig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_05024_amd import binding

    binding.load_library()
    saved = binding.get_params()
    yield binding
    binding.set_params(**saved)


def check_aed_result(H, Hg, Zg, nd, nw, kbot):
    n = H.shape[0]
    assert 0 <= nd <= nw
    assert backward_error(H, Hg, Zg) <= 50 * n * EPS
    assert orthogonality(Zg) <= 50 * n * EPS
    assert np.all(np.tril(Hg, -2) == 0)
    kb = kbot - nd
    if nd > 0:
        assert Hg[kb + 1, kb] == 0.0
        tail = Hg[kb + 1:kbot + 1, kb + 1:kbot + 1]
        sub = np.diag(tail, -1)
        assert not np.any((sub[:-1] != 0) & (sub[1:] != 0))  # quasi-triangular


@pytest.mark.parametrize("nw", [128, 192, 384])
def test_aed_wide_step_interior_block(neig, nw):
    """An AED step on an active block strictly inside H, so that every update
    (rows above the window, columns right of it, all of Z) is exercised."""
    n, ktop, kbot = 900, 37, 900 - 1 - 100
    say(f"aed wide n={n} nw={nw} ktop={ktop} kbot={kbot}")
    H = inputs.random_hessenberg(n, inputs.rng(92, nw))
    H[ktop, ktop - 1] = 0.0
    H[kbot + 1, kbot] = 0.0
    Hd, Zd = to_dev(H), to_dev(np.eye(n))
    nd, sr, si = neig.aed(Hd, Zd, ktop, kbot, nw)
    Hg, Zg = to_host(Hd), to_host(Zd)
    say(f"  nd={nd} ritz={len(sr)} stats rec_aeds={neig.get_stats()['rec_aeds']}")
    check_aed_result(H, Hg, Zg, nd, nw, kbot)
    assert nd > 0  # a random Hessenberg window of this size always deflates some
    assert len(sr) <= nw - nd
    for k in range(len(si)):
        if si[k] > 0:
            assert si[k + 1] == -si[k] and sr[k + 1] == sr[k]
    # untouched outside the similarity: rows below kbot left of the window stay zero
    assert np.all(Hg[kbot + 1:, :kbot + 1] == 0.0)


def constructed(n, nw, k, beta, seed, pairs):
    """H whose trailing nw x nw window is [[A, B], [0, T2]], coupled to the rest
    only through H(kwtop, kwtop-1) = beta.  A (k x k) is the symmetric
    tridiagonal matrix with zero diagonal and unit off-diagonal: its eigenvalues
    2 cos(pi j / (k+1)) are distinct and its eigenvectors are sine vectors, so
    every first component is at least about 0.03.  T2 is upper quasi-triangular
    in standard form with eigenvalues from 3 up (`pairs` 2x2 blocks).  The window
    QR changes only A's rows and columns, so the spike is beta times the first
    row of A's Schur factor: T2's blocks have spike exactly 0 and always deflate;
    A's fail for beta = 1 and deflate for beta = 1e-30."""
    g = np.random.default_rng(seed)
    H = np.triu(g.standard_normal((n, n)), -1)
    kw = n - nw
    H[kw, kw - 1] = beta
    A = np.diag(np.ones(k - 1), 1) + np.diag(np.ones(k - 1), -1)
    m2 = nw - k
    T2 = np.triu(g.standard_normal((m2, m2)) * 0.3, 1)
    np.fill_diagonal(T2, 3.0 + np.arange(m2) * 0.25)
    for p in range(pairs):  # standardised 2x2 blocks [[a, b], [c, a]], b c < 0
        j = 2 + 4 * p
        T2[j, j + 1] = 1.5
        T2[j + 1, j] = -0.5 - 0.1 * p
        T2[j + 1, j + 1] = T2[j, j]
    W = np.zeros((nw, nw))
    W[:k, :k] = A
    W[:k, k:] = g.standard_normal((k, m2))
    W[k:, k:] = T2
    H[kw:, kw:] = W
    return np.asfortranarray(H)


@pytest.mark.parametrize("nw", [64, 160, 384])
@pytest.mark.parametrize("beta,pairs", [(1.0, 0), (1.0, 3), (1e-30, 2)])
def test_aed_deflation_count_is_determinate(neig, nw, beta, pairs):
    n, k = 700, 24
    say(f"aed determinate nw={nw} beta={beta} pairs={pairs}")
    H = constructed(n, nw, k, beta, 11 + nw, pairs)
    Hd, Zd = to_dev(H), to_dev(np.eye(n))
    nd, sr, si = neig.aed(Hd, Zd, 0, n - 1, nw)
    Hg, Zg = to_host(Hd), to_host(Zd)
    check_aed_result(H, Hg, Zg, nd, nw, n - 1)
    expect = nw if beta < 1e-20 else nw - k
    assert nd == expect, (nd, expect)
    # the deflated part carries T2's eigenvalues (and A's when all deflate)
    tail = Hg[n - nd:, n - nd:]
    got = np.sort_complex(np.linalg.eigvals(tail))
    want = np.sort_complex(np.linalg.eigvals(H[n - nd:, n - nd:] if beta >= 1e-20 else H[n - nw:, n - nw:]))
    X, Y = match_eigenvalues(got, want)
    assert np.max(np.abs(X - Y)) <= 1e-10 * np.linalg.norm(H)


@pytest.mark.parametrize("nw,ns", [(192, 64), (384, 128)])
def test_schur_with_wide_windows(neig, nw, ns):
    """Whole reductions with every AED window wide (recursive window solves) and
    many shifts per sweep: random N(0,1) Hessenberg (n = 1000, checked by its
    spectral invariants) and a prescribed spectrum (n = 1200, eigenvalues
    against the prescribed ones)."""
    neig.set_params(nw=nw, ns=ns)
    try:
        n = 1000
        say(f"schur wide nw={nw} ns={ns} random n={n}")
        H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 500 + nw))
        Hd = to_dev(H)
        r = neig.schur(Hd)
        st = neig.get_stats()
        say(f"  info={r.info} aeds={st['aeds']} rec={st['rec_aeds']} sweeps={st['sweeps']}")
        assert r.info == 0
        assert st["rec_aeds"] > 0
        S, Z = to_host(Hd), to_host(r.Z)
        wr, wi = r.wr.cpu().numpy(), r.wi.cpu().numpy()
        assert backward_error(H, S, Z) <= 50 * n * EPS
        assert orthogonality(Z) <= 50 * n * EPS
        assert structure_violations(S, wr, wi) == []
        # random Hessenberg eigenvalues of this order are far too ill-conditioned
        # to compare one by one (the oracle's condition estimates all exceed
        # 1e10); the spectral invariants pin them as a whole
        inv = invariant_errors(H, wr, wi)
        assert inv["trace"] <= 50 * np.sqrt(n) * n * EPS, inv
        assert inv["trace_sq"] <= 50 * n * n * EPS, inv

        n = 1200
        say(f"schur wide nw={nw} ns={ns} prescribed n={n}")
        A, lam_p = inputs.prescribed_matrix(n, inputs.rng(inputs.PRESCRIBED, 77), 0.1 / np.sqrt(n))
        H, _ = inputs.to_hessenberg(A)
        Hd = to_dev(H)
        r = neig.schur(Hd)
        assert r.info == 0
        S, Z = to_host(Hd), to_host(r.Z)
        wr, wi = r.wr.cpu().numpy(), r.wi.cpu().numpy()
        assert backward_error(H, S, Z) <= 50 * n * EPS
        assert orthogonality(Z) <= 50 * n * EPS
        assert structure_violations(S, wr, wi) == []
        X, Y = match_eigenvalues(eigs(wr, wi), lam_p)
        assert np.max(np.abs(X - Y)) <= 1e-8 * np.linalg.norm(H)
    finally:
        neig.set_params(nw=0, ns=0)
