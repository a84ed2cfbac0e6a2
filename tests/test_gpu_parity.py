"""Parity of the HIP path (through the C ABI) with the CPU oracle and with what
mathematics fixes.  Every test needs an MI355X.

Schur forms are not unique (block order, signs), so parity is judged on
invariant quantities: backward error and orthogonality <= 50 n eps, exact
structure of S and of (wr, wi), spectral invariants of the input, and the
eigenvalues matched one to one against the oracle's within
1e-10 ||H|| cond(lambda) (cond from the oracle's own estimate; eigenvalues with
cond >= 1e10 are unpinned and counted, not compared).
"""
import numpy as np
import pytest

import oracle
from checks import (EPS, backward_error, eigs, invariant_errors, match_eigenvalues, orthogonality,
                    structure_violations)
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


def run_gpu(neig, H, Z=None, small=False):
    Hd = to_dev(H)
    Zd = to_dev(np.eye(H.shape[0]) if Z is None else Z)
    fn = neig.small_schur if small else neig.schur
    r = fn(Hd, Zd)
    return to_host(Hd), to_host(r.Z), r.wr.cpu().numpy(), r.wi.cpu().numpy(), r.info


def check_result(H, S, Z, wr, wi, info, tag=""):
    n = H.shape[0]
    assert info == 0, f"{tag}: info={info}"
    be = backward_error(H, S, Z)
    oe = orthogonality(Z)
    assert be <= 50 * n * EPS, f"{tag}: backward error {be:.3e}"
    assert oe <= 50 * n * EPS, f"{tag}: orthogonality {oe:.3e}"
    assert structure_violations(S, wr, wi) == [], tag
    inv = invariant_errors(H, wr, wi)
    assert inv["trace"] <= 50 * np.sqrt(n) * n * EPS, (tag, inv)
    assert inv["trace_sq"] <= 50 * n * n * EPS, (tag, inv)
    return be, oe


def eigen_parity(H, wr, wi, tag=""):
    """Match GPU eigenvalues with the oracle's; compare those with cond < 1e10."""
    S0, Z0, wr0, wi0, info0 = oracle.schur(H)
    assert info0 == 0
    cnd = oracle.cond(S0)
    lo = eigs(wr0, wi0)
    order = np.lexsort((np.sign(wi0), np.abs(wi0), wr0))
    A, B = match_eigenvalues(lo, eigs(wr, wi))
    c = cnd[order]
    nh = np.linalg.norm(H)
    pinned = c * 1e-10 < 1
    err = np.abs(A - B)
    assert np.all(err[pinned] <= 1e-10 * nh * c[pinned]), f"{tag}: max scaled err " \
        f"{np.max(err[pinned] / (nh * c[pinned])):.3e}"
    return float(np.mean(~pinned))


# ---------------------------------------------------------------- in-LDS solver

@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 40, 64, 96])
def test_small_schur_random(neig, n):
    say(f"small_schur n={n}")
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 500 + n))
    S, Z, wr, wi, info = run_gpu(neig, H, small=True)
    check_result(H, S, Z, wr, wi, info, f"small n={n}")
    if n >= 2:
        eigen_parity(H, wr, wi, f"small n={n}")


def test_small_schur_cyclic(neig):
    n = 40
    say(f"small_schur cyclic n={n}")
    H = inputs.cyclic_shift(n)
    S, Z, wr, wi, info = run_gpu(neig, H, small=True)
    check_result(H, S, Z, wr, wi, info, "cyclic")
    roots = np.exp(2j * np.pi * np.arange(n) / n)
    A, B = match_eigenvalues(eigs(wr, wi), roots)
    assert np.max(np.abs(A - B)) <= 1e-12


# ---------------------------------------------------------------- one sweep (implicit-Q theorem)

def oracle_sweep(H, shifts, ilo, ihi):
    """The same sweep as a sequence of double-shift steps (oracle): by the
    implicit-Q theorem both equal Q^T H Q for p(H) = prod (H - s I) = QR."""
    Hc, Zc = H.copy(order="F"), np.eye(H.shape[0], order="F")
    for g in range(len(shifts) // 2):
        a, b = shifts[2 * g], shifts[2 * g + 1]
        tr = (a + b).real
        det = (a * b).real
        Hc, Zc = oracle.francis_step(Hc, Zc, tr, det, ilo, ihi)
    return Hc, Zc


@pytest.mark.parametrize("n,ktop,kbot,nbul,chain,chase_w", [
    (40, 0, 39, 2, 0, 0),       # one chain, one window
    (60, 4, 50, 3, 0, 0),       # interior block: full-width updates outside it
    (150, 0, 149, 6, 2, 16),    # three chains, many small windows
    (200, 0, 199, 8, 4, 40),    # two chains, windows with overlap
    (600, 0, 599, 24, 16, 96),  # the default shape: a full 16-bulge chain and a second one, 96-row windows
    (700, 10, 650, 32, 16, 96),  # two full chains chased concurrently on an interior block
])
def test_sweep_implicit_q(neig, n, ktop, kbot, nbul, chain, chase_w):
    say(f"sweep n={n} [{ktop},{kbot}] bulges={nbul} chain={chain} w={chase_w}")
    g = inputs.rng(90, n)
    H = inputs.random_hessenberg(n, g)
    if ktop > 0:
        H[ktop, ktop - 1] = 0.0
    if kbot + 1 < n:
        H[kbot + 1, kbot] = 0.0
    # shifts far from the spectrum keep p(H) well conditioned
    shifts = []
    for k in range(nbul):
        if k % 2 == 0:
            z = complex(30.0 + 3 * k, 5.0 + k)
            shifts += [z, z.conjugate()]
        else:
            shifts += [complex(-25.0 - k, 0.0), complex(28.0 + k, 0.0)]
    shifts = np.array(shifts)
    neig.set_params(chain=chain, chase_w=chase_w)
    try:
        Hd, Zd = to_dev(H), to_dev(np.eye(n))
        neig.sweep(Hd, Zd, ktop, kbot, shifts.real, shifts.imag)
    finally:
        neig.set_params(chain=0, chase_w=0)
    Hg, Zg = to_host(Hd), to_host(Zd)
    Ho, Zo = oracle_sweep(H, shifts, ktop, kbot)
    assert np.all(np.tril(Hg, -2) == 0)
    assert backward_error(H, Hg, Zg) <= 50 * n * EPS
    assert orthogonality(Zg) <= 50 * n * EPS
    d = np.sign(np.sum(Zo * Zg, axis=0))
    d[d == 0] = 1
    nh = np.linalg.norm(H)
    assert np.linalg.norm(Zg - Zo * d[None, :]) <= 1e-9, np.linalg.norm(Zg - Zo * d[None, :])
    assert np.linalg.norm(Hg - d[:, None] * Ho * d[None, :]) <= 1e-9 * nh


@pytest.mark.parametrize("n,ktop,kbot,nbul,chain,chase_w", [
    (600, 0, 599, 24, 16, 96),
    (700, 10, 650, 32, 16, 96),
    (1500, 0, 1499, 32, 8, 64),   # four chains of 8 in 64-row windows
    (1200, 30, 1100, 40, 4, 40),  # ten chains of 4 on an interior block
    (300, 0, 299, 6, 2, 16),      # many small windows
])
def test_sweep_overlap_matches_one_stream(neig, n, ktop, kbot, nbul, chain, chase_w):
    """The sweep with each step's far updates on the second stream, beside the
    next chase launch, gives the same H and Z, to the bit, as the sweep with
    every update on the call's stream: the same products in the same order."""
    say(f"sweep overlap n={n} [{ktop},{kbot}] bulges={nbul} chain={chain} w={chase_w}")
    H = inputs.random_hessenberg(n, inputs.rng(91, n))
    if ktop > 0:
        H[ktop, ktop - 1] = 0.0
    if kbot + 1 < n:
        H[kbot + 1, kbot] = 0.0
    z = [complex(20.0 + k, 3.0 + 0.5 * k) for k in range(nbul)]
    shifts = np.array([v for c in z for v in (c, c.conjugate())])
    out = {}
    for ov in (2, 1):
        neig.set_params(chain=chain, chase_w=chase_w, overlap=ov)
        try:
            Hd, Zd = to_dev(H), to_dev(np.eye(n))
            neig.sweep(Hd, Zd, ktop, kbot, shifts.real, shifts.imag)
        finally:
            neig.set_params(chain=0, chase_w=0, overlap=0)
        out[ov] = (to_host(Hd), to_host(Zd))
    (H2, Z2), (H1, Z1) = out[2], out[1]
    assert backward_error(H, H1, Z1) <= 50 * n * EPS
    assert orthogonality(Z1) <= 50 * n * EPS
    assert np.array_equal(H1, H2) and np.array_equal(Z1, Z2), (np.abs(H1 - H2).max(), np.abs(Z1 - Z2).max())


# ---------------------------------------------------------------- one AED step

@pytest.mark.parametrize("n,nw", [(120, 40), (200, 96)])
def test_aed_step(neig, n, nw):
    say(f"aed n={n} nw={nw}")
    # a matrix whose bottom part has nearly converged so that AED deflates
    H = inputs.random_hessenberg(n, inputs.rng(91, n))
    H, Z0, _, _, _ = oracle.schur(H, maxit=6)  # a few double-shift steps: still Hessenberg, bottom converging
    H = np.asfortranarray(np.triu(H, -1))
    Hd, Zd = to_dev(H), to_dev(np.eye(n))
    nd, sr, si = neig.aed(Hd, Zd, 0, n - 1, nw)
    Hg, Zg = to_host(Hd), to_host(Zd)
    assert 0 <= nd <= nw
    assert backward_error(H, Hg, Zg) <= 50 * n * EPS
    assert orthogonality(Zg) <= 50 * n * EPS
    assert np.all(np.tril(Hg, -2) == 0)
    kb = n - 1 - nd
    if nd > 0:
        assert Hg[kb + 1, kb] == 0.0
        tail = Hg[kb + 1:, kb + 1:]
        assert np.all(np.tril(tail, -2) == 0)
        sub = np.diag(tail, -1)
        assert not np.any((sub[:-1] != 0) & (sub[1:] != 0))
    # the Ritz values are eigenvalues of the (transformed) window's undeflated part
    assert len(sr) <= nw - nd
    # conjugate pairs adjacent
    for k in range(len(si)):
        if si[k] > 0:
            assert si[k + 1] == -si[k] and sr[k + 1] == sr[k]


# ---------------------------------------------------------------- full solver

@pytest.mark.parametrize("n", [97, 150, 256, 400])
def test_schur_random_hessenberg(neig, n):
    say(f"schur random n={n}")
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, n))
    S, Z, wr, wi, info = run_gpu(neig, H)
    be, oe = check_result(H, S, Z, wr, wi, info, f"random n={n}")
    frac = eigen_parity(H, wr, wi, f"random n={n}")
    say(f"  backward {be:.2e} orth {oe:.2e} unpinned {frac:.2f} stats {neig.get_stats()}")


def test_schur_overlap_sweep_heavy(neig):
    """A sweep-heavy whole reduction (Hessenberg form of a dense uniform[-1,1]
    matrix, 64 shifts in chains of 8, 64-row chase windows) with the sweeps'
    far updates on the second stream: a valid Schur form, and the same one, to
    the bit, as with every update on the call's stream."""
    n = 1500
    say(f"schur overlap, dense uniform n={n}")
    g = inputs.rng(inputs.FULL, 61)
    H, _ = inputs.to_hessenberg(g.uniform(-1.0, 1.0, (n, n)))
    res = {}
    for ov in (2, 1):
        neig.set_params(ns=64, nw=80, chain=8, chase_w=64, overlap=ov)
        try:
            res[ov] = run_gpu(neig, H)
            st = neig.get_stats()
        finally:
            neig.set_params(ns=0, nw=0, chain=0, chase_w=0, overlap=0)
        say(f"  overlap={ov}: sweeps {st['sweeps']} aeds {st['aeds']}")
        assert st["sweeps"] > 0
    S, Z, wr, wi, info = res[1]
    check_result(H, S, Z, wr, wi, info, "overlap")
    for a, b in zip(res[1], res[2]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_schur_plain_n256(neig, seed):
    """The plain 256-order workload: Hessenberg N(0,1), Z from I."""
    say(f"schur plain n=256 seed={seed}")
    H = inputs.random_hessenberg(256, inputs.rng(inputs.PLAIN, seed))
    S, Z, wr, wi, info = run_gpu(neig, H)
    check_result(H, S, Z, wr, wi, info, f"plain seed={seed}")
    eigen_parity(H, wr, wi, f"plain seed={seed}")


@pytest.mark.parametrize("n", [150, 400])
def test_schur_normal_matrix(neig, n):
    say(f"schur normal n={n}")
    A, lam = inputs.normal_matrix(n, inputs.rng(inputs.NORMAL, n))
    H, _ = oracle.hessenberg(A)
    S, Z, wr, wi, info = run_gpu(neig, H)
    check_result(H, S, Z, wr, wi, info, "normal")
    X, Y = match_eigenvalues(eigs(wr, wi), lam)
    assert np.max(np.abs(X - Y)) <= 1e-10 * np.linalg.norm(H)


@pytest.mark.parametrize("n", [300, 600])
def test_schur_prescribed_spectrum(neig, n):
    """U T U^T with a well-conditioned T: eigenvalues equal the prescribed ones
    within 1e-10 ||H|| cond, and Z_in = Q1 gives a Schur form of A."""
    say(f"schur prescribed n={n}")
    A, lam = inputs.prescribed_matrix(n, inputs.rng(inputs.PRESCRIBED, n), 0.1 / np.sqrt(n))
    H, Q1 = inputs.to_hessenberg(A)
    S, Z, wr, wi, info = run_gpu(neig, H, Q1)
    assert info == 0
    assert backward_error(A, S, Z) <= 50 * n * EPS
    assert orthogonality(Z) <= 50 * n * EPS
    assert structure_violations(S, wr, wi) == []
    cnd = oracle.cond(S)
    order = np.lexsort((np.sign(wi), np.abs(wi), wr))
    X, Y = match_eigenvalues(eigs(wr, wi), lam)
    assert np.all(np.abs(X - Y) <= 1e-10 * np.linalg.norm(H) * cnd[order])


def test_schur_cyclic_shift(neig):
    n = 200
    say(f"schur cyclic n={n}")
    H = inputs.cyclic_shift(n)
    S, Z, wr, wi, info = run_gpu(neig, H)
    check_result(H, S, Z, wr, wi, info, "cyclic")
    roots = np.exp(2j * np.pi * np.arange(n) / n)
    A, B = match_eigenvalues(eigs(wr, wi), roots)
    assert np.max(np.abs(A - B)) <= 1e-10


def test_schur_symmetric_tridiagonal(neig):
    n = 300
    say(f"schur tridiagonal n={n}")
    T = inputs.symmetric_tridiagonal(n, inputs.rng(inputs.TRIDIAG, n))
    S, Z, wr, wi, info = run_gpu(neig, T)
    check_result(T, S, Z, wr, wi, info, "tridiag")
    assert np.all(wi == 0)
    assert np.max(np.abs(np.sort(wr) - np.linalg.eigvalsh(T))) <= 50 * n * EPS * np.linalg.norm(T)


def test_schur_graded(neig):
    n = 300
    say(f"schur graded n={n}")
    H = inputs.graded_hessenberg(n, inputs.rng(inputs.GRADED, n))
    S, Z, wr, wi, info = run_gpu(neig, H)
    check_result(H, S, Z, wr, wi, info, "graded")


def test_schur_triangular_and_reducible(neig):
    n = 200
    say("schur triangular / reducible")
    g = inputs.rng(97, 1)
    T = np.asfortranarray(np.triu(g.standard_normal((n, n))))
    S, Z, wr, wi, info = run_gpu(neig, T)
    assert info == 0 and np.array_equal(S, T) and np.array_equal(Z, np.eye(n))
    assert np.array_equal(wr, np.diag(T)) and np.all(wi == 0)
    H = inputs.random_hessenberg(n, inputs.rng(96, 1))
    H[120, 119] = 0.0
    S, Z, wr, wi, info = run_gpu(neig, H)
    check_result(H, S, Z, wr, wi, info, "reducible")
    assert np.all(Z[120:, :120] == 0) and np.all(Z[:120, 120:] == 0)


def test_edge_sizes_and_errors(neig):
    import torch

    say("edge sizes")
    for n in (0, 1, 2):
        H = inputs.random_hessenberg(n, inputs.rng(95, n)) if n else np.zeros((0, 0))
        Hd = to_dev(H) if n else torch.zeros((0, 0), dtype=torch.float64, device="cuda")
        r = neig.schur(Hd)
        assert r.info == 0
        if n:
            check_result(H, to_host(Hd), to_host(r.Z), r.wr.cpu().numpy(), r.wi.cpu().numpy(), r.info)
    H = inputs.random_hessenberg(50, inputs.rng(95, 50))
    H[3, 7] = np.nan
    with pytest.raises(neig.NeigError):
        neig.schur(to_dev(H))


def test_deterministic(neig):
    n = 300
    say("determinism")
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 77))
    a = run_gpu(neig, H)
    b = run_gpu(neig, H)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_iteration_limit_then_resume(neig):
    n = 300
    say("maxit / resume")
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 78))
    neig.set_params(maxit=2)
    try:
        S, Z, wr, wi, info = run_gpu(neig, H)
    finally:
        neig.set_params(maxit=0)
    assert info > 0
    assert backward_error(H, S, Z) <= 50 * n * EPS
    S2, Z2, wr2, wi2, info2 = run_gpu(neig, S, Z)
    check_result(H, S2, Z2, wr2, wi2, info2, "resumed")


def test_norm_stable_criterion(neig):
    n = 256
    say("norm-stable deflation")
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 79))
    neig.set_params(deflation=1)
    try:
        S, Z, wr, wi, info = run_gpu(neig, H)
    finally:
        neig.set_params(deflation=0)
    check_result(H, S, Z, wr, wi, info, "normstable")
