"""Eigenvalue reordering through the C ABI against the oracle: the reordered
form is a valid Schur decomposition of the same matrix, the selected
eigenvalues lead in their order, and the leading invariant subspace equals the
oracle's; trivial selections; a full-size case checked by its properties."""
import numpy as np
import pytest

import oracle
from checks import EPS, backward_error, eigs, orthogonality, structure_violations
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


def schur_case(n, seed, family="random"):
    g = inputs.rng(inputs.NORMAL, 900 + seed)
    if family == "random":
        H = inputs.random_hessenberg(n, g)
    else:
        H, _ = inputs.prescribed_hessenberg(n, g, 0.1 / np.sqrt(n))
    S, Z, wr, wi, info = oracle.schur(H)
    assert info == 0
    return H, S, Z


def run_gpu(neig, S, Z, sel):
    Sd, Zd = to_dev(S), to_dev(Z)
    wr, wi, m, info = neig.reorder(Sd, Zd, sel)
    return to_host(Sd), to_host(Zd), wr.cpu().numpy(), wi.cpu().numpy(), m, info


@pytest.mark.parametrize("n,seed,frac,family", [(30, 0, 0.3, "prescribed"), (80, 1, 0.5, "prescribed"),
                                               (150, 2, 0.2, "prescribed"), (257, 3, 0.5, "prescribed"),
                                               (400, 4, 0.1, "prescribed"), (120, 5, 0.5, "random")])
def test_reorder_matches_oracle(neig, n, seed, frac, family):
    """Prescribed (well-conditioned) spectra pin the subspace; the random family
    (ill-conditioned eigenvalues) is checked for validity and order."""
    H, S, Z = schur_case(n, seed, family)
    sel = (np.random.default_rng(seed).random(n) < frac).astype(np.int32)
    S1, Z1, wr1, wi1, m1, info1 = run_gpu(neig, S, Z, sel)
    S0, Z0, wr0, wi0, m0, info0 = oracle.reorder(S, Z, sel)
    say(f"n={n} selected {m1} (oracle {m0})")
    assert info1 == 0 and info0 == 0 and m1 == m0
    assert backward_error(H, S1, Z1) <= 50 * n * EPS
    assert orthogonality(Z1) <= 50 * n * EPS
    assert structure_violations(S1, wr1, wi1) == []
    cond = oracle.cond(S0)
    l1, l0 = eigs(wr1, wi1), eigs(wr0, wi0)
    scale = np.linalg.norm(H)
    # the leading eigenvalues, in order, where the condition number pins them
    pinned = cond[:m0] * 1e-10 < 1
    assert np.all(np.abs(l1[:m0] - l0[:m0])[pinned] <= 1e-10 * scale * cond[:m0][pinned])
    # the same leading invariant subspace: Z1[:, :m] is orthogonal to Z0[:, m:]
    if 0 < m0 < n and family == "prescribed":
        gap = np.linalg.norm(Z1[:, :m0].T @ Z0[:, m0:])
        say(f"  subspace gap {gap:.2e}")
        assert gap < 1e-7


def test_reorder_trivial_and_bottom_to_top(neig):
    n = 200  # several windows
    H, S, Z = schur_case(n, 7)
    for sel in (np.zeros(n, np.int32), np.ones(n, np.int32)):
        S1, Z1, wr1, wi1, m1, info = run_gpu(neig, S, Z, sel)
        assert info == 0 and m1 == (0 if sel[0] == 0 else n)
        assert np.array_equal(S1, S) and np.array_equal(Z1, Z)
    sel = np.zeros(n, np.int32)
    sel[n - 1] = 1  # the bottom eigenvalue (or pair) to the top, across all windows
    S1, Z1, wr1, wi1, m1, info = run_gpu(neig, S, Z, sel)
    S0, Z0, wr0, wi0, m0, info0 = oracle.reorder(S, Z, sel)
    assert info == 0 and m1 == m0
    assert np.allclose(eigs(wr1, wi1)[:m1], eigs(wr0, wi0)[:m0], rtol=1e-9, atol=1e-12)
    assert backward_error(H, S1, Z1) <= 50 * n * EPS


def test_reorder_full_size_prescribed_n4000(neig):
    """Config-2 size: every eigenvalue with negative real part selected; checked
    by its properties (GPU products) and the spectrum of the leading block."""
    n = 4000
    say(f"reorder n={n}")
    g = inputs.rng(inputs.PRESCRIBED, 4100)
    H, _ = inputs.prescribed_hessenberg(n, g, 0.1 / np.sqrt(n))
    Hd = to_dev(H)
    r = neig.schur(Hd)
    assert r.info == 0
    wr = r.wr.cpu().numpy()
    sel = (wr < 0).astype(np.int32)
    Zd = r.Z
    wr2, wi2, m, info = neig.reorder(Hd, Zd, sel)
    assert info == 0
    H0 = to_dev(H)
    be, oe = gpu_backward_error(H0, Hd, Zd), gpu_orthogonality(Zd)
    say(f"  m={m} backward {be:.2e} orth {oe:.2e}")
    assert be <= 50 * n * EPS and oe <= 50 * n * EPS
    S1 = to_host(Hd)
    wr2, wi2 = wr2.cpu().numpy(), wi2.cpu().numpy()
    assert structure_violations(S1, wr2, wi2) == []
    assert m == int(sel.sum())
    assert np.all(wr2[:m] < 0) and np.all(wr2[m:] >= 0)
    # the multiset of eigenvalues is unchanged (well-conditioned spectrum)
    assert np.allclose(np.sort_complex(eigs(wr2, wi2)), np.sort_complex(eigs(wr, r.wi.cpu().numpy())), atol=1e-9)
