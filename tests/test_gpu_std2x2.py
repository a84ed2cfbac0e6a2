"""The GPU's 2x2 standardisation (the finish step of a real Schur form, Section 2,
eq. 4) on the same 413 blocks that pin the oracle's, through the C ABI.

An order-2 problem goes through the in-LDS QR kernel, whose only work on an
unreduced 2x2 block is the standardising rotation (and, for the batched call,
through the persistent solver's own finish step).  Each result is checked
against what the mathematics fixes and against the oracle's closed form:
orthogonal Z, H = Z S Z^T to a few eps, the standard form (upper triangular
for a real pair; equal diagonal and opposite off-diagonal signs for a complex
pair) with (wr, wi) read off bit for bit, trace and determinant, the roots of
the characteristic polynomial when they are well separated, and the oracle's
eigenvalues.  The one exception is a coupling entry below the device's absolute
negligibility floor DBL_MIN * n / eps (the 1e-300 block), which the kernel
treats as zero: its residual is bounded by that floor instead.
"""
import numpy as np
import pytest

import oracle
from checks import EPS, std2x2_cases, structure_violations
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

DBL_MIN = np.finfo(np.float64).tiny
SMLNUM = DBL_MIN * (2 / EPS)


@pytest.fixture(scope="module")
def neig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_05024_amd import binding

    binding.load_library()
    return binding


def check_block(blk, S, Z, wr, wi, tag):
    a, b, c, d = blk
    B = np.array([[a, b], [c, d]], dtype=np.float64)
    nb = np.linalg.norm(B)
    assert np.linalg.norm(Z.T @ Z - np.eye(2)) <= 8 * EPS, tag
    assert np.linalg.norm(B - Z @ S @ Z.T) <= 16 * EPS * nb + SMLNUM, tag
    assert structure_violations(S, wr, wi) == [], tag
    lam = wr + 1j * wi
    assert abs(lam.sum() - (a + d)) <= 16 * EPS * nb + 2 * SMLNUM, tag
    assert abs(lam.prod() - (a * d - b * c)) <= 32 * EPS * nb * nb + SMLNUM * nb, tag
    disc = (a - d) ** 2 + 4 * b * c
    separated = abs(disc) > 1e-6 * nb * nb and nb > 1e-100
    if separated:
        roots = np.roots([1.0, -(a + d), a * d - b * c])
        got = np.sort_complex(lam)
        ref = np.sort_complex(roots)
        assert np.max(np.abs(got - ref)) <= 1e-9 * nb, (tag, got, ref)
    # the oracle's closed form: same eigenvalues (a nearly defective pair is only
    # determined to about sqrt(eps) |B|)
    _, _, _, (r1, i1, r2, i2) = oracle.std2x2(a, b, c, d)
    ref = np.sort_complex(np.array([complex(r1, i1), complex(r2, i2)]))
    tol = 1e-9 * nb if separated else 4e-8 * nb + SMLNUM
    assert np.max(np.abs(np.sort_complex(lam) - ref)) <= tol, (tag, lam, ref)


def test_std2x2_small_schur(neig):
    cases = std2x2_cases()
    for k, blk in enumerate(cases):
        H = np.array([[blk[0], blk[1]], [blk[2], blk[3]]], dtype=np.float64)
        Hd = to_dev(H)
        r = neig.small_schur(Hd, to_dev(np.eye(2)))
        assert r.info == 0, (k, blk)
        check_block(blk, to_host(Hd), to_host(r.Z), r.wr.cpu().numpy(), r.wi.cpu().numpy(), (k, blk))


def test_std2x2_batched(neig):
    import torch

    cases = std2x2_cases()
    Hs = [np.array([[a, b], [c, d]], dtype=np.float64) for (a, b, c, d) in cases]
    call = neig.schur_batched([to_dev(H) for H in Hs])
    torch.cuda.synchronize()
    info = call.info.cpu().numpy()
    for k, blk in enumerate(cases):
        assert info[k] == 0, (k, blk)
        check_block(blk, to_host(call.Hs[k]), to_host(call.Zs[k]), call.wrs[k].cpu().numpy(),
                    call.wis[k].cpu().numpy(), (k, blk))
