"""Batched Schur reduction (one persistent launch over many problems of uneven
order), through the C ABI: per-problem parity with the oracle and with
prescribed spectra, agreement with the single-problem path, and HIP-graph
capture and replay."""
import numpy as np
import pytest

import oracle
from checks import EPS, backward_error, eigs, match_eigenvalues, orthogonality, structure_violations
from gpu_util import say, to_dev, to_host
from paper_2002_05024_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def neig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_05024_amd import binding

    binding.load_library()
    return binding


def make_batch(sizes, seed):
    """Even entries: random N(0,1) Hessenberg; odd entries: prescribed spectrum
    with a well-conditioned T (std 0.1/sqrt(n)), reduced to Hessenberg form."""
    Hs, spectra = [], []
    for i, n in enumerate(sizes):
        g = inputs.rng(inputs.BATCHED, seed * 1000 + i)
        if i % 2 == 0:
            Hs.append(inputs.random_hessenberg(n, g))
            spectra.append(None)
        else:
            A, lam = inputs.prescribed_matrix(n, g, 0.1 / np.sqrt(n))
            H, _ = inputs.to_hessenberg(A)
            Hs.append(H)
            spectra.append(lam)
    return Hs, spectra


def run_batched(neig, Hs):
    import torch

    c = neig.schur_batched([to_dev(H) for H in Hs])
    torch.cuda.synchronize()
    return c.Hs, c.wrs, c.wis, c.Zs, c.info.cpu().numpy()


def check_problem(H, S, Z, wr, wi, lam, tag):
    n = H.shape[0]
    assert backward_error(H, S, Z) <= 50 * n * EPS, tag
    assert orthogonality(Z) <= 50 * n * EPS, tag
    assert structure_violations(S, wr, wi) == [], tag
    if lam is not None:  # prescribed spectrum: cond of the prescribed eigenvalues ~ 1
        X, Y = match_eigenvalues(eigs(wr, wi), lam)
        assert np.max(np.abs(X - Y)) <= 1e-8 * np.linalg.norm(H), tag
    elif n <= 300:
        S0, Z0, wr0, wi0, info0 = oracle.schur(H)
        cnd = oracle.cond(S0)
        order = np.lexsort((np.sign(wi0), np.abs(wi0), wr0))
        A, B = match_eigenvalues(eigs(wr0, wi0), eigs(wr, wi))
        c = cnd[order]
        pinned = c * 1e-10 < 1
        assert np.all(np.abs(A - B)[pinned] <= 1e-10 * np.linalg.norm(H) * c[pinned]), tag


def test_batched_mixed_sizes(neig):
    sizes = [32, 33, 64, 96, 97, 120, 150, 200, 257, 300, 400, 511, 600, 777, 1024, 45, 2, 1, 5, 90]
    say(f"batched sizes={sizes}")
    Hs, spectra = make_batch(sizes, 1)
    Hd, wrs, wis, Zs, info = run_batched(neig, Hs)
    assert np.all(info == 0), info
    for i, H in enumerate(Hs):
        check_problem(H, to_host(Hd[i]), to_host(Zs[i]), wrs[i].cpu().numpy(), wis[i].cpu().numpy(), spectra[i],
                      f"problem {i} n={H.shape[0]}")


def test_batched_matches_properties_of_single_path(neig):
    """Same inputs through neig_schur one by one and through the batched call:
    both are valid Schur forms with the same spectrum (not bitwise: different
    control parameters)."""
    sizes = [80, 160, 320]
    Hs, _ = make_batch(sizes, 2)
    Hd, wrs, wis, Zs, info = run_batched(neig, Hs)
    for i, H in enumerate(Hs):
        r = neig.schur(to_dev(H))
        A, B = match_eigenvalues(eigs(r.wr.cpu().numpy(), r.wi.cpu().numpy()),
                                 eigs(wrs[i].cpu().numpy(), wis[i].cpu().numpy()))
        S0, Z0, wr0, wi0, info0 = oracle.schur(H)
        cnd = oracle.cond(S0)
        lam0 = eigs(wr0, wi0)
        for a, b in zip(A, B):
            c = cnd[int(np.argmin(np.abs(lam0 - a)))]
            if c * 1e-10 < 1:
                assert abs(a - b) <= 2e-10 * np.linalg.norm(H) * c


def test_batched_invalid_entries_are_skipped(neig):
    """A problem with a bad leading dimension or size gets its own negative info
    and is left untouched; the others are solved."""
    import torch

    Hs, _ = make_batch([50, 60, 70], 4)
    call = neig.batched_tables([to_dev(H) for H in Hs])
    keep = call.Hs[1].clone()
    meta = call.meta.cpu()
    meta[3 + 1] = 10  # ldh of problem 1 < n
    call.meta.copy_(meta.to(call.meta.device))
    neig.launch_batched(call)
    torch.cuda.synchronize()
    info = call.info.cpu().numpy()
    assert info[0] == 0 and info[1] == -4 and info[2] == 0
    assert torch.equal(call.Hs[1], keep)
    for i in (0, 2):
        check_problem(Hs[i], to_host(call.Hs[i]), to_host(call.Zs[i]), call.wrs[i].cpu().numpy(),
                      call.wis[i].cpu().numpy(), None, f"problem {i}")


def test_batched_graph_capture_replays(neig):
    """The batched call is captured in a HIP graph behind the copies that restore
    its inputs, and replayed several times with eager work in between; every
    replay reproduces the eager result bit for bit."""
    import torch

    sizes = [40, 130, 260, 64, 500]
    Hs, _ = make_batch(sizes, 3)
    H0 = [to_dev(H) for H in Hs]
    Z0 = [torch.eye(n, dtype=torch.float64, device="cuda").t().contiguous().t() for n in sizes]
    call = neig.batched_tables([torch.empty_like(h) for h in H0], [torch.empty_like(z) for z in Z0])

    def restore():
        for a, b in zip(call.Hs, H0):
            a.copy_(b)
        for a, b in zip(call.Zs, Z0):
            a.copy_(b)

    restore()
    neig.launch_batched(call)
    torch.cuda.synchronize()
    assert np.all(call.info.cpu().numpy() == 0)
    ref = [t.clone() for t in call.Hs + call.Zs + call.wrs + call.wis]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        restore()
        neig.launch_batched(call, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in call.Hs:
            t.fill_(7.0)  # eager work between replays
        call.info.fill_(5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = call.Hs + call.Zs + call.wrs + call.wis
        for i, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (rep, i)
        assert np.all(call.info.cpu().numpy() == 0)


def test_batched_flop_count(neig):
    """The batched kernel counts the method's operations on the device: integer
    counts, so a batch [A, B, A] counts exactly twice A's work plus B's, every
    problem at least its final 10 m^3 Schur form, and each call (a replayed
    graph included) counts only its own work."""
    import torch

    A, B = make_batch([180, 140], 41)[0]
    counts = {}
    for tag, Hs in (("A", [A]), ("B", [B]), ("ABA", [A, B, A])):
        c = neig.schur_batched([to_dev(H) for H in Hs])
        torch.cuda.synchronize()
        assert np.all(c.info.cpu().numpy() == 0)
        counts[tag] = neig.batched_flops()
        say(f"  flops {tag}: {counts[tag]:.6g}")
    assert counts["A"] > 10 * 180.0 ** 3 / 8 and counts["B"] > 0
    assert counts["ABA"] == 2 * counts["A"] + counts["B"]
    # a second call of the same batch counts the same, not the sum of both
    c = neig.schur_batched([to_dev(A)])
    torch.cuda.synchronize()
    assert neig.batched_flops() == counts["A"]
