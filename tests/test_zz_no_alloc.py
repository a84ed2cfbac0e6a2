"""The batched entry point that allocates nothing (neig_schur_batched_noalloc),
through the C ABI: on two calls in a row, the second with fewer and smaller
problems, it gives bit for bit what neig_schur_batched gives on the same
inputs, and every result passes the per-problem parity checks; batches above
its limit are refused before any work; a captured graph of it replays."""
import numpy as np
import pytest

from checks import EPS, backward_error, orthogonality, structure_violations
from gpu_util import say, to_dev, to_host
from paper_2002_05024_amd import inputs

pytestmark = pytest.mark.gpu

NOALLOC_MAX = 4096


@pytest.fixture(scope="module")
def neig():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2002_05024_amd import binding

    binding.load_library()
    return binding


def make_batch(sizes, seed):
    Hs = []
    for i, n in enumerate(sizes):
        g = inputs.rng(inputs.BATCHED, 7000 + seed * 1000 + i)
        if i % 2 == 0:
            Hs.append(inputs.random_hessenberg(n, g))
        else:
            A, _ = inputs.prescribed_matrix(n, g, 0.1 / np.sqrt(max(n, 1)))
            Hs.append(inputs.to_hessenberg(A)[0])
    return Hs


def solve(neig, Hs, noalloc):
    import torch

    call = neig.batched_tables([to_dev(H) for H in Hs])
    neig.launch_batched(call, noalloc=noalloc)
    torch.cuda.synchronize()
    return call


def compare_calls(neig, Hs, tag):
    import torch

    ref = solve(neig, Hs, noalloc=False)
    got = solve(neig, Hs, noalloc=True)
    assert torch.equal(got.info, ref.info), tag
    assert np.all(got.info.cpu().numpy() == 0), tag
    for i in range(len(Hs)):
        for a, b, what in ((got.Hs[i], ref.Hs[i], "S"), (got.Zs[i], ref.Zs[i], "Z"), (got.wrs[i], ref.wrs[i], "wr"),
                           (got.wis[i], ref.wis[i], "wi")):
            assert torch.equal(a, b), (tag, i, what)
        n = Hs[i].shape[0]
        S, Z = to_host(got.Hs[i]), to_host(got.Zs[i])
        wr, wi = got.wrs[i].cpu().numpy(), got.wis[i].cpu().numpy()
        if n > 0:
            assert backward_error(Hs[i], S, Z) <= 50 * n * EPS, (tag, i)
            assert orthogonality(Z) <= 50 * n * EPS, (tag, i)
        assert structure_violations(S, wr, wi) == [], (tag, i)


def test_noalloc_matches_allocating_entry_two_calls(neig):
    first = [300, 97, 1, 2, 64, 513, 150, 33, 700, 96, 5, 258]
    second = [40, 120, 3, 90]  # fewer and smaller problems: the fixed array keeps the first call's contents
    say(f"noalloc first call sizes={first}")
    compare_calls(neig, make_batch(first, 1), "first")
    say(f"noalloc second call sizes={second}")
    compare_calls(neig, make_batch(second, 2), "second")


def test_noalloc_refuses_batches_above_its_limit(neig):
    import torch

    Hs = make_batch([8], 3)
    call = neig.batched_tables([to_dev(H) for H in Hs])
    lib = neig.load_library()
    import ctypes

    vp = ctypes.c_void_p
    m, p = call.meta.data_ptr(), call.ptrs.data_ptr()
    before = call.Hs[0].clone()
    rc = lib.neig_schur_batched_noalloc(NOALLOC_MAX + 1, vp(m), vp(p), vp(m), vp(p), vp(m), vp(p), vp(p), vp(p),
                                        vp(call.info.data_ptr()), None)
    assert rc == -1
    torch.cuda.synchronize()
    assert torch.equal(call.Hs[0], before)  # nothing ran


def test_noalloc_graph_capture_replays(neig):
    """Captured in a HIP graph behind the copies that restore its inputs and
    replayed with eager work in between: every replay equals the eager result."""
    import torch

    sizes = [40, 130, 260, 64]
    Hs = make_batch(sizes, 4)
    H0 = [to_dev(H) for H in Hs]
    Z0 = [torch.eye(n, dtype=torch.float64, device="cuda").t().contiguous().t() for n in sizes]
    call = neig.batched_tables([torch.empty_like(h) for h in H0], [torch.empty_like(z) for z in Z0])

    def restore():
        for a, b in zip(call.Hs, H0):
            a.copy_(b)
        for a, b in zip(call.Zs, Z0):
            a.copy_(b)

    restore()
    neig.launch_batched(call, noalloc=True)
    torch.cuda.synchronize()
    assert np.all(call.info.cpu().numpy() == 0)
    ref = [t.clone() for t in call.Hs + call.Zs + call.wrs + call.wis]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        restore()
        neig.launch_batched(call, stream=s, noalloc=True)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in call.Hs:
            t.fill_(3.0)
        call.info.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(call.Hs + call.Zs + call.wrs + call.wis, ref)):
            assert torch.equal(a, b), (rep, i)
        assert np.all(call.info.cpu().numpy() == 0)
