"""Host-side logic that needs no GPU: the input generators of the batched and
learned workloads, the training-weight rule, and the autotuner's candidate
filter."""
import os

import numpy as np
import pytest

from paper_2002_05024_amd import inputs


@pytest.mark.parametrize("n", [5, 40, 131])
def test_prescribed_hessenberg_keeps_the_spectrum(n):
    H, lam = inputs.prescribed_hessenberg(n, inputs.rng(90, n), 0.1 / np.sqrt(n))
    assert np.all(np.tril(H, -2) == 0)
    ev = np.linalg.eigvals(H)
    # well-conditioned T: the eigenvalues of H are the prescribed ones
    d = np.abs(np.sort_complex(ev) - np.sort_complex(lam))
    assert d.max() < 1e-10


def test_prescribed_hessenberg_first_column_is_uniform_on_the_sphere():
    """The construction's first basis vector P e1 = w is uniform: the mean of
    w over many draws is ~0 and E[w_k^2] = 1/n."""
    n, draws = 6, 4000
    ws = []
    for k in range(draws):
        g = inputs.rng(91, k)
        inputs.prescribed_quasi_triangular(n, g, 0.0)  # same draw order as the generator
        w = g.standard_normal(n)
        ws.append(w / np.linalg.norm(w))
    ws = np.array(ws)
    assert np.all(np.abs(ws.mean(axis=0)) < 0.05)
    assert np.allclose((ws ** 2).mean(axis=0), 1.0 / n, atol=0.02)


def test_batched_workload_sizes_and_families():
    Hs, lams = inputs.batched_workload(count=12, seed=3, lo=32, hi=64, threads=2)
    assert len(Hs) == 12
    for i, (H, lam) in enumerate(zip(Hs, lams)):
        n = H.shape[0]
        assert 32 <= n <= 64 and H.flags.f_contiguous
        assert np.all(np.tril(H, -2) == 0)
        assert (lam is None) == (i % 2 == 0)
    # deterministic
    Hs2, _ = inputs.batched_workload(count=12, seed=3, lo=32, hi=64, threads=3)
    assert all(np.array_equal(a, b) for a, b in zip(Hs, Hs2))


def test_learned_matrices_three_families():
    from paper_2002_05024_amd import learn

    fams = [learn.make_matrix(i, "train", 60, 80)[0] for i in range(6)]
    assert fams == ["random", "prescribed", "graded"] * 2
    fam, H = learn.make_matrix(2, "train", 60, 80)
    row_scale = np.abs(H).max(axis=1)
    assert row_scale[-1] < 1e-6 * row_scale[0]  # graded: 10^(-8 i / n)
    _, H0 = learn.make_matrix(0, "heldout", 60, 80)
    _, H1 = learn.make_matrix(0, "train", 60, 80)
    assert not np.array_equal(H0, H1)  # held-out matrices are other draws


def test_sample_weights_rule():
    from paper_2002_05024_amd import learn

    # two runs; rewards = deflations / ms
    stats = np.array([[10, 1, 100, 1], [20, 1, 100, 1], [30, 1, 100, 1],   # run 0: rewards 10, 20, 30
                      [5, 1, 90, 1], [5, 1, 90, 1]], dtype=np.float32)      # run 1: all equal
    run = np.array([0, 0, 0, 1, 1])
    w = learn.sample_weights(stats, run, beta=1.0)
    assert w[0] == 0 and w[1] == 0  # at or below the run's median
    assert w[2] == pytest.approx(np.exp(np.log((30 + 1e-3) / (20 + 1e-3))), rel=1e-6)
    assert np.all(w[3:] == 0)


def test_autotune_candidate_filter():
    from paper_2002_05024_amd import autotune

    assert autotune._valid({"nw": 64, "ns": 32, "nmin": 96, "chase_w": 50})
    assert not autotune._valid({"nw": 64, "ns": 32, "nmin": 96, "chase_w": 49})


def test_network_bins_match_the_library():
    from paper_2002_05024_amd import binding, learn

    if not os.path.exists(binding.library_path()):
        pytest.skip("libneig.so not built")
    ns, nw = binding.policy_bins()
    assert tuple(ns) == learn.NS_BINS and tuple(nw) == learn.NW_BINS


def test_run_weights_rule():
    from paper_2002_05024_amd import learn

    k = len(learn.ARMS)
    t_def = np.array([2.0, 2.0, 2.0, 1.0])
    t_run = np.array([2.0, 1.0, 4.0, 1.0])
    arm = np.array([0, 3, 5, -1])
    w = learn.run_weights(t_def, t_run, arm, beta=1.0)
    # an arm as fast as the defaults weighs as much as a default decision;
    # twice as fast: twice as much; twice as slow: half
    assert w[0] == pytest.approx(1.0) and w[3] == pytest.approx(1.0 / k)
    assert w[1] == pytest.approx(2.0) and w[2] == pytest.approx(0.5)
    assert len(set(learn.ARMS)) == k and learn.default_bins(5000) == (3, 4) and learn.default_bins(200) == (1, 2)
    assert learn.default_bins(5000) not in learn.ARMS


def test_run_weights_spread_over_decisions():
    from paper_2002_05024_amd import learn

    # matrix 0: default solve with 1 decision, arm solve with 3; matrix 1: 2 + 2
    t_def = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    t_run = np.array([1.0, 0.5, 0.5, 0.5, 1.0, 1.0, 1.0, 1.0])
    arm = np.array([-1, 2, 2, 2, -1, -1, 4, 4])
    run = np.array([0, 0, 0, 0, 1, 1, 1, 1])
    w = learn.run_weights(t_def, t_run, arm, beta=1.0, run=run)
    k = len(learn.ARMS)
    scale = 2.0  # mean decisions per solve
    assert w[0] == pytest.approx(scale / k)
    assert np.allclose(w[1:4], 2.0 / 3 * scale)  # a solve's weight split over its decisions
    assert np.allclose(w[4:6], 0.5 / k * scale) and np.allclose(w[6:8], 0.5 * scale)


def test_smoothed_targets_follow_the_neighbourhood():
    from paper_2002_05024_amd import learn

    g = np.random.default_rng(0)
    # two well separated groups of matrices; arm F (64 shifts, 48 rows) is
    # faster in group A, slower in group B; the other arm tried is neutral
    XA = g.normal(0.0, 0.1, (20, 24))
    XB = g.normal(5.0, 0.1, (20, 24))
    X = np.vstack([XA, XB])
    F, N = learn.bins_of(64, 48), learn.bins_of(16, 64)
    aF, aN = learn.ARMS.index(F), learn.ARMS.index(N)
    arms = np.array([aF, aN] * 20)
    adv = np.where(np.arange(40) < 20, np.where(arms == aF, 0.3, 0.0), np.where(arms == aF, -0.5, 0.0))
    T = learn.smoothed_targets(X, arms, adv, k=10, beta=8.0)
    default = learn.default_bins(1000)
    for i in range(40):
        probs = dict(T[i])
        assert abs(sum(probs.values()) - 1.0) < 1e-12
        best = max(probs, key=probs.get)
        assert best == (F if i < 20 else default) or (i >= 20 and best == N)
    ids, Xm, am, av = learn.per_matrix_rows(np.array([0, 0, 0, 1, 1]), np.array([-1, -1, 4, -1, 2]),
                                            np.array([2.0] * 5), np.array([2.0, 2.0, 1.0, 2.0, 4.0]),
                                            np.arange(5, dtype=float)[:, None] * np.ones((1, 3)))
    assert list(ids) == [0, 1] and list(am) == [4, 2]
    assert np.allclose(av, [np.log(2.0), np.log(0.5)]) and np.allclose(Xm[:, 0], [0.0, 3.0])


def test_compact_runs_keeps_first_decisions(tmp_path):
    from paper_2002_05024_amd import learn

    # two files of per-run data: matrix 0 (default solve: 2 decisions, arm solve: 3)
    # and matrix 1 (1 + 2); the compact file holds the first decision of each solve
    def part(run, arm, feat0):
        n = len(run)
        return {"feat": np.arange(n, dtype=np.float32)[:, None] + feat0 + np.zeros((1, 24), np.float32),
                "bins": np.zeros((n, 2), np.int32), "stats": np.zeros((n, 4), np.float32),
                "run": np.array(run, np.int32), "t_def": np.full(n, 2.0, np.float32),
                "t_run": np.array([2.0 if a < 0 else 1.0 for a in arm], np.float32),
                "arm": np.array(arm, np.int32), "p_arm": np.full(n, 0.1, np.float32)}
    a = part([0, 0, 0, 0, 0], [-1, -1, 3, 3, 3], 0.0)
    b = part([1, 1, 1], [-1, 5, 5], 100.0)
    fa, fb, out = tmp_path / "a.npz", tmp_path / "b.npz", str(tmp_path / "c.npz")
    np.savez(fa, **a)
    np.savez(fb, **b)
    assert learn.compact_runs([str(fa), str(fb)], out) == 4
    c = np.load(out)
    assert list(c["run"]) == [0, 0, 1, 1] and list(c["arm"]) == [-1, 3, -1, 5]
    assert list(c["feat"][:, 0]) == [0.0, 2.0, 100.0, 101.0]
    full = {k: np.concatenate([a[k], b[k]]) for k in a}
    r1 = learn.per_matrix_rows(full["run"], full["arm"], full["t_def"], full["t_run"], full["feat"])
    r2 = learn.per_matrix_rows(c["run"], c["arm"], c["t_def"], c["t_run"], c["feat"])
    assert all(np.array_equal(x, y) for x, y in zip(r1, r2))


def test_single_tuner_table_buckets_and_keys():
    """The committed single-matrix table: each order falls in one bucket, whose
    entries are valid library parameters (nibble included), and older tables
    without nibble still give their four keys."""
    from paper_2002_05024_amd import autotune_single as at

    table = at.load()
    assert table is not None
    small, large = at.params_for(4000, table), at.params_for(20000, table)
    assert set(small) == set(large) == set(at.KEYS)
    for p in (small, large, {k: table["hard_optimum"][k] for k in at.KEYS}):
        assert at._valid(p) and p["nibble"] in at.GRID["nibble"]
    assert at.params_for(6000, table) == small and at.params_for(6001, table) == large
    old = {"buckets": [{"n_hi": None, "ns": 32, "nw": 64, "chain": 8, "chase_w": 96}]}
    assert at.params_for(100, old) == {"ns": 32, "nw": 64, "chain": 8, "chase_w": 96}
