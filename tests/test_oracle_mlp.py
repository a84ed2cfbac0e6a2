"""Pins of the proposal-network oracle (CPU only): the backward pass against
central finite differences of the loss, the forward pass against hand-set
networks whose outputs are known in closed form, the softmax/cross-entropy
special cases, one Adam step in closed form, and the quantile rule against
numpy's linear-interpolation quantile."""
import numpy as np
import pytest

from oracle import mlp


def tiny_case(B=5, seed=0):
    g = np.random.default_rng(seed)
    theta = mlp.init(seed, mu=g.standard_normal(mlp.NIN) * 0.1, sd=0.5 + g.random(mlp.NIN))
    X = g.standard_normal((B, mlp.NIN))
    a = g.integers(0, 8, B)
    c = g.integers(0, 8, B)
    w = g.random(B) + 0.1
    return theta, X, a, c, w


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    theta, X, a, c, w = tiny_case(seed=seed)
    L, g = mlp.loss_and_grad(theta, X, a, c, w)
    assert abs(L - mlp.loss(theta, X, a, c, w)) < 1e-12
    h = 1e-6
    rng = np.random.default_rng(100 + seed)
    # every bias and a random subset of weights (the whole vector is slow-ish)
    idx = np.concatenate([np.arange(mlp.NPARAM - 16, mlp.NPARAM), rng.choice(mlp.NPARAM, 300, replace=False)])
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, a, c, w) - mlp.loss(tm, X, a, c, w)) / (2 * h)
        if i < 2 * mlp.NIN:
            assert g[i] == 0.0  # normalisation is fixed, not trained
            continue
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_weights_give_bias_logits_and_log8_loss():
    parts = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    parts["sd"] = np.ones(mlp.NIN)
    theta = mlp.pack(parts)
    X = np.random.default_rng(3).standard_normal((4, mlp.NIN))
    z, _ = mlp.forward(theta, X)
    assert np.all(z == 0.0)
    a = np.array([0, 3, 7, 1])
    c = np.array([2, 2, 5, 0])
    w = np.array([1.0, 2.0, 0.5, 0.0])
    # uniform scores: each head's cross-entropy is log 8
    assert mlp.loss(theta, X, a, c, w) == pytest.approx(np.sum(w) * 2 * np.log(8.0) / 4, rel=1e-14)
    parts["b3"] = np.array([np.log(3.0)] + [0.0] * 7 + [0.0] * 8)
    theta = mlp.pack(parts)
    # head 1 scores: bin 0 has weight 3 of a total 3 + 7 = 10
    L = mlp.loss(theta, X[:1], [0], [4], [1.0])
    assert L == pytest.approx(-np.log(0.3) + np.log(8.0), rel=1e-13)


def test_hand_set_network_forward():
    parts = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    parts["mu"] = np.full(mlp.NIN, 1.0)
    parts["sd"] = np.full(mlp.NIN, 2.0)
    parts["W1"][0, 0] = 1.0      # h1[0] = relu((x0 - 1) / 2)
    parts["W2"][5, 0] = 2.0      # h2[5] = relu(2 h1[0] - 0.5)
    parts["b2"][5] = -0.5
    parts["W3"][3, 5] = 1.0      # z[3] = h2[5] + 0.25
    parts["b3"][3] = 0.25
    theta = mlp.pack(parts)
    X = np.zeros((3, mlp.NIN))
    X[:, 0] = [4.0, 1.2, -3.0]
    z, act = mlp.forward(theta, X)
    # x0 = 4: h1 = 1.5, h2 = 2.5, z3 = 2.75; x0 = 1.2: h1 = 0.1, h2 = relu(-0.3) = 0; x0 = -3: h1 = 0
    assert z[0, 3] == pytest.approx(2.75, abs=1e-15)
    assert z[1, 3] == pytest.approx(0.25, abs=1e-15)
    assert z[2, 3] == pytest.approx(0.25, abs=1e-15)
    others = np.delete(z, 3, axis=1)
    assert np.all(others == 0.0)


def test_softmax_invariants():
    z = np.random.default_rng(4).standard_normal((6, 8)) * 30
    p = mlp.softmax(z)
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-15)
    assert np.allclose(mlp.softmax(z + 123.0), p, atol=1e-15)
    assert np.all(np.argmax(p, axis=1) == np.argmax(z, axis=1))


def test_adam_first_step_is_signed_learning_rate():
    theta, X, a, c, w = tiny_case()
    L, g = mlp.loss_and_grad(theta, X, a, c, w)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t1, m1, v1 = mlp.adam_step(theta, g, m, v, 1, lr=1e-2)
    step = theta - t1
    big = np.abs(g) > 1e-4
    # first bias-corrected step: lr * g / (|g| + eps)
    assert np.allclose(step[big], 1e-2 * np.sign(g[big]), rtol=1e-3)
    assert np.all(step[: 2 * mlp.NIN] == 0.0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # fixed entries keep their moments
    m0 = np.full_like(theta, 0.5)
    _, m2, v2 = mlp.adam_step(theta, g, m0, m0, 2)
    assert np.all(m2[: 2 * mlp.NIN] == 0.5) and np.all(v2[: 2 * mlp.NIN] == 0.5)


@pytest.mark.parametrize("k", [1, 2, 7, 100, 1023])
def test_quantile_rule_is_linear_interpolation(k):
    v = np.random.default_rng(k).standard_normal(k)
    probs = 0.05 * np.arange(1, 20)
    assert np.allclose(mlp.quantiles(v, probs), np.quantile(v, probs, method="linear"), atol=1e-14)


# ---------------------------------------------------------------- features

def _graded_block(n, ktop, kbot, logvals, hscale):
    """Hessenberg matrix of order n whose subdiagonal entries in the active
    block are h(k, k-1) = hscale * exp(logvals[k - ktop - 1]), k = ktop+1..kbot;
    everything outside the block (other subdiagonals, the rest of the matrix)
    holds values that would change the features if they were read."""
    g = np.random.default_rng(7)
    H = np.triu(g.standard_normal((n, n)), -1) * 1e3
    for k in range(1, n):
        H[k, k - 1] = 1e-200 if (k <= ktop or k > kbot) else hscale * np.exp(logvals[k - ktop - 1])
    return H


def test_features_closed_form_every_subdiagonal():
    # m - 1 = 301 <= 1024: every subdiagonal entry of the block is used, with
    # log(|h| / scale) = 0, 1/10, ..., 30 (sorted, evenly spaced), so the
    # p-quantile is exactly p * 30; f0 = log m; f20..f23 are passed through
    n, ktop, kbot = 340, 17, 318
    m = kbot - ktop + 1
    hnorm = 3.0 * np.sqrt(n)  # scale hnorm / sqrt(n) = 3
    logs = np.arange(m - 1) / 10.0
    g = np.random.default_rng(3)
    H = _graded_block(n, ktop, kbot, g.permutation(logs), 3.0)  # order along the diagonal is irrelevant
    extra = [0.25, -1.5, 2.0, 0.125]
    f = mlp.features(H, ktop, kbot, hnorm, extra)
    assert f[0] == pytest.approx(np.log(m), abs=1e-15)
    probs = 0.05 * np.arange(1, 20)
    assert np.allclose(f[1:20], probs * 30.0, rtol=0, atol=1e-12)
    assert list(f[20:24]) == extra


@pytest.mark.parametrize("stride", [2, 3])
def test_features_closed_form_sampled_subdiagonal(stride):
    # m - 1 = 1024 * stride > 1024: the sample is k = ktop + 1 + stride * i,
    # i < 1024.  Entries at those offsets carry log values 0, 0.5, ..., 511.5;
    # every other entry of the block carries -600, which would pull the low
    # quantiles down if any were sampled.  p-quantile = 0.5 * 1023 p exactly.
    cnt = 1024 * stride
    ktop = 5
    kbot = ktop + cnt
    n = kbot + 4
    logs = np.full(cnt, -600.0)
    logs[::stride] = 0.5 * np.arange(1024)
    H = _graded_block(n, ktop, kbot, logs, 2.0)
    f = mlp.features(H, ktop, kbot, 2.0 * np.sqrt(n), [0, 0, 0, 0])
    assert f[0] == pytest.approx(np.log(cnt + 1), abs=1e-15)
    probs = 0.05 * np.arange(1, 20)
    assert np.allclose(f[1:20], 0.5 * 1023 * probs, rtol=0, atol=1e-11)


def test_features_single_row_block():
    # m = 1: no subdiagonal entry, the quantile features are zero
    H = _graded_block(8, 3, 3, [], 1.0)
    f = mlp.features(H, 3, 3, 1.0, [1, 2, 3, 4])
    assert f[0] == 0.0 and np.all(f[1:20] == 0.0) and list(f[20:24]) == [1, 2, 3, 4]
