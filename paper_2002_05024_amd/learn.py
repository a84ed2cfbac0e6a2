"""Training and evaluation of the parameter-proposal network.

Stages, each run on a GPU:

``collect``      per-decision exploration (``policy = 2``: every iteration's
                 shift-count and window bins drawn at random), storing each
                 decision's features, bins and the deflations per millisecond
                 that followed it.  (A first design; its rewards are myopic.)
``collect-run``  per-run exploration: every training matrix (three families:
                 random N(0,1), prescribed-spectrum and row-graded Hessenberg,
                 n uniform in [1000, 8000]) is solved with the default rules and
                 with one (shift, window) bin pair held for the whole solve
                 (``policy = 3``); both solves' decisions and times are stored.
``compact``      keeps the first decision of every solve of ``collect-run``
                 files (all that ``train --smooth-k`` reads): the committed
                 training set ``learn_runs_gfx950.npz``.
``train``        fits the network by weighted cross-entropy with the library's
                 own GPU kernels (``neig_mlp_grad`` + ``neig_mlp_adam``); for
                 per-run data a solve weighs exp(beta log(t_default / t_solve))
                 over its exploration probability, and ``--first-only`` keeps
                 the first decision of each solve (a per-matrix proposal).
                 Input normalisation (mu, sd) comes from the data.
``evaluate``     solves held-out matrices with the default rules and with the
                 network (``policy = 4`` by default: the first proposal holds for
                 the whole solve), times both, and checks every result (backward
                 error and orthogonality <= 50 n eps); a result that fails the
                 check with the network is solved again with the default rules.

Inputs are built on the host by worker threads in rounds between the timed
solves (never during one).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SAVED = os.path.join(HERE, "policy_gfx950.npy")
FAMILIES = ("random", "prescribed", "graded")
POLICY = 4  # how the committed network is used: one proposal per matrix
EPS = 2.0 ** -52


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_matrix(index: int, split: str, lo: int = 1000, hi: int = 8000):
    """Matrix ``index`` of a split ('train' or 'heldout'): family index % 3,
    n uniform in [lo, hi]."""
    from . import inputs

    base = 0 if split == "train" else 500_000
    g = inputs.rng(inputs.LEARNED, base + index)
    n = int(g.integers(lo, hi + 1))
    fam = FAMILIES[index % 3]
    if fam == "random":
        H = inputs.random_hessenberg(n, g)
    elif fam == "graded":
        H = inputs.graded_hessenberg(n, g)
    else:
        H, _ = inputs.prescribed_hessenberg(n, g, 0.1 / np.sqrt(n))
    return fam, H


def producer(indices, split, lo, hi, threads=8, depth=None):
    """Yield (index, family, H) in order.  Matrices are built in rounds of
    ``depth`` by ``threads`` workers with single-threaded host BLAS, and a round
    is handed out only when all of it is built: nothing runs on the host while
    a solve is timed (the builders' host-memory traffic delays the solver's
    small device-to-host read-backs and would show up in its time)."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    depth = depth or 2 * threads
    for s0 in range(0, len(indices), depth):
        chunk = indices[s0: s0 + depth]
        with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=threads) as ex:
            mats = list(ex.map(lambda i: make_matrix(i, split, lo, hi), chunk))
        for i, (fam, H) in zip(chunk, mats):
            yield i, fam, H


class Solver:
    """Device buffers sized for the largest n, reused by every solve."""

    def __init__(self, nmax: int):
        import torch

        from . import binding

        self.torch, self.binding = torch, binding
        self.Hbuf = torch.empty(nmax * nmax, dtype=torch.float64, device="cuda")
        self.Zbuf = torch.empty(nmax * nmax, dtype=torch.float64, device="cuda")

    def solve(self, H, check: bool = True):
        """Solve with the current parameters; returns (seconds, info, be, oe)."""
        torch = self.torch
        n = H.shape[0]
        H0 = torch.from_numpy(np.ascontiguousarray(H.T)).cuda().t()
        Hd = self.Hbuf[: n * n].view(n, n).t()  # column-major n x n
        Zd = self.Zbuf[: n * n].view(n, n).t()
        Hd.copy_(H0)
        Zd.zero_()
        Zd.diagonal().fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = self.binding.schur(Hd, Zd)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1000.0
        be = oe = float("nan")
        if check:
            R = torch.mm(torch.mm(Zd, Hd), Zd.t())
            R.sub_(H0)
            be = float(torch.linalg.norm(R) / torch.linalg.norm(H0))
            E = torch.mm(Zd.t(), Zd)
            E.diagonal().sub_(1.0)
            oe = float(torch.linalg.norm(E))
        return sec, r.info, be, oe


def collect(start: int, count: int, out: str, lo: int, hi: int, seed: int, threads: int):
    from . import binding

    binding.load_library()
    solver = Solver(hi)
    feats, bins, stats, runs = [], [], [], []
    t0 = time.time()
    for i, fam, H in producer(list(range(start, start + count)), "train", lo, hi, threads):
        binding.set_params(policy=2, seed=seed * 100_003 + i)
        sec, info, _, _ = solver.solve(H, check=False)
        f, b, s = binding.policy_log()
        feats.append(f)
        bins.append(b)
        stats.append(s)
        runs.append(np.full(len(b), i, dtype=np.int32))
        log(f"[collect] {i} {fam} n={H.shape[0]} {sec:.2f}s info={info} decisions={len(b)} "
            f"elapsed {time.time() - t0:.0f}s")
        if len(runs) % 25 == 0:  # keep what is done if the run is cut short
            _save(out, feats, bins, stats, runs)
    binding.set_params(policy=0)
    _save(out, feats, bins, stats, runs)


# The network's bins (the library's neig_policy_bins): shifts per sweep and
# AED window rows.
NS_BINS = (8, 16, 24, 32, 48, 64, 96, 128)
NW_BINS = (32, 40, 48, 56, 64, 72, 80, 96)


def bins_of(ns: int, nw: int):
    return NS_BINS.index(ns), NW_BINS.index(nw)


# Arms of the per-run exploration: (shift bin, window bin) pairs held for a
# whole solve: 16, 32, 64 or 96 shifts with 48-, 64- or 80-row windows, less
# the default rules' own pair (32 shifts and a 64-row window for active blocks
# of 300 rows or more; 16 and 48 below).
ARMS = [bins_of(a, b) for a in (16, 32, 64, 96) for b in (48, 64, 80) if (a, b) != (32, 64)]
# arms for a focused round of exploration
FOCUSED_ARMS = [bins_of(64, 64), bins_of(96, 64), bins_of(64, 80), bins_of(16, 48)]


def default_bins(m):
    """The bins of the default rules for an active block of order m."""
    return bins_of(32, 64) if m >= 300 else bins_of(16, 48)


def collect_runs(start: int, count: int, out: str, lo: int, hi: int, threads: int, arms=None):
    """Per-run exploration: every training matrix is solved twice, once with the
    default rules (``policy = 1`` with no network: the defaults decide and every
    decision's features are logged) and once with one arm held for the whole
    solve (``policy = 3``); arms cycle per family.  Stores the decisions of both
    solves and, per solve, the time of the default solve and its own."""
    from . import binding

    binding.load_library()
    binding.policy_set(None)
    solver = Solver(hi)
    arms = arms or ARMS
    rec = {"feat": [], "bins": [], "stats": [], "run": [], "t_def": [], "t_run": [], "arm": [], "p_arm": []}
    t0 = time.time()
    for i, fam, H in producer(list(range(start, start + count)), "train", lo, hi, threads):
        arm = arms[(i // 3) % len(arms)]
        binding.set_params(policy=1)
        t_def, info_d, _, _ = solver.solve(H, check=False)
        f0, b0, s0 = binding.policy_log()
        b0 = np.array([default_bins(m) for m in s0[:, 2]], dtype=np.int32).reshape(-1, 2)
        binding.set_params(policy=3, seed=arm[0] + 8 * arm[1])
        t_arm, info_a, _, _ = solver.solve(H, check=False)
        f1, b1, s1 = binding.policy_log()
        for f, b, st, kind, t in ((f0, b0, s0, -1, t_def), (f1, b1, s1, ARMS.index(arm), t_arm)):
            rec["feat"].append(f)
            rec["bins"].append(b)
            rec["stats"].append(st)
            rec["run"].append(np.full(len(b), i, dtype=np.int32))
            rec["t_def"].append(np.full(len(b), t_def, dtype=np.float32))
            rec["t_run"].append(np.full(len(b), t, dtype=np.float32))
            rec["arm"].append(np.full(len(b), kind, dtype=np.int32))
            rec["p_arm"].append(np.full(len(b), 1.0 / len(arms), dtype=np.float32))
        log(f"[collect-run] {i} {fam} n={H.shape[0]} default {t_def:.2f}s arm {arm} {t_arm:.2f}s "
            f"info {info_d}/{info_a} elapsed {time.time() - t0:.0f}s")
        if (i - start + 1) % 10 == 0:
            _save_runs(out, rec)
    binding.set_params(policy=0, seed=0)
    _save_runs(out, rec)


def compact_runs(files, out: str):
    """The first decision of every solve of per-run files, in one file with the
    same fields (default and arm solve of a matrix share its run id)."""
    parts = [np.load(f) for f in files]
    rec = {k: np.concatenate([p[k] for p in parts]) for k in parts[0].files}
    key = rec["run"].astype(np.int64) * 64 + (rec["arm"] + 1)
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)
    tmp = out + ".tmp.npz"
    np.savez_compressed(tmp, **{k: v[first] for k, v in rec.items()})
    os.replace(tmp, out)
    return len(first)


def _save_runs(out, rec):
    tmp = out + ".tmp.npz"
    np.savez_compressed(tmp, **{k: np.concatenate(v) for k, v in rec.items()})
    os.replace(tmp, out)


def run_weights(t_def, t_run, arm, beta: float = 3.0, run=None, p_arm=None):
    """Weights of the per-run data: an arm's solve counts
    exp(beta * log(t_default / t_arm)) times the number of arms (each arm is
    tried on 1/len(ARMS) of the matrices); a default solve counts 1.  With
    ``run`` (one id per solve's decisions; the default and the arm solve of a
    matrix have the same id but different ``arm``) a solve's weight is spread
    evenly over its decisions, so that a solve with more decisions does not
    count more.  ``p_arm`` (per decision) is the probability with which the
    solve's arm was drawn when exploration used fewer arms; the weight scales
    with its inverse.  The network then prefers an arm over the defaults where
    the arm was clearly faster on matrices with similar features."""
    adv = np.log(np.maximum(t_def, 1e-6) / np.maximum(t_run, 1e-6))
    inv_p = len(ARMS) if p_arm is None else 1.0 / np.asarray(p_arm, dtype=np.float64)
    w = np.where(arm >= 0, inv_p * np.exp(np.minimum(beta * adv, 8.0)), 1.0) / len(ARMS)
    if run is not None:
        key = np.asarray(run, dtype=np.int64) * 64 + (np.asarray(arm) + 1)
        _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        w = w / cnt[inv] * cnt.mean()
    return w


def per_matrix_rows(run, arm, t_def, t_run, feat):
    """One row per training matrix of per-run data: the features of its default
    solve's first decision, the arm its other solve held, and that solve's
    advantage log(t_default / t_arm).  Returns (ids, X, arms, adv)."""
    key = run.astype(np.int64) * 64 + (arm + 1)
    _, first = np.unique(key, return_index=True)
    mats = {}
    for i in first:
        d = mats.setdefault(int(run[i]), {})
        if arm[i] < 0:
            d["x"] = feat[i]
        else:
            d["arm"] = int(arm[i])
            d["adv"] = float(np.log(max(t_def[i], 1e-6) / max(t_run[i], 1e-6)))
    ids = np.array(sorted(r for r, d in mats.items() if "x" in d and "arm" in d), dtype=np.int64)
    X = np.array([mats[r]["x"] for r in ids], dtype=np.float64).reshape(len(ids), -1)
    return ids, X, np.array([mats[r]["arm"] for r in ids]), np.array([mats[r]["adv"] for r in ids])


def smoothed_targets(X, arms, adv, k: int = 25, beta: float = 8.0):
    """Per-matrix soft targets over (default, arms): for each matrix, the mean
    advantage of every arm among its k nearest matrices in normalised feature
    space (each matrix tried one arm), then softmax(beta * advantage) with the
    default rules at advantage 0.  Returns a list, per matrix, of
    ((shift bin, window bin), probability)."""
    Z = (X - X.mean(axis=0)) / (X.std(axis=0) + 1e-3)
    out = []
    for i in range(len(X)):
        nb = np.argsort(np.linalg.norm(Z - Z[i], axis=1), kind="stable")[:k]
        by = {}
        for j in nb:
            by.setdefault(int(arms[j]), []).append(adv[j])
        choices = [(default_bins(1000), 0.0)] + [(ARMS[a], float(np.mean(v))) for a, v in sorted(by.items())]
        w = np.exp(beta * np.array([v for _, v in choices]))
        w /= w.sum()
        out.append([(b, float(p)) for (b, _), p in zip(choices, w)])
    return out


def _save(out, feats, bins, stats, runs):
    tmp = out + ".tmp.npz"
    np.savez_compressed(tmp, feat=np.concatenate(feats), bins=np.concatenate(bins), stats=np.concatenate(stats),
                        run=np.concatenate(runs))
    os.replace(tmp, out)


def sample_weights(stats, run, beta: float = 1.5):
    """Reward = deflations per ms after the decision; advantage = log of the
    reward over its run's median reward; weight = exp(beta * advantage) for
    decisions above the median, 0 below (imitate the better half)."""
    r = np.maximum(stats[:, 0], 0.0) / np.maximum(stats[:, 1], 1e-3)
    w = np.zeros_like(r)
    for k in np.unique(run):
        sel = run == k
        med = np.median(r[sel])
        adv = np.log((r[sel] + 1e-3) / (med + 1e-3))
        w[sel] = np.where(adv > 0, np.exp(np.minimum(beta * adv, 5.0)), 0.0)
    return w


def train(data_files, out: str, epochs: int = 30, batch: int = 4096, lr: float = 2e-3, seed: int = 0,
          beta: float = 3.0, first_only: bool = False, smooth_k: int = 0):
    """Fit the network to per-decision data (``collect``) or per-run data
    (``collect-run``, recognised by its per-solve times).  With ``first_only``
    (per-run data) only the first decision of each solve is used, weighted by
    its solve: the network then makes the per-matrix proposal of
    ``policy = 4`` from the features of the whole matrix."""
    import torch

    from . import binding

    binding.load_library()
    parts = [np.load(f) for f in data_files]
    feat = np.concatenate([p["feat"] for p in parts]).astype(np.float64)
    bins = np.concatenate([p["bins"] for p in parts])
    stats = np.concatenate([p["stats"] for p in parts])
    run = np.concatenate([p["run"] for p in parts])
    if smooth_k > 0:
        # per-matrix soft targets from the k nearest training matrices
        ids, Xm, arms, adv = per_matrix_rows(run, np.concatenate([p["arm"] for p in parts]),
                                             np.concatenate([p["t_def"] for p in parts]),
                                             np.concatenate([p["t_run"] for p in parts]), feat)
        rows = [(x, b, pr) for x, tg in zip(Xm, smoothed_targets(Xm, arms, adv, smooth_k, beta)) for b, pr in tg]
        feat = np.array([x for x, _, _ in rows])
        bins = np.array([b for _, b, _ in rows], dtype=np.int32)
        w = np.array([pr for _, _, pr in rows])
        run = np.zeros(len(w), dtype=np.int32)
    elif all("t_def" in p.files for p in parts):
        t_def = np.concatenate([p["t_def"] for p in parts])
        t_run = np.concatenate([p["t_run"] for p in parts])
        arm = np.concatenate([p["arm"] for p in parts])
        p_arm = np.concatenate([p["p_arm"] if "p_arm" in p.files else np.full(len(p["arm"]), 1.0 / len(ARMS))
                                for p in parts])
        if first_only:
            # decisions of one solve are stored together; keep the first of each
            key = run.astype(np.int64) * 64 + (arm + 1)
            _, first = np.unique(key, return_index=True)
            sel = np.zeros(len(run), dtype=bool)
            sel[first] = True
            w = np.where(sel, run_weights(t_def, t_run, arm, beta, p_arm=p_arm), 0.0)
        else:
            w = run_weights(t_def, t_run, arm, beta, run, p_arm)
    else:
        w = sample_weights(stats, run)
    keep = w > 0
    log(f"[train] {len(w)} decisions, {keep.sum()} weighted, from {len(np.unique(run))} runs")
    X, B, W = feat[keep], bins[keep], w[keep]
    W = W / W.mean()
    mu = X.mean(axis=0)
    sd = X.std(axis=0) + 1e-3
    theta = _init_theta(seed, mu, sd)
    dev = torch.device("cuda")
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    ad = torch.tensor(B[:, 0], dtype=torch.int32, device=dev)
    cd = torch.tensor(B[:, 1], dtype=torch.int32, device=dev)
    wd = torch.tensor(W, dtype=torch.float32, device=dev)
    th = torch.tensor(theta, dtype=torch.float32, device=dev)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    g = np.random.default_rng(seed)
    step = 0
    N = Xd.shape[0]
    for ep in range(epochs):
        perm = torch.tensor(g.permutation(N), device=dev)
        tot = 0.0
        for s in range(0, N, batch):
            idx = perm[s: s + batch]
            loss, grad = binding.mlp_grad(Xd[idx].contiguous(), ad[idx].contiguous(), cd[idx].contiguous(),
                                          wd[idx].contiguous(), th)
            step += 1
            binding.mlp_adam(th, grad, m, v, step, lr)
            tot += float(loss.item()) * len(idx)
        log(f"[train] epoch {ep} loss {tot / N:.4f}")
    np.save(out, th.cpu().numpy())
    return th.cpu().numpy()


def _init_theta(seed, mu, sd):
    """He-style random initialisation with zero biases, in the library's layout."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([56, int(seed)])))
    parts = [mu, sd, g.standard_normal((64, 24)) * np.sqrt(2.0 / 24), np.zeros(64),
             g.standard_normal((64, 64)) * np.sqrt(2.0 / 64), np.zeros(64),
             g.standard_normal((16, 64)) * np.sqrt(1.0 / 64), np.zeros(16)]
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def summarize(rows):
    """Totals of an evaluation: default vs judged network time, overall and per family."""
    tot_d = sum(r["t_default"] for r in rows)
    tot_n = sum(r["t_judged"] for r in rows)
    return {"matrices": len(rows), "total_default_s": tot_d, "total_net_s": tot_n,
            "speedup": tot_d / tot_n if tot_n > 0 else None,
            "per_family": {f: {"default_s": sum(r["t_default"] for r in rows if r["family"] == f),
                               "net_s": sum(r["t_judged"] for r in rows if r["family"] == f)}
                           for f in FAMILIES},
            "all_ok": all(r["ok_net"] for r in rows)}


def evaluate(weights: str, start: int, count: int, lo: int, hi: int, min_conf: float, threads: int,
             out: str | None = None, policy: int = POLICY):
    """Held-out matrices solved with the default rules and with the network;
    with ``out`` the rows so far are saved every 10 matrices."""
    from . import binding

    binding.load_library()
    theta = np.load(weights)
    solver = Solver(hi)
    rows = []

    def run_default(H):
        binding.policy_set(None)
        binding.set_params(policy=0)
        return solver.solve(H)

    def run_net(H):
        binding.policy_set(theta, min_conf)
        binding.set_params(policy=policy)
        out = solver.solve(H)
        return out, binding.get_stats()

    warm = True
    for i, fam, H in producer(list(range(start, start + count)), "heldout", lo, hi, threads):
        n = H.shape[0]
        if warm:  # untimed: workspace growth and first-launch costs fall on neither arm
            run_default(H)
            run_net(H)
            warm = False
        # the arm timed first alternates from matrix to matrix
        if i % 2 == 0:
            t_def, info_d, be_d, oe_d = run_default(H)
            (t_net, info_n, be_n, oe_n), st = run_net(H)
        else:
            (t_net, info_n, be_n, oe_n), st = run_net(H)
            t_def, info_d, be_d, oe_d = run_default(H)
        ok = info_n == 0 and be_n <= 50 * n * EPS and oe_n <= 50 * n * EPS
        t_judged = t_net
        if not ok:  # the backward-error check judges: fall back to the default rules
            t2, info_n, be_n, oe_n = run_default(H)
            t_judged += t2
        rows.append({"i": i, "family": fam, "n": n, "t_default": t_def, "t_net": t_net, "t_judged": t_judged,
                     "ok_net": bool(ok), "be_default": be_d, "be_net": be_n, "oe_default": oe_d, "oe_net": oe_n,
                     "used": st["policy_used"], "fallback": st["policy_fallback"]})
        log(f"[eval] {i} {fam} n={n} default {t_def:.3f}s net {t_net:.3f}s ok={ok} "
            f"be {be_d / (n * EPS):.2f}/{be_n / (n * EPS):.2f} n eps")
        if out and len(rows) % 10 == 0:
            _save_eval(out, rows)
    binding.set_params(policy=0)
    binding.policy_set(None)
    if out:
        _save_eval(out, rows)
    return summarize(rows), rows


def _save_eval(path: str, rows) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"summary": summarize(rows), "rows": rows}, f, indent=1)
    os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser(description="proposal network: collect / train / evaluate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=100)
    c.add_argument("--out", required=True)
    c.add_argument("--seed", type=int, default=1)
    cr = sub.add_parser("collect-run")
    cr.add_argument("--start", type=int, default=0)
    cr.add_argument("--count", type=int, default=100)
    cr.add_argument("--out", required=True)
    cr.add_argument("--focused", action="store_true", help="explore only FOCUSED_ARMS")
    cp = sub.add_parser("compact")
    cp.add_argument("data", nargs="+")
    cp.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("data", nargs="+")
    t.add_argument("--out", default=SAVED)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--beta", type=float, default=3.0)
    t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--first-only", action="store_true")
    t.add_argument("--smooth-k", type=int, default=0,
                   help="per-matrix targets smoothed over the k nearest training matrices")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=SAVED)
    e.add_argument("--start", type=int, default=0)
    e.add_argument("--count", type=int, default=200)
    e.add_argument("--min-conf", type=float, default=0.0)
    e.add_argument("--policy", type=int, default=POLICY)
    e.add_argument("--out", default=None)
    for p in (c, cr, e):
        p.add_argument("--lo", type=int, default=1000)
        p.add_argument("--hi", type=int, default=8000)
        p.add_argument("--threads", type=int, default=8)
    args = ap.parse_args()
    if args.cmd == "collect":
        collect(args.start, args.count, args.out, args.lo, args.hi, args.seed, args.threads)
    elif args.cmd == "collect-run":
        collect_runs(args.start, args.count, args.out, args.lo, args.hi, args.threads,
                     FOCUSED_ARMS if args.focused else None)
    elif args.cmd == "compact":
        print(compact_runs(args.data, args.out), flush=True)
    elif args.cmd == "train":
        train(args.data, args.out, args.epochs, batch=args.batch, beta=args.beta, first_only=args.first_only,
              smooth_k=args.smooth_k)
    else:
        summary, rows = evaluate(args.weights, args.start, args.count, args.lo, args.hi, args.min_conf, args.threads,
                                 args.out, args.policy)
        print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
