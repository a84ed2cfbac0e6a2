"""Autotuner for the batched Schur solver's per-size-class parameters.

For each size class of ``neig_schur_batched`` (problems of order up to
``n_hi``) it times the persistent launch on a sample batch drawn from that class
(half random N(0,1) Hessenberg, half prescribed-spectrum Hessenberg) for
candidate settings of the AED window ``nw``, the shifts per sweep ``ns``, the
size ``nmin`` below which a block goes to the in-LDS double-shift QR, and the
chase window ``chase_w`` (Section 3.2: these are the method's tunables), by
coordinate descent from the library's built-in table.  A candidate counts only
if every problem of the sample converges and meets the backward-error and
orthogonality bound 50 n eps (checked with FP64 products on the GPU).  The
winning table can be saved as JSON next to this file and applied with
:func:`apply_saved`.

Usage (on a GPU): ``python -m paper_2002_05024_amd.autotune --out <file>``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
SAVED = os.path.join(HERE, "tuned_batched_gfx950.json")
EPS = 2.0 ** -52

GRID = {
    "nw": [32, 48, 64, 80, 96],
    "ns": [8, 12, 16, 24, 32],
    "nmin": [32, 48, 64, 80, 96],
    "chase_w": [64, 80, 96],
}


def _valid(p) -> bool:
    return 3 * (p["ns"] // 2) + 2 <= p["chase_w"]


def sample_batch(lo: int, hi: int, count: int, seed: int):
    """``count`` problems with n uniform in [lo, hi] from the batched generators."""
    import numpy as np

    from . import inputs

    g = inputs.rng(inputs.BATCHED, 2_000_000 + 1000 * seed + lo)
    sizes = g.integers(lo, hi + 1, size=count)
    out = []
    for i, n in enumerate(sizes):
        H, _ = inputs.batched_problem(7000 + seed, i, int(n))
        out.append(H)
    return out, np.asarray(sizes)


class Bench:
    """Device copies of a sample batch and a timed, checked batched solve."""

    def __init__(self, Hs):
        import torch

        from . import binding

        self.torch = torch
        self.binding = binding
        dev = torch.device("cuda")
        self.H0 = [torch.from_numpy(h.T.copy()).to(dev).t() for h in Hs]
        self.call = binding.batched_tables([torch.empty_like(h) for h in self.H0],
                                           [torch.empty_like(h) for h in self.H0])
        self.eye = [torch.eye(h.shape[0], dtype=torch.float64, device=dev) for h in self.H0]

    def restore(self):
        for a, b in zip(self.call.Hs, self.H0):
            a.copy_(b)
        for a, b in zip(self.call.Zs, self.eye):
            a.copy_(b)

    def run(self, reps: int = 2):
        """Mean seconds per batched launch (HIP events on the current stream) and
        whether every problem converged within 50 n eps."""
        torch = self.torch
        times = []
        for _ in range(reps):
            self.restore()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            self.binding.launch_batched(self.call)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1000.0)
        ok = bool((self.call.info == 0).all().item()) and self.worst_error() <= 50.0 * EPS
        return sum(times) / len(times), ok

    def worst_error(self) -> float:
        """max over problems of max(backward error, orthogonality) / n."""
        torch = self.torch
        worst = 0.0
        for H0, S, Z in zip(self.H0, self.call.Hs, self.call.Zs):
            n = H0.shape[0]
            R = Z @ S @ Z.t() - H0
            be = float(torch.linalg.norm(R) / torch.linalg.norm(H0))
            E = Z.t() @ Z
            E.diagonal().sub_(1.0)
            oe = float(torch.linalg.norm(E))
            worst = max(worst, be / n, oe / n)
        return worst


def _set_all(binding, p):
    binding.set_batched_tune([1 << 30], [p["nw"]], [p["ns"]], [p["nmin"]], [p["chase_w"]])


def tune_class(lo: int, hi: int, start: dict, count: int, passes: int = 2, log=print):
    """Coordinate descent over GRID for problems with n in [lo, hi]."""
    from . import binding

    Hs, _ = sample_batch(lo, hi, count, 0)
    bench = Bench(Hs)
    best = dict(start)
    _set_all(binding, best)
    t_best, ok = bench.run()
    if not ok:
        t_best = float("inf")
    log(f"  [{lo},{hi}] start {best} {t_best * 1e3:.2f} ms ok={ok}")
    for _ in range(passes):
        changed = False
        for key, values in GRID.items():
            for v in values:
                if v == best[key]:
                    continue
                cand = dict(best, **{key: v})
                if not _valid(cand):
                    continue
                _set_all(binding, cand)
                t, ok = bench.run()
                log(f"  [{lo},{hi}] {key}={v}: {t * 1e3:.2f} ms ok={ok}")
                if ok and t < 0.98 * t_best:
                    best, t_best, changed = cand, t, True
        if not changed:
            break
    return best, t_best


def tune(classes=((32, 96), (97, 256), (257, 512), (513, 768), (769, 1024)), count: int = 256, log=print):
    """Tune every class; returns the table in neig_set_batched_tune's form."""
    from . import binding

    base = binding.get_batched_tune()
    table = {"n_hi": [], "nw": [], "ns": [], "nmin": [], "chase_w": [], "ms": []}
    for k, (lo, hi) in enumerate(classes):
        start = {f: base[f][min(k, len(base[f]) - 1)] for f in ("nw", "ns", "nmin", "chase_w")}
        best, t = tune_class(lo, hi, start, count, log=log)
        table["n_hi"].append(hi)
        for f in ("nw", "ns", "nmin", "chase_w"):
            table[f].append(best[f])
        table["ms"].append(round(t * 1e3, 3))
        log(f"class [{lo},{hi}] -> {best} {t * 1e3:.2f} ms")
    apply(table)
    return table


def apply(table) -> None:
    """Install a table (dict with n_hi, nw, ns, nmin, chase_w lists)."""
    from . import binding

    binding.set_batched_tune(table["n_hi"], table["nw"], table["ns"], table["nmin"], table["chase_w"])


def apply_saved(path: str = SAVED) -> bool:
    """Install the saved table if there is one; returns whether it did."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        apply(json.load(f))
    return True


def main():
    ap = argparse.ArgumentParser(description="tune the batched solver's size classes")
    ap.add_argument("--out", default=SAVED)
    ap.add_argument("--count", type=int, default=256, help="problems per class sample")
    args = ap.parse_args()

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t0 = time.time()
    table = tune(count=args.count, log=log)
    table["device"] = "gfx950"
    table["seconds"] = round(time.time() - t0, 1)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table), flush=True)


if __name__ == "__main__":
    main()
