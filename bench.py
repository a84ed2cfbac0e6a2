#!/usr/bin/env python3
"""Schur-reduction benchmark on one MI355X.

Workload: the full-size case -- a random upper Hessenberg matrix of order
n = 20000 (entries on and above the subdiagonal N(0,1), seeded), FP64, with Z
accumulated from the identity; H and Z (3.2 GB each) resident in HBM.

A step is one complete Schur reduction (neig_schur: every AED, sweep, small
solve and the final read-out).  Before each step, untimed, H is restored from a
pristine device copy and Z reset to I.  W warm-up steps, then K timed steps,
each bracketed by synchronisations; the reported value is the mean seconds per
reduction.  The library's timing mode brackets each kernel launch with HIP
events on the call's stream, which gives the live duration of the dominant
kernel (the FP64-MFMA off-diagonal update) for the roofline figure.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--timing", type=int, default=1, help="per-kernel HIP event timing inside the library")
    ap.add_argument("--check", type=int, default=1, help="backward error / orthogonality of the last step")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-n", type=int, default=1200, help="order of the oracle's bounded CPU sample")
    return ap.parse_args()


def make_input(n, seed, device):
    """Random N(0,1) upper Hessenberg, generated on the host with the shared seeded
    generator (row-major fill), stored column-major on the device."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import inputs

    g = inputs.rng(inputs.FULL, seed)
    G = g.standard_normal((n, n))  # row-major fill, same recipe as inputs.random_hessenberg
    Gd = torch.from_numpy(G).to(device)
    del G
    H0 = Gd.t().contiguous().t()  # column-major: element (i, j) at i + j*n
    del Gd
    H0.triu_(-1)
    torch.cuda.synchronize()
    return H0


def backward_and_orth(H0, S, Z):
    """||H0 - Z S Z^T||_F / ||H0||_F and ||Z^T Z - I||_F of the last step, with
    torch FP64 matrix products (a check of the result, outside the timed region)."""
    import torch

    nh = torch.linalg.norm(H0)
    R = torch.mm(torch.mm(Z, S), Z.t())
    R.sub_(H0)
    be = float(torch.linalg.norm(R) / nh)
    del R
    E = torch.mm(Z.t(), Z)
    E.diagonal().sub_(1.0)
    oe = float(torch.linalg.norm(E))
    del E
    torch.cuda.synchronize()
    return be, oe


def cpu_baseline(n_sample, n_target):
    """The oracle (plain single-threaded C, double-shift Francis QR) on a bounded
    sample of the same workload, scaled to the target order by n^3."""
    import oracle
    from paper_2002_05024_amd import inputs

    oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
    H = inputs.random_hessenberg(n_sample, inputs.rng(inputs.FULL, 1000 + n_sample))
    t0 = time.perf_counter()
    S, Z, wr, wi, info = oracle.schur(H)
    dt = time.perf_counter() - t0
    scale = (n_target / n_sample) ** 3
    return {
        "value": dt * scale,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one random N(0,1) Hessenberg matrix of order {n_sample} solved in {dt:.2f} s "
                  f"(info={info}); value = that time x ({n_target}/{n_sample})^3",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch

    from paper_2002_05024_amd import binding

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    binding.load_library()
    n = args.n
    t_gen = time.perf_counter()
    H0 = make_input(n, args.seed, dev)
    H = torch.empty_like(H0)
    Z = torch.empty_like(H0)
    print(f"[bench] input n={n} ready in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    saved = binding.get_params()
    binding.set_params(timing=int(args.timing))

    def restore():
        H.copy_(H0)
        Z.zero_()
        Z.diagonal().fill_(1.0)
        torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        restore()
        t0 = time.perf_counter()
        r = binding.schur(H, Z)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} {time.perf_counter() - t0:.2f}s info={r.info}", file=sys.stderr, flush=True)

    times, stats = [], []
    for k in range(args.steps):
        restore()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        r = binding.schur(H, Z)
        ev1.record(stream)
        torch.cuda.synchronize()
        dt = ev0.elapsed_time(ev1) / 1000.0
        times.append(dt)
        stats.append(binding.get_stats())
        print(f"[bench] step {k} {dt:.3f}s info={r.info}", file=sys.stderr, flush=True)
        if r.info != 0:
            raise SystemExit(f"step {k} did not converge: info={r.info}")
    binding.set_params(**saved)

    sec = sum(times) / len(times)
    st = stats[-1]
    alg_gflops = sum(s["alg_flops"] for s in stats) / sum(times) / 1e9
    exe_gflops = sum(s["gemm_flops"] for s in stats) / sum(times) / 1e9
    line = {
        "metric": "Schur reduction seconds + FP64 GFLOP/s at n=20000; batched solves/sec",
        "value": round(sec, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1000.0, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Schur reduction of a random N(0,1) upper Hessenberg matrix, n={n}, "
                               f"Z accumulated from I", "n": n, "seed": args.seed},
        "gflops_algorithmic": round(alg_gflops, 2),
        "gflops_update_executed": round(exe_gflops, 2),
        "phases_ms": {"aed_host": round(st["t_aed_ms"], 1), "sweep_host": round(st["t_sweep_ms"], 1),
                      "small_host": round(st["t_small_ms"], 1)},
        "counts": {"sweeps": st["sweeps"], "aeds": st["aeds"], "aed_deflated": st["aed_deflated"],
                   "shifts": st["shifts_used"], "exceptional": st["exceptional"],
                   "aed_qr_iters": st["aed_qr_iters"], "aed_swaps": st["aed_swaps"]},
        "aed_cycles_M": {k: round(st[f"aed_cyc_{k}"] / 1e6, 1) for k in ("qr", "defl", "hess")},
    }
    if args.timing:
        upd_ms = sum(s["gpu_update_ms"] for s in stats)
        upd_n = sum(s["n_update"] for s in stats)
        upd_flops = sum(s["gemm_flops"] for s in stats)
        achieved = upd_flops / (upd_ms / 1000.0) / 1e12 if upd_ms > 0 else 0.0
        line["roofline"] = {
            "kernel": "k_update",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
            "traffic": None,
            "avg_launch_us": round(upd_ms * 1000.0 / max(upd_n, 1), 2),
            "flops_per_launch": round(upd_flops / max(upd_n, 1), 1),
        }
        line["gpu_ms_per_step"] = {k: round(sum(s[f"gpu_{k}_ms"] for s in stats) / len(stats), 1)
                                   for k in ("update", "chase", "aed", "small", "other")}
    if args.check:
        be, oe = backward_and_orth(H0, H, Z)
        line["check"] = {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52}
    if args.cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
