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
events on the call's stream, which gives the live per-launch durations behind
the roofline figures: the dominant kernel on this input is the AED window
kernel (a latency-bound FP64 chain on one CU per launch); the FP64-MFMA update
kernel is reported beside it.  A second leg runs the batched workload (512
problems of order 32..1024 in one graph-captured launch) and the same problems
through the single-problem call.

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
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak: 256 CUs x 128 flops/clock x 2.4 GHz
CUS = 256
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
    ap.add_argument("--cpu-n", type=str, default="500,1000,2000",
                    help="orders of the oracle's bounded CPU samples (a n^3 is fitted to them)")
    ap.add_argument("--batched", type=int, default=1, help="also run the batched workload")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--plain-loop", type=int, default=128,
                    help="time this many of the batch's problems solved one neig_schur call at a time")
    ap.add_argument("--single", type=int, default=1, help="run the n=20000 single-matrix workload")
    ap.add_argument("--reorder", type=int, default=1, help="also time the eigenvalue reordering at n=4000")
    ap.add_argument("--hessenberg", type=int, default=20000,
                    help="order of the dense matrix for the Hessenberg-reduction leg (0 skips it)")
    ap.add_argument("--learned", type=int, default=9,
                    help="held-out matrices (n in [1000, 3000]) for the proposal-network leg (0 skips it)")
    ap.add_argument("--plain256", type=int, default=1,
                    help="the n=256 plain workload: GPU and oracle (one core), median of 5")
    ap.add_argument("--hard", type=int, default=20000,
                    help="order of the paper-comparable leg: Hessenberg form (by this library) of a dense "
                         "uniform[-1,1] matrix (0 skips it)")
    ap.add_argument("--prescribed", type=int, default=4000,
                    help="order of the prescribed-spectrum leg (as written and well-conditioned; 0 skips it)")
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


def cpu_baseline(samples, n_target):
    """The oracle (plain single-threaded C, double-shift Francis QR) on bounded
    samples of the same workload -- one random N(0,1) Hessenberg matrix per order
    in ``samples`` -- with t = a n^3 fitted to them (least squares) and
    evaluated at the target order."""
    import numpy as np

    import oracle
    from paper_2002_05024_amd import inputs

    oracle.build() if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")) else None
    ns, ts = [], []
    for n_sample in samples:
        H = inputs.random_hessenberg(n_sample, inputs.rng(inputs.FULL, 1000 + n_sample))
        t0 = time.perf_counter()
        S, Z, wr, wi, info = oracle.schur(H)
        ts.append(time.perf_counter() - t0)
        ns.append(n_sample)
        print(f"[bench] oracle n={n_sample} {ts[-1]:.2f}s info={info}", file=sys.stderr, flush=True)
    x = np.array(ns, dtype=float) ** 3
    a = float(np.dot(x, ts) / np.dot(x, x))
    return {
        "value": a * n_target ** 3,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": "one random N(0,1) Hessenberg matrix per order "
                  + ", ".join(f"n={k}: {t:.2f} s" for k, t in zip(ns, ts))
                  + f"; value = a n^3 at n={n_target} with a = {a:.3e} s fitted by least squares (an extrapolation)",
    }


KERNEL_SOURCES = {"k_aed": "small.hip", "k_small_qr": "small.hip", "k_update_p": "gemm.hip", "k_chase": "chase.hip"}


def kernel_source_sha(kernel):
    """Hash of the source file that defines ``kernel`` and the shared device
    header: a counter summary holds only for the source it was taken on."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2002_05024_amd", "csrc")
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kernel], "neig_dev.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain
    copy of known size), or None when there is none for the current source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_n20000.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha") != kernel_source_sha(kernel):
        return None
    return k["bytes_per_launch"]


def rooflines(stats):
    """Roofline figures of the kernels from the library's per-launch HIP event
    timing: the dominant kernel (most GPU time) as ``roofline``, the others
    beside it.  Algorithmic work per launch: k_aed 10 nw^3 flops (window Schur
    form), k_update 2 w^2 len flops per task, k_chase the bytes of its windows
    (load and store of the window of H, store of U)."""
    aed_ms = sum(s["gpu_aed_ms"] for s in stats)
    # k_aed launches (one or two windows each), including those inside the
    # recursive solves of wide windows
    aed_n = sum(s["aed_launches"] for s in stats)
    aed_fl = sum(s["aed_flops"] for s in stats)
    upd_ms = sum(s["gpu_update_ms"] for s in stats)
    upd_n = sum(s["n_update"] for s in stats)
    upd_fl = sum(s["gemm_flops"] for s in stats)
    out = {}
    if aed_ms > 0:
        ach = aed_fl / (aed_ms / 1000.0) / 1e12
        tr = traffic_per_launch("k_aed")
        out["roofline_aed"] = {
            "kernel": "k_aed", "bound": "alu", "achieved": round(ach, 5), "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / FP64_VECTOR_PEAK_TFLOPS, 7),
            "traffic": tr,
            "avg_launch_us": round(aed_ms * 1000.0 / max(aed_n, 1), 1),
            "flops_per_launch": round(aed_fl / max(aed_n, 1), 1),
            "frac_of_one_cu": round(ach / (FP64_VECTOR_PEAK_TFLOPS / CUS), 5),
        }
    if upd_ms > 0:
        ach = upd_fl / (upd_ms / 1000.0) / 1e12
        out["roofline_update"] = {
            "kernel": "k_update_p", "bound": "mfma", "achieved": round(ach, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / FP64_MFMA_PEAK_TFLOPS, 4),
            "traffic": traffic_per_launch("k_update_p"),
            "avg_launch_us": round(upd_ms * 1000.0 / max(upd_n, 1), 2),
            "flops_per_launch": round(upd_fl / max(upd_n, 1), 1),
        }
        far_ms = sum(s["gpu_update_far_ms"] for s in stats)
        if far_ms > 0:
            # the far parts of overlapped sweep steps, which run beside the next
            # chase launch (included in the figures above)
            far_fl = sum(s["gemm_flops_far"] for s in stats)
            far_n = sum(s["n_update_far"] for s in stats)
            fach = far_fl / (far_ms / 1000.0) / 1e12
            out["roofline_update"]["far_part"] = {
                "achieved": round(fach, 3), "frac": round(fach / FP64_MFMA_PEAK_TFLOPS, 4),
                "launches": int(far_n), "avg_launch_us": round(far_ms * 1000.0 / max(far_n, 1), 2),
                "flop_share": round(far_fl / max(upd_fl, 1.0), 4),
            }
    ch_ms = sum(s["gpu_chase_ms"] for s in stats)
    ch_n = sum(s["n_chase"] for s in stats)
    ch_b = sum(s["chase_bytes"] for s in stats)
    if ch_ms > 0:
        ach = ch_b / (ch_ms / 1000.0) / 1e9
        out["roofline_chase"] = {
            "kernel": "k_chase", "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
            "traffic": traffic_per_launch("k_chase"),
            "avg_launch_us": round(ch_ms * 1000.0 / max(ch_n, 1), 1),
            "bytes_per_launch": round(ch_b / max(ch_n, 1), 1),
            "note": "latency-bound window chase (dependent bulge steps in LDS); HBM is not its limit",
        }
    dominant = "roofline_aed" if aed_ms >= upd_ms else "roofline_update"
    if dominant in out:
        out["roofline"] = dict(out[dominant])
    return out


def timed_solve(H0, dev, reps):
    """Median GPU seconds of neig_schur on a copy of H0 (events on the current
    stream, Z from I; H restored and Z reset untimed before each run) after one
    warm-up, with the last run's stats and result."""
    import torch

    from paper_2002_05024_amd import binding

    n = H0.shape[0]
    H = torch.empty_like(H0)
    Z = torch.empty_like(H0)
    times, stats, r = [], [], None
    for k in range(reps + 1):
        H.copy_(H0)
        Z.zero_()
        Z.diagonal().fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = binding.schur(H, Z)
        e1.record()
        torch.cuda.synchronize()
        if r.info != 0:
            raise SystemExit(f"n={n}: info={r.info}")
        if k > 0:
            times.append(e0.elapsed_time(e1) / 1000.0)
            stats.append(binding.get_stats())
    times.sort()
    return times[len(times) // 2], stats[-1], H, Z, r


def plain256_leg(args, dev):
    """The plain n = 256 workload (random N(0,1) Hessenberg, seed 0, Z from I):
    GPU median of 5 after one warm-up, and the oracle on one host core, median
    of 5, beside it."""
    import numpy as np
    import torch

    import oracle
    from paper_2002_05024_amd import inputs

    n = 256
    H = inputs.random_hessenberg(n, inputs.rng(inputs.PLAIN, 0))
    H0 = torch.from_numpy(np.ascontiguousarray(H.T)).to(dev).t()
    sec, st, S, Z, _ = timed_solve(H0, dev, 5)
    be, oe = backward_and_orth(H0, S, Z)
    tc = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.schur(H)
        tc.append(time.perf_counter() - t0)
    tc.sort()
    return {"workload": "random N(0,1) Hessenberg, n=256, Z from I", "gpu_s": round(sec, 5),
            "oracle_s_one_core": round(tc[2], 4), "gpu_over_oracle_speedup": round(tc[2] / sec, 2),
            "aeds": st["aeds"], "small_solves": st["small_solves"],
            "check": {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52}}


def prescribed_leg(args, dev):
    """The prescribed-spectrum workload: A = U T U^T with 2000 eigenvalues in the
    unit disk (half as conjugate pairs), in Hessenberg form, Z from I; once with
    the strictly upper part of T drawn with standard deviation 0.1 (as written)
    and once with 0.1/sqrt(n) (well-conditioned).  Seconds (median of 3) and the
    method's algorithmic GFLOP/s; the well-conditioned case's eigenvalues are
    checked against the prescribed ones."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import inputs

    from paper_2002_05024_amd import autotune_single, binding

    n = args.prescribed
    saved = binding.get_params()
    tuned = autotune_single.apply(n)
    out = {"params": dict(tuned or {}, source="autotuned table" if tuned else "library defaults")}
    for tag, std, idx in (("as_written_std_0.1", 0.1, 4200), ("well_conditioned_std_0.1_over_sqrt_n",
                                                              0.1 / np.sqrt(n), 4201)):
        t0 = time.perf_counter()
        H, lam = inputs.prescribed_hessenberg(n, inputs.rng(inputs.PRESCRIBED, idx), std)
        print(f"[bench] prescribed {tag} n={n} input in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)
        H0 = torch.from_numpy(np.ascontiguousarray(H.T)).to(dev).t()
        sec, st, S, Z, r = timed_solve(H0, dev, 3)
        be, oe = backward_and_orth(H0, S, Z)
        rec = {"seconds": round(sec, 4), "gflops_algorithmic": round(st["alg_flops"] / sec / 1e9, 1),
               "aeds": st["aeds"], "sweeps": st["sweeps"],
               "check": {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52}}
        if std < 0.1:  # well-conditioned: every eigenvalue against the prescribed spectrum
            got = r.wr.cpu().numpy() + 1j * r.wi.cpu().numpy()

            def key(z):
                return z[np.lexsort((np.sign(z.imag), np.abs(z.imag), z.real))]

            rec["max_eigenvalue_error_vs_prescribed"] = float(np.max(np.abs(key(got) - key(np.asarray(lam)))))
        out[tag] = rec
        del H0, S, Z
        torch.cuda.empty_cache()
    binding.set_params(**saved)
    out["workload"] = (f"prescribed spectrum, n={n}: {n - 2 * (n // 4)} real eigenvalues and {n // 4} conjugate "
                       "pairs in the unit disk, Hessenberg form, Z from I")
    return out


def hard_leg(args, dev):
    """The paper's own kind of input (Section 5: Hessenberg forms of dense
    matrices with entries uniform in [-1, 1]), reduced to Hessenberg form by
    this library's neig_hessenberg (untimed), then one timed Schur reduction with
    Z from I.  On this input the subdiagonal decays and aggressive early
    deflation finds little, so sweeps and their off-diagonal updates carry the
    time; the update kernels' roofline is reported from the library's per-launch
    event timing.  The paper's figure for this order (another machine) is quoted
    as context."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import binding, inputs

    n = args.hard
    t0 = time.perf_counter()
    g = inputs.rng(inputs.FULL, 31)
    A = torch.from_numpy(g.uniform(-1.0, 1.0, (n, n))).to(dev).t()  # column-major view of the row-major fill
    binding.hessenberg(A)
    A.triu_(-1)
    torch.cuda.synchronize()
    print(f"[bench] hard input n={n} ready in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    from paper_2002_05024_amd import autotune_single

    saved = binding.get_params()
    table = autotune_single.load()
    hp = None
    if table and "hard_optimum" in table:
        hp = {k: table["hard_optimum"][k] for k in autotune_single.KEYS if k in table["hard_optimum"]}
        binding.set_params(**hp)
    H = A.clone(memory_format=torch.preserve_format)
    Z = torch.zeros_like(A)

    def solve(timing):
        binding.set_params(timing=timing)
        H.copy_(A)
        Z.zero_()
        Z.diagonal().fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = binding.schur(H, Z)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1000.0, r, binding.get_stats()

    sec, r, st = solve(0)
    print(f"[bench] hard n={n} {sec:.2f}s info={r.info}", file=sys.stderr, flush=True)
    kst = None
    if args.timing:  # a second reduction with HIP events around every launch, for the kernel figures
        _, _, kst = solve(1)
    binding.set_params(**saved)
    out = {"workload": f"Hessenberg form (neig_hessenberg) of a dense uniform[-1,1] matrix, n={n}, Z from I",
           "seconds": round(sec, 3), "info": r.info,
           "params": dict(hp, source="autotuned on another matrix of this kind (n=8000)") if hp else
           {"source": "library defaults"},
           "gflops_algorithmic": round(st["alg_flops"] / sec / 1e9, 1),
           "gflops_update_executed": round(st["gemm_flops"] / sec / 1e9, 1),
           "counts": {"sweeps": st["sweeps"], "aeds": st["aeds"], "shifts": st["shifts_used"],
                      "aed_deflated": st["aed_deflated"]},
           "paper_context": "Table 3, n=20000: StarNEig 85 s on 28 Broadwell cores (one node), ScaLAPACK 158 s"}
    if kst:
        out.update(rooflines([kst]))
        out["gpu_ms"] = {k: round(kst[f"gpu_{k}_ms"], 1) for k in ("update", "chase", "aed", "small", "other")}
    if args.check:
        be, oe = backward_and_orth(A, H, Z)
        out["check"] = {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52}
    del A, H, Z
    torch.cuda.empty_cache()
    return out


def reorder_leg(args, dev):
    """Eigenvalue reordering at the prescribed-spectrum size: the Schur form of a
    4000 x 4000 prescribed-spectrum Hessenberg matrix (well-conditioned strictly
    upper part), then every eigenvalue with negative real part moved to the
    leading block; timed with events around neig_reorder alone."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import binding, inputs

    n = 4000
    H, _ = inputs.prescribed_hessenberg(n, inputs.rng(inputs.PRESCRIBED, 4100), 0.1 / np.sqrt(n))
    Hd = torch.from_numpy(np.ascontiguousarray(H.T)).to(dev).t()
    r = binding.schur(Hd)
    sel = (r.wr.cpu().numpy() < 0).astype(np.int32)
    S0, Z0 = Hd.clone(), r.Z.clone()
    times = []
    for _ in range(2):
        S, Z = S0.clone(), Z0.clone()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wr, wi, m, info = binding.reorder(S, Z, sel)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1000.0)
    st = binding.get_stats()
    return {"workload": f"reorder the Schur form of a prescribed-spectrum Hessenberg matrix, n={n}: "
                        f"{m} eigenvalues with negative real part to the leading block",
            "seconds": round(min(times), 4), "selected": m, "info": info, "windows": st["small_solves"],
            "gflops_update_executed": round(st["gemm_flops"] / min(times) / 1e9, 2)}


def hessenberg_leg(args, dev):
    """Hessenberg reduction of a dense N(0,1) matrix (the step before the Schur
    reduction), Q1 accumulated from the identity; one warm-up at a small order,
    then one timed reduction (events around neig_hessenberg) and the
    backward-error / orthogonality check with GPU products."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import binding, inputs

    n = args.hessenberg
    w = torch.from_numpy(np.ascontiguousarray(inputs.rng(inputs.FULL, 77).standard_normal((256, 256)))).to(dev)
    binding.hessenberg(w.t().contiguous().t())
    g = inputs.rng(inputs.FULL, 78)
    A0 = torch.from_numpy(g.standard_normal((n, n))).to(dev).t()  # column-major view of the row-major fill
    A = A0.clone(memory_format=torch.preserve_format)
    Q = torch.eye(n, dtype=torch.float64, device=dev).t()  # column-major view
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    binding.hessenberg(A, Q)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1000.0
    flops = 10.0 / 3.0 * n ** 3
    gemv_bytes = 8.0 * n ** 3 / 3.0  # each column's product reads the trailing block once
    out = {"workload": f"Hessenberg reduction of a dense N(0,1) matrix, n={n}, Q1 accumulated",
           "seconds": round(sec, 3), "gflops_reduction": round(flops / sec / 1e9, 1),
           "gemv_bytes_algorithmic": gemv_bytes, "gemv_hbm_floor_s": round(gemv_bytes / 8e12, 3),
           "paper_context": "Table 2, n=20000: 53 s (14 Xeon Gold 6132 cores + Tesla V100), 49 s MAGMA"}
    if args.check:
        nrm = torch.linalg.norm(A0)
        R = Q @ A
        R = R @ Q.t()
        R -= A0
        be = float(torch.linalg.norm(R) / nrm)
        del R
        E = Q.t() @ Q
        E.diagonal().sub_(1.0)
        oe = float(torch.linalg.norm(E))
        del E
        out["check"] = {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52,
                        "below_subdiagonal_zero": bool(float(torch.tril(A, -2).abs().max()) == 0.0)}
    del A, A0, Q
    torch.cuda.empty_cache()
    return out


def learned_leg(args, dev):
    """The proposal network against the default rules on the first held-out
    matrices of the learned workload (three families, n in [1000, 3000] to keep
    the leg short), each solved both ways; GPU time by HIP events, every result
    checked (backward error and orthogonality <= 50 n eps)."""
    import os

    from paper_2002_05024_amd import learn

    if not os.path.exists(learn.SAVED):
        return {"skipped": "no trained network"}
    summary, rows = learn.evaluate(learn.SAVED, 0, args.learned, 1000, 3000, 0.0, 8)
    return {"workload": f"{len(rows)} held-out matrices (random / prescribed / graded), n in [1000, 3000]",
            "default_s": round(summary["total_default_s"], 3), "network_s": round(summary["total_net_s"], 3),
            "speedup": round(summary["speedup"], 3), "all_within_50n_eps": summary["all_ok"],
            "per_family": {f: {k: round(v, 3) for k, v in d.items()} for f, d in summary["per_family"].items()},
            "policy": learn.POLICY}


def batched_leg(args, dev):
    """The batched workload: ``batch_count`` problems with n uniform in [32, 1024],
    half random N(0,1) Hessenberg and half prescribed-spectrum Hessenberg, Z from
    I, all resident in HBM, solved by one neig_schur_batched launch captured in a
    HIP graph.  Each timed step restores the inputs (untimed), then replays the
    graph between two events.  Optionally the same problems are solved one by one
    with neig_schur (the plain GPU form) for comparison."""
    import numpy as np
    import torch

    from paper_2002_05024_amd import autotune, binding, inputs

    t0 = time.perf_counter()
    Hs, _ = inputs.batched_workload(args.batch_count, args.seed, threads=min(16, os.cpu_count() or 1))
    sizes = np.array([h.shape[0] for h in Hs])
    H0 = [torch.from_numpy(np.ascontiguousarray(h.T)).to(dev).t() for h in Hs]
    del Hs
    eye = [torch.eye(int(k), dtype=torch.float64, device=dev) for k in sizes]
    tuned = autotune.apply_saved()
    call = binding.batched_tables([torch.empty_like(h) for h in H0], [torch.empty_like(h) for h in H0])
    print(f"[bench] batch of {len(sizes)} ready in {time.perf_counter() - t0:.1f}s (tuned table: {tuned})",
          file=sys.stderr, flush=True)

    def restore():
        for a, b in zip(call.Hs, H0):
            a.copy_(b)
        for a, b in zip(call.Zs, eye):
            a.copy_(b)
        torch.cuda.synchronize()

    restore()
    binding.launch_batched(call)  # eager warm-up
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        binding.launch_batched(call, stream=side)
    torch.cuda.synchronize()
    times = []
    for k in range(args.batch_steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1000.0)
        print(f"[bench] batched step {k} {times[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    info = call.info.cpu().numpy()
    flops = binding.batched_flops()  # counted on the device by the last replay
    worst_be = worst_oe = 0.0
    for h0, S, Z in zip(H0, call.Hs, call.Zs):
        n = h0.shape[0]
        R = torch.mm(torch.mm(Z, S), Z.t())
        R.sub_(h0)
        worst_be = max(worst_be, float(torch.linalg.norm(R) / torch.linalg.norm(h0)) / (n * 2.0 ** -52))
        E = torch.mm(Z.t(), Z)
        E.diagonal().sub_(1.0)
        worst_oe = max(worst_oe, float(torch.linalg.norm(E)) / (n * 2.0 ** -52))
    sec = sum(times) / len(times)
    out = {
        "workload": f"{len(sizes)} Hessenberg problems, n uniform in [32, 1024] (mean {sizes.mean():.0f}), "
                    "half random N(0,1), half prescribed spectrum; Z from I; one graph-captured launch",
        "solves_per_s": round(len(sizes) / sec, 2),
        "ms_per_batch": round(sec * 1e3, 2),
        "steps": args.batch_steps,
        "all_converged": bool((info == 0).all()),
        "worst_backward_error_over_n_eps": round(worst_be, 4),
        "worst_orthogonality_over_n_eps": round(worst_oe, 4),
        "tuned_table": tuned,
        "flops_algorithmic_per_batch": flops,
        "gflops_algorithmic": round(flops / sec / 1e9, 1),
        # one problem per workgroup, each a latency-bound chain on its compute
        # unit: the FP64 vector peak of the chip is the roof it is measured against
        "roofline": {"kernel": "k_batched", "bound": "alu", "achieved": round(flops / sec / 1e12, 4),
                     "peak": 78.6, "unit": "TFLOP/s", "frac": float(f"{flops / sec / 78.6e12:.3g}"),
                     "traffic": None, "avg_launch_us": round(sec * 1e6, 1), "flops_per_launch": flops,
                     "note": "method's operation count, counted on the device by the batched kernel"},
    }
    if args.plain_loop:
        t_plain = 0.0
        restore()
        k = min(args.plain_loop, len(sizes))
        for i in range(k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            r = binding.schur(call.Hs[i], call.Zs[i])
            e1.record()
            torch.cuda.synchronize()
            t_plain += e0.elapsed_time(e1) / 1000.0
            if r.info != 0:
                out["plain_unconverged"] = out.get("plain_unconverged", 0) + 1
        out["plain_loop_solves_per_s"] = round(k / t_plain, 2)
        out["plain_loop_problems"] = f"the first {k} problems of the batch (same size mix), one neig_schur each"
        out["speedup_vs_plain_loop"] = round((len(sizes) / sec) / (k / t_plain), 2)
        print(f"[bench] plain loop {t_plain:.2f}s", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the library runs on a single GPU (multi-GPU sharding is designed, not implemented); --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch

    from paper_2002_05024_amd import binding

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    binding.load_library()
    if not args.single:
        line = {"metric": "Schur reduction seconds + FP64 GFLOP/s at n=20000; batched solves/sec",
                "n_gpus": 1, "dtype": "f64", "data": "synthetic"}
        if args.hard:
            line["hard"] = hard_leg(args, dev)
        if args.plain256:
            line["plain256"] = plain256_leg(args, dev)
        if args.prescribed:
            line["prescribed"] = prescribed_leg(args, dev)
        if args.batched:
            line["batched"] = batched_leg(args, dev)
        if args.reorder:
            line["reorder"] = reorder_leg(args, dev)
        if args.hessenberg:
            line["hessenberg"] = hessenberg_leg(args, dev)
        if args.learned:
            line["learned"] = learned_leg(args, dev)
        print(json.dumps(line), flush=True)
        return
    n = args.n
    t_gen = time.perf_counter()
    H0 = make_input(n, args.seed, dev)
    H = torch.empty_like(H0)
    Z = torch.empty_like(H0)
    print(f"[bench] input n={n} ready in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    saved = binding.get_params()
    from paper_2002_05024_amd import autotune_single

    tuned = autotune_single.apply(n)  # the tuned parameters of this order's bucket, when a table is saved
    binding.set_params(timing=0)

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
    kstats = []
    if args.timing:
        # one more reduction, outside the timed steps, with HIP events around
        # every launch: the per-kernel durations behind the roofline figures
        # (the events add host work, so the timed steps run without them)
        binding.set_params(timing=1)
        restore()
        r = binding.schur(H, Z)
        torch.cuda.synchronize()
        kstats.append(binding.get_stats())
        binding.set_params(timing=0)
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
        "params": dict(tuned or {}, source="autotuned table (paper_2002_05024_amd/tuned_single_gfx950.json)"
                       if tuned else "library defaults"),
    }
    if kstats:
        line.update(rooflines(kstats))
        line["gpu_ms_per_step"] = {k: round(sum(s[f"gpu_{k}_ms"] for s in kstats) / len(kstats), 1)
                                   for k in ("update", "chase", "aed", "small", "other")}
        line["gpu_ms_per_step"]["note"] = "one extra reduction with HIP events around every launch"
    if args.check:
        be, oe = backward_and_orth(H0, H, Z)
        line["check"] = {"backward_error": be, "orthogonality": oe, "bound_50n_eps": 50 * n * 2.0 ** -52}
    if args.batched or args.reorder or args.hessenberg or args.learned or args.plain256 or args.prescribed or \
            args.hard:
        del H, Z, H0
        torch.cuda.empty_cache()
    if args.hard:
        line["hard"] = hard_leg(args, dev)
    if args.plain256:
        line["plain256"] = plain256_leg(args, dev)
    if args.prescribed:
        line["prescribed"] = prescribed_leg(args, dev)
    if args.batched:
        line["batched"] = batched_leg(args, dev)
    if args.reorder:
        line["reorder"] = reorder_leg(args, dev)
    if args.hessenberg:
        line["hessenberg"] = hessenberg_leg(args, dev)
    if args.learned:
        line["learned"] = learned_leg(args, dev)
    if args.cpu_baseline:
        line["cpu_baseline"] = cpu_baseline([int(v) for v in args.cpu_n.split(",") if v], n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
