"""Host model of the overlapped sweep schedule (no GPU).

A multishift sweep chases chains of bulges window by window (Section 3.2); each
chase step ends with update tasks: left strips (a window's rows, the columns
right of it), right strips (the rows above a window, its columns) and the Z
strips.  With overlap on, the library splits a step's updates into a near part
(run before the next chase launch) and a far part (run beside it, on a second
stream), and runs the next step's near part after that far part.  This model
rebuilds the windows of every step and the split exactly as `Solver::sweep`
does, applies random orthogonal window factors in the order the two streams
impose, and checks

* that the far part of a step meets no window of the next step (they run at
  the same time), and that the tasks of one launch never meet;
* that the result equals the one-stream order (each step's chase, then all
  of its left strips, then all right strips and Z).

The GPU tests check the library itself against the one-stream path bit for
bit; this one pins the rule: the naive split (cut every strip at the next
windows' rows/columns) breaks the second property, because a left strip and a
right strip that cross commute only as wholes.
"""
import itertools

import numpy as np
import pytest

MAX_CHAINS = 32


def chain_windows(ktop, kbot, ns, chain, wmax):
    """Each chain's windows (r0, r1): nb bulges three rows apart, a window
    advances until the chain's last bulge leaves it."""
    nbulge = ns // 2
    nbc = min(max(1, min(chain, min(32, (wmax - 2) // 3))), nbulge)
    nchain = (nbulge + nbc - 1) // nbc
    out = []
    for c in range(nchain):
        nb = min(nbc, nbulge - c * nbc)
        tend = kbot - 1 - ktop + 3 * (nb - 1)
        t, ws = 0, []
        while t <= tend:
            r0 = max(ktop, ktop + t - 3 * (nb - 1))
            r1 = min(kbot, r0 + wmax - 1)
            ws.append((r0, r1))
            t = r1 - 3 - ktop + 1 if r1 < kbot else tend + 1
        out.append(ws)
    return out


def schedule(wins):
    """Per step: the windows chased together (a chain joins when its window
    stays clear of the one ahead) and every chain's next window."""
    idx = [0] * len(wins)
    steps = []
    while True:
        prev_r0, prev_done, prev_ran = 0, True, False
        act, any_left = [], False
        for c, ws in enumerate(wins):
            if len(act) >= MAX_CHAINS:
                break
            if idx[c] >= len(ws):
                prev_done, prev_ran = True, False
                continue
            any_left = True
            r0, r1 = ws[idx[c]]
            if not (c == 0 or prev_done or (prev_ran and r1 < prev_r0 - 1)):
                break
            act.append((r0, r1))
            prev_r0, prev_done, prev_ran = r0, False, True
            idx[c] += 1
        if not any_left:
            return steps
        steps.append((act, [ws[idx[c]] for c, ws in enumerate(wins) if idx[c] < len(ws)]))


def rect(t):
    """Rows and columns of H a task covers (None for Z)."""
    kind, _, a, b, c, d = t
    return None if kind == "Z" else (a, b, c, d)


def meets(x, y):
    return x is not None and y is not None and x[0] <= y[1] and y[0] <= x[1] and x[2] <= y[3] and y[2] <= x[3]


def launches(tasks_l, tasks_r):
    """One launch when no left strip meets a right strip, else lefts first."""
    if any(meets(rect(x), rect(y)) for x in tasks_l for y in tasks_r):
        return [tasks_l, tasks_r]
    return [tasks_l + tasks_r]


def split(n, act, nxt, naive=False):
    """Near and far parts of a step's updates, as lists of launches."""
    lo, hi = n, -1
    for r0, r1 in nxt:
        lo, hi = min(lo, max(r0 - 1, 0)), max(hi, r1)
    hi_left = hi
    if not naive:
        for r0, r1 in act:
            if r0 <= hi:
                hi_left = max(hi_left, r1)
    ln, rn, lf, rf = [], [], [], []
    for k, (r0, r1) in enumerate(act):
        b0 = max(r0 - 1, 0)
        if r1 + 1 < n:  # left strip: rows r0..r1, columns r1+1..n-1
            if naive:
                cm = min(max(hi, r1), n - 1)
            else:
                cm = min(max(hi_left, r1), n - 1) if r1 >= lo else r1
            if cm >= r1 + 1:
                ln.append(("L", k, r0, r1, r1 + 1, cm))
            if cm + 1 < n:
                lf.append(("L", k, r0, r1, cm + 1, n - 1))
        if b0 > 0:  # right strip: rows 0..b0-1, columns r0..r1
            rm = min(lo, b0) if (naive or r0 <= hi) else b0
            if rm < b0:
                rn.append(("R", k, rm, b0 - 1, r0, r1))
            if rm > 0:
                rf.append(("R", k, 0, rm - 1, r0, r1))
        rf.append(("Z", k, 0, n - 1, r0, r1))
    return launches(ln, rn), launches(lf, rf)


def chase(H, U, act):
    for k, (r0, r1) in enumerate(act):
        b0 = max(r0 - 1, 0)
        H[r0:r1 + 1, b0:r1 + 1] = U[k].T @ H[r0:r1 + 1, b0:r1 + 1]
        H[b0:r1 + 1, r0:r1 + 1] = H[b0:r1 + 1, r0:r1 + 1] @ U[k]


def apply(H, Z, U, t):
    kind, k, a, b, c, d = t
    if kind == "L":
        H[a:b + 1, c:d + 1] = U[k].T @ H[a:b + 1, c:d + 1]
    elif kind == "R":
        H[a:b + 1, c:d + 1] = H[a:b + 1, c:d + 1] @ U[k]
    else:
        Z[a:b + 1, c:d + 1] = Z[a:b + 1, c:d + 1] @ U[k]


def run(n, ktop, kbot, ns, chain, wmax, seed, naive=False):
    rng = np.random.default_rng(seed)
    steps = schedule(chain_windows(ktop, kbot, ns, chain, wmax))
    Us = [[np.linalg.qr(rng.standard_normal((r1 - r0 + 1,) * 2))[0] for r0, r1 in act] for act, _ in steps]
    H0 = rng.standard_normal((n, n))
    # one stream
    H, Z = H0.copy(), np.eye(n)
    for (act, _), U in zip(steps, Us):
        chase(H, U, act)
        tl, tr = [], []
        for k, (r0, r1) in enumerate(act):
            b0 = max(r0 - 1, 0)
            if r1 + 1 < n:
                tl.append(("L", k, r0, r1, r1 + 1, n - 1))
            if b0 > 0:
                tr.append(("R", k, 0, b0 - 1, r0, r1))
            tr.append(("Z", k, 0, n - 1, r0, r1))
        for t in tl + tr:
            apply(H, Z, U, t)
    ref = (H, Z)
    # two streams: chase(s) beside far(s-1); near(s) after both
    H, Z = H0.copy(), np.eye(n)
    pending = None
    disjoint = True
    for (act, nxt), U in zip(steps, Us):
        chase(H, U, act)
        if pending is not None:
            far, Up = pending
            wins = [(max(r0 - 1, 0), r1, max(r0 - 1, 0), r1) for r0, r1 in act]
            for launch in far:
                for t in launch:
                    disjoint &= not any(meets(rect(t), w) for w in wins)
                    apply(H, Z, Up, t)
        near, far = split(n, act, nxt, naive)
        for launch in near + far:
            for x, y in itertools.combinations(launch, 2):
                assert not meets(rect(x), rect(y)), (x, y)
        for launch in near:
            for t in launch:
                apply(H, Z, U, t)
        pending = (far, U)
    for launch in pending[0]:
        for t in launch:
            apply(H, Z, pending[1], t)
    err = max(np.abs(H - ref[0]).max(), np.abs(Z - ref[1]).max())
    return err, disjoint, max(len(a) for a, _ in steps)


CASES = [(n, ktop, kbot, ns, chain, w)
         for n, ktop, kbot in [(160, 0, 159), (200, 7, 180), (120, 0, 60)]
         for ns, chain, w in [(2, 1, 16), (8, 1, 16), (16, 2, 16), (24, 4, 24), (48, 4, 24), (48, 8, 40),
                              (16, 8, 40)]]


@pytest.mark.parametrize("n,ktop,kbot,ns,chain,w", CASES)
def test_overlapped_schedule_matches_one_stream(n, ktop, kbot, ns, chain, w):
    err, disjoint, _ = run(n, ktop, kbot, ns, chain, w, seed=n + ns + w)
    assert disjoint
    assert err < 1e-10


def test_naive_split_is_wrong():
    """Cutting both strips at the next windows' rows and columns reorders a
    left and a right update that cross (rows of a window behind, columns of one
    ahead) part by part; with several chains this changes the result."""
    errs = []
    for n, ktop, kbot, ns, chain, w in CASES:
        err, disjoint, nmax = run(n, ktop, kbot, ns, chain, w, seed=n + ns + w, naive=True)
        assert disjoint  # the far parts still avoid the next windows
        if nmax > 1:
            errs.append(err)
    assert max(errs) > 1e-3
