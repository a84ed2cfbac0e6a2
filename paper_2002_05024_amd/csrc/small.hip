// small.hip -- one-workgroup kernels that keep a whole small matrix in LDS.
//
//  * k_small_qr: the double-shift QR iteration (the two-shift case of the bulge
//    chase in Section 3.2) on an m x m diagonal block, m <= NEIG_SMALL_MAX, with
//    its orthogonal factor accumulated in LDS.  Used for the final small active
//    blocks and for whole problems that fit.
//  * k_aed: aggressive early deflation (Section 3.2, "AED step") on a trailing
//    window that fits in LDS: window Schur form by the same QR, spike test of
//    every diagonal block from the bottom up, failing blocks moved to the top of
//    the window by swaps of adjacent diagonal blocks (the Bai-Demmel block swap
//    the paper cites), then a Householder Hessenberg reduction of the remaining
//    spike and undeflated part.
//
// Four waves per workgroup.  In the QR iteration the chain of bulge steps is
// latency-bound, so wave 0 runs it alone: each step updates only a near field
// around the bulge (one pass: a mixed 4x3 block on lane 0, the columns to its
// right and the rows above it on other lanes) and hands the next reflector's
// input to every lane through a register broadcast.  Waves 1-3 meanwhile apply
// the previous batch of FB reflectors to the far field (columns right of the
// near field, rows above it, and the accumulated orthogonal factor).  Other
// phases use all four waves with block barriers.
#include "neig_dev.h"
#include <climits>

#define NT 256     // threads per workgroup
#define LANES 64   // wavefront size
#define FB 16      // reflectors per near-field batch

// Optional section timers (compiled in with -DNEIG_PROF): shader clock cycles
// accumulated by thread 0 into g_prof[0..7].
#ifdef NEIG_PROF
__shared__ long long g_prof[8];
#define PROF_T(v) const long long v = clock64()
#define PROF_ADD(slot, t0) do { if (threadIdx.x == 0) g_prof[slot] += clock64() - (t0); } while (0)
#define PROF_CNT(slot, v) do { if (threadIdx.x == 0) g_prof[slot] += (v); } while (0)
#else
#define PROF_CNT(slot, v) do { } while (0)
#define PROF_T(v)
#define PROF_ADD(slot, t0) do { } while (0)
#endif

__device__ __forceinline__ double bcast_lane0(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void refl_apply3(double &a, double &b, double &c, double tau, double v1, double v2) {
    const double t = tau * (a + v1 * b + v2 * c);
    a -= t;
    b -= t * v1;
    c -= t * v2;
}

// Block-wide max / sum (all NT threads call; result in every thread).
__device__ __forceinline__ double block_reduce(double v, bool is_max) {
    __shared__ double red[NT / LANES];
    v = is_max ? wave_max(v) : wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & (LANES - 1)) == 0) red[threadIdx.x / LANES] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < NT / LANES; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
    return r;
}

// rows r, r+1 of M, columns c0..c1: (x, y) <- (cs x + sn y, -sn x + cs y)
__device__ __forceinline__ void lds_rot_rows(double *M, int ld, int r, int c0, int c1, double cs, double sn) {
    for (int j = c0 + (int)threadIdx.x; j <= c1; j += NT) {
        double x = AT(M, ld, r, j), y = AT(M, ld, r + 1, j);
        AT(M, ld, r, j) = cs * x + sn * y;
        AT(M, ld, r + 1, j) = -sn * x + cs * y;
    }
}

// columns c, c+1 of M, rows r0..r1
__device__ __forceinline__ void lds_rot_cols(double *M, int ld, int c, int r0, int r1, double cs, double sn) {
    for (int i = r0 + (int)threadIdx.x; i <= r1; i += NT) {
        double x = AT(M, ld, i, c), y = AT(M, ld, i, c + 1);
        AT(M, ld, i, c) = cs * x + sn * y;
        AT(M, ld, i, c + 1) = -sn * x + cs * y;
    }
}

// Standardise the 2x2 block at (j, j) of the m x m matrix T (rotation applied to
// whole rows and columns of T and to the columns of Q).
__device__ __forceinline__ void lds_standardise(double *T, int ldt, double *Q, int ldq, int m, int j) {
    Std2 o = std2x2(AT(T, ldt, j, j), AT(T, ldt, j, j + 1), AT(T, ldt, j + 1, j), AT(T, ldt, j + 1, j + 1));
    __syncthreads();
    if (!(o.cs == 1.0 && o.sn == 0.0)) {
        lds_rot_rows(T, ldt, j, j + 2, m - 1, o.cs, o.sn);
        lds_rot_cols(T, ldt, j, 0, j - 1, o.cs, o.sn);
        lds_rot_cols(Q, ldq, j, 0, m - 1, o.cs, o.sn);
    }
    if (threadIdx.x == 0) {
        AT(T, ldt, j, j) = o.a; AT(T, ldt, j, j + 1) = o.b;
        AT(T, ldt, j + 1, j) = o.c; AT(T, ldt, j + 1, j + 1) = o.d;
    }
    __syncthreads();
}

// Apply a batch of nb consecutive reflectors (positions k0..k0+nb-1) in order to
// segments of the far field: columns c_lo..c_hi of T (rows k0..k0+nb+1), rows
// 0..r_hi-1 of T (columns k0..k0+nb+1), and, if withq, every row of Q.  Work
// items are spread over threads t0, t0+nth, ...  The coefficients are read into
// registers once; segments of full length take a branch-free path.
__device__ __forceinline__ void far_apply(double *T, int ldt, double *Q, int ldq, int m, int k0, int nb, int c_lo, int c_hi,
                          int r_hi, bool withq, const double *rt, const double *r1, const double *r2, int t0, int nth) {
    const int ncol = (c_hi >= c_lo) ? c_hi - c_lo + 1 : 0;
    const int total = ncol + r_hi + (withq ? m : 0);
    if (t0 >= total) return;
    const int len = (k0 + nb + 2 <= m) ? nb + 2 : m - k0;
    double ct[FB], c1[FB], c2[FB];
#pragma unroll
    for (int t = 0; t < FB; ++t) {
        const bool on = t < nb;
        ct[t] = on ? rt[t] : 0.0;
        c1[t] = on ? r1[t] : 0.0;
        c2[t] = on ? r2[t] : 0.0;
    }
    const bool full = (len == FB + 2);
    for (int it = t0; it < total; it += nth) {
        double *base;
        int stride;
        if (it < ncol) {
            base = &AT(T, ldt, k0, c_lo + it);
            stride = 1;
        } else if (it < ncol + r_hi) {
            base = &AT(T, ldt, it - ncol, k0);
            stride = ldt;
        } else {
            base = &AT(Q, ldq, it - ncol - r_hi, k0);
            stride = ldq;
        }
        double x[FB + 2];
        if (full) {
#pragma unroll
            for (int t = 0; t < FB + 2; ++t) x[t] = base[t * stride];
#pragma unroll
            for (int t = 0; t < FB; ++t) refl_apply3(x[t], x[t + 1], x[t + 2], ct[t], c1[t], c2[t]);
#pragma unroll
            for (int t = 0; t < FB + 2; ++t) base[t * stride] = x[t];
        } else {
#pragma unroll
            for (int t = 0; t < FB + 2; ++t) x[t] = (t < len) ? base[t * stride] : 0.0;
#pragma unroll
            for (int t = 0; t < FB; ++t) refl_apply3(x[t], x[t + 1], x[t + 2], ct[t], c1[t], c2[t]);
#pragma unroll
            for (int t = 0; t < FB + 2; ++t)
                if (t < len) base[t * stride] = x[t];
        }
    }
}

// One bulge step, reflector on rows/columns k..k+M3-1 (M3 = 3, or 2 at the last
// step of a sweep), generated from (x0, x1, x2), recorded for the far field and
// applied to the near field.  Every lane of wave 0 runs the same instructions on
// a 3-vector of its own:
//   lane c (0..31)   column k-1+c, rows k..k+M3-1: c = 0 receives (beta, 0, 0)
//                    when k > l; columns k+M3..cnear take the left reflection;
//   lane 32+t        row k0+t <= min(k+3, i), columns k..k+M3-1: rows k..k+M3-1
//                    first take the left reflection of their entries (from the
//                    column sums of the M3 x M3 diagonal block, which every
//                    lane reads), then every row takes the right reflection.
// The loads come first so that their latency hides behind the reflector's
// dependent chain; only the stores are predicated.  The next generating vector
// (column k, rows k+1..k+3) comes back from the row lanes through readlane.
template <int M3>
__device__ __forceinline__ void near_step(double *T, int ldt, int l, int i, int k, int k0, int cnear, double *rt,
                                          double *r1, double *r2, double &x0, double &x1, double &x2) {
    const int lane = threadIdx.x;
    const int rmax = (k + 3 < i) ? k + 3 : i;
    const bool isRow = lane >= 32;
    const int col = k - 1 + lane;                 // column lanes
    const int row = k0 + lane - 32;               // row lanes
    const bool colOn = !isRow && lane > M3 && col <= cnear;
    const bool betaOn = (lane == 0) && (k > l);
    const bool rowOn = isRow && row <= rmax;
    // the lane's 3-vector as a word offset and stride (idle lanes read word 0
    // and store nothing); integer selects, no branches
    const int off = colOn ? col * ldt + k : (rowOn ? k * ldt + row : 0);
    const int vs = isRow ? ldt : 1;
    double *vec = T + off;
    double v[3];
#pragma unroll
    for (int a = 0; a < M3; ++a) v[a] = vec[a * vs];
    double blk[M3][M3];  // the diagonal block, same addresses for every lane
#pragma unroll
    for (int a = 0; a < M3; ++a)
#pragma unroll
        for (int b = 0; b < M3; ++b) blk[a][b] = AT(T, ldt, k + a, k + b);
    Refl r = make_refl(x0, x1, (M3 == 3) ? x2 : 0.0);
    const double w1 = r.v1, w2 = (M3 == 3) ? r.v2 : 0.0;
    // left reflection of a row lane's entries in rows k..k+M3-1
    const int q = row - k;
    const double lw = (rowOn && q >= 0 && q < M3) ? r.tau * (q == 0 ? 1.0 : (q == 1 ? w1 : w2)) : 0.0;
#pragma unroll
    for (int b = 0; b < M3; ++b) {
        double sc = blk[0][b] + w1 * blk[1][b];
        if (M3 == 3) sc += w2 * blk[2][b];
        v[b] -= lw * sc;
    }
    // the step's own reflection: left for column lanes, right for row lanes
    double s = v[0] + w1 * v[1];
    if (M3 == 3) s += w2 * v[2];
    s *= r.tau;
    v[0] -= s;
    v[1] -= s * w1;
    if (M3 == 3) v[2] -= s * w2;
    if (colOn || rowOn) {
#pragma unroll
        for (int a = 0; a < M3; ++a) vec[a * vs] = v[a];
    }
    if (lane == 0) {
        if (betaOn) {
            AT(T, ldt, k, k - 1) = r.beta;
            AT(T, ldt, k + 1, k - 1) = 0.0;
            if (M3 == 3) AT(T, ldt, k + 2, k - 1) = 0.0;
        }
        rt[k - k0] = r.tau;
        r1[k - k0] = w1;
        r2[k - k0] = w2;
    }
    const int lb = 32 + (k + 1 - k0);
    x0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[0]), lb),
                          __builtin_amdgcn_readlane(__double2loint(v[0]), lb));
    x1 = (k + 2 <= rmax) ? __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[0]), lb + 1),
                                            __builtin_amdgcn_readlane(__double2loint(v[0]), lb + 1))
                         : 0.0;
    x2 = (k + 3 <= rmax) ? __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[0]), lb + 2),
                                            __builtin_amdgcn_readlane(__double2loint(v[0]), lb + 2))
                         : 0.0;
}

// Wave 0: bulge steps k0..k1-1 of the double-shift sweep on rows/cols l..i with
// only the near field updated (columns up to cnear, rows from k0).  (x0, x1, x2)
// carries the generating vector of the next step between calls.  Reflectors with
// tau = 0 are exact no-ops, so no step is special-cased.
__device__ __forceinline__ void near_steps(double *T, int ldt, int l, int i, int k0, int k1, int cnear, double tr, double det,
                           double *rt, double *r1, double *r2, double &x0, double &x1, double &x2) {
    if (k0 == l) {  // the sweep's first step: the bulge from the shift polynomial
        const double h00 = AT(T, ldt, l, l), h01 = AT(T, ldt, l, l + 1);
        const double h10 = AT(T, ldt, l + 1, l), h11 = AT(T, ldt, l + 1, l + 1);
        const double h21 = AT(T, ldt, l + 2, l + 1);
        double sc = fmax(fmax(fabs(h00), fabs(h01)), fmax(fmax(fabs(h10), fabs(h11)), fabs(h21)));
        sc = fmax(sc, fmax(fabs(tr), sqrt(fabs(det))));
        if (sc == 0.0) sc = 1.0;
        const double rs = 1.0 / sc;
        const double a = h00 * rs, b = h01 * rs, c = h10 * rs, d = h11 * rs, e = h21 * rs;
        const double t = tr * rs, dt = det * rs * rs;
        x0 = a * a + b * c - t * a + dt;
        x1 = c * (a + d - t);
        x2 = c * e;
    }
    // three-row reflectors up to k = i - 2, the sweep's last (two-row) one at k = i - 1
    const int k3 = (k1 < i - 1) ? k1 : i - 1;
    int k = k0;
    for (; k < k3; ++k) near_step<3>(T, ldt, l, i, k, k0, cnear, rt, r1, r2, x0, x1, x2);
    if (k < k1) near_step<2>(T, ldt, l, i, k, k0, cnear, rt, r1, r2, x0, x1, x2);
}

// The far-field update of a sweep's last batch of reflectors (columns right of
// its near field, the rows above it, all of Q) may be left pending: every entry
// it writes is strictly above the diagonal, so the deflation scan does not read
// them, and the next sweep's waves 1-3 apply it while wave 0 chases the first
// batch, when that batch's near field lies left of its columns.  Otherwise (and
// before a 2x2 standardisation, shift inputs it may touch, or the end) it is
// applied by all threads at once.
struct FarPending {
    int k0, nb, cnear, buf;  // the batch (k0 < 0: none) and its reflector buffer
};

__device__ __forceinline__ void far_flush(double *T, int ldt, double *Q, int ldq, int m, FarPending &pf,
                                          double (*rq)[3][FB]) {
    if (pf.k0 < 0) return;
    PROF_T(pf0);
    far_apply(T, ldt, Q, ldq, m, pf.k0, pf.nb, pf.cnear + 1, m - 1, pf.k0, true, rq[pf.buf][0], rq[pf.buf][1],
              rq[pf.buf][2], threadIdx.x, NT);
    __syncthreads();
    PROF_ADD(2, pf0);
    pf.k0 = -1;
}

// One implicit double-shift step (all NT threads call) on the active rows l..i
// of the m x m LDS matrix T; updates span all of T and Q's columns, except the
// far field of the last batch, which is left pending in pf.
__device__ __forceinline__ void lds_francis(double *T, int ldt, double *Q, int ldq, int m, int l, int i, double tr, double det,
                                            FarPending &pf, double (*rq)[3][FB]) {
    const int tid = threadIdx.x, wave = tid / LANES;
    PROF_CNT(4, i - l);
    {
        const int k1 = (l + FB < i) ? l + FB : i;
        const int cnear = (k1 + 1 < m - 1) ? k1 + 1 : m - 1;
        if (pf.k0 >= 0 && cnear >= pf.k0) far_flush(T, ldt, Q, ldq, m, pf, rq);
    }
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    bool carried = pf.k0 >= 0;  // the previous sweep's last batch, for waves 1-3
    int pk0 = pf.k0, pnb = pf.nb, pcnear = pf.cnear, pb = pf.buf, cb = carried ? pf.buf ^ 1 : 0;
    for (int k0 = l; k0 <= i - 1; k0 += FB) {
        const int k1 = (k0 + FB < i) ? k0 + FB : i;
        const int cnear = (k1 + 1 < m - 1) ? k1 + 1 : m - 1;
        if (wave == 0) {
            PROF_T(pa);
            if (pk0 >= 0 && !carried && cnear > pcnear)  // previous batch on the columns entering the near field
                far_apply(T, ldt, Q, ldq, m, pk0, pnb, pcnear + 1, cnear, 0, false, rq[pb][0], rq[pb][1], rq[pb][2],
                          tid, LANES);
            near_steps(T, ldt, l, i, k0, k1, cnear, tr, det, rq[cb][0], rq[cb][1], rq[cb][2], x0, x1, x2);
            PROF_ADD(0, pa);
        } else if (pk0 >= 0) {
            // a carried batch's near field is complete: all of its far field here
            const int c_lo = carried ? pcnear + 1 : cnear + 1;
            far_apply(T, ldt, Q, ldq, m, pk0, pnb, c_lo, m - 1, pk0, true, rq[pb][0], rq[pb][1], rq[pb][2],
                      tid - LANES, NT - LANES);
        }
        PROF_T(pw);
        __syncthreads();
        PROF_ADD(1, pw);
        carried = false;
        pk0 = k0;
        pnb = k1 - k0;
        pcnear = cnear;
        pb = cb;
        cb ^= 1;
    }
    pf.k0 = pk0;
    pf.nb = pnb;
    pf.cnear = pcnear;
    pf.buf = pb;
}

// Double-shift QR iteration on the m x m LDS matrix T (upper Hessenberg) with Q
// accumulated.  Returns 0, or i+1 when rows/cols 0..i did not converge within
// maxit iterations.  *iters receives the iteration count.
__device__ __forceinline__ int lds_small_qr(double *T, int ldt, double *Q, int ldq, int m, double hnorm, double smlnum, int maxit,
                            int *iters) {
    __shared__ double rq[2][3][FB];
    const int lane = threadIdx.x & (LANES - 1);
    FarPending pf{-1, 0, 0, 0};
    int i = m - 1, its = 0, total = 0;
    while (i >= 0) {
        PROF_T(pe);
        int l = 0;
        for (int base = i; base >= 1; base -= LANES) {
            const int k = base - lane;
            bool neg = false;
            if (k >= 1)
                neg = negligible_sub(AT(T, ldt, k, k - 1), AT(T, ldt, k - 1, k - 1), AT(T, ldt, k, k), hnorm, smlnum);
            const unsigned long long mask = __ballot(neg);
            if (mask) {
                l = base - (__ffsll(mask) - 1);
                break;
            }
        }
        __syncthreads();
        if (l > 0 && threadIdx.x == 0) AT(T, ldt, l, l - 1) = 0.0;
        __syncthreads();
        PROF_ADD(3, pe);
        if (l == i) {
            --i;
            its = 0;
            continue;
        }
        if (l == i - 1) {
            far_flush(T, ldt, Q, ldq, m, pf, rq);
            lds_standardise(T, ldt, Q, ldq, m, i - 1);
            i -= 2;
            its = 0;
            continue;
        }
        if (total >= maxit) {
            far_flush(T, ldt, Q, ldq, m, pf, rq);
            *iters = total;
            return i + 1;
        }
        ++total;
        ++its;
        // the shift inputs: T(i-1, i) is the only one off the two diagonals
        if (pf.k0 >= 0 && ((i - 1 < pf.k0 && i >= pf.k0 && i <= pf.k0 + pf.nb + 1) ||
                           (i - 1 >= pf.k0 && i - 1 <= pf.k0 + pf.nb + 1 && i > pf.cnear)))
            far_flush(T, ldt, Q, ldq, m, pf, rq);
        double tr, det;
        if (its == 10 || its == 20) {
            const double s = fabs(AT(T, ldt, i, i - 1)) + fabs(AT(T, ldt, i - 1, i - 2));
            const double x = AT(T, ldt, i, i);
            tr = 2.0 * x + 1.5 * s;
            det = x * x + 1.5 * s * x + s * s;
        } else {
            const double a = AT(T, ldt, i - 1, i - 1), b = AT(T, ldt, i - 1, i);
            const double c = AT(T, ldt, i, i - 1), d = AT(T, ldt, i, i);
            tr = a + d;
            det = a * d - b * c;
        }
        __syncthreads();  // every wave has read the shift inputs before wave 0 writes
        lds_francis(T, ldt, Q, ldq, m, l, i, tr, det, pf, rq);
    }
    far_flush(T, ldt, Q, ldq, m, pf, rq);
    *iters = total;
    return 0;
}

// Load the m x m diagonal block of H at (off, off) into T (zeros below the
// subdiagonal) and set Q = I.
__device__ __forceinline__ void lds_load_block(const double *H, int ldh, int off, int m, double *T, int ldt, double *Q, int ldq) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
        const int i = idx % m, j = idx / m;
        AT(T, ldt, i, j) = (i <= j + 1) ? AT(H, ldh, off + i, off + j) : 0.0;
        AT(Q, ldq, i, j) = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
}

// Write T back to H's diagonal block and Q^T to Ut (column-major, ld ldut).
__device__ __forceinline__ void lds_store(double *H, int ldh, int off, int m, const double *T, int ldt, const double *Q, int ldq,
                          double *Ut, int ldut) {
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
        const int i = idx % m, j = idx / m;
        AT(H, ldh, off + i, off + j) = (i <= j + 1) ? AT(T, ldt, i, j) : 0.0;
        AT(Ut, ldut, i, j) = AT(Q, ldq, j, i);
    }
}

extern "C" __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_small_qr(double *H, int ldh, int off, int m, double hnorm, double smlnum, int maxit, double *Ut, int ldut,
           int *status) {
    extern __shared__ double lds[];
    const int ld = m + 1;
    double *T = lds;
    double *Q = lds + (size_t)m * ld;
#ifdef NEIG_PROF
    if (threadIdx.x < 8) g_prof[threadIdx.x] = 0;
    __syncthreads();
    const long long p0 = clock64();
#endif
    lds_load_block(H, ldh, off, m, T, ld, Q, ld);
    int iters = 0;
    const int info = lds_small_qr(T, ld, Q, ld, m, hnorm, smlnum, maxit, &iters);
    __syncthreads();
    lds_store(H, ldh, off, m, T, ld, Q, ld, Ut, ldut);
    if (threadIdx.x == 0) {
        status[0] = info;
        status[1] = iters;
#ifdef NEIG_PROF
        g_prof[7] = clock64() - p0;
        for (int t = 0; t < 8; ++t) ((long long *)(status + 16))[t] = g_prof[t];
#endif
    }
}

// ---------------------------------------------------------------- block swap
//
// Swapping adjacent diagonal blocks A (p x p, on top) and C (q x q) of a
// quasi-triangular matrix [[A B][0 C]]: solve A X - X C = B; the columns of
// [[-X][I]] span C's invariant subspace, so the orthogonal factor Q of their QR
// factorisation gives Q^T [[A B][0 C]] Q = [[C' *][0 A']].  The swap is
// rejected when the computed lower-left block or the reconstruction error is
// not at roundoff level.  Sizes are template parameters so that every array
// below has constant indices and lives in registers.

// Solve the K x K system M x = r by Gaussian elimination with complete
// pivoting; row and column exchanges are done with selects.  Tiny pivots are
// raised to smin.
template <int K>
__device__ __forceinline__ bool solve_cp(double (&M)[K][K], double (&r)[K], double (&x)[K]) {
    int perm[K];
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        perm[i] = i;
#pragma unroll
        for (int j = 0; j < K; ++j) mx = fmax(mx, fabs(M[i][j]));
    }
    const double smin = fmax(NEIG_EPS * mx, NEIG_DBL_MIN);
    double rinv[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        int pr = s, pc = s;
        double best = -1.0;
#pragma unroll
        for (int i = s; i < K; ++i)
#pragma unroll
            for (int j = s; j < K; ++j) {
                const double v = fabs(M[i][j]);
                if (v > best) { best = v; pr = i; pc = j; }
            }
#pragma unroll
        for (int i = s + 1; i < K; ++i) {
            const bool sw = (i == pr);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double a = M[s][j], b = M[i][j];
                M[s][j] = sw ? b : a;
                M[i][j] = sw ? a : b;
            }
            const double a = r[s], b = r[i];
            r[s] = sw ? b : a;
            r[i] = sw ? a : b;
        }
#pragma unroll
        for (int j = s + 1; j < K; ++j) {
            const bool sw = (j == pc);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const double a = M[i][s], b = M[i][j];
                M[i][s] = sw ? b : a;
                M[i][j] = sw ? a : b;
            }
            const int pa = perm[s], pb = perm[j];
            perm[s] = sw ? pb : pa;
            perm[j] = sw ? pa : pb;
        }
        if (fabs(M[s][s]) < smin) M[s][s] = smin;
        const double inv = 1.0 / M[s][s];
        rinv[s] = inv;
#pragma unroll
        for (int i = s + 1; i < K; ++i) {
            const double f = M[i][s] * inv;
#pragma unroll
            for (int j = s; j < K; ++j) M[i][j] -= f * M[s][j];
            r[i] -= f * r[s];
        }
    }
    double y[K];
#pragma unroll
    for (int s = K - 1; s >= 0; --s) {
        double t = r[s];
#pragma unroll
        for (int j = s + 1; j < K; ++j) t -= M[s][j] * y[j];
        y[s] = t * rinv[s];
    }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < K; ++s) v = (perm[s] == i) ? y[s] : v;
        x[i] = v;
        ok = ok && isfinite(v);
    }
    return ok;
}

// The swap transform from a solution X of the Sylvester equation A X - X C = B12
// (A the leading P x P block of B, C the trailing Q x Q block, X(i, j) at index
// i + P j): the columns of [[-X][I]] span C's invariant subspace, Qm is the
// orthogonal factor of their QR factorisation and Bn = Qm^T B Qm.  Returns false
// when Bn's lower-left block or the reconstruction error B - Qm Bn Qm^T is not at
// roundoff level (then the swap is rejected).
template <int P, int Q>
__device__ __forceinline__ bool swap_from_x(const double (&B)[P + Q][P + Q], const double (&X)[P * Q], double bnorm,
                                            double (&Qm)[P + Q][P + Q], double (&Bn)[P + Q][P + Q]) {
    constexpr int N = P + Q;
    constexpr int K = P * Q;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Qm[i][j] = (i == j) ? 1.0 : 0.0;
    double xm = 0.0;
#pragma unroll
    for (int t = 0; t < K; ++t) xm = fmax(xm, fabs(X[t]));
    const double g = 1.0 / fmax(1.0, xm);
    double Y[N][Q];
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i][j] = (i < P) ? -g * X[i + P * j] : ((i - P == j) ? g : 0.0);
    // Householder QR of Y, reflectors accumulated into Qm
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        double v[N];
#pragma unroll
        for (int t = 0; t < N; ++t) v[t] = (t >= c) ? Y[t][c] : 0.0;
        double mx = 0.0;
#pragma unroll
        for (int t = c + 1; t < N; ++t) mx = fmax(mx, fabs(v[t]));
        if (mx == 0.0) continue;
        const double sc = fmax(mx, fabs(v[c]));
        const double rsc = 1.0 / sc;
        double ss = 0.0;
#pragma unroll
        for (int t = c; t < N; ++t) ss += (v[t] * rsc) * (v[t] * rsc);
        const double nrm = sc * sqrt(ss);
        const double alpha = v[c];
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        const double dd = alpha - beta;
        const double qq = 1.0 / (beta * dd);  // one division for 1/beta and 1/(alpha - beta)
        const double tau = -dd * dd * qq;     // (beta - alpha) / beta
        const double inv = beta * qq;         // 1 / (alpha - beta)
#pragma unroll
        for (int t = c + 1; t < N; ++t) v[t] *= inv;
        v[c] = 1.0;
#pragma unroll
        for (int j = c; j < Q; ++j) {
            double d = 0.0;
#pragma unroll
            for (int t = c; t < N; ++t) d += v[t] * Y[t][j];
            d *= tau;
#pragma unroll
            for (int t = c; t < N; ++t) Y[t][j] -= d * v[t];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double d = 0.0;
#pragma unroll
            for (int t = c; t < N; ++t) d += Qm[i][t] * v[t];
            d *= tau;
#pragma unroll
            for (int t = c; t < N; ++t) Qm[i][t] -= d * v[t];
        }
    }
    // Bn = Qm^T (B Qm); B is block upper triangular (rows P.. are zero in
    // columns ..P-1)
    double W[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
#pragma unroll
            for (int k = (i < P ? 0 : P); k < N; ++k) d += B[i][k] * Qm[k][j];
            W[i][j] = d;
        }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) d += Qm[k][i] * W[k][j];
            Bn[i][j] = d;
        }
    const double thresh = fmax(20.0 * NEIG_EPS * bnorm, NEIG_DBL_MIN);
    double low = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j)
#pragma unroll
        for (int i = Q; i < N; ++i) {
            low = fmax(low, fabs(Bn[i][j]));
            Bn[i][j] = 0.0;
        }
    if (!(low <= thresh)) return false;
    // reconstruction: B ~ Qm Bn Qm^T (Bn now block upper triangular: rows Q..
    // are zero in columns ..Q-1)
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
#pragma unroll
            for (int k = (i < Q ? 0 : Q); k < N; ++k) d += Bn[i][k] * Qm[j][k];
            W[i][j] = d;
        }
    double err = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) d += Qm[i][k] * W[k][j];
            err = fmax(err, fabs(d - B[i][j]));
        }
    return err <= thresh;
}

// Closed-form solve of the 2 x 2 Sylvester equation A X - X C = R.  With
// p(z) = z^2 - tr(C) z + det(C) the characteristic polynomial of C,
// Cayley-Hamilton (C^2 = tr(C) C - det(C) I) turns the equation into
// p(A) X = A R + R (C - tr(C) I), a 2 x 2 linear system solved by its adjugate;
// one step of residual correction follows.  Returns false when p(A) is singular
// or the result is not finite (the caller then solves the 4 x 4 system).
__device__ __forceinline__ bool sylv22_closed(const double (&B)[4][4], double (&X)[4]) {
    const double a00 = B[0][0], a01 = B[0][1], a10 = B[1][0], a11 = B[1][1];
    const double c00 = B[2][2], c01 = B[2][3], c10 = B[3][2], c11 = B[3][3];
    const double trc = c00 + c11, detc = c00 * c11 - c01 * c10;
    const double d = a00 + a11 - trc;
    const double p00 = a00 * a00 + a01 * a10 - trc * a00 + detc;
    const double p01 = a01 * d, p10 = a10 * d;
    const double p11 = a10 * a01 + a11 * a11 - trc * a11 + detc;
    const double detp = p00 * p11 - p01 * p10;
    if (!(fabs(detp) > 0.0)) return false;
    const double rd = 1.0 / detp;
    const double q00 = p11 * rd, q01 = -p01 * rd, q10 = -p10 * rd, q11 = p00 * rd;  // p(A)^-1
    // C - tr(C) I = [[-c11, c01], [c10, -c00]]
    double r00 = B[0][2], r01 = B[0][3], r10 = B[1][2], r11 = B[1][3];
    double x00 = 0.0, x01 = 0.0, x10 = 0.0, x11 = 0.0;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const double s00 = a00 * r00 + a01 * r10 - r00 * c11 + r01 * c10;
        const double s01 = a00 * r01 + a01 * r11 + r00 * c01 - r01 * c00;
        const double s10 = a10 * r00 + a11 * r10 - r10 * c11 + r11 * c10;
        const double s11 = a10 * r01 + a11 * r11 + r10 * c01 - r11 * c00;
        x00 += q00 * s00 + q01 * s10;
        x01 += q00 * s01 + q01 * s11;
        x10 += q10 * s00 + q11 * s10;
        x11 += q10 * s01 + q11 * s11;
        if (pass == 0) {  // residual R - (A X - X C)
            r00 = B[0][2] - (a00 * x00 + a01 * x10 - x00 * c00 - x01 * c10);
            r01 = B[0][3] - (a00 * x01 + a01 * x11 - x00 * c01 - x01 * c11);
            r10 = B[1][2] - (a10 * x00 + a11 * x10 - x10 * c00 - x11 * c10);
            r11 = B[1][3] - (a10 * x01 + a11 * x11 - x10 * c01 - x11 * c11);
        }
    }
    X[0] = x00; X[1] = x10; X[2] = x01; X[3] = x11;
    return isfinite(x00) && isfinite(x01) && isfinite(x10) && isfinite(x11);
}

// Closed-form solve of the Sylvester equation when one block is 1x1: for
// (P, Q) = (1, 2) it reads X (a I - C) = R (X a row), for (2, 1) it reads
// (A - c I) X = R (X a column); either is one 2 x 2 system, solved by its
// adjugate, with one step of residual correction.  Returns false when the
// system is singular or the result is not finite (the caller then solves by
// complete pivoting).
template <int P, int Q>
__device__ __forceinline__ bool sylv12_closed(const double (&B)[P + Q][P + Q], double (&X)[2]) {
    static_assert(P * Q == 2, "one 1x1 and one 2x2 block");
    double m00, m01, m10, m11, r0, r1;
    if constexpr (P == 1) {  // [x0 x1] M = [r0 r1], M = a I - C
        m00 = B[0][0] - B[1][1]; m01 = -B[1][2]; m10 = -B[2][1]; m11 = B[0][0] - B[2][2];
        r0 = B[0][1]; r1 = B[0][2];
    } else {  // M [x0; x1] = [r0; r1], M = A - c I
        m00 = B[0][0] - B[2][2]; m01 = B[0][1]; m10 = B[1][0]; m11 = B[1][1] - B[2][2];
        r0 = B[0][2]; r1 = B[1][2];
    }
    const double det = m00 * m11 - m01 * m10;
    if (!(fabs(det) > 0.0)) return false;
    const double rd = 1.0 / det;
    double x0 = 0.0, x1 = 0.0, e0 = r0, e1 = r1;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        if constexpr (P == 1) {  // row vector: e M^-1
            x0 += (e0 * m11 - e1 * m10) * rd;
            x1 += (e1 * m00 - e0 * m01) * rd;
            if (pass == 0) { e0 = r0 - (x0 * m00 + x1 * m10); e1 = r1 - (x0 * m01 + x1 * m11); }
        } else {  // column vector: M^-1 e
            x0 += (m11 * e0 - m01 * e1) * rd;
            x1 += (m00 * e1 - m10 * e0) * rd;
            if (pass == 0) { e0 = r0 - (m00 * x0 + m01 * x1); e1 = r1 - (m10 * x0 + m11 * x1); }
        }
    }
    X[0] = x0; X[1] = x1;
    return isfinite(x0) && isfinite(x1);
}

// Orthogonal Qm (N x N) and the swapped block Bn = Qm^T B Qm for block sizes (P, Q).
template <int P, int Q>
__device__ __forceinline__ bool swap_transform(const double (&B)[P + Q][P + Q], double (&Qm)[P + Q][P + Q],
                                               double (&Bn)[P + Q][P + Q]) {
    constexpr int N = P + Q;
    double bnorm = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) bnorm = fmax(bnorm, fabs(B[i][j]));
    bnorm *= N;  // >= Frobenius norm
    if constexpr (P == 1 && Q == 1) {
        const double a = B[0][0], b = B[0][1], c = B[1][1];
        const double x0 = b, x1 = c - a;
        Qm[0][0] = 1.0; Qm[0][1] = 0.0; Qm[1][0] = 0.0; Qm[1][1] = 1.0;
        if (x0 == 0.0 && x1 == 0.0) {
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = 0; j < N; ++j) Bn[i][j] = B[i][j];
            return true;
        }
        const double rr = hypot(x0, x1);
        const double cs = x0 / rr, sn = x1 / rr;
        Qm[0][0] = cs; Qm[1][0] = sn; Qm[0][1] = -sn; Qm[1][1] = cs;
        Bn[0][0] = c; Bn[0][1] = b; Bn[1][0] = 0.0; Bn[1][1] = a;
        return true;
    } else {
        if constexpr (P == 2 && Q == 2) {
            double Xc[4];
            if (sylv22_closed(B, Xc) && swap_from_x<2, 2>(B, Xc, bnorm, Qm, Bn)) return true;
            PROF_CNT(7, 1);  // the closed form was rejected: 4 x 4 solve
        } else {
            double Xc[2];
            if (sylv12_closed<P, Q>(B, Xc) && swap_from_x<P, Q>(B, Xc, bnorm, Qm, Bn)) return true;
        }
        constexpr int K = P * Q;
        double M[K][K], rhs[K], X[K];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) M[i][j] = 0.0;
        // unknown X(i, j) at index i + P j; equation (i, j): sum_k A(i,k) X(k,j) - sum_k X(i,k) C(k,j) = B(i, P+j)
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int row = i + P * j;
                rhs[row] = B[i][P + j];
#pragma unroll
                for (int k = 0; k < P; ++k) M[row][k + P * j] += B[i][k];
#pragma unroll
                for (int k = 0; k < Q; ++k) M[row][i + P * k] -= B[P + k][P + j];
            }
        if (!solve_cp<K>(M, rhs, X)) return false;
        return swap_from_x<P, Q>(B, X, bnorm, Qm, Bn);
    }
}

// Swap the adjacent diagonal blocks of T at st (sizes P then Q) in place, with
// the transformation applied to whole rows/columns of the nw x nw window and to V.
template <int P, int Q>
__device__ __forceinline__ bool lds_swap_pq(double *T, int ldt, double *V, int ldv, int nw, int st) {
    constexpr int N = P + Q;
    double B[N][N], Qm[N][N], Bn[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) B[i][j] = AT(T, ldt, st + i, st + j);
    const bool ok = swap_transform<P, Q>(B, Qm, Bn);
    __syncthreads();
    if (!ok) return false;
    const int ncol = nw - (st + N);
    const int total = ncol + st + nw;
    for (int it = threadIdx.x; it < total; it += NT) {
        if (it < ncol) {  // rows st..st+N-1 right of the pair: new = Qm^T old
            const int j = st + N + it;
            double o[N];
#pragma unroll
            for (int i = 0; i < N; ++i) o[i] = AT(T, ldt, st + i, j);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) d += Qm[k][i] * o[k];
                AT(T, ldt, st + i, j) = d;
            }
        } else {  // columns st..st+N-1 of the rows above (T) and of V: new = old Qm
            const int i = it - ncol;
            double *M = (i < st) ? T : V;
            const int ld = (i < st) ? ldt : ldv;
            const int row = (i < st) ? i : i - st;
            double o[N];
#pragma unroll
            for (int k = 0; k < N; ++k) o[k] = AT(M, ld, row, st + k);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) d += o[k] * Qm[k][j];
                AT(M, ld, row, st + j) = d;
            }
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) AT(T, ldt, st + i, st + j) = Bn[i][j];
    }
    __syncthreads();
    // the 2x2 blocks of Bn are similar to the old ones but not in standard form;
    // aed_core standardises the deflated ones once, after all swaps
    return true;
}

__device__ __forceinline__ bool lds_swap(double *T, int ldt, double *V, int ldv, int nw, int st, int p, int q) {
    if (p == 1 && q == 1) return lds_swap_pq<1, 1>(T, ldt, V, ldv, nw, st);
    if (p == 1 && q == 2) return lds_swap_pq<1, 2>(T, ldt, V, ldv, nw, st);
    if (p == 2 && q == 1) return lds_swap_pq<2, 1>(T, ldt, V, ldv, nw, st);
    PROF_T(p22);
    const bool ok = lds_swap_pq<2, 2>(T, ldt, V, ldv, nw, st);
    PROF_CNT(5, 1);
    PROF_ADD(6, p22);
    return ok;
}

// ---------------------------------------------------------------- Householder helpers (vector in LDS)

// Turn x[0..len-1] (LDS) into a Householder vector in place: on return
// x[0] = 1, x[1..] = v, *tau and *beta set.  All NT threads call.
__device__ __forceinline__ void lds_house(double *x, int len, double *tau, double *beta) {
    const double alpha = x[0];
    double mx = 0.0;
    for (int t = 1 + (int)threadIdx.x; t < len; t += NT) mx = fmax(mx, fabs(x[t]));
    mx = block_reduce(mx, true);
    if (mx == 0.0) {
        *tau = 0.0;
        *beta = alpha;
        __syncthreads();
        if (threadIdx.x == 0) x[0] = 1.0;
        __syncthreads();
        return;
    }
    const double sc = fmax(mx, fabs(alpha));
    double ss = 0.0;
    for (int t = 1 + (int)threadIdx.x; t < len; t += NT) ss += (x[t] / sc) * (x[t] / sc);
    ss = block_reduce(ss, false) + (alpha / sc) * (alpha / sc);
    const double nrm = sc * sqrt(ss);
    const double b = alpha >= 0.0 ? -nrm : nrm;
    *tau = (b - alpha) / b;
    *beta = b;
    const double inv = 1.0 / (alpha - b);
    __syncthreads();
    for (int t = 1 + (int)threadIdx.x; t < len; t += NT) x[t] *= inv;
    if (threadIdx.x == 0) x[0] = 1.0;
    __syncthreads();
}

// rows r0..r0+len-1 of M, columns c0..c1, from the left by I - tau v v^T
__device__ __forceinline__ void lds_refl_left(double *M, int ld, int r0, int len, int c0, int c1, double tau, const double *v) {
    for (int j = c0 + (int)threadIdx.x; j <= c1; j += NT) {
        double d = 0.0;
        for (int t = 0; t < len; ++t) d += v[t] * AT(M, ld, r0 + t, j);
        d *= tau;
        for (int t = 0; t < len; ++t) AT(M, ld, r0 + t, j) -= d * v[t];
    }
}

// columns c0..c0+len-1 of M (rows r0..r1) and of M2 (rows 0..r2-1), from the right
__device__ __forceinline__ void lds_refl_right2(double *M, int ld, int r0, int r1, double *M2, int ld2, int r2, int c0, int len,
                                double tau, const double *v) {
    const int n1 = (r1 >= r0) ? r1 - r0 + 1 : 0;
    for (int it = threadIdx.x; it < n1 + r2; it += NT) {
        double *A = (it < n1) ? M : M2;
        const int lda = (it < n1) ? ld : ld2;
        const int i = (it < n1) ? r0 + it : it - n1;
        double d = 0.0;
        for (int t = 0; t < len; ++t) d += AT(A, lda, i, c0 + t) * v[t];
        d *= tau;
        for (int t = 0; t < len; ++t) AT(A, lda, i, c0 + t) -= d * v[t];
    }
}

// ---------------------------------------------------------------- AED

// Result of the AED core (returned in every thread).
struct AedOut {
    int nd;       // deflated count
    int nritz;    // Ritz values written
    int infqr;    // rows not converged by the window QR
    int swapfail; // a swap was rejected
    int iters;    // window QR iterations
    int nswap;    // block swaps
    int late;     // deflations found above a failed block
    double spike0;  // new coupling entry h(kwtop, kwtop-1) when nd > 0
    long long cyc_qr, cyc_defl, cyc_hess;
};

// AED on the nw x nw window already in LDS (T upper Hessenberg, V = I), coupled
// to the rest by the spike s (Section 3.2, "AED step"): Schur form of T by the
// window QR, spike test bottom-up with failing blocks moved to the top by block
// swaps, undeflated Ritz values written to sr/si (thread 0), and, if anything
// deflated, the spike and the undeflated part reduced back to Hessenberg form.
// On return T and V hold the transformed window and its orthogonal factor.
// Spike test of the diagonal block at j (size bs) of the AED window: the
// window criterion |s v| <= max(smlnum, eps |lambda|) (criterion 0) or the
// norm-stable |s v| <= max(smlnum, eps ||H||_F) (criterion 1), v the block's
// entries in the first row of V.
__device__ __forceinline__ bool aed_block_deflates(const double *T, const double *V, int ld, double s, int j, int bs,
                                                   double hnorm, double smlnum, int criterion) {
    double sp = fabs(s * AT(V, ld, 0, j));
    if (bs == 2) sp = fmax(sp, fabs(s * AT(V, ld, 0, j + 1)));
    double tol;
    if (criterion == 1) {
        tol = NEIG_EPS * hnorm;
    } else {
        double lam = (bs == 1) ? fabs(AT(T, ld, j, j))
                               : sqrt(fabs(AT(T, ld, j, j) * AT(T, ld, j + 1, j + 1) -
                                           AT(T, ld, j, j + 1) * AT(T, ld, j + 1, j)));
        if (lam == 0.0) lam = fabs(s);
        tol = NEIG_EPS * lam;
    }
    tol = fmax(tol, smlnum);
    return sp <= tol;
}

// Second half of the AED step on a window already in real Schur form (rows
// 0..o.infqr-1 unconverged and never tested): the spike test bottom-up with
// block swaps, standardisation of the deflated 2x2 blocks, the undeflated Ritz
// values, and the reduction of the spike and the undeflated part back to
// Hessenberg form.  T, V and the vector scratch x (nw doubles) may be in LDS or
// in global memory (generic pointers); all NT threads call.
__device__ __forceinline__ void aed_deflate(double *T, double *V, int ld, double *x, int nw, double s, double hnorm,
                                            double smlnum, int criterion, double *sr, double *si, AedOut &o) {
    const int tid = threadIdx.x;
    const long long c1 = clock64();
    o.nswap = 0;
    o.late = 0;
    o.swapfail = 0;
    int top = o.infqr, kend = nw;
    while (kend > top) {
        const int bs = (kend - 2 >= top && AT(T, ld, kend - 1, kend - 2) != 0.0) ? 2 : 1;
        const int j = kend - bs;
        const bool defl = aed_block_deflates(T, V, ld, s, j, bs, hnorm, smlnum, criterion);
        __syncthreads();  // all threads have read the test inputs before any swap writes
        if (defl) {
            if (top > o.infqr) o.late += bs;
            kend -= bs;
            continue;
        }
        int pos = j;
        bool ok = true;
        while (pos > top) {
            const int ba = (pos - 2 >= top && AT(T, ld, pos - 1, pos - 2) != 0.0) ? 2 : 1;
            const int st = pos - ba;
            if (!lds_swap(T, ld, V, ld, nw, st, ba, bs)) {
                ok = false;
                break;
            }
            ++o.nswap;
            pos = st;
        }
        if (!ok) {
            o.swapfail = 1;
            top = kend;
            break;
        }
        top += bs;
    }
    o.nd = nw - kend;
    // standard form for the deflated 2x2 blocks (swaps leave them in any form);
    // a block whose eigenvalues came out real is split into two 1x1 blocks
    for (int j = kend; j + 1 < nw;) {
        if (AT(T, ld, j + 1, j) != 0.0) {
            const double a = AT(T, ld, j, j), b = AT(T, ld, j, j + 1), c = AT(T, ld, j + 1, j), d = AT(T, ld, j + 1, j + 1);
            if (!(a == d && b * c < 0.0)) lds_standardise(T, ld, V, ld, nw, j);
            j += 2;
        } else {
            ++j;
        }
    }
    const long long c2 = clock64();

    // undeflated Ritz values (shift candidates), top to bottom
    int c = 0;
    for (int j = o.infqr; j < kend;) {
        if (j + 1 < kend && AT(T, ld, j + 1, j) != 0.0) {
            if (tid == 0) {
                double re1, im1, re2, im2;
                eig2x2(AT(T, ld, j, j), AT(T, ld, j, j + 1), AT(T, ld, j + 1, j), AT(T, ld, j + 1, j + 1), &re1,
                       &im1, &re2, &im2);
                sr[c] = re1; si[c] = im1; sr[c + 1] = re2; si[c + 1] = im2;
            }
            c += 2;
            j += 2;
        } else {
            if (tid == 0) {
                sr[c] = AT(T, ld, j, j);
                si[c] = 0.0;
            }
            ++c;
            ++j;
        }
    }
    o.nritz = c;
    o.spike0 = 0.0;
    o.cyc_defl = c2 - c1;
    o.cyc_hess = 0;
    if (o.nd == 0) return;

    if (kend > 0 && s != 0.0) {
        __syncthreads();
        for (int t = tid; t < kend; t += NT) x[t] = s * AT(V, ld, 0, t);
        __syncthreads();
        if (kend > 1) {
            double tau, beta;
            lds_house(x, kend, &tau, &beta);
            o.spike0 = beta;
            if (tau != 0.0) {
                lds_refl_left(T, ld, 0, kend, 0, nw - 1, tau, x);
                __syncthreads();
                lds_refl_right2(T, ld, 0, kend - 1, V, ld, nw, 0, kend, tau, x);
                __syncthreads();
            }
            // Householder Hessenberg reduction of the undeflated leading block
            for (int cc = 0; cc + 2 < kend; ++cc) {
                const int len = kend - cc - 1;
                for (int t = tid; t < len; t += NT) x[t] = AT(T, ld, cc + 1 + t, cc);
                __syncthreads();
                double tau2, beta2;
                lds_house(x, len, &tau2, &beta2);
                if (tau2 == 0.0) continue;
                for (int t = tid; t < len; t += NT) AT(T, ld, cc + 1 + t, cc) = (t == 0) ? beta2 : 0.0;
                lds_refl_left(T, ld, cc + 1, len, cc + 1, nw - 1, tau2, x);
                __syncthreads();
                lds_refl_right2(T, ld, 0, kend - 1, V, ld, nw, cc + 1, len, tau2, x);
                __syncthreads();
            }
        } else {
            o.spike0 = x[0];
        }
    }
    __syncthreads();
    o.cyc_hess = clock64() - c2;
}

__device__ __forceinline__ AedOut aed_core(double *T, double *V, int ld, double *x, int nw, double s, double hnorm,
                                           double smlnum, int criterion, int maxit, double *sr, double *si) {
    AedOut o;
    const long long c0 = clock64();
    o.iters = 0;
    o.infqr = lds_small_qr(T, ld, V, ld, nw, hnorm, smlnum, maxit, &o.iters);
    __syncthreads();
    o.cyc_qr = clock64() - c0;
    aed_deflate(T, V, ld, x, nw, s, hnorm, smlnum, criterion, sr, si, o);
    return o;
}

// One AED window of a k_aed launch.  flip = 0: the trailing window of the
// active block [ktop, kbot] (rows/cols kbot-nw+1..kbot, coupled to the rest by
// H(kwtop, kwtop-1)).  flip = 1: the leading window (rows/cols ktop..ktop+nw-1,
// coupled by H(ktop+nw, ktop+nw-1)), handled as the trailing window of the
// flipped block J B^T J (B the active block, J the reversal), which is upper
// Hessenberg again: the window is loaded as J W^T J, the same AED runs on it,
// and the result is mapped back (T -> J T^T J, V -> J V J), so its deflated
// eigenvalues end at the top of the window.
struct AedJob {
    int ktop, kbot, nw, flip;
    double *Vt;   // V^T out (ld ldvt)
    int *status;  // 12 ints (layout below)
    double *sr, *si;
};

struct AedJobs {
    AedJob j[2];
};

// status: [0] nd (deflated count), [1] number of Ritz values written to sr/si,
// [2] 1 if H and the window transform V were updated (the host then applies V^T
// to the rest of H and Z), [3] rows not converged by the window QR, [4] 1 if a
// swap was rejected, [5] window QR iterations, [6] block swaps, [7..9] shader
// clock cycles spent in the window QR, the spike test with its swaps, and the
// re-Hessenberg reduction with the write-back, [10] deflations found above a
// block that failed the test.
extern "C" __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_aed(double *H, int ldh, AedJobs jobs, double hnorm, double smlnum, int criterion, int maxit, int ldvt) {
    extern __shared__ double lds[];
    const AedJob J = jobs.j[blockIdx.x];
    const int nw = J.nw;
    const int ld = nw + 1;
    double *T = lds;
    double *V = lds + (size_t)nw * ld;
    double *x = V + (size_t)nw * ld;  // nw doubles of vector scratch
    int off;
    double s;
    if (!J.flip) {
        off = J.kbot - nw + 1;
        s = (off > J.ktop) ? AT(H, ldh, off, off - 1) : 0.0;
        lds_load_block(H, ldh, off, nw, T, ld, V, ld);
    } else {
        off = J.ktop;
        s = (off + nw <= J.kbot) ? AT(H, ldh, off + nw, off + nw - 1) : 0.0;
        for (int idx = threadIdx.x; idx < nw * nw; idx += NT) {
            const int i = idx % nw, j = idx / nw;
            AT(T, ld, i, j) = (i <= j + 1) ? AT(H, ldh, off + nw - 1 - j, off + nw - 1 - i) : 0.0;
            AT(V, ld, i, j) = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    const AedOut o = aed_core(T, V, ld, x, nw, s, hnorm, smlnum, criterion, maxit, J.sr, J.si);
    if (threadIdx.x == 0) {
        int *status = J.status;
        status[0] = o.nd;
        status[1] = o.nritz;
        status[2] = (o.nd > 0) ? 1 : 0;
        status[3] = o.infqr;
        status[4] = o.swapfail;
        status[5] = o.iters;
        status[6] = o.nswap;
        status[7] = (int)min(o.cyc_qr, (long long)INT_MAX);
        status[8] = (int)min(o.cyc_defl, (long long)INT_MAX);
        status[9] = (int)min(o.cyc_hess, (long long)INT_MAX);
        status[10] = o.late;
    }
    if (o.nd == 0) return;  // H untouched; only the shifts are used
    if (!J.flip) {
        lds_store(H, ldh, off, nw, T, ld, V, ld, J.Vt, ldvt);
        if (off > J.ktop && threadIdx.x == 0) AT(H, ldh, off, off - 1) = o.spike0;
    } else {
        for (int idx = threadIdx.x; idx < nw * nw; idx += NT) {
            const int r = idx % nw, c = idx / nw;
            AT(H, ldh, off + r, off + c) = (r <= c + 1) ? AT(T, ld, nw - 1 - c, nw - 1 - r) : 0.0;
            AT(J.Vt, ldvt, r, c) = AT(V, ld, nw - 1 - c, nw - 1 - r);
        }
        if (off + nw <= J.kbot && threadIdx.x == 0) AT(H, ldh, off + nw, off + nw - 1) = o.spike0;
    }
}

// ---------------------------------------------------------------- reordering window

#define REORDER_WMAX 96

struct ReorderWin {
    int off, w;             // the window: rows/cols off .. off+w-1 of S
    int sel[REORDER_WMAX];  // 1 at the positions of selected eigenvalues of the window
};

// Reorder non-overlapping w x w diagonal windows of the quasi-triangular S, one
// workgroup per window (window b = wins[blockIdx.x]; its factor goes to
// Vt + b * ldvt * ldvt, its status to status + 2 b).  In each window at (off, off): the
// selected blocks move to the top of the window in their order, by swaps of
// adjacent diagonal blocks (the block exchange the paper's reordering phase
// uses), with the window's orthogonal factor accumulated in LDS.  The window
// must not split a 2x2 block.  Afterwards every 2x2 block of the window is put
// in standard form.  Outputs: the window back in S, its factor transposed in
// Vt, status[0] = selected eigenvalues now at the top, status[1] = 1 if a swap
// was rejected (the window is then partly reordered, still a valid Schur form).
// The caller applies Vt to the rest of S and to Z.
extern "C" __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_reorder_window(double *S, int lds_, const ReorderWin *wins, double *Vt_all, int ldvt, int *status_all) {
    extern __shared__ double lds[];
    const ReorderWin &f = wins[blockIdx.x];
    const int off = f.off, w = f.w;
    double *Vt = Vt_all + (size_t)blockIdx.x * ldvt * ldvt;
    int *status = status_all + 2 * blockIdx.x;
    const int ld = w + 1;
    double *T = lds, *V = lds + (size_t)w * ld;
    lds_load_block(S, lds_, off, w, T, ld, V, ld);
    int placed = 0, fail = 0, j = 0;
    while (j < w) {
        const int bs = (j + 1 < w && AT(T, ld, j + 1, j) != 0.0) ? 2 : 1;
        if (!f.sel[j]) {
            j += bs;
            continue;
        }
        int pos = j;
        while (pos > placed) {
            const int ba = (pos - 2 >= placed && AT(T, ld, pos - 1, pos - 2) != 0.0) ? 2 : 1;
            const int st = pos - ba;
            if (!lds_swap(T, ld, V, ld, w, st, ba, bs)) {
                fail = 1;
                break;
            }
            pos = st;
        }
        if (fail) break;
        placed += bs;
        j += bs;
    }
    // standard form for every 2x2 block of the window (swaps leave them in any form)
    for (int k = 0; k + 1 < w;) {
        if (AT(T, ld, k + 1, k) != 0.0) {
            const double a = AT(T, ld, k, k), b = AT(T, ld, k, k + 1), c = AT(T, ld, k + 1, k), d = AT(T, ld, k + 1, k + 1);
            if (!(a == d && b * c < 0.0)) lds_standardise(T, ld, V, ld, w, k);
            k += 2;
        } else {
            ++k;
        }
    }
    lds_store(S, lds_, off, w, T, ld, V, ld, Vt, ldvt);
    if (threadIdx.x == 0) {
        status[0] = placed;
        status[1] = fail;
    }
}
