// chase.hip -- the window task of the multishift sweep (Section 3.2).
//
// One workgroup per diagonal window.  A chain of up to 31 bulges, spaced three
// rows apart, is chased through the window; at each step every active bulge's
// 3-element reflector is applied from the left to the window's rows, from the
// right to the window's columns, and accumulated into the window's orthogonal
// factor U.  Reflectors of one step act on disjoint index triples, so they
// commute, and the left and the right phase are each fully parallel.  The work
// of a phase is a flat list of (bulge, column) or (bulge, row) items, one per
// thread: a bulge at row pos owns the columns pos..r1 from the left and the rows
// up to pos+3 (and every row of U) from the right, and since consecutive bulges
// are three rows apart the per-bulge counts form an arithmetic sequence, so a
// thread finds its bulge in closed form and no lane idles on a column or row
// that a bulge does not touch.  The next step's reflectors are not generated in
// a phase of their own: the item that applies a bulge's right reflection to
// rows pos+1..pos+3 holds, when it is done, the column that generates the
// bulge's next reflector (rows pos+1..pos+3 of column pos), and builds it on
// the spot; another item introduces the bulge that enters at ktop in the next
// step from its shift polynomial.  Two barriers per step.  The window (and U)
// live in LDS with odd leading dimensions (no bank conflicts on strided
// columns); the kernel writes back the window and U^T, which the update kernels
// apply to the rest of H and to Z (the left/right update tasks).
#include "neig_dev.h"

#define CHASE_THREADS 1024
#define CHASE_MAX_BULGES 32

struct ChaseWin {
    int r0, r1;  // reflectors act on rows/cols r0..r1 (U is (r1-r0+1)^2)
    int t0, t1;  // chain steps [t0, t1)
    int chain;   // chain index; its bulges use polynomials chain*nbc + b
    int nb;      // bulges in this chain
};

struct ChaseArgs {
    ChaseWin win[NEIG_MAX_CHAINS];
    int nwin;
    int ktop, kbot;
    int nbc;   // bulges per full chain
    int ldut;  // leading dimension (and slot stride ldut*ldut) of the U^T outputs
};

// First reflector of the bulge introduced at ktop (shifts of its polynomial
// z^2 - tr z + det, scaled), from the leading 3 x 2 corner of the active block
// (local index p of row ktop).
__device__ __forceinline__ Refl chase_intro(const double *Hs, int ldhs, int p, int m3, double tr, double det) {
    const double h00 = AT(Hs, ldhs, p, p), h01 = AT(Hs, ldhs, p, p + 1);
    const double h10 = AT(Hs, ldhs, p + 1, p), h11 = AT(Hs, ldhs, p + 1, p + 1);
    const double h21 = (m3 == 3) ? AT(Hs, ldhs, p + 2, p + 1) : 0.0;
    double sc = fmax(fmax(fabs(h00), fabs(h01)), fmax(fmax(fabs(h10), fabs(h11)), fabs(h21)));
    sc = fmax(sc, fmax(fabs(tr), sqrt(fabs(det))));
    if (sc == 0.0) sc = 1.0;
    const double aa = h00 / sc, bb = h01 / sc, cc = h10 / sc, dd = h11 / sc, ee = h21 / sc;
    const double tt = tr / sc, dt = det / (sc * sc);
    return make_refl(aa * aa + bb * cc - tt * aa + dt, cc * (aa + dd - tt), cc * ee);
}

extern "C" __global__ void __launch_bounds__(CHASE_THREADS)
k_chase(double *H, int ldh, const double *poly, double *Ut, ChaseArgs a) {
    extern __shared__ double lds[];
    // reflectors of the current and of the next step (index: step parity)
    __shared__ double rtau[2][CHASE_MAX_BULGES], rv1[2][CHASE_MAX_BULGES], rv2[2][CHASE_MAX_BULGES];
    __shared__ int rm3[2][CHASE_MAX_BULGES];

    const ChaseWin W = a.win[blockIdx.x];
    const int tid = threadIdx.x;
    const int ktop = a.ktop, kbot = a.kbot;
    const int r0 = W.r0, r1 = W.r1;
    const int b0 = (r0 > 0) ? r0 - 1 : 0;
    const int mb = r1 - b0 + 1;  // LDS block order
    const int w = r1 - r0 + 1;   // U order
    const int ldhs = mb | 1, ldus = w | 1;
    double *Hs = lds;
    double *Us = lds + (size_t)mb * ldhs;
    const int nb = W.nb;
    const double *mypoly = poly + 2 * (size_t)W.chain * a.nbc;

    for (int idx = tid; idx < mb * mb; idx += CHASE_THREADS) {
        const int i = idx % mb, j = idx / mb;
        AT(Hs, ldhs, i, j) = AT(H, ldh, b0 + i, b0 + j);
    }
    for (int idx = tid; idx < w * w; idx += CHASE_THREADS) {
        const int i = idx % w, j = idx / w;
        AT(Us, ldus, i, j) = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();

    // reflectors of the window's first step (one thread per bulge)
    if (tid < CHASE_MAX_BULGES) {
        const int b = tid, buf = W.t0 & 1;
        const int pos = ktop + W.t0 - 3 * b;
        if (b < nb && pos >= ktop && pos <= kbot - 1) {
            const int m3 = (pos <= kbot - 2) ? 3 : 2;
            const int p = pos - b0;
            Refl r;
            if (pos == ktop) {
                r = chase_intro(Hs, ldhs, p, m3, mypoly[2 * b], mypoly[2 * b + 1]);
            } else {
                r = make_refl(AT(Hs, ldhs, p, p - 1), AT(Hs, ldhs, p + 1, p - 1),
                              (m3 == 3) ? AT(Hs, ldhs, p + 2, p - 1) : 0.0);
                AT(Hs, ldhs, p, p - 1) = r.beta;
                AT(Hs, ldhs, p + 1, p - 1) = 0.0;
                if (m3 == 3) AT(Hs, ldhs, p + 2, p - 1) = 0.0;
            }
            rtau[buf][b] = r.tau; rv1[buf][b] = r.v1; rv2[buf][b] = (m3 == 3) ? r.v2 : 0.0;
            rm3[buf][b] = m3;
        }
    }
    __syncthreads();

    const int wave = tid / 64, lane = tid & 63;
    constexpr int NWAVE = CHASE_THREADS / 64;
    for (int t = W.t0; t < W.t1; ++t) {
        const int cur = t & 1, nxt = cur ^ 1;
        // active bulges blo..bhi: ktop <= pos_b = ktop + t - 3 b <= kbot - 1
        const int bhi = min(nb - 1, t / 3);
        const int lag = t - (kbot - 1 - ktop);
        const int blo = (lag > 0) ? (lag + 2) / 3 : 0;
        const int na = bhi - blo + 1;
        const int ptop = ktop + t - 3 * blo;  // row of the leading active bulge
        const bool more = t + 1 < W.t1;

        // left: bulge k (b = blo + k) on rows pos..pos+m3-1 of columns pos..r1;
        // one wave per bulge, one column per lane
        for (int k = wave; k < na; k += NWAVE) {
            const int b = blo + k;
            const int p = ptop - 3 * k - b0;
            const double tau = rtau[cur][b], v1 = rv1[cur][b], v2 = rv2[cur][b];
            const bool three = rm3[cur][b] == 3;
            for (int jl = p + lane; jl < mb; jl += 64) {
                double *c = &AT(Hs, ldhs, p, jl);
                const double x0 = c[0], x1 = c[1], x2 = three ? c[2] : 0.0;
                const double s = tau * (x0 + v1 * x1 + v2 * x2);
                c[0] = x0 - s;
                c[1] = x1 - s * v1;
                if (three) c[2] = x2 - s * v2;
            }
        }
        __syncthreads();

        // right: the last wave holds the leaders (lane k: rows pos+1..min(pos+3,
        // kbot) of bulge blo + k, which then builds the bulge's next reflector)
        // and introduces the bulge that enters at ktop in the next step (lane
        // na); the other waves take 64-row chunks of the rest: every row of U
        // for each bulge, then rows b0..pos of H
        if (wave == NWAVE - 1) {
            const int bin = (t + 1) / 3;  // bulge entering at step t + 1, if any
            const bool intro = more && ((t + 1) % 3 == 0) && bin < nb;
            if (lane < na) {
                const int b = blo + lane;
                const int pos = ptop - 3 * lane;
                const int p = pos - b0;
                const double tau = rtau[cur][b], v1 = rv1[cur][b], v2 = rv2[cur][b];
                const bool three = rm3[cur][b] == 3;
                const int nr = min(pos + 3, kbot) - pos;  // rows pos+1..pos+nr
                double y[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (q < nr) {
                        y[q][0] = AT(Hs, ldhs, p + 1 + q, p);
                        y[q][1] = AT(Hs, ldhs, p + 1 + q, p + 1);
                        y[q][2] = three ? AT(Hs, ldhs, p + 1 + q, p + 2) : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double s = tau * (y[q][0] + v1 * y[q][1] + v2 * y[q][2]);
                    y[q][0] -= s;
                    y[q][1] -= s * v1;
                    y[q][2] -= s * v2;
                }
                if (more && pos + 1 <= kbot - 1) {
                    const int m3n = (pos + 1 <= kbot - 2) ? 3 : 2;
                    const Refl r = make_refl(y[0][0], y[1][0], (m3n == 3) ? y[2][0] : 0.0);
                    y[0][0] = r.beta;
                    y[1][0] = 0.0;
                    if (m3n == 3) y[2][0] = 0.0;
                    rtau[nxt][b] = r.tau; rv1[nxt][b] = r.v1; rv2[nxt][b] = (m3n == 3) ? r.v2 : 0.0;
                    rm3[nxt][b] = m3n;
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (q < nr) {
                        AT(Hs, ldhs, p + 1 + q, p) = y[q][0];
                        AT(Hs, ldhs, p + 1 + q, p + 1) = y[q][1];
                        if (three) AT(Hs, ldhs, p + 1 + q, p + 2) = y[q][2];
                    }
                }
            } else if (lane == na && intro) {
                const int m3 = (ktop <= kbot - 2) ? 3 : 2;
                const Refl r = chase_intro(Hs, ldhs, ktop - b0, m3, mypoly[2 * bin], mypoly[2 * bin + 1]);
                rtau[nxt][bin] = r.tau; rv1[nxt][bin] = r.v1; rv2[nxt][bin] = (m3 == 3) ? r.v2 : 0.0;
                rm3[nxt][bin] = m3;
            }
        } else if (na > 0) {
            const int uc = (w + 63) >> 6;                 // U chunks per bulge
            const int hc1 = ptop - b0 + 1;                // H rows b0..pos of the leading bulge
            // bulges k < m2 have more than 64 such rows (two chunks)
            const int m2 = min(na, max(0, (hc1 - 64 + 2) / 3));
            const int ntask = na * uc + na + m2;
            for (int task = wave; task < ntask; task += NWAVE - 1) {
                int k, row0, nrow, pc;
                double *M;
                int ldm;
                if (task < na * uc) {
                    k = task / uc;
                    row0 = (task - k * uc) * 64;
                    pc = ptop - 3 * k - r0;
                    // U starts as I and each bulge passing a row moves its first
                    // nonzero column left by at most 2, so rows below pc + 2 + 2 nb
                    // are still zero in columns pc..pc+2: nothing to do there
                    nrow = min(w, pc + 3 + 2 * nb);
                    if (row0 >= nrow) continue;
                    M = Us; ldm = ldus;
                } else {
                    const int h = task - na * uc;
                    int c;
                    if (h < 2 * m2) { k = h >> 1; c = h & 1; }
                    else { k = h - m2; c = 0; }
                    row0 = c * 64;
                    nrow = hc1 - 3 * k;
                    pc = ptop - 3 * k - b0;
                    M = Hs; ldm = ldhs;
                }
                const int b = blo + k;
                const double tau = rtau[cur][b], v1 = rv1[cur][b], v2 = rv2[cur][b];
                const bool three = rm3[cur][b] == 3;
                const int row = row0 + lane;
                if (row < nrow) {
                    double *e = &AT(M, ldm, row, pc);
                    const double x0 = e[0], x1 = e[ldm], x2 = three ? e[2 * ldm] : 0.0;
                    const double s = tau * (x0 + v1 * x1 + v2 * x2);
                    e[0] = x0 - s;
                    e[ldm] = x1 - s * v1;
                    if (three) e[2 * ldm] = x2 - s * v2;
                }
            }
        }
        __syncthreads();
    }

    // write back what the window changed: columns r0..r1 (rows b0..r1), the three
    // entries of column b0 below r0, and U^T
    const int off = r0 - b0;
    for (int idx = tid; idx < mb * (mb - off); idx += CHASE_THREADS) {
        const int il = idx % mb, jl = off + idx / mb;
        AT(H, ldh, b0 + il, b0 + jl) = AT(Hs, ldhs, il, jl);
    }
    if (off == 1 && r0 > ktop && tid < 3 && tid + 1 < mb) AT(H, ldh, r0 + tid, b0) = AT(Hs, ldhs, 1 + tid, 0);
    double *Uo = Ut + (size_t)blockIdx.x * a.ldut * a.ldut;
    for (int idx = tid; idx < w * w; idx += CHASE_THREADS) {
        const int r = idx % w, c = idx / w;
        AT(Uo, a.ldut, r, c) = AT(Us, ldus, c, r);
    }
}
