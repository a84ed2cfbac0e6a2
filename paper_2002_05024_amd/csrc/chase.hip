// chase.hip -- the window task of the multishift sweep (Section 3.2).
//
// One workgroup per diagonal window.  A chain of up to 31 bulges, spaced three
// rows apart, is chased through the window: at each step every active bulge's
// 3-element reflector is generated (from the shift polynomial when the bulge is
// introduced at ktop, otherwise from the column to its left), then all
// reflectors are applied from the left to the window's rows, from the right to
// the window's columns, and accumulated into the window's orthogonal factor U.
// Reflectors of one step act on disjoint index triples, so they commute and the
// three phases are each fully parallel; 1024 threads give every thread only a
// few (column, bulge) or (row, bulge) pairs, whose loads are all in flight
// together.  The window (and U) live in LDS; the
// kernel writes back the window and U^T, which the update kernels apply to the
// rest of H and to Z (the left/right update tasks).
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

extern "C" __global__ void __launch_bounds__(CHASE_THREADS)
k_chase(double *H, int ldh, const double *poly, double *Ut, ChaseArgs a) {
    extern __shared__ double lds[];
    __shared__ double rtau[CHASE_MAX_BULGES], rv1[CHASE_MAX_BULGES], rv2[CHASE_MAX_BULGES];
    __shared__ int rpos[CHASE_MAX_BULGES], rm3[CHASE_MAX_BULGES];

    const ChaseWin W = a.win[blockIdx.x];
    const int tid = threadIdx.x;
    const int ktop = a.ktop, kbot = a.kbot;
    const int r0 = W.r0, r1 = W.r1;
    const int b0 = (r0 > 0) ? r0 - 1 : 0;
    const int mb = r1 - b0 + 1;  // LDS block order
    const int w = r1 - r0 + 1;   // U order
    const int ldhs = mb + 1, ldus = w + 1;
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

    for (int t = W.t0; t < W.t1; ++t) {
        // phase A: generate the step's reflectors (one thread per bulge)
        if (tid < CHASE_MAX_BULGES) {
            const int b = tid;
            const int pos = ktop + t - 3 * b;
            if (b < nb && pos >= ktop && pos <= kbot - 1) {
                const int m3 = (pos <= kbot - 2) ? 3 : 2;
                const int p = pos - b0;
                double x0, x1, x2;
                if (pos == ktop) {
                    double h00 = AT(Hs, ldhs, p, p), h01 = AT(Hs, ldhs, p, p + 1);
                    double h10 = AT(Hs, ldhs, p + 1, p), h11 = AT(Hs, ldhs, p + 1, p + 1);
                    double h21 = (m3 == 3) ? AT(Hs, ldhs, p + 2, p + 1) : 0.0;
                    double tr = mypoly[2 * b], det = mypoly[2 * b + 1];
                    double sc = fmax(fmax(fabs(h00), fabs(h01)), fmax(fmax(fabs(h10), fabs(h11)), fabs(h21)));
                    sc = fmax(sc, fmax(fabs(tr), sqrt(fabs(det))));
                    if (sc == 0.0) sc = 1.0;
                    double aa = h00 / sc, bb = h01 / sc, cc = h10 / sc, dd = h11 / sc, ee = h21 / sc;
                    double tt = tr / sc, dt = det / (sc * sc);
                    x0 = aa * aa + bb * cc - tt * aa + dt;
                    x1 = cc * (aa + dd - tt);
                    x2 = cc * ee;
                } else {
                    x0 = AT(Hs, ldhs, p, p - 1);
                    x1 = AT(Hs, ldhs, p + 1, p - 1);
                    x2 = (m3 == 3) ? AT(Hs, ldhs, p + 2, p - 1) : 0.0;
                }
                Refl r = make_refl(x0, x1, x2);
                rtau[b] = r.tau; rv1[b] = r.v1; rv2[b] = (m3 == 3) ? r.v2 : 0.0;
                rpos[b] = pos; rm3[b] = m3;
                if (pos > ktop) {
                    AT(Hs, ldhs, p, p - 1) = r.beta;
                    AT(Hs, ldhs, p + 1, p - 1) = 0.0;
                    if (m3 == 3) AT(Hs, ldhs, p + 2, p - 1) = 0.0;
                }
            } else {
                rpos[b] = -1;
                rtau[b] = 0.0;
            }
        }
        __syncthreads();
        // phase B: from the left, rows pos..pos+2 over columns pos..r1.  Thread
        // (column jl, bulge group g) handles bulges g, g+8, g+16, g+24: their row
        // triples are disjoint, so all loads are issued before any store.
        {
            const int jl = tid & 127, g = tid >> 7;
            if (jl < mb) {
                const int j = b0 + jl;
                double x[4][3];
                int pp[4];
                bool act[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = g + 8 * q;
                    const int pos = (b < nb) ? rpos[b] : -1;
                    act[q] = pos >= 0 && pos <= j && rtau[b] != 0.0;
                    pp[q] = pos - b0;
                    if (act[q]) {
                        x[q][0] = AT(Hs, ldhs, pp[q], jl);
                        x[q][1] = AT(Hs, ldhs, pp[q] + 1, jl);
                        x[q][2] = (rm3[b] == 3) ? AT(Hs, ldhs, pp[q] + 2, jl) : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!act[q]) continue;
                    const int b = g + 8 * q;
                    const double tau = rtau[b], v1 = rv1[b], v2 = rv2[b];
                    const double s = tau * (x[q][0] + v1 * x[q][1] + v2 * x[q][2]);
                    AT(Hs, ldhs, pp[q], jl) = x[q][0] - s;
                    AT(Hs, ldhs, pp[q] + 1, jl) = x[q][1] - s * v1;
                    if (rm3[b] == 3) AT(Hs, ldhs, pp[q] + 2, jl) = x[q][2] - s * v2;
                }
            }
        }
        __syncthreads();
        // phase C: from the right, columns pos..pos+2 over rows b0..min(pos+3, kbot),
        // and the same columns of U over all its rows.  Thread (row slot, bulge
        // group g) handles bulges g, g+4, ..., g+28 (disjoint column triples).
        {
            const int slot = tid & 255, g = tid >> 8;
            const bool isH = slot < 128;
            const int il = isH ? slot : slot - 128;
            if (isH ? (il < mb) : (il < w)) {
                double *M = isH ? Hs : Us;
                const int ldm = isH ? ldhs : ldus;
                const int cbase = isH ? b0 : r0;
                const int gi = b0 + il;  // global row (H only)
                double x[8][3];
                int pc[8];
                bool act[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int b = g + 4 * q;
                    const int pos = (b < nb) ? rpos[b] : -1;
                    bool a = pos >= 0 && rtau[b] != 0.0;
                    if (a && isH) {
                        const int rmax = (pos + 3 < kbot) ? pos + 3 : kbot;
                        a = gi <= rmax;
                    }
                    act[q] = a;
                    pc[q] = pos - cbase;
                    if (a) {
                        x[q][0] = AT(M, ldm, il, pc[q]);
                        x[q][1] = AT(M, ldm, il, pc[q] + 1);
                        x[q][2] = (rm3[b] == 3) ? AT(M, ldm, il, pc[q] + 2) : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (!act[q]) continue;
                    const int b = g + 4 * q;
                    const double tau = rtau[b], v1 = rv1[b], v2 = rv2[b];
                    const double s = tau * (x[q][0] + v1 * x[q][1] + v2 * x[q][2]);
                    AT(M, ldm, il, pc[q]) = x[q][0] - s;
                    AT(M, ldm, il, pc[q] + 1) = x[q][1] - s * v1;
                    if (rm3[b] == 3) AT(M, ldm, il, pc[q] + 2) = x[q][2] - s * v2;
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
