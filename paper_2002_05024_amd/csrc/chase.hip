// chase.hip -- the window task of the multishift sweep (Section 3.2).
//
// One workgroup per diagonal window.  A chain of up to 31 bulges, spaced three
// rows apart, is chased through the window: at each step every active bulge's
// 3-element reflector is generated (from the shift polynomial when the bulge is
// introduced at ktop, otherwise from the column to its left), then all
// reflectors are applied from the left to the window's rows, from the right to
// the window's columns, and accumulated into the window's orthogonal factor U.
// Reflectors of one step act on disjoint index triples, so they commute and the
// three phases are each fully parallel.  The window (and U) live in LDS; the
// kernel writes back the window and U^T, which the update kernels apply to the
// rest of H and to Z (the left/right update tasks).
#include "neig_dev.h"

#define CHASE_THREADS 256
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

    for (int j = 0; j < mb; ++j)
        for (int i = tid; i < mb; i += CHASE_THREADS) AT(Hs, ldhs, i, j) = AT(H, ldh, b0 + i, b0 + j);
    for (int j = 0; j < w; ++j)
        for (int i = tid; i < w; i += CHASE_THREADS) AT(Us, ldus, i, j) = (i == j) ? 1.0 : 0.0;
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
        // phase B: from the left, rows pos..pos+2 over columns pos..r1
        {
            const int jl = tid & 127, half = tid >> 7;
            if (jl < mb) {
                const int j = b0 + jl;
                for (int b = half; b < nb; b += 2) {
                    const int pos = rpos[b];
                    if (pos < 0 || pos > j) continue;
                    const double tau = rtau[b];
                    if (tau == 0.0) continue;
                    const int p = pos - b0;
                    const double v1 = rv1[b], v2 = rv2[b];
                    if (rm3[b] == 3) {
                        double x = AT(Hs, ldhs, p, jl), y = AT(Hs, ldhs, p + 1, jl), z = AT(Hs, ldhs, p + 2, jl);
                        double s = tau * (x + v1 * y + v2 * z);
                        AT(Hs, ldhs, p, jl) = x - s;
                        AT(Hs, ldhs, p + 1, jl) = y - s * v1;
                        AT(Hs, ldhs, p + 2, jl) = z - s * v2;
                    } else {
                        double x = AT(Hs, ldhs, p, jl), y = AT(Hs, ldhs, p + 1, jl);
                        double s = tau * (x + v1 * y);
                        AT(Hs, ldhs, p, jl) = x - s;
                        AT(Hs, ldhs, p + 1, jl) = y - s * v1;
                    }
                }
            }
        }
        __syncthreads();
        // phase C: from the right, columns pos..pos+2 over rows b0..min(pos+3, kbot); and U
        if (tid < 128) {
            const int il = tid;
            if (il < mb) {
                const int i = b0 + il;
                for (int b = 0; b < nb; ++b) {
                    const int pos = rpos[b];
                    if (pos < 0) continue;
                    const int rmax = (pos + 3 < kbot) ? pos + 3 : kbot;
                    if (i > rmax) continue;
                    const double tau = rtau[b];
                    if (tau == 0.0) continue;
                    const int p = pos - b0;
                    const double v1 = rv1[b], v2 = rv2[b];
                    if (rm3[b] == 3) {
                        double x = AT(Hs, ldhs, il, p), y = AT(Hs, ldhs, il, p + 1), z = AT(Hs, ldhs, il, p + 2);
                        double s = tau * (x + v1 * y + v2 * z);
                        AT(Hs, ldhs, il, p) = x - s;
                        AT(Hs, ldhs, il, p + 1) = y - s * v1;
                        AT(Hs, ldhs, il, p + 2) = z - s * v2;
                    } else {
                        double x = AT(Hs, ldhs, il, p), y = AT(Hs, ldhs, il, p + 1);
                        double s = tau * (x + v1 * y);
                        AT(Hs, ldhs, il, p) = x - s;
                        AT(Hs, ldhs, il, p + 1) = y - s * v1;
                    }
                }
            }
        } else {
            const int iu = tid - 128;
            if (iu < w) {
                for (int b = 0; b < nb; ++b) {
                    const int pos = rpos[b];
                    if (pos < 0) continue;
                    const double tau = rtau[b];
                    if (tau == 0.0) continue;
                    const int p = pos - r0;
                    const double v1 = rv1[b], v2 = rv2[b];
                    if (rm3[b] == 3) {
                        double x = AT(Us, ldus, iu, p), y = AT(Us, ldus, iu, p + 1), z = AT(Us, ldus, iu, p + 2);
                        double s = tau * (x + v1 * y + v2 * z);
                        AT(Us, ldus, iu, p) = x - s;
                        AT(Us, ldus, iu, p + 1) = y - s * v1;
                        AT(Us, ldus, iu, p + 2) = z - s * v2;
                    } else {
                        double x = AT(Us, ldus, iu, p), y = AT(Us, ldus, iu, p + 1);
                        double s = tau * (x + v1 * y);
                        AT(Us, ldus, iu, p) = x - s;
                        AT(Us, ldus, iu, p + 1) = y - s * v1;
                    }
                }
            }
        }
        __syncthreads();
    }

    // write back what the window changed: columns r0..r1 (rows b0..r1), the three
    // entries of column b0 below r0, and U^T
    const int off = r0 - b0;
    for (int jl = off; jl < mb; ++jl)
        for (int il = tid; il < mb; il += CHASE_THREADS) AT(H, ldh, b0 + il, b0 + jl) = AT(Hs, ldhs, il, jl);
    if (off == 1 && r0 > ktop && tid < 3 && tid + 1 < mb) AT(H, ldh, r0 + tid, b0) = AT(Hs, ldhs, 1 + tid, 0);
    double *Uo = Ut + (size_t)blockIdx.x * a.ldut * a.ldut;
    for (int c = 0; c < w; ++c)
        for (int r = tid; r < w; r += CHASE_THREADS) AT(Uo, a.ldut, r, c) = AT(Us, ldus, c, r);
}
