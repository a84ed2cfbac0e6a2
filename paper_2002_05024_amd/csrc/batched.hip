// batched.hip -- many independent Schur reductions in one persistent launch.
//
// Each workgroup (4 waves) takes problems from a device work queue (largest
// first) and runs the whole method of Section 3.2 on its problem: splitting at
// negligible subdiagonals, the in-LDS double-shift QR for small blocks,
// aggressive early deflation on the trailing window, and single-chain
// multishift sweeps whose windows are chased in LDS.  The orthogonal factors
// never leave LDS: the workgroup applies them to its problem's off-diagonal
// strips of H and Z in HBM with FP64 matrix-core instructions.  All control
// decisions are taken on the device, so one launch covers the whole batch and
// can be captured in a graph.  Parallelism comes from the batch: one problem per
// CU at a time.
#include "neig_dev.h"

#define B_MAX_BULGES 16
#define B_NBUCKET 6

struct BProb {
    double *H, *Z, *wr, *wi;
    int n, ldh, ldz, pad;
};

struct BTune {
    int nw;      // AED window
    int ns;      // shifts per sweep (<= 2 * B_MAX_BULGES)
    int nmin;    // blocks of at most nmin rows go to the in-LDS QR
    int wchase;  // chase window
};

struct BArgs {
    const BProb *probs;
    const int *order;   // processing order (largest problems first)
    int nprob;
    int *next;          // work counter, zero before the launch; next + 2 (8-byte
                        // aligned) holds the launch's algorithmic flop count
                        // (a double), also zeroed by k_batched_pack
    int *info;          // per problem, in the caller's order
    int bucket_hi[B_NBUCKET];  // problems with n <= bucket_hi[b] use tune[b]
    BTune tune[B_NBUCKET];
    int criterion, nibble, exc, maxit_factor;
};

// ---------------------------------------------------------------- workgroup helpers

// ||H||_F over the Hessenberg part, zeros below the subdiagonal; false on NaN/Inf.
__device__ __forceinline__ bool wg_prep(double *H, int ldh, int n, double *hnorm) {
    double mx = 0.0;
    int bad = 0;
    for (long long idx = threadIdx.x; idx < (long long)n * n; idx += NT) {
        const int i = (int)(idx % n), j = (int)(idx / n);
        if (i > j + 1) {
            AT(H, ldh, i, j) = 0.0;
        } else {
            const double v = AT(H, ldh, i, j);
            if (!isfinite(v)) bad = 1;
            else mx = fmax(mx, fabs(v));
        }
    }
    mx = block_reduce(mx, true);
    const double anybad = block_reduce((double)bad, true);
    if (anybad != 0.0) return false;
    double ssq = 0.0;
    if (mx > 0.0) {
        for (long long idx = threadIdx.x; idx < (long long)n * n; idx += NT) {
            const int i = (int)(idx % n), j = (int)(idx / n);
            if (i <= j + 1) {
                const double v = AT(H, ldh, i, j) / mx;
                ssq += v * v;
            }
        }
    }
    ssq = block_reduce(ssq, false);
    *hnorm = mx * sqrt(ssq);
    return true;
}

// Largest k in [1, kbot] whose subdiagonal is negligible (zeroed), else 0.
__device__ __forceinline__ int wg_scan(double *H, int ldh, int kbot, double hnorm, double smlnum) {
    double best = 0.0;
    for (int k = 1 + (int)threadIdx.x; k <= kbot; k += NT) {
        const double sub = AT(H, ldh, k, k - 1);
        if (sub == 0.0 || negligible_sub(sub, AT(H, ldh, k - 1, k - 1), AT(H, ldh, k, k), hnorm, smlnum)) {
            if (sub != 0.0) AT(H, ldh, k, k - 1) = 0.0;
            best = fmax(best, (double)k);
        }
    }
    return (int)block_reduce(best, true);
}

// C (w x len, in HBM) <- U^T C, U (w x w) in LDS with leading dimension ldu.
// Each 64-column tile of C is staged in LDS (stage: (wp+1) * 64 doubles).
__device__ __forceinline__ void wg_update_left(double *C, int ldc, int w, int len, const double *U, int ldu, double *stage) {
    if (len <= 0 || w <= 0) return;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wp = (w + 15) & ~15, kp = (w + 3) & ~3, nrt = wp >> 4;
    const int lds = wp + 1;
    for (int c0 = 0; c0 < len; c0 += 64) {
        for (int idx = threadIdx.x; idx < wp * 64; idx += NT) {
            const int r = idx % wp, c = idx / wp;
            stage[r + c * lds] = (r < w && c0 + c < len) ? AT(C, ldc, r, c0 + c) : 0.0;
        }
        __syncthreads();
        neig_d4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = (neig_d4){0.0, 0.0, 0.0, 0.0};
        const int cb = 16 * q + li;
        for (int k = 0; k < kp; k += 4) {
            const int kk = k + lk;
            const double b = stage[kk + cb * lds];
#pragma unroll
            for (int rt = 0; rt < 6; ++rt) {
                if (rt < nrt) {
                    const int ar = 16 * rt + li;
                    const double a = (ar < w && kk < w) ? U[kk + ar * ldu] : 0.0;
                    acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[rt], 0, 0, 0);
                }
            }
        }
        const int col = c0 + cb;
        if (col < len) {
#pragma unroll
            for (int rt = 0; rt < 6; ++rt) {
                if (rt < nrt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * rt + lk + 4 * r;
                        if (row < w) AT(C, ldc, row, col) = acc[rt][r];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// C (len x w, in HBM) <- C U, U (w x w) in LDS.
__device__ __forceinline__ void wg_update_right(double *C, int ldc, int len, int w, const double *U, int ldu) {
    if (len <= 0 || w <= 0) return;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wp = (w + 15) & ~15, kp = (w + 3) & ~3, nct = wp >> 4;
    for (int r0 = 0; r0 < len; r0 += 64) {
        const int rbase = r0 + 16 * q;
        const int arow = rbase + li;
        neig_d4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = (neig_d4){0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kp; k += 4) {
            const int kk = k + lk;
            const double a = (arow < len && kk < w) ? AT(C, ldc, arow, kk) : 0.0;
#pragma unroll
            for (int ct = 0; ct < 6; ++ct) {
                if (ct < nct) {
                    const int bc = 16 * ct + li;
                    const double b = (bc < w && kk < w) ? U[kk + bc * ldu] : 0.0;
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[ct], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int ct = 0; ct < 6; ++ct) {
            if (ct < nct) {
                const int col = 16 * ct + li;
                if (col < w) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = rbase + lk + 4 * r;
                        if (row < len) AT(C, ldc, row, col) = acc[ct][r];
                    }
                }
            }
        }
    }
    __syncthreads();
}

// The rest of H and Z after the diagonal block [lo, hi] was transformed by U.
__device__ __forceinline__ void wg_block_updates(double *H, int ldh, double *Z, int ldz, int n, int lo, int hi, const double *U,
                                 int ldu, double *stage) {
    const int w = hi - lo + 1;
    wg_update_left(H + lo + (size_t)(hi + 1) * ldh, ldh, w, n - hi - 1, U, ldu, stage);
    wg_update_right(H + (size_t)lo * ldh, ldh, lo, w, U, ldu);
    wg_update_right(Z + (size_t)lo * ldz, ldz, n, w, U, ldu);
}

// Staging space for left updates of width w: reuse `a` if it is large enough.
__device__ __forceinline__ double *pick_stage(double *a, size_t a_len, double *spare, int w) {
    const size_t need = (size_t)(((w + 15) & ~15) + 1) * 64;
    return (a_len >= need) ? a : spare;
}

// ---------------------------------------------------------------- one chase window (NT threads)

// Chase bulges b = 0..nb-1 (polynomial pairs in ptr/pdet) through steps t0..t1-1
// of the window r0..r1 of the active block ktop..kbot; the window (rows and
// columns b0..r1) and its accumulated factor U live in LDS.
__device__ __forceinline__ void wg_chase_window(double *H, int ldh, int ktop, int kbot, int r0, int r1, int t0, int t1, int nb,
                                const double *ptr, const double *pdet, double *Hs, double *Us) {
    __shared__ double rtau[B_MAX_BULGES], rv1[B_MAX_BULGES], rv2[B_MAX_BULGES];
    __shared__ int rpos[B_MAX_BULGES], rm3[B_MAX_BULGES];
    const int tid = threadIdx.x;
    const int b0 = (r0 > 0) ? r0 - 1 : 0;
    const int mb = r1 - b0 + 1, w = r1 - r0 + 1;
    const int ldhs = mb + 1, ldus = w + 1;
    for (int idx = tid; idx < mb * mb; idx += NT) {
        const int i = idx % mb, j = idx / mb;
        AT(Hs, ldhs, i, j) = AT(H, ldh, b0 + i, b0 + j);
    }
    for (int idx = tid; idx < w * w; idx += NT) {
        const int i = idx % w, j = idx / w;
        AT(Us, ldus, i, j) = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        if (tid < B_MAX_BULGES) {
            const int b = tid;
            const int pos = ktop + t - 3 * b;
            if (b < nb && pos >= ktop && pos <= kbot - 1) {
                const int m3 = (pos <= kbot - 2) ? 3 : 2;
                const int p = pos - b0;
                double x0, x1, x2;
                if (pos == ktop) {
                    const double h00 = AT(Hs, ldhs, p, p), h01 = AT(Hs, ldhs, p, p + 1);
                    const double h10 = AT(Hs, ldhs, p + 1, p), h11 = AT(Hs, ldhs, p + 1, p + 1);
                    const double h21 = (m3 == 3) ? AT(Hs, ldhs, p + 2, p + 1) : 0.0;
                    const double tr = ptr[b], det = pdet[b];
                    double sc = fmax(fmax(fabs(h00), fabs(h01)), fmax(fmax(fabs(h10), fabs(h11)), fabs(h21)));
                    sc = fmax(sc, fmax(fabs(tr), sqrt(fabs(det))));
                    if (sc == 0.0) sc = 1.0;
                    const double rs = 1.0 / sc;
                    const double aa = h00 * rs, bb = h01 * rs, cc = h10 * rs, dd = h11 * rs, ee = h21 * rs;
                    const double tt = tr * rs, dt = det * rs * rs;
                    x0 = aa * aa + bb * cc - tt * aa + dt;
                    x1 = cc * (aa + dd - tt);
                    x2 = cc * ee;
                } else {
                    x0 = AT(Hs, ldhs, p, p - 1);
                    x1 = AT(Hs, ldhs, p + 1, p - 1);
                    x2 = (m3 == 3) ? AT(Hs, ldhs, p + 2, p - 1) : 0.0;
                }
                const Refl r = make_refl(x0, x1, x2);
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
        // left: thread (column, bulge half) handles bulges g, g+2, ... in groups of 4
        {
            const int jl = tid & 127, g = tid >> 7;
            if (jl < mb) {
                const int j = b0 + jl;
                for (int q0 = 0; q0 < B_MAX_BULGES / 2; q0 += 4) {
                    double x[4][3];
                    bool act[4];
                    int pp[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int b = g + 2 * (q0 + q);
                        const int pos = (b < nb) ? rpos[b] : -1;
                        act[q] = pos >= 0 && pos <= j;
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
                        const int b = g + 2 * (q0 + q);
                        const double tau = rtau[b], v1 = rv1[b], v2 = rv2[b];
                        const double sv = tau * (x[q][0] + v1 * x[q][1] + v2 * x[q][2]);
                        AT(Hs, ldhs, pp[q], jl) = x[q][0] - sv;
                        AT(Hs, ldhs, pp[q] + 1, jl) = x[q][1] - sv * v1;
                        if (rm3[b] == 3) AT(Hs, ldhs, pp[q] + 2, jl) = x[q][2] - sv * v2;
                    }
                }
            }
        }
        __syncthreads();
        // right: thread per row slot (H rows, then U rows), bulges in groups of 4
        {
            const bool isH = tid < 128;
            const int il = isH ? tid : tid - 128;
            if (isH ? (il < mb) : (il < w)) {
                double *M = isH ? Hs : Us;
                const int ldm = isH ? ldhs : ldus;
                const int cbase = isH ? b0 : r0;
                const int gi = b0 + il;
                for (int b0g = 0; b0g < B_MAX_BULGES; b0g += 4) {
                    double x[4][3];
                    bool act[4];
                    int pc[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int b = b0g + q;
                        const int pos = (b < nb) ? rpos[b] : -1;
                        bool a = pos >= 0;
                        if (a && isH) a = gi <= ((pos + 3 < kbot) ? pos + 3 : kbot);
                        act[q] = a;
                        pc[q] = pos - cbase;
                        if (a) {
                            x[q][0] = AT(M, ldm, il, pc[q]);
                            x[q][1] = AT(M, ldm, il, pc[q] + 1);
                            x[q][2] = (rm3[b] == 3) ? AT(M, ldm, il, pc[q] + 2) : 0.0;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (!act[q]) continue;
                        const int b = b0g + q;
                        const double tau = rtau[b], v1 = rv1[b], v2 = rv2[b];
                        const double sv = tau * (x[q][0] + v1 * x[q][1] + v2 * x[q][2]);
                        AT(M, ldm, il, pc[q]) = x[q][0] - sv;
                        AT(M, ldm, il, pc[q] + 1) = x[q][1] - sv * v1;
                        if (rm3[b] == 3) AT(M, ldm, il, pc[q] + 2) = x[q][2] - sv * v2;
                    }
                }
            }
        }
        __syncthreads();
    }
    // write back the changed part: columns r0..r1 (rows b0..r1) and column b0 below r0
    const int off = r0 - b0;
    for (int idx = tid; idx < mb * (mb - off); idx += NT) {
        const int il = idx % mb, jl = off + idx / mb;
        AT(H, ldh, b0 + il, b0 + jl) = AT(Hs, ldhs, il, jl);
    }
    if (off == 1 && r0 > ktop && tid < 3 && tid + 1 < mb) AT(H, ldh, r0 + tid, b0) = AT(Hs, ldhs, 1 + tid, 0);
    __syncthreads();
}

// ---------------------------------------------------------------- shifts (thread 0)

// Up to ns shifts from the Ritz values (complex pairs kept together, real values
// paired), smallest magnitude first; returns the count written to (xr, xi).
__device__ __forceinline__ int pick_shifts_dev(const double *rr, const double *ri, int nr, int ns, double *xr, double *xi) {
    // items: complex pair (j, j+1) or a pair of reals
    double mag[64];
    int ia[64], ib[64];
    int nit = 0;
    int realidx[96];
    int nreal = 0;
    for (int t = 0; t < nr && nit < 64;) {
        if (ri[t] != 0.0 && t + 1 < nr) {
            mag[nit] = hypot(rr[t], ri[t]);
            ia[nit] = t;
            ib[nit] = t + 1;
            ++nit;
            t += 2;
        } else {
            if (nreal < 96) realidx[nreal++] = t;
            ++t;
        }
    }
    for (int a = 1; a < nreal; ++a) {  // reals by magnitude
        const int v = realidx[a];
        int b = a - 1;
        while (b >= 0 && fabs(rr[realidx[b]]) > fabs(rr[v])) {
            realidx[b + 1] = realidx[b];
            --b;
        }
        realidx[b + 1] = v;
    }
    for (int a = 0; a + 1 < nreal && nit < 64; a += 2) {
        mag[nit] = fmax(fabs(rr[realidx[a]]), fabs(rr[realidx[a + 1]]));
        ia[nit] = realidx[a];
        ib[nit] = realidx[a + 1];
        ++nit;
    }
    for (int a = 1; a < nit; ++a) {  // stable insertion sort by magnitude
        const double m = mag[a];
        const int x = ia[a], y = ib[a];
        int b = a - 1;
        while (b >= 0 && mag[b] > m) {
            mag[b + 1] = mag[b]; ia[b + 1] = ia[b]; ib[b + 1] = ib[b];
            --b;
        }
        mag[b + 1] = m; ia[b + 1] = x; ib[b + 1] = y;
    }
    int out = 0;
    for (int a = 0; a < nit && out + 2 <= ns; ++a) {
        xr[out] = rr[ia[a]]; xi[out] = ri[ia[a]];
        xr[out + 1] = rr[ib[a]]; xi[out + 1] = ri[ib[a]];
        out += 2;
    }
    return out;
}

// ---------------------------------------------------------------- one problem

// *flops receives the method's own operation count for this problem (the same
// formulas as the single-matrix path's neig_stats.alg_flops: 10 m^3 per window
// or small block solved in LDS, 2 m^2 per row or column its factor is applied
// to, 20 n per bulge position of a sweep); every thread holds the same value.
__device__ __forceinline__ int solve_one(const BProb &P, const BTune &tu, const BArgs &A, double *lds, double *flops) {
    __shared__ double s_rr[NEIG_SMALL_MAX], s_ri[NEIG_SMALL_MAX];
    __shared__ double s_ptr[B_MAX_BULGES * 4], s_pdet[B_MAX_BULGES * 4];
    __shared__ int s_nsh;
    const int tid = threadIdx.x;
    const int n = P.n;
    double *H = P.H, *Z = P.Z;
    const int ldh = P.ldh, ldz = P.ldz;
    if (n <= 0) return 0;
    double hnorm = 0.0;
    if (!wg_prep(H, ldh, n, &hnorm)) return -2;
    const double smlnum = NEIG_DBL_MIN * ((double)n / NEIG_EPS);
    const int nmin = tu.nmin;
    const int maxit = A.maxit_factor * (n > 10 ? n : 10);
    int info = 0;
    int kbot = n - 1, total = 0, ndefl = 0;
    double fl = 0.0;
    while (kbot >= 0) {
        const int ktop = wg_scan(H, ldh, kbot, hnorm, smlnum);
        const int m = kbot - ktop + 1;
        if (m <= nmin) {
            if (m > 1) {  // whole block in LDS, then its factor to the rest
                const int ld = m + 1;
                double *T = lds, *Q = lds + (size_t)m * ld;
                lds_load_block(H, ldh, ktop, m, T, ld, Q, ld);
                int iters = 0;
                const int bad = lds_small_qr(T, ld, Q, ld, m, hnorm, smlnum, 30 * (m > 10 ? m : 10), &iters);
                __syncthreads();
                for (int idx = tid; idx < m * m; idx += NT) {
                    const int i = idx % m, j = idx / m;
                    AT(H, ldh, ktop + i, ktop + j) = (i <= j + 1) ? AT(T, ld, i, j) : 0.0;
                }
                __syncthreads();
                double *stage = pick_stage(T, (size_t)m * ld, Q + (size_t)m * ld, m);
                wg_block_updates(H, ldh, Z, ldz, n, ktop, kbot, Q, ld, stage);
                fl += 10.0 * m * (double)m * m + 2.0 * m * (double)m * (ktop + (n - kbot - 1) + n);
                if (bad > 0) {
                    info = ktop + bad;
                    break;
                }
            }
            kbot = ktop - 1;
            ndefl = 0;
            continue;
        }
        if (++total > maxit) {
            info = kbot + 1;
            break;
        }
        // AED on the trailing window
        int nw = tu.nw < m ? tu.nw : m;
        const int kwtop = kbot - nw + 1;
        const int ld = nw + 1;
        double *T = lds, *V = lds + (size_t)nw * ld, *x = V + (size_t)nw * ld;
        const double s = (kwtop > ktop) ? AT(H, ldh, kwtop, kwtop - 1) : 0.0;
        __syncthreads();
        lds_load_block(H, ldh, kwtop, nw, T, ld, V, ld);
        const AedOut o = aed_core(T, V, ld, x, nw, s, hnorm, smlnum, A.criterion, 30 * (nw > 10 ? nw : 10), s_rr,
                                  s_ri);
        fl += 10.0 * nw * (double)nw * nw;
        if (o.nd > 0) fl += 2.0 * nw * (double)nw * (kwtop + (n - kbot - 1) + n);
        if (o.nd > 0) {
            for (int idx = tid; idx < nw * nw; idx += NT) {
                const int i = idx % nw, j = idx / nw;
                AT(H, ldh, kwtop + i, kwtop + j) = (i <= j + 1) ? AT(T, ld, i, j) : 0.0;
            }
            if (kwtop > ktop && tid == 0) AT(H, ldh, kwtop, kwtop - 1) = o.spike0;
            __syncthreads();
            double *stage = pick_stage(T, (size_t)nw * ld, x + nw, nw);
            wg_block_updates(H, ldh, Z, ldz, n, kwtop, kbot, V, ld, stage);
        }
        kbot -= o.nd;
        ndefl = (o.nd > 0) ? 0 : ndefl + 1;
        const int m2 = kbot - ktop + 1;
        if (m2 <= nmin) continue;
        if (o.nd > 0 && 100 * o.nd > A.nibble * nw) continue;
        // shifts
        int ns = tu.ns;
        if (ns > 2 * B_MAX_BULGES) ns = 2 * B_MAX_BULGES;
        if (ns > m2 / 3) ns = m2 / 3;
        ns -= ns % 2;
        if (ns < 2) ns = 2;
        __syncthreads();
        if (tid == 0) {
            double xr[2 * B_MAX_BULGES], xi[2 * B_MAX_BULGES];
            int got = 0;
            if (ndefl > 0 && ndefl % A.exc == 0) {
                for (int i = kbot; i >= ktop + 2 && got + 2 <= ns; i -= 2) {
                    const double sx = fabs(AT(H, ldh, i, i - 1)) + fabs(AT(H, ldh, i - 1, i - 2));
                    const double c = AT(H, ldh, i, i);
                    xr[got] = c + 0.75 * sx; xi[got] = sqrt(0.4375) * sx;
                    xr[got + 1] = c + 0.75 * sx; xi[got + 1] = -sqrt(0.4375) * sx;
                    got += 2;
                }
            } else {
                got = pick_shifts_dev(s_rr, s_ri, o.nritz, ns, xr, xi);
            }
            if (got < 2) {
                const double a = AT(H, ldh, kbot - 1, kbot - 1), b = AT(H, ldh, kbot - 1, kbot);
                const double c = AT(H, ldh, kbot, kbot - 1), d = AT(H, ldh, kbot, kbot);
                double r1, i1, r2, i2;
                eig2x2(a, b, c, d, &r1, &i1, &r2, &i2);
                if (i1 == 0.0) {
                    const double pick = (fabs(r1 - d) < fabs(r2 - d)) ? r1 : r2;
                    r1 = r2 = pick;
                }
                xr[0] = r1; xi[0] = i1; xr[1] = r2; xi[1] = i2;
                got = 2;
            }
            for (int g = 0; g < got / 2; ++g) {
                s_ptr[g] = xr[2 * g] + xr[2 * g + 1];
                s_pdet[g] = xr[2 * g] * xr[2 * g + 1] - xi[2 * g] * xi[2 * g + 1];
            }
            s_nsh = got;
        }
        __syncthreads();
        // sweep: chains of at most B_MAX_BULGES bulges, one after another
        const int nbulge = s_nsh / 2;
        const int wmax = tu.wchase;
        fl += 20.0 * n * (double)nbulge * (kbot - ktop);
        for (int c0 = 0; c0 < nbulge; c0 += B_MAX_BULGES) {
            const int nb = (nbulge - c0 < B_MAX_BULGES) ? nbulge - c0 : B_MAX_BULGES;
            const int tend = kbot - 1 - ktop + 3 * (nb - 1);
            int t = 0;
            while (t <= tend) {
                const int r0 = (ktop + t - 3 * (nb - 1) > ktop) ? ktop + t - 3 * (nb - 1) : ktop;
                const int r1 = (r0 + wmax - 1 < kbot) ? r0 + wmax - 1 : kbot;
                const int t1 = (r1 < kbot) ? r1 - 3 - ktop + 1 : tend + 1;
                const int b0 = (r0 > 0) ? r0 - 1 : 0;
                const int mb = r1 - b0 + 1, w = r1 - r0 + 1;
                double *Hs = lds, *Us = lds + (size_t)mb * (mb + 1);
                wg_chase_window(H, ldh, ktop, kbot, r0, r1, t, t1, nb, s_ptr + c0, s_pdet + c0, Hs, Us);
                double *stage = pick_stage(Hs, (size_t)mb * (mb + 1), Us + (size_t)w * (w + 1), w);
                wg_update_left(H + r0 + (size_t)(r1 + 1) * ldh, ldh, w, n - r1 - 1, Us, w + 1, stage);
                wg_update_right(H + (size_t)r0 * ldh, ldh, b0, w, Us, w + 1);
                wg_update_right(Z + (size_t)r0 * ldz, ldz, n, w, Us, w + 1);
                t = t1;
            }
        }
    }
    // standardise any decoupled 2x2 block not yet in standard form, then (wr, wi)
    __syncthreads();
    double nflag = 0.0;
    for (int j = tid; j + 1 < n; j += NT) {
        const double c = AT(H, ldh, j + 1, j);
        if (c == 0.0) continue;
        if (j > 0 && AT(H, ldh, j, j - 1) != 0.0) continue;
        if (j + 2 < n && AT(H, ldh, j + 2, j + 1) != 0.0) continue;
        if (!(AT(H, ldh, j, j) == AT(H, ldh, j + 1, j + 1) && AT(H, ldh, j, j + 1) * c < 0.0)) nflag += 1.0;
    }
    nflag = block_reduce(nflag, false);
    for (int j = 0; nflag > 0.0 && j + 1 < n; ++j) {
        const double c = AT(H, ldh, j + 1, j);
        if (c == 0.0) continue;
        if (j > 0 && AT(H, ldh, j, j - 1) != 0.0) continue;
        if (j + 2 < n && AT(H, ldh, j + 2, j + 1) != 0.0) continue;
        const double a = AT(H, ldh, j, j), b = AT(H, ldh, j, j + 1), d = AT(H, ldh, j + 1, j + 1);
        if (a == d && b * c < 0.0) continue;
        const Std2 o = std2x2(a, b, c, d);
        __syncthreads();
        for (int idx = tid; idx < n; idx += NT) {
            if (idx >= j + 2) {
                const double xx = AT(H, ldh, j, idx), yy = AT(H, ldh, j + 1, idx);
                AT(H, ldh, j, idx) = o.cs * xx + o.sn * yy;
                AT(H, ldh, j + 1, idx) = -o.sn * xx + o.cs * yy;
            }
            if (idx < j) {
                const double xx = AT(H, ldh, idx, j), yy = AT(H, ldh, idx, j + 1);
                AT(H, ldh, idx, j) = o.cs * xx + o.sn * yy;
                AT(H, ldh, idx, j + 1) = -o.sn * xx + o.cs * yy;
            }
            const double xx = AT(Z, ldz, idx, j), yy = AT(Z, ldz, idx, j + 1);
            AT(Z, ldz, idx, j) = o.cs * xx + o.sn * yy;
            AT(Z, ldz, idx, j + 1) = -o.sn * xx + o.cs * yy;
        }
        if (tid == 0) {
            AT(H, ldh, j, j) = o.a; AT(H, ldh, j, j + 1) = o.b;
            AT(H, ldh, j + 1, j) = o.c; AT(H, ldh, j + 1, j + 1) = o.d;
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += NT) {
        const bool starts = (j + 1 < n) && AT(H, ldh, j + 1, j) != 0.0;
        const bool ends = (j > 0) && AT(H, ldh, j, j - 1) != 0.0;
        if (starts && !ends) {
            P.wr[j] = AT(H, ldh, j, j);
            P.wi[j] = sqrt(fabs(AT(H, ldh, j, j + 1))) * sqrt(fabs(AT(H, ldh, j + 1, j)));
        } else if (ends && !(j >= 2 && AT(H, ldh, j - 1, j - 2) != 0.0)) {
            P.wr[j] = AT(H, ldh, j, j);
            P.wi[j] = -(sqrt(fabs(AT(H, ldh, j - 1, j))) * sqrt(fabs(AT(H, ldh, j, j - 1))));
        } else {
            P.wr[j] = AT(H, ldh, j, j);
            P.wi[j] = 0.0;
        }
    }
    __syncthreads();
    *flops = fl;
    return info;
}

extern "C" __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) k_batched(BArgs A) {
    extern __shared__ double lds[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(A.next, 1);
        __syncthreads();
        const int k = s_idx;
        __syncthreads();
        if (k >= A.nprob) break;
        const int p = A.order[k];
        const BProb P = A.probs[p];
        if (P.pad) continue;  // rejected by k_batched_pack (uniform across the workgroup)
        int b = 0;
        while (b + 1 < B_NBUCKET && P.n > A.bucket_hi[b]) ++b;
        double fl = 0.0;
        const int info = solve_one(P, A.tune[b], A, lds, &fl);
        if (threadIdx.x == 0) {
            A.info[p] = info;
            atomicAdd((double *)(A.next + 2), fl);
        }
        __syncthreads();
    }
}

// Problem descriptors from the caller's device arrays, per-problem argument
// checks (a rejected problem gets its negative code in info and is skipped), the
// largest-first processing order (rank of each problem by descending order, ties
// by index), and the reset of the work counter.  Everything the persistent kernel
// reads is rebuilt here on the device, so a captured launch pair replays
// correctly with whatever the caller's arrays hold at replay time.
extern "C" __global__ void __launch_bounds__(256) k_batched_pack(BProb *out, int *order, int *next, int *info,
                                                                  const int *n, const int *ldh, const int *ldz,
                                                                  double *const *H, double *const *Z,
                                                                  double *const *wr, double *const *wi, int batch) {
    __shared__ int sk[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const bool mine = b < batch;
    if (b == 0) {
        *next = 0;
        *(double *)(next + 2) = 0.0;  // the launch's flop count
    }
    int key = -1;
    if (mine) {
        BProb p;
        p.H = H[b]; p.Z = Z[b]; p.wr = wr[b]; p.wi = wi[b];
        p.n = n[b]; p.ldh = ldh[b]; p.ldz = ldz[b];
        int code = 0;
        if (p.n < 0) code = -2;
        else if (p.n > 0 && !p.H) code = -3;
        else if (p.ldh < max(1, p.n)) code = -4;
        else if (p.n > 0 && !p.Z) code = -5;
        else if (p.ldz < max(1, p.n)) code = -6;
        else if (p.n > 0 && !p.wr) code = -7;
        else if (p.n > 0 && !p.wi) code = -8;
        p.pad = code;
        out[b] = p;
        if (code) info[b] = code;
        key = max(p.n, -1);  // the key every thread computes for this problem
    }
    // rank = number of problems that come before this one: larger order, or the
    // same order and a smaller index; the sizes pass through LDS 256 at a time
    int rank = 0;
    for (int c0 = 0; c0 < batch; c0 += 256) {
        const int c = c0 + (int)threadIdx.x;
        sk[threadIdx.x] = (c < batch) ? max(n[c], -1) : -2;
        __syncthreads();
        const int lim = min(256, batch - c0);
        for (int u = 0; u < lim; ++u) {
            const int kc = sk[u];
            rank += (kc > key) || (kc == key && c0 + u < b);
        }
        __syncthreads();
    }
    if (mine) order[rank] = b;
}
