// hessenberg.hip -- reduction of a general matrix to upper Hessenberg form,
// A = Q1 H Q1^T (Section 2, eq. 3), by the standard blocked algorithm of
// Section 3.1 (Fig. 2): panels of reflectors I - tau v v^T accumulated in the
// compact WY form I - V T V^T together with Y = A V T; then the trailing update
// A <- (I - V T V^T)^T (A - Y V^T) and the top-part update A <- A - Y V^T.
//
// Per panel column (three launches, all on the caller's stream):
//   k_hrd_a   finish the previous reflector (its v into V, its column of H, the
//             column Y(:, i-1) = tau (A v - Y u)), then apply the panel's earlier
//             reflectors to the new column from the right (a -= Y V(j, :)^T) and
//             form w = V^T a;
//   k_hrd_b   apply them from the left (a -= V T^T w), build the new reflector
//             (alpha, scaled norm of the tail, beta, tau), u = V^T v and the new
//             column of T;
//   k_hrd_gemv  the large matrix-vector product A(:, j+2:n) v over the trailing
//             part, split over row blocks x column chunks (the memory-bound 20%
//             of the flops); the partial sums go to a workspace and are added by
//             the next k_hrd_a.
// The reductions that end each column kernel (w, the tail norm, u) are done by
// the last workgroup to finish (a device-scope counter; no workgroup waits for
// another), in a fixed order, so results do not depend on scheduling.
//
// Per panel (FP64 matrix-core kernels): k_hrd_skinny forms the thin products
// A_top V, Y^T V, A_t^T V and Q V (split over the long dimension), k_hrd_reduce
// sums the partials and applies T (and a correction), and k_hrd_rank applies a
// rank-r update C -= L1 R1^T + L2 R2^T in place.
//
// Index conventions: the panel starts at column k0; its reflectors act on rows
// and columns k0+1..n-1.  "Local row" r = global row - (k0 + 1), 0 <= r < m,
// m = n - k0 - 1.  Reflector i (column j = k0 + i) has v(r) = 0 for r < i,
// v(i) = 1.  V (m x nb) is stored by local rows, Y (n x nb) by global rows.
#include "neig_dev.h"

#define HRD_NB 64        // largest panel width
#define HRD_THREADS 256
#define HRD_RB 256       // rows per workgroup in k_hrd_a / k_hrd_b
#define HRD_GR 512       // rows per workgroup in the GEMV (two per thread)
#define HRD_GC 256       // vector entries per GEMV workgroup (512 for large trailing blocks)
#define HRD_GC_MAX 512

struct HrdState {
    double alpha, beta, tau, scal;
    double s[HRD_NB];     // T^T w for the current column
    double u[HRD_NB];     // V^T v of the newest reflector
    unsigned int count_a, count_b;
};

struct HrdArgs {
    double *A;
    double *V, *Y, *T;     // V, Y: leading dimension ldw; T: HRD_NB x HRD_NB
    double *part;          // per-workgroup partials, HRD_NB + 2 per workgroup
    double *zpart;         // GEMV partials, chunk-major, leading dimension ldw
    HrdState *st;
    int lda, ldw;
    int n, k0, m, i, jb, nch;  // nch: chunks of the previous GEMV
    int cw;                    // vector entries per GEMV chunk (HRD_GC or HRD_GC_MAX)
};

// Sum x[c] (c < 64) over the 64 lanes of a wavefront by recursive halving:
// afterwards lane l returns the total of entry l.  63 shuffles.
template <int S>
__device__ __forceinline__ void hrd_halve(double (&x)[HRD_NB], int lane) {
    const bool up = (lane & S) != 0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double send = up ? x[k] : x[k + S];
        const double keep = up ? x[k + S] : x[k];
        x[k] = keep + __shfl_xor(send, S);
    }
}

__device__ __forceinline__ double hrd_transpose_sum(double (&x)[HRD_NB], int lane) {
    hrd_halve<32>(x, lane);
    hrd_halve<16>(x, lane);
    hrd_halve<8>(x, lane);
    hrd_halve<4>(x, lane);
    hrd_halve<2>(x, lane);
    hrd_halve<1>(x, lane);
    return x[0];
}

// Column sums over the workgroups' partials (nblk rows of stride HRD_NB + 2)
// for the first 64 entries, by all 256 threads: thread (c, q) adds the blocks
// q, q + 4, ... in order, then the four quarter sums are added in order; the
// totals land in out[0..63].  The order is fixed, so results are reproducible.
__device__ __forceinline__ void hrd_sum_partials(const double *part, int nblk, double (*red)[HRD_NB],
                                                 double *out) {
    const int t = threadIdx.x, c = t & 63, q = t >> 6;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = q;
    for (; b + 12 < nblk; b += 16) {
        a0 += part[(size_t)b * (HRD_NB + 2) + c];
        a1 += part[(size_t)(b + 4) * (HRD_NB + 2) + c];
        a2 += part[(size_t)(b + 8) * (HRD_NB + 2) + c];
        a3 += part[(size_t)(b + 12) * (HRD_NB + 2) + c];
    }
    for (; b < nblk; b += 4) a0 += part[(size_t)b * (HRD_NB + 2) + c];
    red[q][c] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (t < HRD_NB) out[t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    __syncthreads();
}

// Stage the panel's T (HRD_NB x HRD_NB) in LDS.
__device__ __forceinline__ void hrd_stage_t(const double *T, double *Ts) {
    for (int idx = threadIdx.x; idx < HRD_NB * HRD_NB; idx += HRD_THREADS) Ts[idx] = T[idx];
    __syncthreads();
}

// (scale, ssq) representation of a sum of squares: value = scale^2 * ssq.
__device__ __forceinline__ void hrd_ssq_merge(double &sc, double &sq, double sc2, double sq2) {
    if (sc2 == 0.0) return;
    if (sc < sc2) {
        const double r = sc / sc2;
        sq = sq2 + sq * r * r;
        sc = sc2;
    } else {
        const double r = sc2 / sc;
        sq += sq2 * r * r;
    }
}

// Finish reflector i-1 (if any) and apply the panel's earlier reflectors to
// column j = k0 + i from the right; partial w = V^T a per workgroup; the last
// workgroup forms s = T^T w.
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_a(HrdArgs p) {
    __shared__ double vrow[HRD_NB];
    __shared__ double uprev[HRD_NB];
    __shared__ double red[HRD_THREADS / 64][HRD_NB];
    __shared__ int is_last;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int i = p.i;
    const int r = blockIdx.x * HRD_RB + t;
    const bool in = r < p.m;
    const size_t g = (size_t)p.k0 + 1 + r;
    const int j = p.k0 + i;
    if (t < i - 1) {
        vrow[t] = AT(p.V, p.ldw, i - 1, t);
        uprev[t] = p.st->u[t];
    }
    __syncthreads();
    const bool last = i == p.jb;  // the panel's last launch only finishes reflector i-1
    double x[HRD_NB];
#pragma unroll
    for (int c = 0; c < HRD_NB; ++c) x[c] = 0.0;
    if (in) {
        // reflector i-1: its vector, its column of H, its column of Y; with one
        // pass over Y(g, 0:i-1) both Y u and the right update Y V(i-1, :)^T
        const double scal = p.st->scal, tau = p.st->tau, beta = p.st->beta;
        const double old = AT(p.A, p.lda, g, j - 1);
        const double vnew = r < i - 1 ? 0.0 : (r == i - 1 ? 1.0 : old * scal);
        AT(p.V, p.ldw, r, i - 1) = vnew;
        if (r >= i - 1) AT(p.A, p.lda, g, j - 1) = (r == i - 1) ? beta : 0.0;
        const double aj = AT(p.A, p.lda, g, j);  // column j, not yet touched by this panel
        // the GEMV partials, eight loads in flight, added in a fixed order
        double z[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int ch = 0;
        for (; ch + 8 <= p.nch; ch += 8) {
            const double *zp = p.zpart + (size_t)ch * p.ldw + r;
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] += zp[u * (size_t)p.ldw];
        }
        for (; ch < p.nch; ++ch) z[0] += p.zpart[(size_t)ch * p.ldw + r];
        const double y = aj + (((z[0] + z[1]) + (z[2] + z[3])) + ((z[4] + z[5]) + (z[6] + z[7])));
        double yu = 0.0, yv = 0.0;
#pragma unroll 8
        for (int c = 0; c < i - 1; ++c) {
            const double yc = AT(p.Y, p.ldw, g, c);
            yu = fma(yc, uprev[c], yu);
            yv = fma(yc, vrow[c], yv);
        }
        const double ycol = tau * (y - yu);
        AT(p.Y, p.ldw, g, i - 1) = ycol;
        if (!last) {
            // right: a -= Y(g, 0:i) V(i-1, 0:i)^T   (V(i-1, i-1) = 1)
            const double a = aj - (yv + ycol);
            AT(p.A, p.lda, g, j) = a;
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c) {
                if (c < i - 1) x[c] = AT(p.V, p.ldw, r, c) * a;
                else if (c == i - 1) x[c] = vnew * a;
            }
        }
    }
    if (last) return;
    const double ws = hrd_transpose_sum(x, lane);
    red[wv][lane] = ws;
    __syncthreads();
    if (t < HRD_NB) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < HRD_THREADS / 64; ++q) s += red[q][t];
        p.part[(size_t)blockIdx.x * (HRD_NB + 2) + t] = s;
    }
    __threadfence();
    __syncthreads();
    if (t == 0) is_last = atomicAdd(&p.st->count_a, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    __shared__ double Ts[HRD_NB * HRD_NB];
    __shared__ double wsum[HRD_NB];
    hrd_sum_partials(p.part, gridDim.x, red, wsum);
    hrd_stage_t(p.T, Ts);
    if (t < i) {
        // s = T^T w, T upper triangular
        double s = 0.0;
        for (int c = 0; c <= t; ++c) s = fma(Ts[c + t * HRD_NB], wsum[c], s);
        p.st->s[t] = s;
    }
    if (t == 0) p.st->count_a = 0;
}

// Left application a -= V s of the earlier reflectors, then the reflector of
// the column's tail: partial scaled sums of squares and u' = V^T tail per
// workgroup; the last workgroup forms alpha, beta, tau, 1/(alpha - beta), u and
// the new column of T.
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_b(HrdArgs p) {
    __shared__ double s[HRD_NB];
    __shared__ double red[HRD_THREADS / 64][HRD_NB];
    __shared__ double rsc[HRD_THREADS / 64], rsq[HRD_THREADS / 64];
    __shared__ int is_last;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int i = p.i;
    const int r = blockIdx.x * HRD_RB + t;
    const bool in = r < p.m;
    const size_t g = (size_t)p.k0 + 1 + r;
    const int j = p.k0 + i;
    if (t < i) s[t] = p.st->s[t];
    __syncthreads();
    double x[HRD_NB];
#pragma unroll
    for (int c = 0; c < HRD_NB; ++c) x[c] = 0.0;
    double sc = 0.0, sq = 0.0;
    if (in) {
        // the row of V is read once: held in x, then replaced by V(r, c) a
        double a = AT(p.A, p.lda, g, j);
        if (i > 0) {
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c)
                if (c < i) x[c] = AT(p.V, p.ldw, r, c);
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c)
                if (c < i) acc = fma(x[c], s[c], acc);
            a -= acc;
            AT(p.A, p.lda, g, j) = a;
        }
        if (r > i) {
            if (a != 0.0) {
                sc = fabs(a);
                sq = 1.0;
            }
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c) x[c] *= a;
        } else {
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c) x[c] = 0.0;
        }
    }
    const double us = hrd_transpose_sum(x, lane);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double sc2 = __shfl_xor(sc, o), sq2 = __shfl_xor(sq, o);
        hrd_ssq_merge(sc, sq, sc2, sq2);
    }
    red[wv][lane] = us;
    if (lane == 0) {
        rsc[wv] = sc;
        rsq[wv] = sq;
    }
    __syncthreads();
    double *mine = p.part + (size_t)blockIdx.x * (HRD_NB + 2);
    if (t < HRD_NB) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < HRD_THREADS / 64; ++q) v += red[q][t];
        mine[t] = v;
    }
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < HRD_THREADS / 64; ++q) hrd_ssq_merge(a, b, rsc[q], rsq[q]);
        mine[HRD_NB] = a;
        mine[HRD_NB + 1] = b;
    }
    __threadfence();
    __syncthreads();
    if (t == 0) is_last = atomicAdd(&p.st->count_b, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    __shared__ double coef[2];
    __shared__ double ufin[HRD_NB];
    __shared__ double usum[HRD_NB];
    __shared__ double Ts[HRD_NB * HRD_NB];
    hrd_sum_partials(p.part, gridDim.x, red, usum);
    hrd_stage_t(p.T, Ts);
    if (t < 64) {
        // the tail's scaled sum of squares: lane l merges blocks l, l + 64, ...
        // in order, then the lanes merge by a fixed butterfly
        double a = 0.0, b = 0.0;
        for (int q = t; q < (int)gridDim.x; q += 64) {
            const double *pq = p.part + (size_t)q * (HRD_NB + 2);
            hrd_ssq_merge(a, b, pq[HRD_NB], pq[HRD_NB + 1]);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double a2 = __shfl_xor(a, o), b2 = __shfl_xor(b, o);
            hrd_ssq_merge(a, b, a2, b2);
        }
        rsc[0] = a;   // every lane holds the same merged pair
        rsq[0] = b;
    }
    __syncthreads();
    if (t == 0) {
        const double a = rsc[0], b = rsq[0];
        const double sigma = a * sqrt(b);
        const double alpha = AT(p.A, p.lda, (size_t)p.k0 + 1 + i, j);
        double beta = alpha, tau = 0.0, scal = 0.0;
        if (sigma != 0.0) {
            const double nrm = hypot(alpha, sigma);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        p.st->alpha = alpha;
        p.st->beta = beta;
        p.st->tau = tau;
        p.st->scal = scal;
        coef[0] = tau;
        coef[1] = scal;
    }
    __syncthreads();
    if (t < i) {
        const double u = AT(p.V, p.ldw, i, t) + coef[1] * usum[t];
        ufin[t] = u;
        p.st->u[t] = u;
    }
    __syncthreads();
    if (t < HRD_NB) {
        // column i of T: T(0:i, i) = -tau T(0:i, 0:i) u, T(i, i) = tau, zero below
        double v = 0.0;
        if (t < i) {
            for (int c = t; c < i; ++c) v = fma(Ts[t + c * HRD_NB], ufin[c], v);
            v *= -coef[0];
        } else if (t == i) {
            v = coef[0];
        }
        p.T[t + (size_t)i * HRD_NB] = v;
    }
    if (t == 0) p.st->count_b = 0;
}

// z(r) = sum over the chunk's entries c of A(k0+1+r, k0+1+c) * scal * a(c),
// a = column j's tail (local entries i+1..m-1).  Grid: row blocks x chunks.
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_gemv(HrdArgs p) {
    __shared__ double v[HRD_GC_MAX];
    const int t = threadIdx.x;
    const int c0 = p.i + 1 + blockIdx.y * p.cw;
    const int cn = min(p.cw, p.m - c0);
    const int j = p.k0 + p.i;
    const size_t base = (size_t)p.k0 + 1;
    const double scal = p.st->scal;
    for (int u = t; u < cn; u += HRD_THREADS) v[u] = AT(p.A, p.lda, base + c0 + u, j) * scal;
    __syncthreads();
    const int r0 = blockIdx.x * HRD_GR + t, r1 = r0 + HRD_THREADS;
    const bool in0 = r0 < p.m, in1 = r1 < p.m;
    const double *col = p.A + (base + c0) * (size_t)p.lda + base;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int c = 0;
    if (in1) {
        // sixteen independent loads in flight per lane before their first use
        const size_t ld = (size_t)p.lda;
        for (; c + 8 <= cn; c += 8) {
            const double *c1 = col + (size_t)c * p.lda;
            double x0[8], x1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                x0[u] = c1[u * ld + r0];
                x1[u] = c1[u * ld + r1];
            }
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                a0 = fma(x0[u], v[c + u], a0);
                a1 = fma(x1[u], v[c + u], a1);
                b0 = fma(x0[u + 1], v[c + u + 1], b0);
                b1 = fma(x1[u + 1], v[c + u + 1], b1);
            }
        }
        for (; c < cn; ++c) {
            const double *c1 = col + (size_t)c * p.lda;
            a0 = fma(c1[r0], v[c], a0);
            a1 = fma(c1[r1], v[c], a1);
        }
    } else if (in0) {
        for (; c + 2 <= cn; c += 2) {
            const double *c1 = col + (size_t)c * p.lda;
            a0 = fma(c1[r0], v[c], a0);
            b0 = fma(c1[r0 + p.lda], v[c + 1], b0);
        }
        for (; c < cn; ++c) a0 = fma(col[(size_t)c * p.lda + r0], v[c], a0);
    }
    double *z = p.zpart + (size_t)blockIdx.y * p.ldw;
    if (in0) z[r0] = a0 + b0;
    if (in1) z[r1] = a1 + b1;
}

// ---------------------------------------------------------------- panel GEMMs

#define HRD_PAD 34   // LDS row pitch (doubles) of 32-wide operand slices: conflict-free reads

struct SkArgs {
    const double *C;   // trans 0: M x K; trans 1: K x M
    const double *V;   // K x nbc
    double *P;         // partials: split s at P + s * sp, M x nbc, leading dimension M
    size_t sp;
    int ldc, ldv, M, K, nbc, kper, trans;
};

__device__ __forceinline__ neig_d4 hrd_mfma(double a, double b, neig_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// P_s(i, c) = sum over k in split s of op(C)(i, k) V(k, c): 64 output rows per
// workgroup, K in 32-wide LDS-staged steps, four waves of 16 rows each; the
// next step's operands are loaded into registers while the matrix cores work
// on the current one.
// Operand layouts of v_mfma_f64_16x16x4_f64 (lane l): A(l%16, l/16),
// B(l/16, l%16); accumulator double r of lane l holds D(l/16 + 4r, l%16).
template <int TRANS>
__device__ __forceinline__ void hrd_skinny_body(const SkArgs &p) {
    __shared__ double Cs[64 * HRD_PAD];
    __shared__ double Vs[64 * HRD_PAD];
    const int t = threadIdx.x, lane = t & 63, q = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int i0 = blockIdx.x * 64;
    const int ks = blockIdx.y * p.kper;
    const int ke = min(p.K, ks + p.kper);
    neig_d4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = (neig_d4){0.0, 0.0, 0.0, 0.0};
    const int nct = (p.nbc + 15) >> 4;
    double rc[8], rv[8];
    auto fetch = [&](int kb) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = t + u * HRD_THREADS;
            int ii, kk;
            if (TRANS == 0) {
                ii = idx & 63;
                kk = idx >> 6;
                rc[u] = (i0 + ii < p.M && kb + kk < ke) ? AT(p.C, p.ldc, i0 + ii, kb + kk) : 0.0;
            } else {
                kk = idx & 31;
                ii = idx >> 5;
                rc[u] = (i0 + ii < p.M && kb + kk < ke) ? AT(p.C, p.ldc, kb + kk, i0 + ii) : 0.0;
            }
            const int vk = idx & 31, vc = idx >> 5;
            rv[u] = (vc < p.nbc && kb + vk < ke) ? AT(p.V, p.ldv, kb + vk, vc) : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = t + u * HRD_THREADS;
            const int ii = TRANS == 0 ? (idx & 63) : (idx >> 5);
            const int kk = TRANS == 0 ? (idx >> 6) : (idx & 31);
            Cs[ii * HRD_PAD + kk] = rc[u];
            Vs[(idx >> 5) * HRD_PAD + (idx & 31)] = rv[u];
        }
    };
    if (ks < ke) fetch(ks);
    for (int kb = ks; kb < ke; kb += 32) {
        store();
        __syncthreads();
        if (kb + 32 < ke) fetch(kb + 32);
#pragma unroll
        for (int k4 = 0; k4 < 32; k4 += 4) {
            const double a = Cs[(16 * q + li) * HRD_PAD + k4 + lk];
            // all four column tiles (V is zero beyond nbc): no runtime branch
            // between the matrix-core instructions
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[ct] = hrd_mfma(a, Vs[(16 * ct + li) * HRD_PAD + k4 + lk], acc[ct]);
        }
        __syncthreads();
    }
    double *P = p.P + (size_t)blockIdx.y * p.sp;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = 16 * ct + li;
        if (ct < nct && col < p.nbc) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int row = i0 + 16 * q + lk + 4 * rr;
                if (row < p.M) P[row + (size_t)col * p.M] = acc[ct][rr];
            }
        }
    }
}

extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_skinny_n(SkArgs p) { hrd_skinny_body<0>(p); }
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_skinny_t(SkArgs p) { hrd_skinny_body<1>(p); }

struct RdArgs {
    const double *P;   // ns partials of M x nbc (leading dimension M), stride sp
    size_t sp;
    int ns;
    const double *X;   // optional M x nbc (leading dimension ldx): subtract X B
    int ldx;
    const double *B;   // nbc x nbc, leading dimension HRD_NB
    const double *T;   // optional nbc x nbc upper triangular, leading dimension HRD_NB
    double *out;
    int ldo, M, nbc;
};

// out = (sum_s P_s - X B) T, row by row; 64 rows per workgroup.
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_reduce(RdArgs p) {
    __shared__ double xs[64 * (HRD_NB + 1)];
    const int t = threadIdx.x;
    const int row = t & 63, cg = t >> 6;
    const int i = blockIdx.x * 64 + row;
    const bool in = i < p.M;
    for (int c = 16 * cg; c < 16 * cg + 16; ++c) {
        double v = 0.0;
        if (in && c < p.nbc) {
            for (int s = 0; s < p.ns; ++s) v += p.P[(size_t)s * p.sp + i + (size_t)c * p.M];
            if (p.X) {
                double acc = 0.0;
                for (int k = 0; k < p.nbc; ++k) acc = fma(AT(p.X, p.ldx, i, k), p.B[k + (size_t)c * HRD_NB], acc);
                v -= acc;
            }
        }
        xs[row * (HRD_NB + 1) + c] = v;
    }
    __syncthreads();
    if (!in) return;
    for (int c = 16 * cg; c < 16 * cg + 16 && c < p.nbc; ++c) {
        double v;
        if (p.T) {
            v = 0.0;
            for (int k = 0; k <= c; ++k) v = fma(xs[row * (HRD_NB + 1) + k], p.T[k + (size_t)c * HRD_NB], v);
        } else {
            v = xs[row * (HRD_NB + 1) + c];
        }
        AT(p.out, p.ldo, i, c) = v;
    }
}

struct RkArgs {
    double *C;
    const double *L1, *R1, *L2, *R2;
    int ldc, ldl1, ldr1, ldl2, ldr2;
    int M, N, r1, r2;
};

// C (M x N) -= L1 R1^T + L2 R2^T, in place: 64 x 64 tile per workgroup, the
// transposed tile accumulated on the matrix cores so that each lane group
// reads and writes 16 consecutive rows of a column; L and R staged in LDS 32
// columns at a time.
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_rank(RkArgs p) {
    __shared__ double Ls[64 * HRD_PAD];
    __shared__ double Rs[64 * HRD_PAD];
    const int t = threadIdx.x, lane = t & 63, q = t >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int i0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    // lane holds D(lk + 4 rr, li) = C^T(col, row): col = c0 + 16 q + lk + 4 rr, row = i0 + 16 it + li
    neig_d4 acc[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int row = i0 + 16 * it + li, col = c0 + 16 * q + lk + 4 * rr;
            acc[it][rr] = (row < p.M && col < p.N) ? AT(p.C, p.ldc, row, col) : 0.0;
        }
    }
    const int rt = p.r1 + p.r2;
    for (int kc = 0; kc < rt; kc += 32) {
        for (int idx = t; idx < 64 * 32; idx += HRD_THREADS) {
            const int ii = idx & 63, kk = idx >> 6;
            const int k = kc + kk;
            double lv = 0.0, rv = 0.0;
            if (k < p.r1) {
                if (i0 + ii < p.M) lv = AT(p.L1, p.ldl1, i0 + ii, k);
                if (c0 + ii < p.N) rv = AT(p.R1, p.ldr1, c0 + ii, k);
            } else if (k < rt) {
                if (i0 + ii < p.M) lv = AT(p.L2, p.ldl2, i0 + ii, k - p.r1);
                if (c0 + ii < p.N) rv = AT(p.R2, p.ldr2, c0 + ii, k - p.r1);
            }
            Ls[ii * HRD_PAD + kk] = lv;
            Rs[ii * HRD_PAD + kk] = -rv;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < 32; k4 += 4) {
            const double a = Rs[(16 * q + li) * HRD_PAD + k4 + lk];
#pragma unroll
            for (int it = 0; it < 4; ++it)
                acc[it] = hrd_mfma(a, Ls[(16 * it + li) * HRD_PAD + k4 + lk], acc[it]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int row = i0 + 16 * it + li, col = c0 + 16 * q + lk + 4 * rr;
            if (row < p.M && col < p.N) AT(p.C, p.ldc, row, col) = acc[it][rr];
        }
    }
}
