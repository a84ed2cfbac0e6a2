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
#define HRD_GC 256       // vector entries per GEMV workgroup

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
    double vnew = 0.0, ycol = 0.0;
    if (in) {
        // reflector i-1: its vector, its column of H, its column of Y
        const double scal = p.st->scal, tau = p.st->tau, beta = p.st->beta;
        const double old = AT(p.A, p.lda, g, j - 1);
        vnew = r < i - 1 ? 0.0 : (r == i - 1 ? 1.0 : old * scal);
        AT(p.V, p.ldw, r, i - 1) = vnew;
        if (r >= i - 1) AT(p.A, p.lda, g, j - 1) = (r == i - 1) ? beta : 0.0;
        double y = AT(p.A, p.lda, g, j);
        for (int ch = 0; ch < p.nch; ++ch) y += p.zpart[(size_t)ch * p.ldw + r];
        double acc = 0.0;
        for (int c = 0; c < i - 1; ++c) acc = fma(AT(p.Y, p.ldw, g, c), uprev[c], acc);
        ycol = tau * (y - acc);
        AT(p.Y, p.ldw, g, i - 1) = ycol;
    }
    if (i == p.jb) return;  // the panel's last finishing launch
    double x[HRD_NB];
#pragma unroll
    for (int c = 0; c < HRD_NB; ++c) x[c] = 0.0;
    if (in) {
        // right: a -= Y(g, 0:i) V(i-1, 0:i)^T   (V(i-1, i-1) = 1)
        double acc = ycol;
        for (int c = 0; c < i - 1; ++c) acc = fma(AT(p.Y, p.ldw, g, c), vrow[c], acc);
        const double a = AT(p.A, p.lda, g, j) - acc;
        AT(p.A, p.lda, g, j) = a;
#pragma unroll
        for (int c = 0; c < HRD_NB; ++c) {
            if (c < i - 1) x[c] = AT(p.V, p.ldw, r, c) * a;
            else if (c == i - 1) x[c] = vnew * a;
        }
    }
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
    if (t < HRD_NB) {
        double w = 0.0;
        for (int b = 0; b < (int)gridDim.x; ++b) w += p.part[(size_t)b * (HRD_NB + 2) + t];
        red[0][t] = w;
    }
    __syncthreads();
    if (t < i) {
        // s = T^T w, T upper triangular
        double s = 0.0;
        for (int c = 0; c <= t; ++c) s = fma(p.T[c + (size_t)t * HRD_NB], red[0][c], s);
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
        double a = AT(p.A, p.lda, g, j);
        if (i > 0) {
            double acc = 0.0;
            for (int c = 0; c < i; ++c) acc = fma(AT(p.V, p.ldw, r, c), s[c], acc);
            a -= acc;
            AT(p.A, p.lda, g, j) = a;
        }
        if (r > i) {
            if (a != 0.0) {
                sc = fabs(a);
                sq = 1.0;
            }
#pragma unroll
            for (int c = 0; c < HRD_NB; ++c)
                if (c < i) x[c] = AT(p.V, p.ldw, r, c) * a;
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
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)gridDim.x; ++q) {
            const double *pq = p.part + (size_t)q * (HRD_NB + 2);
            hrd_ssq_merge(a, b, pq[HRD_NB], pq[HRD_NB + 1]);
        }
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
        double v = 0.0;
        for (int q = 0; q < (int)gridDim.x; ++q) v += p.part[(size_t)q * (HRD_NB + 2) + t];
        const double u = AT(p.V, p.ldw, i, t) + coef[1] * v;
        ufin[t] = u;
        p.st->u[t] = u;
    }
    __syncthreads();
    if (t < HRD_NB) {
        // column i of T: T(0:i, i) = -tau T(0:i, 0:i) u, T(i, i) = tau, zero below
        double v = 0.0;
        if (t < i) {
            for (int c = t; c < i; ++c) v = fma(p.T[t + (size_t)c * HRD_NB], ufin[c], v);
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
    __shared__ double v[HRD_GC];
    const int t = threadIdx.x;
    const int c0 = p.i + 1 + blockIdx.y * HRD_GC;
    const int cn = min(HRD_GC, p.m - c0);
    const int j = p.k0 + p.i;
    const size_t base = (size_t)p.k0 + 1;
    if (t < cn) v[t] = AT(p.A, p.lda, base + c0 + t, j) * p.st->scal;
    __syncthreads();
    const int r0 = blockIdx.x * HRD_GR + t, r1 = r0 + HRD_THREADS;
    const bool in0 = r0 < p.m, in1 = r1 < p.m;
    const double *col = p.A + (base + c0) * (size_t)p.lda + base;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int c = 0;
    if (in1) {
        for (; c + 2 <= cn; c += 2) {
            const double *c1 = col + (size_t)c * p.lda;
            const double *c2 = c1 + p.lda;
            a0 = fma(c1[r0], v[c], a0);
            a1 = fma(c1[r1], v[c], a1);
            b0 = fma(c2[r0], v[c + 1], b0);
            b1 = fma(c2[r1], v[c + 1], b1);
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
// workgroup, K in 32-wide LDS-staged steps, four waves of 16 rows each.
// Operand layouts of v_mfma_f64_16x16x4_f64 (lane l): A(l%16, l/16),
// B(l/16, l%16); accumulator double r of lane l holds D(l/16 + 4r, l%16).
extern "C" __global__ void __launch_bounds__(HRD_THREADS) k_hrd_skinny(SkArgs p) {
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
    for (int kb = ks; kb < ke; kb += 32) {
        for (int idx = t; idx < 64 * 32; idx += HRD_THREADS) {
            int ii, kk;
            double v = 0.0;
            if (p.trans == 0) {
                ii = idx & 63;
                kk = idx >> 6;
                if (i0 + ii < p.M && kb + kk < ke) v = AT(p.C, p.ldc, i0 + ii, kb + kk);
            } else {
                kk = idx & 31;
                ii = idx >> 5;
                if (i0 + ii < p.M && kb + kk < ke) v = AT(p.C, p.ldc, kb + kk, i0 + ii);
            }
            Cs[ii * HRD_PAD + kk] = v;
            const int vk = idx & 31, vc = idx >> 5;
            Vs[vc * HRD_PAD + vk] = (vc < p.nbc && kb + vk < ke) ? AT(p.V, p.ldv, kb + vk, vc) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < 32; k4 += 4) {
            const double a = Cs[(16 * q + li) * HRD_PAD + k4 + lk];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                if (ct < nct) acc[ct] = hrd_mfma(a, Vs[(16 * ct + li) * HRD_PAD + k4 + lk], acc[ct]);
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
