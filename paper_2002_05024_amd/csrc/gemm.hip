// gemm.hip -- the left / right update tasks (Section 3.2): apply a window's
// accumulated orthogonal factor U (w x w, w <= 96, given as U^T) to an
// off-diagonal strip of H or Z, in place, with FP64 matrix-core instructions
// (v_mfma_f64_16x16x4_f64).
//
//   side 0 (left):  C (w x len)  <- U^T C   the rows of a window, right of it
//   side 1 (right): C (len x w)  <- C U     the columns of a window, above it / Z
//
// One launch carries several strips ("tasks"); each workgroup owns a 64-wide
// slice of one strip (64 columns for side 0, 64 rows for side 1), reads all of
// it before writing, so in-place is safe.  U^T is staged in LDS once per
// workgroup.  Four waves; each wave owns one 16-wide column (side 0) or row
// (side 1) tile of the slice and loops over all of the window's 16-row tiles;
// the strip operand comes from LDS (side 0) or from registers loaded all at
// once at the start (side 1).
//
// Operand layouts of v_mfma_f64_16x16x4_f64 (lane l, 64 lanes): A(16x4) element
// (l%16, l/16); B(4x16) element (l/16, l%16); the four accumulator doubles of
// lane l hold D(l/16 + 4r, l%16), r = 0..3.
#include "neig_dev.h"

#define UPD_THREADS 256
#define UPD_MAX_TASKS 48
#define UPD_WMAX 96  // larger factors go to k_update_wide (U^T and the slice would not fit in LDS)
#define UPD_SLICE 64

struct UpdTask {
    double *C;
    const double *Ut;
    int ldc, ldu, w, len, side, tile0;
};

struct UpdArgs {
    UpdTask t[UPD_MAX_TASKS];
    int ntask;
};

__device__ __forceinline__ neig_d4 mfma16(double a, double b, neig_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The body for a window of NRT 16-row tiles (w <= 16 NRT): every loop has a
// compile-time trip count, so the matrix-core instructions issue back to back
// with no branch between them (the zero padding of U^T and of the staged strip
// makes the extra k-steps harmless).
template <int NRT>
__device__ __forceinline__ void upd_body(const UpdTask &T, int tile, double *lds) {
    const int lane = threadIdx.x & 63;
    const int q = threadIdx.x >> 6;
    const int w = T.w;
    constexpr int wp = 16 * NRT;
    const int li = lane & 15, lk = lane >> 4;
    constexpr int ldus = wp + 1;
    double *Us = lds;                       // U^T, wp x wp (zero padded), leading dimension ldus
    double *Cs = lds + (size_t)wp * ldus;   // side 0: the strip's slice
    neig_d4 acc[NRT];
#pragma unroll
    for (int r = 0; r < NRT; ++r) acc[r] = (neig_d4){0.0, 0.0, 0.0, 0.0};

    if (T.side == 0) {
        const int c0 = tile * UPD_SLICE;
        constexpr int ldcs = wp + 1;
        for (int idx = threadIdx.x; idx < wp * UPD_SLICE; idx += UPD_THREADS) {
            const int r = idx % wp, c = idx / wp;
            double v = 0.0;
            if (r < w && c0 + c < T.len) v = AT(T.C, T.ldc, r, c0 + c);
            Cs[r + c * ldcs] = v;
        }
        for (int idx = threadIdx.x; idx < wp * wp; idx += UPD_THREADS) {
            const int r = idx % wp, k = idx / wp;
            Us[r + k * ldus] = (r < w && k < w) ? AT(T.Ut, T.ldu, r, k) : 0.0;
        }
        __syncthreads();
        const int cb = 16 * q + li;
#pragma unroll 4
        for (int k = 0; k < wp; k += 4) {
            const int kk = k + lk;
            const double b = Cs[kk + cb * ldcs];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) acc[rt] = mfma16(Us[(16 * rt + li) + kk * ldus], b, acc[rt]);
        }
        const int col = c0 + 16 * q + li;
        if (col < T.len) {
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * rt + lk + 4 * r;
                    if (row < w) AT(T.C, T.ldc, row, col) = acc[rt][r];
                }
            }
        }
    } else {
        // the wave's 16 rows of the strip, every k at once (all loads in flight
        // together), then U^T from LDS
        const int rbase = tile * UPD_SLICE + 16 * q;
        const int arow = rbase + li;
        double areg[4 * NRT];
#pragma unroll
        for (int s4 = 0; s4 < 4 * NRT; ++s4) {
            const int kk = 4 * s4 + lk;
            areg[s4] = (arow < T.len && kk < w) ? AT(T.C, T.ldc, arow, kk) : 0.0;
        }
        for (int idx = threadIdx.x; idx < wp * wp; idx += UPD_THREADS) {
            const int r = idx % wp, k = idx / wp;
            Us[r + k * ldus] = (r < w && k < w) ? AT(T.Ut, T.ldu, r, k) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < 4 * NRT; ++s4) {
            const int kk = 4 * s4 + lk;
#pragma unroll
            for (int ct = 0; ct < NRT; ++ct) acc[ct] = mfma16(areg[s4], Us[(16 * ct + li) + kk * ldus], acc[ct]);
        }
#pragma unroll
        for (int ct = 0; ct < NRT; ++ct) {
            const int col = 16 * ct + li;
            if (col < w) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rbase + lk + 4 * r;
                    if (row < T.len) AT(T.C, T.ldc, row, col) = acc[ct][r];
                }
            }
        }
    }
}

extern "C" __global__ void __launch_bounds__(UPD_THREADS)
k_update(UpdArgs args) {
    extern __shared__ double lds[];
    int ti = 0;
    const int bid = blockIdx.x;
    while (ti + 1 < args.ntask && args.t[ti + 1].tile0 <= bid) ++ti;
    const UpdTask T = args.t[ti];
    const int tile = bid - T.tile0;
    switch ((T.w + 15) >> 4) {  // uniform per workgroup
        case 1: upd_body<1>(T, tile, lds); break;
        case 2: upd_body<2>(T, tile, lds); break;
        case 3: upd_body<3>(T, tile, lds); break;
        case 4: upd_body<4>(T, tile, lds); break;
        case 5: upd_body<5>(T, tile, lds); break;
        default: upd_body<6>(T, tile, lds); break;
    }
}

// ---------------------------------------------------------------- wide windows
//
// k_update_wide: the same update tasks for factors of order 97..384 (deflation
// windows solved recursively).  U^T no longer fits in LDS, so each workgroup
// stages only its slice of the strip there (all w rows x UPW_SLICE columns for
// side 0, UPW_SLICE rows x all w columns for side 1) and streams U^T from global
// memory (it stays in L2: every workgroup of the launch reads the same factor),
// one register-double-buffered 4-deep k-step ahead.  Wave q owns every fourth
// 16-wide tile along w; the slice is written back through LDS so that the
// global stores are contiguous.
#define UPW_THREADS 256
#define UPW_WMAX 384
#define UPW_SLICE 32

template <int NRT>
__device__ __forceinline__ void upw_body(const UpdTask &T, int tile, double *lds) {
    constexpr int wp = 16 * NRT;  // padded order, a multiple of 64
    constexpr int NT4 = NRT / 4;  // tiles along w per wave
    const int lane = threadIdx.x & 63;
    const int q = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int w = T.w;
    neig_d4 acc[NT4][2];
#pragma unroll
    for (int i = 0; i < NT4; ++i) {
        acc[i][0] = (neig_d4){0.0, 0.0, 0.0, 0.0};
        acc[i][1] = (neig_d4){0.0, 0.0, 0.0, 0.0};
    }
    if (T.side == 0) {
        // slice: rows 0..wp-1 (zero padded) x columns c0..c0+31, leading dimension ldcs
        constexpr int ldcs = wp + 1;
        double *Cs = lds;
        const int c0 = tile * UPW_SLICE;
        for (int idx = threadIdx.x; idx < wp * UPW_SLICE; idx += UPW_THREADS) {
            const int r = idx % wp, c = idx / wp;
            Cs[r + c * ldcs] = (r < w && c0 + c < T.len) ? AT(T.C, T.ldc, r, c0 + c) : 0.0;
        }
        __syncthreads();
        double a0[NT4], a1[NT4];
#pragma unroll
        for (int i = 0; i < NT4; ++i) {
            const int r = 16 * (q + 4 * i) + li;
            a0[i] = (r < w && lk < w) ? AT(T.Ut, T.ldu, r, lk) : 0.0;
        }
        for (int k = 0; k < wp; k += 8) {
            // a0 holds k-step k; load k + 4 into a1 while multiplying
#pragma unroll
            for (int i = 0; i < NT4; ++i) {
                const int r = 16 * (q + 4 * i) + li, kk = k + 4 + lk;
                a1[i] = (r < w && kk < w) ? AT(T.Ut, T.ldu, r, kk) : 0.0;
            }
            {
                const double b0 = Cs[(k + lk) + li * ldcs], b1 = Cs[(k + lk) + (16 + li) * ldcs];
#pragma unroll
                for (int i = 0; i < NT4; ++i) {
                    acc[i][0] = mfma16(a0[i], b0, acc[i][0]);
                    acc[i][1] = mfma16(a0[i], b1, acc[i][1]);
                }
            }
#pragma unroll
            for (int i = 0; i < NT4; ++i) {
                const int r = 16 * (q + 4 * i) + li, kk = k + 8 + lk;
                a0[i] = (r < w && kk < w) ? AT(T.Ut, T.ldu, r, kk) : 0.0;
            }
            {
                const double b0 = Cs[(k + 4 + lk) + li * ldcs], b1 = Cs[(k + 4 + lk) + (16 + li) * ldcs];
#pragma unroll
                for (int i = 0; i < NT4; ++i) {
                    acc[i][0] = mfma16(a1[i], b0, acc[i][0]);
                    acc[i][1] = mfma16(a1[i], b1, acc[i][1]);
                }
            }
        }
        __syncthreads();  // every wave is done reading the slice
#pragma unroll
        for (int i = 0; i < NT4; ++i)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int r = 0; r < 4; ++r) Cs[(16 * (q + 4 * i) + lk + 4 * r) + (16 * ct + li) * ldcs] = acc[i][ct][r];
        __syncthreads();
        for (int idx = threadIdx.x; idx < wp * UPW_SLICE; idx += UPW_THREADS) {
            const int r = idx % wp, c = idx / wp;
            if (r < w && c0 + c < T.len) AT(T.C, T.ldc, r, c0 + c) = Cs[r + c * ldcs];
        }
    } else {
        // slice: rows r0..r0+31 x columns 0..wp-1 (zero padded), leading dimension 33
        constexpr int ldcs = UPW_SLICE + 1;
        double *Cs = lds;
        const int r0 = tile * UPW_SLICE;
        for (int idx = threadIdx.x; idx < wp * UPW_SLICE; idx += UPW_THREADS) {
            const int i = idx % UPW_SLICE, k = idx / UPW_SLICE;
            Cs[i + k * ldcs] = (k < w && r0 + i < T.len) ? AT(T.C, T.ldc, r0 + i, k) : 0.0;
        }
        __syncthreads();
        // B operand: U(kk, col) = U^T(col, kk)
        double b0[NT4], b1[NT4];
#pragma unroll
        for (int i = 0; i < NT4; ++i) {
            const int c = 16 * (q + 4 * i) + li;
            b0[i] = (c < w && lk < w) ? AT(T.Ut, T.ldu, c, lk) : 0.0;
        }
        for (int k = 0; k < wp; k += 8) {
#pragma unroll
            for (int i = 0; i < NT4; ++i) {
                const int c = 16 * (q + 4 * i) + li, kk = k + 4 + lk;
                b1[i] = (c < w && kk < w) ? AT(T.Ut, T.ldu, c, kk) : 0.0;
            }
            {
                const double x0 = Cs[li + (k + lk) * ldcs], x1 = Cs[(16 + li) + (k + lk) * ldcs];
#pragma unroll
                for (int i = 0; i < NT4; ++i) {
                    acc[i][0] = mfma16(x0, b0[i], acc[i][0]);
                    acc[i][1] = mfma16(x1, b0[i], acc[i][1]);
                }
            }
#pragma unroll
            for (int i = 0; i < NT4; ++i) {
                const int c = 16 * (q + 4 * i) + li, kk = k + 8 + lk;
                b0[i] = (c < w && kk < w) ? AT(T.Ut, T.ldu, c, kk) : 0.0;
            }
            {
                const double x0 = Cs[li + (k + 4 + lk) * ldcs], x1 = Cs[(16 + li) + (k + 4 + lk) * ldcs];
#pragma unroll
                for (int i = 0; i < NT4; ++i) {
                    acc[i][0] = mfma16(x0, b1[i], acc[i][0]);
                    acc[i][1] = mfma16(x1, b1[i], acc[i][1]);
                }
            }
        }
        __syncthreads();
        // acc[i][it] lane l: D(lk + 4 r, li) = rows 16 it + lk + 4 r, column 16 (q + 4 i) + li
#pragma unroll
        for (int i = 0; i < NT4; ++i)
#pragma unroll
            for (int it = 0; it < 2; ++it)
#pragma unroll
                for (int r = 0; r < 4; ++r) Cs[(16 * it + lk + 4 * r) + (16 * (q + 4 * i) + li) * ldcs] = acc[i][it][r];
        __syncthreads();
        for (int idx = threadIdx.x; idx < wp * UPW_SLICE; idx += UPW_THREADS) {
            const int i = idx % UPW_SLICE, k = idx / UPW_SLICE;
            if (k < w && r0 + i < T.len) AT(T.C, T.ldc, r0 + i, k) = Cs[i + k * ldcs];
        }
    }
}

extern "C" __global__ void __launch_bounds__(UPW_THREADS) k_update_wide(UpdArgs args) {
    extern __shared__ double lds[];
    int ti = 0;
    const int bid = blockIdx.x;
    while (ti + 1 < args.ntask && args.t[ti + 1].tile0 <= bid) ++ti;
    const UpdTask T = args.t[ti];
    const int tile = bid - T.tile0;
    switch ((T.w + 63) >> 6) {  // uniform per workgroup
        case 2: upw_body<8>(T, tile, lds); break;
        case 3: upw_body<12>(T, tile, lds); break;
        case 4: upw_body<16>(T, tile, lds); break;
        case 5: upw_body<20>(T, tile, lds); break;
        default: upw_body<24>(T, tile, lds); break;
    }
}
