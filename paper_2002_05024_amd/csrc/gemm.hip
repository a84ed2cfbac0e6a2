// gemm.hip -- the left / right update tasks (Section 3.2): apply a window's
// accumulated orthogonal factor U (w x w, w <= 128, given as U^T) to an
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
#define UPD_WMAX 128
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
        case 6: upd_body<6>(T, tile, lds); break;
        case 7: upd_body<7>(T, tile, lds); break;
        default: upd_body<8>(T, tile, lds); break;
    }
}
