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

// ---------------------------------------------------------------- persistent update kernel
//
// k_update_p<NRT>: the update tasks for factors of order w <= 16 NRT <= 96 with
// the factor held in registers.  The launch has a few workgroups per compute
// unit; each loops over 64-wide slices of the tasks' strips (64 columns for
// side 0, 64 rows for side 1).  Workgroup: NRT waves.  Wave q owns the 16-wide
// tile q along w and all four 16-wide tiles across the slice; the part of the
// factor it multiplies with (rows 16q.. of U^T for side 0, columns 16q.. of U
// for side 1, all 4 NRT k-steps) is loaded into registers once per task.  Per
// slice: the slice goes from registers into LDS, the next slice's elements
// (16 per thread) are requested from HBM, the waves multiply from LDS while
// they are in flight, and the results go from the accumulators straight to
// HBM.  With one LDS buffer per workgroup several workgroups share a compute
// unit, so one's barriers and loads overlap another's matrix-core work.
#define UPDP_PER 16  // slice elements per thread
#define UPDP_OOB 0x7ffffff8  // a buffer offset past every slice's range: loads give 0, stores are dropped

typedef unsigned int updp_u2 __attribute__((ext_vector_type(2)));

// Buffer resource over one slice of a strip (raw addressing, range-checked in
// bytes): out-of-range elements of partial slices load as zero and their
// stores are discarded, with no branches.  dword3 is the gfx9 family's
// buffer format word.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t updp_rsrc(const UpdTask &T, int s, int *nvalid) {
    const int base = s * UPD_SLICE;
    const int nv = min(UPD_SLICE, T.len - base);  // columns (side 0) or rows (side 1) of the slice
    *nvalid = nv;
    double *p;
    int bytes;
    if (T.side == 0) {
        p = T.C + (size_t)base * T.ldc;
        bytes = ((nv - 1) * T.ldc + T.w) * 8;
    } else {
        p = T.C + base;
        bytes = ((T.w - 1) * T.ldc + nv) * 8;
    }
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, bytes, 0x00020000);
}

template <int NRT>
__device__ __forceinline__ void updp_load(const UpdTask &T, int s, double (&pre)[UPDP_PER]) {
    constexpr int wp = 16 * NRT;
    int nv;
    const __amdgpu_buffer_rsrc_t rs = updp_rsrc(T, s, &nv);
    const int tid = threadIdx.x;
    if (T.side == 0) {  // element e: row tid % wp, column tid / wp + 4 e (64 NRT threads = 4 wp)
        const int r = tid % wp, c = tid / wp;
#pragma unroll
        for (int e = 0; e < UPDP_PER; ++e) {
            const int off = (r < T.w && c + 4 * e < nv) ? (r + (c + 4 * e) * T.ldc) * 8 : UPDP_OOB;
            pre[e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        }
    } else {  // element e: row tid % 64, column tid / 64 + NRT e
        const int r = tid & 63, c = tid >> 6;
#pragma unroll
        for (int e = 0; e < UPDP_PER; ++e) {
            const int off = (r < nv && c + NRT * e < T.w) ? (r + (c + NRT * e) * T.ldc) * 8 : UPDP_OOB;
            pre[e] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        }
    }
}

template <int NRT>
__device__ __forceinline__ void updp_stage(int side, const double (&pre)[UPDP_PER], double *buf) {
    constexpr int wp = 16 * NRT;
    const int tid = threadIdx.x;
    if (side == 0) {
        const int r = tid % wp, c = tid / wp;
#pragma unroll
        for (int e = 0; e < UPDP_PER; ++e) buf[r + (c + 4 * e) * (wp + 1)] = pre[e];
    } else {
        const int r = tid & 63, c = tid >> 6;
#pragma unroll
        for (int e = 0; e < UPDP_PER; ++e) buf[r + (c + NRT * e) * (UPD_SLICE + 1)] = pre[e];
    }
}

template <int NRT>
__global__ void __launch_bounds__(64 * NRT) __attribute__((amdgpu_waves_per_eu(3))) k_update_p(UpdArgs args,
                                                                                               int nslice) {
    extern __shared__ double lds[];
    constexpr int wp = 16 * NRT;
    constexpr int NK = 4 * NRT;  // k-steps of 4
    const int lane = threadIdx.x & 63;
    const int q = threadIdx.x >> 6;  // tile along w
    const int li = lane & 15, lk = lane >> 4;
    int s = blockIdx.x;
    if (s >= nslice) return;
    int ti = 0;
    while (ti + 1 < args.ntask && args.t[ti + 1].tile0 <= s) ++ti;
    UpdTask T = args.t[ti];
    double frag[NK];
    auto load_frag = [&]() {
        const int rw = 16 * q + li;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int kk = 4 * k + lk;
            frag[k] = (rw < T.w && kk < T.w) ? AT(T.Ut, T.ldu, rw, kk) : 0.0;
        }
        // complete these loads here, so that the slice loads issued later are
        // never waited for by the products that use the factor
        __builtin_amdgcn_s_waitcnt(0);
    };
    load_frag();
    double pre[UPDP_PER];
    updp_load<NRT>(T, s - T.tile0, pre);
    for (;;) {
        __syncthreads();  // every wave is done reading the buffer
        updp_stage<NRT>(T.side, pre, lds);
        __syncthreads();
        const int sn = s + (int)gridDim.x;
        const bool more = sn < nslice;
        int tn = ti;
        if (more) {
            while (tn + 1 < args.ntask && args.t[tn + 1].tile0 <= sn) ++tn;
            updp_load<NRT>(args.t[tn], sn - args.t[tn].tile0, pre);
        }
        neig_d4 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = (neig_d4){0.0, 0.0, 0.0, 0.0};
        int nv;
        const __amdgpu_buffer_rsrc_t rs = updp_rsrc(T, s - T.tile0, &nv);
        if (T.side == 0) {
            constexpr int ldb = wp + 1;
            const double *bp = lds + li * ldb + lk;
            // one k-step's operands read ahead of its products; the scheduling
            // barriers keep the compiler from hoisting every LDS read up front
            double b[4], bn[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = bp[16 * j * ldb];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                if (k + 1 < NK) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) bn[j] = bp[16 * j * ldb + 4 * (k + 1)];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] = mfma16(frag[k], b[j], acc[j]);
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = bn[j];
                __builtin_amdgcn_sched_barrier(0);
            }
            const int row0 = 16 * q + lk;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row0 + 4 * r, col = 16 * j + li;
                    const int off = (row < T.w && col < nv) ? (row + col * T.ldc) * 8 : UPDP_OOB;
                    const double v = acc[j][r];  // a scalar first: a vector element is not an object to bit-cast
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(updp_u2, v), rs, off, 0, 0);
                }
        } else {
            constexpr int lda = UPD_SLICE + 1;
            const double *ap = lds + li + lk * lda;
            double a[4], an[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = ap[16 * j];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                if (k + 1 < NK) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) an[j] = ap[16 * j + 4 * (k + 1) * lda];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] = mfma16(a[j], frag[k], acc[j]);
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = an[j];
                __builtin_amdgcn_sched_barrier(0);
            }
            const int col = 16 * q + li;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * j + lk + 4 * r;
                    const int off = (col < T.w && row < nv) ? (row + col * T.ldc) * 8 : UPDP_OOB;
                    const double v = acc[j][r];  // a scalar first: a vector element is not an object to bit-cast
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(updp_u2, v), rs, off, 0, 0);
                }
        }
        if (!more) break;
        if (tn != ti) {
            ti = tn;
            T = args.t[ti];
            load_frag();
        }
        s = sn;
    }
}
