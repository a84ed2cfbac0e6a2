/*
 * neig.h -- C ABI of libneig: Schur reduction of a real upper Hessenberg matrix
 * on one AMD MI355X (gfx950) GPU.
 *
 * The operation (Section 2, eq. 4 of Myllykoski & Kjelgaard Mikkelsen,
 * "Task-based, GPU-accelerated and robust library for solving dense
 * nonsymmetric eigenvalue problems"): given a real upper Hessenberg H, find an
 * orthogonal Q and an upper quasi-triangular S with 1x1 and 2x2 diagonal blocks
 * such that H = Q S Q^T.  The method is the small-bulge multishift QR algorithm
 * with aggressive early deflation (Section 3.2): AED steps on a trailing window
 * alternate with sweeps that chase chains of 3x3 bulges down the diagonal,
 * window by window, with each window's reflectors accumulated into a small
 * orthogonal matrix that is applied to the off-diagonal parts of H and Z with
 * matrix-matrix products (Section 3.2, the window / left-update / right-update
 * tasks).
 *
 * Conventions for every entry point:
 *   - matrices are FP64, column-major, element (i, j) at p[i + j*ld], ld >= max(1, n);
 *   - pointers marked "device" are GPU memory owned by the caller; the library
 *     never frees or retains them past the call;
 *   - the library owns a per-device workspace it allocates on first use and
 *     frees in neig_finalize();
 *   - return values: 0 success; -k argument k (1-based) invalid; a value
 *     <= -100 is a HIP runtime error (-100 - hipError_t); > 0 as documented per
 *     call.  No C++ exception crosses this interface;
 *   - calls are not thread-safe with respect to each other (one call in flight
 *     per process).
 */
#ifndef NEIG_H
#define NEIG_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Tunables.  A zero field means "library default" (chosen per size). */
typedef struct neig_params {
    int ns;        /* shifts per multishift sweep (even)                                */
    int nw;        /* aggressive-early-deflation window size                             */
    int nmin;      /* active blocks of at most nmin rows go to the in-LDS double-shift QR */
    int chain;     /* bulges per chain (one chase workgroup per chain)                   */
    int chase_w;   /* rows/cols of one chase window held in LDS                          */
    int deflation; /* 0: window criterion |spike| <= eps*|lambda| (LAPACK-style);
                      1: norm-stable criterion |spike| <= eps*||H||_F (Section 5)        */
    int maxit;     /* iteration limit (AED+sweep rounds); 0: 30*max(10, n)               */
    int nibble;    /* percent: an AED that deflates at least this share of its window is
                      followed by another AED instead of a sweep                         */
    int exc;       /* rounds without deflation before exceptional shifts                 */
    int timing;    /* 1: bracket every kernel launch with HIP events on the call's stream and
                      report per-kernel-class GPU time in neig_stats (adds host overhead) */
    int reserved[6];
} neig_params;

/* Counters and timings of the most recent neig_schur call. */
typedef struct neig_stats {
    long long sweeps, aeds, aed_deflated, shifts_used, exceptional, small_solves, swap_failures, iterations;
    double gemm_flops;   /* executed FP64 flops in the off-diagonal update kernels: sum of 2 w^2 len */
    double chase_flops;  /* flops of the reflector applications inside windows                    */
    double small_flops;  /* flops inside the in-LDS QR / AED kernels (estimate)                   */
    double t_total_ms, t_aed_ms, t_sweep_ms, t_small_ms;  /* host wall time per phase           */
    double alg_flops;    /* algorithmic flops of the method: 20 n per bulge position per sweep,
                            10 nw^3 + 2 nw^2 (rows above + columns right + n) per AED / small block */
    /* with timing = 1: GPU time (event intervals) and launch counts per kernel class */
    double gpu_update_ms, gpu_chase_ms, gpu_aed_ms, gpu_small_ms, gpu_other_ms;
    double n_update, n_chase;
    /* inside the AED kernel: window-QR iterations, block swaps, and shader clock
       cycles of its three phases (window QR; spike test and swaps; re-Hessenberg) */
    double aed_qr_iters, aed_swaps, aed_cyc_qr, aed_cyc_defl, aed_cyc_hess;
    double aed_late;     /* deflations found above a block that failed the spike test */
} neig_stats;

/*
 * neig_schur -- real Schur form in place (Section 2, eq. 4; method Section 3.2).
 *   n        order of H (n >= 0).
 *   H, ldh   device; on entry upper Hessenberg (entries below the first
 *            subdiagonal are ignored and set to zero); on exit S, the
 *            standardised real Schur form: exact zeros below the subdiagonal,
 *            1x1 blocks, and 2x2 blocks with equal diagonal entries and
 *            off-diagonal entries of opposite sign (complex pairs only).
 *   Z, ldz   device; on entry an orthogonal matrix (the identity for the
 *            Schur vectors of H, or Q1 from a Hessenberg reduction A = Q1 H Q1^T
 *            (eq. 3) for those of A); on exit Z_in * Q.
 *   wr, wi   device, n doubles each: eigenvalues in the diagonal order of S;
 *            a complex pair at (i, i+1) has wi[i] > 0, wi[i+1] = -wi[i].
 *   stream   HIP stream the work is ordered on; the call returns after it is done.
 * Returns 0; -2 also when H holds a NaN or Inf; > 0 the number of eigenvalues
 * (leading rows/cols 0..info-1) not converged within the iteration limit: H and
 * Z still satisfy H_in = Z S Z^T, so calling again with (S, Z) resumes.
 */
int neig_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi, hipStream_t stream);

/*
 * neig_schur_batched -- neig_schur on `batch` independent problems of uneven
 * order in one call.
 *   n, ldh, ldz  host arrays [batch].
 *   H, Z, wr, wi device arrays [batch] of device pointers (one per problem).
 *   info         device int[batch]: per-problem return value as for neig_schur.
 * Returns 0 or a negative argument / HIP error code for the call as a whole.
 */
int neig_schur_batched(int batch, const int *n, double *const *H, const int *ldh, double *const *Z, const int *ldz,
                       double *const *wr, double *const *wi, int *info, hipStream_t stream);

/*
 * neig_sweep -- one multishift QR sweep (Section 3.2, "Bulge chasing step"):
 * nshifts/2 bulges, each made from the first column of (H - s1 I)(H - s2 I),
 * chased through rows/cols ktop..kbot in chains of overlapping windows, with
 * H (all columns right of and rows above each window) and Z updated.
 *   ktop, kbot   0-based active block; H(ktop, ktop-1) and H(kbot+1, kbot) are
 *                treated as zero.  kbot - ktop >= 2.
 *   nshifts      even, >= 2; shifts sr/si are host arrays with complex
 *                conjugate pairs adjacent (sr equal, si of opposite sign).
 * Returns 0 or a negative code.
 */
int neig_sweep(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nshifts, const double *sr,
               const double *si, hipStream_t stream);

/*
 * neig_aed -- one aggressive early deflation step (Section 3.2, "AED step") on
 * the trailing window rows/cols kbot-nw+1..kbot of the active block ktop..kbot:
 * Schur form of the window, spike test of every diagonal block from the bottom
 * up, failing blocks moved to the top of the window, the remaining spike
 * reduced by a Householder Hessenberg reduction, and the window's orthogonal
 * factor applied to the rest of H and to Z.
 *   nd           host out: number of deflated eigenvalues (rows kbot-nd+1..kbot
 *                are now decoupled and in Schur form).
 *   nshift       host out: number of undeflated Ritz values written to sr/si
 *                (host arrays of at least nw doubles), bottom-most last.
 * Returns 0 or a negative code.
 */
int neig_aed(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nw, int *nd, int *nshift,
             double *sr, double *si, hipStream_t stream);

/*
 * neig_small_schur -- real Schur form of a matrix small enough to live in one
 * workgroup's LDS (n <= the limit neig_get_params reports in nmin's place when
 * nmin is 0), by the double-shift QR iteration (the two-shift case of
 * Section 3.2).  Arguments and results as for neig_schur.  Returns -1 when n
 * exceeds the LDS limit.
 */
int neig_small_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi, hipStream_t stream);

/* Set / read the tunables (process-wide).  neig_set_params returns -k when field k
 * is out of range. */
int neig_set_params(const neig_params *p);
int neig_get_params(neig_params *p);

/* Counters of the most recent neig_schur call. */
int neig_get_stats(neig_stats *s);

/* Free the per-device workspace. */
void neig_finalize(void);

/* Version / build string. */
const char *neig_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NEIG_H */
