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
 * tasks).  Around it: many independent problems in one launch
 * (neig_schur_batched), the Hessenberg reduction that precedes it
 * (neig_hessenberg, Section 3.1), eigenvalue reordering of the result
 * (neig_reorder), and a small network that proposes the shift count and AED
 * window (neig_policy_*, neig_mlp_*).
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
    int policy;    /* shift count and deflation window per iteration:
                      0: the default size rules;
                      1: the proposal network installed by neig_policy_set, falling back to
                         the default rules when it is not confident;
                      2: exploration: uniformly random bins (seeded by `seed`), every
                         decision logged for neig_policy_log;
                      3: fixed bins for the whole call, shift bin seed mod 8 and window
                         bin (seed / 8) mod 8, every decision logged (per-run
                         exploration);
                      4: per-matrix proposal: the network's bins at the first decision
                         hold for the whole call (the default rules when no network is
                         installed or it is not confident); that decision is logged   */
    int seed;      /* seed of the exploration generator                                  */
    int rec_nw;    /* deflation window used inside a recursively solved AED window
                      (nw > 96; at most 96); 0: the default rule for the window's order */
    int rec_ns;    /* shifts per sweep inside a recursively solved AED window            */
    int aed_ends;  /* 0: aggressive early deflation on the trailing window and, while the
                      active block is large and that end keeps deflating, on the leading
                      window too (the same step on the flipped block J B^T J, which is
                      upper Hessenberg again), both in one launch on two compute units;
                      1: the trailing window only                                        */
    int overlap;   /* sweeps: the updates of each chase step are split into the entries the
                      next step's windows cover, applied on the call's stream, and the
                      rest, applied on a second stream beside the next chase launch
                      (Section 3.2: updates run concurrently with the chase);
                      0: for orders of at least 8192; 1: always; 2: never               */
} neig_params;

/* Largest AED window.  Windows of at most 96 rows are solved in one workgroup's
 * LDS; larger ones (Section 3.2: the window's Schur form by a recursive
 * application of the QR algorithm) by the whole method run on the window. */
#define NEIG_AED_MAX 384

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
    double policy_used, policy_fallback;  /* proposals taken from the network / the default rules */
    double aed_flops;    /* algorithmic flops of the LDS AED kernel's windows: 10 nw^3 per launch,
                            including the launches inside recursive window solves          */
    /* AED windows of more than 96 rows: how many, the AED steps and sweeps of the
       recursive solves of those windows (not counted in aeds / sweeps above), and
       the GPU time (timing = 1) of their deflation kernel */
    double rec_aeds, rec_inner_aeds, rec_inner_sweeps, gpu_rec_defl_ms;
    double chase_bytes;  /* algorithmic bytes of the chase windows: 8 (2 mb^2 + w^2) per window
                            (its block of H loaded and stored, its factor stored)            */
    double aeds_top, aed_top_deflated;  /* leading-window AED steps (counted in aeds too) and
                                           the eigenvalues they deflated                    */
    double aed_launches;  /* launches of the LDS AED kernel (one or two windows each)      */
    /* the far parts of overlapped sweep steps (parameter overlap; counted in the
       update totals above too): GPU time (timing = 1), launches, executed flops */
    double gpu_update_far_ms, n_update_far, gemm_flops_far;
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

/* Largest batch one neig_schur_batched call takes. */
#define NEIG_BATCH_MAX 65536

/*
 * neig_schur_batched -- neig_schur on `batch` independent problems of uneven
 * order in one persistent launch (the method of Section 3.2 run per problem by
 * one workgroup that keeps its window factors in LDS; problems are taken from a
 * device work queue, largest first).
 *   batch        0 <= batch <= NEIG_BATCH_MAX.
 *   n, ldh, ldz  device int arrays [batch]: order and leading dimensions.
 *   H, Z, wr, wi device arrays [batch] of device pointers, one per problem, with
 *                the meaning, layout and results of neig_schur's arguments.
 *   info         device int[batch]: per-problem result as neig_schur returns it
 *                (0; -2 also for NaN/Inf in H; -2..-8 for an invalid n, H, ldh,
 *                Z, ldz, wr or wi entry of that problem, which is then left
 *                untouched; > 0 unconverged leading rows).
 *   stream       the work is ordered on this stream; the call returns after
 *                enqueueing it (asynchronous: results are ready once the
 *                stream reaches that point).
 * Every array is read on the device when the work runs, so the call can be
 * captured in a HIP graph and replayed with new contents in the same arrays.
 * All batched calls on a device share one fixed-size library descriptor table:
 * calls (and graph replays) must not overlap in time, e.g. keep them on one
 * stream.  Per-size-class tuning comes from neig_set_batched_tune; the
 * deflation criterion, nibble and exceptional-shift settings from neig_params.
 * Returns 0 or a negative code for the call as a whole (-1 batch out of range).
 */
int neig_schur_batched(int batch, const int *n, double *const *H, const int *ldh, double *const *Z, const int *ldz,
                       double *const *wr, double *const *wi, int *info, hipStream_t stream);

/*
 * neig_batched_flops -- the method's own floating-point operation count for
 * the last neig_schur_batched call on the current device, counted on the
 * device by the batched kernel (Section 3.2's steps: 10 m^3 per AED window or
 * small block brought to Schur form in LDS, 2 m^2 for every row or column of H
 * and Z its orthogonal factor is applied to, 20 n per bulge position of a
 * sweep; the same formulas as neig_stats.alg_flops of the single-matrix path).
 * The count is reset by each call's first kernel, so a graph replay counts
 * its own work.  Waits for the device to finish, then copies the count to
 * *flops (host).  neig_schur_batched_noalloc keeps its own count in its fixed
 * array; this call does not read it.  Returns 0, -1 for a null pointer, or
 * <= -100 for a HIP error (-100 - hipError_t).
 */
int neig_batched_flops(double *flops);

/* Largest batch one neig_schur_batched_noalloc call takes. */
#define NEIG_BATCH_NOALLOC_MAX 4096

/*
 * neig_schur_batched_noalloc -- neig_schur_batched for callers that cannot
 * allocate memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  Same arguments, results, asynchrony and
 * error codes as neig_schur_batched, with the same kernels; it calls no
 * hipMalloc, hipFree or other allocating routine.  Its only scratch (the
 * problem descriptors, the processing order and the work counter, about
 * 213 KB) is a fixed array in device memory that each GPU the library runs on
 * holds until the process ends; its device address is looked up once per
 * device on the first call there.
 *   batch   0 <= batch <= NEIG_BATCH_NOALLOC_MAX; -1 beyond it (nothing runs).
 * Every call on one GPU uses that GPU's one array: calls (and graph replays)
 * that overlap in time on the same GPU race and give undefined results; keep
 * them on one stream.  The array keeps the last call's contents; everything a
 * call reads from it is rewritten by that call's first kernel.
 * Returns 0, a negative code as neig_schur_batched, or <= -100 for a HIP error
 * (also when the array's address cannot be obtained).
 */
int neig_schur_batched_noalloc(int batch, const int *n, double *const *H, const int *ldh, double *const *Z,
                               const int *ldz, double *const *wr, double *const *wi, int *info,
                               hipStream_t stream);

/* Size classes of the batched solver. */
#define NEIG_BATCH_CLASSES 6

/*
 * neig_set_batched_tune -- per-size-class control parameters of
 * neig_schur_batched (Section 3.2: AED window, shifts per sweep, the size below
 * which a block is solved by the in-LDS double-shift QR, and the chase window).
 * A problem of order m uses the first class k with m <= n_hi[k]; the last class
 * takes every larger m (its n_hi is ignored).
 *   nclass          1..NEIG_BATCH_CLASSES.
 *   n_hi            host int[nclass], strictly increasing.
 *   nw, ns, nmin,   host int[nclass]: 2 <= nw, nmin <= 96; ns even, 2..32;
 *   chase_w         3*(ns/2)+2 <= chase_w <= 96.
 * Returns 0 or -k for the first invalid argument k; the table is unchanged on error.
 */
int neig_set_batched_tune(int nclass, const int *n_hi, const int *nw, const int *ns, const int *nmin,
                          const int *chase_w);

/*
 * neig_get_batched_tune -- the current per-size-class table.  *nclass receives
 * NEIG_BATCH_CLASSES; the other host arrays need that many entries.
 */
int neig_get_batched_tune(int *nclass, int *n_hi, int *nw, int *ns, int *nmin, int *chase_w);

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
 * factor applied to the rest of H and to Z.  Windows of at most 96 rows are
 * solved in one workgroup's LDS; 97..NEIG_AED_MAX rows by the whole method run
 * recursively on the window.
 *   nd           host out: number of deflated eigenvalues (rows kbot-nd+1..kbot
 *                are now decoupled and in Schur form).
 *   nshift       host out: number of undeflated Ritz values written to sr/si
 *                (host arrays of at least nw doubles), bottom-most last.
 * Returns 0 or a negative code.
 */
int neig_aed(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nw, int *nd, int *nshift,
             double *sr, double *si, hipStream_t stream);

/*
 * neig_aed_top -- the same deflation step on the leading window of the active
 * block: rows/cols ktop..ktop+nw-1, coupled to the rest of the block by
 * H(ktop+nw, ktop+nw-1).  It is the AED step (Section 3.2) of the flipped
 * block J B^T J (B = H(ktop:kbot, ktop:kbot), J the reversal), which is upper
 * Hessenberg with the window at its bottom; mapped back, the deflated
 * eigenvalues end in a leading quasi-triangular block rows/cols
 * ktop..ktop+nd-1 with H(ktop+nd, ktop+nd-1) = 0.  neig_schur runs it beside
 * the trailing-window step while the active block is large (neig_params
 * aed_ends).  Arguments, updates of H and Z, results and error codes as
 * neig_aed; nw <= 96.  The Ritz values returned are those of the leading
 * window's undeflated part.
 */
int neig_aed_top(int n, double *H, int ldh, double *Z, int ldz, int ktop, int kbot, int nw, int *nd, int *nshift,
                 double *sr, double *si, hipStream_t stream);

/*
 * neig_small_schur -- real Schur form of a matrix small enough to live in one
 * workgroup's LDS (n <= the limit neig_get_params reports in nmin's place when
 * nmin is 0), by the double-shift QR iteration (the two-shift case of
 * Section 3.2).  Arguments and results as for neig_schur.  Returns -1 when n
 * exceeds the LDS limit.
 */
int neig_small_schur(int n, double *H, int ldh, double *Z, int ldz, double *wr, double *wi, hipStream_t stream);

/*
 * neig_hessenberg -- reduction of a general matrix to upper Hessenberg form,
 * A = Q1 H Q1^T (Section 2, eq. 3; the step before the Schur reduction), by
 * the standard blocked Householder algorithm of Section 3.1: panels of 64
 * reflectors reduced with the trailing matrix-vector products on the GPU,
 * accumulated as I - V T V^T with Y = A V T, then the trailing-matrix and
 * top-part updates as FP64 matrix-core products.  Reflector convention:
 * P = I - tau v v^T, v(0) = 1, beta = -sign(alpha) ||x|| (sign(0) = +1),
 * tau = 0 when the tail below the subdiagonal is already zero.
 *   n            order (>= 0).
 *   A, lda       device, column-major; on entry the general matrix, on exit H
 *                with exact zeros below the first subdiagonal.
 *   Q, ldq       device, column-major, or NULL; on exit Q_in * Q1 (pass the
 *                identity for Q1 itself).  NULL skips the accumulation.
 * Workspace (about 4 * 64 * n doubles plus partials) is cached per device.
 * Synchronous.  Returns 0; -1 n < 0; -2 A null; -3 lda < max(1, n);
 * -5 ldq < max(1, n) with Q given; <= -100 HIP error.  Non-finite entries
 * propagate.
 */
int neig_hessenberg(int n, double *A, int lda, double *Q, int ldq, hipStream_t stream);

/*
 * neig_reorder -- eigenvalue reordering of a real Schur decomposition (the
 * phase the paper runs after the Schur reduction): an orthogonal Q such that
 * the selected eigenvalues occupy the leading diagonal block of Q^T S Q, in
 * their original order, by exchanges of adjacent diagonal blocks (the
 * Sylvester-equation construction of Bai and Demmel), organised in windows of
 * at most 96 rows, each moving a group of selected blocks; the windows of one
 * round do not overlap and run concurrently, and their factors are applied to
 * the rest of S and to Z with FP64 matrix-core products.
 *   S, lds   device; on entry a standardised real Schur form (as neig_schur
 *            returns it); on exit the reordered one.
 *   Z, ldz   device; on exit Z_in * Q.
 *   select   host int[n]; nonzero selects the eigenvalue at that diagonal
 *            position (either position of a 2x2 block selects the pair).
 *   wr, wi   device, n doubles each: eigenvalues of the reordered S.
 *   m        host out: number of selected eigenvalues now leading.
 * Synchronous.  Returns 0; 1 if an exchange was rejected by its stability test
 * (S, Z then hold a valid, partly reordered Schur decomposition and *m counts
 * the eigenvalues in place); -k for invalid argument k; <= -100 HIP error.
 */
int neig_reorder(int n, double *S, int lds, double *Z, int ldz, const int *select, double *wr, double *wi, int *m,
                 hipStream_t stream);

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

/*
 * Parameter-proposal network (not part of the paper's method: an addition that
 * chooses the method's two tunables of Section 3.2, the number of shifts of the
 * next sweep and the size of the next deflation window, per iteration).  A
 * 24-64-64-(8+8) perceptron with ReLU hidden layers; the two 8-way heads score
 * the bins neig_policy_bins reports.  Parameters are NEIG_MLP_NPARAM floats laid
 * out as mu[24], sd[24] (fixed input normalisation), W1[64][24], b1[64],
 * W2[64][64], b2[64], W3[16][64], b3[16] (row-major); the input is
 * (x - mu) / sd.
 *
 * Features of one decision (active block [ktop, kbot] of order m, after a
 * deflation window): f0 = log m; f1..f19 = the 5%, 10%, ..., 95% quantiles
 * (linear interpolation between order statistics) of log(|h(k,k-1)| /
 * (||H||_F / sqrt n)) over at most 1024 subdiagonal entries
 * k = ktop+1+floor(i (m-1) / S), i < S = min(m-1, 1024); f20 = log(1e-30 + mean
 * |ritz| / (||H||_F / sqrt n)), f21 = std |ritz| / mean |ritz|, f22 = share of
 * non-real Ritz values, over the undeflated Ritz values of the last window (all
 * three 0 when there are none); f23 = deflations of the last window / its size.
 */
#define NEIG_MLP_NPARAM 6848

/* Bins of the two heads: ns_bins[8] shift counts (8, 16, 24, 32, 48, 64, 96, 128),
 * nw_bins[8] window sizes (32, 40, 48, 56, 64, 72, 80, 96) (host out). */
int neig_policy_bins(int *ns_bins, int *nw_bins);

/*
 * neig_policy_set -- install the network used by params.policy = 1 (host array
 * of NEIG_MLP_NPARAM floats, copied), or remove it (theta NULL).  A proposal is
 * used only when the softmax probability of the chosen bin is at least min_conf
 * on both heads; otherwise the default rules decide.  Returns 0, -1 (nparam),
 * -3 (min_conf not in [0, 1]).
 */
int neig_policy_set(const float *theta, int nparam, float min_conf);

/*
 * neig_policy_log -- the decisions of the most recent neig_schur call with
 * policy 1, 2, 3 or 4.  For decision i < min(count, cap): feat[24 i ..] its features,
 * bins[2 i ..] the (shift, window) bins applied (or proposed, when the default
 * rules decided), stats[4 i ..] = deflations of the next window, milliseconds
 * from the decision to the end of that window, the order m of the active
 * block, and 1 if the bins were applied.  Host arrays.  Returns count (>= 0).
 */
int neig_policy_log(int cap, float *feat, int *bins, float *stats);

/*
 * neig_policy_features -- the features of the active block [ktop, kbot] of H
 * (device, order n, leading dimension ldh) as the solver computes them, with
 * hnorm = ||H||_F and extra[4] (host) = f20..f23, and the installed network's
 * bins and probabilities for them (all host out: feat[24], bins[2], conf[2]).
 * Synchronous.  Returns 0 or -k for invalid argument k.
 */
int neig_policy_features(int n, const double *H, int ldh, int ktop, int kbot, double hnorm, const float *extra,
                         float *feat, int *bins, float *conf, hipStream_t stream);

/*
 * neig_mlp_grad -- loss and gradient of the reward-weighted cross-entropy
 *   L = (1/B) sum_i w_i (-log softmax(z_i[0:8])[a_i] - log softmax(z_i[8:16])[c_i])
 * of a mini-batch, z_i the network's scores of X[i] (FP32 arithmetic).
 *   batch   B >= 1.
 *   X       device float[B][24]; a, c device int[B] in [0, 8); w device float[B].
 *   theta   device float[NEIG_MLP_NPARAM].
 *   grad    device float[NEIG_MLP_NPARAM] out (zero for mu and sd); loss device float out.
 * Asynchronous on `stream`.  Returns 0, -1 (batch), or a HIP error code.
 */
int neig_mlp_grad(int batch, const float *X, const int *a, const int *c, const float *w, const float *theta,
                  float *grad, float *loss, hipStream_t stream);

/*
 * neig_mlp_adam -- one Adam step (Kingma & Ba, bias-corrected) on the trainable
 * entries of theta (device), with moments m, v (device, NEIG_MLP_NPARAM floats,
 * zero before the first step); step >= 1 counts the steps.  Returns 0, -5 (step).
 */
int neig_mlp_adam(float *theta, const float *grad, float *m, float *v, int step, float lr, hipStream_t stream);

/*
 * neig_mlp_infer -- the network's scores with BF16 operands and FP32 sums:
 * weights and each layer's input rounded to BF16 (nearest even), biases FP32.
 *   X device float[B][24]; logits device float[B][16] out; bins device int[B][2]
 *   out (best shift bin, best window bin); conf device float[B][2] out (their
 *   softmax probabilities).  Asynchronous.  Returns 0, -1 (batch).
 */
int neig_mlp_infer(int batch, const float *X, const float *theta, float *logits, int *bins, float *conf,
                   hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* NEIG_H */
