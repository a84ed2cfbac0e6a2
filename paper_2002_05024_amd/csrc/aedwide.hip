// aedwide.hip -- aggressive early deflation on windows too large for one
// workgroup's LDS (Section 3.2, "AED step", whose window is brought to Schur
// form by a recursive application of the QR algorithm).
//
// The host copies the nw x nw window of H into a workspace matrix T (with
// V = I), brings (T, V) to real Schur form by running the whole method on that
// nw x nw problem (AED on its own trailing windows, multishift sweeps, the
// in-LDS QR for its small blocks), and then calls k_aed_wide: the spike test
// bottom-up with block swaps, the deflated 2x2 blocks put in standard form, the
// undeflated Ritz values, and the reduction of the spike and the undeflated
// part back to Hessenberg form -- the same device code the LDS kernel k_aed
// runs, here on T and V in global memory (the window stays in L2).  When
// something deflated, k_win_store writes T back into H and V^T into the
// workspace, and the host applies V to the rest of H and to Z with the update
// kernels.

// T (ldt) <- the nw x nw diagonal block of H at (off, off), zeros below the
// subdiagonal; V (ldv) <- I.
extern "C" __global__ void __launch_bounds__(256) k_win_load(const double *H, int ldh, int off, int nw, double *T,
                                                            int ldt, double *V, int ldv) {
    const size_t total = (size_t)nw * nw;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nw), j = (int)(idx / nw);
        AT(T, ldt, i, j) = (i <= j + 1) ? AT(H, ldh, off + i, off + j) : 0.0;
        AT(V, ldv, i, j) = (i == j) ? 1.0 : 0.0;
    }
}

// The deflation half of the AED step on the window T (real Schur form, rows
// 0..infqr-1 unconverged), V its accumulated factor; one workgroup.  The spike
// is s = H(kwtop, kwtop-1) times the first row of V (0 when kwtop == ktop).
// x: nw doubles of global scratch.  status as k_aed's ([0] nd, [1] Ritz values
// written, [2] 1 if T and V changed, [3] infqr, [4] swap rejected, [5] 0,
// [6] swaps, [7] 0, [8..9] cycles of the spike test and of the re-Hessenberg
// reduction, [10] late deflations); *spike0 receives the new coupling entry.
extern "C" __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_aed_wide(const double *H, int ldh, int ktop, int kbot, double *T, double *V, int ld, int nw, int infqr,
           double hnorm, double smlnum, int criterion, double *x, int *status, double *sr, double *si,
           double *spike0) {
    const int kwtop = kbot - nw + 1;
    const double s = (kwtop > ktop) ? AT(H, ldh, kwtop, kwtop - 1) : 0.0;
    AedOut o;
    o.iters = 0;
    o.infqr = infqr;
    o.cyc_qr = 0;
    aed_deflate(T, V, ld, x, nw, s, hnorm, smlnum, criterion, sr, si, o);
    if (threadIdx.x == 0) {
        status[0] = o.nd;
        status[1] = o.nritz;
        status[2] = (o.nd > 0) ? 1 : 0;
        status[3] = o.infqr;
        status[4] = o.swapfail;
        status[5] = 0;
        status[6] = o.nswap;
        status[7] = 0;
        status[8] = (int)min(o.cyc_defl, (long long)INT_MAX);
        status[9] = (int)min(o.cyc_hess, (long long)INT_MAX);
        status[10] = o.late;
        *spike0 = o.spike0;
    }
}

// Write the transformed window back: H's diagonal block at (kwtop, kwtop) <- T
// (zeros below the subdiagonal), Vt <- V^T, and H(kwtop, kwtop-1) <- *spike0
// when the window does not start the active block.
extern "C" __global__ void __launch_bounds__(256) k_win_store(double *H, int ldh, int ktop, int kwtop, int nw,
                                                             const double *T, const double *V, int ld, double *Vt,
                                                             int ldvt, const double *spike0) {
    const size_t total = (size_t)nw * nw;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nw), j = (int)(idx / nw);
        AT(H, ldh, kwtop + i, kwtop + j) = (i <= j + 1) ? AT(T, ld, i, j) : 0.0;
        AT(Vt, ldvt, j, i) = AT(V, ld, i, j);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && kwtop > ktop) AT(H, ldh, kwtop, kwtop - 1) = *spike0;
}
