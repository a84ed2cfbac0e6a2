// util.hip -- O(n^2) and O(n) passes around the iteration: input preparation,
// the negligible-subdiagonal scan that splits the active block, the final
// read-out of the eigenvalues from the real Schur form (Section 2, eq. 4), and
// small gathers for the host's control decisions.
#include "neig_dev.h"

// Zero entries below the subdiagonal, flag non-finite entries, and produce one
// scaled sum of squares (scale, ssq) per workgroup for ||H||_F.
extern "C" __global__ void __launch_bounds__(256)
k_prep(double *H, int ldh, int n, int *bad, double *part) {
    __shared__ double smax[256], sssq[256];
    double mx = 0.0;
    int nonfinite = 0;
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (i > j + 1) {
                AT(H, ldh, i, j) = 0.0;
            } else {
                double v = AT(H, ldh, i, j);
                if (!isfinite(v)) nonfinite = 1;
                else mx = fmax(mx, fabs(v));
            }
        }
    }
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
        __syncthreads();
    }
    const double scale = smax[0];
    double ssq = 0.0;
    if (scale > 0.0) {
        for (int j = blockIdx.x; j < n; j += gridDim.x) {
            const int top = (j + 2 < n) ? j + 2 : n;
            for (int i = threadIdx.x; i < top; i += blockDim.x) {
                double v = AT(H, ldh, i, j);
                if (isfinite(v)) ssq += (v / scale) * (v / scale);
            }
        }
    }
    sssq[threadIdx.x] = ssq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sssq[threadIdx.x] += sssq[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = scale;
        part[2 * blockIdx.x + 1] = sssq[0];
    }
    if (nonfinite) atomicOr(bad, 1);
}

// Zero every negligible subdiagonal entry h(k,k-1), 1 <= k <= kbot, and record
// the largest such k in *out (which the host clears first).
extern "C" __global__ void __launch_bounds__(256)
k_scan(double *H, int ldh, int kbot, double hnorm, double smlnum, int *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (k > kbot) return;
    const double sub = AT(H, ldh, k, k - 1);
    if (sub == 0.0) {
        atomicMax(out, k);
        return;
    }
    if (negligible_sub(sub, AT(H, ldh, k - 1, k - 1), AT(H, ldh, k, k), hnorm, smlnum)) {
        AT(H, ldh, k, k - 1) = 0.0;
        atomicMax(out, k);
    }
}

// Gather diagonal, subdiagonal and superdiagonal entries of rows lo..hi into buf
// (3 * (hi - lo + 1) doubles) for host-side shift decisions.
extern "C" __global__ void k_gather(const double *H, int ldh, int lo, int hi, double *buf) {
    const int m = hi - lo + 1;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int i = lo + t;
        buf[t] = AT(H, ldh, i, i);
        buf[m + t] = (i > 0) ? AT(H, ldh, i, i - 1) : 0.0;
        buf[2 * m + t] = (i + 1 < hi + 1) ? AT(H, ldh, i, i + 1) : 0.0;
    }
}

// For every decoupled 2x2 diagonal block that is not in standard form, compute
// the standardising rotation; flag[j] = 1 marks block starts needing one.  Rows
// of a part that did not converge (consecutive nonzero subdiagonals) are left
// alone: rotating them would need the rows below as well.
extern "C" __global__ void __launch_bounds__(256)
k_std_check(const double *H, int ldh, int n, int *flag, double *rot, int *count) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j + 1 >= n) return;
    flag[j] = 0;
    const double c = AT(H, ldh, j + 1, j);
    if (c == 0.0) return;
    if (j > 0 && AT(H, ldh, j, j - 1) != 0.0) return;          // not a block start
    if (j + 2 < n && AT(H, ldh, j + 2, j + 1) != 0.0) return;  // not decoupled below (unreduced part)
    const double a = AT(H, ldh, j, j), b = AT(H, ldh, j, j + 1), d = AT(H, ldh, j + 1, j + 1);
    if (a == d && b * c < 0.0) return;
    Std2 o = std2x2(a, b, c, d);
    rot[6 * j + 0] = o.cs; rot[6 * j + 1] = o.sn;
    rot[6 * j + 2] = o.a; rot[6 * j + 3] = o.b; rot[6 * j + 4] = o.c; rot[6 * j + 5] = o.d;
    flag[j] = 1;
    atomicAdd(count, 1);
}

// Apply the standardising rotation of block j to H's rows j, j+1 (right of the
// block), H's columns j, j+1 (above it) and Z's columns j, j+1; then store the
// standardised block.
extern "C" __global__ void __launch_bounds__(256)
k_std_apply(double *H, int ldh, double *Z, int ldz, int n, int j, const double *rot) {
    const double cs = rot[6 * j], sn = rot[6 * j + 1];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) {
        if (idx >= j + 2) {
            double x = AT(H, ldh, j, idx), y = AT(H, ldh, j + 1, idx);
            AT(H, ldh, j, idx) = cs * x + sn * y;
            AT(H, ldh, j + 1, idx) = -sn * x + cs * y;
        }
        if (idx < j) {
            double x = AT(H, ldh, idx, j), y = AT(H, ldh, idx, j + 1);
            AT(H, ldh, idx, j) = cs * x + sn * y;
            AT(H, ldh, idx, j + 1) = -sn * x + cs * y;
        }
        double x = AT(Z, ldz, idx, j), y = AT(Z, ldz, idx, j + 1);
        AT(Z, ldz, idx, j) = cs * x + sn * y;
        AT(Z, ldz, idx, j + 1) = -sn * x + cs * y;
    }
    if (idx == 0) {
        AT(H, ldh, j, j) = rot[6 * j + 2]; AT(H, ldh, j, j + 1) = rot[6 * j + 3];
        AT(H, ldh, j + 1, j) = rot[6 * j + 4]; AT(H, ldh, j + 1, j + 1) = rot[6 * j + 5];
    }
}

// Eigenvalues in the diagonal order of S: 1x1 blocks give (s_jj, 0); a 2x2
// block (a, b; c, a) gives (a, +sqrt|b| sqrt|c|) and (a, -sqrt|b| sqrt|c|).
extern "C" __global__ void __launch_bounds__(256)
k_eigs(const double *H, int ldh, int n, double *wr, double *wi) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool starts = (j + 1 < n) && AT(H, ldh, j + 1, j) != 0.0;
    const bool ends = (j > 0) && AT(H, ldh, j, j - 1) != 0.0;
    if (starts && !ends) {
        const double b = AT(H, ldh, j, j + 1), c = AT(H, ldh, j + 1, j);
        wr[j] = AT(H, ldh, j, j);
        wi[j] = sqrt(fabs(b)) * sqrt(fabs(c));
    } else if (ends && !(j >= 2 && AT(H, ldh, j - 1, j - 2) != 0.0)) {
        const double b = AT(H, ldh, j - 1, j), c = AT(H, ldh, j, j - 1);
        wr[j] = AT(H, ldh, j, j);
        wi[j] = -(sqrt(fabs(b)) * sqrt(fabs(c)));
    } else {
        wr[j] = AT(H, ldh, j, j);
        wi[j] = 0.0;
    }
}

// Set Z to the identity (for callers that pass no initial Z).
extern "C" __global__ void __launch_bounds__(256)
k_identity(double *Z, int ldz, int n) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int i = (int)(idx % n), j = (int)(idx / n);
    AT(Z, ldz, i, j) = (i == j) ? 1.0 : 0.0;
}
