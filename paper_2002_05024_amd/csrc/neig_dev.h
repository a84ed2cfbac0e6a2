// neig_dev.h -- device-side building blocks shared by the libneig kernels (gfx950).
//
// Householder reflectors of length <= 3 (the bulge reflectors of Section 3.2),
// the 2x2 standardisation of a real Schur block (Section 2, eq. 4), the
// negligible-subdiagonal test, and wavefront reductions.  Everything is FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define NEIG_EPS 2.220446049250313e-16      // 2^-52
#define NEIG_DBL_MIN 2.2250738585072014e-308

typedef double neig_d4 __attribute__((ext_vector_type(4)));

// Column-major element access.
#define AT(M, ld, i, j) (M)[(size_t)(j) * (size_t)(ld) + (size_t)(i)]

// Smallest m * (m + 1) * 16 + 4096 byte LDS budget fits NEIG_SMALL_MAX (see the host).
#define NEIG_SMALL_MAX 96
#define NEIG_CHASE_MAX 96   // rows/cols of U in one chase window
#define NEIG_MAX_CHAINS 32

// Reflector P = I - tau v v^T with v = (1, v1, v2) mapping x = (x0, x1, x2) to (beta, 0, 0).
struct Refl {
    double tau, v1, v2, beta;
};

// Square root and reciprocal of an argument well inside the normal range
// (1e-300 .. 1e300): the hardware approximations refined by Newton steps
// (Goldschmidt's coupled iteration for the square root), correct to about one
// unit in the last place.  They skip the range scaling that the general library
// routines add, which sits on the critical path of every bulge step.
__device__ __forceinline__ double sqrt_normal(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

__device__ __forceinline__ double rcp_normal(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ Refl make_refl(double x0, double x1, double x2) {
    Refl r;
    const double s = fabs(x1) + fabs(x2);
    if (s == 0.0) {
        r.tau = 0.0; r.v1 = 0.0; r.v2 = 0.0; r.beta = x0;
        return r;
    }
    const double mx = fmax(fabs(x0), s);
    if (mx > 1e-150 && mx < 1e150) {
        // no overflow or harmful underflow in the squares or in beta (x0 - beta);
        // one division gives both 1/beta and 1/(x0 - beta)
        const double nrm = sqrt_normal(x0 * x0 + x1 * x1 + x2 * x2);
        const double beta = (x0 >= 0.0) ? -nrm : nrm;
        const double d = x0 - beta;
        const double q = rcp_normal(beta * d);
        const double inv = beta * q;  // 1 / (x0 - beta)
        r.tau = -d * d * q;           // (beta - x0) / beta
        r.v1 = x1 * inv;
        r.v2 = x2 * inv;
        r.beta = beta;
        return r;
    }
    const double rs = 1.0 / mx;
    const double a = x0 * rs, b = x1 * rs, c = x2 * rs;
    const double nrm = mx * sqrt(a * a + b * b + c * c);
    const double beta = (x0 >= 0.0) ? -nrm : nrm;
    const double inv = 1.0 / (x0 - beta);
    r.tau = (beta - x0) / beta;
    r.v1 = x1 * inv;
    r.v2 = x2 * inv;
    r.beta = beta;
    return r;
}

// Standardisation of one 2x2 block B = [[a b][c d]] (real Schur form, eq. 4):
// G = [[cs -sn][sn cs]] with G^T B G upper triangular (real eigenvalues) or with
// equal diagonal entries and b' c' < 0 (complex pair).  Reasoning: with
// p = (a - d)/2 a rotation by t turns (p, (b + c)/2) by 2t and keeps (b - c)/2 and
// the trace; p^2 + bc decides real versus complex.
struct Std2 {
    double a, b, c, d, cs, sn;
    double rr1, ri1, rr2, ri2;
};

__device__ __forceinline__ Std2 std2x2(double a, double b, double c, double d) {
    Std2 o;
    o.ri1 = o.ri2 = 0.0;
    if (c == 0.0) {
        o.a = a; o.b = b; o.c = 0.0; o.d = d; o.cs = 1.0; o.sn = 0.0;
        o.rr1 = a; o.rr2 = d;
        return o;
    }
    if (b == 0.0) {
        o.a = d; o.b = -c; o.c = 0.0; o.d = a; o.cs = 0.0; o.sn = 1.0;
        o.rr1 = d; o.rr2 = a;
        return o;
    }
    double p = 0.5 * (a - d);
    double bc = b * c;
    double disc = p * p + bc;
    if (disc >= 0.0) {
        double r = sqrt(disc);
        double z = (p >= 0.0) ? p + r : p - r;
        if (z == 0.0) {
            o.a = a; o.b = b; o.c = 0.0; o.d = d; o.cs = 1.0; o.sn = 0.0;
            o.rr1 = a; o.rr2 = d;
            return o;
        }
        double t = hypot(z, c);
        double cs = z / t, sn = c / t;
        o.cs = cs; o.sn = sn;
        o.a = d + z;
        o.d = d - bc / z;
        o.b = (d - a) * cs * sn + b * cs * cs - c * sn * sn;
        o.c = 0.0;
        o.rr1 = o.a; o.rr2 = o.d;
        return o;
    }
    double q = 0.5 * (b + c), k = 0.5 * (b - c);
    double r = hypot(p, q);
    double cs = 1.0, sn = 0.0;
    if (r != 0.0) {
        double c2 = q / r, s2 = -p / r;
        if (c2 >= 0.0) {
            cs = sqrt(0.5 * (1.0 + c2));
            sn = s2 / (2.0 * cs);
        } else {
            sn = copysign(sqrt(0.5 * (1.0 - c2)), s2);
            cs = s2 / (2.0 * sn);
        }
    }
    double m = 0.5 * (a + d);
    o.cs = cs; o.sn = sn;
    o.a = m; o.d = m; o.b = r + k; o.c = r - k;
    o.rr1 = o.rr2 = m;
    o.ri1 = sqrt(fabs(o.b)) * sqrt(fabs(o.c));
    o.ri2 = -o.ri1;
    return o;
}

// |h(k,k-1)| negligible next to its diagonal neighbours (classic criterion).
__device__ __forceinline__ bool negligible_sub(double sub, double dkm1, double dk, double hnorm, double smlnum) {
    double s = fabs(dkm1) + fabs(dk);
    if (s == 0.0) s = hnorm;
    return fabs(sub) <= fmax(smlnum, NEIG_EPS * s);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Eigenvalues of a 2x2 block (any form): returns real parts and |imag|.
__device__ __forceinline__ void eig2x2(double a, double b, double c, double d, double *r1, double *i1, double *r2,
                                       double *i2) {
    double p = 0.5 * (a - d);
    double disc = p * p + b * c;
    double m = 0.5 * (a + d);
    if (disc >= 0.0) {
        double r = sqrt(disc);
        *r1 = m + r; *r2 = m - r; *i1 = 0.0; *i2 = 0.0;
    } else {
        double r = sqrt(-disc);
        *r1 = m; *r2 = m; *i1 = r; *i2 = -r;
    }
}
