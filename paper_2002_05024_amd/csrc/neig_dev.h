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

// The hardware reciprocal is good to about 2^-24 relative; each Newton step
// squares the error, so two give the reciprocal to within about half a unit in
// the last place (measured on gfx950 over 2^20 arguments spread over 2^+-40).
__device__ __forceinline__ double rcp_normal(double a) {
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
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

// Standardisation of one 2x2 block of a real Schur form (Section 2, eq. 4).
// Result: a rotation G = [[cs -sn][sn cs]] and the block G^T B G, which is upper
// triangular when the eigenvalues are real and otherwise has equal diagonal
// entries and off-diagonal entries of opposite sign.
//
// Construction (two angles, composed):
//  1. Rotating by t changes the diagonal difference to
//     (a - d) cos 2t + (b + c) sin 2t, so tan 2t1 = (d - a) / (b + c) gives a
//     block [[m b1][c1 m]], m the mean of the diagonal.  tan t1 is taken as the
//     root of modulus <= 1 of tan 2t1 = 2 tan t1 / (1 - tan^2 t1).
//  2. The eigenvalues of that block are m +- sqrt(b1 c1).  If b1 and c1 have
//     opposite signs the pair is complex and the block is final.  Otherwise
//     rotating it by t2 leaves (2,1) entry c1 cos^2 t2 - b1 sin^2 t2, which a
//     rotation with (cos t2, sin t2) proportional to (sqrt|b1|, sqrt|c1|)
//     annihilates.
// The output block is formed from B itself by the composed rotation (one
// rounding step on the diagonal), and the entry that is zero in exact
// arithmetic is set to zero.
struct Std2 {
    double a, b, c, d, cs, sn;
};

// G^T [[a b][c d]] G for G = [[C -S][S C]]: out = (0,0), (0,1), (1,0), (1,1).
__device__ __forceinline__ void rot2_similarity(double a, double b, double c, double d, double C, double S,
                                                double (&out)[4]) {
    const double p00 = a * C + b * S, p01 = b * C - a * S;  // B G, first row
    const double p10 = c * C + d * S, p11 = d * C - c * S;  // B G, second row
    out[0] = C * p00 + S * p10;
    out[1] = C * p01 + S * p11;
    out[2] = C * p10 - S * p00;
    out[3] = C * p11 - S * p01;
}

__device__ __forceinline__ Std2 std2x2(double a, double b, double c, double d) {
    Std2 o{a, b, c, d, 1.0, 0.0};
    if (c == 0.0) return o;  // already triangular
    const double big = fmax(fmax(fabs(a), fabs(b)), fmax(fabs(c), fabs(d)));
    const double inv = 1.0 / big;
    // angle 1 (scale-free, so computed on the scaled entries)
    const double u = d * inv - a * inv, v = b * inv + c * inv;
    double t1 = 0.0;
    if (u != 0.0) {
        const double h = hypot(u, v);
        t1 = u / (v >= 0.0 ? v + h : v - h);
    }
    const double C1 = 1.0 / sqrt(1.0 + t1 * t1), S1 = t1 * C1;
    double e[4];
    rot2_similarity(a, b, c, d, C1, S1, e);
    if ((e[1] > 0.0 && e[2] < 0.0) || (e[1] < 0.0 && e[2] > 0.0)) {
        const double m = 0.5 * (e[0] + e[3]);
        o.a = m; o.b = e[1]; o.c = e[2]; o.d = m; o.cs = C1; o.sn = S1;
        return o;
    }
    // angle 2 (real pair)
    const double p = sqrt(fabs(e[1] * inv)), q = sqrt(fabs(e[2] * inv));
    const double r = hypot(p, q);
    const double C2 = (r > 0.0) ? p / r : 1.0, S2 = (r > 0.0) ? q / r : 0.0;
    const double C = C1 * C2 - S1 * S2, S = S1 * C2 + C1 * S2;
    rot2_similarity(a, b, c, d, C, S, e);
    o.a = e[0]; o.b = e[1]; o.c = 0.0; o.d = e[3]; o.cs = C; o.sn = S;
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
