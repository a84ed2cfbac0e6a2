// mlp.hip -- the parameter-proposal network: a 24-64-64-(8+8) perceptron that
// proposes, per iteration of the Schur reduction, one of 8 shift-count bins and
// one of 8 deflation-window bins (the two tunables of the method, Section 3.2).
//
// Parameters are one FP32 vector: mu (24), sd (24) input normalisation (fixed),
// W1 (64x24 row-major), b1 (64), W2 (64x64), b2 (64), W3 (16x64), b3 (16).
// Training runs in FP32: k_mlp_grad computes the loss and gradient of the
// reward-weighted cross-entropy of a mini-batch (one workgroup per 32 samples,
// per-workgroup partial gradients), k_mlp_reduce sums the partials in a fixed
// order, k_mlp_adam applies an Adam step.  Inference rounds weights and layer
// inputs to BF16 (round to nearest even) and accumulates in FP32.
// k_policy computes the 24 features of one iteration from H on the device and
// runs the inference for that one sample.
#include "neig_dev.h"

#define MLP_NIN 24
#define MLP_NH 64
#define MLP_NOUT 16
#define MLP_NBIN 8
#define MLP_TILE 32
#define MLP_O_MU 0
#define MLP_O_SD 24
#define MLP_O_W1 48
#define MLP_O_B1 (MLP_O_W1 + MLP_NH * MLP_NIN)
#define MLP_O_W2 (MLP_O_B1 + MLP_NH)
#define MLP_O_B2 (MLP_O_W2 + MLP_NH * MLP_NH)
#define MLP_O_W3 (MLP_O_B2 + MLP_NH)
#define MLP_O_B3 (MLP_O_W3 + MLP_NOUT * MLP_NH)
#define MLP_NPARAM (MLP_O_B3 + MLP_NOUT)
#define POLICY_SAMPLE 1024

static_assert(MLP_NPARAM == 6848, "parameter layout");

// ---------------------------------------------------------------- training (FP32)

extern "C" __global__ void __launch_bounds__(256) k_mlp_grad(const float *theta, const float *X, const int *act_ns,
                                                              const int *act_nw, const float *wgt, int batch,
                                                              float inv_batch, float *partial, float *loss_partial) {
    __shared__ float xn[MLP_TILE][MLP_NIN];
    __shared__ float h1[MLP_TILE][MLP_NH];
    __shared__ float h2[MLP_TILE][MLP_NH];
    __shared__ float dz[MLP_TILE][MLP_NOUT];
    __shared__ float d2[MLP_TILE][MLP_NH];  // dL/da2
    __shared__ float d1[MLP_TILE][MLP_NH];  // dL/da1
    __shared__ float lred[MLP_TILE];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * MLP_TILE;
    const float *mu = theta + MLP_O_MU, *sd = theta + MLP_O_SD;
    const float *W1 = theta + MLP_O_W1, *b1 = theta + MLP_O_B1;
    const float *W2 = theta + MLP_O_W2, *b2 = theta + MLP_O_B2;
    const float *W3 = theta + MLP_O_W3, *b3 = theta + MLP_O_B3;
    for (int idx = tid; idx < MLP_TILE * MLP_NIN; idx += 256) {
        const int s = idx / MLP_NIN, k = idx % MLP_NIN;
        xn[s][k] = (s0 + s < batch) ? (X[(size_t)(s0 + s) * MLP_NIN + k] - mu[k]) / sd[k] : 0.0f;
    }
    __syncthreads();
    for (int idx = tid; idx < MLP_TILE * MLP_NH; idx += 256) {
        const int s = idx / MLP_NH, o = idx % MLP_NH;
        float acc = b1[o];
        for (int k = 0; k < MLP_NIN; ++k) acc += W1[o * MLP_NIN + k] * xn[s][k];
        h1[s][o] = fmaxf(acc, 0.0f);
    }
    __syncthreads();
    for (int idx = tid; idx < MLP_TILE * MLP_NH; idx += 256) {
        const int s = idx / MLP_NH, o = idx % MLP_NH;
        float acc = b2[o];
        for (int k = 0; k < MLP_NH; ++k) acc += W2[o * MLP_NH + k] * h1[s][k];
        h2[s][o] = fmaxf(acc, 0.0f);
    }
    __syncthreads();
    for (int idx = tid; idx < MLP_TILE * MLP_NOUT; idx += 256) {
        const int s = idx / MLP_NOUT, o = idx % MLP_NOUT;
        float acc = b3[o];
        for (int k = 0; k < MLP_NH; ++k) acc += W3[o * MLP_NH + k] * h2[s][k];
        dz[s][o] = acc;  // logits for now
    }
    __syncthreads();
    // softmax of both heads, cross-entropy, and dL/dz = w/B (p - onehot)
    if (tid < 2 * MLP_TILE) {
        const int s = tid >> 1, head = tid & 1;
        float *zz = &dz[s][head * MLP_NBIN];
        const bool valid = s0 + s < batch;
        const float w = valid ? wgt[s0 + s] : 0.0f;
        const int target = valid ? (head ? act_nw[s0 + s] : act_ns[s0 + s]) : 0;
        float mx = zz[0];
        for (int k = 1; k < MLP_NBIN; ++k) mx = fmaxf(mx, zz[k]);
        float den = 0.0f;
        for (int k = 0; k < MLP_NBIN; ++k) den += expf(zz[k] - mx);
        const float lse = mx + logf(den);
        const float ce = lse - zz[target];
        for (int k = 0; k < MLP_NBIN; ++k) {
            const float pk = expf(zz[k] - lse);
            zz[k] = w * inv_batch * (pk - (k == target ? 1.0f : 0.0f));
        }
        // two heads of one sample sit in adjacent lanes of one wave
        const float other = __shfl_xor(w * inv_batch * ce, 1);
        if (head == 0) lred[s] = w * inv_batch * ce + other;
    }
    __syncthreads();
    // back through layer 3
    for (int idx = tid; idx < MLP_TILE * MLP_NH; idx += 256) {
        const int s = idx / MLP_NH, k = idx % MLP_NH;
        float acc = 0.0f;
        for (int o = 0; o < MLP_NOUT; ++o) acc += dz[s][o] * W3[o * MLP_NH + k];
        d2[s][k] = (h2[s][k] > 0.0f) ? acc : 0.0f;
    }
    __syncthreads();
    for (int idx = tid; idx < MLP_TILE * MLP_NH; idx += 256) {
        const int s = idx / MLP_NH, k = idx % MLP_NH;
        float acc = 0.0f;
        for (int o = 0; o < MLP_NH; ++o) acc += d2[s][o] * W2[o * MLP_NH + k];
        d1[s][k] = (h1[s][k] > 0.0f) ? acc : 0.0f;
    }
    __syncthreads();
    // parameter gradients of this tile: sums over its samples
    float *g = partial + (size_t)blockIdx.x * MLP_NPARAM;
    for (int i = tid; i < MLP_NPARAM; i += 256) {
        float acc = 0.0f;
        if (i < MLP_O_W1) {
            acc = 0.0f;
        } else if (i < MLP_O_B1) {
            const int o = (i - MLP_O_W1) / MLP_NIN, k = (i - MLP_O_W1) % MLP_NIN;
            for (int s = 0; s < MLP_TILE; ++s) acc += d1[s][o] * xn[s][k];
        } else if (i < MLP_O_W2) {
            const int o = i - MLP_O_B1;
            for (int s = 0; s < MLP_TILE; ++s) acc += d1[s][o];
        } else if (i < MLP_O_B2) {
            const int o = (i - MLP_O_W2) / MLP_NH, k = (i - MLP_O_W2) % MLP_NH;
            for (int s = 0; s < MLP_TILE; ++s) acc += d2[s][o] * h1[s][k];
        } else if (i < MLP_O_W3) {
            const int o = i - MLP_O_B2;
            for (int s = 0; s < MLP_TILE; ++s) acc += d2[s][o];
        } else if (i < MLP_O_B3) {
            const int o = (i - MLP_O_W3) / MLP_NH, k = (i - MLP_O_W3) % MLP_NH;
            for (int s = 0; s < MLP_TILE; ++s) acc += dz[s][o] * h2[s][k];
        } else {
            const int o = i - MLP_O_B3;
            for (int s = 0; s < MLP_TILE; ++s) acc += dz[s][o];
        }
        g[i] = acc;
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) l += lred[s];
        loss_partial[blockIdx.x] = l;
    }
}

// grad[i] = sum over workgroups of partial[b][i], in workgroup order; the loss likewise.
extern "C" __global__ void k_mlp_reduce(const float *partial, const float *loss_partial, int nblk, float *grad,
                                        float *loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_NPARAM) {
        float acc = 0.0f;
        for (int b = 0; b < nblk; ++b) acc += partial[(size_t)b * MLP_NPARAM + i];
        grad[i] = acc;
    }
    if (i == MLP_NPARAM) {
        float acc = 0.0f;
        for (int b = 0; b < nblk; ++b) acc += loss_partial[b];
        *loss = acc;
    }
}

// Adam: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
// theta <- theta - lr (m / bc1) / (sqrt(v / bc2) + eps); mu and sd untouched.
// 1 - b1 and 1 - b2 come from the host (in float, 1 - 0.999f loses four digits).
extern "C" __global__ void k_mlp_adam(float *theta, const float *grad, float *m, float *v, float lr, float beta1,
                                      float beta2, float one_m_beta1, float one_m_beta2, float eps, float bc1,
                                      float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_O_W1 || i >= MLP_NPARAM) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + one_m_beta1 * gi;
    const float vi = beta2 * v[i] + one_m_beta2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------- inference (BF16 operands, FP32 sums)

__device__ __forceinline__ float bf16_round(float x) {
    unsigned int u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // Inf / NaN pass through
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// Forward pass of up to 4 samples per workgroup, wave w taking sample w when
// live[w]; x[w] (24 raw features), scratch ha[w], hb[w] (64 each) and the scores
// z[w] (16) in LDS.  Every thread of the workgroup calls this (it synchronises).
__device__ __forceinline__ void mlp_infer_block(const float *theta, float (*x)[MLP_NIN], float (*ha)[MLP_NH],
                                                float (*hb)[MLP_NH], float (*z)[MLP_NOUT], const bool *live) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool on = live[wv];
    const float *mu = theta + MLP_O_MU, *sd = theta + MLP_O_SD;
    const float *W1 = theta + MLP_O_W1, *b1 = theta + MLP_O_B1;
    const float *W2 = theta + MLP_O_W2, *b2 = theta + MLP_O_B2;
    const float *W3 = theta + MLP_O_W3, *b3 = theta + MLP_O_B3;
    if (on && lane < MLP_NIN) hb[wv][lane] = bf16_round((x[wv][lane] - mu[lane]) / sd[lane]);
    __syncthreads();
    if (on) {
        float acc = 0.0f;
        for (int k = 0; k < MLP_NIN; ++k) acc += bf16_round(W1[lane * MLP_NIN + k]) * hb[wv][k];
        ha[wv][lane] = bf16_round(fmaxf(acc + b1[lane], 0.0f));
    }
    __syncthreads();
    if (on) {
        float acc = 0.0f;
        for (int k = 0; k < MLP_NH; ++k) acc += bf16_round(W2[lane * MLP_NH + k]) * ha[wv][k];
        hb[wv][lane] = bf16_round(fmaxf(acc + b2[lane], 0.0f));
    }
    __syncthreads();
    if (on && lane < MLP_NOUT) {
        float acc = 0.0f;
        for (int k = 0; k < MLP_NH; ++k) acc += bf16_round(W3[lane * MLP_NH + k]) * hb[wv][k];
        z[wv][lane] = acc + b3[lane];
    }
    __syncthreads();
}

// Bin with the largest score of one head and its softmax probability.
__device__ __forceinline__ void head_pick(const float *z, int *bin, float *prob) {
    int best = 0;
    float mx = z[0];
    for (int k = 1; k < MLP_NBIN; ++k)
        if (z[k] > mx) {
            mx = z[k];
            best = k;
        }
    float den = 0.0f;
    for (int k = 0; k < MLP_NBIN; ++k) den += expf(z[k] - mx);
    *bin = best;
    *prob = 1.0f / den;
}

// Batched inference: wave w of workgroup b handles samples 4b + w, 4b + w + 4*grid, ...
extern "C" __global__ void __launch_bounds__(256) k_mlp_infer(const float *theta, const float *X, int batch,
                                                               float *logits, int *bins, float *conf) {
    __shared__ float sx[4][MLP_NIN], sa[4][MLP_NH], sb[4][MLP_NH], sz[4][MLP_NOUT];
    __shared__ bool live[4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s0 = blockIdx.x * 4; s0 < batch; s0 += gridDim.x * 4) {
        const int s = s0 + wv;
        if (lane == 0) live[wv] = s < batch;
        if (s < batch && lane < MLP_NIN) sx[wv][lane] = X[(size_t)s * MLP_NIN + lane];
        __syncthreads();
        mlp_infer_block(theta, sx, sa, sb, sz, live);
        if (s < batch) {
            if (lane < MLP_NOUT) logits[(size_t)s * MLP_NOUT + lane] = sz[wv][lane];
            if (lane < 2) {
                int bn;
                float p;
                head_pick(sz[wv] + lane * MLP_NBIN, &bn, &p);
                bins[2 * s + lane] = bn;
                conf[2 * s + lane] = p;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- features + decision for one iteration

// Features of the active block [ktop, kbot] of H (order n, ||H||_F = hnorm):
//   f0       log m, m = kbot - ktop + 1
//   f1..f19  quantiles 5%, 10%, ..., 95% of log(|h(k,k-1)| / (hnorm / sqrt n)) over
//            at most 1024 subdiagonal entries k = ktop+1+floor(i (m-1) / S), i < S
//   f20..f23 supplied by the caller (Ritz-value statistics, previous deflations)
// then the BF16 inference.  out_feat[24]; out_bins[2]; out_conf[2].
extern "C" __global__ void __launch_bounds__(256) k_policy(const double *H, int ldh, int n, int ktop, int kbot,
                                                            double hnorm, float f20, float f21, float f22, float f23,
                                                            const float *theta, float *out_feat, int *out_bins,
                                                            float *out_conf) {
    __shared__ float v[POLICY_SAMPLE];
    __shared__ float x[4][MLP_NIN], ha[4][MLP_NH], hb[4][MLP_NH], z[4][MLP_NOUT];
    __shared__ bool live[4];
    const int tid = threadIdx.x;
    const int m = kbot - ktop + 1;
    const int cnt = m - 1;
    const int S = cnt < POLICY_SAMPLE ? cnt : POLICY_SAMPLE;
    const double scale = (hnorm > 0.0 && n > 0) ? hnorm / sqrt((double)n) : 1.0;
    for (int i = tid; i < POLICY_SAMPLE; i += 256) {
        float val = INFINITY;
        if (i < S) {
            const int k = ktop + 1 + (int)(((long long)i * cnt) / S);
            const double h = fabs(AT(H, ldh, k, k - 1));
            val = (float)log(fmax(h, 1e-300) / scale);
        }
        v[i] = val;
    }
    __syncthreads();
    // bitonic sort of the 1024 values (padding +inf sorts last)
    for (int size = 2; size <= POLICY_SAMPLE; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < POLICY_SAMPLE / 2; i += 256) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const float a = v[lo], b = v[hi];
                if ((a > b) == up) {
                    v[lo] = b;
                    v[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    if (tid < 4) live[tid] = tid == 0;
    if (tid == 0) x[0][0] = logf((float)m);
    if (tid >= 1 && tid <= 19) {
        float q = 0.0f;
        if (S > 0) {
            const float p = 0.05f * (float)tid;
            const float pos = p * (float)(S - 1);
            const int lo = (int)floorf(pos);
            const int hi = lo + 1 < S ? lo + 1 : S - 1;
            q = v[lo] + (pos - (float)lo) * (v[hi] - v[lo]);
        }
        x[0][tid] = q;
    }
    if (tid == 20) x[0][20] = f20;
    if (tid == 21) x[0][21] = f21;
    if (tid == 22) x[0][22] = f22;
    if (tid == 23) x[0][23] = f23;
    __syncthreads();
    mlp_infer_block(theta, x, ha, hb, z, live);
    if (tid < MLP_NIN) out_feat[tid] = x[0][tid];
    if (tid < 2) {
        int bn;
        float p;
        head_pick(z[0] + tid * MLP_NBIN, &bn, &p);
        out_bins[tid] = bn;
        out_conf[tid] = p;
    }
}
