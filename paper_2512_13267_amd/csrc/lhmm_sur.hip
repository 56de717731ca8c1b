// lhmm_sur.hip -- gfx950 kernels and runtime of the stress surrogate: an
// ensemble of MLPs (n_in -> n_hidden -> n_hidden -> n_out, GELU) trained with
// mean-squared error and Adam, evaluated in the LHMM loop with an ensemble
// spread gate (include/lhmm.h, lhmm_sur_*).
//
// Every product is one NT GEMM  C[M x N] = A[M x K] * B[N x K]^T  on BF16
// operands with FP32 accumulation (v_mfma_f32_32x32x16_bf16), one wave per
// 32 x 32 x NT output tile (NT = 4, 2 or 1 as N allows), batched over the
// ensemble members (grid z).  Operand
// fragments are loaded straight from global memory as 16-byte vectors (lane
// l takes row l%32 and k-slice 8*(l/32) .. +7 of A and of B), so every
// operand is kept in the layout whose reduction index is contiguous:
//   forward  Z = X W:  A = X [B x nin],  B = W^T [nh x nin]
//   backward dH = dZ W^T: A = dZ [B x nout], B = W [nin x nout]
//   weights  dW = X^T dZ: A = X^T [nin x B], B = dZ^T [nout x B]
// Epilogues add the bias, apply GELU (keeping the FP32 pre-activation) or
// multiply by GELU'(Z), and write BF16 results in both layouts as needed.
// Dimensions are padded: inputs to a multiple of 32, outputs to 32, batch
// rows to a multiple of 32 (padded rows carry zero gradient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "lhmm.h"
#include "lhmm_internal.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int HIST = LHMM_SUR_HIST;  // gradient samples per feature vector

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi {
    EPI_F32 = 0,      // C -> f32 [M x N]
    EPI_BIAS_F32,     // C + bias -> f32 [M x N]
    EPI_BIAS_GELU,    // Z = C + bias -> f32; H = gelu(Z) -> bf16 [M x N] and [N x M]
    EPI_GELU_GRAD,    // dZ = C * gelu'(Z) -> f32 [M x N], bf16 [M x N] and [N x M]
};

struct Gemm {
    const bf16* A;
    const bf16* B;
    int M, N, K, lda, ldb;
    long sA, sB;       // member strides (elements)
    const float* bias;  // [N] per member
    long sBias;
    const float* Zin;   // EPI_GELU_GRAD: pre-activation [M x N]
    float* Cf;          // f32 output [M x N]
    bf16* Cb;           // bf16 output [M x N] (ld = N)
    bf16* Ct;           // bf16 transposed output [N x M] (ld = ldt)
    int ldt;
    long sC, sCt;       // member strides of the M x N and N x M outputs
    int ksplit, kchunk;  // EPI_F32: grid z = member x k-chunk, partial sums per chunk
};

// One wave computes NT adjacent 32 x 32 output tiles of one member; the A
// fragment of a k-slice is shared by the NT products, and the fragments of
// the next k-slice are loaded while the current ones are multiplied.  The
// accumulation order over k is the same for every NT.
template <int EPI, int NT>
__global__ __launch_bounds__(64) void k_gemm_nt(Gemm g) {
    // with a k-split, z = member x ksplit + chunk and the output at z x sC is
    // the chunk's partial product
    const int z = blockIdx.z;
    const int e = z / g.ksplit, kc = z % g.ksplit;
    const int n0 = blockIdx.x * 32 * NT, m0 = blockIdx.y * 32;
    const int l = threadIdx.x;
    const int koff = kc * g.kchunk;
    const bf16* A = g.A + e * g.sA + (long)(m0 + (l & 31)) * g.lda + 8 * (l >> 5) + koff;
    const bf16* B = g.B + e * g.sB + (long)(n0 + (l & 31)) * g.ldb + 8 * (l >> 5) + koff;
    const long bstep = 32L * g.ldb;
    floatx16 acc[NT];
    bf16x8 b[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        acc[j] = floatx16{};
        b[j] = *(const bf16x8*)(B + j * bstep);
    }
    bf16x8 a = *(const bf16x8*)A;
    const int K = min(g.kchunk, g.K - koff);
    for (int k = 16; k < K; k += 16) {
        const bf16x8 an = *(const bf16x8*)(A + k);
        bf16x8 bn[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) bn[j] = *(const bf16x8*)(B + j * bstep + k);
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[j], acc[j], 0, 0, 0);
        a = an;
#pragma unroll
        for (int j = 0; j < NT; ++j) b[j] = bn[j];
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[j], acc[j], 0, 0, 0);
    const long cbase = z * g.sC, tbase = e * g.sCt;
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int col = n0 + 32 * j + (l & 31);
        float bias = 0.0f;
        if (EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_GELU) bias = g.bias[e * g.sBias + col];
        // value v of the tile sits at row 8 (v / 4) + 4 (l / 32) + v % 4: each
        // group of four is four consecutive rows, stored transposed at once
#pragma unroll
        for (int vg = 0; vg < 4; ++vg) {
            const int row0 = m0 + 8 * vg + 4 * (l >> 5);
            bf16x4 tq;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = row0 + u;
                const long idx = cbase + (long)row * g.N + col;
                const float c = acc[j][4 * vg + u];
                if (EPI == EPI_F32) {
                    g.Cf[idx] = c;
                } else if (EPI == EPI_BIAS_F32) {
                    g.Cf[idx] = c + bias;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = c + bias;
                    const bf16 h = (bf16)gelu_f(z);
                    g.Cb[idx] = h;
                    if (g.Cf) g.Cf[idx] = z;  // the pre-activation and H^T only feed backward
                    tq[u] = h;
                } else {  // EPI_GELU_GRAD
                    const float dz = c * gelu_grad_f(g.Zin[idx]);
                    g.Cf[idx] = dz;
                    const bf16 hb = (bf16)dz;
                    g.Cb[idx] = hb;
                    tq[u] = hb;
                }
            }
            if (EPI == EPI_GELU_GRAD || (EPI == EPI_BIAS_GELU && g.Cf))
                *(bf16x4*)(g.Ct + tbase + (long)col * g.ldt + row0) = tq;
        }
    }
}

// sum the k-chunk partials of every member in chunk order:
// out[e][i] = sum_c part[(e ksplit + c) MN + i]
__global__ void k_splitk_sum(const float* __restrict__ part, int ksplit, long MN, int E, float* __restrict__ out,
                             long ostride) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)E * MN) return;
    const int e = (int)(t / MN);
    const long i = t % MN;
    const float* p = part + (long)e * ksplit * MN + i;
    float s = 0.0f;
    for (int c = 0; c < ksplit; ++c) s += p[(long)c * MN];
    out[e * ostride + i] = s;
}

// caller features (B x n_in, f32) -> padded BF16 inputs X [Bp x nin_p] and
// X^T [nin_p x Bp]; padding rows and columns are zero
__global__ void k_inputs(const float* __restrict__ x, int B, int nin, int Bp, int nin_p, bf16* __restrict__ X,
                         bf16* __restrict__ Xt) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)Bp * nin_p) return;
    const int r = (int)(t / nin_p), c = (int)(t % nin_p);
    const bf16 v = (bf16)((r < B && c < nin) ? x[(long)r * nin + c] : 0.0f);
    X[t] = v;
    if (Xt) Xt[(long)c * Bp + r] = v;
}

// MSE gradient and per-block loss partials for every member:
// dY = 2 (Y - T) / (B n_out) on real rows and columns, 0 on padding.
__global__ void k_loss_grad(const float* __restrict__ Y, long ystride, const float* __restrict__ T, int B, int Bp,
                            int n_out, int nout_p, bf16* __restrict__ dY, bf16* __restrict__ dYt,
                            float* __restrict__ dYf, float* __restrict__ part) {
    __shared__ float sh[256];
    const int e = blockIdx.y;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.0f;
    if (t < (long)Bp * nout_p) {
        const int b = (int)(t / nout_p), j = (int)(t % nout_p);
        float d = 0.0f;
        if (b < B && j < n_out) {
            const float diff = Y[(long)e * ystride + t] - T[(long)b * n_out + j];
            sq = diff * diff;
            d = 2.0f * diff / (float)(B * n_out);
        }
        dYf[(long)e * Bp * nout_p + t] = d;
        dY[(long)e * Bp * nout_p + t] = (bf16)d;
        dYt[(long)e * nout_p * Bp + (long)j * Bp + b] = (bf16)d;
    }
    sh[threadIdx.x] = sq;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)e * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_loss_final(const float* __restrict__ part, int nparts, int B, int n_out, float* __restrict__ loss) {
    const int e = blockIdx.x;
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += part[(long)e * nparts + k];
    loss[e] = (float)(s / (double)(B * n_out));
}

// column sums of f32 [rows x cols] per member (bias gradients) in two
// passes, each in a fixed order.  k_colsum_part: the block of row slice z
// (64 columns x 16 row groups) sums the slice's rows, row group y taking
// every 16th, and adds its 16 partials in order; k_colsum_final adds the
// COLSUM_SLICES slices in order.  Slicing the rows keeps ~16 dependent loads
// per thread where one block per column tile would chain hundreds.
constexpr int COLSUM_SLICES = 16;

__global__ __launch_bounds__(1024) void k_colsum_part(const float* __restrict__ x, int rows, int cols, long stride,
                                                     float* __restrict__ part) {
    __shared__ float sh[16][64];
    const int e = blockIdx.y, z = blockIdx.z;
    const int c = blockIdx.x * 64 + threadIdx.x;
    const int len = (rows + COLSUM_SLICES - 1) / COLSUM_SLICES;
    const int r0 = z * len, r1 = min(rows, r0 + len);
    float s = 0.0f;
    if (c < cols) {
        const float* p = x + e * stride + c;
        for (int r = r0 + (int)threadIdx.y; r < r1; r += 16) s += p[(long)r * cols];
    }
    sh[threadIdx.y][threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.y == 0 && c < cols) {
        float t = 0.0f;
        for (int y = 0; y < 16; ++y) t += sh[y][threadIdx.x];
        part[((long)e * COLSUM_SLICES + z) * cols + c] = t;
    }
}

__global__ void k_colsum_final(const float* __restrict__ part, int cols, int n_members, float* __restrict__ out,
                               long ostride) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n_members * cols) return;
    const int e = (int)(t / cols), c = (int)(t % cols);
    float s = 0.0f;
    for (int z = 0; z < COLSUM_SLICES; ++z) s += part[((long)e * COLSUM_SLICES + z) * cols + c];
    out[e * ostride + c] = s;
}

// Adam on FP32 masters of one weight matrix [rows x cols] per member, then
// BF16 copies W [rows x cols] and W^T [cols x rows]
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int rows, int cols, long stride, int n_members, float lr, float c1,
                       float c2, bf16* __restrict__ wb, bf16* __restrict__ wt) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = (long)rows * cols;
    if (t >= per * n_members) return;
    const int e = (int)(t / per);
    const long q = t % per;
    const long idx = e * stride + q;
    const float gg = g[idx];
    const float mm = 0.9f * m[idx] + 0.1f * gg;
    const float vv = 0.999f * v[idx] + 0.001f * gg * gg;
    m[idx] = mm;
    v[idx] = vv;
    const float wn = w[idx] - lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    w[idx] = wn;
    if (wb) {
        const int r = (int)(q / cols), c = (int)(q % cols);
        const bf16 h = (bf16)wn;
        wb[e * stride + q] = h;
        wt[e * stride + (long)c * rows + r] = h;
    }
}

// member outputs (stride Bmax x nout_p) -> n_members x B x n_out
__global__ void k_outputs(const float* __restrict__ Ysrc, long stride, int nout_p, int E, int B, int nout,
                          float* __restrict__ Y) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)E * B * nout) return;
    const int e = (int)(t / ((long)B * nout));
    const long r = t % ((long)B * nout);
    const int b = (int)(r / nout), j = (int)(r % nout);
    Y[t] = Ysrc[e * stride + (long)b * nout_p + j];
}

// history ring of the in-plane gradient components: sample t of particle b
// goes to slot t mod HIST as (L_xx, L_xy, L_yx, L_yy)
__global__ void k_push_history(float* __restrict__ ring, int n, const double* __restrict__ gradL, long t,
                               float scale) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double* L = gradL + 9 * (long)b;
    float* o = ring + ((long)b * HIST + (int)(t % HIST)) * 4;
    o[0] = (float)(L[0] * scale);
    o[1] = (float)(L[1] * scale);
    o[2] = (float)(L[3] * scale);
    o[3] = (float)(L[4] * scale);
}

// features of particle b after sample t: samples t-HIST+1 .. t (oldest
// first, 4 components each) and the polymer fraction
__global__ void k_features(const float* __restrict__ ring, int n, long t, const float* __restrict__ phi,
                           float* __restrict__ X) {
    constexpr int NF = 4 * HIST + 1;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * NF) return;
    const int b = (int)(i / NF), f = (int)(i % NF);
    float x;
    if (f < 4 * HIST) {
        const int s = f / 4, c = f % 4;
        const int slot = (int)((t + 1 + s) % HIST);  // t + 1 - HIST + s, mod HIST
        x = ring[((long)b * HIST + slot) * 4 + c];
    } else {
        x = phi[b];
    }
    X[i] = x;
}

// ensemble mean and spread gate: spread = sqrt(mean_j var_members(Y_j)),
// flag if spread > threshold x max(|mean|_2, floor)
__global__ void k_gate(const float* __restrict__ Y, int n_members, int B, int Bp, int n_out, int nout_p,
                       float threshold, float floor_, float* __restrict__ mean, unsigned* __restrict__ flag) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float var_sum = 0.0f, norm2 = 0.0f;
    for (int j = 0; j < n_out; ++j) {
        float s = 0.0f, s2 = 0.0f;
        for (int e = 0; e < n_members; ++e) {
            const float y = Y[((long)e * Bp + b) * nout_p + j];
            s += y;
            s2 += y * y;
        }
        const float mu = s / n_members;
        var_sum += fmaxf(s2 / n_members - mu * mu, 0.0f);
        norm2 += mu * mu;
        mean[(long)b * n_out + j] = mu;
    }
    const float spread = sqrtf(var_sum / n_out);
    flag[b] = spread > threshold * fmaxf(sqrtf(norm2), floor_) ? 1u : 0u;
}

// micro stresses (xx, yy, zz, xy, xz, yz) -> deviatoric in-plane targets
// (xx - tr/3, xy, yy - tr/3) x inv_scale
__global__ void k_targets(const double* __restrict__ sigma, int n, float inv_scale, float* __restrict__ T) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double* s = sigma + 6 * (long)b;
    const double tr3 = (s[0] + s[1] + s[2]) / 3.0;
    T[3 * (long)b + 0] = (float)((s[0] - tr3) * inv_scale);
    T[3 * (long)b + 1] = (float)(s[3] * inv_scale);
    T[3 * (long)b + 2] = (float)((s[1] - tr3) * inv_scale);
}

// stress for the macro solver: the micro stress where use_dpd[b], else the
// traceless tensor built from the surrogate mean
__global__ void k_blend(const float* __restrict__ mean, const unsigned* __restrict__ use_dpd,
                        const double* __restrict__ sigma_dpd, int n, float scale, double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double* o = out + 6 * (long)b;
    if (use_dpd && use_dpd[b]) {
        for (int q = 0; q < 6; ++q) o[q] = sigma_dpd[6 * (long)b + q];
    } else {
        const double dxx = (double)mean[3 * (long)b] * scale, dxy = (double)mean[3 * (long)b + 1] * scale,
                     dyy = (double)mean[3 * (long)b + 2] * scale;
        o[0] = dxx;
        o[1] = dyy;
        o[2] = -(dxx + dyy);
        o[3] = dxy;
        o[4] = 0.0;
        o[5] = 0.0;
    }
}

// gradient sample s of the history ring back to micro gradients (n x 9)
__global__ void k_ring_to_grad(const float* __restrict__ ring, int n, long s, float inv_scale,
                               double* __restrict__ gradL) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const float* r = ring + ((long)b * HIST + (int)(s % HIST)) * 4;
    double* L = gradL + 9 * (long)b;
    const double xx = (double)r[0] * inv_scale, xy = (double)r[1] * inv_scale, yx = (double)r[2] * inv_scale;
    L[0] = xx; L[1] = xy; L[2] = 0.0;
    L[3] = yx; L[4] = -xx; L[5] = 0.0;
    L[6] = 0.0; L[7] = 0.0; L[8] = 0.0;
}

// symmetry image of sample b under the in-plane orthogonal map
// Q = Rot(theta_b) (diag(1, -1) if mirror_b): every gradient sample
// L -> Q L Q^T, the stress target S -> Q S Q^T, in place
__global__ void k_augment(float* __restrict__ X, float* __restrict__ T, int n, const float* __restrict__ theta,
                          const unsigned* __restrict__ mirror) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const float c = cosf(theta[b]), s = sinf(theta[b]);
    float q00 = c, q01 = -s, q10 = s, q11 = c;
    if (mirror[b]) {
        q01 = s;
        q11 = -c;
    }
    float* x = X + (long)b * LHMM_SUR_FEATURES;
    for (int k = 0; k < HIST; ++k) {
        const float l00 = x[4 * k], l01 = x[4 * k + 1], l10 = x[4 * k + 2], l11 = x[4 * k + 3];
        // A = Q L, then A Q^T
        const float a00 = q00 * l00 + q01 * l10, a01 = q00 * l01 + q01 * l11;
        const float a10 = q10 * l00 + q11 * l10, a11 = q10 * l01 + q11 * l11;
        x[4 * k] = a00 * q00 + a01 * q01;
        x[4 * k + 1] = a00 * q10 + a01 * q11;
        x[4 * k + 2] = a10 * q00 + a11 * q01;
        x[4 * k + 3] = a10 * q10 + a11 * q11;
    }
    float* y = T + 3 * (long)b;
    const float sxx = y[0], sxy = y[1], syy = y[2];
    const float a00 = q00 * sxx + q01 * sxy, a01 = q00 * sxy + q01 * syy;
    const float a10 = q10 * sxx + q11 * sxy, a11 = q10 * sxy + q11 * syy;
    y[0] = a00 * q00 + a01 * q01;
    y[1] = a00 * q10 + a01 * q11;
    y[2] = a10 * q10 + a11 * q11;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

struct lhmm_sur {
    int E = 0, nin = 0, nin_p = 0, nh = 0, nout = 0, nout_p = 32, Bmax = 0, step = 0;
    int device = 0;  // the device current at create
    hipStream_t stream = nullptr;
    std::vector<void*> bufs;
    // FP32 masters, grads, Adam moments, per member (stride = size of one member's tensor)
    float *W1 = nullptr, *b1 = nullptr, *W2 = nullptr, *b2 = nullptr, *W3 = nullptr, *b3 = nullptr;
    float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
    float *mW1, *mb1, *mW2, *mb2, *mW3, *mb3, *vW1, *vb1, *vW2, *vb2, *vW3, *vb3;
    // BF16 weights in both layouts
    bf16 *W1b, *W1t, *W2b, *W2t, *W3b, *W3t;
    // activations
    bf16 *X, *Xt, *H1, *H1t, *H2, *H2t, *dY, *dYt, *dZ2, *dZ2t, *dZ1, *dZ1t;
    float *Z1, *Z2, *Y, *dYf, *dZ1f, *dZ2f, *part;
    float* part_k = nullptr;  // k-split partials of the weight gradients
    float* part_c = nullptr;  // row-slice partials of the bias gradients
};

namespace {

template <typename T>
int sur_alloc(lhmm_sur* s, T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess)
        return lhmm_fail(LHMM_ERR_OOM, "hipMalloc(%zu) failed", count * sizeof(T));
    s->bufs.push_back(q);
    *p = (T*)q;
    return LHMM_OK;
}

void sur_release(lhmm_sur* s) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void* b : s->bufs) (void)hipFree(b);
    s->bufs.clear();
}

constexpr int KCHUNK = 512;  // k-split chunk of the weight-gradient products

template <int EPI>
void launch_gemm(lhmm_sur* s, const Gemm& g, int zdim) {
    if (g.N % 128 == 0) {
        k_gemm_nt<EPI, 4><<<dim3(g.N / 128, g.M / 32, zdim), 64, 0, s->stream>>>(g);
    } else if (g.N % 64 == 0) {
        k_gemm_nt<EPI, 2><<<dim3(g.N / 64, g.M / 32, zdim), 64, 0, s->stream>>>(g);
    } else {
        k_gemm_nt<EPI, 1><<<dim3(g.N / 32, g.M / 32, zdim), 64, 0, s->stream>>>(g);
    }
}

template <int EPI>
void gemm(lhmm_sur* s, Gemm g) {
    g.ksplit = 1;
    g.kchunk = g.K;
    if (EPI == EPI_F32 && g.K >= 2 * KCHUNK && s->part_k) {
        // weight gradients (K = batch): k-chunks in parallel, then a fixed-order sum
        const int ks = (g.K + KCHUNK - 1) / KCHUNK;
        float* out = g.Cf;
        const long ostride = g.sC;
        g.ksplit = ks;
        g.kchunk = KCHUNK;
        g.Cf = s->part_k;
        g.sC = (long)g.M * g.N;
        launch_gemm<EPI>(s, g, s->E * ks);
        const long n = (long)s->E * g.M * g.N;
        k_splitk_sum<<<(n + 255) / 256, 256, 0, s->stream>>>(s->part_k, ks, (long)g.M * g.N, s->E, out, ostride);
        return;
    }
    launch_gemm<EPI>(s, g, s->E);
}

// bias gradients: out[e][c] = sum over the rows of x[e] (both passes on the stream)
void colsum(lhmm_sur* s, const float* x, int rows, int cols, long stride, float* out, long ostride) {
    k_colsum_part<<<dim3((cols + 63) / 64, s->E, COLSUM_SLICES), dim3(64, 16), 0, s->stream>>>(x, rows, cols, stride,
                                                                                              s->part_c);
    const long n = (long)s->E * cols;
    k_colsum_final<<<(unsigned)((n + 255) / 256), 256, 0, s->stream>>>(s->part_c, cols, s->E, out, ostride);
}

long szW1(const lhmm_sur* s) { return (long)s->nin_p * s->nh; }
long szW2(const lhmm_sur* s) { return (long)s->nh * s->nh; }
long szW3(const lhmm_sur* s) { return (long)s->nh * s->nout_p; }

// Activations of a forward pass: padded BF16 inputs X [Bp x nin_p], per
// member the BF16 hidden activations H1, H2 (member stride sh), their FP32
// pre-activations Z1, Z2 and transposes H1t, H2t (training only, else
// null), and the FP32 outputs Y (member stride sy).
struct Act {
    bf16 *X, *H1, *H1t, *H2, *H2t;
    float *Z1, *Z2, *Y;
    long sh, sy;
};

Act engine_act(const lhmm_sur* s, bool train) {
    Act a{};
    a.X = s->X;
    a.H1 = s->H1;
    a.H2 = s->H2;
    if (train) {
        a.H1t = s->H1t;
        a.H2t = s->H2t;
        a.Z1 = s->Z1;
        a.Z2 = s->Z2;
    }
    a.Y = s->Y;
    a.sh = (long)s->Bmax * s->nh;
    a.sy = (long)s->Bmax * s->nout_p;
    return a;
}

// forward of every member on the first Bp rows of act.X; with the
// pre-activations and transposed activations set (training) they are kept
// for backward
void forward(lhmm_sur* s, int Bp, const Act& act) {
    const bool train = act.Z1 != nullptr;
    Gemm g{};
    // layer 1: Z1 = X W1 + b1
    g.A = act.X; g.lda = s->nin_p; g.sA = 0;
    g.B = s->W1t; g.ldb = s->nin_p; g.sB = szW1(s);
    g.M = Bp; g.N = s->nh; g.K = s->nin_p;
    g.bias = s->b1; g.sBias = s->nh;
    g.Cf = train ? act.Z1 : nullptr; g.Cb = act.H1; g.Ct = act.H1t; g.ldt = Bp; g.sC = act.sh;
    g.sCt = act.sh;
    gemm<EPI_BIAS_GELU>(s, g);
    // layer 2
    g.A = act.H1; g.lda = s->nh; g.sA = act.sh;
    g.B = s->W2t; g.ldb = s->nh; g.sB = szW2(s);
    g.M = Bp; g.N = s->nh; g.K = s->nh;
    g.bias = s->b2; g.sBias = s->nh;
    g.Cf = train ? act.Z2 : nullptr; g.Cb = act.H2; g.Ct = act.H2t; g.ldt = Bp;
    gemm<EPI_BIAS_GELU>(s, g);
    // layer 3: Y = H2 W3 + b3
    g.A = act.H2; g.lda = s->nh; g.sA = act.sh;
    g.B = s->W3t; g.ldb = s->nh; g.sB = szW3(s);
    g.M = Bp; g.N = s->nout_p; g.K = s->nh;
    g.bias = s->b3; g.sBias = s->nout_p;
    g.Cf = act.Y; g.sC = act.sy; g.Cb = nullptr; g.Ct = nullptr;
    gemm<EPI_BIAS_F32>(s, g);
}

constexpr size_t SUR_SCRATCH_BYTES = size_t(32) << 20;  // see `scratch` below

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// bytes of scratch a forward pass of Bp padded rows needs
size_t static_scratch_bytes(const lhmm_sur* s, int Bp) {
    return align256((size_t)Bp * s->nin_p * sizeof(bf16)) + 2 * align256((size_t)s->E * Bp * s->nh * sizeof(bf16)) +
           align256((size_t)s->E * Bp * s->nout_p * sizeof(float));
}

int check_dims(const lhmm_sur_params* p) {
    if (p->n_members < 1 || p->n_members > 64) return lhmm_fail(LHMM_ERR_ARG, "n_members must be 1..64");
    if (p->n_in < 1 || p->n_out < 1 || p->n_out > 32) return lhmm_fail(LHMM_ERR_ARG, "need n_in >= 1, 1 <= n_out <= 32");
    if (p->n_hidden < 32 || p->n_hidden % 32) return lhmm_fail(LHMM_ERR_ARG, "n_hidden must be a positive multiple of 32");
    if (p->max_batch < 1) return lhmm_fail(LHMM_ERR_ARG, "max_batch must be positive");
    return LHMM_OK;
}

}  // namespace

// Scratch of lhmm_sur_forward_static: the activations of one forward pass
// (padded inputs, both hidden layers of every member, outputs) in a
// file-scope device array instead of engine buffers.  Each device holds its
// own copy at its own address until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns on that device (the
// array's name on the host is a stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[SUR_SCRATCH_BYTES];

hipStream_t lhmm_sur_caller_stream(const lhmm_sur* s) { return s->stream; }

void lhmm_sur_dims(const lhmm_sur* s, int* n_members, int* n_in, int* n_out, int* max_batch) {
    *n_members = s->E;
    *n_in = s->nin;
    *n_out = s->nout;
    *max_batch = s->Bmax;
}

extern "C" {

int lhmm_sur_create(const lhmm_sur_params* p, const float* weights, void* stream, lhmm_sur** out) {
    lhmm_clear_error();
    if (!p || !weights || !out) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    *out = nullptr;
    int rc = check_dims(p);
    if (rc != LHMM_OK) return rc;
    lhmm_sur* s = new (std::nothrow) lhmm_sur();
    if (!s) return lhmm_fail(LHMM_ERR_OOM, "host allocation failed");
    s->E = p->n_members;
    s->nin = p->n_in;
    s->nin_p = round_up(p->n_in, 32);
    s->nh = p->n_hidden;
    s->nout = p->n_out;
    s->Bmax = round_up(p->max_batch, 32);
    s->stream = (hipStream_t)stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return lhmm_fail(LHMM_ERR_HIP, "hipGetDevice failed");
    }
    const long E = s->E, w1 = szW1(s), w2 = szW2(s), w3 = szW3(s), nh = s->nh, no = s->nout_p;
    const long Bm = s->Bmax;
    float** f32s[] = {&s->W1, &s->gW1, &s->mW1, &s->vW1};
    for (float** q : f32s) rc = rc ? rc : sur_alloc(s, q, E * w1);
    float** f32h[] = {&s->b1, &s->gb1, &s->mb1, &s->vb1, &s->b2, &s->gb2, &s->mb2, &s->vb2};
    for (float** q : f32h) rc = rc ? rc : sur_alloc(s, q, E * nh);
    float** f32w2[] = {&s->W2, &s->gW2, &s->mW2, &s->vW2};
    for (float** q : f32w2) rc = rc ? rc : sur_alloc(s, q, E * w2);
    float** f32w3[] = {&s->W3, &s->gW3, &s->mW3, &s->vW3};
    for (float** q : f32w3) rc = rc ? rc : sur_alloc(s, q, E * w3);
    float** f32b3[] = {&s->b3, &s->gb3, &s->mb3, &s->vb3};
    for (float** q : f32b3) rc = rc ? rc : sur_alloc(s, q, E * no);
    bf16** wb[] = {&s->W1b, &s->W1t};
    for (bf16** q : wb) rc = rc ? rc : sur_alloc(s, q, E * w1);
    bf16** wb2[] = {&s->W2b, &s->W2t};
    for (bf16** q : wb2) rc = rc ? rc : sur_alloc(s, q, E * w2);
    bf16** wb3[] = {&s->W3b, &s->W3t};
    for (bf16** q : wb3) rc = rc ? rc : sur_alloc(s, q, E * w3);
    rc = rc ? rc : sur_alloc(s, &s->X, Bm * s->nin_p);
    rc = rc ? rc : sur_alloc(s, &s->Xt, Bm * s->nin_p);
    bf16** acts[] = {&s->H1, &s->H1t, &s->H2, &s->H2t, &s->dZ2, &s->dZ2t, &s->dZ1, &s->dZ1t};
    for (bf16** q : acts) rc = rc ? rc : sur_alloc(s, q, E * Bm * nh);
    float** actf[] = {&s->Z1, &s->Z2, &s->dZ1f, &s->dZ2f};
    for (float** q : actf) rc = rc ? rc : sur_alloc(s, q, E * Bm * nh);
    rc = rc ? rc : sur_alloc(s, &s->Y, E * Bm * no);
    rc = rc ? rc : sur_alloc(s, &s->dYf, E * Bm * no);
    rc = rc ? rc : sur_alloc(s, &s->dY, E * Bm * no);
    rc = rc ? rc : sur_alloc(s, &s->dYt, E * Bm * no);
    rc = rc ? rc : sur_alloc(s, &s->part, E * (Bm * no / 256 + 1));
    rc = rc ? rc : sur_alloc(s, &s->part_c, (size_t)E * COLSUM_SLICES * std::max(nh, no));
    if (Bm >= 2 * KCHUNK) {
        const long mn = std::max(std::max(w1, w2), w3);
        rc = rc ? rc : sur_alloc(s, &s->part_k, E * ((Bm + KCHUNK - 1) / KCHUNK) * mn);
    }
    if (rc == LHMM_OK) rc = lhmm_sur_set_weights(s, weights);
    if (rc != LHMM_OK) {
        sur_release(s);
        delete s;
        return rc;
    }
    *out = s;
    return LHMM_OK;
}

int lhmm_sur_set_weights(lhmm_sur* s, const float* weights) {
    lhmm_clear_error();
    if (!s || !weights) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    const int E = s->E, nin = s->nin, nin_p = s->nin_p, nh = s->nh, nout = s->nout, no = s->nout_p;
    const long w1 = szW1(s), w2 = szW2(s), w3 = szW3(s);
    std::vector<float> W1((size_t)E * w1, 0.f), W2((size_t)E * w2, 0.f), W3((size_t)E * w3, 0.f);
    std::vector<float> B1((size_t)E * nh, 0.f), B2((size_t)E * nh, 0.f), B3((size_t)E * no, 0.f);
    const float* q = weights;
    for (int e = 0; e < E; ++e) {
        for (int i = 0; i < nin; ++i)
            for (int j = 0; j < nh; ++j) W1[e * w1 + (long)i * nh + j] = *q++;
        for (int j = 0; j < nh; ++j) B1[(size_t)e * nh + j] = *q++;
        for (int i = 0; i < nh; ++i)
            for (int j = 0; j < nh; ++j) W2[e * w2 + (long)i * nh + j] = *q++;
        for (int j = 0; j < nh; ++j) B2[(size_t)e * nh + j] = *q++;
        for (int i = 0; i < nh; ++i)
            for (int j = 0; j < nout; ++j) W3[e * w3 + (long)i * no + j] = *q++;
        for (int j = 0; j < nout; ++j) B3[(size_t)e * no + j] = *q++;
    }
    const long total = (long)E * ((long)nin * nh + nh + (long)nh * nh + nh + (long)nh * nout + nout);
    for (long i = 0; i < total; ++i)
        if (!std::isfinite(weights[i])) return lhmm_fail(LHMM_ERR_ARG, "non-finite weight %ld", i);
    LHMM_HIPCHK(hipStreamSynchronize(s->stream));
    LHMM_HIPCHK(hipMemcpy(s->W1, W1.data(), W1.size() * 4, hipMemcpyHostToDevice));
    LHMM_HIPCHK(hipMemcpy(s->W2, W2.data(), W2.size() * 4, hipMemcpyHostToDevice));
    LHMM_HIPCHK(hipMemcpy(s->W3, W3.data(), W3.size() * 4, hipMemcpyHostToDevice));
    LHMM_HIPCHK(hipMemcpy(s->b1, B1.data(), B1.size() * 4, hipMemcpyHostToDevice));
    LHMM_HIPCHK(hipMemcpy(s->b2, B2.data(), B2.size() * 4, hipMemcpyHostToDevice));
    LHMM_HIPCHK(hipMemcpy(s->b3, B3.data(), B3.size() * 4, hipMemcpyHostToDevice));
    float* zero[] = {s->mW1, s->vW1, s->mW2, s->vW2, s->mW3, s->vW3, s->mb1, s->vb1, s->mb2, s->vb2, s->mb3, s->vb3,
                     s->gW1, s->gW2, s->gW3, s->gb1, s->gb2, s->gb3};
    const long zs[] = {w1, w1, w2, w2, w3, w3, nh, nh, nh, nh, no, no, w1, w2, w3, nh, nh, no};
    for (int k = 0; k < 18; ++k) LHMM_HIPCHK(hipMemset(zero[k], 0, (size_t)E * zs[k] * 4));
    // BF16 copies: an Adam step with zero learning rate and zero gradient
    // leaves the masters unchanged and writes both layouts
    const int t = 256;
    k_adam<<<(E * w1 + t - 1) / t, t, 0, s->stream>>>(s->W1, s->gW1, s->mW1, s->vW1, nin_p, nh, w1, E, 0.f, 1.f, 1.f,
                                                     s->W1b, s->W1t);
    k_adam<<<(E * w2 + t - 1) / t, t, 0, s->stream>>>(s->W2, s->gW2, s->mW2, s->vW2, nh, nh, w2, E, 0.f, 1.f, 1.f,
                                                     s->W2b, s->W2t);
    k_adam<<<(E * w3 + t - 1) / t, t, 0, s->stream>>>(s->W3, s->gW3, s->mW3, s->vW3, nh, no, w3, E, 0.f, 1.f, 1.f,
                                                     s->W3b, s->W3t);
    LHMM_HIPCHK(hipGetLastError());
    LHMM_HIPCHK(hipStreamSynchronize(s->stream));
    s->step = 0;
    return LHMM_OK;
}

}  // extern "C"

namespace {

// device FP32 tensors of one kind (masters or gradients) -> packed host layout
int copy_packed(lhmm_sur* s, bool grads, float* out) {
    const int E = s->E, nin = s->nin, nh = s->nh, nout = s->nout, no = s->nout_p;
    const long w1 = szW1(s), w2 = szW2(s), w3 = szW3(s);
    std::vector<float> W1((size_t)E * w1), W2((size_t)E * w2), W3((size_t)E * w3), B1((size_t)E * nh),
        B2((size_t)E * nh), B3((size_t)E * no);
    const float* src[6] = {grads ? s->gW1 : s->W1, grads ? s->gb1 : s->b1, grads ? s->gW2 : s->W2,
                           grads ? s->gb2 : s->b2, grads ? s->gW3 : s->W3, grads ? s->gb3 : s->b3};
    std::vector<float>* dst[6] = {&W1, &B1, &W2, &B2, &W3, &B3};
    LHMM_HIPCHK(hipStreamSynchronize(s->stream));
    for (int k = 0; k < 6; ++k)
        LHMM_HIPCHK(hipMemcpy(dst[k]->data(), src[k], dst[k]->size() * 4, hipMemcpyDeviceToHost));
    float* q = out;
    for (int e = 0; e < E; ++e) {
        for (int i = 0; i < nin; ++i)
            for (int j = 0; j < nh; ++j) *q++ = W1[e * w1 + (long)i * nh + j];
        for (int j = 0; j < nh; ++j) *q++ = B1[(size_t)e * nh + j];
        for (int i = 0; i < nh; ++i)
            for (int j = 0; j < nh; ++j) *q++ = W2[e * w2 + (long)i * nh + j];
        for (int j = 0; j < nh; ++j) *q++ = B2[(size_t)e * nh + j];
        for (int i = 0; i < nh; ++i)
            for (int j = 0; j < nout; ++j) *q++ = W3[e * w3 + (long)i * no + j];
        for (int j = 0; j < nout; ++j) *q++ = B3[(size_t)e * no + j];
    }
    return LHMM_OK;
}

}  // namespace

extern "C" {

int lhmm_sur_get_weights(lhmm_sur* s, float* weights) {
    lhmm_clear_error();
    if (!s || !weights) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    return copy_packed(s, false, weights);
}

int lhmm_sur_get_grads(lhmm_sur* s, float* grads) {
    lhmm_clear_error();
    if (!s || !grads) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    return copy_packed(s, true, grads);
}

// B rows of f32 features (device, B x n_in) into the padded BF16 inputs
// (and their transpose, for training)
static int load_inputs(lhmm_sur* s, const float* X, int B, int Bp, bf16* Xp, bf16* Xt) {
    const long n = (long)Bp * s->nin_p;
    k_inputs<<<(n + 255) / 256, 256, 0, s->stream>>>(X, B, s->nin, Bp, s->nin_p, Xp, Xt);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_train_step(lhmm_sur* s, const float* X, const float* T, int32_t B, float lr, float* loss) {
    lhmm_clear_error();
    if (!s || !X || !T) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    if (B < 1 || B > s->Bmax) return lhmm_fail(LHMM_ERR_ARG, "batch %d outside 1..%d", B, s->Bmax);
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return lhmm_fail(LHMM_ERR_ARG, "bad learning rate");
    const int Bp = round_up(B, 32), E = s->E, nh = s->nh, no = s->nout_p;
    const long Bm = s->Bmax;
    int rc = load_inputs(s, X, B, Bp, s->X, s->Xt);
    if (rc != LHMM_OK) return rc;
    forward(s, Bp, engine_act(s, true));
    // dY and loss
    const long nY = (long)Bp * no;
    const int nparts = (int)((nY + 255) / 256);
    // dY, dY^T and the f32 dY use member stride Bp x n_out_p
    k_loss_grad<<<dim3(nparts, E), 256, 0, s->stream>>>(s->Y, Bm * no, T, B, Bp, s->nout, no, s->dY, s->dYt, s->dYf,
                                                        s->part);
    Gemm g{};
    // dW3 = H2^T dY : A = H2t [nh x Bp], B = dYt [no x Bp]
    g.A = s->H2t; g.lda = Bp; g.sA = Bm * nh;
    g.B = s->dYt; g.ldb = Bp; g.sB = (long)no * Bp;
    g.M = nh; g.N = no; g.K = Bp;
    g.Cf = s->gW3; g.sC = szW3(s);
    gemm<EPI_F32>(s, g);
    // dZ2 = (dY W3^T) * gelu'(Z2): A = dY [Bp x no], B = W3b [nh x no]
    g = Gemm{};
    g.A = s->dY; g.lda = no; g.sA = (long)Bp * no;
    g.B = s->W3b; g.ldb = no; g.sB = szW3(s);
    g.M = Bp; g.N = nh; g.K = no;
    g.Zin = s->Z2; g.Cf = s->dZ2f; g.Cb = s->dZ2; g.Ct = s->dZ2t; g.ldt = Bp; g.sC = Bm * nh; g.sCt = Bm * nh;
    gemm<EPI_GELU_GRAD>(s, g);
    // dW2 = H1^T dZ2 : A = H1t [nh x Bp], B = dZ2t [nh x Bp]
    g = Gemm{};
    g.A = s->H1t; g.lda = Bp; g.sA = Bm * nh;
    g.B = s->dZ2t; g.ldb = Bp; g.sB = Bm * nh;
    g.M = nh; g.N = nh; g.K = Bp;
    g.Cf = s->gW2; g.sC = szW2(s);
    gemm<EPI_F32>(s, g);
    // dZ1 = (dZ2 W2^T) * gelu'(Z1): A = dZ2 [Bp x nh], B = W2b [nh x nh]
    g = Gemm{};
    g.A = s->dZ2; g.lda = nh; g.sA = Bm * nh;
    g.B = s->W2b; g.ldb = nh; g.sB = szW2(s);
    g.M = Bp; g.N = nh; g.K = nh;
    g.Zin = s->Z1; g.Cf = s->dZ1f; g.Cb = s->dZ1; g.Ct = s->dZ1t; g.ldt = Bp; g.sC = Bm * nh; g.sCt = Bm * nh;
    gemm<EPI_GELU_GRAD>(s, g);
    // dW1 = X^T dZ1 : A = Xt [nin_p x Bp], B = dZ1t [nh x Bp]
    g = Gemm{};
    g.A = s->Xt; g.lda = Bp; g.sA = 0;
    g.B = s->dZ1t; g.ldb = Bp; g.sB = Bm * nh;
    g.M = s->nin_p; g.N = nh; g.K = Bp;
    g.Cf = s->gW1; g.sC = szW1(s);
    gemm<EPI_F32>(s, g);
    // bias gradients
    colsum(s, s->dYf, Bp, no, (long)Bp * no, s->gb3, no);
    colsum(s, s->dZ2f, Bp, nh, Bm * nh, s->gb2, nh);
    colsum(s, s->dZ1f, Bp, nh, Bm * nh, s->gb1, nh);
    // Adam
    s->step += 1;
    const float c1 = 1.0f - powf(0.9f, (float)s->step), c2 = 1.0f - powf(0.999f, (float)s->step);
    const int t = 256;
    const long w1 = szW1(s), w2 = szW2(s), w3 = szW3(s);
    k_adam<<<(E * w1 + t - 1) / t, t, 0, s->stream>>>(s->W1, s->gW1, s->mW1, s->vW1, s->nin_p, nh, w1, E, lr, c1, c2,
                                                     s->W1b, s->W1t);
    k_adam<<<(E * w2 + t - 1) / t, t, 0, s->stream>>>(s->W2, s->gW2, s->mW2, s->vW2, nh, nh, w2, E, lr, c1, c2,
                                                     s->W2b, s->W2t);
    k_adam<<<(E * w3 + t - 1) / t, t, 0, s->stream>>>(s->W3, s->gW3, s->mW3, s->vW3, nh, no, w3, E, lr, c1, c2,
                                                     s->W3b, s->W3t);
    k_adam<<<(E * nh + t - 1) / t, t, 0, s->stream>>>(s->b1, s->gb1, s->mb1, s->vb1, 1, nh, nh, E, lr, c1, c2,
                                                     nullptr, nullptr);
    k_adam<<<(E * nh + t - 1) / t, t, 0, s->stream>>>(s->b2, s->gb2, s->mb2, s->vb2, 1, nh, nh, E, lr, c1, c2,
                                                     nullptr, nullptr);
    k_adam<<<(E * no + t - 1) / t, t, 0, s->stream>>>(s->b3, s->gb3, s->mb3, s->vb3, 1, no, no, E, lr, c1, c2,
                                                     nullptr, nullptr);
    if (loss) k_loss_final<<<E, 64, 0, s->stream>>>(s->part, nparts, B, s->nout, loss);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_forward(lhmm_sur* s, const float* X, int32_t B, float* Y) {
    lhmm_clear_error();
    if (!s || !X || !Y) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    if (B < 1 || B > s->Bmax) return lhmm_fail(LHMM_ERR_ARG, "batch %d outside 1..%d", B, s->Bmax);
    const int Bp = round_up(B, 32);
    int rc = load_inputs(s, X, B, Bp, s->X, nullptr);
    if (rc != LHMM_OK) return rc;
    const Act act = engine_act(s, false);
    forward(s, Bp, act);
    const long n = (long)s->E * B * s->nout;
    k_outputs<<<(n + 255) / 256, 256, 0, s->stream>>>(act.Y, act.sy, s->nout_p, s->E, B, s->nout, Y);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_forward_static(lhmm_sur* s, const float* X, int32_t B, float* Y) {
    lhmm_clear_error();
    if (!s || !X || !Y) return lhmm_fail(LHMM_ERR_ARG, "null argument");
    if (B < 1) return lhmm_fail(LHMM_ERR_ARG, "batch %d must be positive", B);
    const int Bp = round_up(B, 32);
    const size_t need = static_scratch_bytes(s, Bp);
    if (need > SUR_SCRATCH_BYTES)
        return lhmm_fail(LHMM_ERR_ARG, "batch %d needs %zu bytes of scratch, more than the %zu this entry point holds",
                         B, need, SUR_SCRATCH_BYTES);
    int dev = -1;
    LHMM_HIPCHK(hipGetDevice(&dev));
    if (dev != s->device) return lhmm_fail(LHMM_ERR_ARG, "call with the engine's device %d current (got %d)", s->device, dev);
    if (dev < 0 || dev >= MAX_DEVICES) return lhmm_fail(LHMM_ERR_ARG, "device %d beyond the %d supported", dev, MAX_DEVICES);
    unsigned char* base = nullptr;
    {
        // the scratch's device address, looked up once per device (with that device current)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* ptr = nullptr;
            LHMM_HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return lhmm_fail(LHMM_ERR_HIP, "hipGetSymbolAddress returned no address");
            g_scratch_ptr[dev] = ptr;
        }
        base = (unsigned char*)g_scratch_ptr[dev];
    }
    Act act{};
    size_t off = 0;
    act.X = (bf16*)(base + off);
    off += align256((size_t)Bp * s->nin_p * sizeof(bf16));
    act.H1 = (bf16*)(base + off);
    off += align256((size_t)s->E * Bp * s->nh * sizeof(bf16));
    act.H2 = (bf16*)(base + off);
    off += align256((size_t)s->E * Bp * s->nh * sizeof(bf16));
    act.Y = (float*)(base + off);
    act.sh = (long)Bp * s->nh;
    act.sy = (long)Bp * s->nout_p;
    // every scratch word the pass reads is written by it first (inputs and
    // their zero padding, then each layer), so nothing needs clearing
    int rc = load_inputs(s, X, B, Bp, act.X, nullptr);
    if (rc != LHMM_OK) return rc;
    forward(s, Bp, act);
    const long n = (long)s->E * B * s->nout;
    k_outputs<<<(n + 255) / 256, 256, 0, s->stream>>>(act.Y, act.sy, s->nout_p, s->E, B, s->nout, Y);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_push_history(float* ring, int32_t n, const double* gradL, int64_t t, float scale, void* stream) {
    lhmm_clear_error();
    if (!ring || !gradL || n < 1 || t < 0 || !std::isfinite(scale)) return lhmm_fail(LHMM_ERR_ARG, "bad history arguments");
    k_push_history<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(ring, n, gradL, t, scale);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_features(const float* ring, int32_t n, int64_t t, const float* phi, float* X, void* stream) {
    lhmm_clear_error();
    if (!ring || !phi || !X || n < 1 || t < 0) return lhmm_fail(LHMM_ERR_ARG, "bad feature arguments");
    const long total = (long)n * (4 * HIST + 1);
    k_features<<<(total + 255) / 256, 256, 0, (hipStream_t)stream>>>(ring, n, t, phi, X);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_gate(const float* Y, int32_t n_members, int32_t B, int32_t n_out, float threshold, float floor_,
                  float* mean, uint32_t* flag, void* stream) {
    lhmm_clear_error();
    if (!Y || !mean || !flag || n_members < 1 || B < 1 || n_out < 1) return lhmm_fail(LHMM_ERR_ARG, "bad gate arguments");
    k_gate<<<(B + 255) / 256, 256, 0, (hipStream_t)stream>>>(Y, n_members, B, B, n_out, n_out, threshold, floor_,
                                                           mean, flag);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_targets(const double* sigma, int32_t n, float inv_scale, float* T, void* stream) {
    lhmm_clear_error();
    if (!sigma || !T || n < 1) return lhmm_fail(LHMM_ERR_ARG, "bad target arguments");
    k_targets<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(sigma, n, inv_scale, T);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_blend(const float* mean, const uint32_t* use_dpd, const double* sigma_dpd, int32_t n, float scale,
                   double* sigma_out, void* stream) {
    lhmm_clear_error();
    if (!mean || !sigma_out || n < 1 || (use_dpd && !sigma_dpd)) return lhmm_fail(LHMM_ERR_ARG, "bad blend arguments");
    k_blend<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(mean, use_dpd, sigma_dpd, n, scale, sigma_out);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_history_gradient(const float* ring, int32_t n, int64_t t, float inv_scale, double* gradL, void* stream) {
    lhmm_clear_error();
    if (!ring || !gradL || n < 1 || t < 0) return lhmm_fail(LHMM_ERR_ARG, "bad history arguments");
    k_ring_to_grad<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(ring, n, t, inv_scale, gradL);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_augment(float* X, float* T, int32_t n, const float* theta, const uint32_t* mirror, void* stream) {
    lhmm_clear_error();
    if (!X || !T || !theta || !mirror || n < 1) return lhmm_fail(LHMM_ERR_ARG, "bad augment arguments");
    k_augment<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(X, T, n, theta, mirror);
    LHMM_HIPCHK(hipGetLastError());
    return LHMM_OK;
}

int lhmm_sur_destroy(lhmm_sur* s) {
    lhmm_clear_error();
    if (!s) return LHMM_OK;
    sur_release(s);
    delete s;
    return LHMM_OK;
}

}  // extern "C"
