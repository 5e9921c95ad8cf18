// Learned impedance model on gfx950: MLP 13 -> 64 -> 64 -> 1 (ReLU), BF16
// operands on the matrix cores (v_mfma_f32_16x16x16_bf16), FP32 accumulation,
// FP32 master weights and Adam.
//
// Parameter blob (FP32), kParams floats:
//   mu[13], sigma[13]          input standardisation (not trained)
//   W1[64][13], b1[64], W2[64][64], b2[64], w3[64], b3[1]
// Gradients use the same layout without mu/sigma (kTrain floats).
//
// Rounding points (the CPU check follows them): standardised inputs, W1, W2,
// the post-ReLU first hidden layer, and the back-propagated dH2 and dH1 are
// rounded to BF16 (round to nearest even) where they enter an MFMA; the second
// hidden layer and the output layer stay in FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.hpp"

namespace vtm {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int F = kNumFeatures;  // 13 inputs, padded to 16 on the matrix cores
constexpr int H = 64;
constexpr int kWaves = 4;

__device__ inline short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ inline float bf2f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights staged in LDS as BF16: W1b[64][16] (K padded), W2b[64][64]; FP32 b1, b2, w3, mu, 1/sigma.
struct Smem {
    short W1b[H][16];
    short W2b[H][H];
    float b1[H], b2[H], w3[H], mu[16], isd[16];
    float b3;
    short T[kWaves][16][H];  // per-wave transpose buffer
};

__device__ void stage_weights(const float *__restrict__ P, Smem &s) {
    const float *mu = P, *sd = P + F, *W1 = P + 2 * F, *b1 = W1 + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H;
    for (int i = threadIdx.x; i < H * 16; i += blockDim.x) {
        const int o = i / 16, k = i % 16;
        s.W1b[o][k] = k < F ? f2bf(W1[o * F + k]) : (short)0;
    }
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) s.W2b[i / H][i % H] = f2bf(W2[i]);
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        s.b1[i] = b1[i];
        s.b2[i] = b2[i];
        s.w3[i] = w3[i];
    }
    for (int i = threadIdx.x; i < 16; i += blockDim.x) {
        s.mu[i] = i < F ? mu[i] : 0.f;
        s.isd[i] = i < F ? 1.f / sd[i] : 0.f;
    }
    if (threadIdx.x == 0) s.b3 = w3[H];
    __syncthreads();
}

// Forward pass of 16 rows by one wave.  Lane l = 16*kb + c holds, in the MFMA
// output layout, rows 4*kb + j (j < 4) of columns 16*t + c of each hidden layer.
struct Fwd {
    bf16x4 h1[4];   // BF16 first hidden layer (post-ReLU), per column tile t
    f32x4 h2[4];    // FP32 second hidden layer (post-ReLU)
    float y[4];     // outputs of rows 4*kb + j
};

__device__ inline float xin(const float *__restrict__ X, int64_t row, bool ok, int k, const Smem &s) {
    return (ok && k < F) ? (X[row * F + k] - s.mu[k]) * s.isd[k] : 0.f;
}

// Rows r0 .. r0+15 of a batch: through an index list, or contiguous from row0.
struct Rows {
    const int64_t *idx;
    int64_t row0, r0, n;
    __device__ bool ok(int i) const { return r0 + i < n; }
    __device__ int64_t at(int i) const { return ok(i) ? (idx ? idx[r0 + i] : row0 + r0 + i) : 0; }
};

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ void forward16(const float *__restrict__ X, const Rows &R, Smem &s, int w, Fwd &o) {
    const int l = threadIdx.x & 63, c = l & 15, kb = l >> 4;
    // layer 1: A = standardised inputs (row c, k = 4kb + j)
    bf16x4 a;
    {
        const bool ok = R.ok(c);
        const int64_t r = R.at(c);
        for (int j = 0; j < 4; ++j) a[j] = f2bf(xin(X, r, ok, 4 * kb + j, s));
    }
    for (int t = 0; t < 4; ++t) {
        bf16x4 bw;
        for (int j = 0; j < 4; ++j) bw[j] = s.W1b[16 * t + c][4 * kb + j];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(a, bw, acc);
        for (int j = 0; j < 4; ++j) {
            const float h = fmaxf(acc[j] + s.b1[16 * t + c], 0.f);
            o.h1[t][j] = f2bf(h);
            s.T[w][4 * kb + j][16 * t + c] = o.h1[t][j];
        }
    }
    wave_sync();
    // layer 2: A = H1 rows (row c, k = 16 ks + 4 kb + j) from the transpose buffer
    f32x4 acc2[4];
    for (int t = 0; t < 4; ++t) acc2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < 4; ++ks) {
        bf16x4 ah;
        for (int j = 0; j < 4; ++j) ah[j] = s.T[w][c][16 * ks + 4 * kb + j];
        for (int t = 0; t < 4; ++t) {
            bf16x4 bw;
            for (int j = 0; j < 4; ++j) bw[j] = s.W2b[16 * t + c][16 * ks + 4 * kb + j];
            acc2[t] = mfma(ah, bw, acc2[t]);
        }
    }
    wave_sync();
    float part[4] = {0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 4; ++t)
        for (int j = 0; j < 4; ++j) {
            const float h = fmaxf(acc2[t][j] + s.b2[16 * t + c], 0.f);
            o.h2[t][j] = h;
            part[j] += h * s.w3[16 * t + c];
        }
    // layer 3: sum over the 16 lanes that share kb
    for (int j = 0; j < 4; ++j) {
        float v = part[j];
        for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
        o.y[j] = v + s.b3;
    }
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *__restrict__ P, const float *__restrict__ X, int64_t n,
                                                     float *__restrict__ y) {
    __shared__ Smem s;
    stage_weights(P, s);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, kb = l >> 4, c = l & 15;
    for (int64_t r0 = ((int64_t)blockIdx.x * kWaves + w) * 16; r0 < n; r0 += (int64_t)gridDim.x * kWaves * 16) {
        const Rows R{nullptr, 0, r0, n};
        Fwd o;
        forward16(X, R, s, w, o);
        if (c == 0)
            for (int j = 0; j < 4; ++j)
                if (r0 + 4 * kb + j < n) y[r0 + 4 * kb + j] = o.y[j];
    }
}

// Impedance per VTL from the prediction: Z = exp(clamp(y, lo, hi)) / a_vv.
__global__ void k_z_from_pred(const float *__restrict__ y, const double *__restrict__ avv, int64_t n, double lo, double hi,
                              double *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = (double)y[i];
    d = d < lo ? lo : (d > hi ? hi : d);
    z[i] = exp(d) / avv[i];
}

// Gradient of the mean squared error over rows idx[0..n) (or row0 + i), partial per workgroup.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                  const float *__restrict__ Y, const int64_t *__restrict__ idx,
                                                  int64_t row0, int64_t n, float scale, float *__restrict__ part) {
    __shared__ Smem s;
    __shared__ float red[kTrain + 1];
    stage_weights(P, s);
    for (int i = threadIdx.x; i < kTrain + 1; i += blockDim.x) red[i] = 0.f;
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, kb = l >> 4, c = l & 15;
    f32x4 gW2[4][4], gW1[4];
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gw3[4] = {0.f, 0.f, 0.f, 0.f};
    float gb3 = 0.f, loss = 0.f;
    for (int64_t r0 = ((int64_t)blockIdx.x * kWaves + w) * 16; r0 < n; r0 += (int64_t)gridDim.x * kWaves * 16) {
        const Rows R{idx, row0, r0, n};
        Fwd o;
        forward16(X, R, s, w, o);
        // output error
        float dy[4];
        for (int j = 0; j < 4; ++j) {
            const int r = 4 * kb + j;
            const bool ok = R.ok(r);
            const float e = ok ? o.y[j] - Y[R.at(r)] : 0.f;
            dy[j] = scale * 2.f * e;
            if (c == 0) { loss += e * e; gb3 += dy[j]; }
        }
        // layer 3 and the second hidden layer's gradient (FP32, then BF16 for the MFMAs)
        bf16x4 dh2[4];
        for (int t = 0; t < 4; ++t) {
            const float w3 = s.w3[16 * t + c];
            for (int j = 0; j < 4; ++j) {
                gw3[t] += dy[j] * o.h2[t][j];
                const float g = o.h2[t][j] > 0.f ? dy[j] * w3 : 0.f;
                gb2[t] += g;
                dh2[t][j] = f2bf(g);
                s.T[w][4 * kb + j][16 * t + c] = dh2[t][j];
            }
        }
        // dW2[o][i] += sum_r dH2[r][o] H1[r][i]
        for (int ot = 0; ot < 4; ++ot)
            for (int it = 0; it < 4; ++it) gW2[ot][it] = mfma(dh2[ot], o.h1[it], gW2[ot][it]);
        wave_sync();
        // dH1[r][i] = sum_o dH2[r][o] W2[o][i], masked by the first layer's ReLU
        f32x4 d1[4];
        for (int t = 0; t < 4; ++t) d1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 4; ++ks) {
            bf16x4 ad;
            for (int j = 0; j < 4; ++j) ad[j] = s.T[w][c][16 * ks + 4 * kb + j];
            for (int it = 0; it < 4; ++it) {
                bf16x4 bw;
                for (int j = 0; j < 4; ++j) bw[j] = s.W2b[16 * ks + 4 * kb + j][16 * it + c];
                d1[it] = mfma(ad, bw, d1[it]);
            }
        }
        wave_sync();
        bf16x4 dh1[4];
        for (int it = 0; it < 4; ++it)
            for (int j = 0; j < 4; ++j) {
                const float g = bf2f(o.h1[it][j]) > 0.f ? d1[it][j] : 0.f;
                gb1[it] += g;
                dh1[it][j] = f2bf(g);
            }
        // dW1[i][k] += sum_r dH1[r][i] Xhat[r][k]; B operand lane (kb, c): rows 4kb + j, feature c
        bf16x4 bx;
        for (int j = 0; j < 4; ++j) {
            const int r = 4 * kb + j;
            bx[j] = f2bf(xin(X, R.at(r), R.ok(r), c, s));
        }
        for (int it = 0; it < 4; ++it) gW1[it] = mfma(dh1[it], bx, gW1[it]);
    }
    // reduce the workgroup's waves into LDS (gradient layout: W1, b1, W2, b2, w3, b3), then one partial
    float *rW1 = red, *rb1 = rW1 + H * F, *rW2 = rb1 + H, *rb2 = rW2 + H * H, *rw3 = rb2 + H, *rb3 = rw3 + H;
    for (int ww = 0; ww < kWaves; ++ww) {
        if (w == ww) {
            for (int it = 0; it < 4; ++it)
                for (int j = 0; j < 4; ++j) {
                    const int o_ = 16 * it + 4 * kb + j;
                    if (c < F) rW1[o_ * F + c] += gW1[it][j];
                }
            for (int ot = 0; ot < 4; ++ot)
                for (int it = 0; it < 4; ++it)
                    for (int j = 0; j < 4; ++j) rW2[(16 * ot + 4 * kb + j) * H + 16 * it + c] += gW2[ot][it][j];
            for (int t = 0; t < 4; ++t) {
                atomicAdd(&rb1[16 * t + c], gb1[t]);
                atomicAdd(&rb2[16 * t + c], gb2[t]);
                atomicAdd(&rw3[16 * t + c], gw3[t]);
            }
            if (c == 0) {
                atomicAdd(rb3, gb3);
                atomicAdd(&red[kTrain], loss);
            }
        }
        __syncthreads();
    }
    float *out = part + (int64_t)blockIdx.x * (kTrain + 1);
    for (int i = threadIdx.x; i < kTrain + 1; i += blockDim.x) out[i] = red[i];
}

// Sum of the per-workgroup partials in a fixed order.
__global__ void k_sum_partials(const float *__restrict__ part, int nparts, float *__restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kTrain) return;
    float acc = 0.f;
    for (int p = 0; p < nparts; ++p) acc += part[(int64_t)p * (kTrain + 1) + i];
    g[i] = acc;
}

__global__ void k_adam(float *__restrict__ P, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kTrain) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[2 * F + i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

int mlp_grid(int64_t n) {
    int64_t b = (n + kWaves * 16 - 1) / (kWaves * 16);
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

void launch_mlp_predict(const float *P, const float *X, int64_t n, float *y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_predict, dim3(mlp_grid(n)), dim3(256), 0, st, P, X, n, y);
}

void launch_z_from_pred(const float *y, const double *avv, int64_t n, double lo, double hi, double *z, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_z_from_pred, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, avv, n, lo, hi, z);
}

void launch_mlp_grad(const float *P, const float *X, const float *Y, const int64_t *idx, int64_t row0, int64_t n,
                     float scale, float *part, int nparts, float *g, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(nparts), dim3(256), 0, st, P, X, Y, idx, row0, n, scale, part);
    hipLaunchKernelGGL(k_sum_partials, dim3((kTrain + 1 + 255) / 256), dim3(256), 0, st, part, nparts, g);
}

void launch_adam(float *P, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                 float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((kTrain + 255) / 256), dim3(256), 0, st, P, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace vtm
