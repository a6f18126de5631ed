// HIP kernels for gfx950 of the surrogate network: a multilayer perceptron with d_in inputs,
// `depth` hidden SiLU layers of `width` units and 2 linear outputs, trained with an
// output-weighted mean squared error and Adam.
//
// Precision: the hidden-to-hidden layers run on MFMA (v_mfma_f32_16x16x32_bf16) with BF16
// weights and activations and FP32 accumulation, forward and backward.  The first layer (a few
// inputs) and the output layer (2 outputs) run in FP32, so that the input features and the
// predicted front positions keep FP32 resolution.  Master weights, gradients and Adam moments
// are FP32; Adam refreshes BF16 copies of each hidden weight matrix and of its transpose.
//
// All reductions (bias and output-layer gradients, loss, data statistics) use fixed-order trees,
// so repeated runs give identical results.
#include "sur_internal.h"

namespace scf {
namespace sur {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_prime(float z) {
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// SplitMix64 output function (published constants): counter-based random numbers.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int kThreads = 256;

// Fixed-order block reduction (kThreads threads).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------------------------
// MFMA GEMM, "NT" form: C[m][n] = sum_k A[m*lda + k] * B[n*ldb + k], BF16 operands contiguous in
// k, FP32 accumulation.  One wave per 16 x 16 output tile, four waves per block along n.
// Lane l holds A[m0 + l%16][k0 + 8(l/16) .. +7] and B[n0 + l%16][k0 + 8(l/16) .. +7] and receives
// C[m0 + 4(l/16) + i][n0 + l%16], i = 0..3 (layout checked on the device by the GEMM tests).
// M, N multiples of 16 (N of 64 per block row), K multiple of 32.
// ---------------------------------------------------------------------------------------------
template <class Epi>
__global__ void __launch_bounds__(256)
k_gemm_nt(const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B, int ldb, int K,
          Epi epi) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 16;
    const int n0 = (blockIdx.y * 4 + wave) * 16;
    const int r = lane & 15, g = lane >> 4;
    const __bf16* a = A + (int64_t)(m0 + r) * lda + 8 * g;
    const __bf16* b = B + (int64_t)(n0 + r) * ldb + 8 * g;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf8 fa = *reinterpret_cast<const bf8*>(a + k0);
        const bf8 fb = *reinterpret_cast<const bf8*>(b + k0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
    }
    epi(m0 + 4 * g, n0 + r, acc);
}

// Forward hidden layer: z = acc + bias; keeps z (FP32) for the backward pass and h = silu(z) in
// BF16, both row-major [m][n] and transposed [n][m] (the transposed copy feeds the weight
// gradient, which reduces over m).
struct EpiForward {
    const float* bias;
    float* Z;           // [M][N]
    __bf16* H;          // [M][N]
    __bf16* HT;         // [N][M]
    int N, M;
    __device__ void operator()(int mrow, int n, f4 acc) const {
        bf4 t;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[i] + bias[n];
            Z[(int64_t)(mrow + i) * N + n] = z;
            const __bf16 h = (__bf16)silu(z);
            H[(int64_t)(mrow + i) * N + n] = h;
            t[i] = h;
        }
        *reinterpret_cast<bf4*>(HT + (int64_t)n * M + mrow) = t;
    }
};

// Back-propagation through a hidden layer: acc = dH of the layer below; dz = dH * silu'(z).
struct EpiBackward {
    const float* Zprev;   // [M][N] pre-activations of the layer below
    float* dZ;            // [M][N] FP32 (bias gradient, first-layer weight gradient)
    __bf16* dZb;          // [M][N]
    __bf16* dZbT;         // [N][M]
    int N, M;
    __device__ void operator()(int mrow, int n, f4 acc) const {
        bf4 t;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t o = (int64_t)(mrow + i) * N + n;
            const float dz = acc[i] * silu_prime(Zprev[o]);
            dZ[o] = dz;
            const __bf16 hb = (__bf16)dz;
            dZb[o] = hb;
            t[i] = hb;
        }
        *reinterpret_cast<bf4*>(dZbT + (int64_t)n * M + mrow) = t;
    }
};

// Weight gradient: dW[n_out][k_in] = acc.
struct EpiWeightGrad {
    float* dW;
    int N;
    __device__ void operator()(int mrow, int n, f4 acc) const {
#pragma unroll
        for (int i = 0; i < 4; ++i) dW[(int64_t)(mrow + i) * N + n] = acc[i];
    }
};

// ---------------------------------------------------------------------------------------------
// First layer (FP32): z = Xn W1^T + b1, one thread per (row, unit).
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_first_forward(const float* __restrict__ X, int d_in, const float* __restrict__ W,
                const float* __restrict__ bias, int width, int rows, float* __restrict__ Z,
                __bf16* __restrict__ H, __bf16* __restrict__ HT) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (int64_t)rows * width) return;
    const int m = (int)(i / width), n = (int)(i % width);
    float z = bias[n];
    for (int k = 0; k < d_in; ++k) z += X[(int64_t)m * d_in + k] * W[n * d_in + k];
    Z[i] = z;
    const __bf16 h = (__bf16)silu(z);
    H[i] = h;
    HT[(int64_t)n * rows + m] = h;
}

// First-layer gradients: dW1[n][k] = sum_m dZ1[m][n] Xn[m][k], db1[n] = sum_m dZ1[m][n].
// One block per unit n; one fixed-order reduction per input (k = d_in gives the bias).
__global__ void __launch_bounds__(kThreads)
k_first_grad(const float* __restrict__ dZ, const float* __restrict__ X, int d_in, int width,
             int rows, float* __restrict__ dW, float* __restrict__ db) {
    __shared__ float sh[kThreads];
    const int n = blockIdx.x;
    for (int k = 0; k <= d_in; ++k) {
        float a = 0.0f;
        for (int m = threadIdx.x; m < rows; m += kThreads)
            a += dZ[(int64_t)m * width + n] * (k < d_in ? X[(int64_t)m * d_in + k] : 1.0f);
        a = block_sum(a, sh);
        if (threadIdx.x == 0) {
            if (k < d_in) dW[n * d_in + k] = a;
            else db[n] = a;
        }
    }
}

// Column sums of an FP32 [rows][width] matrix (bias gradients), one block per column.
__global__ void __launch_bounds__(kThreads)
k_colsum(const float* __restrict__ M, int width, int rows, float* __restrict__ out) {
    __shared__ float sh[kThreads];
    const int n = blockIdx.x;
    float a = 0.0f;
    for (int m = threadIdx.x; m < rows; m += kThreads) a += M[(int64_t)m * width + n];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[n] = a;
}

// ---------------------------------------------------------------------------------------------
// Output layer, loss and the first backward step, one wave per row:
//   y_o = b_o + sum_k silu(z_k) W_o[k];  r = y - t;  loss_m = w_m |r|^2 / 2;  dy = w_m r / n
// (n = number of real rows; padding rows carry w = 0)
//   dz_k = (sum_o dy_o W_o[k]) silu'(z_k)  -> dZ (FP32), dZb, dZbT (BF16) of the last layer.
// With T == nullptr only y is computed (inference).
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_output(const float* __restrict__ Z, int width, int rows, const float* __restrict__ W,
         const float* __restrict__ bias, const float* __restrict__ T, const float* __restrict__ w,
         float inv_n, float* __restrict__ Y, float* __restrict__ dY, float* __restrict__ rowloss,
         float* __restrict__ dZ, __bf16* __restrict__ dZb, __bf16* __restrict__ dZbT) {
    const int lane = threadIdx.x & 63;
    const int m = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (m >= rows) return;
    const float* z = Z + (int64_t)m * width;
    float s0 = 0.0f, s1 = 0.0f;
    for (int k = lane; k < width; k += 64) {
        const float h = silu(z[k]);
        s0 += h * W[k];
        s1 += h * W[width + k];
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
    }
    const float y0 = s0 + bias[0], y1 = s1 + bias[1];
    if (lane == 0) {
        Y[2 * m] = y0;
        Y[2 * m + 1] = y1;
    }
    if (!T) return;
    const float r0 = y0 - T[2 * m], r1 = y1 - T[2 * m + 1];
    const float wm = w[m];
    const float d0 = wm * r0 * inv_n, d1 = wm * r1 * inv_n;
    if (lane == 0) {
        dY[2 * m] = d0;
        dY[2 * m + 1] = d1;
        rowloss[m] = 0.5f * wm * (r0 * r0 + r1 * r1);
    }
    for (int k = lane; k < width; k += 64) {
        const float dz = (d0 * W[k] + d1 * W[width + k]) * silu_prime(z[k]);
        dZ[(int64_t)m * width + k] = dz;
        dZb[(int64_t)m * width + k] = (__bf16)dz;
        dZbT[(int64_t)k * rows + m] = (__bf16)dz;
    }
}

// Output-layer gradients: dW_o[k] = sum_m dy_o silu(z_mk), db_o = sum_m dy_o; block per k
// (block `width` computes the bias gradient).
__global__ void __launch_bounds__(kThreads)
k_output_grad(const float* __restrict__ Z, int width, int rows, const float* __restrict__ dY,
              float* __restrict__ dW, float* __restrict__ db) {
    __shared__ float sh[kThreads];
    const int k = blockIdx.x;
    float a0 = 0.0f, a1 = 0.0f;
    for (int m = threadIdx.x; m < rows; m += kThreads) {
        const float h = k < width ? silu(Z[(int64_t)m * width + k]) : 1.0f;
        a0 += dY[2 * m] * h;
        a1 += dY[2 * m + 1] * h;
    }
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    if (threadIdx.x == 0) {
        if (k < width) {
            dW[k] = a0;
            dW[width + k] = a1;
        } else {
            db[0] = a0;
            db[1] = a1;
        }
    }
}

// Sum of the per-row losses (fixed order, one block).
__global__ void __launch_bounds__(kThreads)
k_loss_sum(const float* __restrict__ rowloss, int rows, float inv_n, float* __restrict__ out) {
    __shared__ double sh[kThreads];
    double a = 0.0;
    for (int m = threadIdx.x; m < rows; m += kThreads) a += (double)rowloss[m];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[0] = (float)(a * inv_n);
}

// ---------------------------------------------------------------------------------------------
// Adam (Kingma and Ba, 2015) with bias correction; the step count and the learning rate live on
// the device so that captured graphs advance the one and follow changes of the other.  Hidden weight matrices are copied to BF16, row-major and
// transposed.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m1,
       float* __restrict__ m2, int64_t n, const int64_t* __restrict__ step,
       const float* __restrict__ lr_dev, float b1, float b2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float lr = *lr_dev;
    const float t = (float)(*step + 1);
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float v = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    const float ah = a / (1.0f - powf(b1, t));
    const float vh = v / (1.0f - powf(b2, t));
    theta[i] -= lr * ah / (sqrtf(vh) + eps);
}

__global__ void k_bump64(int64_t* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = *c + 1;
}

// BF16 copies of one (n_out x n_in) FP32 weight matrix, row-major and transposed.
__global__ void __launch_bounds__(kThreads)
k_shadow(const float* __restrict__ W, int n_out, int n_in, __bf16* __restrict__ Wb,
         __bf16* __restrict__ WbT) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (int64_t)n_out * n_in) return;
    const int o = (int)(i / n_in), k = (int)(i % n_in);
    const __bf16 v = (__bf16)W[i];
    Wb[i] = v;
    WbT[(int64_t)k * n_out + o] = v;
}

// ---------------------------------------------------------------------------------------------
// Data: feature statistics (mean, standard deviation, min, max per input; FP64 sums, one block
// per feature), normalisation of an explicit batch, and random minibatches of the stored set.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
k_stats(const float* __restrict__ X, int d_in, int64_t n, float* __restrict__ mean,
        float* __restrict__ stdv, float* __restrict__ lo, float* __restrict__ hi) {
    __shared__ double sh[kThreads];
    __shared__ float sf[kThreads];
    const int k = blockIdx.x;
    double s = 0.0;
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t m = threadIdx.x; m < n; m += kThreads) {
        const float v = X[m * d_in + k];
        s += v;
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    const double mu = block_sum(s, sh) / (double)n;
    double q = 0.0;
    for (int64_t m = threadIdx.x; m < n; m += kThreads) {
        const double d = X[m * d_in + k] - mu;
        q += d * d;
    }
    const double var = block_sum(q, sh) / (double)n;
    // min / max by the same fixed tree
    sf[threadIdx.x] = mn;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sf[threadIdx.x] = fminf(sf[threadIdx.x], sf[threadIdx.x + st]);
        __syncthreads();
    }
    const float gmn = sf[0];
    __syncthreads();
    sf[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) sf[threadIdx.x] = fmaxf(sf[threadIdx.x], sf[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mean[k] = (float)mu;
        stdv[k] = var > 0.0 ? (float)sqrt(var) : 1.0f;
        lo[k] = gmn;
        hi[k] = sf[0];
    }
}

// Normalise rows of X into Xn (and copy targets / weights when given).  With rng set, row i is
// drawn from the stored set (src_rows rows) by a counter-based hash of (seed, step, i).
__global__ void __launch_bounds__(kThreads)
k_gather(const float* __restrict__ X, const float* __restrict__ T, const float* __restrict__ w,
         int64_t src_rows, int d_in, int rows, const float* __restrict__ mean,
         const float* __restrict__ stdv, float* __restrict__ Xn, float* __restrict__ Tb,
         float* __restrict__ wb, int rng, uint64_t seed, const int64_t* __restrict__ step) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    int64_t j = i;
    if (rng) {
        const uint64_t h = mix64(seed ^ mix64((uint64_t)(*step) * 0x100000001B3ull + (uint64_t)i));
        j = (int64_t)(h % (uint64_t)src_rows);
    }
    for (int k = 0; k < d_in; ++k) Xn[(int64_t)i * d_in + k] = (X[j * d_in + k] - mean[k]) / stdv[k];
    if (Tb) {
        Tb[2 * i] = T[2 * j];
        Tb[2 * i + 1] = T[2 * j + 1];
        wb[i] = w[j];
    }
}

// Rows i < n of X (caller's device memory) normalised into Xn as k_gather does; padding rows
// [n, rows) are set to 0 (rows are independent through the network and their outputs unused).
__global__ void __launch_bounds__(kThreads)
k_normalise(const float* __restrict__ X, int64_t n, int d_in, int rows, const float* __restrict__ mean,
            const float* __restrict__ stdv, float* __restrict__ Xn) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    for (int k = 0; k < d_in; ++k)
        Xn[(int64_t)i * d_in + k] = i < n ? (X[(int64_t)i * d_in + k] - mean[k]) / stdv[k] : 0.0f;
}

__global__ void __launch_bounds__(kThreads) k_fill_u8(uint8_t* __restrict__ p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

// Inputs inside the axis-aligned box of the stored training inputs.
__global__ void __launch_bounds__(kThreads)
k_hull(const float* __restrict__ X, int d_in, int rows, const float* __restrict__ lo,
       const float* __restrict__ hi, uint8_t* __restrict__ in) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    uint8_t ok = 1;
    for (int k = 0; k < d_in; ++k) {
        const float v = X[(int64_t)i * d_in + k];
        if (!(v >= lo[k] && v <= hi[k])) ok = 0;
    }
    in[i] = ok;
}

// Parameter initialisation: W uniform in +-1/sqrt(fan_in) from a counter-based hash, b = 0.
__global__ void __launch_bounds__(kThreads)
k_init_params(float* __restrict__ theta, int64_t off, int n_out, int n_in, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nw = (int64_t)n_out * n_in;
    if (i >= nw + n_out) return;
    float v = 0.0f;
    if (i < nw) {
        const uint64_t h = mix64(seed ^ mix64((uint64_t)(off + i)));
        const float u = (float)(h >> 40) * (1.0f / 16777216.0f);   // [0, 1)
        v = (2.0f * u - 1.0f) / sqrtf((float)n_in);
    }
    theta[off + i] = v;
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + kThreads - 1) / kThreads)); }

}  // namespace

hipError_t gemm_forward(const __bf16* Hprev, const __bf16* Wb, const float* bias, int rows, int width,
                        float* Z, __bf16* H, __bf16* HT, hipStream_t s) {
    EpiForward epi{bias, Z, H, HT, width, rows};
    hipLaunchKernelGGL(k_gemm_nt<EpiForward>, dim3(rows / 16, width / 64), dim3(256), 0, s, Hprev,
                       width, Wb, width, width, epi);
    return hipGetLastError();
}

hipError_t gemm_backward(const __bf16* dZb, const __bf16* WbT, const float* Zprev, int rows,
                         int width, float* dZ, __bf16* dZbo, __bf16* dZbTo, hipStream_t s) {
    EpiBackward epi{Zprev, dZ, dZbo, dZbTo, width, rows};
    hipLaunchKernelGGL(k_gemm_nt<EpiBackward>, dim3(rows / 16, width / 64), dim3(256), 0, s, dZb,
                       width, WbT, width, width, epi);
    return hipGetLastError();
}

hipError_t gemm_weight_grad(const __bf16* dZbT, const __bf16* HT, int rows, int width, float* dW,
                            hipStream_t s) {
    EpiWeightGrad epi{dW, width};
    hipLaunchKernelGGL(k_gemm_nt<EpiWeightGrad>, dim3(width / 16, width / 64), dim3(256), 0, s, dZbT,
                       rows, HT, rows, rows, epi);
    return hipGetLastError();
}

hipError_t first_forward(const float* Xn, int d_in, const float* W, const float* b, int width, int rows,
                         float* Z, __bf16* H, __bf16* HT, hipStream_t s) {
    hipLaunchKernelGGL(k_first_forward, grid1((int64_t)rows * width), dim3(kThreads), 0, s, Xn, d_in, W,
                       b, width, rows, Z, H, HT);
    return hipGetLastError();
}

hipError_t first_grad(const float* dZ, const float* Xn, int d_in, int width, int rows, float* dW,
                      float* db, hipStream_t s) {
    hipLaunchKernelGGL(k_first_grad, dim3(width), dim3(kThreads), 0, s, dZ, Xn, d_in, width, rows, dW, db);
    return hipGetLastError();
}

hipError_t colsum(const float* M, int width, int rows, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(width), dim3(kThreads), 0, s, M, width, rows, out);
    return hipGetLastError();
}

hipError_t output_layer(const float* Z, int width, int rows, const float* W, const float* b,
                        const float* T, const float* w, float inv_n, float* Y, float* dY,
                        float* rowloss, float* dZ, __bf16* dZb, __bf16* dZbT, hipStream_t s) {
    hipLaunchKernelGGL(k_output, dim3((rows + 3) / 4), dim3(kThreads), 0, s, Z, width, rows, W, b, T, w,
                       inv_n, Y, dY, rowloss, dZ, dZb, dZbT);
    return hipGetLastError();
}

hipError_t output_grad(const float* Z, int width, int rows, const float* dY, float* dW, float* db,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_output_grad, dim3(width + 1), dim3(kThreads), 0, s, Z, width, rows, dY, dW, db);
    return hipGetLastError();
}

hipError_t loss_sum(const float* rowloss, int rows, float inv_n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kThreads), 0, s, rowloss, rows, inv_n, out);
    return hipGetLastError();
}

hipError_t adam(float* theta, const float* grad, float* m1, float* m2, int64_t n, int64_t* step,
                const float* lr, float b1, float b2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, grid1(n), dim3(kThreads), 0, s, theta, grad, m1, m2, n, step, lr, b1, b2,
                       eps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bump64, dim3(1), dim3(64), 0, s, step);
    return hipGetLastError();
}

hipError_t shadow(const float* W, int n_out, int n_in, __bf16* Wb, __bf16* WbT, hipStream_t s) {
    hipLaunchKernelGGL(k_shadow, grid1((int64_t)n_out * n_in), dim3(kThreads), 0, s, W, n_out, n_in, Wb,
                       WbT);
    return hipGetLastError();
}

hipError_t stats(const float* X, int d_in, int64_t n, float* mean, float* stdv, float* lo, float* hi,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(d_in), dim3(kThreads), 0, s, X, d_in, n, mean, stdv, lo, hi);
    return hipGetLastError();
}

hipError_t gather(const float* X, const float* T, const float* w, int64_t src_rows, int d_in, int rows,
                  const float* mean, const float* stdv, float* Xn, float* Tb, float* wb, int rng,
                  uint64_t seed, const int64_t* step, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, grid1(rows), dim3(kThreads), 0, s, X, T, w, src_rows, d_in, rows, mean,
                       stdv, Xn, Tb, wb, rng, seed, step);
    return hipGetLastError();
}

hipError_t hull(const float* X, int d_in, int rows, const float* lo, const float* hi, uint8_t* in,
                hipStream_t s) {
    hipLaunchKernelGGL(k_hull, grid1(rows), dim3(kThreads), 0, s, X, d_in, rows, lo, hi, in);
    return hipGetLastError();
}

hipError_t normalise(const float* X, int64_t n, int d_in, int rows, const float* mean, const float* stdv,
                     float* Xn, hipStream_t s) {
    hipLaunchKernelGGL(k_normalise, grid1(rows), dim3(kThreads), 0, s, X, n, d_in, rows, mean, stdv, Xn);
    return hipGetLastError();
}

hipError_t fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u8, grid1(n), dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t init_params(float* theta, int64_t off, int n_out, int n_in, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_init_params, grid1((int64_t)n_out * n_in + n_out), dim3(kThreads), 0, s, theta,
                       off, n_out, n_in, seed);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace scf
