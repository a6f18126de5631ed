// Internal interface between the surrogate kernels (sur_kernels.hip) and their host runtime
// (sur_runtime.hip).  Not installed; the public ABI is include/scf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scf {
namespace sur {

constexpr int kMaxIn = 32;   // largest number of input features

// Launchers, asynchronous on stream s.  Matrices are row-major; "T" names a transposed copy.
hipError_t gemm_forward(const __bf16* Hprev, const __bf16* Wb, const float* bias, int rows, int width,
                        float* Z, __bf16* H, __bf16* HT, hipStream_t s);
hipError_t gemm_backward(const __bf16* dZb, const __bf16* WbT, const float* Zprev, int rows,
                         int width, float* dZ, __bf16* dZbo, __bf16* dZbTo, hipStream_t s);
hipError_t gemm_weight_grad(const __bf16* dZbT, const __bf16* HT, int rows, int width, float* dW,
                            hipStream_t s);
hipError_t first_forward(const float* Xn, int d_in, const float* W, const float* b, int width, int rows,
                         float* Z, __bf16* H, __bf16* HT, hipStream_t s);
hipError_t first_grad(const float* dZ, const float* Xn, int d_in, int width, int rows, float* dW,
                      float* db, hipStream_t s);
hipError_t colsum(const float* M, int width, int rows, float* out, hipStream_t s);
hipError_t output_layer(const float* Z, int width, int rows, const float* W, const float* b,
                        const float* T, const float* w, float inv_n, float* Y, float* dY,
                        float* rowloss, float* dZ, __bf16* dZb, __bf16* dZbT, hipStream_t s);
hipError_t output_grad(const float* Z, int width, int rows, const float* dY, float* dW, float* db,
                       hipStream_t s);
hipError_t loss_sum(const float* rowloss, int rows, float inv_n, float* out, hipStream_t s);
hipError_t adam(float* theta, const float* grad, float* m1, float* m2, int64_t n, int64_t* step,
                const float* lr, float b1, float b2, float eps, hipStream_t s);
hipError_t shadow(const float* W, int n_out, int n_in, __bf16* Wb, __bf16* WbT, hipStream_t s);
hipError_t stats(const float* X, int d_in, int64_t n, float* mean, float* stdv, float* lo, float* hi,
                 hipStream_t s);
hipError_t gather(const float* X, const float* T, const float* w, int64_t src_rows, int d_in, int rows,
                  const float* mean, const float* stdv, float* Xn, float* Tb, float* wb, int rng,
                  uint64_t seed, const int64_t* step, hipStream_t s);
hipError_t hull(const float* X, int d_in, int rows, const float* lo, const float* hi, uint8_t* in,
                hipStream_t s);
// Rows i < n of X normalised by (mean, stdv) into Xn (rows >= n entries, padding rows zeroed).
hipError_t normalise(const float* X, int64_t n, int d_in, int rows, const float* mean, const float* stdv,
                     float* Xn, hipStream_t s);
hipError_t fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t init_params(float* theta, int64_t off, int n_out, int n_in, uint64_t seed, hipStream_t s);

}  // namespace sur
}  // namespace scf
