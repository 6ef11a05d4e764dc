// Device building blocks of the learned a1^(2) closure MLP (36 -> 64 -> 64 -> 3,
// GELU): BF16 operands on the matrix cores (v_mfma_f32_16x16x16_bf16), FP32
// accumulation, LDS-resident tiles.  The closure is not part of the paper.
//
// Parameter vector (FP32, 6723 values): W1 (64 x 36, out x in), b1 (64),
// W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3).  Normalisation vector (78):
// x_mean (36), x_std (36), y_mean (3), y_std (3).
// Packed BF16 weights (8768 values, copied verbatim into LDS): W1 as 64 rows
// of stride 52 (inputs 36..51 zero), W2 as 64 rows of stride 68, W3 as 16 rows
// of stride 68 (outputs 3..15 zero; columns 64..67 of W2 and W3 zero).  The
// row strides are 8 bytes modulo 128, so the 8-byte matrix-core operand reads
// of 16 consecutive rows fall on distinct LDS bank pairs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbrr {
namespace mlp {

constexpr int kIn = 36, kInP = 48, kH = 64, kOut = 3, kOutP = 16;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kOut * kH, kNParam = kOffB3 + kOut;
static_assert(kNParam == 6723, "parameter count");
constexpr int kNNorm = 2 * kIn + 2 * kOut;
constexpr int kLd1 = 52, kLdH = 68;  // LDS row strides (BF16 elements) of 48- and 64-wide operands
constexpr int kPW1 = 0, kPW2 = kPW1 + kH * kLd1, kPW3 = kPW2 + kH * kLdH, kNPacked = kPW3 + kOutP * kLdH;
static_assert((kNPacked * 2) % 16 == 0 && (kPW2 * 2) % 16 == 0 && (kPW3 * 2) % 16 == 0, "16-byte packed blocks");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __builtin_bit_cast(float, uint32_t(b) << 16); }

// erf(x) by Abramowitz & Stegun, Handbook of Mathematical Functions, formula
// 7.1.26 (|error| <= 1.5e-7, below the BF16 rounding that follows every
// activation): erf(x) = 1 - t (a1 + t (a2 + ...)) exp(-x^2), t = 1/(1 + p x),
// x >= 0, odd extension.  g = exp(-x^2) is returned for the GELU derivative.
__device__ __forceinline__ float erf_as(float x, float& g) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  g = __expf(-ax * ax);
  const float e = 1.0f - poly * g;
  return x < 0.0f ? -e : e;
}

// GELU in the exact erf form, gelu(z) = z Phi(z) (Phi: standard normal
// distribution function), evaluated as max(z, 0) - |z| Phi(-|z|), an identity
// for every z.  Phi(-x) = 2^H(x) with x = min(|z|, 6) and H the degree-6
// polynomial below, fitted to log2 Phi(-x) on [0, 6] for the smallest largest
// error of x Phi(-x) (Lawson's iteratively reweighted least squares; the fit is
// gelu_fit.py beside this package).  FP32 error on [-12, 12]: at most 2.8e-7,
// 8.1e-8 beyond half an ulp of the result (erf by A&S 7.1.26 above: 3.8e-7);
// beyond |z| = 6 the term dropped is below 6e-9 |z|.  One exponential and
// nine other operations, against two transcendentals and about seventeen.
constexpr float kGeluH[7] = {-9.999930859e-01f, -1.151201725e+00f, -4.587709904e-01f, -5.341210216e-02f,
                             8.080714382e-03f,  -7.692191284e-04f, 3.309273961e-05f};
__device__ __forceinline__ float gelu(float z) {
  // the clamps as medians of three: min(|z|, 6) and max(z, 0) in one operation each
  const float x = __builtin_amdgcn_fmed3f(fabsf(z), 0.0f, 6.0f);
  float h = kGeluH[6];
#pragma unroll
  for (int k = 5; k >= 0; --k) h = fmaf(h, x, kGeluH[k]);
  return fmaf(-fabsf(z), __builtin_amdgcn_exp2f(h), __builtin_amdgcn_fmed3f(z, 0.0f, 3.40282347e38f));
}
// Derivative of the erf form, Phi(z) + z phi(z), with erf by A&S 7.1.26.
__device__ __forceinline__ float gelu_grad(float z) {
  float g;  // exp(-z^2 / 2)
  const float e = erf_as(z * 0.70710678118654752f, g);
  return 0.5f * (1.0f + e) + z * g * 0.39894228040143268f;
}

// Four FP32 values -> four BF16 values, round to nearest even (the matrix
// cores' operand layout: element r in bits 16 r .. 16 r + 15 of the pair).
__device__ __forceinline__ bf16x4 pack_bf16(float a, float b, float c, float d) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  const bf16x2 lo = __builtin_convertvector((f32x2){a, b}, bf16x2);
  const bf16x2 hi = __builtin_convertvector((f32x2){c, d}, bf16x2);
  return __builtin_bit_cast(bf16x4, ((u32x2){__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)}));
}

// One 16 x 16 output tile of A (M x K) * B (K x N) from BF16 values in LDS:
// A(i, k) = A[i * a_rs + k * a_cs], B(k, j) = B[k * b_rs + j * b_cs]; rows
// i0..i0+15, columns j0..j0+15, K a multiple of 16.  Lane l of the wave holds
// the results D[i0 + 4*(l/16) + r][j0 + l%16], r = 0..3 (matrix-core layout).
template <int K>
__device__ __forceinline__ f32x4 tile(const uint16_t* A, int a_rs, int a_cs, const uint16_t* B, int b_rs, int b_cs,
                                      int i0, int j0, f32x4 acc) {
  const int l = threadIdx.x & 63;
  const int ii = i0 + (l & 15), jj = j0 + (l & 15), kk = 4 * (l >> 4);
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = short(A[ii * a_rs + (k0 + kk + r) * a_cs]);
      b[r] = short(B[(k0 + kk + r) * b_rs + jj * b_cs]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Same tile when both operands are contiguous along k (A(i, k) = A[i * lda + k],
// B(k, j) = B[j * ldb + k], lda and ldb multiples of 4, 8-byte aligned rows):
// each lane fetches its four k values of A and of B with one 8-byte LDS read.
template <int K>
__device__ __forceinline__ f32x4 tile_kc(const uint16_t* A, int lda, const uint16_t* B, int ldb, int i0, int j0,
                                         f32x4 acc) {
  const int l = threadIdx.x & 63;
  const bf16x4* ap = reinterpret_cast<const bf16x4*>(A + (i0 + (l & 15)) * lda + 4 * (l >> 4));
  const bf16x4* bp = reinterpret_cast<const bf16x4*>(B + (j0 + (l & 15)) * ldb + 4 * (l >> 4));
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[k0 / 4], bp[k0 / 4], acc, 0, 0, 0);
  return acc;
}

// Row and column of element r of a lane's tile result.
__device__ __forceinline__ int tile_row(int i0, int r) { return i0 + 4 * ((threadIdx.x & 63) >> 4) + r; }
__device__ __forceinline__ int tile_col(int j0) { return j0 + (threadIdx.x & 15); }

// Load the packed BF16 weights into LDS with a block of NT threads, 16 bytes
// per load, every load of a thread issued before its first LDS write.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <int NT>
__device__ __forceinline__ void load_weights(const uint16_t* __restrict__ packed, uint16_t* lds) {
  constexpr int kChunks = kNPacked * 2 / 16, kPer = (kChunks + NT - 1) / NT;
  const u32x4* src = reinterpret_cast<const u32x4*>(packed);
  u32x4* dst = reinterpret_cast<u32x4*>(lds);
  u32x4 v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int c = int(threadIdx.x) + k * NT;
    if (c < kChunks) v[k] = src[c];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int c = int(threadIdx.x) + k * NT;
    if (c < kChunks) dst[c] = v[k];
  }
}

}  // namespace mlp
}  // namespace lbrr
