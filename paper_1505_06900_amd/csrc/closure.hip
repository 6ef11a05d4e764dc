// Learned a1^(2) closure for coarse D2Q9 runs (not part of the paper): data
// kernels (coarse-graining of fine fields, next-step features), MLP training
// (forward + backward on the matrix cores, per-block partial gradients, fixed-
// order reduction, Adam), batched inference, and the fused coarse step that
// adds the predicted correction to a1^(2) before the recursion of Sec. 3.1
// rebuilds the higher-order coefficients (Eq. rel_a1) and the populations are
// reconstructed (Eq. discr_bgk_reg).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "closure.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace lbrr {
namespace {

using namespace mlp;
static_assert(kMlpNPacked == kNPacked && kMlpNParam == kNParam && kMlpNNorm == kNNorm, "closure.hpp sizes");

// ---------------------------------------------------------------------------
// Coarse-graining of fine fields by F x F box averages (acoustic scaling:
// velocities and stresses keep their lattice-unit values):
//   rho_c = box(rho), j_c = box(rho u), u_c = j_c / rho_c,
//   T = box(rho u u) - rho_c u_c u_c          (sub-filter stress),
//   pi1_c = alpha box(pi1) + beta T.
template <class T>
__global__ void __launch_bounds__(256) k_coarsen(const T* __restrict__ rho, const T* __restrict__ u,
                                                 const T* __restrict__ pi1, int nfx, int nfy, int F, double alpha,
                                                 double beta, double* __restrict__ rho_c, double* __restrict__ u_c,
                                                 double* __restrict__ pi1_c) {
  const int ncx = nfx / F, ncy = nfy / F;
  const int64_t nc = int64_t(ncx) * ncy, nfine = int64_t(nfx) * nfy;
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int cx = int(c % ncx), cy = int(c / ncx);
  double sr = 0, sjx = 0, sjy = 0, sxx = 0, sxy = 0, syy = 0, vxx = 0, vxy = 0, vyy = 0;
  for (int dy = 0; dy < F; ++dy) {
    for (int dx = 0; dx < F; ++dx) {
      const int64_t n = int64_t(cy * F + dy) * nfx + (cx * F + dx);
      const double r = double(rho[n]), ux = double(u[n]), uy = double(u[nfine + n]);
      sr += r;
      sjx += r * ux;
      sjy += r * uy;
      sxx += r * ux * ux;
      sxy += r * ux * uy;
      syy += r * uy * uy;
      vxx += double(pi1[n]);
      vxy += double(pi1[nfine + n]);
      vyy += double(pi1[2 * nfine + n]);
    }
  }
  const double inv = 1.0 / double(F * F);
  const double rc = sr * inv, ux = sjx * inv / rc, uy = sjy * inv / rc;
  const double txx = sxx * inv - rc * ux * ux, txy = sxy * inv - rc * ux * uy, tyy = syy * inv - rc * uy * uy;
  rho_c[c] = rc;
  u_c[c] = ux;
  u_c[nc + c] = uy;
  pi1_c[c] = alpha * vxx * inv + beta * txx;
  pi1_c[nc + c] = alpha * vxy * inv + beta * txy;
  pi1_c[2 * nc + c] = alpha * vyy * inv + beta * tyy;
}

// (rho - rho0, u_x, u_y) of the stored D2Q9 state at element offset off.
template <class S>
__device__ __forceinline__ void node_moments3(const S* __restrict__ src, const StepArgs& a, int64_t off,
                                              float (&v)[3]) {
  using R = typename Prec<S>::R;
  R f[9];
  sfor<0, 9>([&](auto I) { f[I] = R(src[int64_t(I) * a.si + off]); });
  const Moments<R> mo = raw_moments<D2Q9, R>(f);
  const Hydro<R> h = hydro<D2Q9, R>(mo, R(a.rho0));
  v[0] = float(h.drho);
  v[1] = float(h.ux);
  v[2] = float(h.uy);
}

// (rho - rho0, u_x, u_y) of every node of a stored D2Q9 state (compact [3][ny][nx]).
template <class S>
__global__ void __launch_bounds__(256) k_node_moments(const S* __restrict__ src, StepArgs a, float* __restrict__ m) {
  const int64_t nodes = int64_t(a.nx) * a.ny;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  float v[3];
  node_moments3<S>(src, a, node_offset(a, uint32_t(n)), v);
  m[n] = v[0];
  m[nodes + n] = v[1];
  m[2 * nodes + n] = v[2];
}

// Pull the 9 pre-collision deviations of node (x, y) from a stored state.
template <class S, class R>
__device__ __forceinline__ void pull9(const S* __restrict__ src, const StepArgs& a, int x, int y, R (&f)[9]) {
  const int xm = (x == 0) ? a.nx - 1 : x - 1, xp = (x == a.nx - 1) ? 0 : x + 1;
  const int ym = (y == 0) ? a.ny - 1 : y - 1, yp = (y == a.ny - 1) ? 0 : y + 1;
  sfor<0, 9>([&](auto I) {
    constexpr int cx = D2Q9::cx(I), cy = D2Q9::cy(I);
    const int xs = (cx == 1) ? xm : ((cx == -1) ? xp : x);
    const int ys = (cy == 1) ? ym : ((cy == -1) ? yp : y);
    f[I] = R(src[int64_t(I) * a.si + int64_t(ys) * a.sy + xs]);
  });
}

// The 36 raw features of node (x, y): pulled deviations, then the 3 x 3
// neighbourhood (dy outer, dx inner) of (rho - rho0, u_x, u_y) of the stored state.
template <class R>
__device__ __forceinline__ void features36(const R (&f)[9], const float* __restrict__ m, const StepArgs& a, int x,
                                           int y, float (&feat)[kIn]) {
  const int64_t nodes = int64_t(a.nx) * a.ny;
#pragma unroll
  for (int i = 0; i < 9; ++i) feat[i] = float(f[i]);
  int k = 9;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    const int yy = (y + dy + a.ny) % a.ny;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int xx = (x + dx + a.nx) % a.nx;
      const int64_t n = int64_t(yy) * a.nx + xx;
      feat[k++] = m[n];
      feat[k++] = m[nodes + n];
      feat[k++] = m[2 * nodes + n];
    }
  }
}

// Features of the next step and labels a_target - plain_weight * (plain
// a1^(2) of the pulled populations) (a_target NULL reads as 0), one thread per node.
template <class S>
__global__ void __launch_bounds__(256) k_features(const S* __restrict__ src, const float* __restrict__ m, StepArgs a,
                                                  const double* __restrict__ a_target, double plain_weight,
                                                  float* __restrict__ feat_out, float* __restrict__ lab_out) {
  using R = typename Prec<S>::R;
  const int64_t nodes = int64_t(a.nx) * a.ny;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int x = int(n % a.nx), y = int(n / a.nx);
  R f[9];
  pull9<S, R>(src, a, x, y, f);
  float feat[kIn];
  features36<R>(f, m, a, x, y, feat);
  for (int k = 0; k < kIn; ++k) feat_out[n * kIn + k] = feat[k];
  const Moments<R> mo = raw_moments<D2Q9, R>(f);
  const Hydro<R> h = hydro<D2Q9, R>(mo, R(a.rho0));
  const double ap[3] = {double(h.axx), double(h.axy), double(h.ayy)};
  for (int c = 0; c < 3; ++c)
    lab_out[n * 3 + c] = float((a_target ? a_target[int64_t(c) * nodes + n] : 0.0) - plain_weight * ap[c]);
}

// ---------------------------------------------------------------------------
// Per-block constants of the inference kernels, staged in LDS: biases b1 (64),
// b2 (64), b3 (3, padded to 4), then x_mean (36), 1/x_std (36), y_mean (3), y_std (3).
constexpr int kCB1 = 0, kCB2 = kCB1 + kH, kCB3 = kCB2 + kH, kCMean = kCB3 + 4, kCInv = kCMean + kIn,
              kCYMean = kCInv + kIn, kCYStd = kCYMean + kOut, kNConst = kCYStd + kOut;
// Per-wave activation region: 64 rows (one per sample) of kLdH BF16 values.
constexpr int kRegion = 64 * kLdH;

__device__ __forceinline__ void load_constants(const float* __restrict__ params, const float* __restrict__ norm,
                                               float* c) {
  for (int k = threadIdx.x; k < kNConst; k += blockDim.x) {
    float v;
    if (k < kCB2) v = params[kOffB1 + k];
    else if (k < kCB3) v = params[kOffB2 + k - kCB2];
    else if (k < kCMean) v = (k - kCB3 < kOut) ? params[kOffB3 + k - kCB3] : 0.0f;
    else if (k < kCInv) v = norm[k - kCMean];
    else if (k < kCYMean) v = 1.0f / norm[kIn + k - kCInv];
    else v = norm[2 * kIn + k - kCYMean];
    c[k] = v;
  }
}

// Forward pass of a group of 64 samples shared by NW waves; every thread of
// the block calls it (barriers inside).  Wave `part` (0..NW-1) of the group
// computes every NW-th output tile of each layer; wave 0 holds the samples
// (sample s = its lane s): it writes their features and reads their outputs.
// The products are computed transposed, features x samples (weights as the
// matrix-core A operand), so a lane's result, four consecutive features of
// one sample, goes to the sample's LDS row with one 8-byte write and is read
// back as the next layer's operand with one 8-byte read.  feat: the lane's raw
// features (wave 0); w: packed weights in LDS; r0, r1: the group's two
// activation regions; c: constants.
template <int NW>
__device__ __forceinline__ void forward_group(const float (&feat)[kIn], int part, const uint16_t* w, uint16_t* r0,
                                              uint16_t* r1, const float* c, float (&out)[kOut]) {
  const int lane = threadIdx.x & 63, q = lane >> 4;
  if (part == 0) {  // standardised BF16 features, row = sample (stride kLd1, inputs 36..47 zero)
    bf16x4* xr = reinterpret_cast<bf16x4*>(r0 + lane * kLd1);
#pragma unroll
    for (int k4 = 0; k4 < kInP / 4; ++k4) {
      bf16x4 v;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 4 * k4 + r;
        v[r] = short(k < kIn ? to_bf16((feat[k] - c[kCMean + k]) * c[kCInv + k]) : uint16_t(0));
      }
      xr[k4] = v;
    }
  }
  __syncthreads();
  // layer 1: H1 = gelu(W1 X + b1), 4 x 4 tiles (features j0, samples s0) -> r1
#pragma unroll
  for (int t = part; t < 16; t += NW) {
    const int j0 = 16 * (t & 3), s0 = 16 * (t >> 2);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kInP>(w + kPW1, kLd1, r0, kLd1, j0, s0, acc);
    const int j = j0 + 4 * q;
    bf16x4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = short(to_bf16(gelu(acc[r] + c[kCB1 + j + r])));
    *reinterpret_cast<bf16x4*>(r1 + (s0 + (lane & 15)) * kLdH + j) = h;
  }
  __syncthreads();
  // layer 2: H2 = gelu(W2 H1 + b2) -> r0
#pragma unroll
  for (int t = part; t < 16; t += NW) {
    const int j0 = 16 * (t & 3), s0 = 16 * (t >> 2);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kH>(w + kPW2, kLdH, r1, kLdH, j0, s0, acc);
    const int j = j0 + 4 * q;
    bf16x4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = short(to_bf16(gelu(acc[r] + c[kCB2 + j + r])));
    *reinterpret_cast<bf16x4*>(r0 + (s0 + (lane & 15)) * kLdH + j) = h;
  }
  __syncthreads();
  // layer 3: Y = W3 H2 + b3 (rows 0..2 of one 16-row tile), FP32 -> r1 as [64][4]
  float* ys = reinterpret_cast<float*>(r1);
#pragma unroll
  for (int t = part; t < 4; t += NW) {
    const int s0 = 16 * t;
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kH>(w + kPW3, kLdH, r0, kLdH, 0, s0, acc);
    if (q == 0) {
#pragma unroll
      for (int o = 0; o < kOut; ++o) ys[(s0 + lane) * 4 + o] = acc[o] + c[kCB3 + o];
    }
  }
  __syncthreads();
  if (part == 0) {
#pragma unroll
    for (int o = 0; o < kOut; ++o) out[o] = ys[lane * 4 + o] * c[kCYStd + o] + c[kCYMean + o];
  }
  __syncthreads();
}

constexpr int kInferWaves = 2;

// Batched inference: raw features (n x 36) -> de-normalised outputs (n x 3).
__global__ void __launch_bounds__(64 * kInferWaves) k_mlp_infer(const float* __restrict__ x, int64_t n,
                                                                const uint16_t* __restrict__ packed,
                                                                const float* __restrict__ params,
                                                                const float* __restrict__ norm, float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) uint16_t w[kNPacked];
  __shared__ __attribute__((aligned(16))) uint16_t reg[kInferWaves][2][kRegion];
  __shared__ __attribute__((aligned(16))) float cst[kNConst];
  load_weights<64 * kInferWaves>(packed, w);
  load_constants(params, norm, cst);
  const int wave = threadIdx.x >> 6;
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t sc = s < n ? s : n - 1;  // every lane takes part in the matrix-core tiles
  float feat[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) feat[k] = x[sc * kIn + k];
  __syncthreads();
  float out[kOut];
  forward_group<1>(feat, 0, w, reg[wave][0], reg[wave][1], cst, out);
  if (s < n)
    for (int o = 0; o < kOut; ++o) y[s * kOut + o] = out[o];
}

// ---------------------------------------------------------------------------
// Training: forward + backward of 32 samples per block (4 waves share the
// tiles), mean-squared error of normalised outputs over the whole batch.
// Writes one partial gradient (kNParam) and one partial squared-error sum per block.
constexpr int kTS = 32;  // samples per block

// Batch rows outside [0, nrows) are clamped to the nearest valid row.
__device__ __forceinline__ int64_t clamp_row(int r, int64_t nrows) {
  return r < 0 ? 0 : (int64_t(r) >= nrows ? nrows - 1 : int64_t(r));
}

__global__ void __launch_bounds__(256) k_mlp_train(const float* __restrict__ x, const float* __restrict__ tgt,
                                                   int64_t nrows, const int* __restrict__ idx, int batch,
                                                   const uint16_t* __restrict__ packed,
                                                   const float* __restrict__ params, const float* __restrict__ norm,
                                                   float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) uint16_t w[kNPacked];
  __shared__ __attribute__((aligned(16))) uint16_t xs[kTS * kLd1];
  __shared__ __attribute__((aligned(16))) uint16_t h1s[kTS * kLdH];
  __shared__ __attribute__((aligned(16))) uint16_t h2s[kTS * kLdH];
  __shared__ __attribute__((aligned(16))) uint16_t dys[kTS * kOutP], dz2s[kTS * kLdH], dz1s[kTS * kLdH];
  __shared__ float z1[kTS * kH], z2[kTS * kH], ys[kTS * kOutP], ts[kTS * kOut], red[kTS * kOut];
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int s0 = blockIdx.x * kTS;
  float* g = gpart + int64_t(blockIdx.x) * kNParam;
  load_weights<256>(packed, w);
  for (int e = threadIdx.x; e < kTS * kInP; e += blockDim.x) {
    const int s = e / kInP, k = e % kInP, si = s0 + s;
    float v = 0.0f;
    if (k < kIn && si < batch) v = (x[clamp_row(idx[si], nrows) * kIn + k] - norm[k]) / norm[kIn + k];
    xs[s * kLd1 + k] = to_bf16(v);
  }
  for (int e = threadIdx.x; e < kTS * kOut; e += blockDim.x) {
    const int s = e / kOut, c = e % kOut, si = s0 + s;
    ts[e] = si < batch ? (tgt[clamp_row(idx[si], nrows) * kOut + c] - norm[2 * kIn + c]) / norm[2 * kIn + kOut + c]
                       : 0.0f;
  }
  __syncthreads();
  // forward ------------------------------------------------------------------
  for (int t = wave; t < 8; t += nw) {  // layer 1: 2 x 4 tiles
    const int i0 = 16 * (t >> 2), j0 = 16 * (t & 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kInP>(xs, kLd1, w + kPW1, kLd1, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) {
      const int i = tile_row(i0, r);
      const float zz = acc[r] + params[kOffB1 + j];
      z1[i * kH + j] = zz;
      h1s[i * kLdH + j] = to_bf16(gelu(zz));
    }
  }
  __syncthreads();
  for (int t = wave; t < 8; t += nw) {  // layer 2
    const int i0 = 16 * (t >> 2), j0 = 16 * (t & 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kH>(h1s, kLdH, w + kPW2, kLdH, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) {
      const int i = tile_row(i0, r);
      const float zz = acc[r] + params[kOffB2 + j];
      z2[i * kH + j] = zz;
      h2s[i * kLdH + j] = to_bf16(gelu(zz));
    }
  }
  __syncthreads();
  for (int t = wave; t < 2; t += nw) {  // layer 3: 2 x 1 tiles
    const int i0 = 16 * t;
    f32x4 acc = {0, 0, 0, 0};
    acc = tile_kc<kH>(h2s, kLdH, w + kPW3, kLdH, i0, 0, acc);
    const int j = tile_col(0);
    for (int r = 0; r < 4; ++r) ys[tile_row(i0, r) * kOutP + j] = acc[r] + (j < kOut ? params[kOffB3 + j] : 0.0f);
  }
  __syncthreads();
  // loss and dY = 2 (y - t) / (3 B) -----------------------------------------------
  for (int e = threadIdx.x; e < kTS * kOutP; e += blockDim.x) {
    const int s = e / kOutP, c = e % kOutP;
    float d = 0.0f;
    if (c < kOut && s0 + s < batch) {
      const float diff = ys[e] - ts[s * kOut + c];
      red[s * kOut + c] = diff * diff;
      d = 2.0f * diff / float(kOut * batch);
    } else if (c < kOut) {
      red[s * kOut + c] = 0.0f;
    }
    ys[e] = d;  // ys now holds dY (FP32)
    dys[e] = to_bf16(d);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float l = 0.0f;
    for (int e = 0; e < kTS * kOut; ++e) l += red[e];
    lpart[blockIdx.x] = l;
  }
  if (threadIdx.x < kOut) {  // db3
    float sacc = 0.0f;
    for (int s = 0; s < kTS; ++s) sacc += ys[s * kOutP + threadIdx.x];
    g[kOffB3 + threadIdx.x] = sacc;
  }
  // dW3 = dY^T H2 (rows o < 3), 1 x 4 tiles, K = samples
  for (int t = wave; t < 4; t += nw) {
    const int j0 = 16 * t;
    f32x4 acc = {0, 0, 0, 0};
    acc = tile<kTS>(dys, 1, kOutP, h2s, kLdH, 1, 0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) {
      const int o = tile_row(0, r);
      if (o < kOut) g[kOffW3 + o * kH + j] = acc[r];
    }
  }
  // dZ2 = (dY W3) * gelu'(z2); z2 keeps dZ2 in FP32
  for (int t = wave; t < 8; t += nw) {
    const int i0 = 16 * (t >> 2), j0 = 16 * (t & 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile<kOutP>(dys, kOutP, 1, w + kPW3, kLdH, 1, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) {
      const int i = tile_row(i0, r);
      const float d = acc[r] * gelu_grad(z2[i * kH + j]);
      z2[i * kH + j] = d;
      dz2s[i * kLdH + j] = to_bf16(d);
    }
  }
  __syncthreads();
  if (threadIdx.x < kH) {  // db2
    float sacc = 0.0f;
    for (int s = 0; s < kTS; ++s) sacc += z2[s * kH + threadIdx.x];
    g[kOffB2 + threadIdx.x] = sacc;
  }
  for (int t = wave; t < 16; t += nw) {  // dW2 = dZ2^T H1, 4 x 4 tiles, K = samples
    const int i0 = 16 * (t >> 2), j0 = 16 * (t & 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile<kTS>(dz2s, 1, kLdH, h1s, kLdH, 1, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) g[kOffW2 + tile_row(i0, r) * kH + j] = acc[r];
  }
  for (int t = wave; t < 8; t += nw) {  // dZ1 = (dZ2 W2) * gelu'(z1)
    const int i0 = 16 * (t >> 2), j0 = 16 * (t & 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile<kH>(dz2s, kLdH, 1, w + kPW2, kLdH, 1, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r) {
      const int i = tile_row(i0, r);
      const float d = acc[r] * gelu_grad(z1[i * kH + j]);
      z1[i * kH + j] = d;
      dz1s[i * kLdH + j] = to_bf16(d);
    }
  }
  __syncthreads();
  if (threadIdx.x < kH) {  // db1
    float sacc = 0.0f;
    for (int s = 0; s < kTS; ++s) sacc += z1[s * kH + threadIdx.x];
    g[kOffB1 + threadIdx.x] = sacc;
  }
  for (int t = wave; t < 12; t += nw) {  // dW1 = dZ1^T X, 4 x 3 tiles, K = samples
    const int i0 = 16 * (t / 3), j0 = 16 * (t % 3);
    f32x4 acc = {0, 0, 0, 0};
    acc = tile<kTS>(dz1s, 1, kLdH, xs, kLd1, 1, i0, j0, acc);
    const int j = tile_col(j0);
    for (int r = 0; r < 4; ++r)
      if (j < kIn) g[kOffW1 + tile_row(i0, r) * kIn + j] = acc[r];
  }
}

// grad[p] = sum over blocks of the partials in a fixed order (eight interleaved
// accumulators keep eight loads in flight per thread); loss = sum / (3 B).
__global__ void __launch_bounds__(256) k_grad_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart,
                                                     int nblocks, int batch, float* __restrict__ grad,
                                                     float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParam) {
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int b = 0;
    for (; b + 8 <= nblocks; b += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += gpart[int64_t(b + u) * kNParam + p];
    }
    for (; b < nblocks; ++b) s[0] += gpart[int64_t(b) * kNParam + p];
    grad[p] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  }
  if (p == 0 && loss) {
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += lpart[b];
    *loss = s / float(kOut * batch);
  }
}

// Column mean / std of x (n x dim): one block per column, fixed-order FP64 sums.
__global__ void __launch_bounds__(256) k_column_stats(const float* __restrict__ x, int64_t n, int dim,
                                                      float* __restrict__ mean, float* __restrict__ sd) {
  __shared__ double red[2][256];
  const int c = blockIdx.x;
  double s = 0.0, q = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = double(x[r * dim + c]);
    s += v;
    q += v * v;
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = q;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = red[0][0] / double(n);
    const double var = red[1][0] / double(n) - m * m;
    mean[c] = float(m);
    sd[c] = var > 0.0 ? float(sqrt(var)) : 1.0f;
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float mk = b1 * m[k] + (1.0f - b1) * g[k];
  const float vk = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// FP32 parameters -> padded BF16 weight blocks (layout of the packed vector above).
__global__ void __launch_bounds__(256) k_pack(const float* __restrict__ params, uint16_t* __restrict__ packed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNPacked) return;
  float v = 0.0f;
  if (e < kPW2) {
    const int o = e / kLd1, k = e % kLd1;
    if (k < kIn) v = params[kOffW1 + o * kIn + k];
  } else if (e < kPW3) {
    const int o = (e - kPW2) / kLdH, k = (e - kPW2) % kLdH;
    if (k < kH) v = params[kOffW2 + o * kH + k];
  } else {
    const int o = (e - kPW3) / kLdH, k = (e - kPW3) % kLdH;
    if (o < kOut && k < kH) v = params[kOffW3 + o * kH + k];
  }
  packed[e] = to_bf16(v);
}

// ---------------------------------------------------------------------------
// Fused coarse D2Q9 step with the closure: pull, moments, features, MLP on the
// matrix cores, a1^(2) += predicted correction, recursion and reconstruction,
// store.  A block handles 64 nodes of a row: wave 0 pulls and later collides
// (one node per lane; lanes past the row end use a wrapped node and do not
// store) while waves 1-3 compute (rho - rho0, u) of the stored state on rows
// y-1, y, y+1 (64 + 2 nodes each) into LDS for the neighbour features; then
// all four waves share the MLP tiles, so a 256^2 grid keeps four waves per
// SIMD busy.
constexpr int kClosureNW = 4;

template <int N, class S>
__global__ void __launch_bounds__(64 * kClosureNW) k_step_closure(const S* __restrict__ src, S* __restrict__ dst, StepArgs a,
                                                                  const uint16_t* __restrict__ packed,
                                                                  const float* __restrict__ params,
                                                                  const float* __restrict__ norm) {
  using R = typename Prec<S>::R;
  __shared__ __attribute__((aligned(16))) uint16_t w[kNPacked];
  __shared__ __attribute__((aligned(16))) uint16_t reg[2][kRegion];
  __shared__ __attribute__((aligned(16))) float cst[kNConst];
  __shared__ float nb[3][66][3];  // (rho - rho0, u) of rows y-1, y, y+1 at x0-1 .. x0+64
  load_weights<64 * kClosureNW>(packed, w);
  load_constants(params, norm, cst);
  const int part = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x0 = blockIdx.x * 64, xr = x0 + lane;
  const bool active = xr < a.nx;
  const int x = active ? xr : xr % a.nx;
  const int y = blockIdx.y;
  R f[9];
  if (part == 0) {
    pull9<S, R>(src, a, x, y, f);
  } else if (part <= 3) {
    const int yy = (y + part - 2 + a.ny) % a.ny;
    for (int k = lane; k < 66; k += 64) {
      const int xx = ((x0 - 1 + k) % a.nx + a.nx) % a.nx;
      float v[3];
      node_moments3<S>(src, a, int64_t(yy) * a.sy + xx, v);
      nb[part - 1][k][0] = v[0];
      nb[part - 1][k][1] = v[1];
      nb[part - 1][k][2] = v[2];
    }
  }
  __syncthreads();
  float feat[kIn];
  if (part == 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) feat[i] = float(f[i]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int c = 0; c < 3; ++c) feat[9 + 3 * (3 * dy + dx) + c] = nb[dy][lane + dx][c];
  }
  float d[kOut];
  forward_group<kClosureNW>(feat, part, w, reg[0], reg[1], cst, d);
  if (part != 0) return;
  const Moments<R> mo = raw_moments<D2Q9, R>(f);
  Hydro<R> h = hydro<D2Q9, R>(mo, R(a.rho0));
  h.axx += R(d[0]);
  h.axy += R(d[1]);
  h.ayy += R(d[2]);
  R C[3][3][3];
  coefficients<D2Q9, N, R>(h, R(a.omega1), C);
  reconstruct<D2Q9, N, R>(C, f);
  if (active) {
    S* out = dst + int64_t(y) * a.sy + x;
    sfor<0, 9>([&](auto I) { __builtin_nontemporal_store(to_store<S, R>(f[I]), out + int64_t(I) * a.si); });
  }
}

template <class S>
hipError_t step_closure_s(int order, const void* src, void* dst, const StepArgs& a, const uint16_t* packed,
                          const float* params, const float* norm, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, a.ny, 1);
  const int bx = 64 * kClosureNW;
  switch (order) {
    case 2:
      hipLaunchKernelGGL((k_step_closure<2, S>), grid, dim3(bx), 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                         a, packed, params, norm);
      break;
    case 3:
      hipLaunchKernelGGL((k_step_closure<3, S>), grid, dim3(bx), 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                         a, packed, params, norm);
      break;
    case 4:
      hipLaunchKernelGGL((k_step_closure<4, S>), grid, dim3(bx), 0, s, static_cast<const S*>(src), static_cast<S*>(dst),
                         a, packed, params, norm);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
hipError_t features_s(const void* src, float* m, const StepArgs& a, const double* a_target, double plain_weight,
                      float* feat, float* lab, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny;
  const unsigned g = unsigned((nodes + 255) / 256);
  hipLaunchKernelGGL((k_node_moments<S>), dim3(g), dim3(256), 0, s, static_cast<const S*>(src), a, m);
  hipLaunchKernelGGL((k_features<S>), dim3(g), dim3(256), 0, s, static_cast<const S*>(src), m, a, a_target,
                     plain_weight, feat, lab);
  return hipGetLastError();
}

}  // namespace

hipError_t closure_step(int order, int storage, const void* src, void* dst, const StepArgs& a,
                        const uint16_t* packed, const float* params, const float* norm, hipStream_t s) {
  switch (storage) {
    case 0: return step_closure_s<double>(order, src, dst, a, packed, params, norm, s);
    case 1: return step_closure_s<float>(order, src, dst, a, packed, params, norm, s);
    case 2: return step_closure_s<_Float16>(order, src, dst, a, packed, params, norm, s);
  }
  return hipErrorInvalidValue;
}

hipError_t closure_features(int storage, const void* src, float* m, const StepArgs& a, const double* a_target,
                            double plain_weight, float* feat, float* lab, hipStream_t s) {
  switch (storage) {
    case 0: return features_s<double>(src, m, a, a_target, plain_weight, feat, lab, s);
    case 1: return features_s<float>(src, m, a, a_target, plain_weight, feat, lab, s);
    case 2: return features_s<_Float16>(src, m, a, a_target, plain_weight, feat, lab, s);
  }
  return hipErrorInvalidValue;
}

hipError_t closure_coarsen(int dtype, const void* rho, const void* u, const void* pi1, int nfx, int nfy, int F,
                           double alpha, double beta, double* rho_c, double* u_c, double* pi1_c, hipStream_t s) {
  const int64_t nc = int64_t(nfx / F) * (nfy / F);
  const unsigned g = unsigned((nc + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL((k_coarsen<double>), dim3(g), dim3(256), 0, s, static_cast<const double*>(rho),
                       static_cast<const double*>(u), static_cast<const double*>(pi1), nfx, nfy, F, alpha, beta, rho_c, u_c,
                       pi1_c);
  else
    hipLaunchKernelGGL((k_coarsen<float>), dim3(g), dim3(256), 0, s, static_cast<const float*>(rho),
                       static_cast<const float*>(u), static_cast<const float*>(pi1), nfx, nfy, F, alpha, beta, rho_c, u_c,
                       pi1_c);
  return hipGetLastError();
}

hipError_t mlp_pack(const float* params, uint16_t* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((kNPacked + 255) / 256), dim3(256), 0, s, params, packed);
  return hipGetLastError();
}

hipError_t mlp_infer(const float* x, int64_t n, const uint16_t* packed, const float* params, const float* norm,
                     float* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 64 * kInferWaves;
  hipLaunchKernelGGL(k_mlp_infer, dim3(unsigned((n + bs - 1) / bs)), dim3(bs), 0, s, x, n, packed, params, norm, y);
  return hipGetLastError();
}

int mlp_train_blocks(int batch) { return (batch + kTS - 1) / kTS; }

hipError_t column_stats(const float* x, int64_t n, int dim, float* mean, float* sd, hipStream_t s) {
  hipLaunchKernelGGL(k_column_stats, dim3(dim), dim3(256), 0, s, x, n, dim, mean, sd);
  return hipGetLastError();
}

hipError_t mlp_gradient(const float* x, const float* t, int64_t nrows, const int* idx, int batch, const uint16_t* packed,
                        const float* params, const float* norm, float* gpart, float* lpart, float* grad, float* loss,
                        hipStream_t s) {
  const int nb = mlp_train_blocks(batch);
  if (nb <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_train, dim3(nb), dim3(256), 0, s, x, t, nrows, idx, batch, packed, params, norm, gpart,
                     lpart);
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, s, gpart, lpart, nb, batch, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float* p, float* m, float* v, const float* g, long long step, float lr, float b1, float b2,
                    float eps, hipStream_t s) {
  const float c1 = 1.0f - float(std::pow(double(b1), double(step)));
  const float c2 = 1.0f - float(std::pow(double(b2), double(step)));
  hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, p, m, v, g, kNParam, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lbrr
