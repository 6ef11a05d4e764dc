// Learned a1^(2) closure for coarse D2Q9 runs (not part of the paper): data
// kernels (coarse-graining of fine fields, next-step features), MLP training
// (forward + backward on the matrix cores, per-block partial gradients, fixed-
// order reduction, Adam), batched inference, and the fused coarse step that
// adds the predicted correction to a1^(2) before the recursion of Sec. 3.1
// rebuilds the higher-order coefficients (Eq. rel_a1) and the populations are
// reconstructed (Eq. discr_bgk_reg).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
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

// Standardised BF16 features of one sample into its LDS row (kInP values,
// inputs kIn .. kInP - 1 zero): (x - mean) * (1 / std).
__device__ __forceinline__ void write_features(const float (&feat)[kIn], const float* mean, const float* inv,
                                               uint16_t* row) {
  bf16x4* xr = reinterpret_cast<bf16x4*>(row);
  float v[kInP];
#pragma unroll
  for (int k = 0; k < kInP; ++k) v[k] = k < kIn ? (feat[k] - mean[k]) * inv[k] : 0.0f;
#pragma unroll
  for (int k4 = 0; k4 < kInP / 4; ++k4) xr[k4] = pack_bf16(v[4 * k4], v[4 * k4 + 1], v[4 * k4 + 2], v[4 * k4 + 3]);
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
// activation regions; c: constants.  The barriers wait for LDS only, so global
// loads a caller issued before the call stay in flight through it.
template <int NW>
__device__ __forceinline__ void forward_group(const float (&feat)[kIn], int part, const uint16_t* w, uint16_t* r0,
                                              uint16_t* r1, const float* c, float (&out)[kOut]) {
  const int lane = threadIdx.x & 63, q = lane >> 4;
  if (part == 0) {  // standardised BF16 features, row = sample (stride kLd1, inputs 36..47 zero)
    write_features(feat, c + kCMean, c + kCInv, r0 + lane * kLd1);
  }
  lds_barrier();
  // layer 1: H1 = gelu(W1 X + b1), 4 x 4 tiles (features j0, samples s0) -> r1
#pragma unroll
  for (int t = part; t < 16; t += NW) {
    const int j0 = 16 * (t & 3), s0 = 16 * (t >> 2), j = j0 + 4 * q;
    f32x4 acc = *reinterpret_cast<const f32x4*>(c + kCB1 + j);
    acc = tile_kc<kInP>(w + kPW1, kLd1, r0, kLd1, j0, s0, acc);
    *reinterpret_cast<bf16x4*>(r1 + (s0 + (lane & 15)) * kLdH + j) =
        pack_bf16(gelu(acc[0]), gelu(acc[1]), gelu(acc[2]), gelu(acc[3]));
  }
  lds_barrier();
  // layer 2: H2 = gelu(W2 H1 + b2) -> r0
#pragma unroll
  for (int t = part; t < 16; t += NW) {
    const int j0 = 16 * (t & 3), s0 = 16 * (t >> 2), j = j0 + 4 * q;
    f32x4 acc = *reinterpret_cast<const f32x4*>(c + kCB2 + j);
    acc = tile_kc<kH>(w + kPW2, kLdH, r1, kLdH, j0, s0, acc);
    *reinterpret_cast<bf16x4*>(r0 + (s0 + (lane & 15)) * kLdH + j) =
        pack_bf16(gelu(acc[0]), gelu(acc[1]), gelu(acc[2]), gelu(acc[3]));
  }
  lds_barrier();
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
  lds_barrier();
  if (part == 0) {
#pragma unroll
    for (int o = 0; o < kOut; ++o) out[o] = ys[lane * 4 + o] * c[kCYStd + o] + c[kCYMean + o];
  }
  lds_barrier();
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
// Matrix-core operands of the fused step: the 16 x 16 x 32 BF16 product, whose
// lane l supplies eight consecutive k of row (A) or column (B) l % 16 from k
// offset 8 (l / 16) of a 32-wide chunk.  A and B take the same k assignment,
// so the product sums matching pairs whatever order the hardware uses.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 join8(bf16x4 lo, bf16x4 hi) {
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Eight BF16 values at k = 32 c + 8 q of a row (p: the row's start, 8-byte
// aligned), zero where k >= kv (the zero padding of a shorter operand).
__device__ __forceinline__ bf16x8 operand8(const uint16_t* p, int c, int q, int kv) {
  const bf16x4* v = reinterpret_cast<const bf16x4*>(p + 32 * c + 8 * q);
  const bf16x8 x = join8(v[0], v[1]);
  return 32 * c + 8 * q < kv ? x : bf16x8{};
}

// v mod n for v >= -1 (periodic index of a halo node): one compare and add
// or subtract in the usual case, the division only for axes shorter than the
// tile and its halo.
__device__ __forceinline__ int wrap(int v, int n) {
  if (v < 0) v += n;
  if (v >= n) v -= n;
  return v < n ? v : v % n;
}

constexpr int kClosureRows = 4;
constexpr int kClosureSamples = 64 * kClosureRows;
constexpr int kClosureHalo = (kClosureRows + 2) * 66;  // nodes whose moments the features read

// A operand of a product whose k runs over the 64 outputs of the previous
// layer as the matrix cores leave them in registers: lane (q, l16) holds rows
// 4 q .. 4 q + 3 of each 16-row output tile, so chunk c of the next product
// takes elements 0..3 from tile 2 c and 4..7 from tile 2 c + 1, i.e.
// k = 32 c + 16 (i / 4) + 4 q + i % 4.  row: the weight row (output feature).
__device__ __forceinline__ bf16x8 operand8_tiles(const uint16_t* row, int c, int q) {
  const bf16x4* v = reinterpret_cast<const bf16x4*>(row + 32 * c + 4 * q);
  return join8(v[0], v[4]);
}

// The fused step's weight operands as its lanes hold them: operand o (0-7:
// W1 tile jt = o / 2, chunk c = o % 2; 8-15: W2 likewise; 16-17: W3 chunk c),
// lane (q, l16), eight BF16 values: image[(o * 64 + lane) * 8 + e].  A lane
// then fetches each operand with one 16-byte load, the wave's 64 loads of an
// operand being one contiguous KiB.  Built from the packed weights.
constexpr int kNOps = 18;
static_assert(kMlpNRegImage == kNOps * 64 * 8, "closure.hpp sizes");

__device__ __forceinline__ bf16x8 step_operand(const uint16_t* packed, int o, int lane) {
  const int q = lane >> 4, l16 = lane & 15;
  if (o < 8) return operand8(packed + kPW1 + (16 * (o >> 1) + l16) * kLd1, o & 1, q, kInP);
  if (o < 16) return operand8_tiles(packed + kPW2 + (16 * ((o - 8) >> 1) + l16) * kLdH, o & 1, q);
  return operand8_tiles(packed + kPW3 + l16 * kLdH, o - 16, q);
}

__global__ void __launch_bounds__(64) k_pack_image(const uint16_t* __restrict__ packed, bf16x8* __restrict__ image) {
  const int o = blockIdx.x;  // one operand per block, one lane per thread
  image[o * 64 + threadIdx.x] = step_operand(packed, o, int(threadIdx.x));
}

// Fused coarse D2Q9 step with the closure: pull, moments, features, MLP on the
// matrix cores, a1^(2) += predicted correction, recursion and reconstruction,
// store.  A block owns 64 columns of kClosureRows consecutive rows and has WPR
// waves per row.  The row's first wave (w < kClosureRows, row y0 + w) pulls,
// and later collides, its 64 nodes (one node per lane; lanes past the row end,
// or on rows past the last, use a wrapped node and do not store).
// (rho - rho0, u) of the stored state on those rows and a one-node halo go to
// LDS for the neighbour features.  The row's WPR waves then share the MLP of
// its 64 samples, 16 at a time (its wave p = w / kClosureRows takes the 4 / WPR
// tiles from p (4 / WPR) on), with every weight and bias in registers: a
// layer's products leave each lane four consecutive outputs of one sample,
// which after the activation are the next layer's operand as they stand
// (operand8_tiles orders the weights to match), so only the standardised
// inputs and the three outputs pass through LDS.  The barriers wait for LDS
// only: the pulled populations stay in flight until the collision.
template <int N, class S, int WPR>
__global__ void __launch_bounds__(kClosureSamples * WPR)
    k_step_closure(const S* __restrict__ src, S* __restrict__ dst, StepArgs a, const uint16_t* __restrict__ packed,
                   const float* __restrict__ params, const float* __restrict__ norm) {
  using R = typename Prec<S>::R;
  constexpr int kThreads = kClosureSamples * WPR, kTiles = 4 / WPR;  // sample tiles of 16 per wave
  // standardised BF16 inputs; the padding keeps the operand reads of k 48 .. 63 (set to zero) of the last row inside
  __shared__ __attribute__((aligned(16))) uint16_t xs[kClosureSamples * kLd1 + 16];
  __shared__ __attribute__((aligned(16))) float ys[kClosureSamples][4];            // network outputs
  __shared__ __attribute__((aligned(16))) float cst[kNNorm];  // x_mean, 1 / x_std, y_mean, y_std
  __shared__ __attribute__((aligned(16))) float nb[kClosureRows + 2][66][4];  // (rho - rho0, u_x, u_y, -)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, l16 = lane & 15;
  // the row's waves share its 64 samples (one wave per row: row = wave, part 0)
  const int row = WPR == 1 ? wave : wave % kClosureRows, part = WPR == 1 ? 0 : wave / kClosureRows;
  const bool owner = part == 0;  // the wave that pulls and collides the row
  const int gx = (a.nx + 63) / 64;
  const int x0 = int(blockIdx.x % unsigned(gx)) * 64, y0 = int(blockIdx.x / unsigned(gx)) * kClosureRows;
  const int xr = x0 + lane, yr = y0 + row;
  const bool active = owner && xr < a.nx && yr < a.ny;
  const int x = xr < a.nx ? xr : xr % a.nx, y = yr < a.ny ? yr : yr % a.ny;
  // global loads first: one normalisation constant per thread, the lane's
  // pulled populations, the stored populations of the halo nodes, then the
  // weight operands and biases (consumed in this order, so that no wait for
  // one load waits for a later one; at most 56 loads in flight per wave)
  const float nv = threadIdx.x < kNNorm ? norm[threadIdx.x] : 0.0f;
  R f[9];
  if (owner) pull9<S, R>(src, a, x, y, f);
  constexpr int kPer = (kClosureHalo + kThreads - 1) / kThreads;
  R p[kPer][9];
#pragma unroll
  for (int h = 0; h < kPer; ++h) {
    const int k = int(threadIdx.x) + h * kThreads;
    if (k < kClosureHalo) {
      const int64_t off = int64_t(wrap(y0 - 1 + k / 66, a.ny)) * a.sy + wrap(x0 - 1 + k % 66, a.nx);
      sfor<0, 9>([&](auto I) { p[h][I] = R(src[int64_t(I) * a.si + off]); });
    }
  }
  // A operands (rows: output features 16 jt + l16) from the register image,
  // one 16-byte load each, and the biases that start the accumulators
  const bf16x8* img = reinterpret_cast<const bf16x8*>(packed + kNPacked) + lane;
  bf16x8 w1[4][2], w2[4][2], w3[2];
  f32x4 b1[4], b2[4];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      w1[jt][c] = img[(2 * jt + c) * 64];
      w2[jt][c] = img[(8 + 2 * jt + c) * 64];
    }
    b1[jt] = *reinterpret_cast<const f32x4*>(params + kOffB1 + 16 * jt + 4 * q);
    b2[jt] = *reinterpret_cast<const f32x4*>(params + kOffB2 + 16 * jt + 4 * q);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) w3[c] = img[(16 + c) * 64];
  const f32x4 b3 = q == 0 ? f32x4{params[kOffB3], params[kOffB3 + 1], params[kOffB3 + 2], 0.0f} : f32x4{0, 0, 0, 0};
  if (threadIdx.x < kNNorm) cst[threadIdx.x] = (threadIdx.x >= kIn && threadIdx.x < 2 * kIn) ? 1.0f / nv : nv;
  // halo moments -> LDS
#pragma unroll
  for (int h = 0; h < kPer; ++h) {
    const int k = int(threadIdx.x) + h * kThreads;
    if (k < kClosureHalo) {
      const Moments<R> mo = raw_moments<D2Q9, R>(p[h]);
      const Hydro<R> hh = hydro<D2Q9, R>(mo, R(a.rho0));
      *reinterpret_cast<f32x4*>(&nb[k / 66][k % 66][0]) = f32x4{float(hh.drho), float(hh.ux), float(hh.uy), 0.0f};
    }
  }
  lds_barrier();
  // features of the lane's node -> its row of xs
  if (owner) {
    float feat[kIn];
#pragma unroll
    for (int i = 0; i < 9; ++i) feat[i] = float(f[i]);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(&nb[row + dy][lane + dx][0]);
#pragma unroll
        for (int c = 0; c < 3; ++c) feat[9 + 3 * (3 * dy + dx) + c] = v[c];
      }
    write_features(feat, cst, cst + kIn, xs + (64 * row + lane) * kLd1);
  }
  lds_barrier();
  // the MLP of the wave's samples, 16 at a time (tile st: samples 64 row + 16 st + l16)
#pragma unroll
  for (int t = 0; t < kTiles; ++t) {
    const int st = part * kTiles + t;
    const uint16_t* xrow = xs + (64 * row + 16 * st + l16) * kLd1;
    const bf16x8 x1[2] = {operand8(xrow, 0, q, kInP), operand8(xrow, 1, q, kInP)};
    bf16x4 h[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {  // H1 = gelu(W1 X + b1)
      f32x4 acc = b1[jt];
#pragma unroll
      for (int c = 0; c < 2; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[jt][c], x1[c], acc, 0, 0, 0);
      h[jt] = pack_bf16(gelu(acc[0]), gelu(acc[1]), gelu(acc[2]), gelu(acc[3]));
    }
    const bf16x8 x2[2] = {join8(h[0], h[1]), join8(h[2], h[3])};
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {  // H2 = gelu(W2 H1 + b2)
      f32x4 acc = b2[jt];
#pragma unroll
      for (int c = 0; c < 2; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[jt][c], x2[c], acc, 0, 0, 0);
      h[jt] = pack_bf16(gelu(acc[0]), gelu(acc[1]), gelu(acc[2]), gelu(acc[3]));
    }
    const bf16x8 x3[2] = {join8(h[0], h[1]), join8(h[2], h[3])};
    f32x4 acc = b3;  // Y = W3 H2 + b3: rows 0..2 of the tile, in lanes 0..15
#pragma unroll
    for (int c = 0; c < 2; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[c], x3[c], acc, 0, 0, 0);
    if (q == 0) *reinterpret_cast<f32x4*>(&ys[64 * row + 16 * st + l16][0]) = acc;
  }
  lds_barrier();
  if (!owner) return;
  const f32x4 yv = *reinterpret_cast<const f32x4*>(&ys[64 * row + lane][0]);
  const Moments<R> mo = raw_moments<D2Q9, R>(f);
  Hydro<R> h = hydro<D2Q9, R>(mo, R(a.rho0));
  const float* ym = cst + 2 * kIn;
  const float* ysd = ym + kOut;
  h.axx += R(yv[0] * ysd[0] + ym[0]);
  h.axy += R(yv[1] * ysd[1] + ym[1]);
  h.ayy += R(yv[2] * ysd[2] + ym[2]);
  R C[3][3][3];
  coefficients<D2Q9, N, R>(h, R(a.omega1), C);
  reconstruct<D2Q9, N, R>(C, f);
  if (active) {
    S* out = dst + int64_t(y) * a.sy + x;
    sfor<0, 9>([&](auto I) { __builtin_nontemporal_store(to_store<S, R>(f[I]), out + int64_t(I) * a.si); });
  }
}

template <class S, int WPR>
hipError_t launch_closure(int order, dim3 grid, const void* src, void* dst, const StepArgs& a, const uint16_t* packed,
                          const float* params, const float* norm, hipStream_t s) {
  const dim3 block(kClosureSamples * WPR);
  switch (order) {
    case 2:
      hipLaunchKernelGGL((k_step_closure<2, S, WPR>), grid, block, 0, s, static_cast<const S*>(src),
                         static_cast<S*>(dst), a, packed, params, norm);
      break;
    case 3:
      hipLaunchKernelGGL((k_step_closure<3, S, WPR>), grid, block, 0, s, static_cast<const S*>(src),
                         static_cast<S*>(dst), a, packed, params, norm);
      break;
    case 4:
      hipLaunchKernelGGL((k_step_closure<4, S, WPR>), grid, block, 0, s, static_cast<const S*>(src),
                         static_cast<S*>(dst), a, packed, params, norm);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
hipError_t step_closure_s(int order, const void* src, void* dst, const StepArgs& a, const uint16_t* packed,
                          const float* params, const float* norm, hipStream_t s) {
  const int64_t blocks = int64_t((a.nx + 63) / 64) * ((a.ny + kClosureRows - 1) / kClosureRows);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid = dim3(unsigned(blocks));
  if constexpr (sizeof(S) == 8) {  // FP64 storage keeps one wave per row: two would spill
    return launch_closure<S, 1>(order, grid, src, dst, a, packed, params, norm, s);
  } else {
    // grids that give at most one block per compute unit leave one wave per SIMD: two waves per row there
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int wpr = blocks <= cus ? 2 : 1;
    if (const char* e = std::getenv("LBRR_CLOSURE_WPR")) {  // 1 or 2; other values are ignored
      const int v = std::atoi(e);
      if (v == 1 || v == 2) wpr = v;
    }
    return wpr == 2 ? launch_closure<S, 2>(order, grid, src, dst, a, packed, params, norm, s)
                    : launch_closure<S, 1>(order, grid, src, dst, a, packed, params, norm, s);
  }
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

hipError_t mlp_pack_step(const float* params, uint16_t* packed_and_image, hipStream_t s) {
  if (hipError_t e = mlp_pack(params, packed_and_image, s); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack_image, dim3(kNOps), dim3(64), 0, s, packed_and_image,
                     reinterpret_cast<bf16x8*>(packed_and_image + kNPacked));
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
