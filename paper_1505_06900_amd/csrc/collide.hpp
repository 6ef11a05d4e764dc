// Register-resident recursive-regularised collision for one lattice node.
//
// Input: the q pulled pre-collision populations of a node, stored as
// deviations d_i = f_i - w_i rho0.  Output (in place): the post-collision
// deviations of Eq. discr_bgk_reg (Sec. 3.5),
//
//   f_i = w_i sum_{|k| <= N} H_k(xi_i) [a0_k + (1 - 1/tau) a1_k] / N_k,
//
// with a0_k = rho u_x^a u_y^b u_z^c (Sec. 2 and the equilibrium recursion of
// Sec. 3.1), a1^(2) = Pi - rho c_s^2 I - rho u u (Sec. 2, P^(1) = a1^(2)) and
// the higher a1_k from the recursion of Sec. 3.1 (Eq. rel_a1) in its closed
// pair-sum form: every pair of indices of k carries a1^(2), the remaining
// indices carry velocities (App. B lists the same expressions order by order,
// with the discrete O(Ma^(n+1)) terms dropped as the paper does).
//
// Formulation (differs from a dense q x q projection on purpose):
//  * moments and reconstruction of the tensor-product lattices (D2Q9, D3Q27)
//    are done axis by axis with three-point transforms, which folds the
//    weights w_i and the Hermite norms N_k = a! b! c! c_s^(2|k|) into
//    per-axis constants;
//  * D3Q19 has no orthogonal Hermite basis (Sec. 3.2): its kept polynomials
//    are those with at least one zero exponent, and the reconstruction solves
//    with their Gram matrix G_kl = sum_i w_i H_k H_l, computed at compile time,
//    before the same unweighted per-axis transforms and a final w_i.  On D3Q19
//    f1 stops at order 3 (see coefficients).
// Everything is unrolled at compile time; coefficients beyond order N are
// never formed.
#pragma once

#include <type_traits>
#include <utility>

#include "lattice.hpp"

namespace lbrr {

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// Raw moments of the deviations: 0th, 1st and 2nd order.
template <class R>
struct Moments {
  R d0, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
};

// Hydrodynamic state of a node.
template <class R>
struct Hydro {
  R drho, rho, ux, uy, uz, jx, jy, jz;
  R axx, ayy, azz, axy, axz, ayz;  // a1^(2) of the pre-collision populations
};

// ---- moments -------------------------------------------------------------

// Tensor-product lattices: sums along x, then y, then z.  f is indexed by the
// D3Q27 position (cx+1) + 3(cy+1) + 9(cz+1) restricted to the lattice.
template <class L, class R>
__device__ __forceinline__ Moments<R> moments_product(const R* f) {
  constexpr int NZ = (L::D == 3) ? 3 : 1;
  R X[3][3][3];  // X[a][cy][cz] = sum_cx cx^a f
  sfor<0, NZ>([&](auto Z) {
    sfor<0, 3>([&](auto Y) {
      constexpr int base = 3 * Y + 9 * Z;
      const R fm = f[base + 0], f0 = f[base + 1], fp = f[base + 2];
      const R s = fp + fm;
      X[0][Y][Z] = s + f0;
      X[1][Y][Z] = fp - fm;
      X[2][Y][Z] = s;
    });
  });
  R Yv[3][3][3];  // Yv[a][b][cz] = sum_{cx,cy} cx^a cy^b f, a + b <= 2
  sfor<0, NZ>([&](auto Z) {
    sfor<0, 3>([&](auto A) {
      const R m = X[A][0][Z], z0 = X[A][1][Z], p = X[A][2][Z];
      const R s = p + m;
      Yv[A][0][Z] = s + z0;
      if constexpr (A <= 1) Yv[A][1][Z] = p - m;
      if constexpr (A == 0) Yv[A][2][Z] = s;
    });
  });
  Moments<R> r;
  if constexpr (L::D == 2) {
    r.d0 = Yv[0][0][0];
    r.jx = Yv[1][0][0];
    r.jy = Yv[0][1][0];
    r.jz = R(0);
    r.pxx = Yv[2][0][0];
    r.pyy = Yv[0][2][0];
    r.pxy = Yv[1][1][0];
    r.pzz = r.pxz = r.pyz = R(0);
  } else {
    auto zs = [&](int a, int b, R& m0, R& m1, R& m2, int need) {
      const R m = Yv[a][b][0], z0 = Yv[a][b][1], p = Yv[a][b][2];
      const R s = p + m;
      m0 = s + z0;
      if (need >= 1) m1 = p - m;
      if (need >= 2) m2 = s;
    };
    R t0, t1, t2;
    zs(0, 0, r.d0, r.jz, r.pzz, 2);
    zs(1, 0, r.jx, r.pxz, t2, 1);
    zs(0, 1, r.jy, r.pyz, t2, 1);
    zs(2, 0, r.pxx, t1, t2, 0);
    zs(0, 2, r.pyy, t1, t2, 0);
    zs(1, 1, r.pxy, t1, t2, 0);
    (void)t0;
  }
  return r;
}

// Sum over the q velocities of cx^A cy^B cz^C f_i (zero terms dropped at compile time).
template <class L, int A, int B, int C, class R>
__device__ __forceinline__ R moment_direct(const R* f) {
  R s = R(-0.0);  // -0 + x == x exactly, so the first add folds away
  sfor<0, L::Q>([&](auto I) {
    constexpr int p = (A == 0 ? 1 : (A == 1 ? L::cx(I) : L::cx(I) * L::cx(I))) *
                      (B == 0 ? 1 : (B == 1 ? L::cy(I) : L::cy(I) * L::cy(I))) *
                      (C == 0 ? 1 : (C == 1 ? L::cz(I) : L::cz(I) * L::cz(I)));
    if constexpr (p == 1) s = s + f[I];
    if constexpr (p == -1) s = s - f[I];
  });
  return s;
}

template <class L, class R>
__device__ __forceinline__ Moments<R> moments_direct(const R* f) {
  Moments<R> r;
  r.d0 = moment_direct<L, 0, 0, 0>(f);
  r.jx = moment_direct<L, 1, 0, 0>(f);
  r.jy = moment_direct<L, 0, 1, 0>(f);
  r.jz = moment_direct<L, 0, 0, 1>(f);
  r.pxx = moment_direct<L, 2, 0, 0>(f);
  r.pyy = moment_direct<L, 0, 2, 0>(f);
  r.pzz = moment_direct<L, 0, 0, 2>(f);
  r.pxy = moment_direct<L, 1, 1, 0>(f);
  r.pxz = moment_direct<L, 1, 0, 1>(f);
  r.pyz = moment_direct<L, 0, 1, 1>(f);
  return r;
}

// f holds the lattice's q populations in lattice order.
template <class L, class R>
__device__ __forceinline__ Moments<R> raw_moments(const R* f) {
  if constexpr (L::kProduct) {
    // product lattices keep the D3Q27 positions (D2Q9: cz = 0 plane, offset 0)
    return moments_product<L, R>(f);
  } else {
    return moments_direct<L, R>(f);
  }
}

// 1/rho for rho = rho0 + drho rounded: the exact rounding error of the sum
// (two-sum) corrects the reciprocal to first order.  Rounding rho to the
// working precision would otherwise bias u = j/rho by up to half an ulp of
// rho0 at every step, an error that accumulates in time.
template <class R>
__device__ __forceinline__ R inv_density(R rho0, R drho, R rho) {
  const R bb = rho - rho0;
  const R err = (rho0 - (rho - bb)) + (drho - bb);
  const R inv = R(1) / rho;
  return inv - inv * inv * err;
}
// FP32: the hardware reciprocal (within 1 ulp) and one Newton step
// r (2 - rho r) in place of the IEEE division sequence; rho is near rho0, far
// from zero, infinity and the denormals.
__device__ __forceinline__ float inv_density(float rho0, float drho, float rho) {
  const float bb = rho - rho0;
  const float err = (rho0 - (rho - bb)) + (drho - bb);
  float inv = __builtin_amdgcn_rcpf(rho);
  inv = __builtin_fmaf(inv, __builtin_fmaf(-rho, inv, 1.0f), inv);
  return inv - inv * inv * err;
}

// rho, u and a1^(2) = Pi - rho cs2 I - rho u u, written with deviations:
// Pi_ab = P'_ab + rho0 cs2 delta_ab, so a1_ab = P'_ab - drho cs2 delta_ab - j_a u_b.
template <class L, class R>
__device__ __forceinline__ Hydro<R> hydro(const Moments<R>& m, R rho0) {
  constexpr R cs2 = R(kCs2);
  Hydro<R> h;
  h.drho = m.d0;
  h.rho = rho0 + m.d0;
  const R inv = inv_density(rho0, m.d0, h.rho);
  h.jx = m.jx;
  h.jy = m.jy;
  h.ux = m.jx * inv;
  h.uy = m.jy * inv;
  h.axx = m.pxx - m.d0 * cs2 - m.jx * h.ux;
  h.ayy = m.pyy - m.d0 * cs2 - m.jy * h.uy;
  h.axy = m.pxy - m.jx * h.uy;
  if constexpr (L::D == 3) {
    h.jz = m.jz;
    h.uz = m.jz * inv;
    h.azz = m.pzz - m.d0 * cs2 - m.jz * h.uz;
    h.axz = m.pxz - m.jx * h.uz;
    h.ayz = m.pyz - m.jy * h.uz;
  } else {
    h.jz = h.uz = h.azz = h.axz = h.ayz = R(0);
  }
  return h;
}

// ---- Hermite coefficients --------------------------------------------------

// Is multi-index (a, b, c) carried by lattice L at order N?
template <class L, int N>
constexpr bool kept(int a, int b, int c) {
  if (a + b + c > N) return false;
  if (L::D == 2 && c != 0) return false;
  if (!L::kProduct && a > 0 && b > 0 && c > 0) return false;  // D3Q19 basis
  return true;
}

// C[a][b][c] = a0_k + omega1 * a1_k for every kept k (deviation form: C[0][0][0] = drho).
// s_xx .. s_yz are omega1 * a1^(2).
template <class L, int N, class R>
__device__ __forceinline__ void coefficients(const Hydro<R>& h, R omega1, R (&C)[3][3][3]) {
  const R sxx = omega1 * h.axx, syy = omega1 * h.ayy, sxy = omega1 * h.axy;
  const R szz = omega1 * h.azz, sxz = omega1 * h.axz, syz = omega1 * h.ayz;
  const R px[3] = {R(1), h.ux, h.ux * h.ux};
  const R py[3] = {R(1), h.uy, h.uy * h.uy};
  const R pz[3] = {R(1), h.uz, h.uz * h.uz};
  sfor<0, 3>([&](auto A) {
    sfor<0, 3>([&](auto B) {
      sfor<0, 3>([&](auto Cc) {
        constexpr int a = A, b = B, c = Cc;
        if constexpr (kept<L, N>(a, b, c)) {
          constexpr int n = a + b + c;
          if constexpr (n == 0) {
            C[a][b][c] = h.drho;
          } else if constexpr (n == 1) {
            C[a][b][c] = (a == 1) ? h.jx : ((b == 1) ? h.jy : h.jz);
          } else {
            // a0: rho u^k, written as j_d times the remaining velocities
            R e;
            if constexpr (a > 0) e = h.jx * px[a - 1] * py[b] * pz[c];
            else if constexpr (b > 0) e = h.jy * py[b - 1] * pz[c];
            else e = h.jz * pz[c - 1];
            // a1: pair sum of the recursion
            R s = R(-0.0);
            if constexpr (!L::kProduct && n == 4) {
              // D3Q19: f1 stops at order 3 while f0 keeps order 4.  The population
              // vector f1^(3) has, on the fourth-order polynomial H_aabb of D3Q19,
              // the moment -a1_cc / 6 (c the axis with exponent 0): the weights
              // couple H_aabb to H_cc only.  With that value in place of the
              // recursion's a1^(4), the order-4 reconstruction below returns
              // f0^(4) + omega1 f1^(3).  (An f1 at order 4 through the same
              // projection makes the rest state grow for tau near 1/2.)
              s = R(-1.0 / 6.0) * (a == 0 ? sxx : (b == 0 ? syy : szz));
            } else {
              if constexpr (a == 2) s = s + sxx * py[b] * pz[c];
              if constexpr (b == 2) s = s + syy * px[a] * pz[c];
              if constexpr (c == 2) s = s + szz * px[a] * py[b];
              if constexpr (a > 0 && b > 0) s = s + R(a * b) * sxy * px[a - 1] * py[b - 1] * pz[c];
              if constexpr (a > 0 && c > 0) s = s + R(a * c) * sxz * px[a - 1] * py[b] * pz[c - 1];
              if constexpr (b > 0 && c > 0) s = s + R(b * c) * syz * px[a] * py[b - 1] * pz[c - 1];
            }
            C[a][b][c] = e + s;
          }
        }
      });
    });
  });
}

// ---- reconstruction ---------------------------------------------------------

// Three-point transform along one axis.  Weighted (product lattices): values
// w(xi) sum_a h_a(xi) C_a / n_a at xi = -1, 0, 1 with h = (1, xi, xi^2 - 1/3),
// w = (1/6, 2/3, 1/6) and n_a = (1, 1/3, 2/9):
//   g(0) = 2/3 C0 - C2,  g(+-1) = 1/6 C0 +- 1/2 C1 + 1/2 C2.
// Plain (D3Q19, after the Gram solve): g(0) = C0 - C2/3, g(+-1) = C0 +- C1 + 2/3 C2.
// Every multiply-add of the transform is an explicit fused multiply-add, so
// the bits of each output do not depend on which other outputs the caller
// uses (a contraction left to the compiler can change with that).
__device__ __forceinline__ float fused(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fused(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The collision conserves mass and momentum (Sec. 2), and the weighted form
// keeps that in any precision: g(0) is formed first and the outer values share
// what is left of C0, g(+-1) = (C0 - g(0))/2 +- C1/2.  Then g(-1) + g(0) + g(+1)
// returns C0 and g(+1) - g(-1) returns C1 up to the round-to-nearest errors of
// the operations alone.  With the sum 1/6 C0 + 1/2 C2 written out instead, the
// rounded constants give 2 fl(1/6) + fl(2/3) = 1 + 2^-25 in FP32, so that every
// weighted transform would scale the zeroth moment of its input by that
// factor: a systematic growth of the momentum of 2^-24 per step in 3D.
template <bool Weighted, bool Has1, bool Has2, class R>
__device__ __forceinline__ void axis3(R c0, R c1, R c2, R& gm, R& g0, R& gp) {
  if constexpr (Weighted) {
    g0 = Has2 ? fused(R(2.0 / 3.0), c0, -c2) : R(2.0 / 3.0) * c0;
    const R t = R(0.5) * (c0 - g0);
    if constexpr (Has1) {
      gm = fused(R(-0.5), c1, t);
      gp = fused(R(0.5), c1, t);
    } else {
      gm = t;
      gp = t;
    }
  } else {
    R t = c0;
    if constexpr (Has2) t = fused(R(2.0 / 3.0), c2, c0);
    if constexpr (Has1) {
      gm = t - c1;
      gp = t + c1;
    } else {
      gm = t;
      gp = t;
    }
    g0 = Has2 ? fused(R(-1.0 / 3.0), c2, c0) : c0;
  }
}

// w_i v for a lattice whose weights are not dyadic (D3Q19: 1/3, 1/18, 1/36).
// In FP32 the weight is split into its rounded value and the remainder, so the
// product carries one rounding of the exact w_i v: a plainly rounded weight
// would scale every population of its class by the same factor at every step
// (fl(1/18) = (1 + 7.5e-9)/18), a drift of mass and momentum.  In FP64 that
// factor is below 1e-16 and the weight is used as rounded.
template <class L, int I, class R>
__device__ __forceinline__ R times_weight(R v) {
  constexpr double w = L::w(I);
  if constexpr (std::is_same_v<R, float>) {
    constexpr float hi = float(w);
    constexpr float lo = float(w - double(hi));
    return fused(hi, v, lo * v);
  } else {
    return R(w) * v;
  }
}

// Gram matrix of the kept D3Q19 polynomials and its inverse (compile time).
template <int N>
struct GramD3Q19 {
  double inv[27][27];
  static constexpr double h(int n, int c) { return n == 0 ? 1.0 : (n == 1 ? double(c) : double(c * c) - kCs2); }
  constexpr GramD3Q19() : inv{} {
    int ks[27] = {};
    int K = 0;
    for (int p = 0; p < 27; ++p)
      if (kept<D3Q19, N>(p / 9, (p / 3) % 3, p % 3)) ks[K++] = p;
    int vx[D3Q19::Q] = {}, vy[D3Q19::Q] = {}, vz[D3Q19::Q] = {};
    double wv[D3Q19::Q] = {};
    for (int j = 0, i = 0; j < 27; ++j) {  // the 19 non-corner velocities in lattice order
      const int a = j % 3 - 1, b = (j / 3) % 3 - 1, c = j / 9 - 1;
      const int s2 = a * a + b * b + c * c;
      if (s2 > 2) continue;
      vx[i] = a;
      vy[i] = b;
      vz[i] = c;
      wv[i] = s2 == 0 ? 1.0 / 3.0 : (s2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
      ++i;
    }
    double hv[27][D3Q19::Q] = {};  // H_k(xi_i) of the kept polynomials
    for (int r = 0; r < K; ++r)
      for (int i = 0; i < D3Q19::Q; ++i)
        hv[r][i] = h(ks[r] / 9, vx[i]) * h((ks[r] / 3) % 3, vy[i]) * h(ks[r] % 3, vz[i]);
    double g[27][54] = {};
    for (int r = 0; r < K; ++r) {
      for (int s = 0; s < K; ++s) {
        double acc = 0.0;
        for (int i = 0; i < D3Q19::Q; ++i) acc += wv[i] * hv[r][i] * hv[s][i];
        g[r][s] = acc;
      }
      g[r][K + r] = 1.0;
    }
    for (int col = 0; col < K; ++col) {  // Gauss-Jordan with partial pivoting
      int piv = col;
      for (int r = col + 1; r < K; ++r)
        if ((g[r][col] < 0 ? -g[r][col] : g[r][col]) > (g[piv][col] < 0 ? -g[piv][col] : g[piv][col])) piv = r;
      for (int s = 0; s < 2 * K; ++s) {
        const double t = g[col][s];
        g[col][s] = g[piv][s];
        g[piv][s] = t;
      }
      const double d = g[col][col];
      for (int s = 0; s < 2 * K; ++s) g[col][s] /= d;
      for (int r = 0; r < K; ++r) {
        if (r == col) continue;
        const double m = g[r][col];
        for (int s = 0; s < 2 * K; ++s) g[r][s] -= m * g[col][s];
      }
    }
    for (int r = 0; r < K; ++r)
      for (int s = 0; s < K; ++s) {
        double v = g[r][K + s];
        // integers exactly (the rows of the zeroth and first moments are 1 and
        // 3 times the identity), zeros of the sparse inverse exactly
        const double n = double(static_cast<long long>(v < 0 ? v - 0.5 : v + 0.5));
        if (v - n < 1e-12 && v - n > -1e-12) v = n;
        inv[ks[r]][ks[s]] = v;
      }
  }
};

template <int N>
struct GramD3Q19Table {
  static constexpr GramD3Q19<N> t{};
};

// At order 4 the inverse Gram matrix couples the six second-order polynomials
// S_a = H_aa (a = x, y, z) and P_ab = H_aabb through a dense 6 x 6 block that
// is symmetric under permutations of the axes:
//   B[S_a]  = s5 S_a  + t3 T + q2 Q + p3 P_bc    (P_bc: the pair without a)
//   B[P_bc] = p18 P_bc + c2 T + c12 Q + s3 S_a    (S_a: the axis not in the pair)
// with T = S_x + S_y + S_z and Q = P_xy + P_xz + P_yz, so the block takes 20
// operations instead of 36.  The constants are read off the inverse, and
// block_ok checks that every entry of the block has this form.
// The block's entries are multiples of 1/3 up to the rounding of the compile-time inversion.
constexpr double nearest_third(double x) {
  const double n = 3.0 * x;
  return double(static_cast<long long>(n < 0 ? n - 0.5 : n + 0.5)) / 3.0;
}
constexpr bool nearly(double x, double y) { return (x - y < 0 ? y - x : x - y) <= 1e-12 * (1.0 + (y < 0 ? -y : y)); }

struct GramBlock19 {
  static constexpr int S[3] = {18, 6, 2};   // (2,0,0), (0,2,0), (0,0,2)
  static constexpr int P[3] = {8, 20, 24};  // pair without x (0,2,2), without y (2,0,2), without z (2,2,0)
  static constexpr const double (&g)[27][27] = GramD3Q19Table<4>::t.inv;
  static constexpr double t3 = nearest_third(g[S[2]][S[0]]), s5 = nearest_third(g[S[2]][S[2]]) - t3;
  static constexpr double q2 = nearest_third(g[S[2]][P[0]]), p3 = nearest_third(g[S[2]][P[2]]) - q2;
  static constexpr double c2 = nearest_third(g[P[0]][S[1]]), s3 = nearest_third(g[P[0]][S[0]]) - c2;
  static constexpr double c12 = nearest_third(g[P[0]][P[1]]), p18 = nearest_third(g[P[0]][P[0]]) - c12;
  static constexpr bool block_ok() {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        if (!nearly(g[S[a]][S[b]], a == b ? s5 + t3 : t3)) return false;
        if (!nearly(g[S[a]][P[b]], a == b ? q2 + p3 : q2)) return false;
        if (!nearly(g[P[a]][S[b]], a == b ? c2 + s3 : c2)) return false;
        if (!nearly(g[P[a]][P[b]], a == b ? c12 + p18 : c12)) return false;
      }
    return true;
  }
  static constexpr bool in_block(int p) { return p == 2 || p == 6 || p == 18 || p == 8 || p == 20 || p == 24; }
};
static_assert(GramBlock19::block_ok(), "the order-4 D3Q19 Gram block has the axis-symmetric form");

// D3Q19 in FP32: the reconstruction does not keep the zeroth and first
// moments exactly.  The constants 2/3 and 1/3 of its plain transforms are
// rounded, which shifts the fractional bits of every rounding that follows
// the same way, and mass and momentum drift by about 1e-11 per node and step.
// The weights are not products, so no per-axis form holds them by
// construction as in the weighted transform.  Instead the populations are
// made to carry the node's own moments, which the collision conserves
// (Sec. 2):
//  * z momentum: the faces (0, 0, +-1) take the part of j_z the other
//    populations of the c_z = +-1 layers lack, half each, keeping their sum;
//  * x and y momentum: the same with the faces (+-1, 0, 0) and (0, +-1, 0);
//  * mass: the rest population is drho minus the sum of the other 18.
// Each is one rounding of a plain sum, with no constant in it.  Only the
// c_z = +-1 layers enter the z step and only layer c_z = 0 is changed after
// it.  A layer-selected rebuild (ZSel = +-1) therefore computes both c_z = +-1
// layers and gets the same bits for them as a full one.
// Lattice index of velocity (cx, cy, cz) (-1 if the lattice lacks it).
template <class L>
constexpr int velocity_index(int cx, int cy, int cz) {
  for (int i = 0; i < L::Q; ++i)
    if (L::cx(i) == cx && L::cy(i) == cy && L::cz(i) == cz) return i;
  return -1;
}

template <class L, class R>
__device__ __forceinline__ void conserve_layers(const R (&C)[3][3][3], R* out) {
  constexpr int zp = velocity_index<L>(0, 0, 1), zm = velocity_index<L>(0, 0, -1);
  R e = R(-0.0);  // z momentum of the c_z = +-1 populations other than the two faces
  sfor<0, L::Q>([&](auto I) {
    if constexpr (I != zp && I != zm) {
      if constexpr (L::cz(I) == 1) e = e + out[I];
      if constexpr (L::cz(I) == -1) e = e - out[I];
    }
  });
  const R s = out[zp] + out[zm];
  const R d = C[0][0][1] - e;  // what the faces must carry: out[zp] - out[zm]
  out[zp] = R(0.5) * (s + d);
  out[zm] = R(0.5) * (s - d);
}

template <class L, class R>
__device__ __forceinline__ void conserve_plane(const R (&C)[3][3][3], R* out) {
  constexpr int xp = velocity_index<L>(1, 0, 0), xm = velocity_index<L>(-1, 0, 0);
  constexpr int yp = velocity_index<L>(0, 1, 0), ym = velocity_index<L>(0, -1, 0);
  constexpr int rest = velocity_index<L>(0, 0, 0);
  R ex = R(-0.0), ey = R(-0.0);
  sfor<0, L::Q>([&](auto I) {
    if constexpr (I != xp && I != xm) {
      if constexpr (L::cx(I) == 1) ex = ex + out[I];
      if constexpr (L::cx(I) == -1) ex = ex - out[I];
    }
    if constexpr (I != yp && I != ym) {
      if constexpr (L::cy(I) == 1) ey = ey + out[I];
      if constexpr (L::cy(I) == -1) ey = ey - out[I];
    }
  });
  const R sx = out[xp] + out[xm], dx = C[1][0][0] - ex;
  out[xp] = R(0.5) * (sx + dx);
  out[xm] = R(0.5) * (sx - dx);
  const R sy = out[yp] + out[ym], dy = C[0][1][0] - ey;
  out[yp] = R(0.5) * (sy + dy);
  out[ym] = R(0.5) * (sy - dy);
  R m = R(-0.0);
  sfor<0, L::Q>([&](auto I) {
    if constexpr (I != rest) m = m + out[I];
  });
  out[rest] = C[0][0][0] - m;
}

// Layer c_z = z - 1 is computed by a reconstruction with layer selection ZSel.
template <bool Conserve, int ZSel>
constexpr bool layer_needed(int z) {
  return ZSel == 2 || z == ZSel + 1 || (Conserve && z != 1);
}

// Post-collision deviations of the lattice's q populations from C.  With
// ZSel = -1 or +1 (3D) the populations with c_z = ZSel are written (D3Q19 in
// FP32 writes both c_z = +-1 layers, see conserve_layers; other entries of
// out are left untouched); ZSel = 2 writes all q.
template <class L, int N, class R, int ZSel = 2>
__device__ __forceinline__ void reconstruct(R (&C)[3][3][3], R* out) {
  static_assert(ZSel == 2 || (L::D == 3 && (ZSel == -1 || ZSel == 1)), "layer selection is 3D only");
  constexpr bool W = L::kProduct;
  constexpr bool kConserve = !W && std::is_same_v<R, float>;
  R B[3][3][3];
  if constexpr (W) {
    sfor<0, 27>([&](auto P) {
      constexpr int a = P / 9, b = (P / 3) % 3, c = P % 3;
      if constexpr (kept<L, N>(a, b, c)) B[a][b][c] = C[a][b][c];
    });
  } else {
    // D3Q19: B = G^-1 C over the kept polynomials (order 4: the second-order
    // block in its axis-symmetric form, GramBlock19)
    constexpr bool kBlock = N >= 4;
    sfor<0, 27>([&](auto P) {
      constexpr int a = P / 9, b = (P / 3) % 3, c = P % 3;
      if constexpr (kept<L, N>(a, b, c) && !(kBlock && GramBlock19::in_block(P))) {
        R s = R(-0.0);
        sfor<0, 27>([&](auto S) {
          constexpr int a2 = S / 9, b2 = (S / 3) % 3, c2 = S % 3;
          if constexpr (kept<L, N>(a2, b2, c2)) {
            constexpr double g = GramD3Q19Table<N>::t.inv[P][S];
            if constexpr (g != 0.0) s = fused(R(g), C[a2][b2][c2], s);
          }
        });
        B[a][b][c] = s;
      }
    });
    if constexpr (kBlock) {
      static_assert(N == 4, "the D3Q19 basis stops at order 4");
      using G = GramBlock19;
      const R sx = C[2][0][0], sy = C[0][2][0], sz = C[0][0][2];
      const R px = C[0][2][2], py = C[2][0][2], pz = C[2][2][0];  // pair without x, y, z
      const R T = sx + sy + sz, Q = px + py + pz;
      const R cs = fused(R(G::t3), T, R(G::q2) * Q), cp = fused(R(G::c2), T, R(G::c12) * Q);
      B[2][0][0] = fused(R(G::s5), sx, fused(R(G::p3), px, cs));
      B[0][2][0] = fused(R(G::s5), sy, fused(R(G::p3), py, cs));
      B[0][0][2] = fused(R(G::s5), sz, fused(R(G::p3), pz, cs));
      B[0][2][2] = fused(R(G::p18), px, fused(R(G::s3), sx, cp));
      B[2][0][2] = fused(R(G::p18), py, fused(R(G::s3), sy, cp));
      B[2][2][0] = fused(R(G::p18), pz, fused(R(G::s3), sz, cp));
    }
  }
  // stage z: B[a][b][*] -> G1[a][b][cz]
  constexpr int NZ = (L::D == 3) ? 3 : 1;
  R G1[3][3][3];
  sfor<0, 3>([&](auto A) {
    sfor<0, 3>([&](auto Bi) {
      constexpr int a = A, b = Bi;
      if constexpr (kept<L, N>(a, b, 0)) {
        if constexpr (L::D == 3) {
          constexpr bool h1 = kept<L, N>(a, b, 1), h2 = kept<L, N>(a, b, 2);
          axis3<W, h1, h2>(B[a][b][0], h1 ? B[a][b][1] : R(0), h2 ? B[a][b][2] : R(0),
                           G1[a][b][0], G1[a][b][1], G1[a][b][2]);
        } else {
          G1[a][b][0] = B[a][b][0];
        }
      }
    });
  });
  // presence of G1[a][b][*]: some kept (a, b, c)
  // stage y: G1[a][*][cz] -> G2[a][cy][cz]
  R G2[3][3][3];
  sfor<0, 3>([&](auto A) {
    sfor<0, NZ>([&](auto Z) {
      constexpr int a = A;
      if constexpr (kept<L, N>(a, 0, 0) && layer_needed<kConserve, ZSel>(int(Z))) {
        constexpr bool h1 = kept<L, N>(a, 1, 0), h2 = kept<L, N>(a, 2, 0);
        axis3<W, h1, h2>(G1[a][0][Z], h1 ? G1[a][1][Z] : R(0), h2 ? G1[a][2][Z] : R(0),
                         G2[a][0][Z], G2[a][1][Z], G2[a][2][Z]);
      }
    });
  });
  // stage x: G2[*][cy][cz] -> populations; D3Q19 multiplies by w_i and skips corners
  sfor<0, NZ>([&](auto Z) {
    if constexpr (layer_needed<kConserve, ZSel>(int(Z))) sfor<0, 3>([&](auto Y) {
      R gm, g0, gp;
      axis3<W, true, true>(G2[0][Y][Z], G2[1][Y][Z], G2[2][Y][Z], gm, g0, gp);
      sfor<0, L::Q>([&](auto I) {
        if constexpr (L::cy(I) + 1 == Y && L::cz(I) + 1 == (L::D == 3 ? int(Z) : 1)) {
          const R v = (L::cx(I) == -1) ? gm : ((L::cx(I) == 0) ? g0 : gp);
          if constexpr (W) out[I] = v;
          else out[I] = times_weight<L, int(I)>(v);
        }
      });
    });
  });
  if constexpr (kConserve) {
    conserve_layers<L>(C, out);
    if constexpr (ZSel == 2) conserve_plane<L>(C, out);
  }
}

// In-place collision of one node's deviations.
template <class L, int N, class R>
__device__ __forceinline__ Hydro<R> collide(R* f, R rho0, R omega1) {
  const Moments<R> m = raw_moments<L, R>(f);
  const Hydro<R> h = hydro<L, R>(m, rho0);
  R C[3][3][3];
  coefficients<L, N, R>(h, omega1, C);
  reconstruct<L, N, R>(C, f);
  return h;
}

}  // namespace lbrr
