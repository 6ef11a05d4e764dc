// Moment-state form of the regularised update.
//
// After the collision of Eq. discr_bgk_reg every population of a node is a
// function of that node's rho, u and a1^(2) alone: f0 from a0_k = rho u^k and
// f1 from a1^(2) through the recursion of Sec. 3.1 (Eq. rel_a1), both
// reconstructed as in Sec. 3.2.  The state of a lattice node can therefore be
// stored as its pre-collision moments
//     m = (rho - rho0, j = rho u, a1^(2))       10 values in 3D, 6 in 2D,
// instead of q populations, and one step of the scheme becomes: rebuild the
// post-collision populations of every node from m, stream them (pull), and
// take the moments of the populations that arrive.  This is the same update
// in exact arithmetic, with 2 x 10 instead of 2 x 27 stored values moved per
// D3Q27 node update.
//
// Storage: field c of node (x, y, z) at element c*si + z*sz + y*sy + x.
// 3D fields: drho, jx, jy, jz, axx, ayy, azz, axy, axz, ayz; 2D: drho, jx,
// jy, axx, ayy, axy.  FP64 or FP32; the collision runs in the same precision.
//
// Step kernel (3D): a block rebuilds the populations of an MX x TY patch of
// nodes of one z-plane (64 x 8 in FP32, 32 x 8 in FP64: 55 KiB of LDS),
// exchanges them through LDS, and the inner (MX-2) x (TY-2) nodes pull
// theirs.  The block marches along z through a chunk of planes: the
// populations rebuilt on plane p with c_z = -1, 0, +1 arrive on planes p-1,
// p, p+1, so each inner thread keeps running moment sums for three target
// planes, and plane p-1 is complete once plane p has been rebuilt.  A chunk of
// lz target planes rebuilds lz + 2 planes; a patch rebuilds its one-node halo
// ring as well.  The halo and chunk overlaps are the price of the 2.7x smaller
// state: about 2 rebuilds per node update and about twice the algorithmic
// bytes read, so the kernel is held by the rebuild arithmetic and by that
// traffic together, not by the stored bytes.  The 2D step (k_mstep2) does the
// same one dimension lower: a row of kRowX nodes marching along y.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace lbrr {

template <class L>
constexpr int kNM = (L::D == 3) ? 10 : 6;

// Patch of rebuilt nodes per block of the 3D step: MX x TY.  A row of the
// patch is read as MX consecutive values of each field starting one node
// before a tile, so it spans one 128-byte line more than it needs; 64 wide,
// that is 3 lines for 62 outputs (FP32) instead of 2 for 30.  Measured,
// D3Q27 FP32 (GLUPS, best chunk length): 32 x 16 patches 36.5 / 33.3 / 30.5
// at 256^3 / 384^3 / 512^3 (the larger boxes only with contiguous tile
// ranges per XCD, otherwise falling to 21-27 past a plane-size threshold),
// 64 x 8 patches 37.1 / 39.8 / 40.8 at 6 planes per chunk in plain block
// order, 64 x 16 (1024 threads) spills registers and ran 33.6-39.1.
template <class S>
struct MPatch {
  static constexpr int MX = sizeof(S) == 4 ? 64 : 32, TY = 8;
};
constexpr int kPrefetch = 2;  // planes of moments in flight ahead of the rebuild

// 2D: nodes per rebuilt row of a block.  Measured, D2Q9 order 4 FP32, GLUPS at
// 2 / 4 / 8 / 16 rows per chunk: 2048^2 rows of 128: 81 / 86 / 82 / 79, of 256:
// 86 / 93 / 89 / 81, of 512: 76 / 81 / 85 / 76; 4096^2 rows of 256: 93 / 100 /
// 94 / 85, of 512: 92 / 102 / 98 / 90 (population storage: 84 and 87).  The
// host picks 4 rows per chunk.
constexpr int kRowX = 256;

// Hydrodynamic state of a node from its stored moments m.
template <class L, class R>
__device__ __forceinline__ Hydro<R> state_hydro(const R (&m)[kNM<L>], R rho0) {
  Hydro<R> h;
  h.drho = m[0];
  h.rho = rho0 + m[0];
  const R inv = inv_density(rho0, m[0], h.rho);
  h.jx = m[1];
  h.jy = m[2];
  h.ux = m[1] * inv;
  h.uy = m[2] * inv;
  if constexpr (L::D == 3) {
    h.jz = m[3];
    h.uz = m[3] * inv;
    h.axx = m[4];
    h.ayy = m[5];
    h.azz = m[6];
    h.axy = m[7];
    h.axz = m[8];
    h.ayz = m[9];
  } else {
    h.jz = h.uz = R(0);
    h.axx = m[3];
    h.ayy = m[4];
    h.axy = m[5];
    h.azz = h.axz = h.ayz = R(0);
  }
  return h;
}

// Stored moments of a node from the moment sums of its arrived populations.
template <class L, class R>
__device__ __forceinline__ void finalize_state(const Moments<R>& s, R rho0, R (&m)[kNM<L>]) {
  const Hydro<R> h = hydro<L, R>(s, rho0);
  m[0] = s.d0;
  m[1] = s.jx;
  m[2] = s.jy;
  if constexpr (L::D == 3) {
    m[3] = s.jz;
    m[4] = h.axx;
    m[5] = h.ayy;
    m[6] = h.azz;
    m[7] = h.axy;
    m[8] = h.axz;
    m[9] = h.ayz;
  } else {
    m[3] = h.axx;
    m[4] = h.ayy;
    m[5] = h.axy;
  }
}

template <class R>
__device__ __forceinline__ void clear(Moments<R>& s) {
  s.d0 = s.jx = s.jy = s.jz = s.pxx = s.pyy = s.pzz = s.pxy = s.pxz = s.pyz = R(0);
}

// Does the lattice carry velocity (cx, cy, cz)?
template <class L>
constexpr bool has_velocity(int cx, int cy, int cz) {
  if (L::D == 2 && cz != 0) return false;
  if (!L::kProduct && cx != 0 && cy != 0 && cz != 0) return false;
  return true;
}

// Add the populations of the layer c_z = CZ that arrive at inner node (tx, ty)
// to its moment sums s: population (cx, cy, CZ) comes from patch node
// (tx - cx, ty - cy).  Sums along x, then y, then the c_z factors.
template <class L, int CZ, int TY, int MX, class R, bool Assign = false>
__device__ __forceinline__ void add_layer(Moments<R>& s, const R (*pop)[TY][MX], int tx, int ty) {
  R r0[3], r1[3], r2[3];  // per row cy: sum of v, cx v, cx^2 v
  sfor<0, 3>([&](auto Y) {
    constexpr int cy = int(Y) - 1;
    R v[3];
    sfor<0, 3>([&](auto X) {
      constexpr int cx = int(X) - 1;
      if constexpr (has_velocity<L>(cx, cy, CZ)) v[X] = pop[velocity_index<L>(cx, cy, CZ)][ty - cy][tx - cx];
      else v[X] = R(0);
    });
    constexpr bool side = has_velocity<L>(-1, cy, CZ);  // the +-1 entries come in pairs
    if constexpr (side) {
      const R e = v[2] + v[0];
      r0[Y] = e + v[1];
      r1[Y] = v[2] - v[0];
      r2[Y] = e;
    } else {
      r0[Y] = v[1];
      r1[Y] = R(0);
      r2[Y] = R(0);
    }
  });
  const R e0 = r0[2] + r0[0];
  const R s00 = e0 + r0[1], s01 = r0[2] - r0[0], s02 = e0;
  const R s10 = (r1[2] + r1[0]) + r1[1], s11 = r1[2] - r1[0];
  const R s20 = (r2[2] + r2[0]) + r2[1];
  if constexpr (Assign) {  // the first layer a target receives (c_z = +1) sets every sum
    static_assert(CZ > 0, "assign with the c_z = +1 layer");
    s.d0 = s00;
    s.jx = s10;
    s.jy = s01;
    s.pxx = s20;
    s.pyy = s02;
    s.pxy = s11;
    s.pzz = s00;
    s.jz = s00;
    s.pxz = s10;
    s.pyz = s01;
    return;
  }
  s.d0 = s.d0 + s00;
  s.jx = s.jx + s10;
  s.jy = s.jy + s01;
  s.pxx = s.pxx + s20;
  s.pyy = s.pyy + s02;
  s.pxy = s.pxy + s11;
  if constexpr (CZ != 0) {
    s.pzz = s.pzz + s00;
    if constexpr (CZ > 0) {
      s.jz = s.jz + s00;
      s.pxz = s.pxz + s10;
      s.pyz = s.pyz + s01;
    } else {
      s.jz = s.jz - s00;
      s.pxz = s.pxz - s10;
      s.pyz = s.pyz - s01;
    }
  }
}

// 2D: add the populations with c_y = CY rebuilt on one row that arrive at
// inner node tx to its moment sums s: population (cx, CY) comes from row node
// tx - cx.
template <class L, int CY, int BX, class R, bool Assign = false>
__device__ __forceinline__ void add_row(Moments<R>& s, const R (*pop)[BX], int tx) {
  R v[3];
  sfor<0, 3>([&](auto X) {
    constexpr int cx = int(X) - 1;
    v[X] = pop[velocity_index<L>(cx, CY, 0)][tx - cx];
  });
  const R e = v[2] + v[0];
  const R s0 = e + v[1], s1 = v[2] - v[0];
  if constexpr (Assign) {  // the first row a target receives (c_y = +1) sets every sum
    static_assert(CY > 0, "assign with the c_y = +1 row");
    s.d0 = s0;
    s.jx = s1;
    s.pxx = e;
    s.pyy = s0;
    s.jy = s0;
    s.pxy = s1;
    s.jz = s.pzz = s.pxz = s.pyz = R(0);
    return;
  }
  s.d0 = s.d0 + s0;
  s.jx = s.jx + s1;
  s.pxx = s.pxx + e;
  if constexpr (CY != 0) {
    s.pyy = s.pyy + s0;
    if constexpr (CY > 0) {
      s.jy = s.jy + s0;
      s.pxy = s.pxy + s1;
    } else {
      s.jy = s.jy - s0;
      s.pxy = s.pxy - s1;
    }
  }
}

// ---- resting walls -----------------------------------------------------------
// Resting no-slip walls on the first and last node of the axes in a.walls: the
// regularised Dirichlet boundary of Sec. 3.7 with u = 0, as the population step
// applies it.  At a wall node a population whose source lies outside the box is
// unknown; it takes the value of its opposite if that one is known (the
// off-equilibrium bounce-back at u = 0, where w_i = w_opp), else w_i (rho - rho0);
// rho - rho0 follows from the zeroth moment of the completed set, the node keeps
// j = 0, and a1^(2) is the second moment of the completed set minus
// (rho - rho0) c_s^2 I.  Every step is linear in the arriving populations, so
// their contributions are summed layer by layer as they arrive: a known
// population whose opposite is unknown counts twice (at xi and at -xi: the
// momentum cancels), and the buried ones enter when the node is finalised.

// Side of the box along one axis: -1 (first node), +1 (last node), 0.
__device__ __forceinline__ int wall_side(int walls, int bit, int v, int n) {
  return (walls >> bit & 1) ? (v == 0 ? -1 : (v == n - 1 ? 1 : 0)) : 0;
}

// Does a population moving along (cx, cy, cz) arrive from outside the box?
__device__ __forceinline__ bool from_outside(int sx, int sy, int sz, int cx, int cy, int cz) {
  return (sx != 0 && cx == -sx) || (sy != 0 && cy == -sy) || (sz != 0 && cz == -sz);
}

// Contribution of the known population v moving along (cx, cy, cz) to the moment
// sums of a wall node (sides sx, sy, sz).
template <class R>
__device__ __forceinline__ void add_known(Moments<R>& s, R v, int cx, int cy, int cz, int sx, int sy, int sz) {
  const bool twice = from_outside(sx, sy, sz, -cx, -cy, -cz);
  const R k = twice ? R(2) * v : v;
  s.d0 = s.d0 + k;
  if (!twice) {
    s.jx = s.jx + R(cx) * v;
    s.jy = s.jy + R(cy) * v;
    s.jz = s.jz + R(cz) * v;
  }
  s.pxx = s.pxx + R(cx * cx) * k;
  s.pyy = s.pyy + R(cy * cy) * k;
  s.pzz = s.pzz + R(cz * cz) * k;
  s.pxy = s.pxy + R(cx * cy) * k;
  s.pxz = s.pxz + R(cx * cz) * k;
  s.pyz = s.pyz + R(cy * cz) * k;
}

// Wall node: the populations of layer c_z = CZ arriving at inner node (tx, ty).
template <class L, int CZ, int TY, int MX, class R>
__device__ __forceinline__ void add_layer_walls(Moments<R>& s, const R (*pop)[TY][MX], int tx, int ty, int sx, int sy,
                                                int sz) {
  sfor<0, 3>([&](auto Y) {
    sfor<0, 3>([&](auto X) {
      constexpr int cx = int(X) - 1, cy = int(Y) - 1;
      if constexpr (has_velocity<L>(cx, cy, CZ)) {
        if (!from_outside(sx, sy, sz, cx, cy, CZ))
          add_known(s, pop[velocity_index<L>(cx, cy, CZ)][ty - cy][tx - cx], cx, cy, CZ, sx, sy, sz);
      }
    });
  });
}

// 2D wall node: the populations with c_y = CY rebuilt on one row arriving at inner node tx.
template <class L, int CY, int BX, class R>
__device__ __forceinline__ void add_row_walls(Moments<R>& s, const R (*pop)[BX], int tx, int sx, int sy) {
  sfor<0, 3>([&](auto X) {
    constexpr int cx = int(X) - 1;
    if (!from_outside(sx, sy, 0, cx, CY, 0)) add_known(s, pop[velocity_index<L>(cx, CY, 0)][tx - cx], cx, CY, 0, sx, sy, 0);
  });
}

// Stored moments of a wall node from its sums (known and bounced populations).
template <class L, class R>
__device__ __forceinline__ void finalize_walls(const Moments<R>& s, int sx, int sy, int sz, R (&m)[kNM<L>]) {
  R wb = R(0), bxx = R(0), byy = R(0), bzz = R(0), bxy = R(0), bxz = R(0), byz = R(0);  // buried: sum w, w xi xi
  sfor<0, L::Q>([&](auto I) {
    constexpr int cx = L::cx(I), cy = L::cy(I), cz = L::cz(I);
    if (from_outside(sx, sy, sz, cx, cy, cz) && from_outside(sx, sy, sz, -cx, -cy, -cz)) {
      const R w = R(L::w(I));
      wb = wb + w;
      bxx = bxx + R(cx * cx) * w;
      byy = byy + R(cy * cy) * w;
      bzz = bzz + R(cz * cz) * w;
      bxy = bxy + R(cx * cy) * w;
      bxz = bxz + R(cx * cz) * w;
      byz = byz + R(cy * cz) * w;
    }
  });
  const R drho = s.d0 / (R(1) - wb);
  constexpr R cs2 = R(kCs2);
  m[0] = drho;
  m[1] = R(0);
  m[2] = R(0);
  if constexpr (L::D == 3) {
    m[3] = R(0);
    m[4] = s.pxx + drho * bxx - drho * cs2;
    m[5] = s.pyy + drho * byy - drho * cs2;
    m[6] = s.pzz + drho * bzz - drho * cs2;
    m[7] = s.pxy + drho * bxy;
    m[8] = s.pxz + drho * bxz;
    m[9] = s.pyz + drho * byz;
  } else {
    m[3] = s.pxx + drho * bxx - drho * cs2;
    m[4] = s.pyy + drho * byy - drho * cs2;
    m[5] = s.pxy + drho * bxy;
  }
}

// Element at a byte offset from a base pointer.
template <class S>
__device__ __forceinline__ S at_offset(const S* base, uint32_t off) {
  return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + off);
}
template <class S>
__device__ __forceinline__ S* ptr_at_offset(S* base, uint32_t off) {
  return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + off);
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// One step of the moment-state update (see the file comment).
template <class L, int N, class S, int TY, int MX, bool W>
__global__ void __launch_bounds__(MX * TY) k_mstep(const S* __restrict__ src, S* __restrict__ dst, StepArgs a) {
  static_assert(L::D == 3, "3D lattices; 2D runs k_mstep2");
  using R = S;
  constexpr int NM = kNM<L>;
  __shared__ R pop[L::Q][TY][MX];
  const int tx = threadIdx.x % MX, ty = threadIdx.x / MX;
  const int gx = (a.nx + MX - 3) / (MX - 2), gy = (a.ny + TY - 3) / (TY - 2);
  // tiles in x, then y, then the z-chunk
  const int t = int(blockIdx.x);
  const int bxi = t % gx, byi = (t / gx) % gy, bz = t / (gx * gy);
  const int x0 = bxi * (MX - 2), y0 = byi * (TY - 2);
  // the patch node this thread rebuilds, and the node it updates if inner
  const int px = wrap(x0 - 1 + tx, a.nx), py = wrap(y0 - 1 + ty, a.ny);
  const bool inner = tx >= 1 && tx <= MX - 2 && ty >= 1 && ty <= TY - 2 && x0 + tx - 1 < a.nx && y0 + ty - 1 < a.ny;
  // Byte offsets of the node within its plane of one field (32 bits: the host
  // checks that a plane fits); the plane and field bases are block-uniform, so
  // each access is a scalar base plus one per-lane 32-bit offset.
  const uint32_t off_in = uint32_t((int64_t(py) * a.sy + px) * int64_t(sizeof(S)));
  const uint32_t off_out = uint32_t((int64_t(y0 + ty - 1) * a.sy + (x0 + tx - 1)) * int64_t(sizeof(S)));
  const R rho0 = R(a.rho0), om = R(a.omega1);

  auto load = [&](int z, R (&m)[NM]) {
    const S* s = src + int64_t(z) * a.sz;
    uint32_t o = off_in;
    asm volatile("" : "+v"(o));  // keeps the scalar-base form of the accesses (see k_mstep_t)
    sfor<0, NM>([&](auto C) { m[C] = at_offset(s + int64_t(C) * a.si, o); });
  };
  // Rebuild the populations of this thread's patch node into LDS; ZS selects
  // all of them (2) or only those with c_z = ZS (the planes next to a chunk).
  auto rebuild = [&](const R (&m)[NM], auto ZS) __attribute__((always_inline)) {
    constexpr int Z = decltype(ZS)::value;
    const Hydro<R> h = state_hydro<L, R>(m, rho0);
    R C[3][3][3];
    coefficients<L, N, R>(h, om, C);
    R f[L::Q];
    reconstruct<L, N, R, Z>(C, f);
    sfor<0, L::Q>([&](auto I) {
      if constexpr (Z == 2 || L::cz(I) == Z) pop[I][ty][tx] = f[I];
    });
  };
  auto put = [&](int z, const R (&m)[NM]) {
    S* d = dst + int64_t(z) * a.sz;
    uint32_t o = off_out;
    asm volatile("" : "+v"(o));
    sfor<0, NM>([&](auto C) { __builtin_nontemporal_store(m[C], ptr_at_offset(d + int64_t(C) * a.si, o)); });
  };
  // walls (W): sides of this thread's target column and row; the side along z
  // depends on the target plane
  const int wsx = W ? wall_side(a.walls, 0, x0 + tx - 1, a.nx) : 0;
  const int wsy = W ? wall_side(a.walls, 1, y0 + ty - 1, a.ny) : 0;
  // Add layer c_z = CZ to the sums of target plane `target`; the c_z = +1 layer
  // is the first a target receives and sets the sums.
  auto add = [&](Moments<R>& sums, auto CZS, int target) __attribute__((always_inline)) {
    constexpr int CZ = decltype(CZS)::value;
    if constexpr (W) {
      const int wsz = wall_side(a.walls, 2, target, a.nz);
      if (wsx != 0 || wsy != 0 || wsz != 0) {
        if constexpr (CZ > 0) clear(sums);
        add_layer_walls<L, CZ, TY, MX, R>(sums, pop, tx, ty, wsx, wsy, wsz);
        return;
      }
    }
    add_layer<L, CZ, TY, MX, R, (CZ > 0)>(sums, pop, tx, ty);
  };
  auto finish = [&](const Moments<R>& sums, int target, R (&m)[NM]) __attribute__((always_inline)) {
    if constexpr (W) {
      const int wsz = wall_side(a.walls, 2, target, a.nz);
      if (wsx != 0 || wsy != 0 || wsz != 0) {
        finalize_walls<L, R>(sums, wsx, wsy, wsz, m);
        return;
      }
    }
    finalize_state<L, R>(sums, rho0, m);
  };
  using layer_m = std::integral_constant<int, -1>;
  using layer_0 = std::integral_constant<int, 0>;
  using layer_p = std::integral_constant<int, 1>;

  {
    // Target planes z0 .. z1-1; planes z0-1 .. z1 are rebuilt, plane k of the
    // march being z0 - 1 + k (k = 0 .. n + 1, n = z1 - z0).  Plane 0 reaches only
    // target z0 (its c_z = +1 populations) and plane n + 1 only target z1 - 1
    // (c_z = -1), so those two rebuild a third of the populations and add one
    // layer.  Plane k adds its c_z = +1 layer to target k (first contribution),
    // c_z = 0 to target k - 1 and c_z = -1 to target k - 2, which is then
    // complete.  Roles rotate with period 3: the moments of plane k sit in
    // buffer k mod 3 (plane k + 2 is loaded into buffer (k + 2) mod 3 while plane
    // k is rebuilt) and the sums of target j in T[j mod 3]; the march is unrolled
    // by 3, so no register is copied between iterations.  The moments of a
    // completed target are kept in registers and stored at the start of the next
    // iteration, next to the prefetch: loads and stores then have one or more
    // whole rebuilds to complete before they are waited for.
    static_assert(kPrefetch == 2, "two planes in flight ahead of the rebuild");
    const int z0 = bz * a.lz;
    const int z1 = (z0 + a.lz < a.nz) ? z0 + a.lz : a.nz;
    const int n = z1 - z0;
    Moments<R> T[3];  // sums of targets j = k, k - 1, k - 2 (mod 3) at plane k
    R B[3][NM];       // moments of planes k, k + 1, k + 2 (mod 3)
    load(wrap(z0 - 1, a.nz), B[0]);
    load(wrap(z0, a.nz), B[1]);
    R out[NM];  // moments of target k - 3, stored during plane k
    // E = 2: plane inside the chunk; +1: plane 0; -1: plane n + 1.  PH = k mod 3.
    auto iteration = [&](int k, auto PHS, auto ES) __attribute__((always_inline)) {
      constexpr int PH = decltype(PHS)::value, E = decltype(ES)::value;
      constexpr int P1 = (PH + 2) % 3, P2 = (PH + 1) % 3;  // (k - 1) mod 3, (k - 2) mod 3
      const int pz = z0 - 1 + k;
      if (k + kPrefetch <= n + 1) load(wrap(pz + kPrefetch, a.nz), B[P1]);  // buffer (k + 2) mod 3
      if (inner && k >= 3) put(z0 + k - 3, out);
      rebuild(B[PH], ES);
      lds_barrier();
      if (inner) {
        if constexpr (E == 1) {
          add(T[PH], layer_p{}, z0);  // target z0 (k = 0)
        } else if constexpr (E == -1) {
          add(T[P2], layer_m{}, z1 - 1);  // target n - 1 = k - 2 is complete
          finish(T[P2], z1 - 1, out);
        } else {
          if (k < n) add(T[PH], layer_p{}, pz + 1);
          add(T[P1], layer_0{}, pz);
          if (k >= 2) {
            add(T[P2], layer_m{}, pz - 1);
            finish(T[P2], pz - 1, out);  // target k - 2 is complete
          }
        }
      }
      lds_barrier();
    };
    using ph0 = std::integral_constant<int, 0>;
    using ph1 = std::integral_constant<int, 1>;
    using ph2 = std::integral_constant<int, 2>;
    using first_plane = std::integral_constant<int, 1>;
    using inner_plane = std::integral_constant<int, 2>;
    using last_plane = std::integral_constant<int, -1>;
    iteration(0, ph0{}, first_plane{});
    int k = 1;
    for (; k + 2 <= n; k += 3) {
      iteration(k, ph1{}, inner_plane{});
      iteration(k + 1, ph2{}, inner_plane{});
      iteration(k + 2, ph0{}, inner_plane{});
    }
    if (k <= n) iteration(k++, ph1{}, inner_plane{});  // k = 1 mod 3 here
    if (k <= n) iteration(k++, ph2{}, inner_plane{});
    // k = n + 1: the last plane
    switch (k % 3) {
      case 0: iteration(k, ph0{}, last_plane{}); break;
      case 1: iteration(k, ph1{}, last_plane{}); break;
      default: iteration(k, ph2{}, last_plane{}); break;
    }
    if (inner) put(z1 - 1, out);
  }
}

// One step of the moment-state update with row-aligned tiles (3D, FP32).  The
// inner tile of a block is 64 nodes of a row, starting at a multiple of 64,
// by TY rows.  TY + 2 waves rebuild the tile's 64 columns on rows y0 - 1 ..
// y0 + TY (one wave per row), and one more wave rebuilds the two halo columns
// (x0 - 1 and the column right after the tile) of those rows, so every field
// row is read as two whole 128-byte lines, and the halo lines are the first and
// last lines of the neighbouring tiles.  A 256-node row takes four tiles.  The
// march along z is that of k_mstep.  LDS holds the patch as TY + 2 rows of 66
// columns: column 0 is the left halo, 1 .. width the tile, width + 1 the right
// halo.
template <class L, int N, class S, int TY, bool W>
__global__ void __launch_bounds__(64 * (TY + 3)) k_mstep_t(const S* __restrict__ src, S* __restrict__ dst,
                                                           StepArgs a) {
  static_assert(L::D == 3, "3D lattices");
  static_assert(2 * (TY + 2) <= 64, "the halo wave holds both halo columns of every patch row");
  using R = S;
  constexpr int NM = kNM<L>, RW = TY + 2, MXL = 66;
  __shared__ R pop[L::Q][RW][MXL];
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
  // Blocks reach the eight XCDs round-robin by id, and each XCD has its own
  // L2.  Blocks b and b + 8 (the same XCD, dispatched one after the other) take
  // x-neighbouring tiles of one tile row (rows y0 .. y0 + TY - 1 of a z-chunk),
  // so the halo columns a block reads are lines its XCD's L2 holds for the
  // neighbour.  Tile rows g >= gy * gz of the last group of eight are empty.
  const int gx = (a.nx + 63) / 64, gy = (a.ny + TY - 1) / TY, gz = (a.nz + a.lz - 1) / a.lz;
  const int b = int(blockIdx.x);
  const int bxi = (b / 8) % gx, g = (b / (8 * gx)) * 8 + b % 8;
  if (g >= gy * gz) return;
  const int byi = g % gy, bz = g / gy;
  const int x0 = bxi * 64, y0 = byi * TY;
  const int width = (a.nx - x0 < 64) ? a.nx - x0 : 64;
  // The node this thread rebuilds: patch row r, LDS column col, lattice node (px, py).
  int r, col, px;
  bool writes;
  if (wave < RW) {
    r = wave;
    writes = lane < width;
    col = lane + 1;
    px = x0 + (writes ? lane : 0);
  } else {
    const bool left = lane < RW;
    writes = lane < 2 * RW;
    r = left ? lane : (writes ? lane - RW : 0);
    col = left ? 0 : width + 1;
    px = wrap(left ? x0 - 1 : x0 + width, a.nx);
  }
  const int py = wrap(y0 - 1 + r, a.ny);
  // the node this thread updates, if inner: (x0 + lane, y0 + r - 1), LDS (lane + 1, r)
  const bool inner = wave < RW && r >= 1 && r <= TY && lane < width && y0 + r - 1 < a.ny;
  const int tc = lane + 1;
  const uint32_t off_in = uint32_t((int64_t(py) * a.sy + px) * int64_t(sizeof(S)));
  const uint32_t off_out =
      inner ? uint32_t((int64_t(y0 + r - 1) * a.sy + (x0 + lane)) * int64_t(sizeof(S))) : 0u;
  const R rho0 = R(a.rho0), om = R(a.omega1);

  auto load = [&](int z, R (&m)[NM]) {
    const S* s = src + int64_t(z) * a.sz;
    // The empty asm hides that the lane offset is the same in every plane of
    // the march.  Without it the compiler hoists a 64-bit copy of the offset
    // out of the loop and adds it to every field's base with a 64-bit lane
    // add; with it each access takes the scalar-base form (scalar field base +
    // 32-bit lane offset) and the adds go away.
    uint32_t o = off_in;
    asm volatile("" : "+v"(o));
    sfor<0, NM>([&](auto C) { m[C] = at_offset(s + int64_t(C) * a.si, o); });
  };
  auto rebuild = [&](const R (&m)[NM], auto ZS) __attribute__((always_inline)) {
    constexpr int Z = decltype(ZS)::value;
    const Hydro<R> h = state_hydro<L, R>(m, rho0);
    R C[3][3][3];
    coefficients<L, N, R>(h, om, C);
    R f[L::Q];
    reconstruct<L, N, R, Z>(C, f);
    if (writes) {
      sfor<0, L::Q>([&](auto I) {
        if constexpr (Z == 2 || L::cz(I) == Z) pop[I][r][col] = f[I];
      });
    }
  };
  auto put = [&](int z, const R (&m)[NM]) {
    S* d = dst + int64_t(z) * a.sz;
    uint32_t o = off_out;
    asm volatile("" : "+v"(o));
    sfor<0, NM>([&](auto C) { __builtin_nontemporal_store(m[C], ptr_at_offset(d + int64_t(C) * a.si, o)); });
  };
  const int wsx = W ? wall_side(a.walls, 0, x0 + lane, a.nx) : 0;
  const int wsy = W ? wall_side(a.walls, 1, y0 + r - 1, a.ny) : 0;
  auto add = [&](Moments<R>& sums, auto CZS, int target) __attribute__((always_inline)) {
    constexpr int CZ = decltype(CZS)::value;
    if constexpr (W) {
      const int wsz = wall_side(a.walls, 2, target, a.nz);
      if (wsx != 0 || wsy != 0 || wsz != 0) {
        if constexpr (CZ > 0) clear(sums);
        add_layer_walls<L, CZ, RW, MXL, R>(sums, pop, tc, r, wsx, wsy, wsz);
        return;
      }
    }
    add_layer<L, CZ, RW, MXL, R, (CZ > 0)>(sums, pop, tc, r);
  };
  auto finish = [&](const Moments<R>& sums, int target, R (&m)[NM]) __attribute__((always_inline)) {
    if constexpr (W) {
      const int wsz = wall_side(a.walls, 2, target, a.nz);
      if (wsx != 0 || wsy != 0 || wsz != 0) {
        finalize_walls<L, R>(sums, wsx, wsy, wsz, m);
        return;
      }
    }
    finalize_state<L, R>(sums, rho0, m);
  };
  using layer_m = std::integral_constant<int, -1>;
  using layer_0 = std::integral_constant<int, 0>;
  using layer_p = std::integral_constant<int, 1>;
  {
    // The march of k_mstep: targets z0 .. z1 - 1, planes z0 - 1 .. z1 rebuilt,
    // register roles rotating with period 3, the two edge planes rebuilding
    // only the layer that reaches the chunk.
    static_assert(kPrefetch == 2, "two planes in flight ahead of the rebuild");
    const int z0 = bz * a.lz;
    const int z1 = (z0 + a.lz < a.nz) ? z0 + a.lz : a.nz;
    const int n = z1 - z0;
    Moments<R> T[3];
    R B[3][NM];
    load(wrap(z0 - 1, a.nz), B[0]);
    load(wrap(z0, a.nz), B[1]);
    // a completed target is stored at once (with 1024 threads a block has 128
    // VGPRs per lane, and holding it for the next iteration spilled)
    auto complete = [&](const Moments<R>& sums, int target) __attribute__((always_inline)) {
      R out[NM];
      finish(sums, target, out);
      put(target, out);
    };
    auto iteration = [&](int k, auto PHS, auto ES) __attribute__((always_inline)) {
      constexpr int PH = decltype(PHS)::value, E = decltype(ES)::value;
      constexpr int P1 = (PH + 2) % 3, P2 = (PH + 1) % 3;
      const int pz = z0 - 1 + k;
      if (k + kPrefetch <= n + 1) load(wrap(pz + kPrefetch, a.nz), B[P1]);
      rebuild(B[PH], ES);
      lds_barrier();
      if (inner) {
        if constexpr (E == 1) {
          add(T[PH], layer_p{}, z0);
        } else if constexpr (E == -1) {
          add(T[P2], layer_m{}, z1 - 1);
          complete(T[P2], z1 - 1);
        } else {
          if (k < n) add(T[PH], layer_p{}, pz + 1);
          add(T[P1], layer_0{}, pz);
          if (k >= 2) {
            add(T[P2], layer_m{}, pz - 1);
            complete(T[P2], pz - 1);
          }
        }
      }
      lds_barrier();
    };
    using ph0 = std::integral_constant<int, 0>;
    using ph1 = std::integral_constant<int, 1>;
    using ph2 = std::integral_constant<int, 2>;
    using first_plane = std::integral_constant<int, 1>;
    using inner_plane = std::integral_constant<int, 2>;
    using last_plane = std::integral_constant<int, -1>;
    iteration(0, ph0{}, first_plane{});
    int k = 1;
    for (; k + 2 <= n; k += 3) {
      iteration(k, ph1{}, inner_plane{});
      iteration(k + 1, ph2{}, inner_plane{});
      iteration(k + 2, ph0{}, inner_plane{});
    }
    if (k <= n) iteration(k++, ph1{}, inner_plane{});
    if (k <= n) iteration(k++, ph2{}, inner_plane{});
    switch (k % 3) {
      case 0: iteration(k, ph0{}, last_plane{}); break;
      case 1: iteration(k, ph1{}, last_plane{}); break;
      default: iteration(k, ph2{}, last_plane{}); break;
    }
  }
}

// One step of the 2D moment-state update.  A block of BX threads rebuilds a
// row of BX nodes (x0 - 1 ... x0 + BX - 2) and marches along y through a
// chunk of a.lz target rows: the populations rebuilt on row p with c_y = -1,
// 0, +1 arrive on rows p - 1, p, p + 1, so each inner thread keeps running
// moment sums for three target rows, and row p - 1 is complete once row p has
// been rebuilt.  Rows of BX nodes keep the loads and stores of a field nearly
// line-aligned (one partial 128-byte line per row and field), and the two-stage
// prefetch ring of the 3D step overlaps them with the rebuilds.
template <class L, int N, class S, int BX, bool W>
__global__ void __launch_bounds__(BX) k_mstep2(const S* __restrict__ src, S* __restrict__ dst, StepArgs a) {
  using R = S;
  constexpr int NM = kNM<L>;
  static_assert(L::D == 2, "2D lattices only");
  __shared__ R pop[L::Q][BX];
  const int tx = threadIdx.x;
  const int x0 = blockIdx.x * (BX - 2);
  const int px = wrap(x0 - 1 + tx, a.nx);
  const bool inner = tx >= 1 && tx <= BX - 2 && x0 + tx - 1 < a.nx;
  const int xo = x0 + tx - 1;
  const R rho0 = R(a.rho0), om = R(a.omega1);
  // byte offsets within a row of one field; row and field bases are block-uniform
  const uint32_t off_in = uint32_t(px) * uint32_t(sizeof(S)), off_out = uint32_t(xo) * uint32_t(sizeof(S));
  auto load = [&](int y, R (&m)[NM]) {
    const S* s = src + int64_t(y) * a.sy;
    sfor<0, NM>([&](auto C) { m[C] = at_offset(s + int64_t(C) * a.si, off_in); });
  };
  auto put = [&](int y, const R (&m)[NM]) {
    S* d = dst + int64_t(y) * a.sy;
    sfor<0, NM>([&](auto C) { __builtin_nontemporal_store(m[C], ptr_at_offset(d + int64_t(C) * a.si, off_out)); });
  };
  // Target rows y0 .. y1-1; rows y0-1 .. y1 are rebuilt, row k of the march
  // being y0 - 1 + k (k = 0 .. n + 1, n = y1 - y0).  Row k adds its c_y = +1
  // populations to target k (first contribution), c_y = 0 to target k - 1 and
  // c_y = -1 to target k - 2, which is then complete.  Register roles rotate
  // with period 3 as in the 3D step: moments of row k in buffer k mod 3, sums
  // of target j in slot j mod 3, the march unrolled by 3 with no copies.
  const int y0 = blockIdx.y * a.lz;
  const int y1 = (y0 + a.lz < a.ny) ? y0 + a.lz : a.ny;
  const int n = y1 - y0;
  Moments<R> T[3];
  R B[3][NM];
  load(wrap(y0 - 1, a.ny), B[0]);
  load(wrap(y0, a.ny), B[1]);
  R out[NM];  // moments of target k - 3, stored during row k
  auto iteration = [&](int k, auto PHS) __attribute__((always_inline)) {
    constexpr int PH = decltype(PHS)::value;
    constexpr int P1 = (PH + 2) % 3, P2 = (PH + 1) % 3;  // (k - 1) mod 3, (k - 2) mod 3
    const int py = y0 - 1 + k;
    if (k + kPrefetch <= n + 1) load(wrap(py + kPrefetch, a.ny), B[P1]);  // buffer (k + 2) mod 3
    if (inner && k >= 3) put(y0 + k - 3, out);
    {
      const Hydro<R> h = state_hydro<L, R>(B[PH], rho0);
      R C[3][3][3];
      coefficients<L, N, R>(h, om, C);
      R f[L::Q];
      reconstruct<L, N, R>(C, f);
      sfor<0, L::Q>([&](auto I) { pop[I][tx] = f[I]; });
    }
    lds_barrier();
    if (inner) {
      if constexpr (W) {
        // walls: sides of the target column and of the target rows py + 1, py, py - 1
        // (with no side the wall sums are the plain sums)
        const int sx = wall_side(a.walls, 0, xo, a.nx);
        if (k < n) {
          clear(T[PH]);
          add_row_walls<L, 1, BX, R>(T[PH], pop, tx, sx, wall_side(a.walls, 1, py + 1, a.ny));
        }
        if (k >= 1 && k <= n) add_row_walls<L, 0, BX, R>(T[P1], pop, tx, sx, wall_side(a.walls, 1, py, a.ny));
        if (k >= 2) {  // target row py - 1 is complete
          const int sm = wall_side(a.walls, 1, py - 1, a.ny);
          add_row_walls<L, -1, BX, R>(T[P2], pop, tx, sx, sm);
          if (sx != 0 || sm != 0) finalize_walls<L, R>(T[P2], sx, sm, 0, out);
          else finalize_state<L, R>(T[P2], rho0, out);
        }
      } else {
        if (k < n) add_row<L, 1, BX, R, true>(T[PH], pop, tx);
        if (k >= 1 && k <= n) add_row<L, 0, BX, R>(T[P1], pop, tx);
        if (k >= 2) {
          add_row<L, -1, BX, R>(T[P2], pop, tx);
          finalize_state<L, R>(T[P2], rho0, out);  // target row py - 1 is complete
        }
      }
    }
    lds_barrier();
  };
  using ph0 = std::integral_constant<int, 0>;
  using ph1 = std::integral_constant<int, 1>;
  using ph2 = std::integral_constant<int, 2>;
  iteration(0, ph0{});
  int k = 1;
  for (; k + 2 <= n + 1; k += 3) {
    iteration(k, ph1{});
    iteration(k + 1, ph2{});
    iteration(k + 2, ph0{});
  }
  if (k <= n + 1) iteration(k++, ph1{});  // k = 1 mod 3 here
  if (k <= n + 1) iteration(k++, ph2{});
  if (inner) put(y1 - 1, out);
}

// Moment state at t = 0 from (rho, u[, pi1]): the pre-collision moments of
// f0(rho, u) + f1(u, pi1), i.e. rho - rho0, rho u and pi1 (Sec. 3.2).
template <class L, class S, class T>
__global__ void __launch_bounds__(256) k_minit(const T* __restrict__ rho, const T* __restrict__ u,
                                               const T* __restrict__ pi1, S* __restrict__ dst, StepArgs a) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = node_offset(a, uint32_t(n));
  const double r = double(rho[n]);
  S m[kNM<L>];
  m[0] = S(r - a.rho0);
  m[1] = S(r * double(u[n]));
  m[2] = S(r * double(u[nodes + n]));
  if constexpr (L::D == 3) {
    m[3] = S(r * double(u[2 * nodes + n]));
    // pi1 order xx, xy, xz, yy, yz, zz -> state order axx, ayy, azz, axy, axz, ayz
    const int perm[6] = {0, 3, 5, 1, 2, 4};
    for (int c = 0; c < 6; ++c) m[4 + c] = pi1 ? S(pi1[perm[c] * nodes + n]) : S(0);
  } else {
    const int perm[3] = {0, 2, 1};  // xx, xy, yy -> axx, ayy, axy
    for (int c = 0; c < 3; ++c) m[3 + c] = pi1 ? S(pi1[perm[c] * nodes + n]) : S(0);
  }
  sfor<0, kNM<L>>([&](auto C) { dst[int64_t(C) * a.si + off] = m[C]; });
}

// rho, u, pi1 (= the stored pre-collision a1^(2)) of the moment state.
template <class L, class S, class T>
__global__ void __launch_bounds__(256) k_mmoments(const S* __restrict__ src, T* __restrict__ rho, T* __restrict__ u,
                                                  T* __restrict__ pi1, StepArgs a) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = node_offset(a, uint32_t(n));
  double m[kNM<L>];
  sfor<0, kNM<L>>([&](auto C) { m[C] = double(src[int64_t(C) * a.si + off]); });
  const double r = a.rho0 + m[0];
  if (rho) rho[n] = T(r);
  if (u) {
    u[n] = T(m[1] / r);
    u[nodes + n] = T(m[2] / r);
    if constexpr (L::D == 3) u[2 * nodes + n] = T(m[3] / r);
  }
  if (pi1) {
    if constexpr (L::D == 3) {
      const int from[6] = {4, 7, 8, 5, 9, 6};  // xx, xy, xz, yy, yz, zz
      for (int c = 0; c < 6; ++c) pi1[c * nodes + n] = T(m[from[c]]);
    } else {
      const int from[3] = {3, 5, 4};  // xx, xy, yy
      for (int c = 0; c < 3; ++c) pi1[c * nodes + n] = T(m[from[c]]);
    }
  }
}

// Per-block partial totals {rho, j_x, j_y, j_z, |j|^2 / (2 rho)} of the moment state.
template <class L, class S>
__global__ void __launch_bounds__(kReduceBlock) k_mtotals(const S* __restrict__ src, double* __restrict__ partials,
                                                          StepArgs a, int64_t per_block) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t begin = int64_t(blockIdx.x) * per_block;
  const int64_t end = begin + per_block < nodes ? begin + per_block : nodes;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t n = begin + threadIdx.x; n < end; n += kReduceBlock) {
    const int64_t off = node_offset(a, uint32_t(n));
    const double r = a.rho0 + double(src[off]);
    const double jx = double(src[a.si + off]), jy = double(src[2 * a.si + off]);
    const double jz = (L::D == 3) ? double(src[3 * a.si + off]) : 0.0;
    acc[0] += r;
    acc[1] += jx;
    acc[2] += jy;
    acc[3] += jz;
    acc[4] += 0.5 * (jx * jx + jy * jy + jz * jz) / r;
  }
  block_sum_store<5>(acc, partials);
}

// Velocity field (FP64) of the moment state.
template <class L, class S>
__global__ void __launch_bounds__(256) k_mvelocity(const S* __restrict__ src, double* __restrict__ u, StepArgs a) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = node_offset(a, uint32_t(n));
  const double inv = 1.0 / (a.rho0 + double(src[off]));
  u[n] = double(src[a.si + off]) * inv;
  u[nodes + n] = double(src[2 * a.si + off]) * inv;
  if constexpr (L::D == 3) u[2 * nodes + n] = double(src[3 * a.si + off]) * inv;
}

// Post-collision deviations of the moment state (what the population form
// stores), compact SoA [q][node] in the state's precision.
template <class L, int N, class S>
__global__ void __launch_bounds__(256) k_mpopulations(const S* __restrict__ src, S* __restrict__ dst, StepArgs a) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = node_offset(a, uint32_t(n));
  S m[kNM<L>];
  sfor<0, kNM<L>>([&](auto C) { m[C] = src[int64_t(C) * a.si + off]; });
  const Hydro<S> h = state_hydro<L, S>(m, S(a.rho0));
  S C[3][3][3];
  coefficients<L, N, S>(h, S(a.omega1), C);
  S f[L::Q];
  reconstruct<L, N, S>(C, f);
  sfor<0, L::Q>([&](auto I) { dst[int64_t(I) * nodes + n] = f[I]; });
}

// ---------------------------------------------------------------------------
// Launchers.  a.lz = z-planes per block of the 3D step (each chunk rebuilds
// lz + 2 planes); the host picks it.  Measured with 32 x 16 patches, 256^3
// D3Q27 FP32: patches of 8, 16 and 32 rows within 6%; dispatching the z-chunks
// of a tile next to each other gave 24-27 GLUPS at 256^3 and 512^3 for lz = 2
// to 32; padding the z-planes off multiples of 64 KiB changed nothing;
// contiguous tile ranges per XCD removed the fall-off at large planes but did
// not beat the 64 x 8 patches in plain order.
template <class L, int N, class S>
hipError_t launch_mstep(const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  if (a.lz < 1) return hipErrorInvalidValue;
  if constexpr (L::D == 2) {
    dim3 grid2(unsigned((a.nx + kRowX - 3) / (kRowX - 2)), unsigned((a.ny + a.lz - 1) / a.lz));
    if (grid2.y > 65535u) return hipErrorInvalidValue;
    if (a.walls)
      hipLaunchKernelGGL((k_mstep2<L, N, S, kRowX, true>), grid2, dim3(kRowX), 0, s, static_cast<const S*>(src),
                         static_cast<S*>(dst), a);
    else
      hipLaunchKernelGGL((k_mstep2<L, N, S, kRowX, false>), grid2, dim3(kRowX), 0, s, static_cast<const S*>(src),
                         static_cast<S*>(dst), a);
    return hipGetLastError();
  } else {
    if (int64_t(a.ny) * a.sy * int64_t(sizeof(S)) >= (int64_t(1) << 32)) return hipErrorInvalidValue;
    if constexpr (sizeof(S) == 4) {
      constexpr int TY = kTileRows;
      const int64_t rows = int64_t((a.ny + TY - 1) / TY) * ((a.nz + a.lz - 1) / a.lz);
      const int64_t nbt = int64_t((a.nx + 63) / 64) * 8 * ((rows + 7) / 8);
      if (nbt >= (int64_t(1) << 31)) return hipErrorInvalidValue;
      if (a.walls)
        hipLaunchKernelGGL((k_mstep_t<L, N, S, TY, true>), dim3(unsigned(nbt)), dim3(64 * (TY + 3)), 0, s,
                           static_cast<const S*>(src), static_cast<S*>(dst), a);
      else
        hipLaunchKernelGGL((k_mstep_t<L, N, S, TY, false>), dim3(unsigned(nbt)), dim3(64 * (TY + 3)), 0, s,
                           static_cast<const S*>(src), static_cast<S*>(dst), a);
      return hipGetLastError();
    }
    constexpr int TY = MPatch<S>::TY, MX = MPatch<S>::MX;
    const int64_t nb = int64_t((a.nx + MX - 3) / (MX - 2)) * ((a.ny + TY - 3) / (TY - 2)) *
                       ((a.nz + a.lz - 1) / a.lz);
    if (nb >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    if (a.walls)
      hipLaunchKernelGGL((k_mstep<L, N, S, TY, MX, true>), dim3(unsigned(nb)), dim3(MX * TY), 0, s,
                         static_cast<const S*>(src), static_cast<S*>(dst), a);
    else
      hipLaunchKernelGGL((k_mstep<L, N, S, TY, MX, false>), dim3(unsigned(nb)), dim3(MX * TY), 0, s,
                         static_cast<const S*>(src), static_cast<S*>(dst), a);
    return hipGetLastError();
  }
}

template <class L, int N, class S>
hipError_t launch_mpopulations(const void* src, void* dst, const StepArgs& a, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  hipLaunchKernelGGL((k_mpopulations<L, N, S>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                     static_cast<const S*>(src), static_cast<S*>(dst), a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_minit(int dtype, const void* rho, const void* u, const void* pi1, void* dst, const StepArgs& a,
                        hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  dim3 grid(unsigned((nodes + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL((k_minit<L, S, double>), grid, dim3(256), 0, s, static_cast<const double*>(rho),
                       static_cast<const double*>(u), static_cast<const double*>(pi1), static_cast<S*>(dst), a);
  else
    hipLaunchKernelGGL((k_minit<L, S, float>), grid, dim3(256), 0, s, static_cast<const float*>(rho),
                       static_cast<const float*>(u), static_cast<const float*>(pi1), static_cast<S*>(dst), a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_mmoments(int dtype, const void* src, void* rho, void* u, void* pi1, const StepArgs& a,
                           hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  dim3 grid(unsigned((nodes + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL((k_mmoments<L, S, double>), grid, dim3(256), 0, s, static_cast<const S*>(src),
                       static_cast<double*>(rho), static_cast<double*>(u), static_cast<double*>(pi1), a);
  else
    hipLaunchKernelGGL((k_mmoments<L, S, float>), grid, dim3(256), 0, s, static_cast<const S*>(src),
                       static_cast<float*>(rho), static_cast<float*>(u), static_cast<float*>(pi1), a);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_mtotals(const void* src, double* partials, int nblocks, double* out, const StepArgs& a,
                          hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t per_block = (nodes + nblocks - 1) / nblocks;
  hipLaunchKernelGGL((k_mtotals<L, S>), dim3(nblocks), dim3(kReduceBlock), 0, s, static_cast<const S*>(src),
                     partials, a, per_block);
  hipLaunchKernelGGL((k_final<5>), dim3(1), dim3(kReduceBlock), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

template <class L, class S>
hipError_t launch_mvelocity(const void* src, double* u, const StepArgs& a, hipStream_t s) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  hipLaunchKernelGGL((k_mvelocity<L, S>), dim3(unsigned((nodes + 255) / 256)), dim3(256), 0, s,
                     static_cast<const S*>(src), u, a);
  return hipGetLastError();
}

}  // namespace lbrr
