// Compile-time velocity sets of the GPU path (D2Q9, D3Q19, D3Q27).
//
// Velocity sets of Sec. 3.2 ("Discretization of the microscopic velocity
// space"): D2Q9 and D3Q27 are tensor products of the three-point
// Gauss-Hermite rule {-1, 0, 1} with weights {1/6, 2/3, 1/6}; D3Q19 keeps
// the rest, face and edge velocities with weights 1/3, 1/18, 1/36.  Sound
// speed c_s^2 = 1/3.
//
// Population order: i = (cx+1) + 3(cy+1) + 9(cz+1) (cz = 0 in 2D); D3Q19
// keeps this order with the eight corner velocities removed.
#pragma once

namespace lbrr {

constexpr double kCs2 = 1.0 / 3.0;

// one-dimensional weight of a velocity component in {-1, 0, 1}
constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

struct D2Q9 {
  static constexpr int Q = 9, D = 2, NMAX = 4;
  static constexpr bool kProduct = true;
  // D3Q27 index of population i
  static constexpr int idx27(int i) { return 9 + i; }
  static constexpr int cx(int i) { return i % 3 - 1; }
  static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
  static constexpr int cz(int) { return 0; }
  static constexpr double w(int i) { return w1d(cx(i)) * w1d(cy(i)); }
};

struct D3Q27 {
  static constexpr int Q = 27, D = 3, NMAX = 6;
  static constexpr bool kProduct = true;
  static constexpr int idx27(int i) { return i; }
  static constexpr int cx(int i) { return i % 3 - 1; }
  static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
  static constexpr int cz(int i) { return i / 9 - 1; }
  static constexpr double w(int i) { return w1d(cx(i)) * w1d(cy(i)) * w1d(cz(i)); }
};

struct D3Q19 {
  static constexpr int Q = 19, D = 3, NMAX = 4;
  static constexpr bool kProduct = false;
  // D3Q27 indices that are not corners (|c|^2 <= 2), in increasing order
  static constexpr int idx27(int i) {
    int n = -1;
    for (int j = 0; j < 27; ++j) {
      const int a = j % 3 - 1, b = (j / 3) % 3 - 1, c = j / 9 - 1;
      if (a * a + b * b + c * c <= 2 && ++n == i) return j;
    }
    return -1;
  }
  static constexpr int cx(int i) { return idx27(i) % 3 - 1; }
  static constexpr int cy(int i) { return (idx27(i) / 3) % 3 - 1; }
  static constexpr int cz(int i) { return idx27(i) / 9 - 1; }
  static constexpr double w(int i) {
    const int s = cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
    return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

}  // namespace lbrr
