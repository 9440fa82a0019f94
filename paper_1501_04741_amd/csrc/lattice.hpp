// Velocity sets of the GPU path, as compile-time tables.
//
// D3Q19 follows the paper's list e_1..e_19 (Section 3), 0-based.  D2Q9 is the
// z = 0 subset of that list in the same order; the scalar lattices D3Q7 and
// D2Q5 are its first 7 and 5 members.  Weights: D3Q19 1/3, 1/18, 1/36; D2Q9
// 4/9, 1/9, 1/36 (c_s^2 = 1/3 for both); D2Q5 1/3, 1/6 (c^2 = 1/3); D3Q7 1/4,
// 1/8 (c^2 = 1/4).  Every loop over these tables is fully unrolled, so each
// lookup folds to a constant.
#pragma once

#include <hip/hip_runtime.h>

namespace lbmk {

template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int ex(int j) {
    constexpr int t[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    return t[j];
  }
  __host__ __device__ static constexpr int ey(int j) {
    constexpr int t[9] = {0, 0, 0, 1, -1, 1, 1, -1, -1};
    return t[j];
  }
  __host__ __device__ static constexpr int ez(int) { return 0; }
  __host__ __device__ static constexpr int opp(int j) {
    constexpr int t[9] = {0, 2, 1, 4, 3, 8, 7, 6, 5};
    return t[j];
  }
  __host__ __device__ static constexpr double w(int j) {
    return j == 0 ? 4.0 / 9.0 : (j < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr double cs2() { return 1.0 / 3.0; }
};

template <>
struct Lat<19> {
  static constexpr int D = 3;
  __host__ __device__ static constexpr int ex(int j) {
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[j];
  }
  __host__ __device__ static constexpr int ey(int j) {
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[j];
  }
  __host__ __device__ static constexpr int ez(int j) {
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return t[j];
  }
  __host__ __device__ static constexpr int opp(int j) {
    constexpr int t[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    return t[j];
  }
  __host__ __device__ static constexpr double w(int j) {
    return j == 0 ? 1.0 / 3.0 : (j < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  __host__ __device__ static constexpr double cs2() { return 1.0 / 3.0; }
};

// Scalar lattices: the first QS velocities of the matching flow lattice.
template <int QS>
struct SLat;

template <>
struct SLat<0> {
  __host__ __device__ static constexpr int ex(int) { return 0; }
  __host__ __device__ static constexpr int ey(int) { return 0; }
  __host__ __device__ static constexpr int ez(int) { return 0; }
  __host__ __device__ static constexpr int opp(int) { return 0; }
  __host__ __device__ static constexpr double w(int) { return 0.0; }
  __host__ __device__ static constexpr double c2() { return 1.0; }
};

template <>
struct SLat<5> {
  __host__ __device__ static constexpr int ex(int j) { return Lat<9>::ex(j); }
  __host__ __device__ static constexpr int ey(int j) { return Lat<9>::ey(j); }
  __host__ __device__ static constexpr int ez(int) { return 0; }
  __host__ __device__ static constexpr int opp(int j) { return Lat<9>::opp(j); }
  __host__ __device__ static constexpr double w(int j) { return j == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
  __host__ __device__ static constexpr double c2() { return 1.0 / 3.0; }
};

template <>
struct SLat<7> {
  __host__ __device__ static constexpr int ex(int j) { return Lat<19>::ex(j); }
  __host__ __device__ static constexpr int ey(int j) { return Lat<19>::ey(j); }
  __host__ __device__ static constexpr int ez(int j) { return Lat<19>::ez(j); }
  __host__ __device__ static constexpr int opp(int j) { return Lat<19>::opp(j); }
  __host__ __device__ static constexpr double w(int j) { return j == 0 ? 1.0 / 4.0 : 1.0 / 8.0; }
  __host__ __device__ static constexpr double c2() { return 1.0 / 4.0; }
};

// Moment basis of the D3Q19 multiple-relaxation-time collision (d'Humieres et
// al., the matrix Section 3.1 cites): row k of U evaluated on velocity j.  Rows:
// density; energy 19|c|^2 - 30; energy square (21|c|^4 - 53|c|^2 + 24)/2;
// momentum c_a and energy flux (5|c|^2 - 9) c_a for a = x, y, z; stresses
// 3c_x^2 - |c|^2, c_y^2 - c_z^2 and their partners times (3|c|^2 - 5);
// off-diagonal stresses c_x c_y, c_y c_z, c_x c_z; third-order moments
// (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z.  The rows are
// mutually orthogonal, so U^{-1} = U^T diag(1 / |row|^2).
struct Mrt19 {
  __host__ __device__ static constexpr int u(int k, int j) {
    const int x = Lat<19>::ex(j), y = Lat<19>::ey(j), z = Lat<19>::ez(j);
    const int c2 = x * x + y * y + z * z;
    switch (k) {
      case 0: return 1;
      case 1: return 19 * c2 - 30;
      case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
      case 3: return x;
      case 4: return (5 * c2 - 9) * x;
      case 5: return y;
      case 6: return (5 * c2 - 9) * y;
      case 7: return z;
      case 8: return (5 * c2 - 9) * z;
      case 9: return 3 * x * x - c2;
      case 10: return (3 * c2 - 5) * (3 * x * x - c2);
      case 11: return y * y - z * z;
      case 12: return (3 * c2 - 5) * (y * y - z * z);
      case 13: return x * y;
      case 14: return y * z;
      case 15: return x * z;
      case 16: return (y * y - z * z) * x;
      case 17: return (z * z - x * x) * y;
      default: return (x * x - y * y) * z;
    }
  }
  __host__ __device__ static constexpr int norm2(int k) {
    int s = 0;
    for (int j = 0; j < 19; ++j) s += u(k, j) * u(k, j);
    return s;
  }
  // rate group of row k: 0 = 1/tau (conserved and viscous rows), 1 energy,
  // 2 energy square, 3 energy flux, 4 fourth-order stresses, 5 third-order
  __host__ __device__ static constexpr int group(int k) {
    constexpr int t[19] = {0, 1, 2, 0, 3, 0, 3, 0, 3, 0, 4, 0, 4, 0, 0, 0, 5, 5, 5};
    return t[k];
  }
};

// Velocity indices of +x and -x (paper's e_2 and e_3) in every lattice.
constexpr int kPX = 1;
constexpr int kMX = 2;

}  // namespace lbmk
