// Discrete velocity sets for the device kernels.
//
// D3Q19 weights 1/3, 1/18, 1/36 are the ones printed with Eq. 16; D2Q9 uses
// 4/9, 1/9, 1/36.  The direction order is canonical (it decides ties in the
// wetting-link rule and the layout of the population arrays):
//   D2Q9  0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
//         5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1)
//   D3Q19 0 rest, 1..6 +x -x +y -y +z -z, 7..18 the twelve edge diagonals
//         (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
//         (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
#pragma once
#include <cstdint>

struct D2Q9 {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  // weights times 36 (exact integers): 16, 4, 1
  static constexpr int w36[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
  // axis directions (+a, -a) for a < D
  static constexpr int axp[3] = {1, 2, 0};
  static constexpr int axm[3] = {3, 4, 0};
};

struct D3Q19 {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  // weights times 36: 12, 2, 1
  static constexpr int w36[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  static constexpr int axp[3] = {1, 3, 5};
  static constexpr int axm[3] = {2, 4, 6};
};

template <class L>
__host__ __device__ constexpr int lat_len2(int q) {
  return L::ex[q] * L::ex[q] + L::ey[q] * L::ey[q] + L::ez[q] * L::ez[q];
}
