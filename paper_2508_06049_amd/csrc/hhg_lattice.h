// Fixed facts about the lattice triangulation of a uniformly refined macro element, in the
// macro's integer index coordinates (i, j[, k]).  Used by host setup and by the kernels.
//
// 2D: the 4-split produces two element shapes per lattice cell,
//     up   = (0,0), (1,0), (0,1)      down = (1,0), (0,1), (1,1).
// 3D: Bey's rule produces, in p = (i, i+j, i+j+k), the Kuhn triangulation of the unit-cube
//     lattice: for every permutation s of the axes the simplex 0, e_s0, e_s0+e_s1, (1,1,1).
//     Mapped back with E0 = (1,-1,0), E1 = (0,1,-1), E2 = (0,0,1) (the images of the p-axes),
//     type s has vertex offsets 0, E_s0, E_s0+E_s1, (1,0,0).
#pragma once

namespace hhg {

// [type][vertex][coordinate]
constexpr int kType3[6][4][3] = {
    {{0, 0, 0}, {1, -1, 0}, {1, 0, -1}, {1, 0, 0}},   // s = (0,1,2)
    {{0, 0, 0}, {1, -1, 0}, {1, -1, 1}, {1, 0, 0}},   // s = (0,2,1)
    {{0, 0, 0}, {0, 1, -1}, {1, 0, -1}, {1, 0, 0}},   // s = (1,0,2)
    {{0, 0, 0}, {0, 1, -1}, {0, 1, 0}, {1, 0, 0}},    // s = (1,2,0)
    {{0, 0, 0}, {0, 0, 1}, {1, -1, 1}, {1, 0, 0}},    // s = (2,0,1)
    {{0, 0, 0}, {0, 0, 1}, {0, 1, 0}, {1, 0, 0}},     // s = (2,1,0)
};
constexpr int kType2[2][3][2] = {
    {{0, 0}, {1, 0}, {0, 1}},
    {{1, 0}, {0, 1}, {1, 1}},
};

// Direction index of an offset (0 = centre, 1..H = +dir, H+1..2H = -dir), -1 if none.
__host__ __device__ constexpr int dir_index3(int a, int b, int c) {
  if (a == 0 && b == 0 && c == 0) return 0;
  if (a == 1 && b == 0 && c == 0) return 1;
  if (a == 0 && b == 1 && c == 0) return 2;
  if (a == 0 && b == 0 && c == 1) return 3;
  if (a == -1 && b == 1 && c == 0) return 4;
  if (a == -1 && b == 0 && c == 1) return 5;
  if (a == 0 && b == -1 && c == 1) return 6;
  if (a == 1 && b == -1 && c == 1) return 7;
  if (a == -1 && b == 0 && c == 0) return 8;
  if (a == 0 && b == -1 && c == 0) return 9;
  if (a == 0 && b == 0 && c == -1) return 10;
  if (a == 1 && b == -1 && c == 0) return 11;
  if (a == 1 && b == 0 && c == -1) return 12;
  if (a == 0 && b == 1 && c == -1) return 13;
  if (a == -1 && b == 1 && c == -1) return 14;
  return -1;
}
__host__ __device__ constexpr int dir_index2(int a, int b) {
  if (a == 0 && b == 0) return 0;
  if (a == 1 && b == 0) return 1;
  if (a == 0 && b == 1) return 2;
  if (a == -1 && b == 1) return 3;
  if (a == -1 && b == 0) return 4;
  if (a == 0 && b == -1) return 5;
  if (a == 1 && b == -1) return 6;
  return -1;
}

// offsets of the directions in the same order
constexpr int kOff3[15][3] = {{0, 0, 0},   {1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {-1, 1, 0},
                              {-1, 0, 1},  {0, -1, 1}, {1, -1, 1}, {-1, 0, 0}, {0, -1, 0},
                              {0, 0, -1},  {1, -1, 0}, {1, 0, -1}, {0, 1, -1}, {-1, 1, -1}};
constexpr int kOff2[7][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1}};

// the lattice direction whose endpoints have the parity pattern p = (i&1) | (j&1)<<1 | (k&1)<<2
// (prolongation: an odd fine node is the midpoint of the coarse edge along this direction)
constexpr int kParDir3[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 1, 0},
                                {0, 0, 1}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};
constexpr int kParDir2[4][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 1}};

}  // namespace hhg
