// Layout of the stored 10^3 box of one 8^3 tile (the tile plus a one-cell halo on
// every side) in the sorted deposit. Box point h = (hx, hy, hz), each 0..9, is cell
// 8 t + h - 1 of the grid for a tile at tile coordinates t. The box is stored so that
// each of its consumers reads contiguous runs: first the 8^3 interior (tile-local
// x, y, z = h - 1, row-major), then the halo grouped by the neighbouring tile whose
// cells it covers: six faces of 64 values (the two free coordinates row-major), twelve
// edges of 8 (along the free axis), eight corners of 1.
//   faces:   face axis f (0..2), side s (0: h_f = 0, 1: h_f = 9): group 2 f + s
//   edges:   free axis g (0..2), sides of the other two axes p < q: group 4 g + 2 s_p + s_q
//   corners: group 4 s_x + 2 s_y + s_z
#pragma once

#include <hip/hip_runtime.h>

namespace pm_tilebox {

constexpr int kSlots = 1000;
constexpr int kFaceBase = 512;
constexpr int kEdgeBase = kFaceBase + 6 * 64;   // 896
constexpr int kCornerBase = kEdgeBase + 12 * 8; // 992

// side of one box coordinate: -1 (0, the low halo), +1 (9, the high halo), 0 (interior)
__host__ __device__ constexpr int side(int h) { return h == 0 ? -1 : (h == 9 ? 1 : 0); }

__host__ __device__ constexpr int slot_of(int hx, int hy, int hz) {
  const int sx = side(hx), sy = side(hy), sz = side(hz);
  const int zeros = (sx == 0) + (sy == 0) + (sz == 0);
  if (zeros == 3) return ((hx - 1) * 8 + (hy - 1)) * 8 + (hz - 1);
  if (zeros == 2) {
    if (sx != 0) return kFaceBase + 64 * (0 + (sx > 0)) + (hy - 1) * 8 + (hz - 1);
    if (sy != 0) return kFaceBase + 64 * (2 + (sy > 0)) + (hx - 1) * 8 + (hz - 1);
    return kFaceBase + 64 * (4 + (sz > 0)) + (hx - 1) * 8 + (hy - 1);
  }
  if (zeros == 1) {
    if (sx == 0) return kEdgeBase + 8 * (0 + 2 * (sy > 0) + (sz > 0)) + (hx - 1);
    if (sy == 0) return kEdgeBase + 8 * (4 + 2 * (sx > 0) + (sz > 0)) + (hy - 1);
    return kEdgeBase + 8 * (8 + 2 * (sx > 0) + (sy > 0)) + (hz - 1);
  }
  return kCornerBase + 4 * (sx > 0) + 2 * (sy > 0) + (sz > 0);
}

// inverse of slot_of: the box point stored at slot (0 .. 999)
__host__ __device__ inline void box_of(int slot, int &hx, int &hy, int &hz) {
  if (slot < kFaceBase) {
    hx = (slot >> 6) + 1;
    hy = ((slot >> 3) & 7) + 1;
    hz = (slot & 7) + 1;
  } else if (slot < kEdgeBase) {
    const int o = slot - kFaceBase, grp = o >> 6, u = ((o >> 3) & 7) + 1, v = (o & 7) + 1;
    const int hs = (grp & 1) ? 9 : 0;
    const int f = grp >> 1;
    hx = f == 0 ? hs : u;
    hy = f == 1 ? hs : (f == 0 ? u : v);
    hz = f == 2 ? hs : v;
  } else if (slot < kCornerBase) {
    const int o = slot - kEdgeBase, grp = o >> 3, c = (o & 7) + 1;
    const int g = grp >> 2, hp = (grp & 2) ? 9 : 0, hq = (grp & 1) ? 9 : 0;
    hx = g == 0 ? c : hp;
    hy = g == 1 ? c : (g == 0 ? hp : hq);
    hz = g == 2 ? c : hq;
  } else {
    const int o = slot - kCornerBase;
    hx = (o & 4) ? 9 : 0;
    hy = (o & 2) ? 9 : 0;
    hz = (o & 1) ? 9 : 0;
  }
}

// Slot, in the box of tile t + d, of cell c = (x, y, z) (tile-local 0..7) of tile t:
// box point c + 1 - 8 d. d = (dx, dy, dz) in {-1, 0, 1}^3 with d_a = -1 only where
// c_a = 0 and d_a = +1 only where c_a = 7 (the neighbours whose halo covers the cell).
// With d known at compile time the group is a constant and only the free coordinates
// remain.
__host__ __device__ constexpr int gather_slot(int dx, int dy, int dz, int x, int y, int z) {
  const int zeros = (dx == 0) + (dy == 0) + (dz == 0);
  if (zeros == 3) return (x * 8 + y) * 8 + z;
  if (zeros == 2) {
    // the neighbour's box point on this axis is 9 for d = -1 (its high face), 0 for +1
    if (dx != 0) return kFaceBase + 64 * (0 + (dx < 0)) + y * 8 + z;
    if (dy != 0) return kFaceBase + 64 * (2 + (dy < 0)) + x * 8 + z;
    return kFaceBase + 64 * (4 + (dz < 0)) + x * 8 + y;
  }
  if (zeros == 1) {
    if (dx == 0) return kEdgeBase + 8 * (0 + 2 * (dy < 0) + (dz < 0)) + x;
    if (dy == 0) return kEdgeBase + 8 * (4 + 2 * (dx < 0) + (dz < 0)) + y;
    return kEdgeBase + 8 * (8 + 2 * (dx < 0) + (dy < 0)) + z;
  }
  return kCornerBase + 4 * (dx < 0) + 2 * (dy < 0) + (dz < 0);
}

}  // namespace pm_tilebox
