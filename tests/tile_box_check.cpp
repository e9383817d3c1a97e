// Host check of the stored tile-box layout of the sorted deposit (tile_box.h): the slot
// map is a bijection of the 10^3 box points onto 0..999, box_of inverts it, and the
// gather's slot rule reads, for every cell of a tile, exactly the box points that its
// one to eight covering tiles stored for that cell, each box point of each tile once
// (periodic ring of three tiles per axis). Prints "ok" and returns 0 when all hold.
#include <cstdio>

#include "tile_box.h"

using namespace pm_tilebox;

int main() {
  int seen[kSlots] = {0};
  for (int hx = 0; hx < 10; ++hx)
    for (int hy = 0; hy < 10; ++hy)
      for (int hz = 0; hz < 10; ++hz) {
        const int s = slot_of(hx, hy, hz);
        if (s < 0 || s >= kSlots) return std::printf("slot out of range\n"), 1;
        ++seen[s];
        int a, b, c;
        box_of(s, a, b, c);
        if (a != hx || b != hy || c != hz) return std::printf("box_of is not the inverse\n"), 1;
      }
  for (int s = 0; s < kSlots; ++s)
    if (seen[s] != 1) return std::printf("slot %d taken %d times\n", s, seen[s]), 1;
  const int T = 3;
  static int used[T][T][T][kSlots];
  for (int tx = 0; tx < T; ++tx)
    for (int ty = 0; ty < T; ++ty)
      for (int tz = 0; tz < T; ++tz)
        for (int x = 0; x < 8; ++x)
          for (int y = 0; y < 8; ++y)
            for (int z = 0; z < 8; ++z)
              for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                  for (int dz = -1; dz <= 1; ++dz) {
                    if ((dx == -1 && x != 0) || (dx == 1 && x != 7)) continue;
                    if ((dy == -1 && y != 0) || (dy == 1 && y != 7)) continue;
                    if ((dz == -1 && z != 0) || (dz == 1 && z != 7)) continue;
                    // box point of tile t + d that holds cell (x, y, z) of tile t
                    const int hx = x + 1 - 8 * dx, hy = y + 1 - 8 * dy, hz = z + 1 - 8 * dz;
                    const int px = (tx + dx + T) % T, py = (ty + dy + T) % T, pz = (tz + dz + T) % T;
                    const int g = 8 * T;
                    if (((8 * px + hx - 1) % g + g) % g != 8 * tx + x ||
                        ((8 * py + hy - 1) % g + g) % g != 8 * ty + y ||
                        ((8 * pz + hz - 1) % g + g) % g != 8 * tz + z)
                      return std::printf("box point is not the cell\n"), 1;
                    if (gather_slot(dx, dy, dz, x, y, z) != slot_of(hx, hy, hz))
                      return std::printf("gather_slot disagrees with slot_of\n"), 1;
                    ++used[px][py][pz][slot_of(hx, hy, hz)];
                  }
  for (int px = 0; px < T; ++px)
    for (int py = 0; py < T; ++py)
      for (int pz = 0; pz < T; ++pz)
        for (int s = 0; s < kSlots; ++s)
          if (used[px][py][pz][s] != 1) return std::printf("box slot read %d times\n", used[px][py][pz][s]), 1;
  std::printf("ok\n");
  return 0;
}
