// Stored order of the single-vector path's 128 x 128 dipole tiles; host
// and device code (the layout kernels, the tile kernel, the small-problem
// kernel) all address tiles through these two functions.
#pragma once

#include <stdint.h>

#include "tdse_split.h"

namespace tdse {

// Stored order of a 128 x 128 dipole tile (lane order of the tile kernel).
// Wave w of the tile workgroup owns columns 16w .. 16w+15; its lane
// (h, q) = (lane >> 4, lane & 15) owns rows q + 16k (k = 0..7) and columns
// 16w + 4h + c (c = 0..3). Load j = 2k + c/2 of wave w fetches one double2
// per lane (columns c, c+1 for even c), 64 consecutive double2 per load.
TDSE_HD inline int64_t tile_pos(int a, int b) {
    const int q = a & 15, k = a >> 4, w = b >> 4, h = (b >> 2) & 3, c = b & 3;
    return 2 * ((int64_t)(w * 16 + 2 * k + (c >> 1)) * 64 + 16 * h + q) + (c & 1);
}
// Inverse of tile_pos: element (row a, column b) stored at position p.
TDSE_HD inline void tile_elem(int64_t p, int *a, int *b) {
    const int e = (int)(p & 1), L = (int)((p >> 1) & 63), j = (int)((p >> 7) & 15), w = (int)(p >> 11);
    const int h = L >> 4, q = L & 15, k = j >> 1, c = 2 * (j & 1) + e;
    *a = q + 16 * k;
    *b = 16 * w + 4 * h + c;
}

}  // namespace tdse
