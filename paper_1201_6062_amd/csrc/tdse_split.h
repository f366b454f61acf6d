// Balanced split of `work` units over `workers` (Sec. 4.1, algorithm for
// splitting generic work): worker `id` gets floor(work/workers) units, plus
// one if id < work mod workers, starting at id*floor(work/workers) +
// min(id, work mod workers). Parts differ in length by at most one and tile
// [0, work) in order. Used (over 16-row units) for row/column segments of
// dipole blocks, for tiles over XCDs, and for work lists over workgroups.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define TDSE_HD __host__ __device__
#else
#define TDSE_HD
#endif

namespace tdse {

TDSE_HD inline int64_t split_start(int64_t work, int64_t workers, int64_t id) {
    int64_t div = work / workers, rem = work % workers;
    return id * div + (id < rem ? id : rem);
}

TDSE_HD inline int64_t split_len(int64_t work, int64_t workers, int64_t id) {
    return work / workers + (id < work % workers ? 1 : 0);
}

// Row/column segments of the single-vector path's dipole blocks: the same
// balanced split, over units of 16 rows (one row group of a 128 x 128 tile)
// rather than single rows, so that every segment but the last is whole row
// groups and a block's padding sits in its last segment only (a streamed
// tile's all-padding row groups and column pairs are never fetched). Segment
// q of n rows over T segments; needs 1 <= T <= ceil(n / 16), and a segment is
// at most 128 rows when T >= ceil(n / 128).
TDSE_HD inline int64_t seg_start(int64_t n, int64_t T, int64_t q) { return 16 * split_start((n + 15) / 16, T, q); }

TDSE_HD inline int64_t seg_len(int64_t n, int64_t T, int64_t q) {
    const int64_t end = 16 * split_start((n + 15) / 16, T, q + 1);
    return (end < n ? end : n) - seg_start(n, T, q);
}

}  // namespace tdse
