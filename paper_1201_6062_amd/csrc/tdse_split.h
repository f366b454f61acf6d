// Balanced split of `work` units over `workers` (Sec. 4.1, algorithm for
// splitting generic work): worker `id` gets floor(work/workers) units, plus
// one if id < work mod workers, starting at id*floor(work/workers) +
// min(id, work mod workers). Parts differ in length by at most one and tile
// [0, work) in order. Used for row/column segments of dipole blocks, for
// tiles over XCDs, and for work lists over workgroups.
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

}  // namespace tdse
