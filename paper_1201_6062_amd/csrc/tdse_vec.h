// Launch descriptors and buffer tables of the single-vector (batch == 1)
// tile kernels: the completion a launch performs, the per-call descriptor its
// captured graphs read, and the plan buffers it reads and writes. Kept apart
// from the rest of the library's internal declarations because these types
// (with vec_kernels.hip) determine the tile kernels' code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdse {

// ---------------------------------------------------------------------------
// Completion of one product (the RK4 stage or Taylor term whose dipole
// product the previous launch computed) and formation of the next input.
enum CompletionKind : int32_t {
    CK_RK4_MID = 0,   // completed RK4 stage s in 1..3
    CK_RK4_END = 1,   // completed RK4 stage 4 (finishes a step)
    CK_TAY_MID = 2,   // completed Taylor term m < p
    CK_TAY_END = 3,   // completed Taylor term p (finishes a step)
    CK_HMUL = -1,     // no completion: write y = E o u + F z (single product)
    CK_ADJ_MID = 4,   // adjoint stage j > 1 of a reversed RK4 step
    CK_ADJ_LAST = 5,  // adjoint stage 1: finishes the reversed step
    CK_RKF = 6,       // Runge-Kutta-Fehlberg stage (slot = stage 0..5; batched path)
};

struct Completion {
    int32_t kind;
    int32_t slot;        // field sample slot of the completed product
    int32_t step_delta;  // step of the completed product = base + off + step_delta
    int32_t first;       // RK4 stage 1: acc = w k (reset); else acc += w k
    double w_acc;        // RK4: b_s; Taylor: unused
    double a_next;       // RK4: alpha_{s+1} (times dt in-kernel); Taylor: dt/m factor
};

// Per-call values that a captured graph reads from device memory, so one
// graph serves every call of the same shape.
constexpr int CHUNK_STEPS = 64;  // steps per captured graph (even: even launch count)

struct CallDesc {
    int64_t base_step;   // first step of the current chunk
    int64_t nsteps;
    const double *field; // [B][nsteps][S]
    double *ckpt;        // may be null
    int64_t ckpt_every;
    double dt;
    int32_t slots;       // S
    int32_t pad_;
    // Field samples of steps base_step-1 .. base_step+CHUNK_STEPS-1 (zero outside
    // [0, nsteps)), staged at a fixed address at the start of every chunk so a
    // launch finds its sample without a dependent load.
    double chunk_field[(CHUNK_STEPS + 1) * 3];
    // Checkpoint row written by a completion that ends step base_step + x
    // (x = 0 .. CHUNK_STEPS), or -1 when that step is not a checkpoint.
    int64_t chunk_ckpt_row[CHUNK_STEPS + 1];
};

// ---------------------------------------------------------------------------
// Single-vector (batch == 1) streaming path.
constexpr int VEC_TILE_MAX = 128;   // max rows/cols of one dipole tile
constexpr int VEC_THREADS = 512;    // 8 waves per tile workgroup

// Products launches that stream the dipole from HBM take patches of at most
// PATCH_MAX x PATCH_MAX tiles of one block per workgroup, leaving
// patch_np(T) row partials per row segment and column partials per column
// segment (one per patch across), where one workgroup per tile leaves T.
constexpr int PATCH_MAX = 4;
__host__ __device__ constexpr int patch_np(int T) { return (T + PATCH_MAX - 1) / PATCH_MAX; }


// Buffers of one parity (a launch reads one parity and writes the other).
struct VecSide {
    double2 *st[3];        // c, acc, u, each [(lmax+1)*n]
    double2 *rowp;         // [lmax][T(seg i)][np(contrib)][VEC_TILE_MAX], np <= T
    double2 *colp;         // [lmax][T(out seg j)][np(contrib)][VEC_TILE_MAX]
};

// Field order: lmax, n, en, dip and side[0] fill the first 64 bytes, the
// kernel-argument words a tile launch needs before its first memory access.
struct VecBuffers {
    int32_t lmax, n;
    const double *en;      // [(lmax+1)*n]
    const double *dip;     // tiles [lmax][T][T][VEC_TILE_MAX * VEC_TILE_MAX], order tile_pos
    VecSide side[2];       // [parity]
    CallDesc *desc;
    int32_t ld, T;
    int32_t gauge;         // TDSE_LENGTH or TDSE_VELOCITY (how the two block uses combine)
};

struct VecLaunch {
    Completion comp;
    int32_t off;     // step offset within chunk of the launch
    int32_t parity;  // launch parity: read st/partials[parity], write [parity^1]
    int32_t finish;  // 1: write c' to the caller's cT (finish launch)
    int32_t slots;   // field samples per step (3 RK4, 1 Taylor)
    int32_t np;      // completions: partials per segment and direction (0: T, one per tile)
    int32_t pad_;
    double *out;     // caller cT for the finish launch
};

}  // namespace tdse
