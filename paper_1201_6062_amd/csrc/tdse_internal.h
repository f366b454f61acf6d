// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/tdse.h"
#include "tdse_split.h"
#include "tdse_tile.h"
#include "tdse_vec.h"

namespace tdse {

// ---------------------------------------------------------------------------
// Error reporting (thread-local text, see tdse_last_error).
void set_error(const std::string &msg);
void clear_error();
tdse_status fail(tdse_status st, const std::string &msg);
tdse_status hip_fail(hipError_t e, const char *what);

#define TDSE_HIP(call)                                        \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::tdse::hip_fail(e_, #call); \
    } while (0)

#define TDSE_HIP_ST(call)                                     \
    do {                                                      \
        tdse_status s_ = (call);                              \
        if (s_ != TDSE_OK) return s_;                         \
    } while (0)

// Uneven group (several batch-1 plans advanced together).
struct GroupTile {
    int32_t inst;           // instance (index into the GroupInst array)
    int16_t l;              // block of the patch
    int8_t i, j;            // patch row / column within the block (patch_np(T) each way)
};
struct GroupSeg {
    int32_t inst;           // instance (index into the GroupInst array)
    int16_t m;              // block of the segment
    int16_t q;              // segment index within the block
};
struct GroupInst {
    VecBuffers b;           // the instance plan's buffers (its own T and segments)
    const double *field;    // [nsteps][3]
    int64_t nsteps;
};
// Single-workgroup propagation of small problems ((lmax+1) n <= 256, n <= 64).
bool small_eligible(int lmax, int n);
// rs[(m, a)] = absolute row sum of the symmetric coupling matrix (row-major
// blocks dip [lmax][n][n], device), [(lmax+1) n] device.
hipError_t coupling_rowsum(const double *dip, int lmax, int n, double *rs, hipStream_t s);
hipError_t small_propagate(const double *en, const double *dip, int gauge, int lmax, int n, int method, int order, double dt,
                           int64_t nsteps, const double *field, const double *c0, double *cT, double *ckpt,
                           int64_t ckpt_every, hipStream_t s);

// Per-call values of a group that its captured graphs read from device memory.
struct GroupDesc {
    int64_t base_round;     // first RK4 stage-round of the current chunk
    double dt;
};
constexpr int GROUP_CHUNK_ROUNDS = 64;  // rounds per captured graph (16 steps)
// One RK4 stage-round (desc->base_round + off) of a group: completion over the
// segment list, then the patch products over the patch list.
hipError_t group_launch_round(const GroupSeg *segs, int nsegs, const GroupTile *tiles, int ntiles,
                              const GroupInst *insts, const GroupDesc *desc, int32_t off, hipStream_t s);
hipError_t group_set_desc(GroupDesc *desc, int64_t base_round, double dt, hipStream_t s);

hipError_t vec_launch_tiles(const VecBuffers &b, const VecLaunch &l, hipStream_t s);
// Bytes of per-call buffers of a single-vector plan (states and partials of
// both parities, the call descriptor) and their placement in one region.
size_t vec_scratch_bytes(int lmax, int n, int T);
void vec_bind_scratch(VecBuffers &vb, char *base, int lmax, int n, int T);
// Single-vector RK4 / Taylor propagation of plan p on the per-call buffers of
// vb; use_graphs: replay the plan's captured chunk graph (vb must then be the
// plan's own buffers).
tdse_status vec_propagate_on(tdse_plan p, const VecBuffers &vb, bool use_graphs, tdse_method m, int order, double dt,
                             int64_t nsteps, const double *field, const double *c0, double *cT, double *ckpt,
                             int32_t K, hipStream_t s);
// NULL, alignment and device-memory check of an argument (TDSE_E_INVAL).
tdse_status check_device_ptr(const void *p, const char *name);

hipError_t vec_launch_combine(const VecBuffers &b, const VecLaunch &l, hipStream_t s);
// Split path: products only, inputs completed by a preceding vec_launch_combine.
hipError_t vec_launch_products(const VecBuffers &b, const VecLaunch &l, hipStream_t s);
hipError_t vec_launch_start(const VecBuffers &b, int32_t parity, const double *c0, int32_t method,
                            hipStream_t s);
hipError_t chunk_begin(CallDesc *d, int64_t base, hipStream_t s);
hipError_t vec_layout(const double *src, double *dst, int lmax, int n, int T, hipStream_t s);
hipError_t vec_untile(const double *tiles, double *dst, int lmax, int n, int T, hipStream_t s);
hipError_t set_desc(CallDesc *d, const CallDesc &v, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched (batch > 1) matrix-core path.
struct BatBuffers {
    double *en;            // [(lmax+1)][np]
    double *d;             // [lmax][np][np]  D_l row-major, zero-padded
    double *dT;            // [lmax][np][np]  D_l^T row-major, zero-padded
    double *u[2];          // [parity][(lmax+1)][np][ldu] stage inputs
    double *c, *acc;       // [(lmax+1)][np][ldu]
    double *kst;           // Runge-Kutta-Fehlberg: stage derivatives k_1..k_5, [5][(lmax+1)][np][ldu]
    const double *field;   // caller [batch][nsteps][S]
    int32_t lmax, n, np, ldu, batch, tm, tn, kc;
    int32_t ks;            // K groups per workgroup (1, or 2: one per neighbour block; 8: the small-batch kernel)
    int32_t gauge;         // TDSE_LENGTH or TDSE_VELOCITY (d holds -Q_l in the velocity gauge)
};

struct BatLaunch {
    int32_t kind;          // CompletionKind of this stage's own product
    int32_t slot, first, parity;
    double w_acc, a_next, dt;
    int64_t step, nsteps;
    int32_t slots, ckpt_row, ckpt_rows, pad_;
    double *ckpt;          // caller checkpoints [batch][ckpt_rows][2n], or null
    double *out;           // tdse_hmul output (caller layout)
    // forward recompute: copy this stage's input u to ustore (internal layout)
    // adjoint: ustore holds the forward input of the stage being reversed
    double *ustore;
    double *gpart;         // per row-tile partials [row tiles][batch]: adjoint field gradient, RKF45
                           // squared error, or (single product, if set) Re <u, H u>
    double p_lam, p_ub;    // adjoint: next input = p_lam * lambda + p_ub * ubar
};

hipError_t bat_layout(const double *src_dip, const double *src_en, BatBuffers &b, hipStream_t s);
hipError_t bat_pack(const BatBuffers &b, const double *c0, int taylor, hipStream_t s);
// c = state, u[0] = u_scale * state, acc = 0, reading the caller layout with
// pulse_stride doubles between pulses.
hipError_t bat_pack_strided(const BatBuffers &b, const double *src, size_t pulse_stride, double u_scale,
                            hipStream_t s);
hipError_t bat_launch_adjoint(const BatBuffers &b, const BatLaunch &l, hipStream_t s);
// grad[b][k][slot] for the steps k0 .. k0+len-1 from the partials of one segment
hipError_t bat_reduce_grad(const double *gpart, int rowtiles, int batch, int64_t k0, int64_t len,
                           int64_t nsteps, int nprod, int rk4, double *grad, hipStream_t s);
hipError_t bat_unpack(const BatBuffers &b, double *out, hipStream_t s);
// err[b * nsteps + k] = sqrt(sum over row tiles of the squared-error partials)
hipError_t bat_reduce_err(const double *gpart, int rowtiles, int batch, int64_t k, int64_t nsteps, double *err,
                          hipStream_t s);
hipError_t bat_ckpt0(const BatBuffers &b, const double *c0, double *ckpt, int rows, hipStream_t s);
hipError_t bat_launch_stage(const BatBuffers &b, const BatLaunch &l, hipStream_t s);

// ---------------------------------------------------------------------------
// Short-iterative Lanczos (caller-layout vectors [batch][len], len = 2 nstates).
// Several pulses (batched plans): the recurrence over many workgroups, grid
// (lzb_chunks(len), batch). normp: [batch][chunks] norm parts; dotp: the
// product's per-(row tile, pulse) parts of Re <v_j, H v_j>, [rowtiles][batch].
int lzb_chunks(int64_t len);
hipError_t lzb_norm_parts(const double *x, int batch, int64_t len, double *normp, hipStream_t s);
hipError_t lzb_update(const double *dotp, int rowtiles, const double *vj, const double *vjm1, double *w,
                      double *alpha, const double *beta, double *normp, int j, int m, int last, int batch,
                      int64_t len, hipStream_t s);
// v = x / |x| into vout (caller layout) and into the plan's product input u[0]
// (j < 0: beta0 = |x|; j >= 0: beta_j with the breakdown rule)
hipError_t lzb_normalize(const BatBuffers &bb, const double *x, const double *normp, double *vout, int j, int m,
                         const double *alpha, double *beta, double *beta0, int64_t len, hipStream_t s);
// One pulse over many workgroups. The Krylov vectors are formed unnormalised
// (x_0 = c, x_{j+1} = H v_j - alpha_j v_j - beta_{j-1} v_{j-1}), each launch
// that forms one leaving per-workgroup parts of |x|^2 in normp; the product
// launch of x_j reads it as is, and the completion (vec_launch_hmul_dot)
// takes the norm from the parts, stores beta (beta0 for j = 0), v_j = x_j /
// beta in place and y = H v_j, with the per-segment parts of Re <v_j, y> in
// dotp. lz_wide_groups: the workgroup count of the launches that leave norm
// parts (normp holds that many).
int lz_wide_groups(int64_t ncplx);
// x_0 = c and its norm parts
hipError_t lz_begin_wide(const double *c, double *x0, double *normp, int64_t ncplx, hipStream_t s);
// alpha_j from dotp; unless last, xnext = w - alpha_j v_j - beta_{j-1} v_{j-1}
// and its norm parts
hipError_t lz_update(const double *dotp, int nseg, const double *vj, const double *vjm1, const double *w,
                     double *xnext, double *alpha, const double *beta, int j, int last, double *normp,
                     int64_t ncplx, hipStream_t s);
// Normalisation of Krylov vector j inside its completion launch.
struct LzNorm {
    const double *normp;  // parts of |x_j|^2
    int32_t nparts;
    int32_t j;
    double *beta0;        // j == 0: receives |x_0|
    const double *alpha;  // alpha_{j-1} (breakdown test)
    double *beta;         // j > 0: receives beta_{j-1} = |x_j| (0 on breakdown)
};
hipError_t vec_launch_hmul_dot(const VecBuffers &b, const VecLaunch &l, double *dotp, const LzNorm &nz,
                               hipStream_t s);
// The update of step j folded into the product launch of the next vector:
// every workgroup sums alpha_j from dotp (workgroup 0 stores it) and forms its
// input segments of x_{j+1} = w - alpha_j v_j - beta_{j-1} v_{j-1}; one owner
// workgroup per segment stores that segment to xnext and its part of
// |x_{j+1}|^2 to normp[m T + q]. Needs lmax >= 1.
struct LzUpdate {
    const double *dotp;   // per-segment parts of alpha_j
    int32_t nseg;
    int32_t j;
    const double *w;      // H v_j
    const double *vj, *vjm1;
    double *xnext;
    double *alpha;
    const double *beta;
    double *normp;
};
hipError_t vec_launch_lz_products(const VecBuffers &b, const LzUpdate &z, hipStream_t s);
// One launch per Krylov product (one pulse, plans on the fused tile path).
// Launch k forms x_k and its products: for k >= 1 every tile workgroup
// completes, for its two input segments, the product of x_{k-1} from the
// previous launch's partials, and forms x_k = H v_{k-1} - alpha_{k-1} v_{k-1}
// - beta_{k-2} v_{k-2} with v_j = x_j / beta_{j-1} (beta_{-1} = beta0 =
// |x_0|); alpha_{k-1} = (sum E|x|^2 + F x^H D x) / |x|^2 of x_{k-1} and its
// norm come from the previous launch's parts, summed in the same order in
// every workgroup (workgroup 0 stores alpha_{k-1} and beta_{k-2}, or beta0
// for k = 1). Launch 0 takes x_0 as it is. Every launch leaves, for x_k:
// the partials (parity k & 1), x^H D x in two parts per tile (real part,
// length gauge; imaginary part, velocity gauge; times 2), and per segment
// sum E|x|^2 and |x|^2 (the segment's owner tile), and the owners store x_k
// (k >= 1).
struct LzFused {
    const double *xprev;   // k >= 1: x_{k-1}; k = 0: x_0
    const double *xprev2;  // x_{k-2} (k >= 2; any valid vector otherwise)
    double *xout;          // x_k (k >= 1)
    const double *qin, *ein, *nin;  // parts of x_{k-1}
    double *qout, *eout, *nout;     // parts of x_k
    const double *fsample; // this step's field sample
    double *alpha, *beta, *beta0;
    int32_t k;
    int32_t pad_;
};
hipError_t vec_launch_lz_fused(const VecBuffers &b, const LzFused &z, hipStream_t s);
// dt_dev: if not null, dt is read from there at run time (captured steps).
// dotp (one pulse, optional): alpha_{m-1} is the sum of its nseg parts.
hipError_t lz_expm(const double *alpha, const double *beta, const double *beta0, double dt, const double *dt_dev,
                   int m, int batch, double *y, const double *dotp, int nseg, hipStream_t s);
hipError_t lz_combine(const double *V, size_t vstride, const double *y, int m, int batch, int64_t ncplx, double *c,
                      double *ckpt, int64_t ckpt_rows, int64_t ckpt_row, hipStream_t s);
// One pulse, one launch per product: alpha_{m-1} and |x_{m-1}| from that
// launch's parts, the exponential, y_j scaled by beta0 / beta_{j-1} (for the
// recombination over the unnormalised x_j).
hipError_t lz_expm_fused(double *alpha, double *beta, double *beta0, const double *qin, const double *ein,
                         const double *nin, int nq, int nseg, const double *fsample, double dt,
                         const double *dt_dev, int m, double *y, hipStream_t s);
// One pulse: c = sum_j y_j v_j as lz_combine, also x0 = c (the next step's
// first Krylov vector, in place over v_0) and its norm parts.
hipError_t lz_combine_wide(double *V, const double *y, int m, int64_t ncplx, double *c, double *ckpt,
                           int64_t ckpt_row, double *normp, hipStream_t s);
hipError_t lz_ckpt0(const double *c0, double *ckpt, int batch, int64_t len, int64_t rows, hipStream_t s);

// ---------------------------------------------------------------------------
// Tile choices (autotuner cache).
struct TileChoice {
    int32_t T;        // single-vector path: tiles per block dimension (0 = default)
    int32_t tm, tn;   // batched path: output tile (0 = default)
    int32_t kc;       // batched path: contraction chunk staged per LDS buffer (0 = default)
    int32_t ks;       // batched path: K groups per workgroup (1, 2; 8 = the small-batch kernel; 0 = default)
};

// Reads $TDSE_TUNE_CACHE (written by tdse_tune) and $TDSE_TILE; leaves the
// arguments unchanged when there is no entry for (lmax, n, batch).
void tune_lookup(int lmax, int n, int batch, TileChoice *tc);
// Plan creation with an optional forced tile choice (used by the tuner).
tdse_status create_plan(tdse_plan *out, const double *energies, const double *dipole, int32_t gauge, int32_t lmax,
                        int32_t n, int32_t batch, hipStream_t s, const TileChoice *force);

}  // namespace tdse

// ---------------------------------------------------------------------------
struct tdse_group_s {
    std::vector<tdse_plan> plans;
    // per member: its blocks tiled at the default tile count, owned by the
    // group, where the plan itself was built with another count (else null)
    std::vector<double *> retiled;
    // work list and instance table of the last call (host copies stay alive
    // until the next call, so the asynchronous uploads can read them)
    std::vector<tdse::GroupTile> tiles;
    std::vector<tdse::GroupSeg> segs;
    std::vector<tdse::GroupInst> insts;
    tdse::GroupTile *d_tiles = nullptr;
    tdse::GroupSeg *d_segs = nullptr;
    tdse::GroupInst *d_insts = nullptr;
    size_t tiles_cap = 0, segs_cap = 0, insts_cap = 0;
    tdse::GroupDesc *d_desc = nullptr;
    // captured chunks of GROUP_CHUNK_ROUNDS rounds, keyed by their grid sizes
    // (tiles << 32 | segments: the active prefix of the work lists)
    std::map<int64_t, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
};

struct tdse_plan_s {
    int32_t lmax = 0, n = 0, batch = 1;
    // spectrum bounds for the stability test: max |E| and the largest absolute
    // row sum of the coupling (>= its spectral norm)
    double emax = 0.0, dnorm = 0.0;
    // tdse_propagate_adaptive workspace (first use): field samples, two states, errors
    double *ada_mem = nullptr;
    size_t ada_bytes = 0;
    int32_t gauge = 0;           // tdse_gauge of the coupling blocks
    int device = 0;
    // device copies of the Hamiltonian
    double *en = nullptr;
    double *dip = nullptr;
    int32_t ld = 0;
    // single-vector path
    int32_t T = 1;
    bool small = false;          // whole propagation in one workgroup
    bool split = false;          // separate completion and product launches (large problems)
    double *scratch = nullptr;   // one allocation holding states, partials, descriptor
    size_t scratch_bytes = 0;
    tdse::VecBuffers vb{};
    // batched path
    tdse::BatBuffers bb{};
    double *bat_mem = nullptr;
    // adjoint workspace (allocated on first use): forward-recompute state,
    // segment store of stage inputs, gradient partials, internal checkpoints
    double *adj_mem = nullptr;
    size_t adj_bytes = 0;
    // Lanczos workspace (allocated on first use): basis, product, coefficients
    double *lz_mem = nullptr;
    size_t lz_bytes = 0;
    // Runge-Kutta-Fehlberg workspace (batched plans, first use): k_1..k_5, error partials
    double *rkf_mem = nullptr;
    tdse_plan adj_plan = nullptr;   // batched twin of a batch-1 plan, for the adjoint
    // captured chunk graphs keyed by (method, order, chunk steps, parity)
    std::map<std::string, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
};
