// Single-vector (batch == 1) propagation kernels for gfx950.
//
// One launch per dipole product (an RK4 stage or a Taylor term; appendix B).
// The block-tridiagonal product of Sec. 4 is cut into tiles: tile (l, i, j)
// covers rows i and columns j of the stored superdiagonal block D_l
// (Sec. 5 stores only D_l; the l+1 -> l block is its transpose). Row and
// column segments come from the balanced split of Sec. 4.1. One workgroup
// reads its tile once and produces both uses of it:
//   row partial    r[a] = sum_b D_l[a,b] u_{l+1}[b]   (towards z_l, rows i)
//   column partial p[b] = sum_a D_l[a,b] u_l[a]       (towards z_{l+1}, cols j)
// so every stored dipole element is read once per product and no atomics
// are used (the paper's optimisation notes, Sec. 5.2). The partials of one
// launch are reduced in fixed order by the prologue of the next launch, which
// also completes the RK4 stage / Taylor term (the vector sums of Eqs.
// RKDeriv / RKFinal) and forms the next product's input, so a whole stage is
// one kernel. The prologue's loads are issued before the tile loads, so the
// completion arithmetic runs while the tile is still streaming in.
//
// Tiles are assigned to workgroups so that a tile always lands on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs) and each XCD
// works on a contiguous range of tiles.
#include "tdse_internal.h"
#include "tdse_reduce.h"

namespace tdse {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Coupling product of a state entry from its row-use part r (the block above,
// D_l u_{l+1}) and column-use part s (the block below, D_{l-1}^T u_{l-1}):
// length gauge r + s; velocity gauge, with the blocks holding Q of
// P = -i Q: -i (r - s).
__device__ __forceinline__ double2 couple(int gauge, double2 r, double2 s) {
    if (gauge) return make_double2(r.y - s.y, -(r.x - s.x));
    return make_double2(r.x + s.x, r.y + s.y);
}
template <int G>
__device__ __forceinline__ double2 couple_g(double2 r, double2 s) {
    if constexpr (G != 0) return make_double2(r.y - s.y, -(r.x - s.x));
    else return make_double2(r.x + s.x, r.y + s.y);
}

// 16-byte access to partials and state. Plain (cached) accesses: with the
// non-temporal hint a product at Lmax=15, N=500 took 6% longer -- the next
// launch's reads of the partials then came from further out.
typedef double dv2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld2(const double2 *p) {
    dv2_t v = *reinterpret_cast<const dv2_t *>(p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double2 *p, double2 v) {
    *reinterpret_cast<dv2_t *>(p) = dv2_t{v.x, v.y};
}
// Store through a pointer the compiler cannot trace to a kernel argument
// (one loaded from memory, or held in registers with pin_sgpr): spelled as a
// global-address-space store (a generic/flat store would also count against
// the LDS counter and force waits on the tile stream).
typedef __attribute__((address_space(1))) dv2_t gdv2_t;
__device__ __forceinline__ void st_global(double2 *p, double2 v) {
    dv2_t w = {v.x, v.y};
    *(gdv2_t *)(p) = w;
}
__device__ __forceinline__ double2 ld_global(const double2 *p) {
    const dv2_t v = *(const gdv2_t *)(p);
    return make_double2(v.x, v.y);
}

// Tile loads that may be skipped (all-padding parts of a tile), as raw buffer
// loads over the one tile: a skipped load gets an offset past the buffer's
// end, which the hardware answers with zeros and no memory access. Every load
// is issued either way, so the wait counter stays exact; with loads under
// branches the compiler has to wait for all of them before the first use of
// anything loaded earlier. Used by the Krylov products launch (the
// recurrence's alpha is needed early) and, with the LDS bit, by the patch
// products launch (its explicit waits count every load). 0x00020000: the
// fourth descriptor word for untyped buffer access on gfx9-family GPUs.
constexpr int TILE_BYTES = VEC_TILE_MAX * VEC_TILE_MAX * 8;
constexpr int TILE_SKIP = 0x40000000;  // offset of a skipped load (past the end)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const double *dip, int tile) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(dip) + (size_t)tile * (TILE_BYTES / 8), 0,
                                             TILE_BYTES, 0x00020000);
}
__device__ __forceinline__ double2 tile_ld(__amdgpu_buffer_rsrc_t rs, int off) {
    const dv2_t v = __builtin_bit_cast(dv2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    return make_double2(v.x, v.y);
}

// Keeps a wave-uniform value in scalar registers at this point of the
// program: the scalar load that produces it is issued here rather than sunk
// towards its first use, where its round trip would join the critical path.
// (An empty statement with a register operand: no instruction is emitted.)
template <typename T>
__device__ __forceinline__ void pin_sgpr(T &v) {
    asm volatile("" : "+s"(v));
}

// Workgroup barrier that orders LDS only. __syncthreads() also orders global
// memory, which on gfx9 waits for every outstanding global load and store
// (vmcnt(0)) -- including the tile stream this kernel wants to keep in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// y = H u_prev = E0 u + F z ; k = -i y. Then the RK4 / Taylor bookkeeping.
__device__ __forceinline__ void apply_completion(const Completion &cp, double dt, double F,
                                                 double E0, double2 z, double2 &c,
                                                 double2 &acc, double2 &u) {
    double yr = fma(F, z.x, E0 * u.x);
    double yi = fma(F, z.y, E0 * u.y);
    double kr = yi, ki = -yr;
    switch (cp.kind) {
    case CK_RK4_MID: {
        double w = cp.w_acc;
        if (cp.first) {
            acc.x = w * kr;
            acc.y = w * ki;
        } else {
            acc.x = fma(w, kr, acc.x);
            acc.y = fma(w, ki, acc.y);
        }
        double a = cp.a_next * dt;
        u.x = fma(a, kr, c.x);
        u.y = fma(a, ki, c.y);
        break;
    }
    case CK_RK4_END: {
        // c' = c + dt (acc + k4 / 6)
        double sx = fma(cp.w_acc, kr, acc.x), sy = fma(cp.w_acc, ki, acc.y);
        c.x = fma(dt, sx, c.x);
        c.y = fma(dt, sy, c.y);
        u = c;
        acc = make_double2(0.0, 0.0);
        break;
    }
    case CK_TAY_MID: {
        double s = cp.a_next * dt;  // dt / m
        double tr = s * kr, ti = s * ki;
        acc.x += tr;
        acc.y += ti;
        u = make_double2(tr, ti);
        break;
    }
    default: {  // CK_TAY_END
        double s = cp.a_next * dt;
        acc.x = fma(s, kr, acc.x);
        acc.y = fma(s, ki, acc.y);
        c = acc;
        u = acc;
        break;
    }
    }
}

// Buffer pointers by parity, selected without indexing the kernel-argument
// struct at run time (that would turn into a dependent memory load).
__device__ __forceinline__ double2 *st_ptr(const VecBuffers &b, int par, int v) {
    if (v == 0) return par ? b.side[1].st[0] : b.side[0].st[0];
    if (v == 1) return par ? b.side[1].st[1] : b.side[0].st[1];
    return par ? b.side[1].st[2] : b.side[0].st[2];
}
__device__ __forceinline__ double2 *rowp_ptr(const VecBuffers &b, int par) { return par ? b.side[1].rowp : b.side[0].rowp; }
__device__ __forceinline__ double2 *colp_ptr(const VecBuffers &b, int par) { return par ? b.side[1].colp : b.side[0].colp; }

__device__ __forceinline__ bool is_end(int kind) { return kind == CK_RK4_END || kind == CK_TAY_END; }

// Field sample of the product a launch completes, from the chunk's staged copy.
__device__ __forceinline__ double field_of(const CallDesc *d, const VecLaunch &L) {
    return d->chunk_field[(L.off + L.comp.step_delta + 1) * L.slots + L.comp.slot];
}

// Sum of the partials of one kind for state entry e of segment (m, q):
// rows=true: the np row partials of segment (m, q) (tiles (m, q, 0..T-1) when
// np == T, one per tile; one per patch column of block m for patch
// products); rows=false: the np column partials of segment (m, q) from block
// m-1, in ascending order. The TP >= np loads are unconditional (indices
// clamped into the buffer) and invalid terms are dropped afterwards, so the
// loads issue back to back.
template <int TP>
struct PartialLoads {
    double2 v[TP];
    bool valid;
};

template <int TP>
__device__ __forceinline__ PartialLoads<TP> load_partials(const VecBuffers &b, int T, int np, int par, bool rows,
                                                          int m, int q, int e) {
    PartialLoads<TP> p;
    p.valid = rows ? (m < b.lmax) : (m > 0);
    const int hi = b.lmax > 0 ? b.lmax - 1 : 0;
    int mb = rows ? m : m - 1;
    mb = mb < 0 ? 0 : (mb > hi ? hi : mb);
    double2 *pr = rowp_ptr(b, par), *pc = colp_ptr(b, par);
    const double2 *base = (rows ? pr : pc) + ((size_t)(mb * T + q) * np) * VEC_TILE_MAX + e;
#pragma unroll
    for (int k = 0; k < TP; ++k) p.v[k] = ld2(base + (size_t)(k < np ? k : np - 1) * VEC_TILE_MAX);
    return p;
}

// Fixed-order sum of the loaded partials (contributions k = 0 .. np-1).
template <int TP>
__device__ __forceinline__ double2 add_partials(const PartialLoads<TP> &p, int np) {
    double zx = 0.0, zy = 0.0;
#pragma unroll
    for (int k = 0; k < TP; ++k) {
        zx += k < np ? p.v[k].x : 0.0;
        zy += k < np ? p.v[k].y : 0.0;
    }
    return p.valid ? make_double2(zx, zy) : make_double2(0.0, 0.0);
}

template <int TP>
__device__ __forceinline__ double2 sum_partials(const VecBuffers &b, int T, int np, int par, bool rows, int m,
                                                int q, int e) {
    return add_partials<TP>(load_partials<TP>(b, T, np, par, rows, m, q, e), np);
}

// Where (if anywhere) a launch's completion writes a checkpoint. Both
// descriptor words are read unconditionally and combined with selects, so
// the two scalar loads issue together and nothing branches on the first.
struct CkptTarget {
    double2 *slot;  // checkpoint row for this launch's completed step, or null
};

__device__ __forceinline__ CkptTarget ckpt_target(const VecBuffers &b, const VecLaunch &L,
                                                  const CallDesc *d) {
    double *ck = d->ckpt;
    const int64_t row = d->chunk_ckpt_row[L.off + L.comp.step_delta + 1];
    const bool on = (ck != nullptr) & is_end(L.comp.kind) & (row >= 0);
    CkptTarget t;
    t.slot = on ? reinterpret_cast<double2 *>(ck) + (size_t)row * (size_t)(b.lmax + 1) * b.n : nullptr;
    return t;
}

// Store the completed state of one entry (owner workgroup only) and, at the
// end of a step that is a checkpoint, c into the caller's checkpoint buffer.
__device__ __forceinline__ void store_state(const VecBuffers &b, const VecLaunch &L,
                                            const CkptTarget &ct, size_t gi, double2 c,
                                            double2 acc, double2 u) {
    const int par = L.parity;
    st2(st_ptr(b, par ^ 1, 0) + gi, c);
    st2(st_ptr(b, par ^ 1, 1) + gi, acc);
    st2(st_ptr(b, par ^ 1, 2) + gi, u);
    if (ct.slot) st_global(ct.slot + gi, c);
}

// Swap of 32-bit lane data between two registers: permlane32_swap exchanges
// the upper 32 lanes of x with the lower 32 lanes of y, permlane16_swap the
// odd 16-lane rows of x with the even rows of y. Adding the two results
// reduces x over lane bit 5 (resp. 4) in the lanes where that bit is clear and
// y in the lanes where it is set.
template <int BIT>
__device__ __forceinline__ double swap_reduce(double x, double y) {
    const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    const unsigned xl = (unsigned)bx, xh = (unsigned)(bx >> 32), yl = (unsigned)by, yh = (unsigned)(by >> 32);
    unsigned rl0, rl1, rh0, rh1;
    if constexpr (BIT == 5) {
        auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        rl0 = l[0], rl1 = l[1], rh0 = h[0], rh1 = h[1];
    } else {
        auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        rl0 = l[0], rl1 = l[1], rh0 = h[0], rh1 = h[1];
    }
    const double a = __longlong_as_double(((long long)rh0 << 32) | rl0);
    const double c = __longlong_as_double(((long long)rh1 << 32) | rl1);
    return a + c;
}

// LDS of a tile workgroup.
struct TileLds {
    double2 uA[VEC_TILE_MAX], uB[VEC_TILE_MAX];    // product inputs: segments (l, i), (l+1, j)
    double2 zc[2 * VEC_TILE_MAX];                  // column-partial sums for the completing threads
    double2 rbuf[VEC_THREADS / 64][VEC_TILE_MAX];  // [wave][row]
    double2 cbuf[VEC_TILE_MAX][17];                // [column][row class], padded
};

// Tile products of workgroup (l, i, j) from the tile data dv (tile_pos
// order, this lane's 16 loads) and the inputs in lds.uA / lds.uB: writes the
// row partials (towards z_l, rows i) and column partials (towards z_{l+1},
// columns j) to the partial buffers of parity npar.
// QF (Krylov products): also returns, in the row threads, this row's term of
// the tile's part of the quadratic form, conj(u_A[a]) (D_tile u_B)[a] -- its
// real part (length gauge) or imaginary part (velocity gauge, QF = 2); 0 in
// every other thread.
template <int QF = 0>
__device__ __forceinline__ double tile_products(const VecBuffers &b, TileLds &lds, const double2 (&dv)[16], int T,
                                                int l, int i, int j, int RA, int RB, int npar) {
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    // Output bases held in scalar registers: the two partial stores below sit
    // in branches on the thread index, and merged into one store they would
    // otherwise pick the base by a per-lane load of the kernel argument (a
    // vector load whose wait also drains every earlier store of the wave).
    double2 *colp_out = colp_ptr(b, npar), *rowp_out = rowp_ptr(b, npar);
    pin_sgpr(colp_out);
    pin_sgpr(rowp_out);
    // ---- tile products. Lane (h, qq) holds rows qq + 16k and columns
    // cb .. cb+3: dv[2k] = D[row k][cb, cb+1], dv[2k+1] = D[row k][cb+2, cb+3].
    const int h = lane >> 4, qq = lane & 15;
    const int cb = wv * 16 + 4 * h;
    const double2 ub0 = lds.uB[cb], ub1 = lds.uB[cb + 1], ub2 = lds.uB[cb + 2], ub3 = lds.uB[cb + 3];
    double2 cp[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) cp[c] = make_double2(0.0, 0.0);
    double tr[8], ti[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double2 d01 = dv[2 * k], d23 = dv[2 * k + 1];
        const double2 ua = lds.uA[qq + 16 * k];
        tr[k] = fma(d23.y, ub3.x, fma(d23.x, ub2.x, fma(d01.y, ub1.x, d01.x * ub0.x)));
        ti[k] = fma(d23.y, ub3.y, fma(d23.x, ub2.y, fma(d01.y, ub1.y, d01.x * ub0.y)));
        cp[0].x = fma(d01.x, ua.x, cp[0].x);
        cp[0].y = fma(d01.x, ua.y, cp[0].y);
        cp[1].x = fma(d01.y, ua.x, cp[1].x);
        cp[1].y = fma(d01.y, ua.y, cp[1].y);
        cp[2].x = fma(d23.x, ua.x, cp[2].x);
        cp[2].y = fma(d23.x, ua.y, cp[2].y);
        cp[3].x = fma(d23.y, ua.x, cp[3].x);
        cp[3].y = fma(d23.y, ua.y, cp[3].y);
    }
    // Row partials over the wave's 16 columns: reduce over lane bits 5 and 4
    // (the four column groups h). Afterwards a lane holds rows
    // qq + 16 (k + 2 bit4 + 4 bit5), k = 0, 1.
    double sr[4], si[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sr[k] = swap_reduce<5>(tr[k], tr[k + 4]);
        si[k] = swap_reduce<5>(ti[k], ti[k + 4]);
    }
    const int rcls = 2 * (h & 1) + 4 * (h >> 1);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double zr = swap_reduce<4>(sr[k], sr[k + 2]), zi = swap_reduce<4>(si[k], si[k + 2]);
        lds.rbuf[wv][qq + 16 * (k + rcls)] = make_double2(zr, zi);
    }
    // Column partials over the lane's 8 rows, per row class qq.
#pragma unroll
    for (int c = 0; c < 4; ++c) lds.cbuf[cb + c][qq] = cp[c];
    lds_barrier();

    if (t < VEC_TILE_MAX) {
        if (t < RB) {  // column partial of column t: sum over the 16 row classes
            double2 s = lds.cbuf[t][0];
#pragma unroll
            for (int k = 1; k < 16; ++k) s = cadd(s, lds.cbuf[t][k]);
            double2 *cpo = colp_out + ((size_t)(l * T + j) * T + i) * VEC_TILE_MAX;
            st_global(cpo + t, s);
        }
    } else if (t < 2 * VEC_TILE_MAX) {  // row partial of row a: sum over the 8 waves' columns
        const int a = t - VEC_TILE_MAX;
        if (a < RA) {
            double2 s = lds.rbuf[0][a];
#pragma unroll
            for (int k = 1; k < VEC_THREADS / 64; ++k) s = cadd(s, lds.rbuf[k][a]);
            double2 *rp = rowp_out + ((size_t)(l * T + i) * T + j) * VEC_TILE_MAX;
            st_global(rp + a, s);
            if constexpr (QF == 1) {
                const double2 ua = lds.uA[a];
                return fma(ua.x, s.x, ua.y * s.y);
            } else if constexpr (QF == 2) {
                const double2 ua = lds.uA[a];
                return fma(ua.x, s.y, -(ua.y * s.x));
            }
        }
    }
    return 0.0;
}

// One tile workgroup of the fused path: completes the previous product for
// segments A = (l, i) and B = (l+1, j) and produces this launch's row and
// column partials of tile (l, i, j). T is the number of tiles per block
// dimension (a compile-time constant where TP == T).
template <int TP, int G>
__device__ __forceinline__ void tile_body(const VecBuffers &b, const VecLaunch &L, int T, int l, int i, int j,
                                          int r0, int RA, int c0, int RB) {
    const int n = b.n;
    const int tile = (l * T + i) * T + j;

    __shared__ TileLds lds;

    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int par = L.parity;

    // ---- prologue loads: entry pe of segment A = (l, i) or B = (l+1, j).
    // Threads t and t+256 share an entry: the first loads the row partials
    // and the state, the second the column partials.
    const int pe = t & 255, half = __builtin_amdgcn_readfirstlane(t >> 8);  // wave-uniform
    const bool isB = pe >= VEC_TILE_MAX;
    const int e = pe & (VEC_TILE_MAX - 1);
    const int m = isB ? l + 1 : l, q = isB ? j : i, len = isB ? RB : RA, s0 = isB ? c0 : r0;
    const int ec = e < len ? e : len - 1;
    const size_t gi = (size_t)m * n + s0 + ec;
    const PartialLoads<TP> pl = load_partials<TP>(b, T, T, par, half == 0, m, q, ec);
    // The state is read by the completing half only.
    double2 c_in = make_double2(0.0, 0.0), acc_in = c_in, u_in = c_in;
    double E0 = 0.0;
    if (half == 0) {
        c_in = ld2(st_ptr(b, par, 0) + gi);
        acc_in = ld2(st_ptr(b, par, 1) + gi);
        u_in = ld2(st_ptr(b, par, 2) + gi);
        E0 = b.en[gi];
    }

    // ---- tile loads (stored in lane order, tile_pos): load jj of wave wv
    // reads 64 consecutive double2, one per lane. Rows and columns past the
    // segment are stored as zeros.
    const double2 *Dt = reinterpret_cast<const double2 *>(b.dip) +
                        (size_t)tile * (VEC_TILE_MAX * VEC_TILE_MAX / 2) + wv * 16 * 64 + lane;
    // The partial sums wait for the prologue loads only (issued first); they
    // are placed after the first EARLY tile loads are in flight, so the tile
    // stream is not held back by the prologue. With 8 partials per entry the
    // remaining loads are issued after the sum to stay within 128 VGPRs (with
    // 16 partials, all of them).
    constexpr int EARLY = TP <= 4 ? 16 : (TP <= 8 ? 8 : 0);
    double2 dv[16];
#pragma unroll
    for (int r = 0; r < EARLY; ++r) dv[r] = Dt[r * 64];
    __builtin_amdgcn_sched_barrier(0);
    // Per-call values (field sample, dt, checkpoint row) from the descriptor:
    // scalar loads issued behind the vector loads, first waited for by the
    // completion, so they add no round trip of their own to the launch.
    const CallDesc *d = b.desc;
    double F = field_of(d, L), dt = d->dt;
    CkptTarget ct = ckpt_target(b, L, d);
    pin_sgpr(F);
    pin_sgpr(dt);
    pin_sgpr(ct.slot);
    __builtin_amdgcn_sched_barrier(0);
    const double2 zpart = add_partials<TP>(pl, T);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = EARLY; r < 16; ++r) dv[r] = Dt[r * 64];

    // ---- completion of the previous product (overlaps the tile stream).
    if (half == 1) lds.zc[pe] = zpart;
    lds_barrier();
    double2 c = c_in, acc = acc_in, u = make_double2(0.0, 0.0);
    bool owner = false;
    if (half == 0) {
        if (e < len) {
            u = u_in;
            apply_completion(L.comp, dt, F, E0, couple_g<G>(zpart, lds.zc[pe]), c, acc, u);
            owner = isB ? (l == b.lmax - 1 && i == 0) : (j == 0);
        }
        (isB ? lds.uB : lds.uA)[e] = u;
    }
    lds_barrier();
    tile_products(b, lds, dv, T, l, i, j, RA, RB, par ^ 1);
    // The completed state is stored after the products: one counter covers
    // vector loads and stores, so a store issued before them would be waited
    // for together with the last tile loads.
    if (owner) store_state(b, L, ct, gi, c, acc, u);
}

// Start and length of segment q of n split over T (seg_start / seg_len: the
// Sec. 4.1 split over 16-row units), without a dependent load: T is a
// compile-time constant where TP == T.
__device__ __forceinline__ void segment_of(int n, int T, int q, int *start, int *len) {
    const int U = (n + 15) >> 4, div = U / T, rem = U - div * T;
    const int s = q * div + (q < rem ? q : rem), end = 16 * (s + div + (q < rem ? 1 : 0));
    *start = 16 * s;
    *len = (end < n ? end : n) - 16 * s;
}

// G: compile-time gauge (0 length, 1 velocity) of the fused kernel.
// The words a launch needs before its first memory access (the tile, the
// read side's partials and state, lmax and n: 14 dwords) come as leading
// scalar arguments as well as inside b. Leading scalar arguments are
// preloaded into scalar registers before the wave starts (kernel-argument
// preloading, built with -amdgpu-kernarg-preload-count), so the prologue's
// loads do not wait for a kernel-argument fetch: 5.24 -> 5.06 us per
// product at Lmax=15, N=500. (Preloading E, the call descriptor and the
// field sample's index instead of acc and u, which then sit at fixed
// offsets from c, measured 5.19 us.)
template <int TP, int G>
__global__ __launch_bounds__(VEC_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void vec_tiles_kernel(
    const double *dip, double2 *st_c, double2 *st_acc, double2 *st_u, double2 *rowp, double2 *colp, int32_t lmax,
    int32_t n, VecBuffers bk, VecLaunch L) {
    VecBuffers b = bk;
    b.dip = dip;
    b.side[0].st[0] = st_c;
    b.side[0].st[1] = st_acc;
    b.side[0].st[2] = st_u;
    b.side[0].rowp = rowp;
    b.side[0].colp = colp;
    b.lmax = lmax;
    b.n = n;
    // TP == T for T <= 8, so the tile decode divides by compile-time constants.
    const int T = TP <= 8 ? TP : b.T;
    const int ntiles = b.lmax * T * T;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);  // Sec. 4.1 split over XCDs
    const int l = tile / (T * T), rem = tile - l * T * T, i = rem / T, j = rem - i * T;
    int r0, RA, c0, RB;
    segment_of(b.n, T, i, &r0, &RA);
    segment_of(b.n, T, j, &c0, &RB);
    // The launcher hands every launch its buffers in parity-0 order (see
    // vec_launch_tiles), so no buffer pointer is chosen at run time.
    VecLaunch L0 = L;
    L0.parity = 0;
    tile_body<TP, G>(b, L0, T, l, i, j, r0, RA, c0, RB);
}

// ---------------------------------------------------------------------------
// Patch products: the products launch of the split path and of uneven
// groups, where the dipole streams from HBM. A workgroup takes a patch of
// PI x PJ tiles (at most PATCH_MAX each way; the Sec. 4.1 split of a block's
// T tile rows and columns over patch_np(T) patches each way) of one block
// D_l: tile rows ti0 .. ti0+PI-1, tile columns tj0 .. tj0+PJ-1. Each wave
// streams its 16 KB slice of every tile of the patch (wave w: columns 16w ..
// 16w+15, the tile_pos order of the fused kernel) straight into LDS with
// buffer loads that carry the LDS bit: LOOK loads of 1 KB in flight per wave
// through a ring of PATCH_RING slots, so no registers are tied up by data in
// flight and the stream runs on across tile boundaries. Parts of a tile that
// are all padding are not fetched (out-of-range offsets).
//   Row partials (towards z_l) accumulate over the patch's PJ tiles of a
//   tile row in registers and are kept per tile row; column partials
//   (towards z_{l+1}) accumulate over the patch's PI tile rows. Both are
//   summed across lanes and waves only once the patch's stream has ended:
//   the columns over the 16 row classes of a wave by lane shuffles, the rows
//   over the 8 waves in the ring's LDS. Nothing waits on the other waves
//   while the stream runs.
// A patch leaves one row partial per row segment and one column partial per
// column segment, so a segment collects patch_np(T) of each (T when every
// tile is a workgroup of its own), and the workgroup turns over once per
// patch rather than once per tile. The LDS (144 KB) admits one workgroup
// per CU: 8 waves, LOOK KB in flight per wave.
constexpr int PATCH_RING = 16;  // 1 KB slots per wave: one tile slice, so load r of a tile uses slot r
// Loads in flight per wave: 8, 10, 12 and 14 measured within 1% of each
// other on both streaming workloads (10 the fastest by a hair).
constexpr int PATCH_LOOK = 10;

typedef __attribute__((address_space(3))) void lds_void_t;

struct PatchLds {
    char ring[VEC_THREADS / 64][PATCH_RING][1024];  // [wave][slot]; after the stream, the row sums
    double2 uA[PATCH_MAX][VEC_TILE_MAX];            // inputs of the row segments (l, ti0 + ii)
    double2 uB[PATCH_MAX][VEC_TILE_MAX];            // inputs of the column segments (l+1, tj0 + jj)
};

// What a patch workgroup reads and writes, copied into scalar registers at
// kernel entry (a group's instance buffers live in device memory, and every
// explicit wait below is a compiler memory barrier that would otherwise have
// them re-read, each re-read waiting for the whole stream).
struct PatchArgs {
    const double *dip;     // tiles of the plan
    const double2 *u;      // product inputs: the stage inputs completed by the preceding combine launch
    double2 *rowp, *colp;  // partials written (np per segment and direction)
    int n, T;
};

__device__ __forceinline__ PatchArgs patch_args(const VecBuffers &b, int par) {
    PatchArgs a{b.dip, st_ptr(b, par ^ 1, 2), rowp_ptr(b, par ^ 1), colp_ptr(b, par ^ 1), b.n, b.T};
    pin_sgpr(a.dip);
    pin_sgpr(a.u);
    pin_sgpr(a.rowp);
    pin_sgpr(a.colp);
    pin_sgpr(a.n);
    pin_sgpr(a.T);
    return a;
}

// Stream state of one tile of a patch: a buffer descriptor over the tile (no
// records past the patch's last tile, so loads beyond it fetch nothing) and
// the tile's valid rows and columns.
struct PatchTile {
    __amdgpu_buffer_rsrc_t rs;
    int ra, rb;
};

// Tile row / column of the patch that the stream visits at position x of n:
// in order, or (rev) from the last one back.
__device__ __forceinline__ int patch_pos(int x, int n, int rev) { return rev ? n - 1 - x : x; }

// The tile visited at stream position (ii, jj) (ii == PI: past the last one).
__device__ __forceinline__ PatchTile patch_tile(const PatchArgs &A, int l, int ti0, int tj0, int PI, int PJ, int rev,
                                                int ii, int jj) {
    const int T = A.T;
    const bool live = ii < PI;
    const int i = ti0 + (live ? patch_pos(ii, PI, rev) : 0), j = tj0 + patch_pos(jj, PJ, rev);
    int r0, ra, c0, rb;
    segment_of(A.n, T, i, &r0, &ra);
    segment_of(A.n, T, j, &c0, &rb);
    PatchTile pt;
    pt.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(A.dip) + (size_t)((l * T + i) * T + j) * (TILE_BYTES / 8),
                                              0, live ? TILE_BYTES : 0, 0x00020000);
    pt.ra = live ? ra : 0;
    pt.rb = live ? rb : 0;
    return pt;
}

// Load r of this wave's slice of a tile into ring slot r: lane (h, q) of wave
// w fetches the double2 at 64 (16 w + r) + 16 h + q, i.e. rows q + 16 (r/2),
// columns 16 w + 4 h + 2 (r % 2) + {0, 1}; row groups at or past ra and
// column pairs at or past rb are not fetched.
__device__ __forceinline__ void patch_issue(const PatchTile &pt, int r, char *ring, int lane_off, int cb) {
    const bool need = 16 * (r >> 1) < pt.ra && cb + 2 * (r & 1) < pt.rb;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(pt.rs, (lds_void_t *)(ring + r * 1024), 16,
                                             need ? lane_off + r * 1024 : TILE_SKIP, 0, 0, 0);
}

// Workgroup barrier for LDS written with ds instructions only (a barrier with
// a memory fence would also wait for the ring's loads).
__device__ __forceinline__ void patch_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// LDS accesses of the patch kernel, through byte pointers: the compiler then
// does not tie them to the ring's in-flight loads (it would wait for every
// one of them before any access to the workgroup's LDS). The ring is read
// only after an explicit wait for the loads that fill it; the other arrays
// are written with ds instructions only.
__device__ __forceinline__ double2 lds_ld2(const char *p) {
    const dv2_t v = *reinterpret_cast<const dv2_t *>(p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void lds_st2(char *p, double2 v) { *reinterpret_cast<dv2_t *>(p) = dv2_t{v.x, v.y}; }

// Patch (pr, pc) of block l: reads the inputs A.u, writes the partials in
// the np-per-segment layout. LOOK (even, 8 .. 14): loads in flight per wave.
// rev: visit the patch's tiles from the last back to the first. Launches
// alternate the direction, so each starts on the tiles the one before it
// streamed last, part of which the GPU's memory-side cache (MALL) still holds:
// a products launch over 504 MB of tiles takes about 8% less time than with
// one direction throughout.
template <int LOOK>
__device__ __forceinline__ void patch_body(const PatchArgs &A, int np, int l, int pr, int pc, int rev) {
    static_assert(LOOK % 2 == 0 && LOOK >= 4 && LOOK <= PATCH_RING - 2, "a slot is refilled only after its data was used");
    __shared__ PatchLds lds;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int h = lane >> 4, qq = lane & 15, cb = wv * 16 + 4 * h;
    const int T = A.T, n = A.n;
    const int ti0 = (int)split_start(T, np, pr), PI = (int)split_len(T, np, pr);
    const int tj0 = (int)split_start(T, np, pc), PJ = (int)split_len(T, np, pc);
    const double2 *u = A.u;
    char *ring = lds.ring[wv][0], *ring0 = lds.ring[0][0];
    char *uab = reinterpret_cast<char *>(&lds.uA[0][0]), *ubb = reinterpret_cast<char *>(&lds.uB[0][0]);
    const int lane_off = wv * 16 * 1024 + lane * 16;

    // ---- inputs into LDS, zero past each segment: thread t loads entry
    // t % 128 of row segment t / 128 and of column segment t / 128
    double2 ua_in, ub_in;
    {
        const int x = t >> 7, e = t & (VEC_TILE_MAX - 1);
        int r0, ra, c0, rb;
        segment_of(n, T, ti0 + (x < PI ? x : 0), &r0, &ra);
        segment_of(n, T, tj0 + (x < PJ ? x : 0), &c0, &rb);
        const bool oka = x < PI && e < ra, okb = x < PJ && e < rb;
        const double2 va = ld_global(u + (size_t)l * n + r0 + (oka ? e : 0));
        const double2 vb = ld_global(u + (size_t)(l + 1) * n + c0 + (okb ? e : 0));
        ua_in = oka ? va : make_double2(0.0, 0.0);
        ub_in = okb ? vb : make_double2(0.0, 0.0);
    }
    // The ring starts zeroed: slots a skipped load leaves alone then hold
    // zeros or an earlier tile's (finite) values, which only meet zero inputs
    // or feed partials that are not stored.
#pragma unroll
    for (int r = 0; r < PATCH_RING; ++r) *reinterpret_cast<dv2_t *>(ring + r * 1024 + lane * 16) = dv2_t{0.0, 0.0};
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");

    // ---- the stream: loads 0 .. LOOK-1 of the first tile
    PatchTile cur = patch_tile(A, l, ti0, tj0, PI, PJ, rev, 0, 0);
#pragma unroll
    for (int r = 0; r < LOOK; ++r) patch_issue(cur, r, ring, lane_off, cb);
    lds_st2(uab + t * 16, ua_in);  // uA[t / 128][t % 128]
    lds_st2(ubb + t * 16, ub_in);
    patch_barrier();
    // the data of loads 0 and 1 (each step below reads the next pair ahead)
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOOK - 2) : "memory");
    double2 d0 = lds_ld2(ring + lane * 16), d1 = lds_ld2(ring + 1024 + lane * 16);

    double2 col[PATCH_MAX][4];
#pragma unroll
    for (int jj = 0; jj < PATCH_MAX; ++jj)
#pragma unroll
        for (int c = 0; c < 4; ++c) col[jj][c] = make_double2(0.0, 0.0);
    // row sums of each tile row, reduced over the wave's column groups:
    // rows[ii][k] holds rows qq + 16 (k + rcls) (k = 0, 1) of tile row ii
    const int rcls = 2 * (h & 1) + 4 * (h >> 1);
    double2 rows[PATCH_MAX][2];
#pragma unroll
    for (int x = 0; x < PATCH_MAX; ++x) rows[x][0] = rows[x][1] = make_double2(0.0, 0.0);

    // (tile rows unrolled: the row sums then stay in registers)
#pragma unroll
    for (int ii = 0; ii < PATCH_MAX; ++ii) {
        if (ii >= PI) break;
        const int ai = patch_pos(ii, PI, rev);  // tile row of the patch
        double2 ua[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) ua[k] = lds_ld2(uab + (ai * VEC_TILE_MAX + qq + 16 * k) * 16);
        double tr[8], ti[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) tr[k] = ti[k] = 0.0;
#pragma unroll
        for (int jj = 0; jj < PATCH_MAX; ++jj) {
            if (jj < PJ) {
                const bool row_end = jj + 1 >= PJ;
                const PatchTile nxt =
                    patch_tile(A, l, ti0, tj0, PI, PJ, rev, row_end ? ii + 1 : ii, row_end ? 0 : jj + 1);
                const int aj = patch_pos(jj, PJ, rev);  // tile column of the patch
                double2 ub[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) ub[c] = lds_ld2(ubb + (aj * VEC_TILE_MAX + cb + c) * 16);
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) {
                    // keep LOOK loads ahead: this tile's loads up to 15, then the next tile's
                    const int r = 2 * kk + LOOK;
                    if (r < PATCH_RING) {
                        patch_issue(cur, r, ring, lane_off, cb);
                        patch_issue(cur, r + 1, ring, lane_off, cb);
                    } else {
                        patch_issue(nxt, r - PATCH_RING, ring, lane_off, cb);
                        patch_issue(nxt, r + 1 - PATCH_RING, ring, lane_off, cb);
                    }
                    // the pair after this one has landed: read it ahead
                    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LOOK - 2) : "memory");
                    const int rn = (2 * kk + 2) & (PATCH_RING - 1);
                    const double2 n0 = lds_ld2(ring + rn * 1024 + lane * 16);
                    const double2 n1 = lds_ld2(ring + (rn + 1) * 1024 + lane * 16);
                    // d0 = D[row qq+16kk][cb, cb+1], d1 = D[row qq+16kk][cb+2, cb+3]
                    tr[kk] = fma(d1.y, ub[3].x, fma(d1.x, ub[2].x, fma(d0.y, ub[1].x, fma(d0.x, ub[0].x, tr[kk]))));
                    ti[kk] = fma(d1.y, ub[3].y, fma(d1.x, ub[2].y, fma(d0.y, ub[1].y, fma(d0.x, ub[0].y, ti[kk]))));
                    const double2 a = ua[kk];
                    col[jj][0].x = fma(d0.x, a.x, col[jj][0].x);
                    col[jj][0].y = fma(d0.x, a.y, col[jj][0].y);
                    col[jj][1].x = fma(d0.y, a.x, col[jj][1].x);
                    col[jj][1].y = fma(d0.y, a.y, col[jj][1].y);
                    col[jj][2].x = fma(d1.x, a.x, col[jj][2].x);
                    col[jj][2].y = fma(d1.x, a.y, col[jj][2].y);
                    col[jj][3].x = fma(d1.y, a.x, col[jj][3].x);
                    col[jj][3].y = fma(d1.y, a.y, col[jj][3].y);
                    d0 = n0;
                    d1 = n1;
                }
                cur = nxt;
            }
        }
        // row sums of tile row ii over the wave's column groups (lane bits 5, 4)
        double sr[4], si[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sr[k] = swap_reduce<5>(tr[k], tr[k + 4]);
            si[k] = swap_reduce<5>(ti[k], ti[k + 4]);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
            rows[ii][k] = make_double2(swap_reduce<4>(sr[k], sr[k + 2]), swap_reduce<4>(si[k], si[k + 2]));
    }
    // ---- the stream has ended (its last loads fetch nothing); every wave's
    // ring is free once all waves are here
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    patch_barrier();
    // row partials: the 8 waves' sums of each row, in a fixed order (rows[x]
    // holds the tile row visited x-th; past PI, zeros into unused space)
#pragma unroll
    for (int x = 0; x < PATCH_MAX; ++x) {
        const int ax = x < PI ? patch_pos(x, PI, rev) : x;
#pragma unroll
        for (int k = 0; k < 2; ++k)
            lds_st2(ring0 + ((ax * (VEC_THREADS / 64) + wv) * VEC_TILE_MAX + qq + 16 * (k + rcls)) * 16, rows[x][k]);
    }
    patch_barrier();
    {
        const int x = t >> 7, a = t & (VEC_TILE_MAX - 1);
        int r0, ra;
        segment_of(n, T, ti0 + (x < PI ? x : 0), &r0, &ra);
        if (x < PI && a < ra) {
            const char *base = ring0 + (x * (VEC_THREADS / 64) * VEC_TILE_MAX + a) * 16;
            double2 z = lds_ld2(base);
#pragma unroll
            for (int w = 1; w < VEC_THREADS / 64; ++w) z = cadd(z, lds_ld2(base + w * VEC_TILE_MAX * 16));
            st_global(A.rowp + ((size_t)(l * T + ti0 + x) * np + pc) * VEC_TILE_MAX + a, z);
        }
    }
    // column partials: sum over the 16 row classes (lane bits 3..0), halving
    // the values each step; lane (h, q) ends with tile column jj = q / 4,
    // column cb + q % 4
    double v[8 * PATCH_MAX];
#pragma unroll
    for (int jj = 0; jj < PATCH_MAX; ++jj)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[(jj * 4 + c) * 2] = col[jj][c].x;
            v[(jj * 4 + c) * 2 + 1] = col[jj][c].y;
        }
#pragma unroll
    for (int bit = 3; bit >= 0; --bit) {
        const int half = 2 << bit;
        const bool hi = (lane >> bit) & 1;
#pragma unroll
        for (int x = 0; x < half; ++x) {
            const double send = hi ? v[x] : v[x + half];
            const double keep = hi ? v[x + half] : v[x];
            v[x] = keep + __shfl_xor(send, 1 << bit);
        }
    }
    {
        const int jj = qq >> 2, cc = cb + (qq & 3);  // jj: the tile column visited jj-th
        const int aj = jj < PJ ? patch_pos(jj, PJ, rev) : 0;
        int c0, rb;
        segment_of(n, T, tj0 + aj, &c0, &rb);
        if (jj < PJ && cc < rb)
            st_global(A.colp + ((size_t)(l * T + tj0 + aj) * np + pr) * VEC_TILE_MAX + cc, make_double2(v[0], v[1]));
    }
}

// Products launch of the split path (after a vec_combine launch): one
// workgroup per patch, patch_np(T)^2 patches per block.
template <int LOOK>
__global__ __launch_bounds__(VEC_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void vec_patch_kernel(VecBuffers b, VecLaunch L) {
    const int np = patch_np(b.T);
    const int w = blockIdx.x, per = np * np;
    const int l = w / per, rem = w - l * per;
    patch_body<LOOK>(patch_args(b, L.parity), np, l, rem / np, rem - (rem / np) * np, L.parity);
}

// Products launch of the next Krylov vector with the recurrence's update
// folded in (one pulse, lmax >= 1): the input segments are x_{j+1} = w -
// alpha_j v_j - beta_{j-1} v_{j-1}, alpha_j summed from the per-segment parts
// in every workgroup (while the tile loads are in flight). Segment (m, q) is
// owned by tile (m, q, 0) for m < lmax (its row-side input) and by tile
// (lmax - 1, 0, q) for m = lmax (its column-side input); the owner stores the
// segment of x_{j+1} and its part of |x_{j+1}|^2.
template <int TP>
__global__ __launch_bounds__(VEC_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void vec_lz_products_kernel(VecBuffers b, LzUpdate z) {
    __shared__ TileLds lds;
    __shared__ double red[VEC_THREADS / 64];
    __shared__ double nred[4];
    const int T = TP <= 8 ? TP : b.T;
    const int ntiles = b.lmax * T * T;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);
    const int l = tile / (T * T), rem = tile - l * T * T, i = rem / T, j = rem - i * T;
    int r0, RA, c0, RB;
    segment_of(b.n, T, i, &r0, &RA);
    segment_of(b.n, T, j, &c0, &RB);
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(b.dip, tile);
    const int lofs = (wv * 16 * 64 + lane) * 16;
    const bool isB = t >= VEC_TILE_MAX, seg_thread = t < 2 * VEC_TILE_MAX;
    const int e = t & (VEC_TILE_MAX - 1), len = isB ? RB : RA;
    const int sm = isB ? l + 1 : l;
    const size_t gi = (size_t)sm * b.n + (isB ? c0 : r0) + (e < len ? e : len - 1);
    // (plain doubles: vector-type members assigned under branches were kept
    // in scratch memory)
    double xr = 0.0, xi = 0.0, vr = 0.0, vi = 0.0, pr = 0.0, pi = 0.0;
    if (seg_thread) {
        const double2 x = ld2(reinterpret_cast<const double2 *>(z.w) + gi);
        const double2 v = ld2(reinterpret_cast<const double2 *>(z.vj) + gi);
        xr = x.x;
        xi = x.y;
        vr = v.x;
        vi = v.y;
        if (z.j > 0) {
            const double2 q = ld2(reinterpret_cast<const double2 *>(z.vjm1) + gi);
            pr = q.x;
            pi = q.y;
        }
    }
    const double bprev = z.j > 0 ? z.beta[z.j - 1] : 0.0;
    // Up to 2 * VEC_THREADS parts: two loads per thread at clamped indices,
    // issued before the tile loads, so that waiting for them leaves the tile
    // stream in flight (a loop would wait inside it, before the tile loads
    // are issued). More parts: a loop after the tile loads.
    const int nseg = z.nseg;
    const bool fixed = nseg <= 2 * VEC_THREADS;
    double d0 = 0.0, d1 = 0.0;
    if (fixed) {
        d0 = z.dotp[t < nseg ? t : nseg - 1];
        d1 = z.dotp[t + VEC_THREADS < nseg ? t + VEC_THREADS : nseg - 1];
    }
    const int cb = wv * 16 + 4 * (lane >> 4);
    double2 dv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const bool need = 16 * (r >> 1) < RA && cb + 2 * (r & 1) < RB;
        dv[r] = tile_ld(rs, need ? lofs + r * 64 * 16 : TILE_SKIP);
    }
    double dpart = (t < nseg ? d0 : 0.0) + (t + VEC_THREADS < nseg ? d1 : 0.0);
    if (!fixed)
        for (int k = t; k < nseg; k += VEC_THREADS) dpart += z.dotp[k];
    const double a = block_sum<VEC_THREADS>(dpart, red);
    if (w == 0 && t == 0) z.alpha[z.j] = a;
    // same operation order as lz_update_kernel
    xr -= a * vr;
    xi -= a * vi;
    if (z.j > 0) {
        xr -= bprev * pr;
        xi -= bprev * pi;
    }
    const bool live = seg_thread && e < len;
    const bool own = isB ? (l == b.lmax - 1 && i == 0) : (j == 0);
    if (live && own) st_global(reinterpret_cast<double2 *>(z.xnext) + gi, make_double2(xr, xi));
    if (seg_thread) {
        const double n2 = wave_sum(live ? fma(xr, xr, xi * xi) : 0.0);
        if (lane == 0) nred[wv] = n2;
        (isB ? lds.uB : lds.uA)[e] = live ? make_double2(xr, xi) : make_double2(0.0, 0.0);
    }
    lds_barrier();
    if (own && (t == 0 || t == VEC_TILE_MAX)) z.normp[sm * T + (isB ? j : i)] = nred[wv] + nred[wv + 1];
    tile_products(b, lds, dv, T, l, i, j, RA, RB, 0);
}

// One launch per Krylov product (see LzFused). The structure follows
// tile_body: prologue loads (half 0: row partials, x_{k-1}, x_{k-2}, E; half
// 1: column partials), the previous launch's parts, the tile stream, then the
// sums, the formation of this tile's two input segments of x_k, the tile
// products with the tile's quadratic-form term, and the parts of x_k.
template <int TP, int G>
__device__ __forceinline__ void lz_tile_body(const VecBuffers &b, const LzFused &z, int T, int l, int i, int j,
                                             int r0, int RA, int c0, int RB) {
    const int n = b.n;
    const int tile = (l * T + i) * T + j;
    __shared__ TileLds lds;
    __shared__ double red[3][VEC_THREADS / 64];
    __shared__ double sred[4][2];  // [wave of the input threads][e-part, n-part]
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int pe = t & 255, half = __builtin_amdgcn_readfirstlane(t >> 8);
    const bool isB = pe >= VEC_TILE_MAX;
    const int e = pe & (VEC_TILE_MAX - 1);
    const int m = isB ? l + 1 : l, q = isB ? j : i, len = isB ? RB : RA, s0 = isB ? c0 : r0;
    const int ec = e < len ? e : len - 1;
    const size_t gi = (size_t)m * n + s0 + ec;
    const int k = z.k;
    // prologue (the partials exist for k = 0 too; their values are unused then)
    const PartialLoads<TP> pl = load_partials<TP>(b, T, T, 0, half == 0, m, q, ec);
    double2 xp = make_double2(0.0, 0.0), xp2 = xp;
    double E0 = 0.0;
    if (half == 0) {
        xp = ld2(reinterpret_cast<const double2 *>(z.xprev) + gi);
        xp2 = ld2(reinterpret_cast<const double2 *>(z.xprev2) + gi);
        E0 = b.en[gi];
    }
    // parts of x_{k-1}: two per tile (at most 2 VEC_THREADS on this path, L
    // T^2 <= 512) and one per segment (at most 2 VEC_THREADS); loads at
    // clamped indices
    const int nq = 2 * b.lmax * T * T, nseg = (b.lmax + 1) * T;
    const int t2 = t + VEC_THREADS;
    const double qv0 = z.qin[t < nq ? t : nq - 1], qv1 = z.qin[t2 < nq ? t2 : nq - 1];
    const double ev0 = z.ein[t < nseg ? t : nseg - 1], nv0 = z.nin[t < nseg ? t : nseg - 1];
    const double ev1 = z.ein[t2 < nseg ? t2 : nseg - 1], nv1 = z.nin[t2 < nseg ? t2 : nseg - 1];
    // alpha_{k-2} and beta_{k-3} (beta0 for k = 2), stored by earlier launches
    const double a_pp = k >= 2 ? z.alpha[k - 2] : 0.0;
    const double b_ppp = k >= 3 ? z.beta[k - 3] : (k == 2 ? *z.beta0 : 0.0);
    const double F = *z.fsample;

    const double2 *Dt = reinterpret_cast<const double2 *>(b.dip) +
                        (size_t)tile * (VEC_TILE_MAX * VEC_TILE_MAX / 2) + wv * 16 * 64 + lane;
    constexpr int EARLY = TP <= 4 ? 16 : (TP <= 8 ? 8 : 0);
    double2 dv[16];
    // (in consumption order: the products use loads 2k and 2k + 1 together)
#pragma unroll
    for (int r = 0; r < EARLY; ++r) {
        dv[r] = Dt[r * 64];
        __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    // sums of the parts (every workgroup, same order)
    double qs = (t < nq ? qv0 : 0.0) + (t2 < nq ? qv1 : 0.0);
    double es = (t < nseg ? ev0 : 0.0) + (t2 < nseg ? ev1 : 0.0);
    double ns = (t < nseg ? nv0 : 0.0) + (t2 < nseg ? nv1 : 0.0);
    qs = wave_sum(qs);
    es = wave_sum(es);
    ns = wave_sum(ns);
    if (lane == 0) {
        red[0][wv] = qs;
        red[1][wv] = es;
        red[2][wv] = ns;
    }
    const double2 zpart = add_partials<TP>(pl, T);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = EARLY; r < 16; ++r) dv[r] = Dt[r * 64];
    if (half == 1) lds.zc[pe] = zpart;
    lds_barrier();
    double Q = red[0][0], Es = red[1][0], Ns = red[2][0];
#pragma unroll
    for (int w = 1; w < VEC_THREADS / 64; ++w) {
        Q += red[0][w];
        Es += red[1][w];
        Ns += red[2][w];
    }
    // beta_{k-2} = |x_{k-1}| (beta0 for k = 1) with the breakdown rule,
    // alpha_{k-1}, and the scales of v_{k-1} and v_{k-2}
    double bprev = sqrt(Ns);
    if (k >= 2 && bprev <= 1e-13 * (fabs(a_pp) + (k >= 3 ? b_ppp : 0.0))) bprev = 0.0;
    const double s1 = bprev > 0.0 ? 1.0 / bprev : 0.0;
    const double s2 = b_ppp > 0.0 ? 1.0 / b_ppp : 0.0;
    const double alpha = (Es + F * Q) * (s1 * s1);
    if (blockIdx.x == 0 && t == 0 && k >= 1) {
        z.alpha[k - 1] = alpha;
        if (k == 1) *z.beta0 = bprev;
        else z.beta[k - 2] = bprev;
    }
    // this tile's input segments of x_k
    double2 x = make_double2(0.0, 0.0);
    double epart = 0.0, npart = 0.0;
    bool owner = false;
    if (half == 0) {
        if (e < len) {
            if (k == 0) {
                x = xp;
            } else {
                const double2 w = couple_g<G>(zpart, lds.zc[pe]);
                const double2 v = make_double2(xp.x * s1, xp.y * s1);
                const double yr = fma(F, w.x * s1, E0 * v.x), yi = fma(F, w.y * s1, E0 * v.y);
                x.x = yr - alpha * v.x;
                x.y = yi - alpha * v.y;
                if (k >= 2) {
                    x.x -= bprev * (xp2.x * s2);
                    x.y -= bprev * (xp2.y * s2);
                }
            }
            const double a2 = fma(x.x, x.x, x.y * x.y);
            npart = a2;
            epart = E0 * a2;
            owner = isB ? (l == b.lmax - 1 && i == 0) : (j == 0);
        }
        (isB ? lds.uB : lds.uA)[e] = x;
        epart = wave_sum(epart);
        npart = wave_sum(npart);
        if (lane == 0) {
            sred[wv][0] = epart;
            sred[wv][1] = npart;
        }
    }
    lds_barrier();
    // the owner of each input segment stores its parts (threads 0 and 128:
    // the first thread of each half's segment)
    const bool seg_owner = isB ? (l == b.lmax - 1 && i == 0) : (j == 0);
    if (half == 0 && (pe == 0 || pe == VEC_TILE_MAX) && seg_owner) {
        const int sg = m * T + q, w0 = pe >> 6;
        z.eout[sg] = sred[w0][0] + sred[w0 + 1][0];
        z.nout[sg] = sred[w0][1] + sred[w0 + 1][1];
    }
    const double wq = tile_products<G == 0 ? 1 : 2>(b, lds, dv, T, l, i, j, RA, RB, 1);
    if (owner && k >= 1) st_global(reinterpret_cast<double2 *>(z.xout) + gi, x);
    // the two row waves' sums are two parts each (no barrier needed)
    if (wv == 2 || wv == 3) {
        const double sq = wave_sum(wq);
        if (lane == 0) z.qout[2 * tile + (wv - 2)] = 2.0 * sq;
    }
}

// As the tile kernel, with the words its first loads need (the tile, the
// read side's partials, x_{k-1}, x_{k-2}, lmax, n and k) as leading scalar
// arguments, preloaded into scalar registers.
template <int TP, int G>
__global__ __launch_bounds__(VEC_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void vec_lz_fused_kernel(
    const double *dip, double2 *rowp, double2 *colp, const double *xprev, const double *xprev2, int32_t lmax,
    int32_t n, int32_t k, VecBuffers bk, LzFused zk) {
    VecBuffers b = bk;
    b.dip = dip;
    b.side[0].rowp = rowp;
    b.side[0].colp = colp;
    b.lmax = lmax;
    b.n = n;
    LzFused z = zk;
    z.xprev = xprev;
    z.xprev2 = xprev2;
    z.k = k;
    const int T = TP <= 8 ? TP : b.T;
    const int ntiles = b.lmax * T * T;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);
    const int l = tile / (T * T), rem = tile - l * T * T, i = rem / T, j = rem - i * T;
    int r0, RA, c0, RB;
    segment_of(b.n, T, i, &r0, &RA);
    segment_of(b.n, T, j, &c0, &RB);
    lz_tile_body<TP, G>(b, z, T, l, i, j, r0, RA, c0, RB);
}

// Uneven group: every RK4 stage-round of the active instances is one
// combine launch over their segments (work list of (instance, m, q)) and one
// patch products launch over their blocks' patches (work list of (instance,
// l, patch row, patch column)); each instance brings its own buffers, tile
// count and field samples.
// RK4 launch schedule: round 4k+s completes stage s of step k (stage 4 of
// step k-1 for s == 0) and forms the input of the next stage.
__device__ __forceinline__ VecLaunch group_round_launch(int64_t round) {
    const int s = (int)(round & 3);
    VecLaunch L{};
    L.parity = (int)(round & 1);
    L.slots = 3;
    if (s == 0) L.comp = {CK_RK4_END, 2, -1, 0, 1.0 / 6.0, 0.0};
    else if (s == 1) L.comp = {CK_RK4_MID, 0, 0, 1, 1.0 / 6.0, 0.5};
    else if (s == 2) L.comp = {CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 0.5};
    else L.comp = {CK_RK4_MID, 1, 0, 0, 2.0 / 6.0, 1.0};
    return L;
}

// A group launch belongs to round desc->base_round + off; instances whose
// last round has passed leave at once (the grid covers the instances active
// at the start of a chunk of rounds).
__global__ __launch_bounds__(VEC_TILE_MAX) void vec_group_combine_kernel(const GroupSeg *segs, const GroupInst *insts,
                                                                          const GroupDesc *desc, int32_t off) {
    const GroupSeg gs = segs[blockIdx.x];
    const GroupInst &gi = insts[gs.inst];
    const int64_t round = desc->base_round + off;
    if (round >= 4 * gi.nsteps) return;
    const VecBuffers &b = gi.b;  // read in place: a local copy would be indexed through scratch
    const VecLaunch L = group_round_launch(round);
    const int e = threadIdx.x;
    const int len = (int)seg_len(b.n, b.T, gs.q);
    if (e >= len) return;
    const int64_t step = (round >> 2) + L.comp.step_delta;
    const double F = (step >= 0 && step < gi.nsteps) ? gi.field[step * 3 + L.comp.slot] : 0.0;
    const size_t g = (size_t)gs.m * b.n + seg_start(b.n, b.T, gs.q) + e;
    const int par = L.parity;
    // partials of the patch products launch (groups stream at T <= 8: at most two per segment)
    const int np = patch_np(b.T);
    const double2 z = couple(b.gauge, sum_partials<2>(b, b.T, np, par, true, gs.m, gs.q, e),
                             sum_partials<2>(b, b.T, np, par, false, gs.m, gs.q, e));
    double2 c = ld2(st_ptr(b, par, 0) + g), acc = ld2(st_ptr(b, par, 1) + g), u = ld2(st_ptr(b, par, 2) + g);
    apply_completion(L.comp, desc->dt, F, b.en[g], z, c, acc, u);
    store_state(b, L, CkptTarget{nullptr}, g, c, acc, u);
}

// Products round of a group: one workgroup per patch (GroupTile i, j: the
// patch's row and column within its block).
template <int LOOK>
__global__ __launch_bounds__(VEC_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void vec_group_patch_kernel(const GroupTile *tiles, const GroupInst *insts, const GroupDesc *desc, int32_t off) {
    const GroupTile gt = tiles[blockIdx.x];
    const GroupInst &gi = insts[gt.inst];
    const int64_t round = desc->base_round + off;
    if (round >= 4 * gi.nsteps) return;
    const PatchArgs A = patch_args(gi.b, (int)(round & 1));
    patch_body<LOOK>(A, patch_np(A.T), gt.l, gt.i, gt.j, (int)(round & 1));
}

__global__ void group_desc_kernel(GroupDesc *desc, int64_t base_round, double dt) {
    desc->base_round = base_round;
    desc->dt = dt;
}

// Completion only (no products): the completion launch of the split path,
// the final completion of a propagation, every launch when lmax == 0 (no
// dipole blocks, z == 0), and the single product of tdse_hmul (kind CK_HMUL:
// y = E o u + F z). TP bounds the partials per segment, np = L.np (or T).
template <int TP>
__global__ __launch_bounds__(VEC_TILE_MAX) void vec_combine_kernel(VecBuffers b, VecLaunch L) {
    const int T = b.T, np = L.np > 0 ? L.np : T;
    const int seg = blockIdx.x;
    const int m = seg / T, q = seg - m * T;
    const int s0 = (int)seg_start(b.n, T, q), len = (int)seg_len(b.n, T, q);
    const int e = threadIdx.x;
    if (e >= len) return;
    const CallDesc *d = b.desc;
    const int par = L.parity;
    const double F = field_of(d, L);
    const size_t gi = (size_t)m * b.n + s0 + e;
    double2 z = make_double2(0.0, 0.0);
    if (b.lmax > 0)
        z = couple(b.gauge, sum_partials<TP>(b, T, np, par, true, m, q, e),
                   sum_partials<TP>(b, T, np, par, false, m, q, e));
    double2 c = ld2(st_ptr(b, par, 0) + gi), acc = ld2(st_ptr(b, par, 1) + gi), u = ld2(st_ptr(b, par, 2) + gi);
    const double E0 = b.en[gi];
    if (L.comp.kind == CK_HMUL) {
        double yr = fma(F, z.x, E0 * u.x), yi = fma(F, z.y, E0 * u.y);
        reinterpret_cast<double2 *>(L.out)[gi] = make_double2(yr, yi);
        return;
    }
    apply_completion(L.comp, d->dt, F, E0, z, c, acc, u);
    store_state(b, L, ckpt_target(b, L, d), gi, c, acc, u);
    if (L.finish) reinterpret_cast<double2 *>(L.out)[gi] = c;
}

// Completion of the product of Krylov vector j (one pulse): the norm of the
// unnormalised x_j from the parts its forming launch left, beta (with the
// recurrence's breakdown rule: beta_{j-1} <= 1e-13 (|alpha_{j-1}| +
// beta_{j-2}) counts as zero), v_j = x_j / beta in place, y = H v_j = (E o x_j
// + F D x_j) / beta, and this segment's part of Re <v_j, y>, summed over the
// segment in a fixed order: dotp[segment].
// HASD: the plan has dipole blocks (lmax > 0); the two cases are separate
// straight-line bodies, so the loads issue without a branch between them
// (after a join the compiler waits for every outstanding load).
template <int TP, bool HASD>
__device__ __forceinline__ void hmul_dot_body(const VecBuffers &b, const VecLaunch &L, double *dotp,
                                              const LzNorm &nz) {
    __shared__ double red[VEC_TILE_MAX / 64];
    const int T = b.T, np = L.np > 0 ? L.np : T;
    const int seg = blockIdx.x;
    const int m = seg / T, q = seg - m * T;
    const int s0 = (int)seg_start(b.n, T, q), len = (int)seg_len(b.n, T, q);
    const int e = threadIdx.x;
    const int par = L.parity;
    const double F = field_of(b.desc, L);
    // the breakdown test's alpha_{j-1} and beta_{j-2}: loaded up front and
    // unconditionally (clamped indices; the unused values are dropped below)
    const double aprev_ld = nz.alpha[nz.j > 0 ? nz.j - 1 : 0];
    const double bprev_ld = nz.beta[nz.j > 1 ? nz.j - 2 : 0];
    const bool live = e < len;
    const int ee = live ? e : 0;
    const size_t gi = (size_t)m * b.n + s0 + ee;
    double2 *up = st_ptr(b, par, 2) + gi;
    // every load first, in the order the values are needed (unconditional,
    // at in-bounds indices): the vector entry, its energy, this thread's first
    // norm part, then the partials
    const double2 x = ld2(up);
    const double E0 = b.en[gi];
    const int nparts = nz.nparts;
    const double n0 = nz.normp[e < nparts ? e : nparts - 1];
    PartialLoads<TP> pr, pc;
    if constexpr (HASD) {
        pr = load_partials<TP>(b, T, np, par, true, m, q, ee);
        pc = load_partials<TP>(b, T, np, par, false, m, q, ee);
    }
    double nsum = e < nparts ? n0 : 0.0;
    if (nparts > VEC_TILE_MAX)  // (a loop here would wait for every load above)
        for (int k = e + VEC_TILE_MAX; k < nparts; k += VEC_TILE_MAX) nsum += nz.normp[k];
    double bj = sqrt(block_sum<VEC_TILE_MAX>(nsum, red));
    const double bprev = nz.j > 1 ? bprev_ld : 0.0;
    if (nz.j > 0 && bj <= 1e-13 * (fabs(aprev_ld) + bprev)) bj = 0.0;
    const double inv = bj > 0.0 ? 1.0 / bj : 0.0;
    if (seg == 0 && e == 0) {
        if (nz.j == 0) *nz.beta0 = bj;
        else nz.beta[nz.j - 1] = bj;
    }
    double2 z = make_double2(0.0, 0.0);
    if constexpr (HASD) z = couple(b.gauge, add_partials<TP>(pr, np), add_partials<TP>(pc, np));
    double dot = 0.0;
    if (live) {
        const double2 v = make_double2(x.x * inv, x.y * inv);
        const double yr = fma(F, z.x * inv, E0 * v.x), yi = fma(F, z.y * inv, E0 * v.y);
        st2(up, v);
        reinterpret_cast<double2 *>(L.out)[gi] = make_double2(yr, yi);
        dot = fma(v.x, yr, v.y * yi);
    }
    const double part = block_sum<VEC_TILE_MAX>(dot, red);
    if (e == 0) dotp[seg] = part;
}

template <int TP>
__global__ __launch_bounds__(VEC_TILE_MAX) void vec_hmul_dot_kernel(VecBuffers b, VecLaunch L, double *dotp,
                                                                    LzNorm nz) {
    if (b.lmax > 0) hmul_dot_body<TP, true>(b, L, dotp, nz);
    else hmul_dot_body<TP, false>(b, L, dotp, nz);
}

__global__ void vec_start_kernel(VecBuffers b, int par, const double2 *c0, int taylor) {
    const size_t ns = (size_t)(b.lmax + 1) * b.n;
    const size_t np = (size_t)b.lmax * b.T * b.T * VEC_TILE_MAX;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const double2 zero = make_double2(0.0, 0.0);
    double2 *sc = par ? b.side[1].st[0] : b.side[0].st[0];
    double2 *sa = par ? b.side[1].st[1] : b.side[0].st[1];
    double2 *su = par ? b.side[1].st[2] : b.side[0].st[2];
    double2 *rp = par ? b.side[1].rowp : b.side[0].rowp;
    double2 *cp = par ? b.side[1].colp : b.side[0].colp;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < ns; g += stride) {
        double2 c = c0[g];
        sc[g] = c;
        sa[g] = make_double2(taylor ? c.x : 0.0, taylor ? c.y : 0.0);
        su[g] = zero;
    }
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < np; g += stride) {
        rp[g] = zero;
        cp[g] = zero;
    }
}

// Re-layout of the caller's row-major blocks [lmax][n][n] into tiles
// [lmax][T][T][VEC_TILE_MAX * VEC_TILE_MAX] in tile_pos order, zero outside
// each tile's extent.
__global__ void vec_layout_kernel(const double *src, double *dst, int lmax, int n, int T) {
    const size_t tile_elems = (size_t)VEC_TILE_MAX * VEC_TILE_MAX;
    const size_t total = (size_t)lmax * T * T * tile_elems;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const size_t tile = g / tile_elems, w = g - tile * tile_elems;
        int a, bcol;
        tile_elem((int64_t)w, &a, &bcol);
        const int l = (int)(tile / (T * T)), rem = (int)(tile % (T * T)), i = rem / T, j = rem % T;
        const int RA = (int)seg_len(n, T, i), RB = (int)seg_len(n, T, j);
        double v = 0.0;
        if (a < RA && bcol < RB) {
            const int r = (int)seg_start(n, T, i) + a, c = (int)seg_start(n, T, j) + bcol;
            v = src[((size_t)l * n + r) * n + c];
        }
        dst[g] = v;
    }
}

// Inverse of vec_layout_kernel: tiles back to row-major [lmax][n][n].
__global__ void vec_untile_kernel(const double *tiles, double *dst, int lmax, int n, int T) {
    const size_t total = (size_t)lmax * n * n;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(g % n);
        const size_t rg = g / n;
        const int r = (int)(rg % n), l = (int)(rg / n);
        int i = 0, j = 0;
        while (i + 1 < T && seg_start(n, T, i + 1) <= r) ++i;
        while (j + 1 < T && seg_start(n, T, j + 1) <= c) ++j;
        const int a = r - (int)seg_start(n, T, i), bcol = c - (int)seg_start(n, T, j);
        dst[g] = tiles[(((size_t)l * T + i) * T + j) * VEC_TILE_MAX * VEC_TILE_MAX + tile_pos(a, bcol)];
    }
}

hipError_t vec_untile(const double *tiles, double *dst, int lmax, int n, int T, hipStream_t s) {
    hipLaunchKernelGGL(vec_untile_kernel, dim3(1024), dim3(256), 0, s, tiles, dst, lmax, n, T);
    return hipGetLastError();
}

hipError_t vec_layout(const double *src, double *dst, int lmax, int n, int T, hipStream_t s) {
    hipLaunchKernelGGL(vec_layout_kernel, dim3(1024), dim3(256), 0, s, src, dst, lmax, n, T);
    return hipGetLastError();
}

__global__ void set_desc_kernel(CallDesc *d, CallDesc v) {
    d->base_step = v.base_step;
    d->nsteps = v.nsteps;
    d->field = v.field;
    d->ckpt = v.ckpt;
    d->ckpt_every = v.ckpt_every;
    d->dt = v.dt;
    d->slots = v.slots;
}

// Stage the field samples of steps base-1 .. base+CHUNK_STEPS-1.
__global__ void chunk_begin_kernel(CallDesc *d, int64_t base) {
    const int S = d->slots;
    const int64_t nst = d->nsteps;
    const double *f = d->field;
    for (int x = threadIdx.x; x < (CHUNK_STEPS + 1) * S; x += blockDim.x) {
        const int64_t step = base - 1 + x / S;
        d->chunk_field[x] = (step >= 0 && step < nst) ? f[step * S + x % S] : 0.0;
    }
    const int64_t K = d->ckpt_every;
    for (int x = threadIdx.x; x <= CHUNK_STEPS; x += blockDim.x) {
        const int64_t ends = base + x;  // a completion at chunk offset x-1 ends this step
        d->chunk_ckpt_row[x] = (ends <= nst && ends % K == 0) ? ends / K : -1;
    }
    if (threadIdx.x == 0) d->base_step = base;
}

hipError_t set_desc(CallDesc *d, const CallDesc &v, hipStream_t s) {
    hipLaunchKernelGGL(set_desc_kernel, dim3(1), dim3(1), 0, s, d, v);
    return hipGetLastError();
}
hipError_t chunk_begin(CallDesc *d, int64_t base, hipStream_t s) {
    hipLaunchKernelGGL(chunk_begin_kernel, dim3(1), dim3(256), 0, s, d, base);
    return hipGetLastError();
}

// Compiled bounds on the number of tiles per block dimension.
#define TDSE_TP_DISPATCH(T, KERNEL, ...)                                        \
    do {                                                                        \
        switch (T) {                                                            \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;              \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;              \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;              \
        case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;              \
        case 5: hipLaunchKernelGGL(KERNEL<5>, __VA_ARGS__); break;              \
        case 6: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;              \
        case 7: hipLaunchKernelGGL(KERNEL<7>, __VA_ARGS__); break;              \
        case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;              \
        default:                                                                \
            if ((T) <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);         \
            else return hipErrorInvalidValue;                                   \
        }                                                                       \
    } while (0)

typedef void (*TilesKernel)(const double *, double2 *, double2 *, double2 *, double2 *, double2 *, int32_t, int32_t,
                            VecBuffers, VecLaunch);
template <int G>
static TilesKernel tiles_kernel_for(int T) {
    switch (T) {
    case 1: return vec_tiles_kernel<1, G>;
    case 2: return vec_tiles_kernel<2, G>;
    case 3: return vec_tiles_kernel<3, G>;
    case 4: return vec_tiles_kernel<4, G>;
    case 5: return vec_tiles_kernel<5, G>;
    case 6: return vec_tiles_kernel<6, G>;
    case 7: return vec_tiles_kernel<7, G>;
    case 8: return vec_tiles_kernel<8, G>;
    default: return T <= 16 ? vec_tiles_kernel<16, G> : nullptr;
    }
}

// The fused kernel reads the parity-0 buffers and writes the parity-1 ones: a
// launch of parity 1 is passed the buffer pairs exchanged instead, so the
// kernel's pointers are fixed kernel-argument words (a pointer picked by a
// run-time parity becomes a dependent load at kernel entry).
static VecBuffers parity_view(const VecBuffers &b, int parity) {
    VecBuffers v = b;
    if (parity) {
        v.side[0] = b.side[1];
        v.side[1] = b.side[0];
    }
    return v;
}

hipError_t vec_launch_tiles(const VecBuffers &b, const VecLaunch &l, hipStream_t s) {
    const int ntiles = b.lmax * b.T * b.T;
    TilesKernel k = b.gauge ? tiles_kernel_for<1>(b.T) : tiles_kernel_for<0>(b.T);
    if (!k) return hipErrorInvalidValue;
    VecLaunch l0 = l;
    l0.parity = 0;
    const VecBuffers v = parity_view(b, l.parity);
    hipLaunchKernelGGL(k, dim3(ntiles), dim3(VEC_THREADS), 0, s, v.dip, v.side[0].st[0], v.side[0].st[1],
                       v.side[0].st[2], v.side[0].rowp, v.side[0].colp, v.lmax, v.n, v, l0);
    return hipGetLastError();
}
hipError_t vec_launch_combine(const VecBuffers &b, const VecLaunch &l, hipStream_t s) {
    if (l.np > b.T) return hipErrorInvalidValue;
    TDSE_TP_DISPATCH(l.np > 0 ? l.np : b.T, vec_combine_kernel, dim3((b.lmax + 1) * b.T), dim3(VEC_TILE_MAX), 0, s, b,
                     l);
    return hipGetLastError();
}
hipError_t vec_launch_lz_products(const VecBuffers &b, const LzUpdate &z, hipStream_t s) {
    if (b.lmax == 0) return hipErrorInvalidValue;
    TDSE_TP_DISPATCH(b.T, vec_lz_products_kernel, dim3(b.lmax * b.T * b.T), dim3(VEC_THREADS), 0, s, b, z);
    return hipGetLastError();
}
typedef void (*LzFusedKernel)(const double *, double2 *, double2 *, const double *, const double *, int32_t, int32_t,
                              int32_t, VecBuffers, LzFused);
template <int G>
static LzFusedKernel lz_fused_kernel_for(int T) {
    switch (T) {
    case 1: return vec_lz_fused_kernel<1, G>;
    case 2: return vec_lz_fused_kernel<2, G>;
    case 3: return vec_lz_fused_kernel<3, G>;
    case 4: return vec_lz_fused_kernel<4, G>;
    case 5: return vec_lz_fused_kernel<5, G>;
    case 6: return vec_lz_fused_kernel<6, G>;
    case 7: return vec_lz_fused_kernel<7, G>;
    case 8: return vec_lz_fused_kernel<8, G>;
    default: return T <= 16 ? vec_lz_fused_kernel<16, G> : nullptr;
    }
}
// Launch k reads the partials of parity (k - 1) & 1 and writes parity k & 1:
// through the parity view, always "read side 0, write side 1".
hipError_t vec_launch_lz_fused(const VecBuffers &b, const LzFused &z, hipStream_t s) {
    const int ntiles = b.lmax * b.T * b.T;
    if (b.lmax == 0 || ntiles > VEC_THREADS || (b.lmax + 1) * b.T > 2 * VEC_THREADS) return hipErrorInvalidValue;
    LzFusedKernel k = b.gauge ? lz_fused_kernel_for<1>(b.T) : lz_fused_kernel_for<0>(b.T);
    if (!k) return hipErrorInvalidValue;
    const VecBuffers v = parity_view(b, (z.k + 1) & 1);
    hipLaunchKernelGGL(k, dim3(ntiles), dim3(VEC_THREADS), 0, s, v.dip, v.side[0].rowp, v.side[0].colp, z.xprev,
                       z.xprev2, v.lmax, v.n, z.k, v, z);
    return hipGetLastError();
}
hipError_t vec_launch_hmul_dot(const VecBuffers &b, const VecLaunch &l, double *dotp, const LzNorm &nz,
                               hipStream_t s) {
    if (l.np > b.T) return hipErrorInvalidValue;
    TDSE_TP_DISPATCH(l.np > 0 ? l.np : b.T, vec_hmul_dot_kernel, dim3((b.lmax + 1) * b.T), dim3(VEC_TILE_MAX), 0, s,
                     b, l, dotp, nz);
    return hipGetLastError();
}
hipError_t vec_launch_products(const VecBuffers &b, const VecLaunch &l, hipStream_t s) {
    const int np = patch_np(b.T);
    if (b.lmax == 0 || b.T > 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(vec_patch_kernel<PATCH_LOOK>, dim3(b.lmax * np * np), dim3(VEC_THREADS), 0, s, b, l);
    return hipGetLastError();
}
hipError_t group_launch_round(const GroupSeg *segs, int nsegs, const GroupTile *tiles, int ntiles,
                              const GroupInst *insts, const GroupDesc *desc, int32_t off, hipStream_t s) {
    hipLaunchKernelGGL(vec_group_combine_kernel, dim3(nsegs), dim3(VEC_TILE_MAX), 0, s, segs, insts, desc, off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(vec_group_patch_kernel<PATCH_LOOK>, dim3(ntiles), dim3(VEC_THREADS), 0, s, tiles, insts, desc, off);
    return hipGetLastError();
}
hipError_t group_set_desc(GroupDesc *desc, int64_t base_round, double dt, hipStream_t s) {
    hipLaunchKernelGGL(group_desc_kernel, dim3(1), dim3(1), 0, s, desc, base_round, dt);
    return hipGetLastError();
}

hipError_t vec_launch_start(const VecBuffers &b, int32_t parity, const double *c0, int32_t method,
                            hipStream_t s) {
    hipLaunchKernelGGL(vec_start_kernel, dim3(256), dim3(256), 0, s, b, parity,
                       reinterpret_cast<const double2 *>(c0), method == TDSE_TAYLOR ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tdse
