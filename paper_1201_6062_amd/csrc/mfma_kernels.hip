// Batched propagation (batch > 1 pulses sharing one Hamiltonian) on the FP64
// matrix cores of gfx950.
//
// With B pulses the state of partial wave l is a complex n x B matrix; stored
// as a real n x 2B matrix U_l (columns: pulse b real part, then imaginary
// part) the dipole product of Sec. 4 becomes two real GEMMs per block,
//   Z_m = D_m U_{m+1} + D_{m-1}^T U_{m-1},
// because the dipole is real (Sec. 5 stores it as real doubles). One
// workgroup owns an output tile of Z_m over the full contraction of both
// neighbour blocks, so no partial sums leave the workgroup, and the RK4 stage
// or Taylor term (appendix B) is completed in the epilogue with each pulse's
// own field sample. The plan keeps D and D^T, each row-major, so both
// products stream their left operand as k-major panels.
//
// v_mfma_f64_16x16x4f64 lane layout (wave64, measured on gfx950): A[i][k]
// comes from lane 16k + i, B[k][j] from lane 16k + j, and output register r
// of lane L holds row L/16 + 4r of column L % 16.
#include "tdse_internal.h"
#include "tdse_validate.h"

namespace tdse {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double dv2b_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void bat_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// partner lane (L ^ 1) through DPP quad_perm(1,0,3,2)
__device__ __forceinline__ double bat_xor1(double v) {
    long long x = __double_as_longlong(v);
    int lo = __builtin_amdgcn_mov_dpp((int)(x & 0xffffffffll), 0xB1, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0xB1, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Runge-Kutta-Fehlberg 4(5) tableau (stage times 0, 1/4, 3/8, 12/13, 1, 1/2):
// stage inputs u_{i+1} = c + dt sum_{q<=i} A[i+1][q] k_q, fifth-order
// weights B5 (the solution carried forward: the paper propagates the pair's
// fifth-order solution, Sec. 5.1) and E = B5 - B4 (the embedded error
// estimate, B4 the fourth-order weights).
__constant__ double RKF_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
__constant__ double RKF_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};
__constant__ double RKF_E[6] = {16.0 / 135.0 - 25.0 / 216.0, 0.0, 6656.0 / 12825.0 - 1408.0 / 2565.0,
                                28561.0 / 56430.0 - 2197.0 / 4104.0, -9.0 / 50.0 + 1.0 / 5.0, 2.0 / 55.0};

// Stride of one 1 KB group of a staged panel with rows of W doubles: 128 B
// of padding after each group (the four 16-lane row groups of a fragment
// read then fall into two LDS bank sets); with a three-deep ring, 64 B after
// each group of a 128-wide panel (one row per group: its rows then fall
// into four bank sets, just as evenly spread), so that two workgroups' rings
// fit one CU's LDS.
template <int W, int DEPTH>
__host__ __device__ constexpr int panel_group() { return 1024 + (DEPTH == 3 && W == 128 ? 64 : 128); }

template <int TM, int TN, int KC, int DEPTH = 2>
struct BatTile {
    static constexpr int THREADS = 256;
    static constexpr int WM = TM / 2, WN = TN / 2;       // 2 x 2 waves
    static constexpr int SM = WM / 16, SN = WN / 16;     // 16 x 16 subtiles per wave
    // The K panels go from global memory straight into LDS (global_load_lds):
    // one instruction moves 64 lanes x 16 B = 1 KB, i.e. 128 / TM rows of the
    // A panel (128 / TN rows of B), each such group followed by padding.
    static constexpr int A_RPI = 128 / TM, B_RPI = 128 / TN;
    static constexpr int GROUP_A = panel_group<TM, DEPTH>(), GROUP_B = panel_group<TN, DEPTH>();
    static constexpr int A_GROUPS = KC / A_RPI, B_GROUPS = KC / B_RPI;
    static constexpr int A_PER_W = A_GROUPS / 4, B_PER_W = B_GROUPS / 4;  // instructions per wave
    static constexpr int A_BYTES = A_GROUPS * GROUP_A, B_BYTES = B_GROUPS * GROUP_B;
};

typedef __attribute__((address_space(3))) void lds_void_t;

// byte offset of element (k, x) of a staged panel with rows of W doubles
template <int W, int DEPTH = 2>
__device__ __forceinline__ int panel_off(int k, int x) {
    constexpr int RPI = 128 / W;
    return (k / RPI) * panel_group<W, DEPTH>() + ((k % RPI) * W + x) * 8;
}

// One K chunk of a workgroup: start the direct-to-LDS loads of the next
// chunk into (wa, wb) when wa is non-null -- wave wv moves row groups
// wv, wv+4, ... of both panels -- then run the chunk's MFMAs from (la, lb)
// when la is non-null. The restrict qualifiers tell the compiler that the
// panels being read and the ones being filled do not overlap, so it does
// not wait for the new loads before reading the current panels.
template <int TM, int TN, int KC, bool PIN = false, int DEPTH = 2>
__device__ __forceinline__ void bat_chunk(const char *__restrict__ la, const char *__restrict__ lb,
                                          char *__restrict__ wa, char *__restrict__ wb,
                                          const double *__restrict__ pa, const double *__restrict__ pb,
                                          int Np, int ldu, int lane, int wv,
                                          d4_t (&acc)[BatTile<TM, TN, KC>::SM][BatTile<TM, TN, KC>::SN]) {
    using C = BatTile<TM, TN, KC, DEPTH>;
    if (DEPTH == 3 && wa) {
        // Buffer loads with the LDS bit: the compiler does not track these
        // against LDS reads (it would wait for every panel in flight before
        // reading the current one, the previous chunk's loads included);
        // the kernel's explicit waits order them.
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(pa), 0, 0x7fffffff, 0x00020000);
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(pb), 0, 0x7fffffff, 0x00020000);
#pragma unroll
        for (int q = 0; q < C::A_PER_W; ++q) {
            const int g = wv + 4 * q, k = g * C::A_RPI + lane / (TM / 2), x = 2 * (lane % (TM / 2));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_t *)(wa + g * C::GROUP_A), 16, (k * Np + x) * 8, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < C::B_PER_W; ++q) {
            const int g = wv + 4 * q, k = g * C::B_RPI + lane / (TN / 2), x = 2 * (lane % (TN / 2));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void_t *)(wb + g * C::GROUP_B), 16, (k * ldu + x) * 8, 0, 0, 0);
        }
    } else if (wa) {
#pragma unroll
        for (int q = 0; q < C::A_PER_W; ++q) {
            const int g = wv + 4 * q, k = g * C::A_RPI + lane / (TM / 2), x = 2 * (lane % (TM / 2));
            __builtin_amdgcn_global_load_lds((const void *)(pa + (size_t)k * Np + x),
                                             (lds_void_t *)(wa + g * C::GROUP_A), 16, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < C::B_PER_W; ++q) {
            const int g = wv + 4 * q, k = g * C::B_RPI + lane / (TN / 2), x = 2 * (lane % (TN / 2));
            __builtin_amdgcn_global_load_lds((const void *)(pb + (size_t)k * ldu + x),
                                             (lds_void_t *)(wb + g * C::GROUP_B), 16, 0, 0);
        }
    }
    if (!la) return;
    const int wy = wv >> 1, wx = wv & 1;
    if constexpr (!PIN) {
        // fragments of k-step ks+1 are read while the products of ks run
        double af[2][C::SM], bf[2][C::SN];
        auto frag = [&](int ks, int slot) {
            const int kr = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
                af[slot][i] =
                    *reinterpret_cast<const double *>(la + panel_off<TM, DEPTH>(kr, wy * C::WM + i * 16 + (lane & 15)));
#pragma unroll
            for (int j = 0; j < C::SN; ++j)
                bf[slot][j] =
                    *reinterpret_cast<const double *>(lb + panel_off<TN, DEPTH>(kr, wx * C::WN + j * 16 + (lane & 15)));
        };
        frag(0, 0);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            if (ks + 1 < KC / 4) frag(ks + 1, (ks + 1) & 1);
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
#pragma unroll
                for (int j = 0; j < C::SN; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks & 1][i], bf[ks & 1][j], acc[i][j], 0, 0, 0);
        }
    } else {
        // PIN (kernels with two K groups, the skinny grids of few pulses):
        // the fragments of k-step ks+2 are read while the products of ks run,
        // from a ring of three sets, and a scheduling barrier keeps the reads
        // ahead of the products (the scheduler would otherwise sink them
        // behind the products and wait for them at once). At 256 pulses the
        // one-group kernels keep the compiler's schedule: the barrier cost
        // 1.6% there.
        constexpr int D = 2, NSLOT = 3;
        double af[NSLOT][C::SM], bf[NSLOT][C::SN];
        auto frag = [&](int ks, int slot) {
            const int kr = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
                af[slot][i] =
                    *reinterpret_cast<const double *>(la + panel_off<TM, DEPTH>(kr, wy * C::WM + i * 16 + (lane & 15)));
#pragma unroll
            for (int j = 0; j < C::SN; ++j)
                bf[slot][j] =
                    *reinterpret_cast<const double *>(lb + panel_off<TN, DEPTH>(kr, wx * C::WN + j * 16 + (lane & 15)));
        };
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (d < KC / 4) frag(d, d);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            if (ks + D < KC / 4) frag(ks + D, (ks + D) % NSLOT);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
#pragma unroll
                for (int j = 0; j < C::SN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks % NSLOT][i], bf[ks % NSLOT][j], acc[i][j],
                                                                     0, 0, 0);
        }
    }
}

// ADJ = false: forward RK4 / Taylor stage (or a single product).
// ADJ = true: one stage of the discrete adjoint of an RK4 step, run in
// reverse: the product input is the co-state kbar of the stage derivative,
// ubar = i H(F) kbar (since (-iH)^H = iH for real symmetric H), the co-state
// of c accumulates sum ubar, and the field gradient Im((D kbar)^H u) is
// reduced per row tile (u = the forward input of the stage).
// KS = 2: the workgroup holds two groups of four waves, one per neighbour
// block (the row use of D_m and the transposed use of D_{m-1}), each with its
// own panels; the second group's accumulators are added to the first's in
// LDS before the epilogue. For grids of few tiles (few pulses): twice the
// waves per CU.
// DEPTH: panels in flight. 2: the next chunk's panels load while this
// chunk's products run, and every chunk ends waiting for all of them. 3: the
// panels of the chunk after next are issued at the start of each chunk, and
// a chunk waits only for its own (one chunk's loads stay in flight across
// the barrier).
template <int TM, int TN, int KC, bool ADJ, int KS, int DEPTH = 2>
__global__ __launch_bounds__(256 * KS) __attribute__((amdgpu_waves_per_eu(1, 2))) void bat_stage_kernel(BatBuffers b, BatLaunch L) {
    using C = BatTile<TM, TN, KC, DEPTH>;
    static_assert(DEPTH == 2 || (DEPTH == 3 && KS == 1), "three-deep rings for one K group");
    static_assert(C::A_PER_W >= 1 && C::B_PER_W >= 1 && C::A_GROUPS % 4 == 0 && C::B_GROUPS % 4 == 0,
                  "panel groups must split evenly over the 4 waves");
    const int Np = b.np, ldu = b.ldu, lmax = b.lmax;
    const int RT = Np / TM, CT = ldu / TN;
    const int ntiles = (lmax + 1) * RT * CT;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);
    const int m = tile / (RT * CT), rem = tile - m * RT * CT, rt = rem / CT, ct = rem - rt * CT;
    const int r0 = rt * TM, c0 = ct * TN;

    __shared__ __attribute__((aligned(16))) char lds_a[KS][DEPTH][C::A_BYTES];
    __shared__ __attribute__((aligned(16))) char lds_b[KS][DEPTH][C::B_BYTES];

    const int t = threadIdx.x % 256, lane = t & 63, wv = t >> 6;
    const int kg = KS == 2 ? (int)(threadIdx.x >> 8) : 0;  // K group of this wave
    const int wy = wv >> 1, wx = wv & 1;
    const int par = L.parity;
    const double *U = par ? b.u[1] : b.u[0];

    // K chunks: first the row use of D_m against U_{m+1}, then the transposed
    // use of D_{m-1} against U_{m-1}.
    const int kchunks = Np / KC;
    const bool has_up = m < lmax, has_dn = m > 0;
    const int nchunks = kchunks * ((has_up ? 1 : 0) + (has_dn ? 1 : 0));
    const size_t blk = (size_t)Np * Np;

    // Panel sources of chunk kc.
    auto a_src = [&](int kc) -> const double * {
        const bool up = has_up && kc < kchunks;
        const int k0 = (up ? kc : kc - (has_up ? kchunks : 0)) * KC;
        return up ? b.dT + (size_t)m * blk + (size_t)k0 * Np + r0
                  : b.d + (size_t)(m - 1) * blk + (size_t)k0 * Np + r0;
    };
    auto b_src = [&](int kc) -> const double * {
        const bool up = has_up && kc < kchunks;
        const int k0 = (up ? kc : kc - (has_up ? kchunks : 0)) * KC;
        return U + ((size_t)(up ? m + 1 : m - 1) * Np + k0) * ldu + c0;
    };

    d4_t acc[C::SM][C::SN];
#pragma unroll
    for (int i = 0; i < C::SM; ++i)
#pragma unroll
        for (int j = 0; j < C::SN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    // Chunks [kbeg, kbeg + kcnt) of this wave's K group. With two groups a
    // tile with both neighbours gives each group one; a tile with one gives
    // it to group 0. Both groups pass the same niter barriers.
    const bool both = has_up && has_dn;
    const int kbeg = KS == 2 && both ? kg * kchunks : 0;
    const int kcnt = KS == 1 ? nchunks : (both ? kchunks : (kg == 0 ? nchunks : 0));
    const int niter = KS == 1 ? nchunks : (nchunks > 0 ? kchunks : 0);
    char(*la)[C::A_BYTES] = lds_a[kg];
    char(*lb)[C::B_BYTES] = lds_b[kg];
    if constexpr (DEPTH == 3) {
        // chunks 0 and 1 in flight; chunk q waits for its own panels only
        constexpr int LPW = C::A_PER_W + C::B_PER_W;  // loads per wave and chunk
#pragma unroll
        for (int d = 0; d < 2; ++d)
            if (d < kcnt)
                bat_chunk<TM, TN, KC, false, 3>(nullptr, nullptr, la[d], lb[d], a_src(kbeg + d), b_src(kbeg + d), Np,
                                                ldu, lane, wv, acc);
        for (int q = 0; q < kcnt; ++q) {
            if (q + 1 < kcnt) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(LPW) : "memory");
            else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            // every wave's part of chunk q has landed, and every wave is done
            // with chunk q - 1, whose buffer the loads below refill
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
            const int nb = (q + 2) % 3;
            const bool next = q + 2 < kcnt;
            bat_chunk<TM, TN, KC, false, 3>(la[q % 3], lb[q % 3], next ? la[nb] : nullptr, next ? lb[nb] : nullptr,
                                            next ? a_src(kbeg + q + 2) : nullptr, next ? b_src(kbeg + q + 2) : nullptr,
                                            Np, ldu, lane, wv, acc);
        }
    } else if (niter > 0) {
        if (kcnt > 0)
            bat_chunk<TM, TN, KC, KS == 2>(nullptr, nullptr, la[0], lb[0], a_src(kbeg), b_src(kbeg), Np, ldu, lane, wv, acc);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        bat_lds_barrier();
        for (int q = 0; q < niter; ++q) {
            if (q < kcnt) {
                const int buf = q & 1;
                const bool next = q + 1 < kcnt;
                bat_chunk<TM, TN, KC, KS == 2>(la[buf], lb[buf], next ? la[buf ^ 1] : nullptr, next ? lb[buf ^ 1] : nullptr,
                                      next ? a_src(kbeg + q + 1) : nullptr, next ? b_src(kbeg + q + 1) : nullptr, Np,
                                      ldu, lane, wv, acc);
            }
            // the next chunk's panels have landed and every wave is done with this one
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            bat_lds_barrier();
        }
    }
    if constexpr (KS == 2) {
        // group 1's accumulators onto group 0's (one addition per element)
        __shared__ double kred[TM * TN];
        if (kg == 1) {
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
#pragma unroll
                for (int j = 0; j < C::SN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) kred[(((wv * C::SM + i) * C::SN + j) * 4 + r) * 64 + lane] = acc[i][j][r];
        }
        bat_lds_barrier();
        if (kg == 0) {
#pragma unroll
            for (int i = 0; i < C::SM; ++i)
#pragma unroll
                for (int j = 0; j < C::SN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += kred[(((wv * C::SM + i) * C::SN + j) * 4 + r) * 64 + lane];
        }
    }

    // ---- epilogue. It runs one row subtile i at a time: first every load of
    // that subtile's SN x 4 entries (state, stage input, energies, stored
    // stage derivatives), then the arithmetic and the stores. Loads placed
    // after the previous entry's stores would each wait for their own round
    // trip (the compiler cannot move a load above a store it cannot prove
    // disjoint), one latency per entry instead of one per subtile.
    const int B = b.batch;
    const int64_t step = L.step;
    const double dt = L.dt;
    double *Un = par ? b.u[0] : b.u[1];
    double gsum[C::SN];
    double Fj[C::SN];
#pragma unroll
    for (int j = 0; j < C::SN; ++j) {
        gsum[j] = 0.0;
        const int col = c0 + wx * C::WN + j * 16 + (lane & 15);
        Fj[j] = (col >> 1) < B ? b.field[((size_t)(col >> 1) * L.nsteps + step) * L.slots + L.slot] : 0.0;
    }
    const bool rkf = L.kind == CK_RKF;
    const int st = L.slot;
    const size_t kstride = (size_t)(lmax + 1) * Np * ldu;
    // (with two K groups, group 0 completes the stage; group 1 only passes
    // the barriers below)
#pragma unroll
    for (int i = 0; i < (kg == 0 ? C::SM : 0); ++i) {
#pragma unroll
        for (int j = 0; j < C::SN; ++j) {
            // the loads of this (i, j) group's four entries, then their arithmetic
            size_t gi[4];
            double uo[4], cv[4], av[4], us[4], E0[4], kq[4][5];
            const int colg = c0 + wx * C::WN + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wy * C::WM + i * 16 + (lane >> 4) + 4 * r;
                E0[r] = b.en[(size_t)m * Np + row];
                gi[r] = ((size_t)m * Np + row) * ldu + colg;
                uo[r] = U[gi[r]];
                cv[r] = b.c[gi[r]];
                av[r] = b.acc[gi[r]];
                us[r] = ADJ ? L.ustore[gi[r]] : 0.0;
            }
            if (!ADJ && rkf) {
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    if (q < st) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) kq[r][q] = b.kst[(size_t)q * kstride + gi[r]];
                    }
            }
            const bool is_im = colg & 1;
            const int pulse = colg >> 1;
            const double F = Fj[j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wy * C::WM + i * 16 + (lane >> 4) + 4 * r;
                const size_t g = gi[r];
                // coupling product of this column (z) and of its real/imaginary
                // partner (zp); velocity gauge: -i times the contraction
                const double zc = acc[i][j][r], zcp = bat_xor1(zc);
                const double z = b.gauge ? (is_im ? -zcp : zcp) : zc;
                const double zp = b.gauge ? (is_im ? zc : -zc) : zcp;
                const double u0 = uo[r], up = bat_xor1(u0);
                if constexpr (ADJ) {
                    // ubar = i (E0 kbar + F w): re = -(E0 kbar_im + F w_im), im = E0 kbar_re + F w_re
                    const double ub = (is_im ? 1.0 : -1.0) * fma(F, zp, E0[r] * up);
                    const double usp = bat_xor1(us[r]);
                    // Im(w^H u) = sum (w_re u_im - w_im u_re)
                    gsum[j] += (is_im ? -z : z) * usp;
                    const double lam = cv[r];
                    const double cb = (L.first ? lam : av[r]) + ub;
                    if (L.kind == CK_ADJ_MID) {
                        b.acc[g] = cb;
                        Un[g] = fma(L.p_lam, lam, L.p_ub * ub);
                    } else {  // CK_ADJ_LAST: cb is the co-state of c at the step's start
                        b.c[g] = cb;
                        Un[g] = L.p_lam * cb;
                    }
                } else {
                    // own component of y = E0 u + F z and of k = -i y:
                    // k_re = y_im, k_im = -y_re
                    const double yre = is_im ? fma(F, zp, E0[r] * up) : fma(F, z, E0[r] * u0);
                    const double yim = is_im ? fma(F, z, E0[r] * u0) : fma(F, zp, E0[r] * up);
                    const double k = is_im ? -yre : yim;
                    if (L.kind == CK_HMUL) {  // single product y = H u (tdse_hmul; Krylov products)
                        if (pulse < B && row < b.n)
                            L.out[(size_t)pulse * 2 * (lmax + 1) * b.n + 2 * ((size_t)m * b.n + row) +
                                  (is_im ? 1 : 0)] = is_im ? yim : yre;
                        gsum[j] = fma(u0, is_im ? yim : yre, gsum[j]);  // this column's part of Re <u, y>
                        continue;
                    }
                    if (L.ustore) L.ustore[g] = u0;  // forward recompute for the adjoint
                    double c = cv[r];
                    double a = av[r];
                    double unext;
                    switch (L.kind) {
                    case CK_RK4_MID:
                        a = L.first ? L.w_acc * k : fma(L.w_acc, k, a);
                        unext = fma(L.a_next * dt, k, c);
                        b.acc[g] = a;
                        break;
                    case CK_RK4_END:
                        c = fma(dt, fma(L.w_acc, k, a), c);
                        unext = c;
                        b.c[g] = c;
                        break;
                    case CK_TAY_MID: {
                        const double tm = L.a_next * dt * k;
                        a = (L.first ? c : a) + tm;
                        unext = tm;
                        b.acc[g] = a;
                        break;
                    }
                    case CK_RKF: {
                        // stage st: keep k_st, then the next stage input, or after
                        // the sixth stage the fifth-order step and its error estimate
                        double sacc = 0.0, serr = 0.0;
#pragma unroll
                        for (int q = 0; q < 5; ++q)
                            if (q < st) {
                                sacc = fma(st < 5 ? RKF_A[st + 1][q] : RKF_B5[q], kq[r][q], sacc);
                                serr = fma(RKF_E[q], kq[r][q], serr);
                            }
                        if (st < 5) {
                            b.kst[(size_t)st * kstride + g] = k;
                            unext = fma(dt, fma(RKF_A[st + 1][st], k, sacc), c);
                        } else {
                            c = fma(dt, fma(RKF_B5[5], k, sacc), c);
                            const double e = dt * fma(RKF_E[5], k, serr);
                            gsum[j] = fma(e, e, gsum[j]);
                            unext = c;
                            b.c[g] = c;
                        }
                        break;
                    }
                    default: {  // CK_TAY_END
                        const double tm = L.a_next * dt * k;
                        c = (L.first ? c : a) + tm;
                        unext = c;
                        b.c[g] = c;
                        break;
                    }
                    }
                    Un[g] = unext;
                    const bool ends = L.kind == CK_RK4_END || L.kind == CK_TAY_END || (L.kind == CK_RKF && L.slot == 5);
                    if (L.ckpt && ends && pulse < B && row < b.n) {
                        // caller layout [B][rows][2 n]
                        L.ckpt[((size_t)pulse * L.ckpt_rows + L.ckpt_row) * 2 * (size_t)(lmax + 1) * b.n +
                               2 * ((size_t)m * b.n + row) + (is_im ? 1 : 0)] = c;
                    }
                }
            }
        }
    }
    if (ADJ || (((L.kind == CK_RKF && L.slot == 5) || L.kind == CK_HMUL) && L.gpart != nullptr)) {
        // Per-pulse partial of this row tile (adjoint: the field gradient;
        // Runge-Kutta-Fehlberg: the squared error estimate; single product:
        // Re <u, H u>, the Krylov recurrence's alpha): rows of one lane
        // (i, r), then the four 16-lane row groups, then the real/imaginary
        // column pair, then the two row halves of the tile.
        __shared__ double gred[2][TN];
#pragma unroll
        for (int j = 0; j < C::SN; ++j) {
            double g = gsum[j];
            g += __shfl_xor(g, 16);
            g += __shfl_xor(g, 32);
            g += bat_xor1(g);
            if (lane < 16 && kg == 0) gred[wy][wx * C::WN + j * 16 + lane] = g;
        }
        bat_lds_barrier();
        if (t < TN / 2 && kg == 0) {
            const int pulse = c0 / 2 + t;
            if (pulse < B) L.gpart[(size_t)(m * RT + rt) * B + pulse] = gred[0][2 * t] + gred[1][2 * t];
        }
    }
}

// ---------------------------------------------------------------------------
// Small batches (2B <= 64 real columns): one workgroup of eight waves per
// 32-row tile and all columns, the contraction (both neighbour blocks, K =
// 2 Np) split into eight contiguous k ranges, one per wave. A wave streams its
// operands from global memory straight into registers -- no LDS staging and no
// barrier inside the k loop -- keeping DEPTH k-steps of loads in flight, and
// runs 4 NG MFMAs per k-step on them. Every operand is k-major (D^T rows for
// the row use of D_m, D rows for the transposed use of D_{m-1}, U rows), so
// one 16-byte load per lane covers four k rows of 32 consecutive entries:
// lane 16q + i takes entries 2i, 2i + 1 of row k0 + q. For A that is two
// 16-row MFMA operands (the even and the odd rows of the tile); for U the
// real and the imaginary column of 16 pulses. The eight partial tiles are
// summed in LDS in wave order (a fixed order: bitwise reproducible) and the
// epilogue -- the same completions as the kernel above, on complex entries --
// is spread over all 512 threads, each owning whole (row, pulse) entries.
template <int NG>
struct SkinnyTile {
    static constexpr int TM = 32, TN = 32 * NG, WAVES = 8;
    static constexpr int NACC = 2 * NG * 2;          // (row parity, column group, re/im)
    static constexpr int SLOTS = NACC * 4;           // doubles of accumulator per lane
};

// The words the first loads need (both dipole copies, the stage input read,
// Np, ldu and lmax: 9 dwords) come as leading scalar arguments, which are
// preloaded into scalar registers before the wave starts (built with
// -amdgpu-kernarg-preload-count), so the k loop's first loads do not wait for
// a kernel-argument fetch.
template <int NG, bool ADJ, int DEPTH, int CHUNK>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void bat_skinny_kernel(
    const double *dp, const double *dTp, const double *U, int32_t Np, int32_t ldu, int32_t lmax, BatBuffers bk,
    BatLaunch L) {
    static_assert(CHUNK % DEPTH == 0, "a chunk holds whole rounds of the load ring");
    using S = SkinnyTile<NG>;
    BatBuffers b = bk;
    b.d = const_cast<double *>(dp);
    b.dT = const_cast<double *>(dTp);
    b.np = Np;
    b.ldu = ldu;
    b.lmax = lmax;
    const int RT = Np / S::TM, CT = ldu / S::TN;
    const int ntiles = (lmax + 1) * RT * CT;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);
    const int m = tile / (RT * CT), rem = tile - m * RT * CT, rt = rem / CT, ct = rem - rt * CT;
    const int r0 = rt * S::TM, c0 = ct * S::TN;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: buffer descriptors stay scalar
    const int q = lane >> 4, li = lane & 15;  // U: the stage input read (b.u[L.parity])

    // ---- this wave's k range: with both neighbour blocks, waves 0-3 split the
    // row use of D_m and waves 4-7 the transposed use of D_{m-1}; with one,
    // all eight split it.
    const bool has_up = m < lmax, has_dn = m > 0;
    const int nks = Np / 4;
    const bool up = (has_up && has_dn) ? wv < 4 : has_up;
    const int nparts = (has_up && has_dn) ? 4 : 8, part = (has_up && has_dn) ? (wv & 3) : wv;
    // k-steps [ks0, ks0 + len) of the block, by the balanced split of Sec. 4.1
    const int len = (has_up || has_dn) ? (int)split_len(nks, nparts, part) : 0;
    const int ks0 = (has_up || has_dn) ? (int)split_start(nks, nparts, part) : 0;
    const size_t blk = (size_t)Np * Np;
    const double *A = up ? b.dT + (size_t)(has_up ? m : 0) * blk : b.d + (size_t)(has_dn ? m - 1 : 0) * blk;
    const double *Bm = U + (size_t)(up ? (has_up ? m + 1 : 0) : (has_dn ? m - 1 : 0)) * Np * ldu;
    // Raw buffer loads: the descriptor of k-step ks starts at that step's
    // first row and covers the rows left in this wave's range, so a load past
    // the range (the look-ahead of the last k-steps) returns zeros without
    // touching memory; every load is issued either way and the wait counts
    // stay exact. Base and size are scalar, the lane offset is one register.
    const double *A0 = A + (size_t)4 * ks0 * Np, *B0 = Bm + (size_t)4 * ks0 * ldu;
    const int oa = (q * Np + r0 + 2 * li) * 8, ob = (q * ldu + c0 + 2 * li) * 8;  // lane byte offsets
    auto rsrc = [&](const double *base, int ks, int ld) {
        const int left = len - ks;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base) + (size_t)ks * 4 * ld, 0,
                                                 left > 0 ? left * 4 * ld * 8 : 0, 0x00020000);
    };

    d4_t acc[2][NG][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int g = 0; g < NG; ++g) acc[p][g][0] = acc[p][g][1] = d4_t{0.0, 0.0, 0.0, 0.0};

    if (len > 0) {
        dv2b_t ra[DEPTH], rb[DEPTH][NG];
        auto load = [&](int slot, int ks) {
            ra[slot] = __builtin_bit_cast(dv2b_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc(A0, ks, Np), oa, 0, 0));
            const __amdgpu_buffer_rsrc_t rb_s = rsrc(B0, ks, ldu);
#pragma unroll
            for (int g = 0; g < NG; ++g)
                rb[slot][g] = __builtin_bit_cast(dv2b_t, __builtin_amdgcn_raw_buffer_load_b128(rb_s, ob + 256 * g, 0, 0));
        };
        auto mfmas = [&](int slot) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int g = 0; g < NG; ++g)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[p][g][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[slot][p], rb[slot][g][c], acc[p][g][c],
                                                                            0, 0, 0);
        };
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) load(d, d);
        // CHUNK k-steps fully unrolled per trip (the launcher picks CHUNK >=
        // the longest k range, so a wave normally makes one trip: at a loop
        // back edge the compiler waits for every load in flight). A range
        // shorter than the chunk ends with products of the zeros that the
        // loads past it returned.
        for (int ks = 0; ks < len; ks += CHUNK) {
#pragma unroll
            for (int d = 0; d < CHUNK; ++d) {
                mfmas(d % DEPTH);
                load(d % DEPTH, ks + DEPTH + d);
                // keep each slot's reload right behind its products (the
                // scheduler would otherwise gather the reloads at the end)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // ---- epilogue operands of this thread's entries, requested before the
    // reduction so their latency overlaps it. Thread (v, lane) owns the
    // accumulator slots P = NPER v .. NPER v + NPER - 1 of every wave, P =
    // ((g 2 + p) 4 + r): rows r0 + 2 (q + 4 r) + p, pulse c0/2 + 16 g + li.
    constexpr int NPER = 2 * NG * 4 / 8;  // (g, p, r) slots per thread: 2 (NG = 2) or 1
    const int B = b.batch;
    double *Un = L.parity ? b.u[0] : b.u[1];
    size_t gi[NPER];
    int row[NPER], pulse[NPER];
    dv2b_t uo[NPER], cc[NPER], aa[NPER], us[NPER];
    double E0[NPER], F[NPER];
#pragma unroll
    for (int e = 0; e < NPER; ++e) {
        const int P = NPER * wv + e, g = P >> 3, p = (P >> 2) & 1, r = P & 3;
        row[e] = r0 + 2 * (q + 4 * r) + p;
        pulse[e] = c0 / 2 + 16 * g + li;
        gi[e] = ((size_t)m * Np + row[e]) * ldu + 2 * pulse[e];
        uo[e] = *reinterpret_cast<const dv2b_t *>(U + gi[e]);
        cc[e] = *reinterpret_cast<const dv2b_t *>(b.c + gi[e]);
        aa[e] = (ADJ || !L.first || L.kind == CK_RK4_END || L.kind == CK_RKF) ? *reinterpret_cast<const dv2b_t *>(b.acc + gi[e])
                                                                              : dv2b_t{0.0, 0.0};
        us[e] = (ADJ && L.ustore) ? *reinterpret_cast<const dv2b_t *>(L.ustore + gi[e]) : dv2b_t{0.0, 0.0};
        E0[e] = b.en[(size_t)m * Np + row[e]];
        F[e] = pulse[e] < B ? b.field[((size_t)pulse[e] * L.nsteps + L.step) * L.slots + L.slot] : 0.0;
    }

    // ---- fixed-order sum of the eight partial tiles
    __shared__ double red[S::WAVES][S::SLOTS][64];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[wv][((((g * 2 + p) * 4 + r) * 2) + c)][lane] = acc[p][g][c][r];
    bat_lds_barrier();
    const double dt = L.dt;
    double gsum = 0.0;  // this thread's part of the pulse's tile partial (adjoint, RKF error)
#pragma unroll
    for (int e = 0; e < NPER; ++e) {
        const int P = NPER * wv + e;
        double cr = 0.0, ci = 0.0;
#pragma unroll
        for (int k = 0; k < S::WAVES; ++k) {
            cr += red[k][2 * P][lane];
            ci += red[k][2 * P + 1][lane];
        }
        // coupling product z of this entry; velocity gauge: -i times the contraction
        const double zr = b.gauge ? ci : cr, zi = b.gauge ? -cr : ci;
        const double ur = uo[e][0], ui = uo[e][1];
        const bool live = pulse[e] < B && row[e] < b.n;
        if constexpr (ADJ) {
            // ubar = i (E0 kbar + F w); gradient part Im(w^H u) = w_re u_im - w_im u_re
            const double ubr = -fma(F[e], zi, E0[e] * ui), ubi = fma(F[e], zr, E0[e] * ur);
            gsum = fma(zr, us[e][1], gsum);
            gsum = fma(-zi, us[e][0], gsum);
            const double lr = cc[e][0], lim = cc[e][1];
            const double cbr = (L.first ? lr : aa[e][0]) + ubr, cbi = (L.first ? lim : aa[e][1]) + ubi;
            if (L.kind == CK_ADJ_MID) {
                *reinterpret_cast<dv2b_t *>(b.acc + gi[e]) = dv2b_t{cbr, cbi};
                *reinterpret_cast<dv2b_t *>(Un + gi[e]) =
                    dv2b_t{fma(L.p_lam, lr, L.p_ub * ubr), fma(L.p_lam, lim, L.p_ub * ubi)};
            } else {
                *reinterpret_cast<dv2b_t *>(b.c + gi[e]) = dv2b_t{cbr, cbi};
                *reinterpret_cast<dv2b_t *>(Un + gi[e]) = dv2b_t{L.p_lam * cbr, L.p_lam * cbi};
            }
        } else {
            // y = E0 u + F z, k = -i y
            const double yr = fma(F[e], zr, E0[e] * ur), yi = fma(F[e], zi, E0[e] * ui);
            const double kr = yi, ki = -yr;
            if (L.kind == CK_HMUL) {
                if (live)
                    *reinterpret_cast<dv2b_t *>(L.out + (size_t)pulse[e] * 2 * (lmax + 1) * b.n +
                                                2 * ((size_t)m * b.n + row[e])) = dv2b_t{yr, yi};
                gsum = fma(ur, yr, gsum);  // this entry's part of Re <u, y>
                gsum = fma(ui, yi, gsum);
                continue;
            }
            if (L.ustore) *reinterpret_cast<dv2b_t *>(L.ustore + gi[e]) = uo[e];
            double c_r = cc[e][0], c_i = cc[e][1], a_r = aa[e][0], a_i = aa[e][1], n_r, n_i;
            switch (L.kind) {
            case CK_RK4_MID: {
                a_r = L.first ? L.w_acc * kr : fma(L.w_acc, kr, a_r);
                a_i = L.first ? L.w_acc * ki : fma(L.w_acc, ki, a_i);
                const double ad = L.a_next * dt;
                n_r = fma(ad, kr, c_r);
                n_i = fma(ad, ki, c_i);
                *reinterpret_cast<dv2b_t *>(b.acc + gi[e]) = dv2b_t{a_r, a_i};
                break;
            }
            case CK_RK4_END:
                c_r = fma(dt, fma(L.w_acc, kr, a_r), c_r);
                c_i = fma(dt, fma(L.w_acc, ki, a_i), c_i);
                n_r = c_r;
                n_i = c_i;
                *reinterpret_cast<dv2b_t *>(b.c + gi[e]) = dv2b_t{c_r, c_i};
                break;
            case CK_TAY_MID: {
                const double tr = L.a_next * dt * kr, ti = L.a_next * dt * ki;
                a_r = (L.first ? c_r : a_r) + tr;
                a_i = (L.first ? c_i : a_i) + ti;
                n_r = tr;
                n_i = ti;
                *reinterpret_cast<dv2b_t *>(b.acc + gi[e]) = dv2b_t{a_r, a_i};
                break;
            }
            case CK_RKF: {
                const int st = L.slot;
                const size_t kstride = (size_t)(lmax + 1) * Np * ldu;
                double sr = 0.0, si = 0.0, er = 0.0, ei = 0.0;
                // the stored stage derivatives, all requested before the first is used
                dv2b_t kq[5];
#pragma unroll
                for (int qq = 0; qq < 5; ++qq)
                    if (qq < st) kq[qq] = *reinterpret_cast<const dv2b_t *>(b.kst + (size_t)qq * kstride + gi[e]);
#pragma unroll
                for (int qq = 0; qq < 5; ++qq)
                    if (qq < st) {
                        const double wgt = st < 5 ? RKF_A[st + 1][qq] : RKF_B5[qq];
                        sr = fma(wgt, kq[qq][0], sr);
                        si = fma(wgt, kq[qq][1], si);
                        er = fma(RKF_E[qq], kq[qq][0], er);
                        ei = fma(RKF_E[qq], kq[qq][1], ei);
                    }
                if (st < 5) {
                    *reinterpret_cast<dv2b_t *>(b.kst + (size_t)st * kstride + gi[e]) = dv2b_t{kr, ki};
                    n_r = fma(dt, fma(RKF_A[st + 1][st], kr, sr), c_r);
                    n_i = fma(dt, fma(RKF_A[st + 1][st], ki, si), c_i);
                } else {
                    c_r = fma(dt, fma(RKF_B5[5], kr, sr), c_r);
                    c_i = fma(dt, fma(RKF_B5[5], ki, si), c_i);
                    const double xr = dt * fma(RKF_E[5], kr, er), xi = dt * fma(RKF_E[5], ki, ei);
                    gsum = fma(xr, xr, gsum);
                    gsum = fma(xi, xi, gsum);
                    n_r = c_r;
                    n_i = c_i;
                    *reinterpret_cast<dv2b_t *>(b.c + gi[e]) = dv2b_t{c_r, c_i};
                }
                break;
            }
            default: {  // CK_TAY_END
                const double tr = L.a_next * dt * kr, ti = L.a_next * dt * ki;
                c_r = (L.first ? c_r : a_r) + tr;
                c_i = (L.first ? c_i : a_i) + ti;
                n_r = c_r;
                n_i = c_i;
                *reinterpret_cast<dv2b_t *>(b.c + gi[e]) = dv2b_t{c_r, c_i};
                break;
            }
            }
            *reinterpret_cast<dv2b_t *>(Un + gi[e]) = dv2b_t{n_r, n_i};
            const bool ends = L.kind == CK_RK4_END || L.kind == CK_TAY_END || (L.kind == CK_RKF && L.slot == 5);
            if (L.ckpt && ends && live)
                *reinterpret_cast<dv2b_t *>(L.ckpt + ((size_t)pulse[e] * L.ckpt_rows + L.ckpt_row) * 2 *
                                                         (size_t)(lmax + 1) * b.n +
                                            2 * ((size_t)m * b.n + row[e])) = dv2b_t{c_r, c_i};
        }
    }
    if (ADJ || (((L.kind == CK_RKF && L.slot == 5) || L.kind == CK_HMUL) && L.gpart != nullptr)) {
        // per-pulse sum over the tile's 32 rows: the thread's own entries, the
        // four row groups q of the wave, then (in LDS, in wave order) the waves
        // holding the same column group
        gsum += __shfl_xor(gsum, 16);
        gsum += __shfl_xor(gsum, 32);
        __shared__ double gred[S::WAVES][16];
        if (lane < 16) gred[wv][lane] = gsum;
        bat_lds_barrier();
        constexpr int WPG = S::WAVES / NG;  // waves per column group
        if (t < S::TN / 2) {
            const int g = t >> 4, j = t & 15, pl = c0 / 2 + t;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < WPG; ++k) s += gred[g * WPG + k][j];
            if (pl < B) L.gpart[(size_t)(m * RT + rt) * B + pl] = s;
        }
    }
}

// caller layout [B][2 n] <-> internal [lmax+1][Np][ldu]
__global__ void bat_pack_kernel(BatBuffers b, const double *c0, int taylor_acc) {
    const size_t total = (size_t)(b.lmax + 1) * b.np * b.ldu;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)(g % b.ldu);
        const size_t rowg = g / b.ldu;
        const int row = (int)(rowg % b.np), m = (int)(rowg / b.np);
        const int pulse = col >> 1, comp = col & 1;
        double v = 0.0;
        if (pulse < b.batch && row < b.n)
            v = c0[(size_t)pulse * 2 * (b.lmax + 1) * b.n + 2 * ((size_t)m * b.n + row) + comp];
        b.c[g] = v;
        b.u[0][g] = v;
        b.acc[g] = taylor_acc ? v : 0.0;
    }
}

__global__ void bat_unpack_kernel(BatBuffers b, double *out) {
    const size_t total = (size_t)b.batch * 2 * (b.lmax + 1) * b.n;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const size_t per = (size_t)2 * (b.lmax + 1) * b.n;
        const int pulse = (int)(g / per);
        const size_t w = g % per;
        const size_t j = w / 2;
        const int comp = (int)(w & 1);
        const int m = (int)(j / b.n), row = (int)(j % b.n);
        out[g] = b.c[((size_t)m * b.np + row) * b.ldu + 2 * pulse + comp];
    }
}

__global__ void bat_ckpt0_kernel(BatBuffers b, const double *c0, double *ckpt, int rows) {
    const size_t per = (size_t)2 * (b.lmax + 1) * b.n;
    const size_t total = (size_t)b.batch * per;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const size_t pulse = g / per, w = g % per;
        ckpt[(pulse * rows) * per + w] = c0[g];
    }
}

// Row-major D and D^T with rows and columns zero-padded to Np. d feeds the
// column (transposed) use of a block; in the velocity gauge it holds -Q so
// that one contraction gives Q_m U_{m+1} - Q_{m-1}^T U_{m-1}.
__global__ void bat_layout_kernel(const double *src, double *d, double *dT, int lmax, int n, int Np, double dsign) {
    const size_t total = (size_t)lmax * Np * Np;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(g % Np);
        const size_t rg = g / Np;
        const int r = (int)(rg % Np), l = (int)(rg / Np);
        double v = 0.0, vt = 0.0;
        if (r < n && c < n) {
            v = dsign * src[((size_t)l * n + r) * n + c];
            vt = src[((size_t)l * n + c) * n + r];
        }
        d[g] = v;
        dT[g] = vt;
    }
}

__global__ void bat_energy_kernel(const double *src, double *dst, int lmax, int n, int Np) {
    const size_t total = (size_t)(lmax + 1) * Np;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(g % Np), l = (int)(g / Np);
        dst[g] = r < n ? src[(size_t)l * n + r] : 0.0;
    }
}

hipError_t bat_layout(const double *src_dip, const double *src_en, BatBuffers &b, hipStream_t s) {
    if (b.lmax > 0)
        hipLaunchKernelGGL(bat_layout_kernel, dim3(2048), dim3(256), 0, s, src_dip, b.d, b.dT, b.lmax, b.n, b.np,
                           b.gauge == TDSE_VELOCITY ? -1.0 : 1.0);
    hipLaunchKernelGGL(bat_energy_kernel, dim3(64), dim3(256), 0, s, src_en, b.en, b.lmax, b.n, b.np);
    return hipGetLastError();
}

hipError_t bat_pack(const BatBuffers &b, const double *c0, int taylor, hipStream_t s) {
    hipLaunchKernelGGL(bat_pack_kernel, dim3(1024), dim3(256), 0, s, b, c0, taylor);
    return hipGetLastError();
}
__global__ void bat_reduce_err_kernel(const double *gpart, int rowtiles, int batch, int64_t k, int64_t nsteps,
                                      double *err) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double s = 0.0;
    for (int rt = 0; rt < rowtiles; ++rt) s += gpart[(size_t)rt * batch + b];
    err[(size_t)b * nsteps + k] = sqrt(s);
}

hipError_t bat_reduce_err(const double *gpart, int rowtiles, int batch, int64_t k, int64_t nsteps, double *err,
                          hipStream_t s) {
    hipLaunchKernelGGL(bat_reduce_err_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, gpart, rowtiles, batch, k,
                       nsteps, err);
    return hipGetLastError();
}

hipError_t bat_unpack(const BatBuffers &b, double *out, hipStream_t s) {
    hipLaunchKernelGGL(bat_unpack_kernel, dim3(1024), dim3(256), 0, s, b, out);
    return hipGetLastError();
}
hipError_t bat_ckpt0(const BatBuffers &b, const double *c0, double *ckpt, int rows, hipStream_t s) {
    hipLaunchKernelGGL(bat_ckpt0_kernel, dim3(1024), dim3(256), 0, s, b, c0, ckpt, rows);
    return hipGetLastError();
}

template <bool ADJ>
static hipError_t bat_launch(const BatBuffers &b, const BatLaunch &l, hipStream_t s) {
    const int ntiles = (b.lmax + 1) * (b.np / b.tm) * (b.ldu / b.tn);
    const dim3 g(ntiles), blk(256), blk2(512);
    if (b.ks == 8) {  // small-batch kernel: 32-row tiles, 32 or 64 columns
        if (b.tm != 32 || (b.tn != 32 && b.tn != 64)) return hipErrorInvalidValue;
        // the longest k range of a wave: a quarter of a block's k-steps when
        // a tile has both neighbour blocks, an eighth when it has one
        const int nks = b.np / 4, maxlen = b.lmax >= 2 ? (nks + 3) / 4 : (nks + 7) / 8;
        const int chunk = maxlen <= 8 ? 8 : maxlen <= 16 ? 16 : maxlen <= 32 ? 32 : 64;
#define TDSE_SKINNY(NG_, CH_)                                                                      \
    if (b.tn == 32 * NG_ && chunk == CH_) {                                                        \
        hipLaunchKernelGGL((bat_skinny_kernel<NG_, ADJ, 8, CH_>), g, blk2, 0, s, b.d, b.dT,      \
                           l.parity ? b.u[1] : b.u[0], b.np, b.ldu, b.lmax, b, l);            \
        return hipGetLastError();                                                                  \
    }
        TDSE_SKINNY(2, 8) TDSE_SKINNY(2, 16) TDSE_SKINNY(2, 32) TDSE_SKINNY(2, 64)
        TDSE_SKINNY(1, 8) TDSE_SKINNY(1, 16) TDSE_SKINNY(1, 32) TDSE_SKINNY(1, 64)
#undef TDSE_SKINNY
        return hipErrorInvalidValue;
    }
    // The default shape of large batches keeps two chunks' panels in flight
    // (161 against 162 us per stage at 256 pulses, 181 against 186 us for a
    // Runge-Kutta-Fehlberg stage); with 128 x 128 tiles the three-deep ring
    // measured slower (186 us: one workgroup per CU).
    if (b.ks == 1 && b.tm == 128 && b.tn == 64 && b.kc == 16) {
        hipLaunchKernelGGL((bat_stage_kernel<128, 64, 16, ADJ, 1, 3>), g, blk, 0, s, b, l);
        return hipGetLastError();
    }
#define TDSE_BAT(TM_, TN_, KC_)                                                                \
    if (b.tm == TM_ && b.tn == TN_ && b.kc == KC_ && b.ks == 1) {                              \
        hipLaunchKernelGGL((bat_stage_kernel<TM_, TN_, KC_, ADJ, 1>), g, blk, 0, s, b, l);   \
        return hipGetLastError();                                                              \
    }
#define TDSE_BAT2(TM_, TN_, KC_)                                                               \
    if (b.tm == TM_ && b.tn == TN_ && b.kc == KC_ && b.ks == 2) {                              \
        hipLaunchKernelGGL((bat_stage_kernel<TM_, TN_, KC_, ADJ, 2>), g, blk2, 0, s, b, l);  \
        return hipGetLastError();                                                              \
    }
    TDSE_BAT2(32, 64, 32)
    TDSE_BAT2(32, 32, 16)
    TDSE_BAT(128, 128, 16)
    TDSE_BAT(64, 128, 16)
    TDSE_BAT(64, 64, 16)
    TDSE_BAT(64, 32, 16)
    TDSE_BAT(32, 64, 16)
    TDSE_BAT(32, 32, 16)
    TDSE_BAT(128, 64, 32)
    TDSE_BAT(64, 128, 32)
    TDSE_BAT(64, 64, 32)
    TDSE_BAT(32, 64, 32)
#undef TDSE_BAT
#undef TDSE_BAT2
    return hipErrorInvalidValue;
}

hipError_t bat_launch_stage(const BatBuffers &b, const BatLaunch &l, hipStream_t s) {
    return bat_launch<false>(b, l, s);
}
hipError_t bat_launch_adjoint(const BatBuffers &b, const BatLaunch &l, hipStream_t s) {
    return bat_launch<true>(b, l, s);
}

__global__ void bat_pack_strided_kernel(BatBuffers b, const double *src, size_t pulse_stride, double u_scale) {
    const size_t total = (size_t)(b.lmax + 1) * b.np * b.ldu;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)(g % b.ldu);
        const size_t rowg = g / b.ldu;
        const int row = (int)(rowg % b.np), m = (int)(rowg / b.np);
        const int pulse = col >> 1, comp = col & 1;
        double v = 0.0;
        if (pulse < b.batch && row < b.n) v = src[(size_t)pulse * pulse_stride + 2 * ((size_t)m * b.n + row) + comp];
        b.c[g] = v;
        b.u[0][g] = u_scale * v;
        b.acc[g] = 0.0;
    }
}

hipError_t bat_pack_strided(const BatBuffers &b, const double *src, size_t pulse_stride, double u_scale,
                            hipStream_t s) {
    hipLaunchKernelGGL(bat_pack_strided_kernel, dim3(1024), dim3(256), 0, s, b, src, pulse_stride, u_scale);
    return hipGetLastError();
}

// gpart layout for one segment: [step][product j][row tiles][batch]. RK4:
// stage 1 -> slot 0, stages 2 and 3 -> slot 1, stage 4 -> slot 2; Taylor:
// all terms of a step -> its one sample.
// Field gradient of a segment from the per-row-tile partials: for every
// (pulse, step) the sum over row tiles of each product's partial (in row-tile
// order), then the stage weights of the map. A block takes 64 (pulse, step)
// items; four threads share an item's products, neighbouring items are
// neighbouring pulses (the partials of one product and row tile are
// contiguous over the pulses).
constexpr int GRAD_ITEMS = 64;
__global__ __launch_bounds__(4 * GRAD_ITEMS) void bat_reduce_grad_kernel(const double *gpart, int rowtiles, int batch,
                                                                          int64_t k0, int64_t len, int64_t nsteps,
                                                                          int nprod, int rk4, double *grad) {
    __shared__ double sj[GRAD_ITEMS][TAYLOR_MAX_ORDER];
    const int t = threadIdx.x, it = t % GRAD_ITEMS, sub = t / GRAD_ITEMS;
    const int64_t total = (int64_t)batch * len;
    const int64_t g = (int64_t)blockIdx.x * GRAD_ITEMS + it;
    const bool live = g < total;
    const int pulse = live ? (int)(g % batch) : 0;
    const int64_t kl = live ? g / batch : 0;
    if (live) {
        for (int j = sub; j < nprod; j += 4) {
            const double *p = gpart + ((size_t)(kl * nprod + j) * rowtiles) * batch + pulse;
            double acc = 0.0;
            for (int rt = 0; rt < rowtiles; ++rt) acc += p[(size_t)rt * batch];
            sj[it][j] = acc;
        }
    }
    __syncthreads();
    if (!live || sub != 0) return;
    if (rk4) {
        double *out = grad + ((size_t)pulse * nsteps + (k0 + kl)) * 3;
        out[0] = sj[it][0];
        out[1] = sj[it][2] + sj[it][1];
        out[2] = sj[it][3];
    } else {
        double tsum = 0.0;
        for (int q = nprod - 1; q >= 0; --q) tsum += sj[it][q];
        grad[(size_t)pulse * nsteps + (k0 + kl)] = tsum;
    }
}

hipError_t bat_reduce_grad(const double *gpart, int rowtiles, int batch, int64_t k0, int64_t len,
                           int64_t nsteps, int nprod, int rk4, double *grad, hipStream_t s) {
    const int64_t items = (int64_t)batch * len;
    const int blocks = (int)((items + GRAD_ITEMS - 1) / GRAD_ITEMS);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(bat_reduce_grad_kernel, dim3(blocks), dim3(4 * GRAD_ITEMS), 0, s, gpart, rowtiles, batch, k0,
                       len, nsteps, nprod, rk4, grad);
    return hipGetLastError();
}

}  // namespace tdse
