// Whole propagation in one workgroup, for small problems ((lmax+1) n <= 256
// states, n <= 64): the latency-bound regime where a launch per product would
// cost more than the product itself.
//
// Rows come in groups of R = 4 consecutive states of one block (3 or 2 for
// the larger blocks), each group owned by 4 lanes. Row a of H's off-diagonal blocks (Sec. 4, the block
// product after Eq. ode) is the concatenation of row a of D_m (towards
// u_{m+1}) and column a of D_{m-1} (towards u_{m-1}): lanes 0 and 1 of a group
// hold the two halves of the first for the group's four rows, lanes 2 and 3
// the two halves of the second, in registers for the whole run. Every u entry
// a lane reads from LDS (double-buffered) then feeds four rows: the product
// is bound by those LDS reads, and one lane per row read each entry once per
// row. A lane's elements multiply consecutive entries of u, so its reads are
// one base address plus compile-time offsets. The group sums its partials
// with DPP in a fixed order, and lane r < R of the group completes the RK4 stage
// or Taylor term (appendix B) of row r, with c and the stage accumulator kept
// in its registers. One LDS barrier per product; field samples are staged
// into LDS 64 steps at a time, one chunk ahead.
#include "tdse_internal.h"

namespace tdse {


__device__ __forceinline__ double small_dpp(double v, int ctrl_sel) {
    long long b = __double_as_longlong(v);
    int lo, hi;
    if (ctrl_sel == 1) {  // xor 1
        lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0xB1, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, true);
    } else {  // xor 2
        lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x4E, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x4E, 0xF, 0xF, true);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct SmallArgs {
    const double *en;      // [(lmax+1) n]
    const double *dip;     // tiles of the single-vector layout (T == 1)
    const double *field;   // [nsteps][S]
    const double *c0;
    double *cT;
    double *ckpt;          // [nsteps/K + 1][2 ns] or null
    int64_t nsteps, ckpt_every;
    double dt;
    int32_t lmax, n, method, order, gauge;
};

// Entries of one u buffer in LDS: the states plus room for the reads of the
// lanes whose elements run past their block (those elements are zero).
constexpr int SMALL_UBUF = 256 + 64;

// EPL: compiled bound on the dipole elements per lane and row, ceil(n / 2) <=
// EPL; R: rows per lane group (4; 3 or 2 for the larger blocks, whose
// elements would not fit the registers four rows at a time with more than
// one wave per SIMD); MAXT: threads per workgroup it is compiled for.
template <int EPL, int R, int MAXT>
__global__ __launch_bounds__(MAXT) void small_propagate_kernel(SmallArgs A) {
    constexpr int SMALL_R = R;
    const int n = A.n, lmax = A.lmax, ns = (lmax + 1) * n;
    const int S = A.method == TDSE_RK4 ? 3 : 1;
    const int t = threadIdx.x;
    const int grp = t >> 2, g = t & 3;
    const int rg_per_block = (n + SMALL_R - 1) / SMALL_R;
    const int m = grp / rg_per_block, a0 = (grp - m * rg_per_block) * SMALL_R;
    const bool live_grp = m <= lmax;
    const int a = a0 + g;                       // the row this lane completes (lanes g < R)
    const bool live = live_grp && g < SMALL_R && a < n;
    const int es = live ? m * n + a : 0;
    const int half = (n + 1) / 2;  // elements per lane and row

    __shared__ double2 ubuf[2][SMALL_UBUF];
    __shared__ double fbuf[2][64 * 3];
    __shared__ double tay_scale[64];  // dt / (p + 1) of Taylor term p + 1

    // dipole elements of this lane for the group's rows a0 + r (zero where the
    // element does not exist): lanes 0, 1: row a0 + r of D_m, columns
    // b = (g & 1) half + k, times u_{m+1}[b]; lanes 2, 3: column a0 + r of
    // D_{m-1}, rows b = (g & 1) half + k, times u_{m-1}[b]
    const bool up = g < 2;
    const int b0 = (g & 1) * half;
    double d[SMALL_R][EPL];
    const size_t tile = (size_t)VEC_TILE_MAX * VEC_TILE_MAX;
#pragma unroll
    for (int r = 0; r < SMALL_R; ++r)
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int ar = a0 + r, bb = b0 + k;
            double v = 0.0;
            if (live_grp && ar < n && k < half && bb < n) {
                if (up) {
                    if (m < lmax) v = A.dip[(size_t)m * tile + tile_pos(ar, bb)];
                } else {
                    // velocity gauge: the column use enters with a minus sign, -i (r - s)
                    if (m > 0) v = (A.gauge ? -1.0 : 1.0) * A.dip[(size_t)(m - 1) * tile + tile_pos(bb, ar)];
                }
            }
            d[r][k] = v;
        }
    // first u entry this lane reads; a missing neighbour block reads entries
    // 0.. instead (its elements are zero)
    int ubase = up ? (m + 1) * n + b0 : (m - 1) * n + b0;
    if ((up && m >= lmax) || (!up && m <= 0) || !live_grp) ubase = 0;
    const double E0 = live ? A.en[es] : 0.0;
    double2 c = make_double2(0.0, 0.0), acc = c;
    if (live) c = reinterpret_cast<const double2 *>(A.c0)[es];
    for (int x = t; x < 2 * SMALL_UBUF; x += blockDim.x) ubuf[x / SMALL_UBUF][x % SMALL_UBUF] = make_double2(0.0, 0.0);
    if (t < 64) tay_scale[t] = A.dt / (double)(t + 1);
    __syncthreads();
    if (live) {
        ubuf[0][es] = c;
        if (A.ckpt) reinterpret_cast<double2 *>(A.ckpt)[es] = c;
    }
    // field samples of steps 0..63
    for (int x = t; x < 64 * S; x += blockDim.x) {
        const int64_t st = x / S;
        fbuf[0][x] = st < A.nsteps ? A.field[st * S + x % S] : 0.0;
    }
    __syncthreads();

    const double dt = A.dt;
    const int nprod = A.method == TDSE_RK4 ? 4 : A.order;
    int par = 0;
    for (int64_t step = 0; step < A.nsteps; ++step) {
        const int fb = (int)((step >> 6) & 1), fo = (int)(step & 63);
        // stage next chunk's field samples (read at the next chunk boundary)
        if (fo == 0) {
            for (int x = t; x < 64 * S; x += blockDim.x) {
                const int64_t st = step + 64 + x / S;
                fbuf[fb ^ 1][x] = st < A.nsteps ? A.field[st * S + x % S] : 0.0;
            }
        }
        for (int p = 0; p < nprod; ++p) {
            // this lane's partial dot products of the group's four rows
            const double2 *ub = &ubuf[par][ubase];
            double zr[SMALL_R], zi[SMALL_R];
#pragma unroll
            for (int r = 0; r < SMALL_R; ++r) zr[r] = zi[r] = 0.0;
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const double2 u = ub[k];
#pragma unroll
                for (int r = 0; r < SMALL_R; ++r) {
                    zr[r] = fma(d[r][k], u.x, zr[r]);
                    zi[r] = fma(d[r][k], u.y, zi[r]);
                }
                // keep at most 8 LDS reads in flight
                if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            // group sums in a fixed order (lanes 0+1, 2+3, then the pairs)
#pragma unroll
            for (int r = 0; r < SMALL_R; ++r) {
                zr[r] += small_dpp(zr[r], 1);
                zi[r] += small_dpp(zi[r], 1);
                zr[r] += small_dpp(zr[r], 2);
                zi[r] += small_dpp(zi[r], 2);
            }
            // lane g takes row a0 + g
            double zrs = zr[0], zis = zi[0];
#pragma unroll
            for (int r = 1; r < SMALL_R; ++r) {
                zrs = g == r ? zr[r] : zrs;
                zis = g == r ? zi[r] : zis;
            }
            if (A.gauge) {  // z = -i (r - s): (x + iy) -> (y - ix)
                const double tt = zrs;
                zrs = zis;
                zis = -tt;
            }
            if (live) {
                const double2 u = ubuf[par][es];
                int slot = 0;
                if (A.method == TDSE_RK4) slot = p == 0 ? 0 : (p == 3 ? 2 : 1);
                const double F = fbuf[fb][fo * S + slot];
                // k = -i (E0 u + F z)
                const double yr = fma(F, zrs, E0 * u.x), yi = fma(F, zis, E0 * u.y);
                const double kr = yi, ki = -yr;
                double2 un;
                if (A.method == TDSE_RK4) {
                    if (p == 0) {
                        acc = make_double2(kr * (1.0 / 6.0), ki * (1.0 / 6.0));
                        un = make_double2(fma(0.5 * dt, kr, c.x), fma(0.5 * dt, ki, c.y));
                    } else if (p < 3) {
                        acc = make_double2(fma(1.0 / 3.0, kr, acc.x), fma(1.0 / 3.0, ki, acc.y));
                        const double al = p == 1 ? 0.5 * dt : dt;
                        un = make_double2(fma(al, kr, c.x), fma(al, ki, c.y));
                    } else {
                        c = make_double2(fma(dt, fma(1.0 / 6.0, kr, acc.x), c.x),
                                         fma(dt, fma(1.0 / 6.0, ki, acc.y), c.y));
                        un = c;
                    }
                } else {
                    // Taylor term T_{p+1} = (dt / (p+1)) k, accumulated onto c
                    const double sc = tay_scale[p];
                    un = make_double2(sc * kr, sc * ki);
                    acc = p == 0 ? make_double2(c.x + un.x, c.y + un.y)
                                 : make_double2(acc.x + un.x, acc.y + un.y);
                    if (p == nprod - 1) {
                        c = acc;
                        un = c;
                    }
                }
                ubuf[par ^ 1][es] = un;
            }
            par ^= 1;
            __syncthreads();
        }
        if (A.ckpt && live && (step + 1) % A.ckpt_every == 0)
            reinterpret_cast<double2 *>(A.ckpt)[(size_t)((step + 1) / A.ckpt_every) * ns + es] = c;
    }
    if (live) reinterpret_cast<double2 *>(A.cT)[es] = c;
}

bool small_eligible(int lmax, int n) { return n <= 64 && (lmax + 1) * n <= 256; }

// Absolute row sums of the symmetric coupling matrix: for state (m, a) the
// row a of D_m (towards block m+1) and the column a of D_{m-1} (towards block
// m-1); neighbouring threads take neighbouring a, so both walks read
// consecutive addresses across the wave.
__global__ void coupling_rowsum_kernel(const double *dip, int lmax, int n, double *rs) {
    const size_t ns = (size_t)(lmax + 1) * n;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < ns; g += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(g / n), a = (int)(g % n);
        double s = 0.0;
        if (m < lmax) {
            const double *row = dip + ((size_t)m * n + a) * n;
            for (int b = 0; b < n; ++b) s += fabs(row[b]);
        }
        if (m > 0) {
            const double *col = dip + (size_t)(m - 1) * n * n + a;
            for (int b = 0; b < n; ++b) s += fabs(col[(size_t)b * n]);
        }
        rs[g] = s;
    }
}

hipError_t coupling_rowsum(const double *dip, int lmax, int n, double *rs, hipStream_t s) {
    hipLaunchKernelGGL(coupling_rowsum_kernel, dim3(256), dim3(256), 0, s, dip, lmax, n, rs);
    return hipGetLastError();
}

hipError_t small_propagate(const double *en, const double *dip, int gauge, int lmax, int n, int method, int order, double dt,
                           int64_t nsteps, const double *field, const double *c0, double *cT, double *ckpt,
                           int64_t ckpt_every, hipStream_t s) {
    SmallArgs A{en, dip, field, c0, cT, ckpt, nsteps, ckpt_every > 0 ? ckpt_every : 1, dt, lmax, n, method, order, gauge};
    // four lanes per group of R rows; with (lmax + 1) n <= 256 that is at most
    // 1024 threads for n <= 16 and 512 for n <= 32 (four rows per group); for
    // n <= 52 four rows where 256 threads suffice (one wave per SIMD: the
    // 4 x 26 elements take most of its registers), else three; beyond, two
    // rows (at most 512 threads)
    const int epl = (n + 1) / 2;  // dipole elements per lane and row
    auto threads_for = [&](int R) { return ((((lmax + 1) * ((n + R - 1) / R)) * 4 + 63) / 64) * 64; };
    const dim3 one(1);
    if (epl <= 8) {
        hipLaunchKernelGGL((small_propagate_kernel<8, 4, 1024>), one, dim3(threads_for(4)), 0, s, A);
    } else if (epl <= 16) {
        hipLaunchKernelGGL((small_propagate_kernel<16, 4, 512>), one, dim3(threads_for(4)), 0, s, A);
    } else if (epl <= 26 && threads_for(4) <= 256) {
        hipLaunchKernelGGL((small_propagate_kernel<26, 4, 256>), one, dim3(threads_for(4)), 0, s, A);
    } else if (epl <= 26) {
        if (threads_for(3) > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((small_propagate_kernel<26, 3, 512>), one, dim3(threads_for(3)), 0, s, A);
    } else {
        if (threads_for(2) > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((small_propagate_kernel<32, 2, 512>), one, dim3(threads_for(2)), 0, s, A);
    }
    return hipGetLastError();
}

}  // namespace tdse
