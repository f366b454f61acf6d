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
// one kernel.
//
// Tiles are assigned to workgroups so that a tile always lands on the same
// XCD (workgroups are dispatched round-robin over the 8 XCDs); with a fixed
// grid, each XCD's L2 keeps serving the same share of the dipole from one
// launch to the next.
#include "tdse_internal.h"

namespace tdse {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

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

// z for state (m, segment q, entry e): row partials of tiles (m, q, *) then
// column partials of tiles (m-1, *, q), each in ascending tile order.
__device__ __forceinline__ double2 reduce_z(const VecBuffers &b, int par, int m, int q, int e) {
    const int T = b.T;
    double zx = 0.0, zy = 0.0;
    if (m < b.lmax) {
        const double2 *p = b.rowp[par] + ((size_t)(m * T + q) * T) * VEC_TILE_MAX + e;
        for (int jj = 0; jj < T; ++jj) {
            double2 v = p[(size_t)jj * VEC_TILE_MAX];
            zx += v.x;
            zy += v.y;
        }
    }
    if (m > 0) {
        const double2 *p = b.colp[par] + ((size_t)((m - 1) * T + q) * T) * VEC_TILE_MAX + e;
        for (int ii = 0; ii < T; ++ii) {
            double2 v = p[(size_t)ii * VEC_TILE_MAX];
            zx += v.x;
            zy += v.y;
        }
    }
    return make_double2(zx, zy);
}

__device__ __forceinline__ bool is_end(int kind) { return kind == CK_RK4_END || kind == CK_TAY_END; }

__device__ __forceinline__ double field_of(const CallDesc *d, const VecLaunch &L, int64_t &step) {
    step = d->base_step + L.off + L.comp.step_delta;
    return (step >= 0 && step < d->nsteps) ? d->field[step * d->slots + L.comp.slot] : 0.0;
}

// One entry of the state: complete the previous product, return the next
// input u, and (if this workgroup owns the entry) store the new state.
__device__ __forceinline__ double2 complete_entry(const VecBuffers &b, const VecLaunch &L,
                                                  const CallDesc *d, double dt, double F,
                                                  int64_t step, int m, int q, int e, int s0,
                                                  bool owner) {
    const int par = L.parity;
    size_t gi = (size_t)m * b.n + s0 + e;
    double2 z = reduce_z(b, par, m, q, e);
    double2 c = b.st[par][0][gi], acc = b.st[par][1][gi], u = b.st[par][2][gi];
    apply_completion(L.comp, dt, F, b.en[gi], z, c, acc, u);
    if (owner) {
        b.st[par ^ 1][0][gi] = c;
        b.st[par ^ 1][1][gi] = acc;
        b.st[par ^ 1][2][gi] = u;
        if (d->ckpt && is_end(L.comp.kind)) {
            int64_t kk = step + 1;
            if (kk % d->ckpt_every == 0) {
                size_t ns = (size_t)(b.lmax + 1) * b.n;
                reinterpret_cast<double2 *>(d->ckpt)[(size_t)(kk / d->ckpt_every) * ns + gi] = c;
            }
        }
    }
    return u;
}

__global__ __launch_bounds__(VEC_THREADS) void vec_tiles_kernel(VecBuffers b, VecLaunch L) {
    const int T = b.T, n = b.n;
    const int ntiles = b.lmax * T * T;
    const int w = blockIdx.x;
    const int tile = (int)split_start(ntiles, 8, w & 7) + (w >> 3);
    const int l = tile / (T * T), rem = tile - l * T * T, i = rem / T, j = rem - i * T;
    const int r0 = (int)split_start(n, T, i), RA = (int)split_len(n, T, i);
    const int c0 = (int)split_start(n, T, j), RB = (int)split_len(n, T, j);

    __shared__ double2 uA[VEC_TILE_MAX], uB[VEC_TILE_MAX];
    __shared__ double2 cpart[VEC_THREADS / 64][VEC_TILE_MAX];

    const CallDesc *d = b.desc;
    const double dt = d->dt;
    int64_t step;
    const double F = field_of(d, L, step);
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;

    // Issue this wave's tile loads first; they overlap the prologue.
    const int a0 = wv * 16;
    const double *Drow = b.dip + ((size_t)l * n + r0) * b.ld + c0;
    double dv0[16], dv1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int a = a0 + r;
        const double *p = Drow + (size_t)a * b.ld;
        dv0[r] = (a < RA && lane < RB) ? p[lane] : 0.0;
        dv1[r] = (a < RA && lane + 64 < RB) ? p[lane + 64] : 0.0;
    }

    // Prologue: complete the previous product for segments A = (l, i), B = (l+1, j).
    if (t < 2 * VEC_TILE_MAX) {
        const bool isB = t >= VEC_TILE_MAX;
        const int e = t & (VEC_TILE_MAX - 1);
        const int m = isB ? l + 1 : l, q = isB ? j : i, len = isB ? RB : RA, s0 = isB ? c0 : r0;
        double2 u = make_double2(0.0, 0.0);
        if (e < len) {
            const bool owner = isB ? (l == b.lmax - 1 && i == 0) : (j == 0);
            u = complete_entry(b, L, d, dt, F, step, m, q, e, s0, owner);
        }
        (isB ? uB : uA)[e] = u;
    }
    __syncthreads();

    // Tile products.
    const double2 ub0 = uB[lane], ub1 = uB[lane + 64];
    double2 cp0 = make_double2(0.0, 0.0), cp1 = make_double2(0.0, 0.0);
    double tr[16], ti[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const double2 ua = uA[(a0 + r) & (VEC_TILE_MAX - 1)];
        cp0.x = fma(dv0[r], ua.x, cp0.x);
        cp0.y = fma(dv0[r], ua.y, cp0.y);
        cp1.x = fma(dv1[r], ua.x, cp1.x);
        cp1.y = fma(dv1[r], ua.y, cp1.y);
        tr[r] = fma(dv1[r], ub1.x, dv0[r] * ub0.x);
        ti[r] = fma(dv1[r], ub1.y, dv0[r] * ub0.y);
    }
    // Transpose-reduce the 16 row partials over the 64 lanes: after the
    // xor-8/4/2/1 exchanges lane L holds row (L & 15) summed over its 16-lane
    // group; xor-16/32 finish the sum.
#pragma unroll
    for (int h = 8; h >= 1; h >>= 1) {
        const bool up = (lane & h) != 0;
#pragma unroll
        for (int k = 0; k < h; ++k) {
            double sr = up ? tr[k] : tr[k + h], si = up ? ti[k] : ti[k + h];
            double kr = up ? tr[k + h] : tr[k], ki = up ? ti[k + h] : ti[k];
            tr[k] = kr + __shfl_xor(sr, h);
            ti[k] = ki + __shfl_xor(si, h);
        }
    }
    double rs = tr[0] + __shfl_xor(tr[0], 16);
    double is = ti[0] + __shfl_xor(ti[0], 16);
    rs += __shfl_xor(rs, 32);
    is += __shfl_xor(is, 32);

    const int npar = L.parity ^ 1;
    {
        const int a = a0 + (lane & 15);
        if (lane < 16 && a < RA) {
            double2 *rp = b.rowp[npar] + ((size_t)(l * T + i) * T + j) * VEC_TILE_MAX;
            rp[a] = make_double2(rs, is);
        }
    }
    cpart[wv][lane] = cp0;
    cpart[wv][lane + 64] = cp1;
    __syncthreads();
    if (t < VEC_TILE_MAX && t < RB) {
        double2 s = cpart[0][t];
#pragma unroll
        for (int k = 1; k < VEC_THREADS / 64; ++k) s = cadd(s, cpart[k][t]);
        double2 *cpo = b.colp[npar] + ((size_t)(l * T + j) * T + i) * VEC_TILE_MAX;
        cpo[t] = s;
    }
}

// Completion only (no products): the final completion of a propagation, and
// every launch when lmax == 0 (no dipole blocks, z == 0).
__global__ __launch_bounds__(VEC_TILE_MAX) void vec_combine_kernel(VecBuffers b, VecLaunch L) {
    const int T = b.T;
    const int seg = blockIdx.x;
    const int m = seg / T, q = seg - m * T;
    const int s0 = (int)split_start(b.n, T, q), len = (int)split_len(b.n, T, q);
    const int e = threadIdx.x;
    if (e >= len) return;
    const CallDesc *d = b.desc;
    int64_t step;
    const double F = field_of(d, L, step);
    size_t gi = (size_t)m * b.n + s0 + e;
    if (L.comp.kind < 0) {  // hmul: y = E0 u + F z
        double2 z = reduce_z(b, L.parity, m, q, e);
        double2 u = b.st[L.parity][2][gi];
        double yr = fma(F, z.x, b.en[gi] * u.x), yi = fma(F, z.y, b.en[gi] * u.y);
        reinterpret_cast<double2 *>(L.out)[gi] = make_double2(yr, yi);
        return;
    }
    double2 u = complete_entry(b, L, d, d->dt, F, step, m, q, e, s0, true);
    (void)u;
    if (L.finish) reinterpret_cast<double2 *>(L.out)[gi] = b.st[L.parity ^ 1][0][gi];
}

__global__ void vec_start_kernel(VecBuffers b, int par, const double2 *c0, int taylor) {
    const size_t ns = (size_t)(b.lmax + 1) * b.n;
    const size_t np = (size_t)b.lmax * b.T * b.T * VEC_TILE_MAX;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const double2 zero = make_double2(0.0, 0.0);
    double2 *sc = par ? b.st[1][0] : b.st[0][0];
    double2 *sa = par ? b.st[1][1] : b.st[0][1];
    double2 *su = par ? b.st[1][2] : b.st[0][2];
    double2 *rp = par ? b.rowp[1] : b.rowp[0];
    double2 *cp = par ? b.colp[1] : b.colp[0];
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

__global__ void set_desc_kernel(CallDesc *d, CallDesc v) { *d = v; }
__global__ void set_desc_base_kernel(CallDesc *d, int64_t base) { d->base_step = base; }

hipError_t set_desc(CallDesc *d, const CallDesc &v, hipStream_t s) {
    hipLaunchKernelGGL(set_desc_kernel, dim3(1), dim3(1), 0, s, d, v);
    return hipGetLastError();
}
hipError_t set_desc_base(CallDesc *d, int64_t base, hipStream_t s) {
    hipLaunchKernelGGL(set_desc_base_kernel, dim3(1), dim3(1), 0, s, d, base);
    return hipGetLastError();
}

hipError_t vec_launch_tiles(const VecBuffers &b, const VecLaunch &l, hipStream_t s) {
    const int ntiles = b.lmax * b.T * b.T;
    hipLaunchKernelGGL(vec_tiles_kernel, dim3(ntiles), dim3(VEC_THREADS), 0, s, b, l);
    return hipGetLastError();
}
hipError_t vec_launch_combine(const VecBuffers &b, const VecLaunch &l, hipStream_t s) {
    hipLaunchKernelGGL(vec_combine_kernel, dim3((b.lmax + 1) * b.T), dim3(VEC_TILE_MAX), 0, s, b, l);
    return hipGetLastError();
}
hipError_t vec_launch_start(const VecBuffers &b, int32_t parity, const double *c0, int32_t method,
                            hipStream_t s) {
    hipLaunchKernelGGL(vec_start_kernel, dim3(256), dim3(256), 0, s, b, parity,
                       reinterpret_cast<const double2 *>(c0), method == TDSE_TAYLOR ? 1 : 0);
    return hipGetLastError();
}

}  // namespace tdse
