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

template <int TM, int TN, int KC>
struct BatTile {
    static constexpr int THREADS = 256;
    static constexpr int WM = TM / 2, WN = TN / 2;       // 2 x 2 waves
    static constexpr int SM = WM / 16, SN = WN / 16;     // 16 x 16 subtiles per wave
    static constexpr int A_ELEMS = KC * TM, B_ELEMS = KC * TN;
    static constexpr int A_PER_T = A_ELEMS / 2 / THREADS, B_PER_T = B_ELEMS / 2 / THREADS;  // double2 each
};

// ADJ = false: forward RK4 / Taylor stage (or a single product).
// ADJ = true: one stage of the discrete adjoint of an RK4 step, run in
// reverse: the product input is the co-state kbar of the stage derivative,
// ubar = i H(F) kbar (since (-iH)^H = iH for real symmetric H), the co-state
// of c accumulates sum ubar, and the field gradient Im((D kbar)^H u) is
// reduced per row tile (u = the forward input of the stage).
template <int TM, int TN, int KC, bool ADJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void bat_stage_kernel(BatBuffers b, BatLaunch L) {
    using C = BatTile<TM, TN, KC>;
    static_assert(C::A_PER_T >= 1 && C::B_PER_T >= 1, "tile too small for 256 threads");
    const int Np = b.np, ldu = b.ldu, lmax = b.lmax;
    const int RT = Np / TM, CT = ldu / TN;
    const int ntiles = (lmax + 1) * RT * CT;
    const int w = blockIdx.x;
    const int xcd = w & 7, per = ntiles >> 3, extra = ntiles & 7;
    const int tile = xcd * per + (xcd < extra ? xcd : extra) + (w >> 3);
    const int m = tile / (RT * CT), rem = tile - m * RT * CT, rt = rem / CT, ct = rem - rt * CT;
    const int r0 = rt * TM, c0 = ct * TN;

    __shared__ double As[2][KC][TM];
    __shared__ double Bs[2][KC][TN];

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wy = wv >> 1, wx = wv & 1;
    const int par = L.parity;
    const double *U = par ? b.u[1] : b.u[0];

    // K chunks: first the row use of D_m against U_{m+1}, then the transposed
    // use of D_{m-1} against U_{m-1}.
    const int kchunks = Np / KC;
    const bool has_up = m < lmax, has_dn = m > 0;
    const int nchunks = kchunks * ((has_up ? 1 : 0) + (has_dn ? 1 : 0));
    const size_t blk = (size_t)Np * Np;

    auto a_src = [&](int kc) -> const double * {
        const bool up = has_up && kc < kchunks;
        const int k0 = (up ? kc : kc - (has_up ? kchunks : 0)) * KC;
        return up ? b.dT + (size_t)m * blk + (size_t)k0 * Np + r0
                  : b.d + (size_t)(m - 1) * blk + (size_t)k0 * Np + r0;
    };
    auto b_src = [&](int kc) -> const double * {
        const bool up = has_up && kc < kchunks;
        const int k0 = (up ? kc : kc - (has_up ? kchunks : 0)) * KC;
        const int lb = up ? m + 1 : m - 1;
        return U + ((size_t)lb * Np + k0) * ldu + c0;
    };

    double2 ra[C::A_PER_T], rb[C::B_PER_T];
    auto gload = [&](int kc) {
        const double *pa = a_src(kc), *pb = b_src(kc);
#pragma unroll
        for (int q = 0; q < C::A_PER_T; ++q) {
            const int e = t + C::THREADS * q, k = e / (TM / 2), i2 = e % (TM / 2);
            ra[q] = *reinterpret_cast<const double2 *>(pa + (size_t)k * Np + 2 * i2);
        }
#pragma unroll
        for (int q = 0; q < C::B_PER_T; ++q) {
            const int e = t + C::THREADS * q, k = e / (TN / 2), j2 = e % (TN / 2);
            rb[q] = *reinterpret_cast<const double2 *>(pb + (size_t)k * ldu + 2 * j2);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < C::A_PER_T; ++q) {
            const int e = t + C::THREADS * q, k = e / (TM / 2), i2 = e % (TM / 2);
            *reinterpret_cast<double2 *>(&As[buf][k][2 * i2]) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < C::B_PER_T; ++q) {
            const int e = t + C::THREADS * q, k = e / (TN / 2), j2 = e % (TN / 2);
            *reinterpret_cast<double2 *>(&Bs[buf][k][2 * j2]) = rb[q];
        }
    };

    d4_t acc[C::SM][C::SN];
#pragma unroll
    for (int i = 0; i < C::SM; ++i)
#pragma unroll
        for (int j = 0; j < C::SN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    if (nchunks > 0) {
        gload(0);
        sstore(0);
        bat_lds_barrier();
        for (int kc = 0; kc < nchunks; ++kc) {
            const int buf = kc & 1;
            if (kc + 1 < nchunks) gload(kc + 1);
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                double af[C::SM], bf[C::SN];
#pragma unroll
                for (int i = 0; i < C::SM; ++i) af[i] = As[buf][kr][wy * C::WM + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < C::SN; ++j) bf[j] = Bs[buf][kr][wx * C::WN + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < C::SM; ++i)
#pragma unroll
                    for (int j = 0; j < C::SN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
            if (kc + 1 < nchunks) {
                sstore(buf ^ 1);
                bat_lds_barrier();
            }
        }
    }

    // ---- epilogue
    const int B = b.batch;
    const int64_t step = L.step;
    const double dt = L.dt;
    double *Un = par ? b.u[0] : b.u[1];
    double gsum[C::SN];
#pragma unroll
    for (int j = 0; j < C::SN; ++j) gsum[j] = 0.0;
#pragma unroll
    for (int i = 0; i < C::SM; ++i) {
#pragma unroll
        for (int j = 0; j < C::SN; ++j) {
            const int col = c0 + wx * C::WN + j * 16 + (lane & 15);
            const bool is_im = col & 1;
            const int pulse = col >> 1;
            double F = 0.0;
            if (pulse < B) F = b.field[((size_t)pulse * L.nsteps + step) * L.slots + L.slot];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + wy * C::WM + i * 16 + (lane >> 4) + 4 * r;
                const size_t gi = ((size_t)m * Np + row) * ldu + col;
                const double E0 = b.en[(size_t)m * Np + row];
                const double z = acc[i][j][r], zp = bat_xor1(z);
                const double uo = U[gi], up = bat_xor1(uo);
                if constexpr (ADJ) {
                    // ubar = i (E0 kbar + F w): re = -(E0 kbar_im + F w_im), im = E0 kbar_re + F w_re
                    const double ub = (is_im ? 1.0 : -1.0) * fma(F, zp, E0 * up);
                    const double us = L.ustore[gi], usp = bat_xor1(us);
                    // Im(w^H u) = sum (w_re u_im - w_im u_re)
                    gsum[j] += (is_im ? -z : z) * usp;
                    const double lam = b.c[gi];
                    const double cb = (L.first ? lam : b.acc[gi]) + ub;
                    if (L.kind == CK_ADJ_MID) {
                        b.acc[gi] = cb;
                        Un[gi] = fma(L.p_lam, lam, L.p_ub * ub);
                    } else {  // CK_ADJ_LAST: cb is the co-state of c at the step's start
                        b.c[gi] = cb;
                        Un[gi] = L.p_lam * cb;
                    }
                } else {
                    // own component of y = E0 u + F z and of k = -i y:
                    // k_re = y_im, k_im = -y_re
                    const double yre = is_im ? fma(F, zp, E0 * up) : fma(F, z, E0 * uo);
                    const double yim = is_im ? fma(F, z, E0 * uo) : fma(F, zp, E0 * up);
                    const double k = is_im ? -yre : yim;
                    if (L.kind == CK_HMUL) {  // single product y = H u (tdse_hmul)
                        if (pulse < B && row < b.n)
                            L.out[(size_t)pulse * 2 * (lmax + 1) * b.n + 2 * ((size_t)m * b.n + row) +
                                  (is_im ? 1 : 0)] = is_im ? yim : yre;
                        continue;
                    }
                    if (L.ustore) L.ustore[gi] = uo;  // forward recompute for the adjoint
                    double c = b.c[gi];
                    double a = b.acc[gi];
                    double unext;
                    switch (L.kind) {
                    case CK_RK4_MID:
                        a = L.first ? L.w_acc * k : fma(L.w_acc, k, a);
                        unext = fma(L.a_next * dt, k, c);
                        b.acc[gi] = a;
                        break;
                    case CK_RK4_END:
                        c = fma(dt, fma(L.w_acc, k, a), c);
                        unext = c;
                        b.c[gi] = c;
                        break;
                    case CK_TAY_MID: {
                        const double tm = L.a_next * dt * k;
                        a = (L.first ? c : a) + tm;
                        unext = tm;
                        b.acc[gi] = a;
                        break;
                    }
                    default: {  // CK_TAY_END
                        const double tm = L.a_next * dt * k;
                        c = (L.first ? c : a) + tm;
                        unext = c;
                        b.c[gi] = c;
                        break;
                    }
                    }
                    Un[gi] = unext;
                    if (L.ckpt && (L.kind == CK_RK4_END || L.kind == CK_TAY_END) && pulse < B && row < b.n) {
                        // caller layout [B][rows][2 n]
                        L.ckpt[((size_t)pulse * L.ckpt_rows + L.ckpt_row) * 2 * (size_t)(lmax + 1) * b.n +
                               2 * ((size_t)m * b.n + row) + (is_im ? 1 : 0)] = c;
                    }
                }
            }
        }
    }
    if constexpr (ADJ) {
        // Gradient partial of this row tile for each pulse of the column tile:
        // rows of one lane (i, r), then the four 16-lane row groups, then the
        // real/imaginary column pair, then the two row halves of the tile.
        __shared__ double gred[2][TN];
#pragma unroll
        for (int j = 0; j < C::SN; ++j) {
            double g = gsum[j];
            g += __shfl_xor(g, 16);
            g += __shfl_xor(g, 32);
            g += bat_xor1(g);
            if (lane < 16) gred[wy][wx * C::WN + j * 16 + lane] = g;
        }
        bat_lds_barrier();
        if (t < TN / 2) {
            const int pulse = c0 / 2 + t;
            if (pulse < B) L.gpart[(size_t)(m * RT + rt) * B + pulse] = gred[0][2 * t] + gred[1][2 * t];
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

// Row-major D and D^T with rows and columns zero-padded to Np.
__global__ void bat_layout_kernel(const double *src, double *d, double *dT, int lmax, int n, int Np) {
    const size_t total = (size_t)lmax * Np * Np;
    for (size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(g % Np);
        const size_t rg = g / Np;
        const int r = (int)(rg % Np), l = (int)(rg / Np);
        double v = 0.0, vt = 0.0;
        if (r < n && c < n) {
            v = src[((size_t)l * n + r) * n + c];
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
        hipLaunchKernelGGL(bat_layout_kernel, dim3(2048), dim3(256), 0, s, src_dip, b.d, b.dT, b.lmax, b.n, b.np);
    hipLaunchKernelGGL(bat_energy_kernel, dim3(64), dim3(256), 0, s, src_en, b.en, b.lmax, b.n, b.np);
    return hipGetLastError();
}

hipError_t bat_pack(const BatBuffers &b, const double *c0, int taylor, hipStream_t s) {
    hipLaunchKernelGGL(bat_pack_kernel, dim3(1024), dim3(256), 0, s, b, c0, taylor);
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
    const dim3 g(ntiles), blk(256);
#define TDSE_BAT(TM_, TN_, KC_)                                                                \
    if (b.tm == TM_ && b.tn == TN_ && b.kc == KC_) {                                           \
        hipLaunchKernelGGL((bat_stage_kernel<TM_, TN_, KC_, ADJ>), g, blk, 0, s, b, l);      \
        return hipGetLastError();                                                              \
    }
    TDSE_BAT(128, 128, 16)
    TDSE_BAT(128, 64, 16)
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

// gpart layout for one segment: [step][stage j-1][row tiles][batch];
// stage 1 -> slot 0, stages 2 and 3 -> slot 1, stage 4 -> slot 2.
__global__ void bat_reduce_grad_kernel(const double *gpart, int rowtiles, int batch, int64_t k0, int64_t len,
                                       int64_t nsteps, double *grad) {
    const int64_t total = (int64_t)batch * len;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int pulse = (int)(g / len);
        const int64_t kl = g % len;
        double sj[4];
        for (int j = 0; j < 4; ++j) {
            const double *p = gpart + ((size_t)(kl * 4 + j) * rowtiles) * batch + pulse;
            double acc = 0.0;
            for (int rt = 0; rt < rowtiles; ++rt) acc += p[(size_t)rt * batch];
            sj[j] = acc;
        }
        double *out = grad + ((size_t)pulse * nsteps + (k0 + kl)) * 3;
        out[0] = sj[0];
        out[1] = sj[2] + sj[1];
        out[2] = sj[3];
    }
}

hipError_t bat_reduce_grad(const double *gpart, int rowtiles, int batch, int64_t k0, int64_t len,
                           int64_t nsteps, double *grad, hipStream_t s) {
    hipLaunchKernelGGL(bat_reduce_grad_kernel, dim3(64), dim3(256), 0, s, gpart, rowtiles, batch, k0, len, nsteps,
                       grad);
    return hipGetLastError();
}

}  // namespace tdse
