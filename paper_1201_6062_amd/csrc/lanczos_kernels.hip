// Short-iterative Lanczos (Krylov) propagation, the propagator the paper's
// optimisation notes (Sec. 5.2) name to build on a fast product. Per step,
// with H frozen at the step's field sample:
//   v_1 = c / |c|,  v_{j+1} beta_j = H v_j - alpha_j v_j - beta_{j-1} v_{j-1},
//   alpha_j = Re <v_j, H v_j>,  c' = |c| V exp(-i dt T) e_1,
// T the tridiagonal of the alphas and betas. The products H v_j are the
// plan's own product kernels; these kernels do the per-pulse reductions,
// the recurrence, the small exponential and the recombination. Vectors are in
// the caller layout [pulse][2 n] (interleaved complex). With several pulses
// the recurrence runs over many workgroups per pulse, alpha from parts the
// batched product leaves. A single pulse on a plan of
// the fused tile path takes one launch per product (vec_lz_fused_kernel, over
// unnormalised vectors, with alpha and the norms summed from parts the
// previous launch left); on a split-path plan two: alpha from the completion
// launch's per-segment dots, the update folded into the next product launch,
// each vector normalised inside its own product's completion launch. Every
// reduction has a fixed order.
#include "tdse_internal.h"
#include "tdse_reduce.h"

namespace tdse {

// Loops over a pulse's vector take LZ_BATCH elements per thread at a time,
// every load of a batch issued before its first use (a loop that used each
// load at once would wait for every one in turn); within a thread the
// elements are still combined in ascending order.
constexpr int LZ_BATCH = 4;

// ---- Several pulses: the products run batched on the matrix cores; the
// recurrence runs over many workgroups, grid (chunks, pulses), each workgroup
// one chunk of LZB_CHUNK doubles of one pulse's vector. alpha_j comes from the
// per-(row tile, pulse) parts of Re <v_j, H v_j> that the product's epilogue
// leaves; norms from per-chunk parts. Every workgroup of a pulse sums the
// same parts in the same order, so all of them hold the same value.
constexpr int LZB_THREADS = 256;
constexpr int LZB_CHUNK = LZB_THREADS * LZ_BATCH;

int lzb_chunks(int64_t len) { return (int)((len + LZB_CHUNK - 1) / LZB_CHUNK); }

// normp[b * G + g]: chunk g's part of |x_b|^2 (x in the caller layout [B][len]).
__global__ __launch_bounds__(LZB_THREADS) void lzb_norm_parts_kernel(const double *x, int64_t len, double *normp) {
    __shared__ double red[LZB_THREADS / 64];
    const int g = blockIdx.x, b = blockIdx.y, G = gridDim.x;
    const double *xb = x + (size_t)b * len;
    const int64_t e0 = (int64_t)g * LZB_CHUNK + threadIdx.x;
    double v[LZ_BATCH];
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) {
        const int64_t e = e0 + r * LZB_THREADS;
        v[r] = e < len ? xb[e] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) s = fma(v[r], v[r], s);
    s = block_sum<LZB_THREADS>(s, red);
    if (threadIdx.x == 0) normp[(size_t)b * G + g] = s;
}

// alpha_j = sum over row tiles of the product's parts (dotp [rowtiles][B]);
// unless last: w -= alpha_j v_j + beta_{j-1} v_{j-1} over this chunk and its
// part of |w|^2. Workgroup (0, b) stores alpha_j.
__global__ __launch_bounds__(LZB_THREADS) void lzb_update_kernel(const double *dotp, int rowtiles, const double *vj,
                                                                 const double *vjm1, double *w, double *alpha,
                                                                 const double *beta, double *normp, int j, int m,
                                                                 int last, int64_t len) {
    __shared__ double red[LZB_THREADS / 64];
    const int g = blockIdx.x, b = blockIdx.y, G = gridDim.x, B = gridDim.y;
    double pa = 0.0;
    for (int rt = threadIdx.x; rt < rowtiles; rt += LZB_THREADS) pa += dotp[(size_t)rt * B + b];
    const double a = block_sum<LZB_THREADS>(pa, red);
    if (g == 0 && threadIdx.x == 0) alpha[(size_t)b * m + j] = a;
    if (last) return;
    const double bprev = j > 0 ? beta[(size_t)b * m + j - 1] : 0.0;
    const size_t off = (size_t)b * len;
    const int64_t e0 = (int64_t)g * LZB_CHUNK + threadIdx.x;
    double x[LZ_BATCH], v[LZ_BATCH], pv[LZ_BATCH];
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) {
        const int64_t e = e0 + r * LZB_THREADS;
        const bool in = e < len;
        x[r] = in ? w[off + e] : 0.0;
        v[r] = in ? vj[off + e] : 0.0;
        pv[r] = in && j > 0 ? vjm1[off + e] : 0.0;
    }
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) {
        const int64_t e = e0 + r * LZB_THREADS;
        double xr = x[r] - a * v[r];
        if (j > 0) xr -= bprev * pv[r];
        if (e < len) w[off + e] = xr;
        s2 = fma(xr, xr, s2);
    }
    s2 = block_sum<LZB_THREADS>(s2, red);
    if (threadIdx.x == 0) normp[(size_t)b * G + g] = s2;
}

// v = x / |x| per pulse, |x| from the per-chunk parts: j < 0 (the start of a
// step, x = c): beta0[b] = |c|; j >= 0: beta_j = |w| with the breakdown rule
// (beta_j <= 1e-13 (|alpha_j| + beta_{j-1}) counts as zero, and v = 0). v is
// written in the caller layout (vout) and into the batched plan's product
// input (u, layout [lmax+1][np][ldu], column 2b / 2b+1 = re / im of pulse b),
// which the next product reads.
__global__ __launch_bounds__(LZB_THREADS) void lzb_normalize_kernel(const double *x, const double *normp,
                                                                    double *vout, double *u, int lmax, int n, int np,
                                                                    int ldu, int j, int m, const double *alpha,
                                                                    double *beta, double *beta0, int64_t len) {
    __shared__ double red[LZB_THREADS / 64];
    const int g = blockIdx.x, b = blockIdx.y, G = gridDim.x;
    double nb = sqrt(block_sum_array<LZB_THREADS>(normp + (size_t)b * G, G, red));
    if (j >= 0) {
        const double bprev = j > 0 ? beta[(size_t)b * m + j - 1] : 0.0;
        if (nb <= 1e-13 * (fabs(alpha[(size_t)b * m + j]) + bprev)) nb = 0.0;
    }
    if (g == 0 && threadIdx.x == 0) {
        if (j < 0) beta0[b] = nb;
        else beta[(size_t)b * m + j] = nb;
    }
    const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
    const size_t off = (size_t)b * len;
    const int64_t e0 = (int64_t)g * LZB_CHUNK + threadIdx.x;
    double xv[LZ_BATCH];
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) {
        const int64_t e = e0 + r * LZB_THREADS;
        xv[r] = e < len ? x[off + e] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < LZ_BATCH; ++r) {
        const int64_t e = e0 + r * LZB_THREADS;
        if (e >= len) continue;
        const double v = xv[r] * inv;
        vout[off + e] = v;
        const int64_t st = e >> 1;  // state index m n + row
        const int blk = (int)(st / n), row = (int)(st - (int64_t)blk * n);
        u[((size_t)blk * np + row) * ldu + 2 * b + (e & 1)] = v;
    }
}

// Value of the previous (lane - 1) and next (lane + 1) lane, zero at the ends
// of the wave: DPP whole-wave shifts by one lane (controls 0x138 and 0x130 of
// the gfx9-family DPP encoding), two 32-bit moves per double.
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_prev(double v) { return lane_shift<0x138>(v); }
__device__ __forceinline__ double lane_next(double v) { return lane_shift<0x130>(v); }

// exp(-i dt T) e_1 for the tridiagonal T held one row per lane (a: diagonal,
// bu / bl: the entries right / left of it; zero outside the matrix), as the
// Taylor series of 16 terms over s sub-steps, s chosen so that dt |T| / s <=
// 1/2 (|T| bounded by its largest Gershgorin row sum): truncation below 1e-17
// per sub-step. Lane j returns component j.
__device__ __forceinline__ void lz_exp_series(double a, double bu, double bl, double dt, bool in, int j, double &yr,
                                              double &yi) {
    double g = fabs(a) + bu + bl;
    for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o));
    const int sub = (int)fmax(1.0, ceil(2.0 * dt * g));
    const double h = dt / sub;
    double ck[16];  // h / k, k = 1 .. 16
#pragma unroll
    for (int k = 0; k < 16; ++k) ck[k] = h / (k + 1);
    yr = (j == 0) ? 1.0 : 0.0;
    yi = 0.0;
    for (int st = 0; st < sub; ++st) {
        double tr = yr, ti = yi, sr = yr, si = yi;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // (T t)_j = a t_j + bl t_{j-1} + bu t_{j+1} (neighbour lanes
            // outside the wave read as zero)
            const double pr = lane_prev(tr), pi = lane_prev(ti);
            const double nr = lane_next(tr), ni = lane_next(ti);
            const double qr = fma(bu, nr, fma(bl, pr, a * tr));
            const double qi = fma(bu, ni, fma(bl, pi, a * ti));
            // t <- (-i h / k) (T t): (-i c)(x + iy) = c y - i c x
            tr = in ? ck[k] * qi : 0.0;
            ti = in ? -ck[k] * qr : 0.0;
            sr += tr;
            si += ti;
        }
        yr = sr;
        yi = si;
    }
}

// y = beta0 exp(-i dt T) e_1 for every pulse, one wave per pulse (lane j holds
// component j, m <= 64). The exponential is the Taylor series of 16 terms
// over s sub-steps, s chosen so that dt |T| / s <= 1/2 (|T| bounded by its
// largest Gershgorin row sum): truncation below 1e-17 per sub-step.
__global__ __launch_bounds__(64) void lz_expm_kernel(const double *alpha, const double *beta, const double *beta0,
                                                     double dt_arg, const double *dt_dev, int m, double2 *y,
                                                     const double *dotp, int nseg) {
    const int b = blockIdx.x, j = threadIdx.x;
    const double dt = dt_dev ? *dt_dev : dt_arg;  // a captured step reads the call's dt from device memory
    const bool in = j < m;
    // one pulse with dotp: alpha_{m-1} from its per-segment parts
    double alast = 0.0;
    if (dotp) {
        for (int k = j; k < nseg; k += 64) alast += dotp[k];
        alast = wave_sum(alast);
    }
    const double a = in ? (dotp && j == m - 1 ? alast : alpha[(size_t)b * m + j]) : 0.0;
    const double bu = (in && j + 1 < m) ? beta[(size_t)b * m + j] : 0.0;       // T[j][j+1]
    const double bl = (in && j > 0) ? beta[(size_t)b * m + j - 1] : 0.0;       // T[j][j-1]
    double yr, yi;
    lz_exp_series(a, bu, bl, dt, in, j, yr, yi);
    if (in) {
        const double nb = beta0[b];
        y[(size_t)b * m + j] = make_double2(nb * yr, nb * yi);
    }
}

// One pulse, one launch per Krylov product: the last vector's alpha and norm
// from the parts its launch left, the exponential, and y_j scaled by
// beta0 / beta_{j-1} (beta_{-1} = beta0), so that c = sum_j y_j x_j over the
// unnormalised vectors x_j. qin/ein/nin: the parts of x_{m-1}.
constexpr int LZ_EXPM_FUSED_THREADS = 256;
__global__ __launch_bounds__(LZ_EXPM_FUSED_THREADS) void lz_expm_fused_kernel(double *alpha, double *beta, double *beta0,
                                                           const double *qin, const double *ein, const double *nin,
                                                           int nq, int nseg, const double *fsample,
                                                           const double *dt_dev, double dt_arg, int m, double2 *y) {
    // the parts over the whole workgroup (up to four of each kind per
    // thread in one round of loads), then the exponential on wave 0
    __shared__ double red[3][LZ_EXPM_FUSED_THREADS / 64];
    const int t = threadIdx.x, j = t;
    const double dt = dt_dev ? *dt_dev : dt_arg;
    const bool in = j < m;
    double qs = 0.0, es = 0.0, ns = 0.0;
    for (int k0 = 0; k0 < nq || k0 < nseg; k0 += 4 * LZ_EXPM_FUSED_THREADS) {
        double qv[4], ev[4], nv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = k0 + r * LZ_EXPM_FUSED_THREADS + t;
            qv[r] = k < nq ? qin[k] : 0.0;
            ev[r] = k < nseg ? ein[k] : 0.0;
            nv[r] = k < nseg ? nin[k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            qs += qv[r];
            es += ev[r];
            ns += nv[r];
        }
    }
    qs = wave_sum(qs);
    es = wave_sum(es);
    ns = wave_sum(ns);
    if ((t & 63) == 0) {
        red[0][t >> 6] = qs;
        red[1][t >> 6] = es;
        red[2][t >> 6] = ns;
    }
    __syncthreads();
    if (t >= 64) return;
    qs = red[0][0];
    es = red[1][0];
    ns = red[2][0];
#pragma unroll
    for (int w = 1; w < LZ_EXPM_FUSED_THREADS / 64; ++w) {
        qs += red[0][w];
        es += red[1][w];
        ns += red[2][w];
    }
    const double F = *fsample;
    // beta_{m-2} (beta0 for m = 1) with the breakdown rule, then alpha_{m-1}
    double blast = sqrt(ns);
    if (m >= 2 && blast <= 1e-13 * (fabs(alpha[m - 2]) + (m >= 3 ? beta[m - 3] : 0.0))) blast = 0.0;
    const double sl = blast > 0.0 ? 1.0 / blast : 0.0;
    const double alast = (es + F * qs) * (sl * sl);
    // beta_q for q = 0 .. m-2 (the last from blast)
    auto beta_of = [&](int q) { return q == m - 2 ? blast : beta[q]; };
    const double a = in ? (j == m - 1 ? alast : alpha[j]) : 0.0;
    const double bu = (in && j + 1 < m) ? beta_of(j) : 0.0;
    const double bl = (in && j > 0) ? beta_of(j - 1) : 0.0;
    const double b0 = m == 1 ? blast : *beta0;
    double yr, yi;
    lz_exp_series(a, bu, bl, dt, in, j, yr, yi);
    if (in) {
        const double bj = j == 0 ? b0 : beta_of(j - 1);  // |x_j| as used: v_j = x_j / bj
        const double sc = bj > 0.0 ? b0 / bj : 0.0;
        y[j] = make_double2(sc * yr, sc * yi);
    }
    if (j == 0) {
        alpha[m - 1] = alast;
        if (m == 1) *beta0 = blast;
        else beta[m - 2] = blast;
    }
}

// c = sum_j y_j v_j (complex y_j, complex vectors), and the checkpoint row if
// one is due. Grid-stride over the complex entries of all pulses.
__global__ void lz_combine_kernel(const double *V, size_t vstride, const double2 *y, int m, int batch,
                                  int64_t ncplx, double *c, double *ckpt, int64_t ckpt_rows, int64_t ckpt_row) {
    const int64_t total = (int64_t)batch * ncplx;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(g / ncplx);
        const int64_t e = g - (int64_t)b * ncplx;
        double sr = 0.0, si = 0.0;
        int j = 0;
        for (; j + 8 <= m; j += 8) {  // loads of eight vectors before their sums
            double2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = reinterpret_cast<const double2 *>(V + (size_t)(j + q) * vstride)[g];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double2 yj = y[(size_t)b * m + j + q];
                sr = fma(yj.x, v[q].x, fma(-yj.y, v[q].y, sr));
                si = fma(yj.x, v[q].y, fma(yj.y, v[q].x, si));
            }
        }
        for (; j < m; ++j) {
            const double2 yj = y[(size_t)b * m + j];
            const double2 v = reinterpret_cast<const double2 *>(V + (size_t)j * vstride)[g];
            sr = fma(yj.x, v.x, fma(-yj.y, v.y, sr));
            si = fma(yj.x, v.y, fma(yj.y, v.x, si));
        }
        reinterpret_cast<double2 *>(c)[g] = make_double2(sr, si);
        if (ckpt)
            reinterpret_cast<double2 *>(ckpt)[((size_t)b * ckpt_rows + ckpt_row) * ncplx + e] = make_double2(sr, si);
    }
}

__global__ void lz_ckpt0_kernel(const double *c0, double *ckpt, int batch, int64_t len, int64_t rows) {
    const int64_t total = (int64_t)batch * len;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = g / len, e = g - b * len;
        ckpt[(size_t)b * rows * len + e] = c0[g];
    }
}

// One pulse over many workgroups (a single workgroup would stream the
// vectors through one CU). Each Krylov vector is formed unnormalised with
// per-workgroup parts of its squared norm; its product launch reads it as is
// and the completion launch after it (vec_hmul_dot_kernel) sums the parts,
// normalises the vector in place and scales the product. Every workgroup that
// needs a sum reduces the same parts in the same order (block_sum_array), so
// all of them hold the same value.
constexpr int LZ_WIDE_THREADS = 256;

// x_0 = c; normp[workgroup] = this workgroup's part of |c|^2.
__global__ __launch_bounds__(LZ_WIDE_THREADS) void lz_begin_wide_kernel(const double2 *c, double2 *x0,
                                                                        double *normp, int64_t ncplx) {
    __shared__ double red[LZ_WIDE_THREADS / 64];
    double s2 = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * LZ_WIDE_THREADS + threadIdx.x; g < ncplx;
         g += (int64_t)gridDim.x * LZ_WIDE_THREADS) {
        const double2 x = c[g];
        x0[g] = x;
        s2 = fma(x.x, x.x, fma(x.y, x.y, s2));
    }
    const double part = block_sum<LZ_WIDE_THREADS>(s2, red);
    if (threadIdx.x == 0) normp[blockIdx.x] = part;
}

// alpha_j = sum of the per-segment parts of Re <v_j, w> (w = H v_j); unless
// last, xnext = w - alpha_j v_j - beta_{j-1} v_{j-1} and this workgroup's
// part of |xnext|^2 to normp[workgroup]. Workgroup 0 stores alpha_j. The
// first element's operands are loaded before the alpha reduction.
__global__ __launch_bounds__(LZ_WIDE_THREADS) void lz_update_kernel(const double *dotp, int nseg, const double2 *vj,
                                                                    const double2 *vjm1, const double2 *w,
                                                                    double2 *xnext, double *alpha,
                                                                    const double *beta, int j, int last,
                                                                    double *normp, int64_t ncplx) {
    __shared__ double red[LZ_WIDE_THREADS / 64];
    int64_t g = (int64_t)blockIdx.x * LZ_WIDE_THREADS + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * LZ_WIDE_THREADS;
    const double2 zero = make_double2(0.0, 0.0);
    double2 x = zero, v = zero, pv = zero;
    if (!last && g < ncplx) {
        x = w[g];
        v = vj[g];
        if (j > 0) pv = vjm1[g];
    }
    const double a = block_sum_array<LZ_WIDE_THREADS>(dotp, nseg, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] = a;
    if (last) return;
    const double bprev = j > 0 ? beta[j - 1] : 0.0;
    double s2 = 0.0;
    while (g < ncplx) {
        x.x -= a * v.x;
        x.y -= a * v.y;
        if (j > 0) {
            x.x -= bprev * pv.x;
            x.y -= bprev * pv.y;
        }
        xnext[g] = x;
        s2 = fma(x.x, x.x, fma(x.y, x.y, s2));
        g += stride;
        if (g < ncplx) {
            x = w[g];
            v = vj[g];
            if (j > 0) pv = vjm1[g];
        }
    }
    const double part = block_sum<LZ_WIDE_THREADS>(s2, red);
    if (threadIdx.x == 0) normp[blockIdx.x] = part;
}

// c = sum_j y_j v_j (as lz_combine_kernel, one pulse), the checkpoint row if
// one is due, x_0 = c over v_0 (each thread reads its entries of every v_j
// before it writes that entry of v_0) and the norm parts of x_0.
__global__ __launch_bounds__(LZ_WIDE_THREADS) void lz_combine_wide_kernel(double2 *V, int64_t vstride2,
                                                                          const double2 *y, int m, int64_t ncplx,
                                                                          double2 *c, double2 *ckpt,
                                                                          double *normp) {
    __shared__ double red[LZ_WIDE_THREADS / 64];
    double s2 = 0.0;
    for (int64_t g = (int64_t)blockIdx.x * LZ_WIDE_THREADS + threadIdx.x; g < ncplx;
         g += (int64_t)gridDim.x * LZ_WIDE_THREADS) {
        double sr = 0.0, si = 0.0;
        // in groups of eight, all loads of a group issued before its sums
        int j = 0;
        for (; j + 8 <= m; j += 8) {
            double2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = V[(size_t)(j + q) * vstride2 + g];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double2 yj = y[j + q];
                sr = fma(yj.x, v[q].x, fma(-yj.y, v[q].y, sr));
                si = fma(yj.x, v[q].y, fma(yj.y, v[q].x, si));
            }
        }
        for (; j < m; ++j) {
            const double2 yj = y[j];
            const double2 v = V[(size_t)j * vstride2 + g];
            sr = fma(yj.x, v.x, fma(-yj.y, v.y, sr));
            si = fma(yj.x, v.y, fma(yj.y, v.x, si));
        }
        const double2 r = make_double2(sr, si);
        c[g] = r;
        if (ckpt) ckpt[g] = r;
        V[g] = r;
        s2 = fma(sr, sr, fma(si, si, s2));
    }
    const double part = block_sum<LZ_WIDE_THREADS>(s2, red);
    if (threadIdx.x == 0) normp[blockIdx.x] = part;
}

int lz_wide_groups(int64_t ncplx) {
    const int64_t g = (ncplx + LZ_WIDE_THREADS - 1) / LZ_WIDE_THREADS;
    return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

hipError_t lz_begin_wide(const double *c, double *x0, double *normp, int64_t ncplx, hipStream_t s) {
    hipLaunchKernelGGL(lz_begin_wide_kernel, dim3(lz_wide_groups(ncplx)), dim3(LZ_WIDE_THREADS), 0, s,
                       reinterpret_cast<const double2 *>(c), reinterpret_cast<double2 *>(x0), normp, ncplx);
    return hipGetLastError();
}

hipError_t lz_update(const double *dotp, int nseg, const double *vj, const double *vjm1, const double *w,
                     double *xnext, double *alpha, const double *beta, int j, int last, double *normp,
                     int64_t ncplx, hipStream_t s) {
    hipLaunchKernelGGL(lz_update_kernel, dim3(last ? 1 : lz_wide_groups(ncplx)), dim3(LZ_WIDE_THREADS), 0, s, dotp,
                       nseg, reinterpret_cast<const double2 *>(vj), reinterpret_cast<const double2 *>(vjm1),
                       reinterpret_cast<const double2 *>(w), reinterpret_cast<double2 *>(xnext), alpha, beta, j,
                       last, normp, ncplx);
    return hipGetLastError();
}

hipError_t lz_combine_wide(double *V, const double *y, int m, int64_t ncplx, double *c, double *ckpt,
                           int64_t ckpt_row, double *normp, hipStream_t s) {
    hipLaunchKernelGGL(lz_combine_wide_kernel, dim3(lz_wide_groups(ncplx)), dim3(LZ_WIDE_THREADS), 0, s,
                       reinterpret_cast<double2 *>(V), ncplx, reinterpret_cast<const double2 *>(y), m, ncplx,
                       reinterpret_cast<double2 *>(c),
                       ckpt ? reinterpret_cast<double2 *>(ckpt) + (size_t)ckpt_row * ncplx : nullptr, normp);
    return hipGetLastError();
}

hipError_t lzb_norm_parts(const double *x, int batch, int64_t len, double *normp, hipStream_t s) {
    hipLaunchKernelGGL(lzb_norm_parts_kernel, dim3(lzb_chunks(len), batch), dim3(LZB_THREADS), 0, s, x, len, normp);
    return hipGetLastError();
}
hipError_t lzb_update(const double *dotp, int rowtiles, const double *vj, const double *vjm1, double *w,
                      double *alpha, const double *beta, double *normp, int j, int m, int last, int batch,
                      int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(lzb_update_kernel, dim3(lzb_chunks(len), batch), dim3(LZB_THREADS), 0, s, dotp, rowtiles, vj,
                       vjm1, w, alpha, beta, normp, j, m, last, len);
    return hipGetLastError();
}
hipError_t lzb_normalize(const BatBuffers &bb, const double *x, const double *normp, double *vout, int j, int m,
                         const double *alpha, double *beta, double *beta0, int64_t len, hipStream_t s) {
    hipLaunchKernelGGL(lzb_normalize_kernel, dim3(lzb_chunks(len), bb.batch), dim3(LZB_THREADS), 0, s, x, normp, vout,
                       bb.u[0], bb.lmax, bb.n, bb.np, bb.ldu, j, m, alpha, beta, beta0, len);
    return hipGetLastError();
}
hipError_t lz_expm(const double *alpha, const double *beta, const double *beta0, double dt, const double *dt_dev,
                   int m, int batch, double *y, const double *dotp, int nseg, hipStream_t s) {
    hipLaunchKernelGGL(lz_expm_kernel, dim3(batch), dim3(64), 0, s, alpha, beta, beta0, dt, dt_dev, m,
                       reinterpret_cast<double2 *>(y), dotp, nseg);
    return hipGetLastError();
}
hipError_t lz_expm_fused(double *alpha, double *beta, double *beta0, const double *qin, const double *ein,
                         const double *nin, int nq, int nseg, const double *fsample, double dt,
                         const double *dt_dev, int m, double *y, hipStream_t s) {
    hipLaunchKernelGGL(lz_expm_fused_kernel, dim3(1), dim3(LZ_EXPM_FUSED_THREADS), 0, s, alpha, beta, beta0, qin, ein,
                       nin, nq, nseg,
                       fsample, dt_dev, dt, m, reinterpret_cast<double2 *>(y));
    return hipGetLastError();
}
hipError_t lz_combine(const double *V, size_t vstride, const double *y, int m, int batch, int64_t ncplx, double *c,
                      double *ckpt, int64_t ckpt_rows, int64_t ckpt_row, hipStream_t s) {
    hipLaunchKernelGGL(lz_combine_kernel, dim3(1024), dim3(256), 0, s, V, vstride,
                       reinterpret_cast<const double2 *>(y), m, batch, ncplx, c, ckpt, ckpt_rows, ckpt_row);
    return hipGetLastError();
}
hipError_t lz_ckpt0(const double *c0, double *ckpt, int batch, int64_t len, int64_t rows, hipStream_t s) {
    hipLaunchKernelGGL(lz_ckpt0_kernel, dim3(256), dim3(256), 0, s, c0, ckpt, batch, len, rows);
    return hipGetLastError();
}

}  // namespace tdse
