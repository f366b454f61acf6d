/*
 * Plain FP64 CPU oracle for the TDSE propagation of O Broin & Nikolopoulos,
 * "An OpenCL implementation for the solution of TDSE on GPU and CPU
 * architectures" (arXiv:1201.6062).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct
 * reference that the HIP library is checked against. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it. It shares
 * no code, header or table with the HIP library.
 *
 * Problem (Sec. 3, Eqs. tdse_ode and tdse_ode_c; Sec. 4, Eq. ode):
 *   dc/dt = -i H(t) c,   H(t) = diag(E) + F(t) D,
 * over partial waves l = 0..lmax with n states each (state j = l*n + a).
 * D is block tridiagonal (Sec. 3, dipole selection rules, Fig. Matrix): the
 * only non-zero blocks couple l and l+1. Only the superdiagonal blocks
 * D_l = D_{l,l+1} (n x n, row-major, rows in block l, columns in block l+1)
 * are given (Sec. 5); the subdiagonal block is D_l^T, so H is real symmetric.
 * The derivative is the block matrix-vector product of Sec. 4:
 *   (H u)_l = E_l u_l + F (D_l u_{l+1} + D_{l-1}^T u_{l-1}).
 *
 * The velocity gauge of Sec. 5 replaces F D by A(t) P with the momentum
 * coupling P = -i Q (oracle_set_gauge); every function below then uses it.
 *
 * Complex vectors are interleaved (re, im) doubles. All arithmetic is double,
 * in natural ascending index order, with no blocking or reordering. Build
 * without FMA contraction (-ffp-contract=off) so every product is rounded
 * once before its sum.
 *
 * Parity pins (tests/test_oracle_pins.py): dense brute-force H on tiny
 * systems, field-free discrete-map closed form, two-level Rabi closed form,
 * eigendecomposition of the per-step polynomial propagator, RK4 convergence
 * order against a high-accuracy ODE solve, Taylor-4 = RK4 identity, norm
 * contraction, linearity, and for the adjoint the dot-product identity,
 * tangent-linear agreement and central finite differences; for the Taylor
 * adjoint the dot-product identity, finite differences and its agreement
 * with the RK4 adjoint where Taylor-4 and RK4 coincide.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RE(v, j) (v)[2 * (size_t)(j)]
#define IM(v, j) (v)[2 * (size_t)(j) + 1]

/*
 * Gauge of the coupling blocks (Sec. 5). Length gauge (0): the blocks are the
 * real dipole D_l and the coupling is real symmetric, H = E + F D. Velocity
 * gauge (1): the blocks hold the real matrix Q_l of the momentum coupling
 * P = -i Q (P_{l,l+1} = -i Q_l, P_{l+1,l} = +i Q_l^T, so P is Hermitian and
 * imaginary) and F is the vector potential A(t): H = E + A P.
 */
static int g_gauge = 0;
void oracle_set_gauge(int gauge) { g_gauge = gauge; }

/* z = D u (the field-coupling part of H, without the field factor). */
void oracle_dmul(int lmax, int n, const double *dip, const double *u, double *z)
{
    size_t ns = (size_t)(lmax + 1) * n;
    for (size_t j = 0; j < ns; ++j) { RE(z, j) = 0.0; IM(z, j) = 0.0; }
    for (int l = 0; l <= lmax; ++l) {
        for (int a = 0; a < n; ++a) {
            double ur = 0.0, ui = 0.0, dr = 0.0, di = 0.0;
            /* block l+1 -> l: row a of block l times u_{l+1} */
            if (l < lmax) {
                const double *row = dip + ((size_t)l * n + a) * n;
                for (int b = 0; b < n; ++b) {
                    size_t jb = (size_t)(l + 1) * n + b;
                    ur += row[b] * RE(u, jb);
                    ui += row[b] * IM(u, jb);
                }
            }
            /* block l-1 -> l: column a of block l-1 (its transpose) times u_{l-1} */
            if (l > 0) {
                const double *blk = dip + (size_t)(l - 1) * n * n;
                for (int b = 0; b < n; ++b) {
                    size_t jb = (size_t)(l - 1) * n + b;
                    dr += blk[(size_t)b * n + a] * RE(u, jb);
                    di += blk[(size_t)b * n + a] * IM(u, jb);
                }
            }
            size_t ja = (size_t)l * n + a;
            if (g_gauge == 0) {
                RE(z, ja) = ur + dr;
                IM(z, ja) = ui + di;
            } else {
                /* -i Q_l u_{l+1} + i Q_{l-1}^T u_{l-1} = -i (up - down); -i (x + iy) = y - ix */
                RE(z, ja) = ui - di;
                IM(z, ja) = -(ur - dr);
            }
        }
    }
}

/* y = H(F) u = E o u + F (D u)  (velocity gauge: E o u + A (P u)). */
void oracle_hmul(int lmax, int n, const double *en, const double *dip, double f,
                 const double *u, double *y)
{
    size_t ns = (size_t)(lmax + 1) * n;
    oracle_dmul(lmax, n, dip, u, y);
    for (size_t j = 0; j < ns; ++j) {
        double zr = RE(y, j), zi = IM(y, j);
        RE(y, j) = en[j] * RE(u, j) + f * zr;
        IM(y, j) = en[j] * IM(u, j) + f * zi;
    }
}

/* k = -i H(F) u  (Sec. 4: M = -iH). (-i)(x + iy) = y - ix. */
static void deriv(int lmax, int n, const double *en, const double *dip, double f,
                  const double *u, double *k, double *tmp)
{
    size_t ns = (size_t)(lmax + 1) * n;
    oracle_hmul(lmax, n, en, dip, f, u, tmp);
    for (size_t j = 0; j < ns; ++j) {
        RE(k, j) = IM(tmp, j);
        IM(k, j) = -RE(tmp, j);
    }
}

/* w = a + s * b (complex vectors, real scalar s). */
static void axpy(size_t ns, const double *a, double s, const double *b, double *w)
{
    for (size_t j = 0; j < 2 * ns; ++j) w[j] = a[j] + s * b[j];
}

/*
 * Classic fourth-order Runge-Kutta (appendix B, Eqs. RKFinal and RKDeriv;
 * the classic tableau c = (0, 1/2, 1/2, 1), a21 = a32 = 1/2, a43 = 1,
 * b = (1, 2, 2, 1)/6). field[k*3 + s] is the field at t_k + (0, dt/2, dt)[s];
 * stages 2 and 3 both use the midpoint sample.
 * c holds c(0) on entry and c(nsteps*dt) on return.
 */
int oracle_rk4(int lmax, int n, const double *en, const double *dip, double dt,
               int64_t nsteps, const double *field, double *c)
{
    size_t ns = (size_t)(lmax + 1) * n;
    double *k1 = malloc(16 * ns), *k2 = malloc(16 * ns), *k3 = malloc(16 * ns);
    double *k4 = malloc(16 * ns), *u = malloc(16 * ns), *tmp = malloc(16 * ns);
    if (!k1 || !k2 || !k3 || !k4 || !u || !tmp) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        const double *F = field + 3 * s;
        deriv(lmax, n, en, dip, F[0], c, k1, tmp);
        axpy(ns, c, 0.5 * dt, k1, u);
        deriv(lmax, n, en, dip, F[1], u, k2, tmp);
        axpy(ns, c, 0.5 * dt, k2, u);
        deriv(lmax, n, en, dip, F[1], u, k3, tmp);
        axpy(ns, c, dt, k3, u);
        deriv(lmax, n, en, dip, F[2], u, k4, tmp);
        for (size_t j = 0; j < 2 * ns; ++j)
            c[j] = c[j] + (dt / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
    }
    free(k1); free(k2); free(k3); free(k4); free(u); free(tmp);
    return 0;
}

/*
 * Truncated Taylor series propagator (appendix B, Eq. taylor): with H frozen
 * over the step at the sample field[k], c(t+dt) = sum_{m=0..order}
 * (-i dt H)^m / m! c(t), built from the scaled terms T_0 = c,
 * T_m = (-i dt / m) H T_{m-1}. This is the reading of the garbled recursion
 * in appendix B that reproduces Eq. taylor.
 */
int oracle_taylor(int lmax, int n, const double *en, const double *dip, int order,
                  double dt, int64_t nsteps, const double *field, double *c)
{
    size_t ns = (size_t)(lmax + 1) * n;
    double *t = malloc(16 * ns), *h = malloc(16 * ns), *acc = malloc(16 * ns);
    if (!t || !h || !acc) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        memcpy(t, c, 16 * ns);
        memcpy(acc, c, 16 * ns);
        for (int m = 1; m <= order; ++m) {
            oracle_hmul(lmax, n, en, dip, field[s], t, h);
            double sc = dt / (double)m;
            /* (-i sc)(x + iy) = sc*y - i sc*x */
            for (size_t j = 0; j < ns; ++j) {
                RE(t, j) = sc * IM(h, j);
                IM(t, j) = -sc * RE(h, j);
            }
            for (size_t j = 0; j < 2 * ns; ++j) acc[j] = acc[j] + t[j];
        }
        memcpy(c, acc, 16 * ns);
    }
    free(t); free(h); free(acc);
    return 0;
}

/*
 * Tangent-linear RK4: propagates (c, dc) for a field perturbation dfield
 * (same layout as field). Differentiating f(F, u) = -i (E o u + F D u):
 *   df = -i H(F) du - i dF (D u).
 * Independent of the adjoint below; used to check it.
 */
int oracle_rk4_tangent(int lmax, int n, const double *en, const double *dip, double dt,
                       int64_t nsteps, const double *field, const double *dfield,
                       double *c, double *dc)
{
    size_t ns = (size_t)(lmax + 1) * n;
    double *k[4], *dk[4];
    double *u = malloc(16 * ns), *du = malloc(16 * ns), *tmp = malloc(16 * ns);
    double *z = malloc(16 * ns);
    for (int i = 0; i < 4; ++i) { k[i] = malloc(16 * ns); dk[i] = malloc(16 * ns); }
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const int slot[4] = {0, 1, 1, 2};
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int i = 0; i < 4; ++i) {
            if (i == 0) {
                memcpy(u, c, 16 * ns);
                memcpy(du, dc, 16 * ns);
            } else {
                axpy(ns, c, alpha[i] * dt, k[i - 1], u);
                axpy(ns, dc, alpha[i] * dt, dk[i - 1], du);
            }
            double F = field[3 * s + slot[i]], dF = dfield[3 * s + slot[i]];
            deriv(lmax, n, en, dip, F, u, k[i], tmp);
            deriv(lmax, n, en, dip, F, du, dk[i], tmp);
            oracle_dmul(lmax, n, dip, u, z);
            for (size_t j = 0; j < ns; ++j) {       /* -i dF z */
                RE(dk[i], j) = RE(dk[i], j) + dF * IM(z, j);
                IM(dk[i], j) = IM(dk[i], j) - dF * RE(z, j);
            }
        }
        for (size_t j = 0; j < 2 * ns; ++j) {
            c[j] = c[j] + (dt / 6.0) * (k[0][j] + 2.0 * k[1][j] + 2.0 * k[2][j] + k[3][j]);
            dc[j] = dc[j] + (dt / 6.0) * (dk[0][j] + 2.0 * dk[1][j] + 2.0 * dk[2][j] + dk[3][j]);
        }
    }
    for (int i = 0; i < 4; ++i) { free(k[i]); free(dk[i]); }
    free(u); free(du); free(tmp); free(z);
    return 0;
}

/*
 * Discrete adjoint of the RK4 map above, for a real loss L(c(T)).
 * Convention: dL = Re(lambda^H dc), lambda = dL/dRe c + i dL/dIm c.
 * On entry lam = lambda_T; on return lam = lambda_0 and grad[k*3+s] =
 * dL/dfield[k*3+s]. Each step reverses the stages in order 4, 3, 2, 1:
 * with kbar_i the co-state of stage derivative k_i and u_i its input,
 *   ubar_i = i H(F_i) kbar_i            (since (-iH)^H = iH, H real symmetric)
 *   g(F_i) += Im((D kbar_i)^H u_i)      (from d k_i / dF = -i D u_i)
 * and kbar_i receives b_i dt lambda plus a_{i+1,i} dt ubar_{i+1}.
 * Forward states c_k are stored for every step and the stage inputs are
 * recomputed from them.
 */
int oracle_rk4_adjoint(int lmax, int n, const double *en, const double *dip, double dt,
                       int64_t nsteps, const double *field, const double *c0,
                       double *lam, double *grad)
{
    size_t ns = (size_t)(lmax + 1) * n;
    double *cs = malloc(16 * ns * (size_t)(nsteps + 1));
    double *u[4], *k[4];
    for (int i = 0; i < 4; ++i) { u[i] = malloc(16 * ns); k[i] = malloc(16 * ns); }
    double *tmp = malloc(16 * ns), *kb = malloc(16 * ns), *ub = malloc(16 * ns);
    double *cb = malloc(16 * ns), *z = malloc(16 * ns);
    if (!cs || !tmp || !kb || !ub || !cb || !z) return -1;
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
    static const int slot[4] = {0, 1, 1, 2};

    memcpy(cs, c0, 16 * ns);
    for (int64_t s = 0; s < nsteps; ++s) {
        double *c = cs + 2 * ns * (size_t)s, *cn = cs + 2 * ns * (size_t)(s + 1);
        memcpy(cn, c, 16 * ns);
        oracle_rk4(lmax, n, en, dip, dt, 1, field + 3 * s, cn);
    }
    for (int64_t s = 0; s < 3 * nsteps; ++s) grad[s] = 0.0;

    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *c = cs + 2 * ns * (size_t)s;
        /* Recompute the stage inputs u_i and derivatives k_i of step s. */
        for (int i = 0; i < 4; ++i) {
            if (i == 0) memcpy(u[0], c, 16 * ns);
            else axpy(ns, c, alpha[i] * dt, k[i - 1], u[i]);
            deriv(lmax, n, en, dip, field[3 * s + slot[i]], u[i], k[i], tmp);
        }
        memcpy(cb, lam, 16 * ns);                   /* c' = c + ... gives cbar = lambda */
        /* ub holds ubar_{i+1} (zero before stage 4). */
        for (size_t j = 0; j < 2 * ns; ++j) ub[j] = 0.0;
        for (int i = 3; i >= 0; --i) {
            double F = field[3 * s + slot[i]];
            double a_next = (i < 3) ? alpha[i + 1] : 0.0;
            for (size_t j = 0; j < 2 * ns; ++j) kb[j] = bw[i] * dt * lam[j] + a_next * dt * ub[j];
            /* g += Im((D kb)^H u_i) = sum Re(z) Im(u) - Im(z) Re(u). */
            oracle_dmul(lmax, n, dip, kb, z);
            double g = 0.0;
            for (size_t j = 0; j < ns; ++j) g += RE(z, j) * IM(u[i], j) - IM(z, j) * RE(u[i], j);
            grad[3 * s + slot[i]] += g;
            /* ub = i H(F) kb: i (x + iy) = -y + ix. */
            oracle_hmul(lmax, n, en, dip, F, kb, tmp);
            for (size_t j = 0; j < ns; ++j) {
                RE(ub, j) = -IM(tmp, j);
                IM(ub, j) = RE(tmp, j);
            }
            for (size_t j = 0; j < 2 * ns; ++j) cb[j] = cb[j] + ub[j];
        }
        memcpy(lam, cb, 16 * ns);
    }
    for (int i = 0; i < 4; ++i) { free(u[i]); free(k[i]); }
    free(cs); free(tmp); free(kb); free(ub); free(cb); free(z);
    return 0;
}

/*
 * Discrete adjoint of the Taylor map above (same convention as the RK4
 * adjoint: dL = Re(lambda^H dc); on entry lam = lambda_T, on return
 * lam = lambda_0 and grad[k] = dL/dfield[k]). One step is
 *   c' = T_0 + T_1 + ... + T_p,  T_0 = c,  T_m = a_m H(F) T_{m-1},
 * with a_m = -i dt / m. Every T_m reaches c' directly and through T_{m+1}, so
 * with lambda the co-state of c' the co-states of the terms are
 *   Tbar_p = lambda,  Tbar_{m-1} = lambda + conj(a_m) H Tbar_m  (m = p..1),
 * using H^T = H (real symmetric), and the co-state of c is Tbar_0. The field
 * enters every term through dT_m / dF = a_m D T_{m-1}, so
 *   g(F) = sum_m Re(Tbar_m^H a_m D T_{m-1}) = sum_m (dt / m) Im((D Tbar_m)^H T_{m-1}).
 * Forward states c_k are stored for every step; the terms of a step are
 * recomputed from c_k.
 */
int oracle_taylor_adjoint(int lmax, int n, const double *en, const double *dip, int order, double dt,
                          int64_t nsteps, const double *field, const double *c0, double *lam, double *grad)
{
    size_t ns = (size_t)(lmax + 1) * n;
    double *cs = malloc(16 * ns * (size_t)(nsteps + 1));
    double *terms = malloc(16 * ns * (size_t)(order + 1));
    double *tb = malloc(16 * ns), *h = malloc(16 * ns), *z = malloc(16 * ns);
    if (!cs || !terms || !tb || !h || !z) return -1;

    memcpy(cs, c0, 16 * ns);
    for (int64_t s = 0; s < nsteps; ++s) {
        double *cn = cs + 2 * ns * (size_t)(s + 1);
        memcpy(cn, cs + 2 * ns * (size_t)s, 16 * ns);
        oracle_taylor(lmax, n, en, dip, order, dt, 1, field + s, cn);
    }
    for (int64_t s = 0; s < nsteps; ++s) grad[s] = 0.0;

    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double F = field[s];
        /* recompute T_0 .. T_{p-1} of step s */
        memcpy(terms, cs + 2 * ns * (size_t)s, 16 * ns);
        for (int m = 1; m < order; ++m) {
            const double *tp = terms + 2 * ns * (size_t)(m - 1);
            double *tm = terms + 2 * ns * (size_t)m;
            oracle_hmul(lmax, n, en, dip, F, tp, h);
            double sc = dt / (double)m;
            for (size_t j = 0; j < ns; ++j) {
                RE(tm, j) = sc * IM(h, j);
                IM(tm, j) = -sc * RE(h, j);
            }
        }
        memcpy(tb, lam, 16 * ns);                    /* Tbar_p = lambda */
        for (int m = order; m >= 1; --m) {
            const double *tprev = terms + 2 * ns * (size_t)(m - 1);
            const double sc = dt / (double)m;
            /* g += (dt/m) Im((D Tbar_m)^H T_{m-1}) */
            oracle_dmul(lmax, n, dip, tb, z);
            double g = 0.0;
            for (size_t j = 0; j < ns; ++j) g += RE(z, j) * IM(tprev, j) - IM(z, j) * RE(tprev, j);
            grad[s] += sc * g;
            /* Tbar_{m-1} = lambda + (i dt/m) H Tbar_m ; i (x + iy) = -y + ix */
            oracle_hmul(lmax, n, en, dip, F, tb, h);
            for (size_t j = 0; j < ns; ++j) {
                RE(tb, j) = RE(lam, j) - sc * IM(h, j);
                IM(tb, j) = IM(lam, j) + sc * RE(h, j);
            }
        }
        memcpy(lam, tb, 16 * ns);                    /* lambda_s = Tbar_0 */
    }
    free(cs); free(terms); free(tb); free(h); free(z);
    return 0;
}

/*
 * Runge-Kutta-Fehlberg 4(5) (the embedded pair of appendix B's RK family):
 * six stages at t_k + c_i dt with c = (0, 1/4, 3/8, 12/13, 1, 1/2) and
 * Fehlberg's coefficients a_ij; c advances with the fifth-order weights b5
 * (Sec. 5.1: the paper propagates the pair's fifth-order solution) and
 * err[k] = |dt sum_i (b5_i - b4_i) k_i|_2 is the embedded estimate of step k
 * (b4: the fourth-order weights). field[k*6 + i] is the field at stage i of
 * step k.
 */
int oracle_rkf45(int lmax, int n, const double *en, const double *dip, double dt, int64_t nsteps,
                 const double *field, double *c, double *err)
{
    static const double A[6][5] = {
        {0, 0, 0, 0, 0},
        {1.0 / 4.0, 0, 0, 0, 0},
        {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
        {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
        {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
        {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
    static const double B4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
    static const double B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};
    size_t ns = (size_t)(lmax + 1) * n;
    double *k[6];
    for (int i = 0; i < 6; ++i) k[i] = malloc(16 * ns);
    double *u = malloc(16 * ns), *tmp = malloc(16 * ns);
    if (!u || !tmp) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int i = 0; i < 6; ++i) {
            for (size_t j = 0; j < 2 * ns; ++j) {
                double acc = 0.0;
                for (int q = 0; q < i; ++q) acc += A[i][q] * k[q][j];
                u[j] = c[j] + dt * acc;
            }
            deriv(lmax, n, en, dip, field[6 * s + i], u, k[i], tmp);
        }
        double e2 = 0.0;
        for (size_t j = 0; j < 2 * ns; ++j) {
            double acc5 = 0.0, de = 0.0;
            for (int i = 0; i < 6; ++i) {
                acc5 += B5[i] * k[i][j];
                de += (B5[i] - B4[i]) * k[i][j];
            }
            c[j] = c[j] + dt * acc5;
            e2 += (dt * de) * (dt * de);
        }
        if (err) err[s] = sqrt(e2);
    }
    for (int i = 0; i < 6; ++i) free(k[i]);
    free(u); free(tmp);
    return 0;
}
