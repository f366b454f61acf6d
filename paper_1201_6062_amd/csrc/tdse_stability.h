// Host-only stability bounds of the step maps on the imaginary axis (no HIP
// calls, so every rule here can be exercised without a GPU).
//
// For the linear system dc/dt = -i H c with H Hermitian, one step of an
// explicit Runge-Kutta method or of the truncated Taylor series (appendix B)
// multiplies each eigencomponent of H by R(-i dt lambda), where R is the
// method's stability polynomial: the degree-p Taylor polynomial of exp for
// Taylor-p and for RK4 (p = 4: classic RK4 on a linear autonomous system is
// Taylor-4), and 1 + sum_k gamma_k z^k with gamma_k = b^T A^{k-1} 1 for the
// Runge-Kutta-Fehlberg pair (A its stage matrix, b the fifth-order weights
// that advance the solution, as the paper's propagator does, Sec. 5.1). The step is stable when |R(i theta)| <= 1 for
// every |theta| <= dt ||H||; ||H|| <= max|E| + |F| ||D|| and ||D||_2 <= the
// largest absolute row sum of the symmetric coupling matrix.
#pragma once

#include <math.h>

#include "../../include/tdse.h"

namespace tdse {

// Rounding allowance of the stability test: |R(i theta)|^2 <= 1 + STAB_TOL.
// Taylor orders p = 1, 2 (mod 4) and the Fehlberg pair's fifth-order
// solution amplify for every theta > 0 (|R|^2 - 1 ~ theta^(p+1), theta^(p+2),
// or theta^6 (1/360 - 1/1040) for Fehlberg, whose z^6 coefficient is 1/2080),
// so their interval is only as wide as this allowance lets it be.
constexpr double STAB_TOL = 1e-14;

// Fehlberg's 4(5) pair: stage matrix (stage times 0, 1/4, 3/8, 12/13, 1, 1/2)
// and the fifth-order weights.
constexpr double FEHLBERG_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0}};
constexpr double FEHLBERG_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};

// Coefficients r[0..deg] of the method's stability polynomial; returns deg
// (0 for methods without one: the Lanczos propagator is unitary).
inline int stability_poly(int method, int order, double *r /* [33] */) {
    if (method == TDSE_RK4 || method == TDSE_TAYLOR) {
        const int p = method == TDSE_RK4 ? 4 : order;
        r[0] = 1.0;
        for (int k = 1; k <= p; ++k) r[k] = r[k - 1] / k;
        return p;
    }
    if (method == TDSE_RKF45) {
        double v[6] = {1, 1, 1, 1, 1, 1};  // A^{k-1} 1
        r[0] = 1.0;
        for (int k = 1; k <= 6; ++k) {
            double g = 0.0;
            for (int i = 0; i < 6; ++i) g += FEHLBERG_B5[i] * v[i];
            r[k] = g;
            double w[6];
            for (int i = 0; i < 6; ++i) {
                w[i] = 0.0;
                for (int j = 0; j < 6; ++j) w[i] += FEHLBERG_A[i][j] * v[j];
            }
            for (int i = 0; i < 6; ++i) v[i] = w[i];
        }
        return 6;
    }
    return 0;
}

// |R(i theta)|^2 for polynomial coefficients r[0..deg].
inline double amplification2(const double *r, int deg, double theta) {
    double re = 0.0, im = 0.0, pw = 1.0;  // (i theta)^k = i^k theta^k
    for (int k = 0; k <= deg; ++k) {
        switch (k & 3) {
        case 0: re += r[k] * pw; break;
        case 1: im += r[k] * pw; break;
        case 2: re -= r[k] * pw; break;
        default: im -= r[k] * pw; break;
        }
        pw *= theta;
    }
    return re * re + im * im;
}

// Largest theta such that |R(i s)|^2 <= 1 + STAB_TOL for every 0 <= s <=
// theta (a scan in steps of 1e-3, then bisection to 1e-12 relative);
// infinity for the unitary Lanczos propagator.
inline double stability_bound(int method, int order) {
    double r[33];
    const int deg = stability_poly(method, order, r);
    if (deg == 0) return INFINITY;
    const double step = 1e-3;
    double lo = 0.0;
    // below the first grid point the amplification can already exceed the
    // tolerance (p = 1, 2): bisect on [0, step] then
    double hi = step;
    while (amplification2(r, deg, hi) <= 1.0 + STAB_TOL && hi < 64.0) {
        lo = hi;
        hi += step;
    }
    if (hi >= 64.0) return 64.0;
    for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (amplification2(r, deg, mid) <= 1.0 + STAB_TOL) lo = mid;
        else hi = mid;
    }
    return lo;
}

// True when |R(i theta)| <= 1 on a whole interval [0, theta*] of positive
// width (RK4, Taylor orders p = 0, 3 mod 4); false when the step amplifies
// every oscillation (Taylor p = 1, 2 mod 4, the Fehlberg pair): the sign of
// the lowest-order non-vanishing coefficient of |R(i theta)|^2 - 1 as a
// polynomial in theta (coefficients below 1e-12 of their largest term count
// as cancelled).
inline bool has_stability_interval(int method, int order) {
    double r[33];
    const int deg = stability_poly(method, order, r);
    if (deg == 0) return true;
    double re[33] = {0}, im[33] = {0};
    for (int k = 0; k <= deg; ++k) {
        const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;  // i^k = sg (k even) or sg i (k odd)
        if (k & 1) im[k] = sg * r[k];
        else re[k] = sg * r[k];
    }
    for (int m = 1; m <= 2 * deg; ++m) {
        double c = 0.0, big = 0.0;
        for (int i = 0; i <= m; ++i) {
            const int j = m - i;
            if (i > deg || j > deg) continue;
            const double t = re[i] * re[j] + im[i] * im[j];
            c += t;
            big = fabs(t) > big ? fabs(t) : big;
        }
        if (fabs(c) > 1e-12 * big) return c < 0.0;
    }
    return true;
}

// theta = dt (emax + fmax dnorm) against the method's bound: TDSE_E_UNSTABLE
// when it exceeds it (a sufficient test: every eigenvalue of dt H(F) for
// |F| <= fmax lies within +-theta).
inline tdse_status check_stability(int method, int order, double dt, double emax, double fmax, double dnorm,
                                   double *theta_out, double *bound_out) {
    const double theta = dt * (emax + fabs(fmax) * dnorm);
    const double bound = stability_bound(method, order);
    if (theta_out) *theta_out = theta;
    if (bound_out) *bound_out = bound;
    return theta <= bound ? TDSE_OK : TDSE_E_UNSTABLE;
}

}  // namespace tdse
