// Host-only checks of the library's argument validation, work split and
// dipole tile order.
// Built with g++ (no HIP) by tests/test_abi_cpu.py; prints one line per
// failed check and exits non-zero if any failed.
#include <math.h>
#include <stdio.h>

#include <complex>

#include "tdse_split.h"
#include "tdse_stability.h"
#include "tdse_tile.h"
#include "tdse_validate.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

int main() {
    using namespace tdse;
    // Sec. 4.1 split: exact tiling, lengths differ by at most one.
    for (int w = 0; w < 300; ++w)
        for (int p = 1; p < 40; ++p) {
            int64_t pos = 0, mn = 1 << 30, mx = -1;
            for (int i = 0; i < p; ++i) {
                CHECK(split_start(w, p, i) == pos);
                int64_t l = split_len(w, p, i);
                pos += l;
                mn = l < mn ? l : mn;
                mx = l > mx ? l : mx;
            }
            CHECK(pos == w);
            CHECK(mx - mn <= 1);
        }
    // Dipole segments: the split over 16-row units tiles [0, n) in order;
    // every segment but the last is whole units, none is empty, and none
    // exceeds 128 rows when T >= ceil(n / 128).
    for (int n = 1; n < 1200; n += (n < 300 ? 1 : 7))
        for (int T = 1; T <= (n + 15) / 16 && T <= 24; ++T) {
            int64_t pos = 0;
            for (int q = 0; q < T; ++q) {
                const int64_t st = seg_start(n, T, q), ln = seg_len(n, T, q);
                CHECK(st == pos);
                CHECK(ln >= 1);
                if (q + 1 < T) CHECK(ln % 16 == 0);
                if (T >= (n + 127) / 128) CHECK(ln <= 128);
                CHECK(st == 16 * split_start((n + 15) / 16, T, q));
                pos += ln;
            }
            CHECK(pos == n);
        }
    // Patches: patch_np(T) per block dimension, each at most 4 tiles wide.
    for (int T = 1; T <= 16; ++T) {
        const int np = (T + 3) / 4;
        for (int p = 0; p < np; ++p) CHECK(split_len(T, np, p) >= 1 && split_len(T, np, p) <= 4);
    }
    // Tile order: a bijection of [0,128)^2 onto [0,16384); lane (h, q) of
    // wave w reads double2 number 64 (16 w + jj) + 16 h + q in load jj and
    // finds rows q + 16k, columns 16w + 4h + c there.
    {
        static int seen[128 * 128];
        for (int a = 0; a < 128; ++a)
            for (int b = 0; b < 128; ++b) {
                const int64_t p = tile_pos(a, b);
                CHECK(p >= 0 && p < 128 * 128);
                if (p < 0 || p >= 128 * 128) continue;
                ++seen[p];
                int a2 = -1, b2 = -1;
                tile_elem(p, &a2, &b2);
                CHECK(a2 == a && b2 == b);
                const int64_t d2 = p >> 1, lane = d2 & 63, w = d2 >> 10, jj = (d2 >> 6) & 15;
                CHECK((lane & 15) == (a & 15) && jj / 2 == a / 16);
                CHECK(w == b / 16 && (lane >> 4) == (b % 16) / 4 && 2 * (jj & 1) + (p & 1) == b % 4);
            }
        for (int p = 0; p < 128 * 128; ++p) CHECK(seen[p] == 1);
    }
    std::string why;
    int dummy = 0;
    CHECK(validate_create(nullptr, &dummy, &dummy, 1, 1, 1, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, nullptr, &dummy, 1, 1, 1, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, nullptr, 1, 1, 1, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, nullptr, 0, 5, 1, &why) == TDSE_OK);
    CHECK(validate_create(&dummy, &dummy, &dummy, -1, 5, 1, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, &dummy, 3, 0, 1, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, &dummy, 3, 5, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, &dummy, 1 << 20, 1 << 20, 1 << 10, &why) == TDSE_E_INVAL);
    CHECK(validate_create(&dummy, &dummy, &dummy, 15, 500, 256, &why) == TDSE_OK);
    CHECK(validate_propagate(false, 0, 0, 0.1, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 2, 0, 0.1, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 1, 0, 0.1, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 1, 33, 0.1, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 1, 32, 0.1, 1, false, 0, &why) == TDSE_OK);
    CHECK(validate_propagate(true, 0, 0, -0.1, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 0, 0, NAN, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 0, 0, INFINITY, 1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 0, 0, 0.1, -1, false, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 0, 0, 0.1, 0, false, 0, &why) == TDSE_OK);
    CHECK(validate_propagate(true, 0, 0, 0.1, 5, true, 0, &why) == TDSE_E_INVAL);
    CHECK(validate_propagate(true, 0, 0, 0.1, 5, true, 1, &why) == TDSE_OK);
    // Stability polynomials against the step maps themselves: one step of
    // dy/dt = -i lam y run stage by stage (RK4 tableau; Fehlberg's tableau with
    // its fifth-order weights; the Taylor recursion) equals R(-i dt lam).
    {
        typedef std::complex<double> cd;
        for (double th : {0.1, 0.7, 1.9, 2.5, 3.1}) {
            const cd z(0.0, -th);  // dt * (-i lam), lam = th / dt
            double r[33];
            // RK4
            cd k1 = z, k2 = z * (1.0 + 0.5 * k1), k3 = z * (1.0 + 0.5 * k2), k4 = z * (1.0 + k3);
            cd y = 1.0 + (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
            int deg = stability_poly(TDSE_RK4, 0, r);
            CHECK(fabs(std::norm(y) - amplification2(r, deg, th)) < 1e-13);
            // Taylor-p
            for (int p = 1; p <= 12; ++p) {
                cd t = 1.0, acc = 1.0;
                for (int m = 1; m <= p; ++m) {
                    t *= z / (double)m;
                    acc += t;
                }
                deg = stability_poly(TDSE_TAYLOR, p, r);
                CHECK(fabs(std::norm(acc) - amplification2(r, deg, th)) < 1e-12);
            }
            // Fehlberg, fifth-order solution
            cd k[6];
            for (int i = 0; i < 6; ++i) {
                cd u = 1.0;
                for (int j = 0; j < i; ++j) u += FEHLBERG_A[i][j] * k[j];
                k[i] = z * u;
            }
            cd yf = 1.0;
            for (int i = 0; i < 6; ++i) yf += FEHLBERG_B5[i] * k[i];
            deg = stability_poly(TDSE_RKF45, 0, r);
            CHECK(fabs(std::norm(yf) - amplification2(r, deg, th)) < 1e-13);
        }
        double r[33];
        stability_poly(TDSE_RKF45, 0, r);
        // fifth order: the exponential's coefficients up to z^5
        CHECK(fabs(r[1] - 1.0) < 1e-15 && fabs(r[2] - 0.5) < 1e-15 && fabs(r[3] - 1.0 / 6.0) < 1e-15 &&
              fabs(r[4] - 1.0 / 24.0) < 1e-15 && fabs(r[5] - 1.0 / 120.0) < 1e-15);
        // bounds: classic values on the imaginary axis
        CHECK(fabs(stability_bound(TDSE_RK4, 0) - 2.0 * sqrt(2.0)) < 1e-6);
        CHECK(fabs(stability_bound(TDSE_TAYLOR, 4) - 2.0 * sqrt(2.0)) < 1e-6);
        CHECK(fabs(stability_bound(TDSE_TAYLOR, 3) - sqrt(3.0)) < 1e-6);
        CHECK(stability_bound(TDSE_TAYLOR, 1) < 2e-7);  // explicit Euler amplifies at once
        CHECK(stability_bound(TDSE_TAYLOR, 8) > stability_bound(TDSE_RK4, 0));
        // Fehlberg's fifth-order solution: z^6 coefficient 1/2080, so
        // |R|^2 - 1 = theta^6 (1/360 - 1/1040) + ... (1/360 from the degree-5
        // Taylor part)
        CHECK(fabs(r[6] - 1.0 / 2080.0) < 1e-15);
        CHECK(fabs(stability_bound(TDSE_RKF45, 0) - pow(1e-14 / (1.0 / 360 - 1.0 / 1040), 1.0 / 6)) < 1e-4);
        for (int p = 1; p <= 16; ++p)
            CHECK(has_stability_interval(TDSE_TAYLOR, p) == (p % 4 == 0 || p % 4 == 3));
        CHECK(has_stability_interval(TDSE_RK4, 0) && !has_stability_interval(TDSE_RKF45, 0));
        CHECK(isinf(stability_bound(TDSE_LANCZOS, 8)));
        // the bound is the first crossing of 1 + STAB_TOL
        for (int m : {TDSE_RK4}) {
            const double b = stability_bound(m, 0);
            const int deg = stability_poly(m, 0, r);
            for (double s = 0.0; s <= b; s += b / 997.0) CHECK(amplification2(r, deg, s) <= 1.0 + STAB_TOL);
            CHECK(amplification2(r, deg, b * (1.0 + 1e-6)) > 1.0 + STAB_TOL);
        }
        double th = 0.0, bd = 0.0;
        // c5-like: dt 0.01, max|E| 29.6, field 0.1, row-sum bound 133
        CHECK(check_stability(TDSE_RK4, 0, 0.01, 29.6, 0.1, 133.0, &th, &bd) == TDSE_OK);
        CHECK(fabs(th - 0.01 * (29.6 + 13.3)) < 1e-12 && fabs(bd - 2.0 * sqrt(2.0)) < 1e-6);
        CHECK(check_stability(TDSE_RK4, 0, 0.1, 29.6, 0.0, 133.0, &th, &bd) == TDSE_E_UNSTABLE);
        CHECK(check_stability(TDSE_RK4, 0, 0.05, 29.6, 0.1, 133.0, &th, &bd) == TDSE_OK);
        CHECK(check_stability(TDSE_RK4, 0, 0.05, 29.6, -0.4, 133.0, &th, &bd) == TDSE_E_UNSTABLE);
        CHECK(check_stability(TDSE_LANCZOS, 12, 10.0, 29.6, 1.0, 133.0, &th, &bd) == TDSE_OK);
    }
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
