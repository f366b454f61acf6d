// Host-only checks of the library's argument validation, work split and
// dipole tile order.
// Built with g++ (no HIP) by tests/test_abi_cpu.py; prints one line per
// failed check and exits non-zero if any failed.
#include <math.h>
#include <stdio.h>

#include "tdse_split.h"
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
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
