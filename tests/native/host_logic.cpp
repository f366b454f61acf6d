// Host-only checks of the library's argument validation and work split.
// Built with g++ (no HIP) by tests/test_abi_cpu.py; prints one line per
// failed check and exits non-zero if any failed.
#include <math.h>
#include <stdio.h>

#include "tdse_split.h"
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
