// Host AddressSanitizer / UBSan run of libplbm's host layer (coefficient
// table, descriptor defaults, validation, sizes, status strings) on valid,
// degenerate and hostile inputs.  Exit status 0: no sanitizer report and
// every documented outcome observed.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "plbm.h"
#include "plbm_internal.h"

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { std::fprintf(stderr, "expectation failed: %s line %d\n", #c, __LINE__); ++fails; } } while (0)

static unsigned rnd(unsigned &s)
{
    s = s * 1664525u + 1013904223u;
    return s >> 8;
}

int main()
{
    double c[PLBM_MAX_Q1D * PLBM_MAX_Q1D];
    // coefficient table: valid sets of every size, duplicates, non-finite, bad q
    const double v[8] = {0, 1, -1, 3, -3, 2, -2, 5};
    for (int q = 1; q <= PLBM_MAX_Q1D; ++q) EXPECT(plbm_coeffs(q, v, c) == PLBM_OK);
    const double dup[3] = {1, 1, 0};
    EXPECT(plbm_coeffs(3, dup, c) == PLBM_ESINGULAR);
    const double nanv[2] = {0, std::numeric_limits<double>::quiet_NaN()};
    EXPECT(plbm_coeffs(2, nanv, c) == PLBM_EINVAL);
    EXPECT(plbm_coeffs(0, v, c) == PLBM_EINVAL && plbm_coeffs(9, v, c) == PLBM_EINVAL);
    EXPECT(plbm_coeffs(3, nullptr, c) == PLBM_EINVAL && plbm_coeffs(3, v, nullptr) == PLBM_EINVAL);
    const double close[2] = {0, 1e-300};
    (void)plbm_coeffs(2, close, c);                 // any status, no fault
    // descriptors
    plbm_desc d;
    EXPECT(plbm_desc_default(&d, 2, 64, 48, 1.5, PLBM_F32) == PLBM_OK);
    EXPECT(plbm_buffer_elems(&d) == (size_t)25 * 64 * 48 && plbm_elem_bytes(&d) == 4);
    EXPECT(plbm_desc_default(&d, 3, 16, 12, 1.5, PLBM_F64) == PLBM_OK && d.nz == 12);
    EXPECT(plbm_desc_default(&d, 1, 1 << 30, 1, 1.0, PLBM_F64) == PLBM_OK);
    EXPECT(plbm_desc_default(&d, 1, (1 << 30) + 1, 1, 1.0, PLBM_F64) != PLBM_OK);
    EXPECT(plbm_desc_default(nullptr, 2, 8, 8, 1.0, PLBM_F64) == PLBM_EINVAL);
    EXPECT(plbm_buffer_elems(nullptr) == 0 && plbm_elem_bytes(nullptr) == 0);
    // hostile descriptors: random fields must validate or be refused, never fault
    unsigned s = 12345u;
    int ok = 0;
    for (int it = 0; it < 200000; ++it) {
        plbm_desc e;
        plbm_desc_default(&e, 2, 64, 64, 1.5, PLBM_F64);
        switch (rnd(s) % 10) {
        case 0: e.dim = (int)(rnd(s) % 7) - 2; break;
        case 1: e.nx = (int)rnd(s) - (1 << 23); break;
        case 2: e.ny = (int)(rnd(s) % 100000) - 10; break;
        case 3: e.q1d = (int)(rnd(s) % 12) - 2; break;
        case 4: e.storage = (int)(rnd(s) % 7) - 2; break;
        case 5: e.v[rnd(s) % PLBM_MAX_Q1D] = (double)((int)(rnd(s) % 13) - 6) * 0.5; break;
        case 6: e.omega = (double)((int)(rnd(s) % 50) - 10) / 10.0; break;
        case 7: e.nz = (int)(rnd(s) % 9) - 2; e.dim = 3; break;
        case 8: e.bc = (int)(rnd(s) % 4) - 1; break;
        default: e.c[rnd(s) % 64] = std::numeric_limits<double>::infinity(); break;
        }
        if (plbm::validate(&e) == PLBM_OK) {
            ++ok;
            const size_t n = plbm_buffer_elems(&e);
            EXPECT(n > 0 && plbm_elem_bytes(&e) > 0);
        } else {
            EXPECT(plbm_buffer_elems(&e) == 0);
        }
    }
    EXPECT(ok > 1000);
    for (int st = -10; st <= 2; ++st) EXPECT(plbm_strerror(st) != nullptr);
    if (fails) std::fprintf(stderr, "%d failures\n", fails);
    return fails ? 1 : 0;
}
