// Host checks of the tile shapes the launch planner and the kernels share
// (hs_internal.h): every (dtype, batch, closed/open) shape gives each tile
// row a thread and fits its LDS budget; closed complex64 launches of 5
// states use the CU's whole 160 KiB for 4096-row tiles, every other shape at
// most 128 KiB; closed complex128 launches of 2 states hold 4096 rows; and a
// device limit below the budget shrinks the tile instead.  Exits non-zero on
// a failure.
#include <cstdio>

#include "../../paper_2606_16959_amd/csrc/hs_internal.h"

static int failures = 0;

static void expect(bool ok, const char *what, int c128, int batch, int open, long long got) {
    if (!ok) {
        std::printf("FAIL %s c128=%d batch=%d open=%d got=%lld\n", what, c128, batch, open, got);
        ++failures;
    }
}

int main() {
    int cases = 0;
    for (int c128 = 0; c128 <= 1; ++c128)
        for (int open = 0; open <= 1; ++open)
            for (int batch = 1; batch <= 8; ++batch) {
                const int esz = c128 ? 16 : 8;
                const int rows = hs::tile_threads(c128, batch, open) * hs::tile_rpt(c128, batch, open);
                const int T = hs::tile_rows_cap(c128, batch, open);
                const int budget = hs::tile_lds_bytes(c128, batch, open);
                expect(T >= 2 && (T & (T - 1)) == 0, "tile rows a power of two", c128, batch, open, T);
                expect(T <= rows, "every tile row has a thread", c128, batch, open, T);
                expect((long long)T * batch * esz <= budget, "tile fits its LDS budget", c128, batch, open,
                       (long long)T * batch * esz);
                expect(budget == ((!c128 && !open && batch == 5) ? 163840 : 131072), "LDS budget", c128, batch,
                       open, budget);
                expect(hs::tile_rpt(c128, batch, open) % 2 == 0, "rows come in pairs", c128, batch, open,
                       hs::tile_rpt(c128, batch, open));
                // a device limit of 128 KiB per workgroup halves the 5-state tile
                const int T128 = hs::tile_rows_cap(c128, batch, open, 131072);
                expect(T128 <= T && (long long)T128 * batch * esz <= 131072, "128 KiB device limit", c128, batch,
                       open, T128);
                ++cases;
            }
    // the shapes the performance record depends on
    expect(hs::tile_rows_cap(false, 1) == 8192, "complex64, 1 state", 0, 1, 0, hs::tile_rows_cap(false, 1));
    expect(hs::tile_rows_cap(false, 4) == 4096, "complex64, 4 states", 0, 4, 0, hs::tile_rows_cap(false, 4));
    expect(hs::tile_rows_cap(false, 5) == 4096, "complex64, 5 states", 0, 5, 0, hs::tile_rows_cap(false, 5));
    expect(hs::tile_rows_cap(false, 5, false, 131072) == 2048, "complex64, 5 states, 128 KiB", 0, 5, 0,
           hs::tile_rows_cap(false, 5, false, 131072));
    for (int b = 6; b <= 8; ++b)
        expect(hs::tile_rows_cap(false, b) == 2048, "complex64, 6-8 states", 0, b, 0, hs::tile_rows_cap(false, b));
    expect(hs::tile_rows_cap(true, 1) == 4096, "complex128, 1 state", 1, 1, 0, hs::tile_rows_cap(true, 1));
    expect(hs::tile_rows_cap(true, 2) == 4096, "complex128, 2 states", 1, 2, 0, hs::tile_rows_cap(true, 2));
    expect(hs::tile_rows_cap(true, 4) == 2048, "complex128, 4 states", 1, 4, 0, hs::tile_rows_cap(true, 4));
    expect(hs::tile_rows_cap(true, 8) == 1024, "complex128, 8 states", 1, 8, 0, hs::tile_rows_cap(true, 8));
    if (failures) return 1;
    std::printf("%d shapes checked\n", cases);
    return 0;
}
