// Host checks of the level-major chunk order of stored diagonals
// (storage_order.h): for every small N = 2^n, split bit s, chunk bits c and
// offset d that is a multiple of 2^s, the positions of the N - |d| entries
// are a permutation of [0, N - |d|) (checked against the inverse map written
// from the layout's description: column, level, place in the chunk); an even
// entry and its successor stay adjacent; s = c = 0 is the identity; and the
// entries a strided tile reads (every level of a window of rows) fall into
// one contiguous stretch per chunk column.  Exits non-zero on a failure.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../paper_2606_16959_amd/csrc/storage_order.h"

static int fail(const char *what, int n, int s, int c, long long d) {
    std::printf("FAIL %s n=%d s=%d c=%d d=%lld\n", what, n, s, c, d);
    return 1;
}

int main() {
    long long cases = 0;
    for (int n = 1; n <= 12; ++n) {
        const int64_t N = int64_t(1) << n;
        for (int s = 0; s <= n; ++s)
            for (int c = (s ? 1 : 0); c <= s; ++c) {
                if (s == 0 && c != 0) continue;
                for (int64_t m = -((N - 1) >> s); m <= ((N - 1) >> s); ++m) {
                    const int64_t d = m << s;
                    const int64_t len = N - (d < 0 ? -d : d);
                    const int64_t clr = (len >> s) << c;
                    std::vector<int> seen(len, 0);
                    for (int64_t i = 0; i < len; ++i) {
                        const int64_t p = hs::perm_pos(i, s, c, clr);
                        if (p < 0 || p >= len || seen[p]++) return fail("not a permutation", n, s, c, d);
                        if (hs::perm_pos32((int)i, s, c, (int)clr) != p) return fail("32-bit form differs", n, s, c, d);
                        if (s == 0 && p != i) return fail("natural order is not the identity", n, s, c, d);
                        if ((i & 1) == 0 && i + 1 < len && c >= 1 && hs::perm_pos(i + 1, s, c, clr) != p + 1)
                            return fail("pair split", n, s, c, d);
                    }
                    if (s > 0) {
                        // inverse: position q = column * clr + level * 2^c + k holds
                        // entry i = level * 2^s + column * 2^c + k
                        const int64_t C = int64_t(1) << c;
                        for (int64_t q = 0; q < len; ++q) {
                            const int64_t col = q / clr, rem = q % clr;
                            const int64_t i = ((rem / C) << s) + (col << c) + (rem % C);
                            if (hs::perm_pos(i, s, c, clr) != q) return fail("inverse", n, s, c, d);
                        }
                        // a tile of all levels over a window of W = 2^c rows starting at w0
                        // (a multiple of W) reads entries level * 2^s + w0 + j: one stretch
                        for (int64_t w0 = 0; w0 < (int64_t(1) << s); w0 += C) {
                            int64_t lo = -1, cnt = 0;
                            for (int64_t lev = 0; lev < (len >> s); ++lev)
                                for (int64_t j = 0; j < C; ++j) {
                                    const int64_t p = hs::perm_pos((lev << s) + w0 + j, s, c, clr);
                                    if (lo < 0) lo = p;
                                    if (p != lo + cnt) return fail("tile window not contiguous", n, s, c, d);
                                    ++cnt;
                                }
                        }
                    }
                    ++cases;
                }
            }
    }
    std::printf("storage order: %lld cases checked\n", cases);
    return 0;
}
