// Storage order of the stored diagonals (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hs {

// Storage order of a stored diagonal of length len = N - |d|.  Entry i (the
// coefficient A[r, r + d] with i = min(r, r + d), Eq. 6) sits at
//   perm_pos(i) = ((i mod 2^s) >> c) * ((len >> s) << c) + ((i >> s) << c) + (i mod 2^c),
// that is, i's low s bits split into a chunk column (bits c..s-1) and a
// position in the chunk (bits 0..c-1), with every "level" i >> s of a column
// stored one chunk after the other.  s = c = 0 is the natural order
// (position i).  Requires len to be a multiple of 2^s, which holds when
// every offset of the factor is a multiple of 2^s.  A strided tile reads,
// per diagonal, all levels of a window of consecutive low rows; in this order
// those entries lie in one short run per chunk column instead of one run per
// level 2^s entries apart (one page-table entry each when 2^s entries span a
// page).  The positions are a permutation of [0, len): the diagonal keeps
// exactly N - |d| entries.
__host__ __device__ __forceinline__ int64_t perm_pos(int64_t i, int s, int c, int64_t clr) {
    return ((i & ((int64_t(1) << s) - 1)) >> c) * clr + ((i >> s) << c) + (i & ((int64_t(1) << c) - 1));
}
// The same in 32-bit arithmetic (tile kernels: N <= 2^30, positions < 2^30).
__host__ __device__ __forceinline__ int perm_pos32(int i, int s, int c, int clr) {
    return ((i & ((1 << s) - 1)) >> c) * clr + ((i >> s) << c) + (i & ((1 << c) - 1));
}

}  // namespace hs
