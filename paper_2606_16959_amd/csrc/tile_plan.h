// Launch planning shared by the factor and operator APIs (host only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <tuple>
#include <vector>

#include "hs_internal.h"

namespace hs {
namespace plan {

inline int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= v) ++l;
    return l;
}

inline size_t elem_bytes(int dtype) { return dtype == HS_C128 ? 16 : 8; }

// Tile geometry for coupling hull [lb, hb) of bits.
struct Geo {
    int qb = 0, kb = 0, logW = 0, nlw_log = 0, T = 0;
    bool ok = false;
};

// LDS a tile may use: the compile-time budget, capped by the current
// device's per-workgroup limit (queried once).
inline int lds_budget() {
    static const int v = [] {
        int dev = 0, lim = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
            lim = 65536;
        return std::min(lim, (int)HS_TILE_LDS_MAX_BYTES);
    }();
    return v;
}

// Largest tile (rows) one launch of `batch` states over N rows uses: the
// kernel's capacity (closed or open launch), halved (down to 1024 rows) while
// the grid would have fewer than 256 tiles, one per compute unit.
inline int tile_rows_max(int dtype, int batch, long long N, bool open = false) {
    int T = tile_rows_cap(dtype == HS_C128, batch, open, lds_budget());
    while (T > 1024 && N / T < 256) T >>= 1;
    return T;
}

// Launch-plan tuning knobs, read from the environment at every evolve (a
// handle keeps one plan per batch size and knob setting): HAMSIM_WMIN_BYTES (shortest run of consecutive rows a
// strided tile may have, default 256), HAMSIM_MAX_FUSE (factors per launch,
// default 8), HAMSIM_PAIR_LDS (which closed complex64 launches whose every
// diagonal pairs run the pair kernel: 2 all, odd offsets of contiguous tiles
// included; 1 all except one-state strided launches whose row runs are
// under 1 KiB and whose diagonals are stored in natural order --
// translation-bound launches, where the row-by-row kernel measured faster;
// 0 none; same results; default 1),
// HAMSIM_XCD_SWIZZLE (which launches deal each XCD one contiguous
// eighth of the tiles instead of every eighth tile: 0 none, 1 all, 2 strided
// tiles only, 3 contiguous tiles only; default 3: strided launches of
// complex64 states measured 1-4% faster without it, contiguous ones faster
// with it).
inline int env_int(const char *name, int dflt, int lo, int hi) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    long x = std::strtol(v, &end, 10);
    if (end == v) return dflt;
    return (int)std::min<long>(hi, std::max<long>(lo, x));
}
struct PlanKey {
    int chunk, fuse, wmin_bytes, max_fuse, swizzle, pairs;
    bool operator<(const PlanKey &o) const {
        return std::tie(chunk, fuse, wmin_bytes, max_fuse, swizzle, pairs) <
               std::tie(o.chunk, o.fuse, o.wmin_bytes, o.max_fuse, o.swizzle, o.pairs);
    }
};
inline PlanKey plan_key(int chunk, bool fuse) {
    return PlanKey{chunk, fuse ? 1 : 0, env_int("HAMSIM_WMIN_BYTES", 256, 8, 1 << 20),
                   env_int("HAMSIM_MAX_FUSE", kMaxRun, 1, kMaxRun),
                   env_int("HAMSIM_XCD_SWIZZLE", 3, 0, 3), env_int("HAMSIM_PAIR_LDS", 1, 0, 2)};
}
// Whether a launch of geometry `g` deals contiguous eighths of its tiles to the XCDs.
inline bool swizzled(int mode, const Geo &g) {
    return mode == 1 || (mode == 2 && g.qb > 0) || (mode == 3 && g.qb == 0);
}
inline int w_min(int dtype, const PlanKey &k) { return std::max(1, k.wmin_bytes / (dtype == HS_C128 ? 16 : 8)); }

inline Geo geometry(int lb, int hb, int n, int Tmax) {
    Geo g;
    hb = std::min(hb, n);
    lb = std::min(lb, hb);
    const int logT = std::min(ilog2(Tmax), n);
    if (hb <= logT) {               // contiguous tile of 2^logT rows
        g.qb = 0; g.kb = logT; g.logW = 0; g.nlw_log = 0; g.T = 1 << logT; g.ok = true;
        return g;
    }
    // here lb >= 1, so logW = min(logT - kb, lb) is 0 only when kb == logT;
    // a thread owns two adjacent rows, so a strided tile needs W >= 2
    const int kb = hb - lb;
    if (kb >= logT) return g;
    g.qb = lb;
    g.kb = kb;
    g.logW = std::min(logT - kb, lb);
    g.nlw_log = lb - g.logW;
    g.T = 1 << (kb + g.logW);
    g.ok = true;
    return g;
}

// Geometry and descriptors of an open launch of an arbitrary operator
// (x and y distinct): stride the tile by the largest power of two dividing
// every offset when that keeps long row runs, else contiguous tiles.
inline Geo generic_geometry(const long long *offsets, int nd, long long N, int dtype, int chunk) {
    uint64_t orall = 0;
    long long maxabs = 0;
    for (int j = 0; j < nd; ++j) {
        const long long a = offsets[j] < 0 ? -offsets[j] : offsets[j];
        orall |= (uint64_t)a;
        maxabs = std::max(maxabs, a);
    }
    const int n = ilog2(N);
    const int Tmax = tile_rows_max(dtype, chunk, N, true);
    const PlanKey key = plan_key(chunk, true);
    const int q = orall ? __builtin_ctzll(orall) : 0;
    Geo geo = geometry(0, 0, n, Tmax);
    if (N < 2 || (N & (N - 1))) {
        // N not a power of two (or 1): contiguous tiles of the smallest power
        // of two >= N (at least one row pair, at most Tmax); the last tile is partial
        int lt = 1;
        while ((1ll << lt) < N && (2ll << lt) <= Tmax) ++lt;
        geo = Geo{};
        geo.kb = lt;
        geo.T = 1 << lt;
        geo.ok = true;
        return geo;
    }
    if (orall && (1 << std::min(q, 20)) >= w_min(dtype, key) && maxabs >= Tmax) {
        const int need = ilog2(maxabs >> q) + 1;     // levels reaching the farthest offset
        const int logT = std::min(ilog2(Tmax), n);
        const int kb = std::min(need + 1, logT - ilog2(w_min(dtype, key)));
        if (kb >= 1) {
            Geo g2 = geometry(q, q + kb, n, Tmax);
            if (g2.ok && g2.qb > 0) geo = g2;
        }
    }
    return geo;
}

inline void fill_descs(const long long *offsets, const void *const *ptrs, int nd, long long N, const Geo &geo,
                       std::vector<DiagDesc> &hd) {
    hd.resize(nd);
    for (int j = 0; j < nd; ++j) {
        const long long d = offsets[j];
        DiagDesc &dd = hd[j];
        dd = DiagDesc{};
        dd.ptr = ptrs[j];
        dd.off = (int32_t)d;
        const long long lowmask = (1ll << geo.qb) - 1;
        dd.regular = (d & lowmask) == 0;
        dd.m = dd.regular ? (int32_t)(d >> geo.qb) : 0;
        dd.lo = (int32_t)std::max<long long>(0, -d);
        dd.hi = (int32_t)std::min<long long>(N, N - d);
    }
}

// Whether launches over `chunk` states of N rows write with non-temporal stores.
inline int32_t stream_out(int chunk, long long N, int dtype) {
    return (size_t)chunk * (size_t)N * elem_bytes(dtype) >= kStreamOutBytes ? 1 : 0;
}

inline TileArgs open_args(const Geo &geo, const DiagDesc *ddev, int nd, const void *x, void *y, long long N) {
    TileArgs a{};
    a.y = y;
    a.x = x;
    a.stride = N;
    a.N = (int32_t)N;
    a.nf = 1;
    a.dstart[0] = 0;
    a.dstart[1] = nd;
    a.desc = ddev;
    a.qb = geo.qb; a.kb = geo.kb; a.logW = geo.logW; a.nlw_log = geo.nlw_log; a.T = geo.T;
    a.nrm2 = nullptr;
    a.viol = nullptr;
    a.swizzle = 0;
    a.ragged = (N % geo.T) != 0;
    a.stream_out = 0;
    a.pairs = 0;
    return a;
}

}  // namespace plan
}  // namespace hs
