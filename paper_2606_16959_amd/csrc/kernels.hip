// HIP kernels for gfx950 (MI355X): factor construction, the DIA tile kernel
// (single factor or a fused run of factors), the single-diagonal kernel and
// the FP64 reductions.  The state update is bandwidth-bound (about one
// complex FMA per stored coefficient), so nothing here uses MFMA; the
// kernels are built around coalesced 8/16-byte streams along each diagonal,
// LDS staging of the state tile and wave64 shuffle reductions.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "hs_internal.h"
#include "storage_order.h"

namespace hs {

template <typename R>
struct alignas(2 * sizeof(R)) C2 {
    R re, im;
};

// acc += c * x, in a fixed order of fused multiply-adds (the same in every
// kernel, so results do not depend on which kernel or batch size ran).
__device__ __forceinline__ void cfma(C2<float> &acc, C2<float> c, C2<float> x) {
    acc.re = __builtin_fmaf(c.re, x.re, acc.re);
    acc.re = __builtin_fmaf(-c.im, x.im, acc.re);
    acc.im = __builtin_fmaf(c.re, x.im, acc.im);
    acc.im = __builtin_fmaf(c.im, x.re, acc.im);
}
__device__ __forceinline__ void cfma(C2<double> &acc, C2<double> c, C2<double> x) {
    acc.re = __builtin_fma(c.re, x.re, acc.re);
    acc.re = __builtin_fma(-c.im, x.im, acc.re);
    acc.im = __builtin_fma(c.re, x.im, acc.im);
    acc.im = __builtin_fma(c.im, x.re, acc.im);
}

template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> v, R s) {
    return C2<R>{v.re * s, v.im * s};
}

// nrm2 points at the squared norm of state 0 inside [batch][4] reduction
// records (state b at nrm2[4 b]); null means no rescaling.
template <typename R>
__device__ __forceinline__ R inv_norm(const double *nrm2, int b) {
    return nrm2 ? (R)(1.0 / sqrt(nrm2[4 * b])) : (R)1;
}

// ------------------------------------------------------------ construction

// E(x) = sum_k c_k (-1)^{popcount(x & z_k)};  out[x] = exp(-i dt E(x)), FP64.
__global__ void phase_table_kernel(int64_t N, int nz, const uint64_t *__restrict__ zm,
                                   const double *__restrict__ cf, double dt,
                                   double *__restrict__ out) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < N;
         x += (int64_t)gridDim.x * blockDim.x) {
        double E = 0.0;
        for (int k = 0; k < nz; ++k) E += cf[k] * ((__popcll((uint64_t)x & zm[k]) & 1) ? -1.0 : 1.0);
        double s, c;
        sincos(-dt * E, &s, &c);
        out[2 * x] = c;
        out[2 * x + 1] = s;
    }
}

// One diagonal per blockIdx.y.  Entry i of diagonal d sits at row r = i - min(d, 0),
// column p = r + d.  Value: L[loc(r), loc(p)] (times D[p]) when r and p agree
// outside the support, else exactly 0; computed in FP64, stored as R at the
// entry's position in the factor's storage order (perm_pos).
template <typename R>
__global__ void construct_kernel(ConstructArgs a) {
    const int j = blockIdx.y;
    const int64_t d = a.offs[j];
    const int64_t len = (int64_t)a.N - (d < 0 ? -d : d);
    const int64_t neg = d < 0 ? d : 0;
    const int64_t clr = (len >> a.perm_s) << a.perm_c;
    C2<R> *out = reinterpret_cast<C2<R> *>(a.base) + a.elem_off[j];
    const uint64_t outside = ~(uint64_t)a.smask;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i - neg, p = r + d;
        double vr = 0.0, vi = 0.0;
        if (a.L == nullptr) {
            if (r == p) vr = 1.0;
        } else if ((((uint64_t)(r ^ p)) & outside) == 0) {
            uint32_t la = 0, lb = 0;
            if (a.contiguous) {
                la = (uint32_t)(r >> a.lb) & (uint32_t)(a.K - 1);
                lb = (uint32_t)(p >> a.lb) & (uint32_t)(a.K - 1);
            } else {
                for (int q = 0; q < a.nbits; ++q) {
                    la |= (uint32_t)((r >> a.bits[q]) & 1) << q;
                    lb |= (uint32_t)((p >> a.bits[q]) & 1) << q;
                }
            }
            const int64_t e = (int64_t)la * a.K + lb;
            vr = a.L[2 * e];
            vi = a.L[2 * e + 1];
        }
        if (a.phase && (vr != 0.0 || vi != 0.0)) {
            const double pr = a.phase[2 * p], pi = a.phase[2 * p + 1];
            const double tr = vr * pr - vi * pi;
            const double ti = vr * pi + vi * pr;
            vr = tr;
            vi = ti;
        }
        out[perm_pos(i, a.perm_s, a.perm_c, clr)] = C2<R>{(R)vr, (R)vi};
    }
}

// dst[k] = entry start + k of a diagonal stored in the order (s, c)
template <typename R>
__global__ void perm_gather_kernel(const C2<R> *__restrict__ src, C2<R> *__restrict__ dst, int64_t start,
                                   int64_t count, int64_t len, int s, int c) {
    const int64_t clr = (len >> s) << c;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[perm_pos(start + k, s, c, clr)];
}

// ------------------------------------------------------------ DIA tile kernel
//
// A workgroup owns one tile of T = 2^kb * W rows:
//   row(i) = hi * 2^(qb+kb) + (i >> logW) * 2^qb + lw * W + (i & (W-1)),
// i.e. all 2^kb "levels" of the bits [qb, qb+kb) times a window of W
// consecutive low rows (contiguous tiles: qb = 0, W = 1, T = 2^kb).
// The state rows of the tile (all B states) are staged once into LDS with
// coalesced loads.  Every row then sums, in ascending-offset order, the stored
// coefficient of each diagonal times the partner amplitude x[r + d]: from LDS
// when the partner row lies in the tile, else (open launches) from global
// memory if the coefficient is nonzero.  Every stored coefficient is read
// exactly once, by the thread that owns its row, along the diagonal in
// consecutive addresses.
//
// A thread owns pairs of adjacent rows (local indices i, i+1 with i even;
// a strided tile has an even W and a contiguous one W = 1 with qb = 0, so
// the two rows are adjacent in the state too).  For an
// even offset the two coefficients are adjacent and 16-byte aligned
// (diagonals start on 256-byte boundaries), so complex64 pairs are fetched
// with one 16-byte load; odd offsets use two 8-byte loads.  Loads are issued
// for all pairs of a diagonal before any is consumed, with clamped indices and
// masks instead of branches, so a wave keeps many loads in flight.
//
// Closed launches (factors built by this library, whose nonzeros only couple
// rows inside one tile) run in place and do not read outside the tile: a
// nonzero out-of-tile coefficient only raises the violation flag.  A fused
// launch applies several factors in turn on the tile held in LDS.

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) f2v g_f2;
typedef const __attribute__((address_space(1))) f4v g_f4;
typedef const __attribute__((address_space(1))) d2v g_d2;

#ifndef HS_TILE_NT
#define HS_TILE_NT 1          // streaming (non-temporal) hint on coefficient and state loads
#endif
#if HS_TILE_NT
#define HS_LOAD(ptr) __builtin_nontemporal_load(ptr)
#else
#define HS_LOAD(ptr) (*(ptr))
#endif

// Single entries (odd offsets: the two rows of a pair read halves of the
// same 16-byte granule, so these loads keep the default cache policy and the
// second one hits in L2).
__device__ __forceinline__ C2<float> ld1(const C2<float> *p, int i) {
    const f2v v = *((g_f2 *)(p) + i);
    return C2<float>{v.x, v.y};
}
__device__ __forceinline__ C2<double> ld1(const C2<double> *p, int i) {
    const d2v v = HS_LOAD((g_d2 *)(p) + i);
    return C2<double>{v.x, v.y};
}
// entries i and i+1 (i even)
__device__ __forceinline__ void ld2(const C2<float> *p, int i, C2<float> &a, C2<float> &b) {
    const f4v v = HS_LOAD((g_f4 *)(p) + (i >> 1));
    a = C2<float>{v.x, v.y};
    b = C2<float>{v.z, v.w};
}
__device__ __forceinline__ void ld2(const C2<double> *p, int i, C2<double> &a, C2<double> &b) {
    a = ld1(p, i);
    b = ld1(p, i + 1);
}
// entries i and i + 1 for any i (8-byte aligned 16-byte load)
typedef float f4u __attribute__((ext_vector_type(4))) __attribute__((aligned(8)));
typedef const __attribute__((address_space(1))) f4u g_f4u;
__device__ __forceinline__ void ld2u(const C2<float> *p, int i, C2<float> &a, C2<float> &b) {
    const f4u v = HS_LOAD((g_f4u *)(p + i));
    a = C2<float>{v.x, v.y};
    b = C2<float>{v.z, v.w};
}

typedef __attribute__((address_space(1))) f4v g_f4w;
typedef __attribute__((address_space(1))) d2v g_d2w;
// one complex128 row of an output state (STREAM: non-temporal)
template <bool STREAM>
__device__ __forceinline__ void st1(C2<double> *p, int i, C2<double> a) {
    const d2v u = {a.re, a.im};
    if (STREAM) __builtin_nontemporal_store(u, (g_d2w *)(p) + i);
    else *((g_d2w *)(p) + i) = u;
}
// rows i and i + 1 (i even) of an output state: one 16-byte store for
// complex64, two for complex128; STREAM streams them past the caches (a
// compile-time choice: with a run-time branch the compiler merges the two
// stores and drops the hint)
template <bool STREAM>
__device__ __forceinline__ void st2(C2<float> *p, int i, C2<float> a, C2<float> b) {
    const f4v v = {a.re, a.im, b.re, b.im};
    if (STREAM) __builtin_nontemporal_store(v, (g_f4w *)(p) + (i >> 1));
    else *((g_f4w *)(p) + (i >> 1)) = v;
}
template <bool STREAM>
__device__ __forceinline__ void st2(C2<double> *p, int i, C2<double> a, C2<double> b) {
    const d2v u = {a.re, a.im}, v = {b.re, b.im};
    if (STREAM) {
        __builtin_nontemporal_store(u, (g_d2w *)(p) + i);
        __builtin_nontemporal_store(v, (g_d2w *)(p) + i + 1);
    } else {
        *((g_d2w *)(p) + i) = u;
        *((g_d2w *)(p) + i + 1) = v;
    }
}

// State rows staged by open launches keep the default cache policy: other
// tiles read them again as out-of-tile partners, and those reads should hit.
__device__ __forceinline__ void ld2_cached(const C2<float> *p, int i, C2<float> &a, C2<float> &b) {
    const f4v v = *((g_f4 *)(p) + (i >> 1));
    a = C2<float>{v.x, v.y};
    b = C2<float>{v.z, v.w};
}
__device__ __forceinline__ C2<double> ld1_cached(const C2<double> *p, int i) {
    const d2v u = *((g_d2 *)(p) + i);
    return C2<double>{u.x, u.y};
}
__device__ __forceinline__ void ld2_cached(const C2<double> *p, int i, C2<double> &a, C2<double> &b) {
    const d2v u = *((g_d2 *)(p) + i);
    const d2v v = *((g_d2 *)(p) + i + 1);
    a = C2<double>{u.x, u.y};
    b = C2<double>{v.x, v.y};
}

// wave64 butterfly sum (fixed order)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R>
__device__ __forceinline__ C2<R> cmask(C2<R> c, bool keep) {
    return keep ? c : C2<R>{(R)0, (R)0};
}

#ifndef HS_TILE_PF_ACC
#define HS_TILE_PF_ACC 3       // registers counted per accumulator register in tile_pf's estimate
#endif
#ifndef HS_TILE_INFLIGHT
#define HS_TILE_INFLIGHT 8     // coefficient pair loads a thread keeps outstanding (complex64; half for complex128)
#endif

// Diagonals whose coefficients a thread keeps in flight.  A thread of one or
// two row pairs (large batches, small tiles) would otherwise wait on a single
// short load per diagonal; it keeps about HS_TILE_INFLIGHT pair loads
// outstanding (half as many for complex128), cut while an estimate of the
// kernel's registers (a fixed part, per-pair indexing, the accumulators and
// the buffers) would pass what NT threads per workgroup leave each thread.
// Threads with more pairs already have enough loads per diagonal.
template <typename R>
constexpr int tile_pf(int B, int P, int NT) {
    const int wc = (int)sizeof(R) / 2;                  // VGPRs per complex value
    const int budget = (NT >= 1024 ? 128 : 256) - 8;
    const int inflight = sizeof(R) == 8 ? HS_TILE_INFLIGHT / 2 : HS_TILE_INFLIGHT;
    int pf = P <= 2 && inflight / P > 1 ? inflight / P : 1;
    while (pf > 1 && 40 + 14 * P + HS_TILE_PF_ACC * P * B * wc + 2 * pf * P * wc > budget) --pf;
    return pf;
}

// Coefficients of one diagonal for every row pair a thread owns (masked
// loads: invalid rows read entry 0 and are zeroed when consumed).  PERM: the
// diagonal may be stored out of natural order (perm_pos with its ps, pc; an
// even entry and its successor stay adjacent, so pairs are still one load).
template <typename R, int P, int NT, bool SINGLE = false, bool PERM = false>
__device__ __forceinline__ void load_diag(C2<R> (&c)[P][2], const DiagDesc &dd, int tid, int T,
                                          int base, int qb, int logW) {
    const C2<R> *cp = reinterpret_cast<const C2<R> *>(dd.ptr);
    const int neg = dd.off < 0 ? dd.off : 0;
    const int len = dd.hi - dd.lo;            // N - |d| entries
    const int W = 1 << logW;
    if constexpr (sizeof(R) == 8) {
        // complex128: the rows of pair p are (2p + k) NT + tid (tile_lidx), one
        // 16-byte load each
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = (2 * p + k) * NT + tid;
                int e = base + ((i >> logW) << qb) + (i & (W - 1)) + neg;
                e = (e >= 0 && e < len && i < T) ? e : 0;
                if (PERM) e = perm_pos32(e, dd.ps, dd.pc, dd.plr);
                c[p][k] = ld1(cp, e);
            }
        return;
    }
    // SINGLE: entry-wise loads (a diagonal of odd length ends inside a pair)
    if (!SINGLE && (dd.off & 1) == 0) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            const int r0 = base + ((i0 >> logW) << qb) + (i0 & (W - 1));
            int e = r0 + neg;
            e = (e >= 0 && e < len && i0 < T) ? e : 0;   // even d: pairs never straddle lo/hi
            if (PERM) e = perm_pos32(e, dd.ps, dd.pc, dd.plr);
            ld2(cp, e, c[p][0], c[p][1]);
        }
    } else {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            const int r0 = base + ((i0 >> logW) << qb) + (i0 & (W - 1));
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                int e = r0 + k + neg;
                e = (e >= 0 && e < len && i0 < T) ? e : 0;
                if (PERM) e = perm_pos32(e, dd.ps, dd.pc, dd.plr);
                c[p][k] = ld1(cp, e);
            }
        }
    }
}

// HORNER (open launches only): the output row is x0[r] + alpha * (A x)[r],
// one Horner stage of a polynomial in A applied to a state.
// RAG (open contiguous launches only): N need not be a multiple of the tile;
// rows at or past N are neither loaded nor stored.
// STREAM (not with RAG): the output is written with non-temporal stores.
// PERM (closed launches only): some diagonals are stored out of natural
// order (perm_pos); the others carry ps = pc = 0.
template <typename R, int B, int RPT, bool CLOSED, bool HORNER = false, int NT = kTileThreads, bool RAG = false,
          bool STREAM = false, bool PERM = false>
__global__ __launch_bounds__(NT) void dia_tile_kernel(TileArgs a) {
    static_assert(!PERM || (CLOSED && !RAG && !HORNER), "out-of-order storage only in closed launches");
    static_assert(RPT % 2 == 0, "rows come in pairs");
    constexpr int P = RPT / 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<R> *lds = reinterpret_cast<C2<R> *>(smem_raw);
    const int T = a.T;
    const int tid = threadIdx.x;
    const int qb = a.qb, kb = a.kb, logW = a.logW;
    const int W = 1 << logW;
    const int L = 1 << kb;
    int blk = blockIdx.x;
    if (a.swizzle && (gridDim.x & 7) == 0) {
        // workgroups are dealt to the 8 XCDs round-robin: give each XCD one
        // contiguous eighth of the tiles
        blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
    }
    const int hi = blk >> a.nlw_log;
    const int lw = blk & ((1 << a.nlw_log) - 1);
    const int base = (hi << (qb + kb)) | (lw << logW);
    const C2<R> *x = reinterpret_cast<const C2<R> *>(a.x);  // may alias y (in place)
    C2<R> *y = reinterpret_cast<C2<R> *>(a.y);

    R scale[B];
#pragma unroll
    for (int b = 0; b < B; ++b) scale[b] = inv_norm<R>(a.nrm2, b);

    // Local index of row k (0 or 1) of the thread's pair p.  complex64: two
    // adjacent rows, i0 = 2 tid + 2 NT p and i0 + 1 (one 16-byte load or store
    // for both); complex128: rows (2p + k) NT + tid, so that each 16-byte
    // load, store and LDS access of a wave covers consecutive addresses
    // (adjacent rows would give every instruction half of each cache line).
    constexpr bool SPLIT = sizeof(R) == 8;
    auto lidx = [&](int p, int k) { return SPLIT ? (2 * p + k) * NT + tid : 2 * tid + 2 * NT * p + k; };
    auto row_of = [&](int i) { return base + ((i >> logW) << qb) + (i & (W - 1)); };

    // stage the tile: issue every load, then write LDS
    {
        C2<R> u[P][2][B];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if constexpr (SPLIT) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int i = lidx(p, k);
                    const int r = i < T ? row_of(i) : base;
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        if (RAG) u[p][k][b] = r < a.N ? x[b * a.stride + r] : C2<R>{(R)0, (R)0};
                        else if (CLOSED) u[p][k][b] = ld1(x + b * a.stride, r);
                        else u[p][k][b] = ld1_cached(x + b * a.stride, r);
                    }
                }
                continue;
            }
            const int i0 = lidx(p, 0);
            const int r0 = i0 < T ? row_of(i0) : base;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (RAG) {
                    const C2<R> z{(R)0, (R)0};
                    u[p][0][b] = r0 < a.N ? x[b * a.stride + r0] : z;
                    u[p][1][b] = r0 + 1 < a.N ? x[b * a.stride + r0 + 1] : z;
                } else if (CLOSED) {
                    ld2(x + b * a.stride, r0, u[p][0][b], u[p][1][b]);
                } else {
                    ld2_cached(x + b * a.stride, r0, u[p][0][b], u[p][1][b]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = lidx(p, k);
                if (i < T)
#pragma unroll
                    for (int b = 0; b < B; ++b) lds[b * T + i] = cscale(u[p][k][b], scale[b]);
            }
    }

    // Coefficients of PF consecutive diagonals are in flight at once: after
    // buffer u is consumed for diagonal j it is refilled with diagonal j + PF,
    // across factor boundaries (coefficient loads do not depend on the tile).
    // Threads with few row pairs (large batches) keep about HS_TILE_INFLIGHT
    // 16-byte pair loads outstanding instead of one per diagonal.
    constexpr int PF = CLOSED ? tile_pf<R>(B, P, NT) : 1;
    const int total = a.dstart[a.nf];
    C2<R> acc[P][2][B];
    bool viol = false;
    auto clear_acc = [&]() {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int b = 0; b < B; ++b) acc[p][k][b] = C2<R>{(R)0, (R)0};
    };
    // acc += (diagonal dd) x (tile in LDS), row by row
    auto apply = [&](const C2<R> (&cc)[P][2], const DiagDesc &dd) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int r0 = row_of(lidx(p, 0));
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = lidx(p, k);
                const int r = SPLIT ? row_of(i) : r0 + k;
                const bool valid = i < T && r >= dd.lo && r < dd.hi;
                const C2<R> cv = cmask(cc[p][k], valid);
                bool in;
                int loc;
                if (dd.regular) {
                    const int lvl = (i >> logW) + dd.m;
                    in = (unsigned)lvl < (unsigned)L;
                    loc = i + dd.m * W;
                } else {
                    const int pr = r + dd.off;
                    in = (pr >> (qb + kb)) == hi && ((pr & ((1 << qb) - 1)) >> logW) == lw;
                    loc = (((pr >> qb) & (L - 1)) << logW) | (pr & (W - 1));
                }
                const bool nz = cv.re != (R)0 || cv.im != (R)0;
                const int sl = in ? loc : (i < T ? i : 0);
                const C2<R> ce = cmask(cv, in);
#pragma unroll
                for (int b = 0; b < B; ++b) cfma(acc[p][k][b], ce, lds[b * T + sl]);
                if (!in && nz) {
                    if (CLOSED) {
                        viol = true;
                    } else {
                        const int pr = r + dd.off;
#pragma unroll
                        for (int b = 0; b < B; ++b)
                            cfma(acc[p][k][b], cv, cscale(x[b * a.stride + pr], scale[b]));
                    }
                }
            }
        }
    };
    // the finished factor's output becomes the next factor's input tile
    auto acc_to_lds = [&]() {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = lidx(p, k);
                if (i < T)
#pragma unroll
                    for (int b = 0; b < B; ++b) lds[b * T + i] = acc[p][k][b];
            }
        __syncthreads();
    };

    // Open launches: a row whose partner lies outside the tile gathers it
    // from global memory.  For complex64 launches of one or two states the
    // gathers of G row pairs are issued before any is used (the gathered
    // values take 8 registers), so their latencies overlap; each row still
    // adds its LDS term first and its gathered term second, as the
    // one-row-at-a-time order would.  Other open launches have no registers
    // to spare (open complex128 and larger batches run at the 128-register
    // limit of 1024-thread workgroups) and gather row by row in the loop below.
    constexpr int kGather = sizeof(R) == 8 ? 0 : 8 / (2 * B * 2);
    constexpr int G = kGather >= P ? P : (kGather >= 1 ? kGather : 1);
    auto apply_open = [&](const C2<R> (&cc)[P][2], const DiagDesc &dd) {
#pragma unroll
        for (int g0 = 0; g0 < P; g0 += G) {
            C2<R> gv[G][2][B];
            C2<R> gc[G][2];
            bool gn[G][2];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const int p = g0 + q;
                const int r0 = row_of(lidx(p, 0));
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int i = lidx(p, k);
                    const int r = SPLIT ? row_of(i) : r0 + k;
                    const bool valid = i < T && r >= dd.lo && r < dd.hi;
                    const C2<R> cv = cmask(cc[p][k], valid);
                    bool in;
                    int loc;
                    if (dd.regular) {
                        const int lvl = (i >> logW) + dd.m;
                        in = (unsigned)lvl < (unsigned)L;
                        loc = i + dd.m * W;
                    } else {
                        const int pr = r + dd.off;
                        in = (pr >> (qb + kb)) == hi && ((pr & ((1 << qb) - 1)) >> logW) == lw;
                        loc = (((pr >> qb) & (L - 1)) << logW) | (pr & (W - 1));
                    }
                    const bool nz = cv.re != (R)0 || cv.im != (R)0;
                    const int sl = in ? loc : (i < T ? i : 0);
                    const C2<R> ce = cmask(cv, in);
#pragma unroll
                    for (int b = 0; b < B; ++b) cfma(acc[p][k][b], ce, lds[b * T + sl]);
                    gn[q][k] = !in && nz;
                    gc[q][k] = cv;
                    if (gn[q][k]) {
                        const int pr = r + dd.off;
#pragma unroll
                        for (int b = 0; b < B; ++b) gv[q][k][b] = x[b * a.stride + pr];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    if (gn[q][k])
#pragma unroll
                        for (int b = 0; b < B; ++b)
                            cfma(acc[g0 + q][k][b], gc[q][k], cscale(gv[q][k][b], scale[b]));
        }
    };

    if constexpr (PF == 1) {
        // The next diagonal's coefficients are loaded once this one's are
        // used.  The body is `apply` written out: this form compiles to the
        // code the one-state kernels were tuned and profiled with (the lambda
        // form schedules slightly differently).
        C2<R> c[P][2];
        load_diag<R, P, NT, RAG, PERM>(c, a.desc[0], tid, T, base, qb, logW);
        __syncthreads();
        int dj = 0;
        for (int f = 0; f < a.nf; ++f) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int b = 0; b < B; ++b) acc[p][k][b] = C2<R>{(R)0, (R)0};
            for (; dj < a.dstart[f + 1]; ++dj) {
                const DiagDesc dd = a.desc[dj];
                if constexpr (!CLOSED && kGather > 0) {
                    apply_open(c, dd);
                } else {
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const int r0 = row_of(lidx(p, 0));
#pragma unroll
                        for (int k = 0; k < 2; ++k) {
                            const int i = lidx(p, k);
                            const int r = SPLIT ? row_of(i) : r0 + k;
                            const bool valid = i < T && r >= dd.lo && r < dd.hi;
                            const C2<R> cv = cmask(c[p][k], valid);
                            bool in;
                            int loc;
                            if (dd.regular) {
                                const int lvl = (i >> logW) + dd.m;
                                in = (unsigned)lvl < (unsigned)L;
                                loc = i + dd.m * W;
                            } else {
                                const int pr = r + dd.off;
                                in = (pr >> (qb + kb)) == hi && ((pr & ((1 << qb) - 1)) >> logW) == lw;
                                loc = (((pr >> qb) & (L - 1)) << logW) | (pr & (W - 1));
                            }
                            const bool nz = cv.re != (R)0 || cv.im != (R)0;
                            const int sl = in ? loc : (i < T ? i : 0);
                            const C2<R> ce = cmask(cv, in);
#pragma unroll
                            for (int b = 0; b < B; ++b) cfma(acc[p][k][b], ce, lds[b * T + sl]);
                            if (!in && nz) {
                                if (CLOSED) {
                                    viol = true;
                                } else {
                                    const int pr = r + dd.off;
#pragma unroll
                                    for (int b = 0; b < B; ++b)
                                        cfma(acc[p][k][b], cv, cscale(x[b * a.stride + pr], scale[b]));
                                }
                            }
                        }
                    }
                }
                if (dj + 1 < total) load_diag<R, P, NT, RAG, PERM>(c, a.desc[dj + 1], tid, T, base, qb, logW);
            }
            if (f + 1 < a.nf) {
                __syncthreads();
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int i = lidx(p, k);
                        if (i < T)
#pragma unroll
                            for (int b = 0; b < B; ++b) lds[b * T + i] = acc[p][k][b];
                    }
                __syncthreads();
            }
        }
    } else {
        C2<R> c[PF][P][2];
#pragma unroll
        for (int u = 0; u < PF; ++u)
            if (u < total) load_diag<R, P, NT, RAG, PERM>(c[u], a.desc[u], tid, T, base, qb, logW);
        __syncthreads();
        clear_acc();
        int f = 0, fend = a.dstart[1];
        for (int d0 = 0; d0 < total; d0 += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int dj = d0 + u;
                if (dj < total) {                 // uniform over the workgroup
                    if (dj == fend) {             // first diagonal of the next factor
                        acc_to_lds();
                        clear_acc();
                        ++f;
                        fend = a.dstart[f + 1];
                    }
                    const DiagDesc dd = a.desc[dj];
                    apply(c[u], dd);
                    if (dj + PF < total) load_diag<R, P, NT, RAG, PERM>(c[u], a.desc[dj + PF], tid, T, base, qb, logW);
                }
            }
        }
    }

    if (a.norm_out) {
        // FP64 sum of |y|^2 over the tile's rows, per state: rows in a fixed
        // order per thread, a wave butterfly, then the waves in order.  The
        // state tile in LDS is no longer needed once every thread is here.
        double ss[B];
#pragma unroll
        for (int b = 0; b < B; ++b) ss[b] = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = lidx(p, k);
                if (i < T && (!RAG || row_of(i) < a.N))
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const double re = (double)acc[p][k][b].re, im = (double)acc[p][k][b].im;
                        ss[b] += re * re + im * im;
                    }
            }
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
        const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double v = wave_sum(ss[b]);
            if (lane == 0) red[wave * B + b] = v;
        }
        __syncthreads();
        if (tid < B) {
            double tsum = 0.0;
            for (int w = 0; w < NT / 64; ++w) tsum += red[w * B + tid];
            double *o = a.norm_out + ((size_t)tid * gridDim.x + blockIdx.x) * 4;
            o[0] = 0.0;
            o[1] = 0.0;
            o[2] = tsum;
            o[3] = 0.0;
        }
    }
    if (HORNER) {
        const C2<R> *x0 = reinterpret_cast<const C2<R> *>(a.x0);
        const C2<R> al{(R)a.alpha_re, (R)a.alpha_im};
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = lidx(p, 0), i1 = lidx(p, 1);
            const int r0 = i0 < T ? row_of(i0) : base;
            const int r1 = SPLIT ? (i1 < T ? row_of(i1) : base) : r0 + 1;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                C2<R> v0, v1;
                if (RAG) {
                    const C2<R> z{(R)0, (R)0};
                    v0 = r0 < a.N ? x0[b * a.stride + r0] : z;
                    v1 = r1 < a.N ? x0[b * a.stride + r1] : z;
                } else if (SPLIT) {
                    v0 = ld1(x0 + b * a.stride, r0);
                    v1 = ld1(x0 + b * a.stride, r1);
                } else {
                    ld2(x0 + b * a.stride, r0, v0, v1);
                }
                cfma(v0, al, acc[p][0][b]);
                cfma(v1, al, acc[p][1][b]);
                acc[p][0][b] = v0;
                acc[p][1][b] = v1;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if constexpr (SPLIT) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = lidx(p, k);
                if (i < T) {
                    const int r = row_of(i);
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        if (!RAG) st1<STREAM>(y + b * a.stride, r, acc[p][k][b]);
                        else if (r < a.N) y[b * a.stride + r] = acc[p][k][b];
                    }
                }
            }
            continue;
        }
        const int i0 = lidx(p, 0);
        if (i0 < T) {
            const int r0 = row_of(i0);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (!RAG) {
                    st2<STREAM>(y + b * a.stride, r0, acc[p][0][b], acc[p][1][b]);
                } else {
                    if (!RAG || r0 < a.N) y[b * a.stride + r0] = acc[p][0][b];
                    if (!RAG || r0 + 1 < a.N) y[b * a.stride + r0 + 1] = acc[p][1][b];
                }
            }
        }
    }
    if (CLOSED && viol) atomicOr(a.viol, 1);
}

// ------------------------------------------------------------ pair kernel
//
// Closed complex64 launches in which every diagonal "pairs": the partners of
// a thread's two rows are adjacent LDS entries starting on an even one.  That
// holds for every diagonal of a strided tile (offsets are multiples of 2^qb
// and W is even, so both rows of a pair sit on one level) and for a
// contiguous tile whose offsets are all even.  Then both rows are in or out
// of the tile together, the two coefficients of a pair are one 16-byte load,
// and the two partners of every state one 16-byte LDS load (lanes read
// consecutive 16-byte words: no bank conflicts).  The LDS stride between
// states is a compile-time constant (the instantiation's row capacity), so
// per-state LDS offsets are immediates.  The loop body has no branch between
// diagonals of different shapes, so the coefficient loads of the next PF
// diagonals stay in flight while this one is used.
//
// A coefficient whose partner lies outside the tile is zero for factors built
// here (closure); such a row reads its own LDS entry and a nonzero value only
// raises the violation flag.  Each row adds the same products in the same
// order as the row-by-row kernel, with the same operands wherever the
// coefficient is nonzero, so the two kernels give the same values.
template <int B, int RPT, int NT>
constexpr int pair_lds_rows() {
    int rows = NT * RPT;
    while (rows > 2 && (long)rows * B * 8 > tile_lds_bytes(false, B, false)) rows >>= 1;
    return rows;
}

#ifndef HS_PAIR_PF_BASE
#define HS_PAIR_PF_BASE 30     // registers of the pair kernel besides per-pair indexing, accumulators, LDS operands and the load ring
#endif
// Diagonals whose coefficients a thread of the pair kernel keeps in flight:
// about HS_TILE_INFLIGHT pair loads, cut while an estimate of its registers
// (a fixed part, the accumulators and LDS operands, the ring of P * PF pairs)
// would pass what NT
// threads per workgroup leave each thread.
template <int B, int P, int NT>
constexpr int pair_pf() {
    const int budget = NT >= 1024 ? 128 : 256;
    int pf = HS_TILE_INFLIGHT / P >= 1 ? HS_TILE_INFLIGHT / P : 1;
    while (pf > 1 && HS_PAIR_PF_BASE + 14 * P + 8 * P * B + 4 * P * pf > budget) --pf;
    return pf;
}

template <int B, int RPT, int NT, bool STREAM, bool PERM = false, bool ODD = false>
__global__ __launch_bounds__(NT) void dia_pair_kernel(TileArgs a) {
    using R = float;
    static_assert(RPT % 2 == 0, "rows come in pairs");
    static_assert(!(PERM && ODD), "odd offsets occur in contiguous tiles, which keep natural order");
    // odd offsets with 6-8 states (one row pair per thread): pick a row's
    // entry when used, which frees registers of the ring
    constexpr bool SEL_AT_USE = ODD && B >= 5 && RPT == 2;
    constexpr int P = RPT / 2;
    constexpr int TS = pair_lds_rows<B, RPT, NT>();       // LDS rows per state (>= T)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<R> *lds = reinterpret_cast<C2<R> *>(smem_raw);
    const int T = a.T;
    const int tid = threadIdx.x;
    const int qb = a.qb, kb = a.kb, logW = a.logW;
    const int W = 1 << logW;
    const int L = 1 << kb;
    int blk = blockIdx.x;
    if (a.swizzle && (gridDim.x & 7) == 0) blk = (blk & 7) * (gridDim.x >> 3) + (blk >> 3);
    const int hi = blk >> a.nlw_log;
    const int lw = blk & ((1 << a.nlw_log) - 1);
    const int base = (hi << (qb + kb)) | (lw << logW);
    const C2<R> *x = reinterpret_cast<const C2<R> *>(a.x);  // may alias y (in place)
    C2<R> *y = reinterpret_cast<C2<R> *>(a.y);
    R scale[B];
#pragma unroll
    for (int b = 0; b < B; ++b) scale[b] = inv_norm<R>(a.nrm2, b);
    auto row_of = [&](int i) { return base + ((i >> logW) << qb) + (i & (W - 1)); };

    {
        C2<R> u[P][2][B];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            const int r0 = i0 < T ? row_of(i0) : base;
#pragma unroll
            for (int b = 0; b < B; ++b) ld2(x + b * a.stride, r0, u[p][0][b], u[p][1][b]);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            if (i0 < T)
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    lds[b * TS + i0] = cscale(u[p][0][b], scale[b]);
                    lds[b * TS + i0 + 1] = cscale(u[p][1][b], scale[b]);
                }
        }
    }

    // Coefficients of PF diagonals are in flight: about HS_TILE_INFLIGHT
    // 16-byte pair loads per thread, so that a workgroup of few row pairs per
    // thread (large batches: one workgroup per CU) still keeps the CU's share
    // of HBM busy while it computes.
    // (the odd-offset path's clamps and selects take registers of the
    // ring: at most 4 diagonals in flight there, one fewer than otherwise)
    constexpr int PF0 = pair_pf<B, P, NT>();
    constexpr int PF = !ODD ? PF0 : (PF0 - 1 < 1 ? 1 : (PF0 - 1 > 4 ? 4 : PF0 - 1));
    const int total = a.dstart[a.nf];
    C2<R> acc[P][2][B];
    bool viol = false;
    auto clear_acc = [&]() {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int b = 0; b < B; ++b) acc[p][k][b] = C2<R>{(R)0, (R)0};
    };
    // coefficient pair of every row pair (even offsets: a pair is in or out
    // of the diagonal's range as a whole; out-of-range pairs read entry 0 and
    // are zeroed when used).  Diagonal j >= total is a placeholder of no
    // entries: every lane reads entry 0 of the last diagonal (one cached
    // line) and the values are never used; it keeps the number of loads per
    // loop iteration fixed, so their waits stay exact.  PERM: the diagonal
    // may be stored out of natural order (perm_pos keeps an even entry and its
    // successor adjacent, and entry 0 in place).
    auto load = [&](C2<R> (&c)[P][2], int j) {
        const DiagDesc &dd = a.desc[j < total ? j : total - 1];
        const C2<R> *cp = reinterpret_cast<const C2<R> *>(dd.ptr);
        const int neg = dd.off < 0 ? dd.off : 0;
        const int len = j < total ? dd.hi - dd.lo : 0;
        if (ODD && (dd.off & 1)) {
            // odd offset (contiguous tile, one-row windows): the pair's
            // entries e, e + 1 start at any entry.  The load stays inside
            // the diagonal's N - |d| >= 2 entries (clamped start el); each
            // row's entry is taken from the loaded pair here, or when used
            // (SEL_AT_USE).
            const int lim = dd.hi - dd.lo;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int i0 = 2 * tid + 2 * NT * p;
                const int e = row_of(i0) + neg;
                const int el = min(max(e, 0), lim - 2);
                if (SEL_AT_USE) {
                    ld2u(cp, el, c[p][0], c[p][1]);
                } else {
                    C2<R> v0, v1;
                    ld2u(cp, el, v0, v1);
                    c[p][0] = e == el ? v0 : v1;
                    c[p][1] = e + 1 == el ? v0 : v1;
                }
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            int e = row_of(i0) + neg;
            e = (e >= 0 && e < len && i0 < T) ? e : 0;
            if (PERM) e = perm_pos32(e, dd.ps, dd.pc, dd.plr);
            ld2(cp, e, c[p][0], c[p][1]);
        }
    };
    auto apply = [&](const C2<R> (&cc)[P][2], const DiagDesc &dd) {
        const int mW = dd.m * W;
        if (ODD && (dd.off & 1)) {
            // odd offset: rows i0, i0 + 1 meet partners s, s + 1 (s = i0 + m,
            // odd); each row has its own range and closure test.  The LDS
            // read of the partner pair is clamped into the tile; in a wave
            // whose pairs all lie inside it, no selects are needed.
            const int neg = dd.off < 0 ? dd.off : 0, lim = dd.hi - dd.lo;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int i0 = 2 * tid + 2 * NT * p;
                const int r0 = row_of(i0);
                const bool v0 = i0 < T && r0 >= dd.lo && r0 < dd.hi;
                const bool v1 = i0 < T && r0 + 1 >= dd.lo && r0 + 1 < dd.hi;
                // the loaded pair starts at el = e clamped into the diagonal:
                // a pair with one row out of range finds its in-range entry
                // in it (the other row is zeroed)
                C2<R> k0 = cc[p][0], k1 = cc[p][1];
                if (SEL_AT_USE) {
                    const int e = r0 + neg, el = min(max(e, 0), lim - 2);
                    k0 = e == el ? cc[p][0] : cc[p][1];
                    k1 = e + 1 == el ? cc[p][0] : cc[p][1];
                }
                const C2<R> c0 = cmask(k0, v0), c1 = cmask(k1, v1);
                const int sp = i0 + mW;
                const bool in0 = (unsigned)sp < (unsigned)T, in1 = (unsigned)(sp + 1) < (unsigned)T;
                viol = viol || (!in0 && (c0.re != (R)0 || c0.im != (R)0)) ||
                       (!in1 && (c1.re != (R)0 || c1.im != (R)0));
                const int sl = min(max(sp, 0), T - 2);
                const bool exact = sp == sl, low = sp + 1 == sl;
                if (__all(exact)) {
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        cfma(acc[p][0][b], c0, lds[b * TS + sl]);
                        cfma(acc[p][1][b], c1, lds[b * TS + sl + 1]);
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const C2<R> lo = lds[b * TS + sl], hi = lds[b * TS + sl + 1];
                        cfma(acc[p][0][b], c0, exact ? lo : hi);
                        cfma(acc[p][1][b], c1, low ? lo : hi);
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            const int r0 = row_of(i0);
            const bool valid = i0 < T && r0 >= dd.lo && r0 < dd.hi;
            const C2<R> c0 = cmask(cc[p][0], valid), c1 = cmask(cc[p][1], valid);
            const bool in = (unsigned)((i0 >> logW) + dd.m) < (unsigned)L;
            const int sl = in ? i0 + mW : (i0 < T ? i0 : 0);
            const bool nz = c0.re != (R)0 || c0.im != (R)0 || c1.re != (R)0 || c1.im != (R)0;
            viol = viol || (!in && nz);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const f4v v = *reinterpret_cast<const f4v *>(&lds[b * TS + sl]);
                cfma(acc[p][0][b], c0, C2<R>{v.x, v.y});
                cfma(acc[p][1][b], c1, C2<R>{v.z, v.w});
            }
        }
    };
    int f = 0, fend = a.dstart[1];
    // before the first diagonal of the next factor: the finished factor's
    // output becomes the tile
    auto next_factor = [&](int dj) {
        if (dj == fend) {             // uniform over the workgroup
            __syncthreads();
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int i0 = 2 * tid + 2 * NT * p;
                if (i0 < T)
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        lds[b * TS + i0] = acc[p][0][b];
                        lds[b * TS + i0 + 1] = acc[p][1][b];
                    }
            }
            __syncthreads();
            clear_acc();
            ++f;
            fend = a.dstart[f + 1];
        }
    };

    C2<R> c[PF][P][2];
#pragma unroll
    for (int u = 0; u < PF; ++u) load(c[u], u);
    __syncthreads();
    clear_acc();
    int d0 = 0;
    for (; d0 + PF <= total; d0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            next_factor(d0 + u);
            apply(c[u], a.desc[d0 + u]);
            load(c[u], d0 + u + PF);
        }
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        if (d0 + u < total) {
            next_factor(d0 + u);
            apply(c[u], a.desc[d0 + u]);
        }
    }

    if (a.norm_out) {
        double ss[B];
#pragma unroll
        for (int b = 0; b < B; ++b) ss[b] = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            if (i0 < T) {
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const double re = (double)acc[p][k][b].re, im = (double)acc[p][k][b].im;
                        ss[b] += re * re + im * im;
                    }
            }
        }
        __syncthreads();
        double *red = reinterpret_cast<double *>(smem_raw);
        const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const double v = wave_sum(ss[b]);
            if (lane == 0) red[wave * B + b] = v;
        }
        __syncthreads();
        if (tid < B) {
            double tsum = 0.0;
            for (int w = 0; w < NT / 64; ++w) tsum += red[w * B + tid];
            double *o = a.norm_out + ((size_t)tid * gridDim.x + blockIdx.x) * 4;
            o[0] = 0.0;
            o[1] = 0.0;
            o[2] = tsum;
            o[3] = 0.0;
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i0 = 2 * tid + 2 * NT * p;
        if (i0 < T) {
            const int r0 = row_of(i0);
#pragma unroll
            for (int b = 0; b < B; ++b) st2<STREAM>(y + b * a.stride, r0, acc[p][0][b], acc[p][1][b]);
        }
    }
    if (viol) atomicOr(a.viol, 1);
}

// ------------------------------------------------------------ whole evolution
//
// Small states (at most 8192 complex64 or 4096 complex128 rows): one
// workgroup per state holds the whole state in LDS and applies every factor
// of every step in one launch -- no launch per factor run and step, no state
// traffic between steps.  Thread t owns row pairs (2t + 2 NT p, +1), as the
// tile kernel's contiguous tiles do; every partner row is in LDS.  Each row
// sums, per factor, its diagonals in ascending-offset order with the same
// fused multiply-adds as the tile kernel, starting from zero, so the values
// are the same as those of one launch per fused run and step.
//
// The diagonals are visited in a fixed walk (step s: its part's list of
// entries).  A ring of KD slots holds the coefficients of the next KD
// diagonals (KD = 8 / P, so that a thread has about 8 row-pair loads
// outstanding) with each one's offset and end-of-factor mark: a slot is
// refilled from the walk KD diagonals ahead of its use, across factor and
// step boundaries, so using a diagonal reads no table.  The cursor and the
// walk entries are uniform over the workgroup.
struct WholeCursor {
    int s, k, kend;
    __device__ __forceinline__ static int part_of(const WholeArgs &a, int st) {
        return a.steps == 1 ? 0 : st == 0 ? 1 : st == a.steps - 1 ? 3 : 2;
    }
    __device__ __forceinline__ void start(const WholeArgs &a) {
        s = 0;
        const int part = part_of(a, 0);
        k = a.part_off[part];
        kend = a.part_off[part + 1];
    }
    __device__ __forceinline__ bool done(const WholeArgs &a) const { return s >= a.steps; }
    __device__ __forceinline__ void next(const WholeArgs &a) {
        if (++k < kend) return;
        if (++s < a.steps) {
            const int part = part_of(a, s);
            k = a.part_off[part];
            kend = a.part_off[part + 1];
        }
    }
};

#ifndef HS_WHOLE_KD
#define HS_WHOLE_KD 8          // row-pair coefficient loads per thread the whole-evolution kernel keeps in flight
#endif

template <typename R, int P, int NT>
__global__ __launch_bounds__(NT) void dia_whole_kernel(WholeArgs a) {
    constexpr int KD = HS_WHOLE_KD / P >= 1 ? HS_WHOLE_KD / P : 1;   // diagonals in flight
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<R> *lds = reinterpret_cast<C2<R> *>(smem_raw);
    const int N = a.N;
    const int tid = threadIdx.x;
    C2<R> *psi = reinterpret_cast<C2<R> *>(a.psi) + (int64_t)blockIdx.x * a.stride;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i0 = 2 * tid + 2 * NT * p;
        if (i0 < N) {
            C2<R> u0, u1;
            ld2_cached(psi, i0, u0, u1);
            lds[i0] = u0;
            lds[i0 + 1] = u1;
        }
    }
    C2<R> c[KD][P][2];
    int soff[KD];
    uint32_t slast[KD];
    WholeCursor fetch;
    fetch.start(a);
    // refill slot u with the diagonal at the fetch cursor (zero outside
    // [lo, hi) and past N; past the walk's end: an empty placeholder)
    auto refill = [&](int u) {
        const bool live = !fetch.done(a);
        const WholeEntry e = a.walk[live ? fetch.k : 0];
        const C2<R> *cp = reinterpret_cast<const C2<R> *>(e.ptr);
        const int neg = e.off < 0 ? e.off : 0;
        const int len = live ? e.hi - e.lo : 0;
        soff[u] = e.off;
        slast[u] = e.last;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int ei = i0 + j + neg;
                const bool ok = ei >= 0 && ei < len && i0 < N;
                c[u][p][j] = cmask(ld1(cp, ok ? ei : 0), ok);
            }
        }
        if (live) fetch.next(a);
    };
#pragma unroll
    for (int u = 0; u < KD; ++u) refill(u);
    __syncthreads();
    C2<R> acc[P][2];
#pragma unroll
    for (int p = 0; p < P; ++p) acc[p][0] = acc[p][1] = C2<R>{(R)0, (R)0};
    // use slot u for the next diagonal of the walk
    auto consume = [&](int u) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int pr = i0 + j + soff[u];
                const int sl = (pr >= 0 && pr < N) ? pr : (i0 < N ? i0 + j : 0);
                cfma(acc[p][j], c[u][p][j], lds[sl]);
            }
        }
    };
    // the factor is complete: it becomes the state
    auto end_factor = [&]() {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i0 = 2 * tid + 2 * NT * p;
            if (i0 < N) {
                lds[i0] = acc[p][0];
                lds[i0 + 1] = acc[p][1];
            }
            acc[p][0] = acc[p][1] = C2<R>{(R)0, (R)0};
        }
        __syncthreads();
    };
    // the walk's length over all steps; full rounds of KD diagonals refill
    // every slot (a fixed number of loads per round), the rest only consume
    auto plen = [&](int q) { return a.part_off[q + 1] - a.part_off[q]; };
    const int64_t total = a.steps == 1 ? plen(0)
                                       : (int64_t)plen(1) + (int64_t)(a.steps - 2) * plen(2) + plen(3);
    int64_t done = 0;
    for (; done + KD <= total; done += KD) {
#pragma unroll
        for (int u = 0; u < KD; ++u) {
            const bool last = slast[u] != 0;
            consume(u);
            refill(u);
            if (last) end_factor();
        }
    }
#pragma unroll
    for (int u = 0; u < KD; ++u) {
        if (done + u < total) {
            consume(u);
            if (slast[u] != 0) end_factor();
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i0 = 2 * tid + 2 * NT * p;
        if (i0 < N) st2<false>(psi, i0, lds[i0], lds[i0 + 1]);
    }
}

// Single main-diagonal factor applied `steps` times: y[i] = v[i]^steps x[i]
// for N even, each thread two adjacent entries (one 16-byte load of the
// coefficients and of each state for complex64), the powers taken as
// `steps` successive complex multiplications in registers in the order of
// one step at a time, so the result equals `steps` single-step passes bit
// for bit while the diagonal and the states cross HBM once.  In place
// allowed.  STREAM: non-temporal output stores.
template <typename R, int B, bool STREAM>
__global__ __launch_bounds__(256) void diag_steps_kernel(C2<R> *y, const C2<R> *x, const C2<R> *__restrict__ v,
                                                         int64_t N, int steps, const double *nrm2) {
    R scale[B];
#pragma unroll
    for (int b = 0; b < B; ++b) scale[b] = inv_norm<R>(nrm2, b);
    const int64_t npairs = N >> 1;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < npairs;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(2 * q);
        C2<R> c0, c1;
        ld2(v, i, c0, c1);
        C2<R> u[B][2];
#pragma unroll
        for (int b = 0; b < B; ++b) ld2(x + b * N, i, u[b][0], u[b][1]);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            C2<R> a0 = cscale(u[b][0], scale[b]), a1 = cscale(u[b][1], scale[b]);
            for (int s = 0; s < steps; ++s) {
                C2<R> t0{(R)0, (R)0}, t1{(R)0, (R)0};
                cfma(t0, c0, a0);
                cfma(t1, c1, a1);
                a0 = t0;
                a1 = t1;
            }
            st2<STREAM>(y + b * N, i, a0, a1);
        }
    }
}

template <typename R>
__global__ void scale_kernel(C2<R> *psi, int64_t N, const double *nrm2) {
    const int b = blockIdx.y;
    const R s = inv_norm<R>(nrm2, b);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        psi[b * N + i] = cscale(psi[b * N + i], s);
}

// ------------------------------------------------------------ reductions
// Pass 1: block g of state b sums elements g*256+t, stepping by G*256, in
// FP64; wave64 butterfly, then the four waves in fixed order.  Pass 2: one
// block per state sums the G partials in a fixed tree.  No atomics, so the
// result is bit-reproducible.

template <typename TA, typename TB, bool DOT>
__global__ __launch_bounds__(256) void reduce_partial_kernel(const void *A, const void *Bv, int64_t N,
                                                             int G, double *partial) {
    const int b = blockIdx.y;
    const C2<TA> *pa = reinterpret_cast<const C2<TA> *>(A) + b * N;
    const C2<TB> *pb = reinterpret_cast<const C2<TB> *>(Bv) + b * N;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)G * 256) {
        const C2<TA> u = pa[i];
        const double ar = (double)u.re, ai = (double)u.im;
        s[2] += ar * ar + ai * ai;
        if (DOT) {
            const C2<TB> w = pb[i];
            const double br = (double)w.re, bi = (double)w.im;
            s[0] += ar * br + ai * bi;
            s[1] += ar * bi - ai * br;
            s[3] += br * br + bi * bi;
        }
    }
    __shared__ double red[4][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(s[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        partial[((int64_t)b * G + blockIdx.x) * 4 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const double *partial, int G, double *out) {
    const int b = blockIdx.x;
    __shared__ double red[256][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = threadIdx.x; g < G; g += 256)
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += partial[((int64_t)b * G + g) * 4 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[b * 4 + threadIdx.x] = red[0][threadIdx.x];
}

// Fidelity records: out[b] = (Re, Im <phi|psi>, <phi|phi>, <psi|psi>, F) from
// the reduction records, F = (Re^2 + Im^2) / (<phi|phi> <psi|psi>) evaluated
// as separate roundings (no fused multiply-add), as the host evaluates it.
__global__ void fidelity_records_kernel(const double *rec, int batch, double *out) {
#pragma clang fp contract(off)
    const int b = threadIdx.x;
    if (b < batch) {
        const double re = rec[4 * b], im = rec[4 * b + 1], np = rec[4 * b + 2], nq = rec[4 * b + 3];
        out[5 * b + 0] = re;
        out[5 * b + 1] = im;
        out[5 * b + 2] = np;
        out[5 * b + 3] = nq;
        out[5 * b + 4] = (re * re + im * im) / (np * nq);
    }
}

// ------------------------------------------------------------ launchers

static inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

static inline int grid_for(int64_t n, int per_block, int cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

int launch_phase_table(int64_t N, int nz, const uint64_t *zm, const double *cf, double dt,
                       double *out, void *stream) {
    hipLaunchKernelGGL(phase_table_kernel, dim3(grid_for(N, 256, 1 << 20)), dim3(256), 0, S(stream),
                       N, nz, zm, cf, dt, out);
    return (int)hipGetLastError();
}

int launch_construct(const ConstructArgs &a, int nd, int64_t max_len, bool c128, void *stream) {
    dim3 grid(grid_for(max_len, 256, 1 << 16), nd);
    if (c128)
        hipLaunchKernelGGL(construct_kernel<double>, grid, dim3(256), 0, S(stream), a);
    else
        hipLaunchKernelGGL(construct_kernel<float>, grid, dim3(256), 0, S(stream), a);
    return (int)hipGetLastError();
}

int launch_perm_gather(const void *src, void *dst, int64_t start, int64_t count, int64_t len, int s, int c,
                       bool c128, void *stream) {
    if (count <= 0) return 0;
    if (start < 0 || start + count > len || s < c || c < 0 || s > 30) return (int)hipErrorInvalidValue;
    const int g = grid_for(count, 256, 1 << 16);
    if (c128)
        hipLaunchKernelGGL(perm_gather_kernel<double>, dim3(g), dim3(256), 0, S(stream),
                           static_cast<const C2<double> *>(src), static_cast<C2<double> *>(dst), start, count, len,
                           s, c);
    else
        hipLaunchKernelGGL(perm_gather_kernel<float>, dim3(g), dim3(256), 0, S(stream),
                           static_cast<const C2<float> *>(src), static_cast<C2<float> *>(dst), start, count, len, s,
                           c);
    return (int)hipGetLastError();
}

enum TileMode { kOpen = 0, kClosed = 1, kHorner = 2 };

static std::mutex &lds_attr_mutex() {
    static std::mutex m;
    return m;
}

// Launch with the smallest rows-per-thread instantiation (power of two, down
// to one row pair) that still gives every tile row a thread: a tile smaller
// than the kernel's capacity would otherwise issue masked loads and FMAs.
template <typename R, int B, int RPT, bool CLOSED, bool HORNER, int NT, bool RAG = false, bool STREAM = false,
          bool PERM = false>
static int tile_launch(const TileArgs &a, int rows_per_thread, size_t lds, int grid, void *stream) {
    if constexpr (RPT > 2) {
        if (rows_per_thread <= RPT / 2)
            return tile_launch<R, B, RPT / 2, CLOSED, HORNER, NT, RAG, STREAM, PERM>(a, rows_per_thread, lds, grid,
                                                                                    stream);
    }
    auto kern = dia_tile_kernel<R, B, RPT, CLOSED, HORNER, NT, RAG, STREAM, PERM>;
    if (lds > 65536) {
        // allow this instantiation the dynamic LDS the launch needs (raised
        // only when a larger launch arrives; the planner keeps lds within the
        // device's per-workgroup limit)
        static std::atomic<int> allowed{65536};
        int cur = allowed.load();
        while ((int)lds > cur) {
            std::lock_guard<std::mutex> lock(lds_attr_mutex());
            cur = allowed.load();
            if ((int)lds <= cur) break;
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return (int)e;
            allowed.store((int)lds);
            cur = (int)lds;
        }
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, S(stream), a);
    return (int)hipGetLastError();
}

// The pair kernel with the smallest rows-per-thread instantiation that
// gives every tile row a thread (as tile_launch).
template <int B, int RPT, int NT, bool STREAM, bool PERM = false, bool ODD = false>
static int pair_launch(const TileArgs &a, int rows_per_thread, int grid, void *stream) {
    if constexpr (RPT > 2) {
        if (rows_per_thread <= RPT / 2)
            return pair_launch<B, RPT / 2, NT, STREAM, PERM, ODD>(a, rows_per_thread, grid, stream);
    }
    constexpr int TS = pair_lds_rows<B, RPT, NT>();
    if (a.T > TS) return (int)hipErrorInvalidValue;
    // odd offsets: contiguous tiles of one-row windows only
    if (ODD && (a.qb != 0 || a.logW != 0 || a.T != (1 << a.kb))) return (int)hipErrorInvalidValue;
    auto kern = dia_pair_kernel<B, RPT, NT, STREAM, PERM, ODD>;
    const size_t lds = (size_t)TS * B * sizeof(C2<float>);
    if (lds > 65536) {
        static std::atomic<int> allowed{65536};
        int cur = allowed.load();
        while ((int)lds > cur) {
            std::lock_guard<std::mutex> lock(lds_attr_mutex());
            cur = allowed.load();
            if ((int)lds <= cur) break;
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return (int)e;
            allowed.store((int)lds);
            cur = (int)lds;
        }
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, S(stream), a);
    return (int)hipGetLastError();
}

template <typename R, int B>
static int tile_dispatch_b(const TileArgs &a, int mode, void *stream) {
    constexpr bool c128 = sizeof(R) == 8;
    constexpr int RPT = tile_rpt(c128, B);
    constexpr int RPT_OPEN = tile_rpt(c128, B, true);
    constexpr int NTC = tile_threads(c128, B);
    constexpr int NTO = tile_threads(c128, B, true);
    const size_t lds = (size_t)a.T * B * sizeof(C2<R>);
    // every tile row must belong to a thread, and the tile must fit the LDS
    // budget; only open contiguous launches may end in a partial tile
    const int nt = mode == kClosed ? NTC : NTO;
    const int rpt = mode == kClosed ? RPT : RPT_OPEN;
    if (a.T < 2 || a.T > nt * rpt || lds > (size_t)tile_lds_bytes(c128, B, mode != kClosed)) return (int)hipErrorInvalidValue;
    // a thread's row pair must be adjacent state rows: strided tiles need W >= 2
    if (a.qb != 0 && a.logW < 1) return (int)hipErrorInvalidValue;
    const bool rag = a.ragged != 0;
    if ((a.N % a.T != 0) != rag) return (int)hipErrorInvalidValue;
    if (rag && (mode == kClosed || a.qb != 0 || a.logW != 0 || a.nlw_log != 0 || a.swizzle))
        return (int)hipErrorInvalidValue;
    const int grid = (int)((a.N + a.T - 1) / a.T);
    const int need = (a.T + nt - 1) / nt;
    const bool st = a.stream_out != 0;         // ragged launches keep plain stores
    // diagonals stored out of natural order are read by closed launches only
    if (a.perm && mode != kClosed) return (int)hipErrorInvalidValue;
    const bool pm = a.perm != 0;
    if constexpr (sizeof(R) == 4) {
        if (mode == kClosed && a.pairs == 2) {      // some diagonals have odd offsets
            if (pm) return (int)hipErrorInvalidValue;
            return st ? pair_launch<B, RPT, NTC, true, false, true>(a, need, grid, stream)
                      : pair_launch<B, RPT, NTC, false, false, true>(a, need, grid, stream);
        }
        if (mode == kClosed && a.pairs) {
            if (pm)
                return st ? pair_launch<B, RPT, NTC, true, true>(a, need, grid, stream)
                          : pair_launch<B, RPT, NTC, false, true>(a, need, grid, stream);
            return st ? pair_launch<B, RPT, NTC, true>(a, need, grid, stream)
                      : pair_launch<B, RPT, NTC, false>(a, need, grid, stream);
        }
    }
    if (mode == kClosed) {
        if (pm)
            return st ? tile_launch<R, B, RPT, true, false, NTC, false, true, true>(a, need, lds, grid, stream)
                      : tile_launch<R, B, RPT, true, false, NTC, false, false, true>(a, need, lds, grid, stream);
        return st ? tile_launch<R, B, RPT, true, false, NTC, false, true>(a, need, lds, grid, stream)
                  : tile_launch<R, B, RPT, true, false, NTC>(a, need, lds, grid, stream);
    }
    if (mode == kOpen)
        return rag  ? tile_launch<R, B, RPT_OPEN, false, false, NTO, true>(a, need, lds, grid, stream)
               : st ? tile_launch<R, B, RPT_OPEN, false, false, NTO, false, true>(a, need, lds, grid, stream)
                    : tile_launch<R, B, RPT_OPEN, false, false, NTO>(a, need, lds, grid, stream);
    return rag  ? tile_launch<R, B, RPT_OPEN, false, true, NTO, true>(a, need, lds, grid, stream)
           : st ? tile_launch<R, B, RPT_OPEN, false, true, NTO, false, true>(a, need, lds, grid, stream)
                : tile_launch<R, B, RPT_OPEN, false, true, NTO>(a, need, lds, grid, stream);
}

template <typename R>
static int tile_dispatch(const TileArgs &a, int batch, int mode, void *stream) {
    switch (batch) {
        case 1: return tile_dispatch_b<R, 1>(a, mode, stream);
        case 2: return tile_dispatch_b<R, 2>(a, mode, stream);
        case 3: return tile_dispatch_b<R, 3>(a, mode, stream);
        case 4: return tile_dispatch_b<R, 4>(a, mode, stream);
        case 5: return tile_dispatch_b<R, 5>(a, mode, stream);
        case 6: return tile_dispatch_b<R, 6>(a, mode, stream);
        case 7: return tile_dispatch_b<R, 7>(a, mode, stream);
        case 8: return tile_dispatch_b<R, 8>(a, mode, stream);
        default: return (int)hipErrorInvalidValue;
    }
}

int launch_tile(const TileArgs &a, int batch, bool c128, bool closed, void *stream) {
    const int mode = closed ? kClosed : kOpen;
    return c128 ? tile_dispatch<double>(a, batch, mode, stream) : tile_dispatch<float>(a, batch, mode, stream);
}

int launch_tile_horner(const TileArgs &a, int batch, bool c128, void *stream) {
    if (!a.x0) return (int)hipErrorInvalidValue;
    return c128 ? tile_dispatch<double>(a, batch, kHorner, stream)
                : tile_dispatch<float>(a, batch, kHorner, stream);
}


template <typename R, int P, int NT>
static int whole_launch(const WholeArgs &a, int batch, void *stream) {
    auto kern = dia_whole_kernel<R, P, NT>;
    const size_t lds = (size_t)a.N * sizeof(C2<R>);
    if (lds > 65536) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(batch), dim3(NT), lds, S(stream), a);
    return (int)hipGetLastError();
}

// threads and row pairs per thread for N rows: 2 NT P >= N
template <typename R>
static int whole_dispatch(const WholeArgs &a, int batch, void *stream) {
    const int N = a.N;
    if (N <= 128) return whole_launch<R, 1, 64>(a, batch, stream);
    if (N <= 256) return whole_launch<R, 1, 128>(a, batch, stream);
    if (N <= 512) return whole_launch<R, 1, 256>(a, batch, stream);
    if (N <= 1024) return whole_launch<R, 1, 512>(a, batch, stream);
    if (N <= 2048) return whole_launch<R, 2, 512>(a, batch, stream);
    if (N <= 4096) return whole_launch<R, 4, 512>(a, batch, stream);
    if constexpr (sizeof(R) == 4) {
        if (N <= 8192) return whole_launch<R, 8, 512>(a, batch, stream);
    }
    return (int)hipErrorInvalidValue;
}

int launch_whole(const WholeArgs &a, int batch, bool c128, void *stream) {
    if (a.N < 2 || (a.N & 1) || batch < 1 || a.steps < 1 || a.part_off[4] < 1) return (int)hipErrorInvalidValue;
    return c128 ? whole_dispatch<double>(a, batch, stream) : whole_dispatch<float>(a, batch, stream);
}

template <typename R, bool STREAM>
static int diag_steps_dispatch(void *y, const void *x, const void *v, int64_t N, int batch, int steps,
                               const double *nrm2, void *stream) {
    C2<R> *py = reinterpret_cast<C2<R> *>(y);
    const C2<R> *px = reinterpret_cast<const C2<R> *>(x);
    const C2<R> *pv = reinterpret_cast<const C2<R> *>(v);
    const dim3 g(grid_for(N >> 1, 256, 1 << 20)), blk(256);
    switch (batch) {
#define HS_DSTEP_CASE(BB) \
    case BB: hipLaunchKernelGGL((diag_steps_kernel<R, BB, STREAM>), g, blk, 0, S(stream), py, px, pv, N, steps, nrm2); break;
        HS_DSTEP_CASE(1) HS_DSTEP_CASE(2) HS_DSTEP_CASE(3) HS_DSTEP_CASE(4)
        HS_DSTEP_CASE(5) HS_DSTEP_CASE(6) HS_DSTEP_CASE(7) HS_DSTEP_CASE(8)
#undef HS_DSTEP_CASE
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_diag_steps(void *y, const void *x, const void *diag, int64_t N, int batch, int steps,
                      const double *nrm2, bool c128, bool stream_out, void *stream) {
    if (N < 2 || (N & 1) || steps < 1) return (int)hipErrorInvalidValue;
    if (c128)
        return stream_out ? diag_steps_dispatch<double, true>(y, x, diag, N, batch, steps, nrm2, stream)
                          : diag_steps_dispatch<double, false>(y, x, diag, N, batch, steps, nrm2, stream);
    return stream_out ? diag_steps_dispatch<float, true>(y, x, diag, N, batch, steps, nrm2, stream)
                      : diag_steps_dispatch<float, false>(y, x, diag, N, batch, steps, nrm2, stream);
}

int launch_scale(void *psi, int64_t N, int batch, const double *nrm2, bool c128, void *stream) {
    dim3 g(grid_for(N, 256, 1 << 14), batch);
    if (c128)
        hipLaunchKernelGGL(scale_kernel<double>, g, dim3(256), 0, S(stream),
                           reinterpret_cast<C2<double> *>(psi), N, nrm2);
    else
        hipLaunchKernelGGL(scale_kernel<float>, g, dim3(256), 0, S(stream),
                           reinterpret_cast<C2<float> *>(psi), N, nrm2);
    return (int)hipGetLastError();
}

int launch_reduce(const void *A, int ta, const void *Bv, int tb, int batch, int64_t N,
                  double *partial, int G, double *out, bool dot, void *stream) {
    dim3 g(G, batch), blk(256);
    if (!dot) {
        if (ta == HS_C128)
            hipLaunchKernelGGL((reduce_partial_kernel<double, double, false>), g, blk, 0, S(stream), A, A, N, G, partial);
        else
            hipLaunchKernelGGL((reduce_partial_kernel<float, float, false>), g, blk, 0, S(stream), A, A, N, G, partial);
    } else {
        if (ta == HS_C128 && tb == HS_C128)
            hipLaunchKernelGGL((reduce_partial_kernel<double, double, true>), g, blk, 0, S(stream), A, Bv, N, G, partial);
        else if (ta == HS_C128)
            hipLaunchKernelGGL((reduce_partial_kernel<double, float, true>), g, blk, 0, S(stream), A, Bv, N, G, partial);
        else if (tb == HS_C128)
            hipLaunchKernelGGL((reduce_partial_kernel<float, double, true>), g, blk, 0, S(stream), A, Bv, N, G, partial);
        else
            hipLaunchKernelGGL((reduce_partial_kernel<float, float, true>), g, blk, 0, S(stream), A, Bv, N, G, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(batch), blk, 0, S(stream), partial, G, out);
    return (int)hipGetLastError();
}

int launch_fidelity_records(const double *rec, int batch, double *out, void *stream) {
    hipLaunchKernelGGL(fidelity_records_kernel, dim3(1), dim3(64), 0, S(stream), rec, batch, out);
    return (int)hipGetLastError();
}

int launch_reduce_partials(const double *partial, int G, int batch, double *out, void *stream) {
    hipLaunchKernelGGL(reduce_final_kernel, dim3(batch), dim3(256), 0, S(stream), partial, G, out);
    return (int)hipGetLastError();
}

}  // namespace hs
