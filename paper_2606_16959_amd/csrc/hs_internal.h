// Internal structures of the hamsim library (host planning + device launch).
#pragma once

#include <complex>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hamsim.h"

namespace hs {

constexpr double kTau = 1e-15;          // |L[a,b]| <= kTau counts as zero
constexpr int kMaxRun = 8;              // factors fused into one launch
constexpr int kMaxDiagsPerLaunch = 128; // descriptors per launch
constexpr size_t kDiagAlignBytes = 256; // start of every stored diagonal

struct Term {
    uint64_t x = 0, z = 0;  // X-part and Z-part masks (Y sets both)
    int ny = 0;             // number of Y characters
    double c = 0.0;         // real coefficient
};

struct Factor {
    double dt = 0.0;                // time step of this factor's exponential
    bool has_diag = false;          // carries D = exp(-i dt E(x)) on the right
    std::vector<int> terms;         // member term indices (application order)
    std::vector<int64_t> offs;      // ascending diagonal offsets d = col - row
    uint64_t smask = 0;             // support (X or Z bits of any member)
    std::vector<int> bits;          // support bits, ascending
    uint64_t xmask_union = 0;       // bits any member flips
    int xlb = 0, xhb = 0;           // hull [xlb, xhb) of xmask_union (empty: 0,0)
    std::vector<std::complex<double>> L;  // K x K local unitary, row-major
    std::vector<size_t> elem_off;   // element offset of each diagonal
    size_t elems_total = 0;         // elements incl. alignment padding
    int perm_s = 0, perm_c = 0;     // storage order of every diagonal (perm_pos,
                                    // storage_order.h); 0, 0 = natural
    void *dev = nullptr;            // device buffer (built handles)
};

struct Plan {
    int n = 0;
    int64_t N = 0;
    double t = 0.0, dt = 0.0;
    int steps = 0, budget = 0;
    unsigned flags = 0;
    std::vector<Term> terms;
    std::vector<int> diag;          // Z-only term indices
    int order = 1;                  // product formula: 1, 2 (symmetric) or 4 (Suzuki)
    std::vector<Factor> factors;    // distinct stored factors
    std::vector<int> seq;           // factor indices applied in one step, in order
    int joint = -1;                 // factor that joins the last and first of consecutive steps
};

// Host-side planning (no device calls).  Returns HS_OK or an error with msg.
hs_status make_plan(int n_qubits, int n_terms, const char *const *strings, const double *coeffs,
                    double t, int steps, int budget, unsigned flags, Plan &out, std::string &msg);
void layout_factor(Factor &f, int64_t N, size_t elem_bytes);

// ------------------------------------------------------------------ kernels

// One stored diagonal as seen by the tile kernel.
struct DiagDesc {
    const void *ptr;   // entries, element type = state element type
    int32_t off;       // d
    int32_t m;         // d >> qb when regular
    int32_t regular;   // d is a multiple of 2^qb
    int32_t lo, hi;    // rows r with 0 <= r + d < N: [lo, hi)
    int32_t ps, pc;    // storage order (perm_pos, storage_order.h): split bit s and chunk bits c;
                       // 0, 0 = natural
    int32_t plr;       // ((N - |d|) >> s) << c: entries between consecutive chunk columns
    int32_t pad;
};

struct TileArgs {
    void *y;
    const void *x;
    int64_t stride;          // elements between consecutive states (= N)
    int32_t N;
    int32_t nf;              // factors in this launch
    int32_t dstart[kMaxRun + 1];
    const DiagDesc *desc;
    int32_t qb, kb, logW, nlw_log, T;
    const double *nrm2;      // per-state squared norms to divide out, or null
    int *viol;               // closure-violation flag (closed launches)
    int32_t swizzle;         // deal contiguous eighths of the tiles to the 8 XCDs
    const void *x0;          // Horner launches: y = x0 + alpha (A x), x0 read at the row only
    double alpha_re, alpha_im;
    int32_t ragged;          // open contiguous launch whose last tile passes row N (any N)
    double *norm_out;        // or null: per tile and state, the FP64 sum of |y|^2 over the
                             // tile's rows at [(b * gridDim.x + tile) * 4 + 2] (others 0)
    int32_t stream_out;      // write y with non-temporal stores (see kStreamOutBytes)
    int32_t pairs;           // closed complex64 launch in the pair kernel: 1 even offsets only,
                             // 2 some odd offsets (contiguous tiles)
    int32_t perm;            // closed launch with a diagonal stored out of natural order (ps > 0)
};

// States of at least this many bytes (the chunk of up to HS_MAX_BATCH states
// that a call takes through all its launches before the next chunk) are
// written with non-temporal stores: they cannot stay in the 256 MB
// last-level cache until the next launch reads them, and streaming them past
// it measured 3-6% faster; smaller states keep the default policy so that the
// next launch finds them cached.
constexpr size_t kStreamOutBytes = size_t(128) << 20;

struct ConstructArgs {
    void *base;              // factor buffer
    const int64_t *offs;     // [nd]
    const uint64_t *elem_off;// [nd]
    const double *L;         // K*K interleaved complex
    const double *phase;     // N interleaved complex, or null
    int32_t N;
    int32_t K;
    uint32_t smask;
    int32_t contiguous;      // support is [lb, lb+k)
    int32_t lb;
    int32_t nbits;
    int8_t bits[16];
    int32_t perm_s, perm_c;  // storage order of the factor's diagonals (perm_pos)
};

// launchers (kernels.hip); all return hipError_t as int
int launch_phase_table(int64_t N, int nz, const uint64_t *zm, const double *cf, double dt,
                       double *out, void *stream);
int launch_construct(const ConstructArgs &a, int nd, int64_t max_len, bool c128, void *stream);
// dst[k] = entry start + k of a diagonal of length len stored in the order
// (s, c) (perm_pos), for k < count: the natural order of a stored range
int launch_perm_gather(const void *src, void *dst, int64_t start, int64_t count, int64_t len, int s, int c,
                       bool c128, void *stream);
int launch_tile(const TileArgs &a, int batch, bool c128, bool closed, void *stream);
// open launch with the Horner epilogue y = x0 + alpha (A x); y may alias x0, not x
int launch_tile_horner(const TileArgs &a, int batch, bool c128, void *stream);
// Whole evolution of small states in one launch (one workgroup per state,
// the state held in LDS).  Each step part is a list of entries, one per
// diagonal it applies in order: the diagonal's storage and range, and
// whether it is the last diagonal of its factor.
struct WholeEntry {
    const void *ptr;            // entries of the diagonal, the state's element type
    int32_t off, lo, hi;        // offset d; rows r with 0 <= r + d < N: [lo, hi)
    uint32_t last;              // 1 for the last diagonal of a factor
};
struct WholeArgs {
    void *psi;                  // [batch][stride] states of the handle's dtype
    int64_t stride;
    int32_t N;
    int32_t steps;
    const WholeEntry *walk;     // concatenated entry lists of the step parts
    int32_t part_off[5];        // part q applies walk[part_off[q] .. part_off[q+1])
};
// Largest state (rows) the whole-evolution kernel holds: 8192 complex64 or
// 4096 complex128 rows (64 KiB of LDS).
constexpr int kWholeRowsC64 = 8192;
constexpr int kWholeRowsC128 = 4096;
int launch_whole(const WholeArgs &a, int batch, bool c128, void *stream);
// the single-diagonal factor applied `steps` times in one pass (N even)
int launch_diag_steps(void *y, const void *x, const void *diag, int64_t N, int batch, int steps,
                      const double *nrm2, bool c128, bool stream_out, void *stream);
int launch_reduce(const void *A, int ta, const void *B, int tb, int batch, int64_t N,
                  double *partial, int G, double *out, bool dot, void *stream);
int launch_scale(void *psi, int64_t N, int batch, const double *nrm2, bool c128, void *stream);
// records [batch][4] from per-block partials [batch][G][4], in a fixed order
int launch_reduce_partials(const double *partial, int G, int batch, double *out, void *stream);
// [batch][5] fidelity records (Re, Im, <phi|phi>, <psi|psi>, F) from reduction records (batch <= 64)
int launch_fidelity_records(const double *rec, int batch, double *out, void *stream);

// general operators in the diagonal layout (dia_ops.hip)
struct PauliDiaArgs {
    int64_t N;
    const int64_t *offs;          // [nd] candidate offsets
    double *const *out;           // [nd] output diagonals (FP64 complex)
    int n_cls;                    // distinct X-masks
    const uint64_t *cls_mask;     // [n_cls]
    const int *cls_ptr;           // [n_cls + 1] into the term arrays
    const uint64_t *zmask;        // terms sorted by X-mask
    const double *coeff;
    const int *ny;
};
struct SpgemmArgs {
    int64_t N;
    const int64_t *a_offs;
    const double *const *a_ptr;
    const double *const *b_ptr;
    const int64_t *c_offs;
    double *const *c_ptr;
    const int *cptr;              // [nc + 1] contributor ranges
    const int *pairs;             // [2 * n_pairs] (index into A, index into B)
    double scale_re, scale_im;
    double *block_max;            // [nc][gridDim.x] largest entry modulus per block
};
struct DiaAddArgs {
    int64_t N;
    const int64_t *offs;
    const int *ia, *ib;           // source diagonal per output diagonal, -1 = none
    const double *const *a_ptr;
    const double *const *b_ptr;
    double *const *out;
};
int dia_grid_x(int64_t len);
int launch_pauli_dia(const PauliDiaArgs &a, int nd, void *stream);
int launch_spgemm(const SpgemmArgs &a, int nd, int gx, bool store, void *stream);
int launch_dia_add(const DiaAddArgs &a, int nd, void *stream);
int launch_dia_maxabs(const double *const *ptrs, const int64_t *offs, int64_t N, int nd, int gx,
                      double *block_max, void *stream);
int launch_dia_fill(double *out, int64_t len, double re, double im, void *stream);
int launch_diag_exp(const double *h, double *out, int64_t len, double dt, void *stream);
void set_last_error(const std::string &m);   // message returned by hs_last_error()
// Whether [p, p + bytes) is device (or managed) memory of the current device
// and lies inside one allocation; otherwise false with a message naming `what`.
// A host address handed to a kernel would fault the GPU, so every entry point
// that takes caller memory checks it before enqueuing work.
bool device_range_ok(const void *p, size_t bytes, const char *what, std::string &msg);
hs_status parse_terms(int n, int n_terms, const char *const *strings, const double *coeffs,
                      std::vector<Term> &terms, std::string &msg);
int launch_dia_to_c64(const double *const *src, float *const *dst, const int64_t *offs, int64_t N,
                      int nd, void *stream);

constexpr int kReduceBlocks = 1024;   // partial sums per state (fixed: determinism)

// Tile-kernel shape (compile-time; the launch planner and the kernels must agree).
#ifndef HS_TILE_THREADS
#define HS_TILE_THREADS 512
#endif
#ifndef HS_TILE_ACC_C64
#define HS_TILE_ACC_C64 16     // complex accumulators per thread (rows x batch), complex64
#endif
#ifndef HS_TILE_ACC_C64_OPEN
#define HS_TILE_ACC_C64_OPEN 8 // the same for open launches (out-of-tile gathers want more waves)
#endif
#ifndef HS_TILE_ACC_C128
#define HS_TILE_ACC_C128 8     // same for complex128
#endif
#ifndef HS_TILE_LDS_BYTES
#define HS_TILE_LDS_BYTES 131072 // largest staged tile (all states); the planner also
                                 // respects the device's per-workgroup LDS limit
#endif
#ifndef HS_TILE_LDS_MAX_BYTES
#define HS_TILE_LDS_MAX_BYTES 163840 // a CU's whole LDS: closed complex64 launches of 5
                                     // states stage 4096-row tiles in it
#endif
// LDS budget of a tile: the general one, or the whole LDS for the one shape
// that needs it to double its tile (5 complex64 states, closed)
constexpr int tile_lds_bytes(bool c128, int batch, bool open) {
    return (!c128 && !open && batch == 5) ? HS_TILE_LDS_MAX_BYTES : HS_TILE_LDS_BYTES;
}
constexpr int kTileThreads = HS_TILE_THREADS;

// Closed complex128 launches of two to four states run twice the default
// threads with half the rows each (2048-row tiles): 16 waves per CU instead
// of 8, measured 4-6% faster; for one state the same change was slower.
constexpr bool tile_c128_pair_wide(bool c128, int batch, bool open) {
    return c128 && !open && batch >= 2 && batch <= 4;
}
// Rows per thread for a launch of `batch` states: the accumulator budget
// split over the batch rounded up to a power of two, at least one row pair.
constexpr int tile_rpt(bool c128, int batch, bool open = false) {
    int bp = 1;
    while (bp < batch) bp <<= 1;
    if (tile_c128_pair_wide(c128, batch, open)) bp *= 2;
    const int acc = c128 ? HS_TILE_ACC_C128 : (open ? HS_TILE_ACC_C64_OPEN : HS_TILE_ACC_C64);
    if (tile_lds_bytes(c128, batch, open) > HS_TILE_LDS_BYTES) return 4;   // 4096-row tiles
    if (c128 && !open && batch == 2) return 4;   // 4096-row tiles (128 KiB): 3 launches for
                                                 // a 24-qubit MaxCut step instead of 4
    return acc / bp >= 2 ? acc / bp : 2;
}
// Threads per workgroup: closed complex64 launches of 3-8 states use twice
// the default, so a 2048-row tile (128 KiB of LDS, one workgroup per CU) still
// runs 16 waves per CU with one row pair per thread; open launches of either
// dtype do too (8192-row tiles for one state), and closed complex128
// launches of two states.
constexpr int tile_threads(bool c128, int batch, bool open = false) {
    return (open || (!c128 && batch > 2) || tile_c128_pair_wide(c128, batch, open)) ? 2 * kTileThreads
                                                                                    : kTileThreads;
}
// Rows of the largest tile: all threads' rows, capped by an LDS budget.
constexpr int tile_rows_cap(bool c128, int batch, bool open = false, int lds_bytes = HS_TILE_LDS_MAX_BYTES) {
    const int rows = tile_threads(c128, batch, open) * tile_rpt(c128, batch, open);
    const int budget = lds_bytes < tile_lds_bytes(c128, batch, open) ? lds_bytes : tile_lds_bytes(c128, batch, open);
    const int lds_rows = budget / (batch * (c128 ? 16 : 8));
    int cap = 1;
    while (cap * 2 <= rows && cap * 2 <= lds_rows) cap *= 2;
    return cap;
}

}  // namespace hs
