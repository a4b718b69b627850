// C ABI of the hamsim library (declared in include/hamsim.h): handle
// lifetime, device construction of the factor diagonals, the evolve loop
// (launch planning: tile geometry and fusion of consecutive factors), the
// generic DIA SpMV and the FP64 reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "hs_internal.h"
#include "tile_plan.h"

using hs::DiagDesc;
using hs::Factor;
using hs::Plan;
using hs::TileArgs;
using namespace hs::plan;

namespace {

thread_local std::string g_err;

hs_status fail(hs_status s, const std::string &m) {
    g_err = m;
    return s;
}

}  // namespace

namespace hs {
void set_last_error(const std::string &m) { g_err = m; }

bool device_range_ok(const void *p, size_t bytes, const char *what, std::string &msg) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        msg = std::string(what) + ": no current device";
        return false;
    }
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        msg = std::string(what) + " is not device memory (a host address?)";
        return false;
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) {
        msg = std::string(what) + " is not device memory (a host address?)";
        return false;
    }
    if (at.type == hipMemoryTypeDevice && at.device != dev) {
        msg = std::string(what) + " lives on device " + std::to_string(at.device) + ", the current device is " +
              std::to_string(dev);
        return false;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) == hipSuccess && base && size) {
        const char *lo = static_cast<const char *>(base);
        if (static_cast<const char *>(p) + bytes > lo + size) {
            msg = std::string(what) + " extends past the end of its allocation";
            return false;
        }
    } else {
        (void)hipGetLastError();      // pool allocations may not report a range
    }
    return true;
}
}  // namespace hs

namespace {

hs_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? HS_ENOMEM : HS_EDEVICE;
}

#define HS_HIP(call, what)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, what);    \
    } while (0)

struct Run {
    int first = 0;              // position of the first factor in the step sequence
    std::vector<int> factors;   // factor indices at consecutive sequence positions
    Geo geo;
    int launch_batch = 1;       // states per launch (1 when the chunk does not fit)
    bool elementwise = false;   // a single main-diagonal factor
    bool open = false;          // no closed tile holds the factor's coupling range: open
                                // launch into the scratch state, then copied back
    bool pairs = false;         // closed complex64 launch whose every diagonal pairs: the
                                // partners of a thread's two rows are adjacent LDS entries
                                // (regular offset; even-aligned unless the offset is odd)
    bool pairs_odd = false;     // ... and some offset is odd (contiguous tile, one-row windows):
                                // the pair kernel's odd-offset path
    bool perm = false;          // some diagonal is stored out of natural order (perm_pos)
    int desc_start = 0;
    std::vector<int> dstart;    // per factor, relative to desc_start (size nf + 1)
};

// The factor sequence of each part of an evolution of several steps.  With a
// joint factor J the steps of a symmetric product run s_0 .. s_{L-2} J, then
// (s_1 .. s_{L-2} J) for the middle steps, then s_1 .. s_{L-1}; part 0 is a
// lone step.  Without a joint every part is the plain step.
enum { kPartLone = 0, kPartFirst = 1, kPartMiddle = 2, kPartLast = 3, kParts = 4 };

std::vector<int> part_sequence(const Plan &P, int part) {
    const auto &q = P.seq;
    if (P.joint < 0 || part == kPartLone) return q;
    std::vector<int> out;
    const size_t L = q.size();
    const size_t a = part == kPartFirst ? 0 : 1;
    const size_t b = part == kPartLast ? L : L - 1;
    for (size_t i = a; i < b; ++i) out.push_back(q[i]);
    if (part != kPartLast) out.push_back(P.joint);
    return out;
}

struct EvolvePlan {
    int swizzle = 0;
    bool needs_scratch = false;  // some run is open
    std::vector<Run> runs[kParts];
    std::vector<DiagDesc> host_desc;
    DiagDesc *dev_desc = nullptr;
};

}  // namespace

struct hs_factors_s {
    Plan plan;
    bool built = false;
    int dtype = HS_C64;
    int device = 0;
    int *viol_dev = nullptr;
    double *work_dev = nullptr;      // [8][G][4] partials, then [8][4] records
    double *norm_dev = nullptr;      // per-tile norm partials of the step's last launch, on demand
    size_t norm_bytes = 0;
    void *scratch_dev = nullptr;     // output of open launches (HS_MAX_BATCH states), on demand
    size_t scratch_bytes = 0;
    hipStream_t alloc_stream = nullptr;   // device memory is stream-ordered on this stream
    std::map<PlanKey, EvolvePlan> plans;
    std::mutex mu;
    // whole-evolution tables (small states), built on first use
    bool whole_ready = false;
    std::vector<hs::WholeEntry> whole_walk;
    int32_t whole_part_off[5] = {0, 0, 0, 0, 0};
    hs::WholeEntry *whole_walk_dev = nullptr;
    bool any_perm = false;           // a factor is stored out of natural order (perm_pos)

    double *partials() { return work_dev; }
    double *records() { return work_dev + (size_t)HS_MAX_BATCH * hs::kReduceBlocks * 4; }

    // Stream-ordered frees (hipFree would wait for the whole device, stalling
    // other handles' work on other streams).
    ~hs_factors_s() {
        for (auto &f : plan.factors)
            if (f.dev) (void)hipFreeAsync(f.dev, alloc_stream);
        for (auto &kv : plans)
            if (kv.second.dev_desc) (void)hipFreeAsync(kv.second.dev_desc, alloc_stream);
        if (viol_dev) (void)hipFreeAsync(viol_dev, alloc_stream);
        if (scratch_dev) (void)hipFreeAsync(scratch_dev, alloc_stream);
        if (norm_dev) (void)hipFreeAsync(norm_dev, alloc_stream);
        if (work_dev) (void)hipFreeAsync(work_dev, alloc_stream);
        if (whole_walk_dev) (void)hipFreeAsync(whole_walk_dev, alloc_stream);
    }
};

namespace {

// The launches of every step part (host only): greedy fusion extends a run
// while the union of coupling hulls still fits one closed tile with rows runs
// of at least w_min elements; each run gets its tile geometry and kernel form.
void form_runs(const Plan &P, int dtype, const PlanKey &key, EvolvePlan &ep) {
    const int n = P.n;
    const int batch = key.chunk;
    const bool fuse = key.fuse != 0;
    const int Tmax = tile_rows_max(dtype, batch, P.N);
    const int Wmin = w_min(dtype, key);
    const size_t sc = elem_bytes(dtype);
    ep = EvolvePlan();
    ep.swizzle = key.swizzle;
    const int max_fuse = key.max_fuse;
    for (int part = 0; part < (P.joint < 0 ? 1 : kParts); ++part) {
        // runs are consecutive positions of the part's factor sequence
        const std::vector<int> seq = part_sequence(P, part);
        std::vector<Run> &runs = ep.runs[part];
        const int F = (int)seq.size();
        int f = 0;
        while (f < F) {
            Run run;
            run.first = f;
            run.factors.push_back(seq[f]);
            const Factor &F0 = P.factors[seq[f]];
            int lb = F0.xlb, hb = F0.xhb;
            bool empty = F0.xmask_union == 0;
            if (F0.offs.size() == 1 && F0.offs[0] == 0 && empty) {
                run.elementwise = true;
            }
            int ndiag = (int)F0.offs.size();
            int g = f + 1;
            while (fuse && g < F && (int)run.factors.size() < max_fuse) {
                const Factor &G = P.factors[seq[g]];
                int nlb = lb, nhb = hb;
                if (G.xmask_union) {
                    if (empty) { nlb = G.xlb; nhb = G.xhb; }
                    else { nlb = std::min(lb, G.xlb); nhb = std::max(hb, G.xhb); }
                }
                const Geo geo = geometry(nlb, nhb, n, Tmax);
                const bool good = geo.ok && (geo.qb == 0 || (1 << geo.logW) >= Wmin);
                if (!good || ndiag + (int)G.offs.size() > hs::kMaxDiagsPerLaunch) break;
                run.factors.push_back(seq[g]);
                run.elementwise = false;
                ndiag += (int)G.offs.size();
                lb = nlb; hb = nhb;
                if (G.xmask_union) empty = false;
                ++g;
            }
            run.launch_batch = batch;
            run.geo = geometry(empty ? 0 : lb, empty ? 0 : hb, n, Tmax);
            if (!run.geo.ok) {            // orbit wider than the batched tile: one state per launch
                run.launch_batch = 1;
                run.geo = geometry(lb, hb, n, tile_rows_max(dtype, 1, P.N));
            }
            if (!run.geo.ok) {            // no closed tile at all (a single factor): open launch
                const Factor &Fo = P.factors[run.factors[0]];
                std::vector<long long> o(Fo.offs.begin(), Fo.offs.end());
                run.launch_batch = batch;
                run.geo = generic_geometry(o.data(), (int)o.size(), P.N, dtype, batch);
                run.open = true;
                ep.needs_scratch = true;
            }
            run.pairs = key.pairs && dtype == HS_C64 && !run.open && !run.elementwise;
            bool permuted = false;
            for (int k : run.factors) permuted = permuted || P.factors[k].perm_s > 0;
            if (key.pairs == 1 && run.geo.qb > 0 && run.launch_batch == 1 && ((size_t)1 << run.geo.logW) * sc < 1024 &&
                !permuted)
                run.pairs = false;
            const int64_t lowmask = (int64_t(1) << run.geo.qb) - 1;
            // odd offsets pair in contiguous tiles (the pair kernel's odd-offset path)
            const bool odd_ok = key.pairs >= 1 && run.geo.qb == 0 && run.geo.logW == 0 && !permuted;
            for (int k : run.factors)
                for (int64_t d : P.factors[k].offs) {
                    if ((d & lowmask) != 0) run.pairs = false;
                    if (run.geo.logW == 0 && (d & 1)) {
                        if (odd_ok && P.N - (d < 0 ? -d : d) >= 2)
                            run.pairs_odd = true;
                        else
                            run.pairs = false;
                    }
                }
            if (!run.pairs) run.pairs_odd = false;
            runs.push_back(run);
            f = g;
        }
    }
    for (int part = 1; P.joint < 0 && part < kParts; ++part) ep.runs[part] = ep.runs[0];
}

// Storage order of every factor (perm_pos): a factor that the one-state plan
// (default fusion) applies only in closed strided launches, whose level
// stride 2^qb rows spans at least HAMSIM_PERM_MIN_BYTES (default 1 MiB, where
// every level of a tile lies on its own 2 MB page; 0: never), is stored with
// s = qb of the launch with the smallest qb.  Its chunks hold
// HAMSIM_PERM_CHUNK_WINDOWS (default 4) of that launch's windows of W
// consecutive rows, or HAMSIM_PERM_CHUNK_BYTES when that is set (nonzero):
// neighbouring tiles, which run at the same time on other compute units, then
// read each level's chunk together.  On the n = 26 TFIM step (complex64) the
// launch whose levels lie 2 MiB apart took 3.14 ms in natural order, 2.84 ms
// with 256-byte chunks and 2.64 ms with chunks of four windows (8 windows:
// 2.92 ms).  Levels 32 KiB apart gained 3% the same way (2.63 -> 2.55 ms), but
// launches of other batch sizes, which read the same storage through tiles of
// another shape, lost up to 2% (8 states of the n = 24 MaxCut step), so the
// default leaves them in natural order.
void choose_storage_order(Plan &P, int dtype) {
    for (auto &f : P.factors) f.perm_s = f.perm_c = 0;
    const int min_bytes = env_int("HAMSIM_PERM_MIN_BYTES", 1 << 20, 0, 1 << 30);
    if (min_bytes == 0) return;
    const size_t sc = elem_bytes(dtype);
    const int chunk_bytes = env_int("HAMSIM_PERM_CHUNK_BYTES", 0, 0, 1 << 24);
    const int chunk_windows = env_int("HAMSIM_PERM_CHUNK_WINDOWS", 4, 1, 1 << 12);
    EvolvePlan ep;
    form_runs(P, dtype, plan_key(1, true), ep);
    std::vector<int> smin(P.factors.size(), -1), wlog(P.factors.size(), 0);
    for (int part = 0; part < kParts; ++part)
        for (const Run &run : ep.runs[part]) {
            const bool strided = !run.open && !run.elementwise && run.geo.qb > 0;
            for (int k : run.factors) {
                const int q = strided ? run.geo.qb : 0;
                if (smin[k] < 0 || q < smin[k]) {
                    smin[k] = q;
                    wlog[k] = run.geo.logW;
                }
            }
        }
    for (size_t k = 0; k < P.factors.size(); ++k) {
        Factor &F = P.factors[k];
        const int q = smin[k];
        if (q <= 0 || q > 30 || ((size_t)1 << q) * sc < (size_t)min_bytes) continue;
        bool multiple = true;
        for (int64_t d : F.offs) multiple = multiple && ((d < 0 ? -d : d) & ((int64_t(1) << q) - 1)) == 0;
        if (!multiple) continue;
        // chunk entries: a power of two, at least 2 (pairs stay adjacent), at most 2^q
        const int64_t want = chunk_bytes ? (int64_t)chunk_bytes / (int64_t)sc
                                         : ((int64_t)chunk_windows << wlog[k]);
        const int c = std::min(q, std::max(1, ilog2(std::max<int64_t>(2, want))));
        F.perm_s = q;
        F.perm_c = c;
    }
}

// The runs of one plan key with their descriptors on the device.
hs_status make_evolve_plan(hs_factors_s *h, const PlanKey &key, EvolvePlan &ep, void *stream) {
    const Plan &P = h->plan;
    const size_t sc = elem_bytes(h->dtype);
    form_runs(P, h->dtype, key, ep);
    for (int part = 0; part < kParts; ++part) {
        if (part > 0 && P.joint < 0) {
            ep.runs[part] = ep.runs[0];
            continue;
        }
        for (Run &run : ep.runs[part]) {
            run.desc_start = (int)ep.host_desc.size();
            run.dstart.assign(1, 0);
            run.perm = false;
            for (int k : run.factors) {
                const Factor &Fk = P.factors[k];
                for (size_t j = 0; j < Fk.offs.size(); ++j) {
                    const int64_t d = Fk.offs[j];
                    DiagDesc dd{};
                    dd.ptr = static_cast<const char *>(Fk.dev) + Fk.elem_off[j] * sc;
                    dd.off = (int32_t)d;
                    const int64_t lowmask = (int64_t(1) << run.geo.qb) - 1;
                    dd.regular = (d & lowmask) == 0;
                    dd.m = dd.regular ? (int32_t)(d >> run.geo.qb) : 0;
                    dd.lo = (int32_t)std::max<int64_t>(0, -d);
                    dd.hi = (int32_t)std::min<int64_t>(P.N, P.N - d);
                    dd.ps = Fk.perm_s;
                    dd.pc = Fk.perm_c;
                    dd.plr = (int32_t)(((P.N - (d < 0 ? -d : d)) >> Fk.perm_s) << Fk.perm_c);
                    if (Fk.perm_s > 0) run.perm = true;
                    ep.host_desc.push_back(dd);
                }
                run.dstart.push_back((int)(ep.host_desc.size() - run.desc_start));
            }
            // out-of-order storage is read by closed tile launches only
            if (run.perm && (run.open || run.elementwise))
                return fail(HS_EDEVICE, "a factor stored out of natural order in an open or elementwise launch");
        }
    }
    const size_t bytes = ep.host_desc.size() * sizeof(DiagDesc);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&ep.dev_desc), std::max<size_t>(bytes, 64), st),
           "hipMallocAsync(descriptors)");
    // the host table lives as long as the plan, so an ordered async copy is safe
    hipError_t e = hipMemcpyAsync(ep.dev_desc, ep.host_desc.data(), bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(ep.dev_desc, st);
        ep.dev_desc = nullptr;
        return hip_fail(e, "hipMemcpy(descriptors)");
    }
    return HS_OK;
}

// Whether the step's last launch can also produce the FP64 norm partials
// (a closed tile launch whose LDS holds the per-wave sums).
bool run_makes_norm(const Run &run) { return !run.elementwise && !run.open && run.geo.T >= 64; }

hs_status launch_run(hs_factors_s *h, const EvolvePlan &ep, const Run &run, void *psi, int chunk,
                     const double *nrm2_records, void *stream, double *norm_partials = nullptr) {
    const Plan &P = h->plan;
    const bool c128 = h->dtype == HS_C128;
    const size_t sc = elem_bytes(h->dtype);
    if (run.elementwise) {
        const Factor &Fk = P.factors[run.factors[0]];
        int e = hs::launch_diag_steps(psi, psi, Fk.dev, P.N, chunk, 1, nrm2_records, c128,
                                      stream_out(chunk, P.N, h->dtype), stream);
        if (e) return hip_fail((hipError_t)e, "diag kernel launch");
        return HS_OK;
    }
    const int lbatch = run.launch_batch;
    for (int b0 = 0; b0 < chunk; b0 += lbatch) {
        TileArgs a{};
        char *p = static_cast<char *>(psi) + (size_t)b0 * P.N * sc;
        a.y = run.open ? h->scratch_dev : p;
        a.x = p;
        a.stride = P.N;
        a.N = (int32_t)P.N;
        a.nf = (int32_t)run.factors.size();
        for (int k = 0; k <= a.nf; ++k) a.dstart[k] = run.dstart[k];
        a.desc = ep.dev_desc + run.desc_start;
        a.qb = run.geo.qb;
        a.kb = run.geo.kb;
        a.logW = run.geo.logW;
        a.nlw_log = run.geo.nlw_log;
        a.T = run.geo.T;
        a.nrm2 = nrm2_records ? nrm2_records + 4 * b0 : nullptr;
        a.viol = run.open ? nullptr : h->viol_dev;
        a.swizzle = swizzled(ep.swizzle, run.geo) ? 1 : 0;
        a.stream_out = stream_out(chunk, P.N, h->dtype);
        a.pairs = run.pairs ? (run.pairs_odd ? 2 : 1) : 0;
        a.perm = run.perm ? 1 : 0;
        // partials of state b0 + b at [((b0 + b) * tiles + tile) * 4]
        a.norm_out = norm_partials ? norm_partials + (size_t)b0 * (P.N / run.geo.T) * 4 : nullptr;
        const int nb = std::min(lbatch, chunk - b0);
        int e = hs::launch_tile(a, nb, c128, !run.open, stream);
        if (e) return hip_fail((hipError_t)e, "tile kernel launch");
        if (run.open)
            HS_HIP(hipMemcpyAsync(p, h->scratch_dev, (size_t)nb * P.N * sc, hipMemcpyDeviceToDevice,
                                  reinterpret_cast<hipStream_t>(stream)), "copy back");
    }
    return HS_OK;
}

// Rows up to which hs_evolve runs a whole evolution in one launch
// (HAMSIM_WHOLE_MAX_ROWS, capped by the kernel's limit; 0 never).  The
// default is where one workgroup per state stops beating the launch per run
// and step on MI355X: 2048 complex64 rows (n <= 11: 1.3-3x faster, n = 12
// and 13 up to 2.7x slower) and 1024 complex128 rows.
int64_t whole_max_rows(int dtype) {
    const int lim = dtype == HS_C128 ? hs::kWholeRowsC128 : hs::kWholeRowsC64;
    const int dflt = dtype == HS_C128 ? 1024 : 2048;
    return env_int("HAMSIM_WHOLE_MAX_ROWS", dflt, 0, lim);
}

// The whole-evolution kernel's walk: for each step part, one entry per
// diagonal it applies, in order (factor by factor, ascending offsets).
hs_status make_whole_tables(hs_factors_s *h, void *stream) {
    const Plan &P = h->plan;
    const size_t sc = elem_bytes(h->dtype);
    h->whole_walk.clear();
    for (int q = 0; q < kParts; ++q) {
        h->whole_part_off[q] = (int32_t)h->whole_walk.size();
        for (int fi : part_sequence(P, q)) {
            const Factor &F = P.factors[fi];
            for (size_t j = 0; j < F.offs.size(); ++j) {
                const int64_t d = F.offs[j];
                hs::WholeEntry e{};
                e.ptr = static_cast<const char *>(F.dev) + F.elem_off[j] * sc;
                e.off = (int32_t)d;
                e.lo = (int32_t)std::max<int64_t>(0, -d);
                e.hi = (int32_t)std::min<int64_t>(P.N, P.N - d);
                e.last = j + 1 == F.offs.size() ? 1u : 0u;
                h->whole_walk.push_back(e);
            }
        }
    }
    h->whole_part_off[kParts] = (int32_t)h->whole_walk.size();
    if (h->whole_walk.empty()) return fail(HS_EINVAL, "no diagonals to apply");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t nw = h->whole_walk.size() * sizeof(hs::WholeEntry);
    HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&h->whole_walk_dev), nw, st), "hipMallocAsync(whole walk)");
    // the host vector lives as long as the handle, so an ordered async copy is safe
    HS_HIP(hipMemcpyAsync(h->whole_walk_dev, h->whole_walk.data(), nw, hipMemcpyHostToDevice, st), "whole walk");
    h->whole_ready = true;
    return HS_OK;
}

hs_status check_handle(hs_factors f) {
    if (!f) return fail(HS_EINVAL, "null handle");
    return HS_OK;
}

}  // namespace

extern "C" {

const char *hs_last_error(void) { return g_err.c_str(); }
int hs_abi_version(void) { return 1; }

hs_status hs_plan(int n_qubits, int n_terms, const char *const *pauli_terms, const double *coeffs,
                  double t, int steps, int budget, unsigned flags, hs_factors *out) {
    if (!out) return fail(HS_EINVAL, "null output handle");
    *out = nullptr;
    hs_factors_s *h = new (std::nothrow) hs_factors_s();
    if (!h) return fail(HS_ENOMEM, "host allocation failed");
    std::string msg;
    hs_status s = hs::make_plan(n_qubits, n_terms, pauli_terms, coeffs, t, steps, budget, flags,
                                h->plan, msg);
    if (s != HS_OK) {
        delete h;
        return fail(s, msg);
    }
    for (auto &f : h->plan.factors) hs::layout_factor(f, h->plan.N, 8);
    *out = h;
    g_err.clear();
    return HS_OK;
}

static hs_status build_device(hs_factors_s *h, void *stream) {
    Plan &P = h->plan;
    const size_t sc = elem_bytes(h->dtype);
    const bool c128 = h->dtype == HS_C128;
    HS_HIP(hipGetDevice(&h->device), "hipGetDevice");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    h->alloc_stream = st;
    choose_storage_order(P, h->dtype);
    for (auto &f : P.factors) h->any_perm = h->any_perm || f.perm_s > 0;
    for (auto &f : P.factors) {
        hs::layout_factor(f, P.N, sc);
        HS_HIP(hipMallocAsync(&f.dev, f.elems_total * sc, st), "hipMallocAsync(factor diagonals)");
    }
    HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&h->viol_dev), sizeof(int), st), "hipMallocAsync(flag)");
    HS_HIP(hipMemsetAsync(h->viol_dev, 0, sizeof(int), st), "hipMemsetAsync(flag)");
    HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&h->work_dev),
                          sizeof(double) * ((size_t)HS_MAX_BATCH * hs::kReduceBlocks * 4 + HS_MAX_BATCH * 4), st),
           "hipMallocAsync(workspace)");

    // temporaries: phase table and per-factor tables
    std::vector<void *> temps;
    std::vector<std::vector<uint64_t>> host_keep;   // sources of async uploads, alive until the sync
    std::vector<std::vector<double>> host_keep_d;
    auto cleanup = [&]() {
        for (void *p : temps) (void)hipFreeAsync(p, st);
    };
    auto upload = [&](const void *src, size_t bytes, void **dst) -> hipError_t {
        // host sources stay alive until the stream is synchronised below
        hipError_t e = hipMallocAsync(dst, std::max<size_t>(bytes, 16), st);
        if (e != hipSuccess) return e;
        temps.push_back(*dst);
        return hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    void *dzm = nullptr, *dcf = nullptr;
    if (!P.diag.empty()) {
        host_keep.emplace_back();
        host_keep_d.emplace_back();
        std::vector<uint64_t> &zm = host_keep.back();
        std::vector<double> &cf = host_keep_d.back();
        for (int k : P.diag) {
            zm.push_back(P.terms[k].z);
            cf.push_back(P.terms[k].c);
        }
        if ((e = upload(zm.data(), zm.size() * 8, &dzm)) != hipSuccess ||
            (e = upload(cf.data(), cf.size() * 8, &dcf)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "phase table setup");
        }
    }
    // one FP64 phase table exp(-i h E(x)) per distinct time step h of the
    // factors that carry D
    std::map<double, double *> phases;
    for (auto &f : P.factors) {
        if (!f.has_diag || phases.count(f.dt)) continue;
        double *phase = nullptr;
        if ((e = hipMallocAsync(reinterpret_cast<void **>(&phase), (size_t)P.N * 16, st)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "phase table setup");
        }
        temps.push_back(phase);
        int le = hs::launch_phase_table(P.N, (int)P.diag.size(), static_cast<uint64_t *>(dzm),
                                        static_cast<double *>(dcf), f.dt, phase, stream);
        if (le) { cleanup(); return hip_fail((hipError_t)le, "phase table kernel"); }
        phases[f.dt] = phase;
    }
    for (auto &f : P.factors) {
        hs::ConstructArgs a{};
        a.base = f.dev;
        a.N = (int32_t)P.N;
        a.smask = (uint32_t)f.smask;
        host_keep.emplace_back(f.elem_off.begin(), f.elem_off.end());
        const std::vector<uint64_t> &eo = host_keep.back();
        void *doffs = nullptr, *deo = nullptr, *dL = nullptr;
        if ((e = upload(f.offs.data(), f.offs.size() * 8, &doffs)) != hipSuccess ||
            (e = upload(eo.data(), eo.size() * 8, &deo)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "factor table upload");
        }
        a.offs = static_cast<int64_t *>(doffs);
        a.elem_off = static_cast<uint64_t *>(deo);
        if (!f.terms.empty()) {
            if ((e = upload(f.L.data(), f.L.size() * 16, &dL)) != hipSuccess) {
                cleanup();
                return hip_fail(e, "local unitary upload");
            }
            a.L = static_cast<double *>(dL);
            a.K = 1 << f.bits.size();
            a.nbits = (int)f.bits.size();
            for (int q = 0; q < a.nbits; ++q) a.bits[q] = (int8_t)f.bits[q];
            a.lb = f.bits.empty() ? 0 : f.bits[0];
            a.contiguous = f.bits.empty() || f.bits.back() - f.bits.front() + 1 == (int)f.bits.size();
        } else {
            a.L = nullptr;
            a.K = 1;
        }
        a.phase = f.has_diag ? phases[f.dt] : nullptr;
        a.perm_s = f.perm_s;
        a.perm_c = f.perm_c;
        int le = hs::launch_construct(a, (int)f.offs.size(), P.N, c128, stream);
        if (le) { cleanup(); return hip_fail((hipError_t)le, "construct kernel"); }
    }
    e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    cleanup();
    if (e != hipSuccess) return hip_fail(e, "construction");
    h->built = true;
    return HS_OK;
}

hs_status hs_build_factors(int n_qubits, int n_terms, const char *const *pauli_terms,
                           const double *coeffs, double t, int steps, int budget, hs_dtype dtype,
                           unsigned flags, void *stream, hs_factors *out) {
    if (!out) return fail(HS_EINVAL, "null output handle");
    *out = nullptr;
    if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_EINVAL, "dtype must be HS_C64 or HS_C128");
    hs_factors h = nullptr;
    hs_status s = hs_plan(n_qubits, n_terms, pauli_terms, coeffs, t, steps, budget, flags, &h);
    if (s != HS_OK) return s;
    h->dtype = dtype;
    s = build_device(h, stream);
    if (s != HS_OK) {
        std::string keep = g_err;
        delete h;
        g_err = keep;
        return s;
    }
    *out = h;
    g_err.clear();
    return HS_OK;
}

hs_status hs_evolve(hs_factors f, void *psi, int batch, int steps, void *stream, unsigned flags) {
    if (hs_status s = check_handle(f)) return s;
    if (!f->built) return fail(HS_EINVAL, "handle was planned, not built");
    if (!psi) return fail(HS_EINVAL, "null state pointer");
    if (batch < 1) return fail(HS_EINVAL, "batch must be >= 1");
    if (steps < 0) return fail(HS_EINVAL, "steps must be >= 0");
    if (flags & ~(unsigned)(HS_RENORM | HS_NO_FUSE)) return fail(HS_EINVAL, "unknown evolve flag");
    if (reinterpret_cast<uintptr_t>(psi) % 16) return fail(HS_EINVAL, "state pointer must be 16-byte aligned");
    const Plan &P = f->plan;
    const size_t sc = elem_bytes(f->dtype);
    {
        // checked before the zero-step return, so a caller can validate a
        // state without enqueuing work
        std::string msg;
        if (!hs::device_range_ok(psi, (size_t)batch * P.N * sc, "state", msg)) return fail(HS_EINVAL, msg);
    }
    if (steps == 0) return HS_OK;
    std::lock_guard<std::mutex> lock(f->mu);
    int cur_dev = 0;
    HS_HIP(hipGetDevice(&cur_dev), "hipGetDevice");
    if (cur_dev != f->device) return fail(HS_EINVAL, "current device differs from the build device");
    if (!(flags & (HS_RENORM | HS_NO_FUSE)) && P.N <= whole_max_rows(f->dtype) && !f->any_perm) {
        // a small state: the whole evolution of every state in one launch
        if (!f->whole_ready)
            if (hs_status s = make_whole_tables(f, stream)) return s;
        hs::WholeArgs w{};
        w.psi = psi;
        w.stride = P.N;
        w.N = (int32_t)P.N;
        w.steps = steps;
        w.walk = f->whole_walk_dev;
        for (int q = 0; q <= kParts; ++q) w.part_off[q] = f->whole_part_off[q];
        int e = hs::launch_whole(w, batch, f->dtype == HS_C128, stream);
        if (e) return hip_fail((hipError_t)e, "whole-evolution kernel launch");
        return HS_OK;
    }
    const bool fuse = !(flags & HS_NO_FUSE);
    const bool renorm = (flags & HS_RENORM) != 0;
    for (int c0 = 0; c0 < batch; c0 += HS_MAX_BATCH) {
        const int chunk = std::min(HS_MAX_BATCH, batch - c0);
        const PlanKey key = plan_key(chunk, fuse);
        auto it = f->plans.find(key);
        if (it == f->plans.end()) {
            EvolvePlan ep;
            if (hs_status s = make_evolve_plan(f, key, ep, stream)) return s;
            it = f->plans.emplace(key, std::move(ep)).first;
        }
        const EvolvePlan &ep = it->second;
        if (ep.needs_scratch && f->scratch_bytes < (size_t)chunk * P.N * sc) {
            // stream-ordered: the old buffer's last use precedes this point on `stream`
            hipStream_t hst = reinterpret_cast<hipStream_t>(stream);
            if (f->scratch_dev) HS_HIP(hipFreeAsync(f->scratch_dev, hst), "hipFreeAsync(scratch)");
            f->scratch_dev = nullptr;
            f->scratch_bytes = 0;
            const size_t bytes = (size_t)chunk * P.N * sc;
            HS_HIP(hipMallocAsync(&f->scratch_dev, bytes, hst), "hipMallocAsync(scratch)");
            f->scratch_bytes = bytes;
        }
        if (renorm) {
            // the step's last launch sums |y|^2 per tile: room for its partials
            size_t need = 0;
            for (int q = 0; q < kParts; ++q)
                if (!ep.runs[q].empty() && run_makes_norm(ep.runs[q].back()))
                    need = std::max(need, (size_t)chunk * (P.N / ep.runs[q].back().geo.T) * 4 * sizeof(double));
            if (need > f->norm_bytes) {
                hipStream_t hst = reinterpret_cast<hipStream_t>(stream);
                if (f->norm_dev) HS_HIP(hipFreeAsync(f->norm_dev, hst), "hipFreeAsync(norm partials)");
                f->norm_dev = nullptr;
                f->norm_bytes = 0;
                HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&f->norm_dev), need, hst),
                       "hipMallocAsync(norm partials)");
                f->norm_bytes = need;
            }
        }
        void *p = static_cast<char *>(psi) + (size_t)c0 * P.N * sc;
        const std::vector<Run> &lone = ep.runs[kPartLone];
        if (!renorm && P.joint < 0 && lone.size() == 1 && lone[0].elementwise) {
            // a step that is one diagonal factor: all steps in one pass (the
            // same multiplications, one step after the other, per entry)
            const Factor &Fk = P.factors[lone[0].factors[0]];
            int e = hs::launch_diag_steps(p, p, Fk.dev, P.N, chunk, steps, nullptr, f->dtype == HS_C128,
                                          stream_out(chunk, P.N, f->dtype), stream);
            if (e) return hip_fail((hipError_t)e, "diag kernel launch");
            continue;
        }
        const double *rec = f->records() + 2;    // squared norm of state b at rec[4 b]
        for (int s = 0; s < steps; ++s) {
            const int part = steps == 1 ? kPartLone
                             : s == 0 ? kPartFirst : s == steps - 1 ? kPartLast : kPartMiddle;
            const std::vector<Run> &runs = ep.runs[part];
            const bool fused_norm = renorm && run_makes_norm(runs.back());
            for (size_t ri = 0; ri < runs.size(); ++ri) {
                const double *nrm = (renorm && s > 0 && ri == 0) ? rec : nullptr;
                double *np = (fused_norm && ri + 1 == runs.size()) ? f->norm_dev : nullptr;
                if (hs_status st = launch_run(f, ep, runs[ri], p, chunk, nrm, stream, np)) return st;
            }
            if (fused_norm) {
                const int tiles = (int)(P.N / runs.back().geo.T);
                int e = hs::launch_reduce_partials(f->norm_dev, tiles, chunk, f->records(), stream);
                if (e) return hip_fail((hipError_t)e, "norm reduction");
            } else if (renorm) {
                int e = hs::launch_reduce(p, f->dtype, p, f->dtype, chunk, P.N, f->partials(),
                                          hs::kReduceBlocks, f->records(), false, stream);
                if (e) return hip_fail((hipError_t)e, "norm reduction");
            }
        }
        if (renorm) {
            int e = hs::launch_scale(p, P.N, chunk, rec, f->dtype == HS_C128, stream);
            if (e) return hip_fail((hipError_t)e, "scale kernel");
        }
    }
    return HS_OK;
}

hs_status hs_factors_info(hs_factors f, int *n_qubits, int *n_factors, int *n_terms,
                          int *n_diag_terms, int *dtype, double *dt, int *steps) {
    if (hs_status s = check_handle(f)) return s;
    if (n_qubits) *n_qubits = f->plan.n;
    if (n_factors) *n_factors = (int)f->plan.factors.size();
    if (n_terms) *n_terms = (int)f->plan.terms.size();
    if (n_diag_terms) *n_diag_terms = (int)f->plan.diag.size();
    if (dtype) *dtype = f->dtype;
    if (dt) *dt = f->plan.dt;
    if (steps) *steps = f->plan.steps;
    return HS_OK;
}

hs_status hs_diag_terms(hs_factors f, int *term_idx, int cap) {
    if (hs_status s = check_handle(f)) return s;
    if (cap < (int)f->plan.diag.size() || (!term_idx && !f->plan.diag.empty()))
        return fail(HS_EINVAL, "output too small");
    std::copy(f->plan.diag.begin(), f->plan.diag.end(), term_idx);
    return HS_OK;
}

static hs_status get_factor(hs_factors f, int k, const Factor **out) {
    if (hs_status s = check_handle(f)) return s;
    if (k < 0 || k >= (int)f->plan.factors.size()) return fail(HS_EINVAL, "factor index out of range");
    *out = &f->plan.factors[k];
    return HS_OK;
}

hs_status hs_factor_info(hs_factors f, int k, int *has_diag, int *n_group_terms, int *n_diags,
                         unsigned long long *support_mask, size_t *bytes) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (has_diag) *has_diag = F->has_diag ? 1 : 0;
    if (n_group_terms) *n_group_terms = (int)F->terms.size();
    if (n_diags) *n_diags = (int)F->offs.size();
    if (support_mask) *support_mask = F->smask;
    if (bytes) *bytes = F->elems_total * elem_bytes(f->dtype);
    return HS_OK;
}

hs_status hs_step_sequence(hs_factors f, int *seq, int cap, int *len) {
    if (hs_status s = check_handle(f)) return s;
    const auto &q = f->plan.seq;
    if (len) *len = (int)q.size();
    if (seq) {
        if (cap < (int)q.size()) return fail(HS_EINVAL, "output too small");
        std::copy(q.begin(), q.end(), seq);
    }
    return HS_OK;
}

hs_status hs_step_joint(hs_factors f, int *factor) {
    if (hs_status s = check_handle(f)) return s;
    if (!factor) return fail(HS_EINVAL, "null output");
    *factor = f->plan.joint;
    return HS_OK;
}

hs_status hs_factor_step(hs_factors f, int k, double *h) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (!h) return fail(HS_EINVAL, "null output");
    *h = F->dt;
    return HS_OK;
}

hs_status hs_factor_terms(hs_factors f, int k, int *term_idx, int cap) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (cap < (int)F->terms.size() || (!term_idx && !F->terms.empty())) return fail(HS_EINVAL, "output too small");
    std::copy(F->terms.begin(), F->terms.end(), term_idx);
    return HS_OK;
}

hs_status hs_factor_offsets(hs_factors f, int k, long long *offsets, int cap) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (cap < (int)F->offs.size() || !offsets) return fail(HS_EINVAL, "output too small");
    for (size_t j = 0; j < F->offs.size(); ++j) offsets[j] = (long long)F->offs[j];
    return HS_OK;
}

hs_status hs_factor_copy_diagonal(hs_factors f, int k, int j, long long start, long long count,
                                  void *host_dst, void *stream) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (!f->built) return fail(HS_EINVAL, "handle was planned, not built");
    if (j < 0 || j >= (int)F->offs.size()) return fail(HS_EINVAL, "diagonal index out of range");
    const int64_t d = F->offs[j];
    const long long len = f->plan.N - (d < 0 ? -d : d);
    if (start < 0 || count < 0 || start + count > len || !host_dst)
        return fail(HS_EINVAL, "range outside the diagonal's N - |d| entries");
    if (count == 0) return HS_OK;
    const size_t sc = elem_bytes(f->dtype);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const char *src = static_cast<const char *>(F->dev) + F->elem_off[j] * sc;
    if (F->perm_s == 0) {
        HS_HIP(hipMemcpyAsync(host_dst, src + (size_t)start * sc, (size_t)count * sc, hipMemcpyDeviceToHost, st),
               "hipMemcpyAsync(diagonal)");
        HS_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        return HS_OK;
    }
    // stored out of natural order: gather the range in pieces of at most
    // 2^22 entries into a temporary, copying each piece to the host
    const long long piece = std::min<long long>(count, 1ll << 22);
    void *tmp = nullptr;
    HS_HIP(hipMallocAsync(&tmp, (size_t)piece * sc, st), "hipMallocAsync(diagonal copy)");
    hipError_t he = hipSuccess;
    for (long long k0 = 0; k0 < count && he == hipSuccess; k0 += piece) {
        const long long m = std::min(piece, count - k0);
        const int e = hs::launch_perm_gather(src, tmp, start + k0, m, len, F->perm_s, F->perm_c,
                                             f->dtype == HS_C128, stream);
        he = e ? (hipError_t)e
               : hipMemcpyAsync(static_cast<char *>(host_dst) + (size_t)k0 * sc, tmp, (size_t)m * sc,
                                hipMemcpyDeviceToHost, st);
        // the next piece reuses the temporary: wait for this copy first
        if (he == hipSuccess) he = hipStreamSynchronize(st);
    }
    const hipError_t fe = hipFreeAsync(tmp, st);
    const hipError_t se = hipStreamSynchronize(st);
    if (he != hipSuccess) return hip_fail(he, "diagonal gather");
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync(diagonal copy)");
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    return HS_OK;
}

hs_status hs_factor_storage(hs_factors f, int k, int *split_bit, int *chunk_bits) {
    const Factor *F = nullptr;
    if (hs_status s = get_factor(f, k, &F)) return s;
    if (split_bit) *split_bit = F->perm_s;
    if (chunk_bits) *chunk_bits = F->perm_c;
    return HS_OK;
}

hs_status hs_step_launches(hs_factors f, int batch, unsigned flags, int part, int *n_launches,
                           int *first_factor, int *n_factors, int cap) {
    if (hs_status s = check_handle(f)) return s;
    if (!f->built) return fail(HS_EINVAL, "handle was planned, not built");
    if (batch < 1 || !n_launches) return fail(HS_EINVAL, "batch >= 1 and an output are required");
    if (part < 0 || part >= kParts) return fail(HS_EINVAL, "part must be 0..3");
    if (flags & ~(unsigned)(HS_RENORM | HS_NO_FUSE)) return fail(HS_EINVAL, "unknown evolve flag");
    std::lock_guard<std::mutex> lock(f->mu);
    const int chunk = std::min(HS_MAX_BATCH, batch);
    const bool fuse = !(flags & HS_NO_FUSE);
    const PlanKey key = plan_key(chunk, fuse);
    auto it = f->plans.find(key);
    if (it == f->plans.end()) {
        EvolvePlan ep;
        if (hs_status s = make_evolve_plan(f, key, ep, f->alloc_stream)) return s;
        it = f->plans.emplace(key, std::move(ep)).first;
        HS_HIP(hipStreamSynchronize(f->alloc_stream), "hipStreamSynchronize");
    }
    const auto &runs = it->second.runs[part];
    *n_launches = (int)runs.size();
    if (first_factor && n_factors) {
        if (cap < (int)runs.size()) return fail(HS_EINVAL, "output too small");
        for (size_t i = 0; i < runs.size(); ++i) {
            first_factor[i] = runs[i].first;
            n_factors[i] = (int)runs[i].factors.size();
        }
    }
    return HS_OK;
}

static size_t footprint_bytes(const Plan &P, int dtype, int batch) {
    const size_t sc = elem_bytes(dtype);
    size_t total = 0;
    for (const auto &F : P.factors) {
        const size_t align = hs::kDiagAlignBytes / sc;
        for (int64_t d : F.offs) {
            const size_t len = (size_t)(P.N - (d < 0 ? -d : d));
            total += (len + align - 1) / align * align * sc;
        }
    }
    total += (size_t)batch * P.N * sc;                                // the states
    bool open = false;                                                // a factor no closed tile holds
    for (const auto &F : P.factors)
        if (F.xmask_union && !geometry(F.xlb, F.xhb, P.n, tile_rows_max(dtype, 1, P.N)).ok) open = true;
    if (open) total += (size_t)std::min(batch, HS_MAX_BATCH) * P.N * sc;   // its scratch state
    // per-tile norm partials when renormalising (tiles of at least 64 rows)
    total += (size_t)std::min(batch, HS_MAX_BATCH) * (size_t)(P.N / 64 + 1) * 4 * sizeof(double);
    total += sizeof(double) * ((size_t)HS_MAX_BATCH * hs::kReduceBlocks * 4 + HS_MAX_BATCH * 4);
    total += 64 * 1024;                                               // descriptors, flag
    return total;
}

hs_status hs_footprint(hs_factors f, int batch, size_t *bytes) {
    if (hs_status s = check_handle(f)) return s;
    if (batch < 1 || !bytes) return fail(HS_EINVAL, "batch >= 1 and an output are required");
    *bytes = footprint_bytes(f->plan, f->dtype, batch);
    return HS_OK;
}

hs_status hs_footprint_dtype(hs_factors f, int batch, hs_dtype dtype, size_t *bytes) {
    if (hs_status s = check_handle(f)) return s;
    if (batch < 1 || !bytes) return fail(HS_EINVAL, "batch >= 1 and an output are required");
    if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_EINVAL, "dtype must be HS_C64 or HS_C128");
    *bytes = footprint_bytes(f->plan, dtype, batch);
    return HS_OK;
}

hs_status hs_check(hs_factors f, void *stream, int *violated) {
    if (hs_status s = check_handle(f)) return s;
    if (!f->built || !violated) return fail(HS_EINVAL, "built handle and output required");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int v = 0;
    HS_HIP(hipMemcpyAsync(&v, f->viol_dev, sizeof(int), hipMemcpyDeviceToHost, st), "hipMemcpyAsync(flag)");
    HS_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    *violated = v;
    return HS_OK;
}

hs_status hs_free_factors(hs_factors f) {
    if (!f) return HS_OK;
    delete f;
    return HS_OK;
}

hs_status hs_dia_spmv(int n_diags, const long long *offsets, const void *const *diags, const void *x,
                      void *y, int batch, long long N, hs_dtype dtype, void *stream) {
    if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_EINVAL, "bad dtype");
    if (n_diags < 1 || n_diags > 65535 || !offsets || !diags || !x || !y || batch < 1)
        return fail(HS_EINVAL, "bad arguments");
    if (N < 1 || N > (1ll << HS_MAX_QUBITS)) return fail(HS_EINVAL, "N must be in [1, 2^30]");
    const size_t sc = elem_bytes(dtype);
    const char *xb = static_cast<const char *>(x);
    char *yb = static_cast<char *>(y);
    const size_t span = (size_t)batch * N * sc;
    if (xb < yb + span && yb < xb + span) return fail(HS_EINVAL, "x and y overlap");
    if (reinterpret_cast<uintptr_t>(x) % 16 || reinterpret_cast<uintptr_t>(y) % 16)
        return fail(HS_EINVAL, "x and y must be 16-byte aligned");
    for (int j = 0; j < n_diags; ++j) {
        if (offsets[j] <= -N || offsets[j] >= N) return fail(HS_EINVAL, "offset out of range");
        if (j && offsets[j] <= offsets[j - 1]) return fail(HS_EINVAL, "offsets must ascend strictly");
        if (!diags[j]) return fail(HS_EINVAL, "null diagonal pointer");
        if (reinterpret_cast<uintptr_t>(diags[j]) % 16) return fail(HS_EINVAL, "diagonals must be 16-byte aligned");
        std::string msg;
        const size_t len = (size_t)(N - (offsets[j] < 0 ? -offsets[j] : offsets[j]));
        if (!hs::device_range_ok(diags[j], len * sc, "diagonal", msg)) return fail(HS_EINVAL, msg);
    }
    {
        std::string msg;
        if (!hs::device_range_ok(x, span, "x", msg) || !hs::device_range_ok(y, span, "y", msg))
            return fail(HS_EINVAL, msg);
    }
    std::vector<DiagDesc> hd;
    for (int c0 = 0; c0 < batch; c0 += HS_MAX_BATCH) {
        const int chunk = std::min(HS_MAX_BATCH, batch - c0);
        const Geo geo = generic_geometry(offsets, n_diags, N, dtype, chunk);
        fill_descs(offsets, diags, n_diags, N, geo, hd);
        DiagDesc *ddev = nullptr;
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&ddev), sizeof(DiagDesc) * n_diags, st),
               "hipMallocAsync(descriptors)");
        hipError_t e = hipMemcpyAsync(ddev, hd.data(), sizeof(DiagDesc) * n_diags, hipMemcpyHostToDevice, st);
        TileArgs a = open_args(geo, ddev, n_diags, xb + (size_t)c0 * N * sc, yb + (size_t)c0 * N * sc, N);
        a.stream_out = stream_out(chunk, N, dtype);
        if (e == hipSuccess) e = (hipError_t)hs::launch_tile(a, chunk, dtype == HS_C128, false, stream);
        hipError_t e2 = hipStreamSynchronize(st);
        (void)hipFreeAsync(ddev, st);
        if (e != hipSuccess) return hip_fail(e, "dia_spmv launch");
        if (e2 != hipSuccess) return hip_fail(e2, "dia_spmv");
    }
    return HS_OK;
}

static hs_status reduce_call(const void *A, int ta, const void *B, int tb, int batch, long long N,
                             void *stream, bool dot, std::vector<double> &rec) {
    const int G = hs::kReduceBlocks;
    double *work = nullptr;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    HS_HIP(hipMallocAsync(reinterpret_cast<void **>(&work), sizeof(double) * ((size_t)batch * G * 4 + (size_t)batch * 4), st),
           "hipMallocAsync(reduce)");
    double *out = work + (size_t)batch * G * 4;
    int le = hs::launch_reduce(A, ta, B, tb, batch, N, work, G, out, dot, stream);
    rec.assign((size_t)batch * 4, 0.0);
    hipError_t e = (hipError_t)le;
    if (e == hipSuccess) e = hipMemcpyAsync(rec.data(), out, sizeof(double) * batch * 4, hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFreeAsync(work, st);
    if (e != hipSuccess) return hip_fail(e, "reduction");
    if (e2 != hipSuccess) return hip_fail(e2, "reduction");
    return HS_OK;
}

hs_status hs_norm2(const void *psi, int batch, long long N, hs_dtype dtype, void *stream, double *out) {
    if (!psi || !out || batch < 1 || N < 1) return fail(HS_EINVAL, "bad arguments");
    if (dtype != HS_C64 && dtype != HS_C128) return fail(HS_EINVAL, "bad dtype");
    {
        std::string msg;
        if (!hs::device_range_ok(psi, (size_t)batch * N * elem_bytes(dtype), "state", msg)) return fail(HS_EINVAL, msg);
    }
    std::vector<double> rec;
    if (hs_status s = reduce_call(psi, dtype, psi, dtype, batch, N, stream, false, rec)) return s;
    for (int b = 0; b < batch; ++b) out[b] = rec[4 * b + 2];
    return HS_OK;
}

hs_status hs_fidelity(const void *phi, int phi_dtype, const void *psi, int psi_dtype, int batch,
                      long long N, void *stream, double *out) {
    if (!phi || !psi || !out || batch < 1 || N < 1) return fail(HS_EINVAL, "bad arguments");
    for (int t : {phi_dtype, psi_dtype})
        if (t != HS_C64 && t != HS_C128) return fail(HS_EINVAL, "bad dtype");
    {
        std::string msg;
        if (!hs::device_range_ok(phi, (size_t)batch * N * elem_bytes(phi_dtype), "phi", msg) ||
            !hs::device_range_ok(psi, (size_t)batch * N * elem_bytes(psi_dtype), "psi", msg))
            return fail(HS_EINVAL, msg);
    }
    std::vector<double> rec;
    if (hs_status s = reduce_call(phi, phi_dtype, psi, psi_dtype, batch, N, stream, true, rec)) return s;
    for (int b = 0; b < batch; ++b) {
        const double re = rec[4 * b], im = rec[4 * b + 1], np = rec[4 * b + 2], nq = rec[4 * b + 3];
        out[5 * b + 0] = re;
        out[5 * b + 1] = im;
        out[5 * b + 2] = np;
        out[5 * b + 3] = nq;
        out[5 * b + 4] = (re * re + im * im) / (np * nq);
    }
    return HS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- no allocation
//
// Scratch of hs_fidelity_noalloc: the FP64 reduction partials of up to
// HS_MAX_BATCH states ([8][kReduceBlocks][4]) and their records ([8][4]),
// 256.25 KiB in every GPU the library runs on, held until the process ends.
// Host code never uses the array's name as an address: each device's copy is
// found once with hipGetSymbolAddress and its pointer kept per device.
namespace {
constexpr size_t kNoAllocPartials = (size_t)HS_MAX_BATCH * hs::kReduceBlocks * 4;
constexpr size_t kNoAllocDoubles = kNoAllocPartials + (size_t)HS_MAX_BATCH * 4;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

static double *noalloc_scratch(std::string &msg) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        msg = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    if (dev < 0 || dev >= kNoAllocDevices) {
        msg = "device index beyond the 64 devices the scratch table covers";
        return nullptr;
    }
    static std::mutex mu;
    static double *ptr[kNoAllocDevices] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        ptr[dev] = static_cast<double *>(p);
    }
    return ptr[dev];
}

extern "C" hs_status hs_fidelity_noalloc(const void *phi, int phi_dtype, const void *psi, int psi_dtype, int batch,
                                         long long N, void *stream, double *out_dev) {
    if (!phi || !psi || !out_dev || N < 1) return fail(HS_EINVAL, "bad arguments");
    if (batch < 1 || batch > HS_MAX_BATCH)
        return fail(HS_EINVAL, "batch must be 1.." + std::to_string(HS_MAX_BATCH) +
                                   ": the static scratch holds the partial sums of that many states");
    for (int t : {phi_dtype, psi_dtype})
        if (t != HS_C64 && t != HS_C128) return fail(HS_EINVAL, "bad dtype");
    std::string msg;
    if (!hs::device_range_ok(phi, (size_t)batch * N * elem_bytes(phi_dtype), "phi", msg) ||
        !hs::device_range_ok(psi, (size_t)batch * N * elem_bytes(psi_dtype), "psi", msg) ||
        !hs::device_range_ok(out_dev, (size_t)batch * 5 * sizeof(double), "out", msg))
        return fail(HS_EINVAL, msg);
    double *s = noalloc_scratch(msg);
    if (!s) return fail(HS_EDEVICE, msg);
    double *rec = s + kNoAllocPartials;
    // every partial and record the kernels read is written by this call first
    int e = hs::launch_reduce(phi, phi_dtype, psi, psi_dtype, batch, N, s, hs::kReduceBlocks, rec, true, stream);
    if (e) return hip_fail((hipError_t)e, "reduction");
    e = hs::launch_fidelity_records(rec, batch, out_dev, stream);
    if (e) return hip_fail((hipError_t)e, "fidelity records");
    return HS_OK;
}
