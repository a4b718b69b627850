// C ABI for general operators in the diagonal layout (declared in
// include/hamsim.h): construction from Pauli strings, SpGEMM, the truncated
// Taylor exponential (paper: Alg. 2), the diagonal-budget step search
// (Section 3.1 flowchart, Eq. 5) and the single-propagator simulation loop
// (Alg. 3).  Entries are FP64 complex unless converted to complex64 for the
// state update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "hs_internal.h"
#include "tile_plan.h"

using namespace hs::plan;
using hs::DiagDesc;
using hs::TileArgs;

namespace {
hs_status dfail(hs_status s, const std::string &m);
}  // namespace

struct hs_dia_s {
    int64_t N = 0;
    int dtype = HS_C128;
    std::vector<int64_t> offs;          // ascending
    std::vector<void *> ptr;            // one stream-ordered allocation per diagonal
    hipStream_t st = nullptr;           // allocation stream
    int64_t *d_offs = nullptr;          // device copies of offs / ptr (lazy)
    void **d_ptrs = nullptr;

    size_t elem() const { return dtype == HS_C128 ? 16 : 8; }
    int64_t len(size_t j) const { return N - (offs[j] < 0 ? -offs[j] : offs[j]); }
    ~hs_dia_s() {
        for (void *p : ptr)
            if (p) (void)hipFreeAsync(p, st);
        if (d_offs) (void)hipFreeAsync(d_offs, st);
        if (d_ptrs) (void)hipFreeAsync(d_ptrs, st);
    }
};

namespace {

hs_status dfail(hs_status s, const std::string &m) {
    hs::set_last_error(m);
    return s;
}

hs_status dhip(hipError_t e, const char *what) {
    hs::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? HS_ENOMEM : HS_EDEVICE;
}

#define DHIP(call, what)                                  \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return dhip(e_, what);      \
    } while (0)

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// empty operator with the given offsets, diagonals allocated (not filled)
hs_status dia_alloc(int64_t N, int dtype, const std::vector<int64_t> &offs, hipStream_t st, hs_dia *out) {
    *out = nullptr;
    hs_dia A = new (std::nothrow) hs_dia_s();
    if (!A) return dfail(HS_ENOMEM, "host allocation failed");
    A->N = N;
    A->dtype = dtype;
    A->offs = offs;
    A->st = st;
    A->ptr.assign(offs.size(), nullptr);
    for (size_t j = 0; j < offs.size(); ++j) {
        hipError_t e = hipMallocAsync(&A->ptr[j], std::max<size_t>(16, (size_t)A->len(j) * A->elem()), st);
        if (e != hipSuccess) {
            delete A;
            return dhip(e, "hipMallocAsync(diagonal)");
        }
    }
    *out = A;
    return HS_OK;
}

hs_status dia_tables(hs_dia A) {
    if (A->d_offs) return HS_OK;
    const size_t nd = std::max<size_t>(1, A->offs.size());
    DHIP(hipMallocAsync(reinterpret_cast<void **>(&A->d_offs), nd * 8, A->st), "hipMallocAsync(table)");
    DHIP(hipMallocAsync(reinterpret_cast<void **>(&A->d_ptrs), nd * 8, A->st), "hipMallocAsync(table)");
    // host vectors live as long as A
    DHIP(hipMemcpyAsync(A->d_offs, A->offs.data(), A->offs.size() * 8, hipMemcpyHostToDevice, A->st), "upload");
    DHIP(hipMemcpyAsync(A->d_ptrs, A->ptr.data(), A->ptr.size() * 8, hipMemcpyHostToDevice, A->st), "upload");
    return HS_OK;
}

// temporary device copies of host tables, freed stream-ordered
struct Temps {
    hipStream_t st;
    std::vector<void *> ptrs;
    explicit Temps(hipStream_t s) : st(s) {}
    ~Temps() {
        for (void *p : ptrs) (void)hipFreeAsync(p, st);
    }
    template <typename T>
    hipError_t up(const std::vector<T> &v, T **dst) {
        void *p = nullptr;
        hipError_t e = hipMallocAsync(&p, std::max<size_t>(16, v.size() * sizeof(T)), st);
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        *dst = static_cast<T *>(p);
        if (v.empty()) return hipSuccess;
        return hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    }
};

hs_status max_of_blocks(double *dev, size_t count, hipStream_t st, double *out) {
    std::vector<double> h(count);
    DHIP(hipMemcpyAsync(h.data(), dev, count * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    double m = 0.0;
    for (double v : h) m = std::max(m, v);
    *out = m;
    return HS_OK;
}

// C = scale * A B (A, B FP64).  store == false computes only the largest entry
// modulus (no output allocated).  Offsets of C: every a + b in (-N, N).
hs_status spgemm(hs_dia A, hs_dia B, double sre, double sim, bool store, hipStream_t st, hs_dia *C,
                 double *norm) {
    const int64_t N = A->N;
    std::map<int64_t, std::vector<std::pair<int, int>>> contrib;
    for (size_t ia = 0; ia < A->offs.size(); ++ia)
        for (size_t ib = 0; ib < B->offs.size(); ++ib) {
            const int64_t c = A->offs[ia] + B->offs[ib];
            if (c <= -N || c >= N) continue;
            contrib[c].push_back({(int)ia, (int)ib});
        }
    std::vector<int64_t> coffs;
    std::vector<int> cptr{0}, pairs;
    for (auto &kv : contrib) {
        coffs.push_back(kv.first);
        for (auto &pq : kv.second) {
            pairs.push_back(pq.first);
            pairs.push_back(pq.second);
        }
        cptr.push_back((int)pairs.size() / 2);
    }
    if (coffs.size() > 65535) return dfail(HS_ETOOLARGE, "product has more than 65535 diagonals");
    hs_dia Cn = nullptr;
    if (store) {
        if (hs_status s = dia_alloc(N, HS_C128, coffs, st, &Cn)) return s;
    }
    if (hs_status s = dia_tables(A)) { delete Cn; return s; }
    if (hs_status s = dia_tables(B)) { delete Cn; return s; }
    Temps tmp(st);
    hs::SpgemmArgs a{};
    a.N = N;
    a.a_offs = A->d_offs;
    a.a_ptr = reinterpret_cast<const double *const *>(A->d_ptrs);
    a.b_ptr = reinterpret_cast<const double *const *>(B->d_ptrs);
    a.scale_re = sre;
    a.scale_im = sim;
    int64_t *dco = nullptr;
    int *dcp = nullptr, *dpairs = nullptr;
    double **dcptr = nullptr;
    std::vector<double *> cp(coffs.size(), nullptr);
    if (store)
        for (size_t j = 0; j < coffs.size(); ++j) cp[j] = static_cast<double *>(Cn->ptr[j]);
    const int gx = hs::dia_grid_x(N);
    double *bmax = nullptr;
    hipError_t e;
    if ((e = tmp.up(coffs, &dco)) != hipSuccess || (e = tmp.up(cptr, &dcp)) != hipSuccess ||
        (e = tmp.up(pairs, &dpairs)) != hipSuccess || (e = tmp.up(cp, &dcptr)) != hipSuccess) {
        delete Cn;
        return dhip(e, "spgemm tables");
    }
    std::vector<double> zeros((size_t)gx * coffs.size(), 0.0);
    if ((e = tmp.up(zeros, &bmax)) != hipSuccess) { delete Cn; return dhip(e, "spgemm tables"); }
    a.c_offs = dco;
    a.c_ptr = dcptr;
    a.cptr = dcp;
    a.pairs = dpairs;
    a.block_max = bmax;
    int le = hs::launch_spgemm(a, (int)coffs.size(), gx, store, st);
    if (le) { delete Cn; return dhip((hipError_t)le, "spgemm kernel"); }
    if (hs_status s = max_of_blocks(bmax, zeros.size(), st, norm)) { delete Cn; return s; }
    if (store) *C = Cn;
    return HS_OK;
}

hs_status identity(int64_t N, hipStream_t st, hs_dia *out) {
    if (hs_status s = dia_alloc(N, HS_C128, {0}, st, out)) return s;
    int le = hs::launch_dia_fill(static_cast<double *>((*out)->ptr[0]), N, 1.0, 0.0, st);
    if (le) { delete *out; *out = nullptr; return dhip((hipError_t)le, "fill kernel"); }
    return HS_OK;
}

// U + T with the union of offsets
hs_status dia_sum(hs_dia U, hs_dia T, hipStream_t st, hs_dia *out) {
    std::set<int64_t> un(U->offs.begin(), U->offs.end());
    un.insert(T->offs.begin(), T->offs.end());
    std::vector<int64_t> offs(un.begin(), un.end());
    hs_dia R = nullptr;
    if (hs_status s = dia_alloc(U->N, HS_C128, offs, st, &R)) return s;
    std::vector<int> ia(offs.size(), -1), ib(offs.size(), -1);
    for (size_t j = 0; j < offs.size(); ++j) {
        auto a = std::lower_bound(U->offs.begin(), U->offs.end(), offs[j]);
        if (a != U->offs.end() && *a == offs[j]) ia[j] = (int)(a - U->offs.begin());
        auto b = std::lower_bound(T->offs.begin(), T->offs.end(), offs[j]);
        if (b != T->offs.end() && *b == offs[j]) ib[j] = (int)(b - T->offs.begin());
    }
    if (hs_status s = dia_tables(U)) { delete R; return s; }
    if (hs_status s = dia_tables(T)) { delete R; return s; }
    if (hs_status s = dia_tables(R)) { delete R; return s; }
    Temps tmp(st);
    int *dia_ = nullptr, *dib = nullptr;
    hipError_t e;
    if ((e = tmp.up(ia, &dia_)) != hipSuccess || (e = tmp.up(ib, &dib)) != hipSuccess) {
        delete R;
        return dhip(e, "sum tables");
    }
    hs::DiaAddArgs a{};
    a.N = U->N;
    a.offs = R->d_offs;
    a.ia = dia_;
    a.ib = dib;
    a.a_ptr = reinterpret_cast<const double *const *>(U->d_ptrs);
    a.b_ptr = reinterpret_cast<const double *const *>(T->d_ptrs);
    a.out = reinterpret_cast<double *const *>(R->d_ptrs);
    int le = hs::launch_dia_add(a, (int)offs.size(), st);
    if (le) { delete R; return dhip((hipError_t)le, "sum kernel"); }
    e = hipStreamSynchronize(st);       // temporaries above are freed on return
    if (e != hipSuccess) { delete R; return dhip(e, "sum"); }
    *out = R;
    return HS_OK;
}

// Largest entry modulus of each diagonal of A (FP64, A complex128).
hs_status diag_maxima(hs_dia A, hipStream_t st, std::vector<double> &out) {
    if (hs_status s = dia_tables(A)) return s;
    const int gx = hs::dia_grid_x(A->N);
    const size_t nd = A->offs.size();
    Temps tmp(st);
    std::vector<double> blocks((size_t)gx * nd, 0.0);
    double *bmax = nullptr;
    DHIP(tmp.up(blocks, &bmax), "maxabs table");
    int le = hs::launch_dia_maxabs(reinterpret_cast<const double *const *>(A->d_ptrs), A->d_offs, A->N,
                                   (int)nd, gx, bmax, st);
    if (le) return dhip((hipError_t)le, "maxabs kernel");
    DHIP(hipMemcpyAsync(blocks.data(), bmax, blocks.size() * sizeof(double), hipMemcpyDeviceToHost, st),
         "download");
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    out.assign(nd, 0.0);
    for (size_t j = 0; j < nd; ++j)
        for (int b = 0; b < gx; ++b) out[j] = std::max(out[j], blocks[j * gx + b]);
    return HS_OK;
}

// Scaling rule for the Taylor series: the smallest s >= 0 with
// |dt| nu / 2^s <= 1/2, nu = sum over H's diagonals (ascending offset) of
// their largest entry modulus, which bounds ||H||_1, ||H||_inf and ||H||_2.
hs_status auto_squarings(hs_dia H, double dt, hipStream_t st, int *s_out) {
    std::vector<double> mx;
    if (hs_status s = diag_maxima(H, st, mx)) return s;
    double nu = 0.0;
    for (double v : mx) nu += v;
    const double x = std::fabs(dt) * nu;
    int s = 0;
    while (x > 0.5 * std::ldexp(1.0, s)) ++s;
    *s_out = s;
    return HS_OK;
}

// Alg. 2 with scaling and squaring: the Taylor series of X = -i H dt / 2^s,
// then s squarings U <- U U by SpGEMM.  squarings < 0 selects s by the rule
// above.
hs_status spme_impl(hs_dia H, double dt, double tol, int max_iter, int squarings, hipStream_t st,
                    hs_dia *out, int *K) {
    *out = nullptr;
    *K = 0;
    if (H->dtype != HS_C128) return dfail(HS_EINVAL, "the exponential needs a complex128 operator");
    if (H->offs.size() == 1 && H->offs[0] == 0) {      // diagonal: exact, elementwise
        hs_dia U = nullptr;
        if (hs_status s = dia_alloc(H->N, HS_C128, {0}, st, &U)) return s;
        int le = hs::launch_diag_exp(static_cast<double *>(H->ptr[0]), static_cast<double *>(U->ptr[0]), H->N, dt, st);
        if (le) { delete U; return dhip((hipError_t)le, "diagonal exponential"); }
        DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        *out = U;
        return HS_OK;
    }
    int sq = squarings;
    if (sq < 0)
        if (hs_status s = auto_squarings(H, dt, st, &sq)) return s;
    const double h = std::ldexp(dt, -sq);               // dt / 2^s, exact
    hs_dia U = nullptr, T = nullptr;
    if (hs_status s = identity(H->N, st, &U)) return s;
    if (hs_status s = identity(H->N, st, &T)) { delete U; return s; }
    for (int k = 1; k <= max_iter; ++k) {
        const double sre = 0.0, sim = -h / k;          // T_k = T_{k-1} (-i h H) / k
        // The stopping test needs only T_k's largest entry: a first pass
        // computes it without storing T_k, so the final (dropped) term, the
        // largest one, never occupies memory.  Kept terms are computed again
        // with storage (same arithmetic, same values).
        double norm = 0.0;
        hs_status s = spgemm(T, H, sre, sim, false, st, nullptr, &norm);
        if (s) { delete U; delete T; return s; }
        if (norm < tol) break;
        hs_dia Tn = nullptr;
        s = spgemm(T, H, sre, sim, true, st, &Tn, &norm);
        delete T;
        T = Tn;
        if (s) { delete U; return s; }
        hs_dia Un = nullptr;
        s = dia_sum(U, T, st, &Un);
        if (s) { delete U; delete T; return s; }
        delete U;
        U = Un;
        *K = k;
    }
    delete T;
    for (int j = 0; j < sq; ++j) {
        hs_dia Un = nullptr;
        double unused = 0.0;
        hs_status s = spgemm(U, U, 1.0, 0.0, true, st, &Un, &unused);
        delete U;
        if (s) return s;
        U = Un;
    }
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    *out = U;
    return HS_OK;
}

}  // namespace

extern "C" {

hs_status hs_dia_from_pauli(int n, int n_terms, const char *const *pauli_terms, const double *coeffs,
                            void *stream, hs_dia *out) {
    if (!out) return dfail(HS_EINVAL, "null output");
    *out = nullptr;
    if (n < 1 || n > HS_MAX_QUBITS) return dfail(n > HS_MAX_QUBITS ? HS_ETOOLARGE : HS_EINVAL, "n_qubits outside [1, 30]");
    if (n_terms < 1 || !pauli_terms || !coeffs) return dfail(HS_EINVAL, "need terms and coefficients");
    std::vector<hs::Term> terms;
    std::string msg;
    if (hs_status s = hs::parse_terms(n, n_terms, pauli_terms, coeffs, terms, msg)) return dfail(s, msg);
    const int64_t N = int64_t(1) << n;
    // terms grouped by X-mask; candidate offsets: every sign pattern of each mask
    std::map<uint64_t, std::vector<int>> cls;
    for (int k = 0; k < n_terms; ++k) cls[terms[k].x].push_back(k);
    std::set<int64_t> cand;
    for (auto &kv : cls) {
        std::vector<int64_t> part{0};
        for (int q = 0; q < n; ++q) {
            if (!((kv.first >> q) & 1)) continue;
            std::vector<int64_t> nx;
            for (int64_t v : part) {
                nx.push_back(v + (int64_t(1) << q));
                nx.push_back(v - (int64_t(1) << q));
            }
            part.swap(nx);
            if (part.size() > 65536) return dfail(HS_ETOOLARGE, "too many candidate diagonals");
        }
        cand.insert(part.begin(), part.end());
        if (cand.size() > 65535) return dfail(HS_ETOOLARGE, "too many candidate diagonals");
    }
    std::vector<int64_t> offs(cand.begin(), cand.end());
    hipStream_t st = S(stream);
    hs_dia A = nullptr;
    if (hs_status s = dia_alloc(N, HS_C128, offs, st, &A)) return s;
    std::vector<uint64_t> masks, zm;
    std::vector<int> cptr{0}, ny;
    std::vector<double> cf;
    for (auto &kv : cls) {
        masks.push_back(kv.first);
        for (int k : kv.second) {
            zm.push_back(terms[k].z);
            cf.push_back(terms[k].c);
            ny.push_back(terms[k].ny);
        }
        cptr.push_back((int)zm.size());
    }
    {
        Temps tmp(st);
        hs::PauliDiaArgs a{};
        uint64_t *dm = nullptr, *dz = nullptr;
        int *dcp = nullptr, *dny = nullptr;
        double *dcf = nullptr;
        hipError_t e;
        if ((e = tmp.up(masks, &dm)) != hipSuccess || (e = tmp.up(zm, &dz)) != hipSuccess ||
            (e = tmp.up(cptr, &dcp)) != hipSuccess || (e = tmp.up(ny, &dny)) != hipSuccess ||
            (e = tmp.up(cf, &dcf)) != hipSuccess) {
            delete A;
            return dhip(e, "term tables");
        }
        if (hs_status s = dia_tables(A)) { delete A; return s; }
        a.N = N;
        a.offs = A->d_offs;
        a.out = reinterpret_cast<double *const *>(A->d_ptrs);
        a.n_cls = (int)masks.size();
        a.cls_mask = dm;
        a.cls_ptr = dcp;
        a.zmask = dz;
        a.coeff = dcf;
        a.ny = dny;
        int le = hs::launch_pauli_dia(a, (int)offs.size(), st);
        if (le) { delete A; return dhip((hipError_t)le, "pauli kernel"); }
        // drop diagonals that are exactly zero (cancelling terms, e.g. XX + YY)
        const int gx = hs::dia_grid_x(N);
        std::vector<double> zeros((size_t)gx * offs.size(), 0.0);
        double *bmax = nullptr;
        if ((e = tmp.up(zeros, &bmax)) != hipSuccess) { delete A; return dhip(e, "maxabs table"); }
        le = hs::launch_dia_maxabs(reinterpret_cast<const double *const *>(A->d_ptrs), A->d_offs, N,
                                   (int)offs.size(), gx, bmax, st);
        if (le) { delete A; return dhip((hipError_t)le, "maxabs kernel"); }
        e = hipMemcpyAsync(zeros.data(), bmax, zeros.size() * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { delete A; return dhip(e, "maxabs"); }
        std::vector<int64_t> keep;
        std::vector<void *> kp;
        for (size_t j = 0; j < offs.size(); ++j) {
            double m = 0.0;
            for (int b = 0; b < gx; ++b) m = std::max(m, zeros[j * gx + b]);
            if (m > 0.0) {
                keep.push_back(offs[j]);
                kp.push_back(A->ptr[j]);
            } else {
                (void)hipFreeAsync(A->ptr[j], st);
            }
            A->ptr[j] = nullptr;
        }
        A->offs = keep;
        A->ptr = kp;
        (void)hipFreeAsync(A->d_offs, st);
        (void)hipFreeAsync(A->d_ptrs, st);
        A->d_offs = nullptr;
        A->d_ptrs = nullptr;
    }
    *out = A;
    return HS_OK;
}

hs_status hs_dia_from_host(long long N, int n_diags, const long long *offsets, const double *const *host_diags,
                           void *stream, hs_dia *out) {
    if (!out) return dfail(HS_EINVAL, "null output");
    *out = nullptr;
    if (N < 1 || N > (1ll << HS_MAX_QUBITS)) return dfail(HS_EINVAL, "N must be in [1, 2^30]");
    if (n_diags < 1 || n_diags > 65535 || !offsets || !host_diags) return dfail(HS_EINVAL, "bad diagonals");
    std::vector<int64_t> offs(offsets, offsets + n_diags);
    for (int j = 0; j < n_diags; ++j) {
        if (offs[j] <= -N || offs[j] >= N) return dfail(HS_EINVAL, "offset out of range");
        if (j && offs[j] <= offs[j - 1]) return dfail(HS_EINVAL, "offsets must ascend strictly");
        if (!host_diags[j]) return dfail(HS_EINVAL, "null diagonal");
    }
    hipStream_t st = S(stream);
    hs_dia A = nullptr;
    if (hs_status s = dia_alloc(N, HS_C128, offs, st, &A)) return s;
    for (int j = 0; j < n_diags; ++j) {
        hipError_t e = hipMemcpyAsync(A->ptr[j], host_diags[j], (size_t)A->len(j) * 16, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) { delete A; return dhip(e, "upload"); }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) { delete A; return dhip(e, "upload"); }
    *out = A;
    return HS_OK;
}

hs_status hs_dia_info(hs_dia A, long long *N, int *n_diags, int *dtype) {
    if (!A) return dfail(HS_EINVAL, "null operator");
    if (N) *N = A->N;
    if (n_diags) *n_diags = (int)A->offs.size();
    if (dtype) *dtype = A->dtype;
    return HS_OK;
}

hs_status hs_dia_offsets(hs_dia A, long long *offsets, int cap) {
    if (!A || !offsets || cap < (int)A->offs.size()) return dfail(HS_EINVAL, "bad arguments");
    for (size_t j = 0; j < A->offs.size(); ++j) offsets[j] = A->offs[j];
    return HS_OK;
}

hs_status hs_dia_copy_diagonal(hs_dia A, int j, long long start, long long count, void *host_dst, void *stream) {
    if (!A || j < 0 || j >= (int)A->offs.size() || !host_dst) return dfail(HS_EINVAL, "bad arguments");
    if (start < 0 || count < 0 || start + count > A->len(j)) return dfail(HS_EINVAL, "range outside the diagonal");
    hipStream_t st = S(stream);
    DHIP(hipMemcpyAsync(host_dst, static_cast<char *>(A->ptr[j]) + start * A->elem(), count * A->elem(),
                        hipMemcpyDeviceToHost, st), "download");
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    return HS_OK;
}

hs_status hs_dia_spgemm(hs_dia A, hs_dia B, void *stream, hs_dia *C) {
    if (!A || !B || !C) return dfail(HS_EINVAL, "null argument");
    *C = nullptr;
    if (A->N != B->N) return dfail(HS_EINVAL, "dimension mismatch");
    if (A->dtype != HS_C128 || B->dtype != HS_C128) return dfail(HS_EINVAL, "SpGEMM needs complex128 operators");
    double norm = 0.0;
    hs_status s = spgemm(A, B, 1.0, 0.0, true, S(stream), C, &norm);
    if (s == HS_OK) {
        hipError_t e = hipStreamSynchronize(S(stream));
        if (e != hipSuccess) return dhip(e, "spgemm");
    }
    return s;
}

hs_status hs_dia_maxabs(hs_dia A, void *stream, double *out) {
    if (!A || !out) return dfail(HS_EINVAL, "null argument");
    if (A->dtype != HS_C128) return dfail(HS_EINVAL, "needs a complex128 operator");
    hipStream_t st = S(stream);
    if (hs_status s = dia_tables(A)) return s;
    const int gx = hs::dia_grid_x(A->N);
    Temps tmp(st);
    std::vector<double> zeros((size_t)gx * A->offs.size(), 0.0);
    double *bmax = nullptr;
    DHIP(tmp.up(zeros, &bmax), "maxabs table");
    int le = hs::launch_dia_maxabs(reinterpret_cast<const double *const *>(A->d_ptrs), A->d_offs, A->N,
                                   (int)A->offs.size(), gx, bmax, st);
    if (le) return dhip((hipError_t)le, "maxabs kernel");
    return max_of_blocks(bmax, zeros.size(), st, out);
}

hs_status hs_spme(hs_dia H, double dt, double tol, int max_iter, int squarings, void *stream, hs_dia *U,
                  int *n_terms) {
    if (!H || !U) return dfail(HS_EINVAL, "null argument");
    if (!(tol > 0.0) || max_iter < 1 || !std::isfinite(dt)) return dfail(HS_EINVAL, "bad tolerance or iterations");
    if (squarings > 60) return dfail(HS_EINVAL, "squarings must be <= 60");
    int K = 0;
    hs_status s = spme_impl(H, dt, tol, max_iter, squarings, S(stream), U, &K);
    if (n_terms) *n_terms = K;
    return s;
}

hs_status hs_estimate_timesteps(hs_dia H, double t, int budget, double tol, int max_iter, void *stream,
                                int *steps) {
    if (!H || !steps || budget < 1 || !(tol > 0.0) || max_iter < 1 || !std::isfinite(t))
        return dfail(HS_EINVAL, "bad arguments");
    if (H->dtype != HS_C128) return dfail(HS_EINVAL, "the exponential needs a complex128 operator");
    if (H->offs.size() == 1 && H->offs[0] == 0) {
        *steps = 1;
        return HS_OK;
    }
    hipStream_t st = S(stream);
    // Taylor term k at step dt is T_k = (-i dt)^k H^k / k!: its largest entry
    // is |dt|^k / k! * max|H^k| and its structural offsets are H^k's, so one
    // sequence of powers of H serves every probe of the search.  max|H^k|
    // comes from a pass that stores nothing; H^(k-1) is stored only when a
    // probe reaches term k with the count so far within the budget, so a
    // stored power never holds more than `budget` diagonals.
    std::vector<double> mk{0.0};                    // mk[k] = max |H^k|
    std::vector<size_t> uk{1};                      // uk[k] = |offsets of H^0 .. H^k|
    std::set<int64_t> un{0};
    std::vector<std::set<int64_t>> upto{un};        // upto[k] = offsets of H^0 .. H^k
    std::vector<int64_t> poffs{0};                  // structural offsets of H^(mk.size() - 1)
    hs_dia P = H;                                   // H^p, owned when p >= 2
    int p = 1;
    auto release = [&]() {
        if (P != H) delete P;
        P = nullptr;
    };
    auto power = [&](int k) -> hs_status {          // extend the tables to term k
        while ((int)mk.size() <= k) {
            const int j = (int)mk.size();
            double m = 0.0;
            if (j == 1) {
                if (hs_status s = hs_dia_maxabs(H, st, &m)) return s;
            } else {
                while (p < j - 1) {                 // H^(p+1), within the budget (see above)
                    hs_dia Pn = nullptr;
                    double unused = 0.0;
                    if (hs_status s = spgemm(P, H, 1.0, 0.0, true, st, &Pn, &unused)) return s;
                    if (P != H) delete P;
                    P = Pn;
                    ++p;
                }
                if (hs_status s = spgemm(P, H, 1.0, 0.0, false, st, nullptr, &m)) return s;
            }
            std::set<int64_t> nx;
            for (int64_t a : poffs)
                for (int64_t b : H->offs)
                    if (a + b > -H->N && a + b < H->N) nx.insert(a + b);
            poffs.assign(nx.begin(), nx.end());
            un.insert(nx.begin(), nx.end());
            mk.push_back(m);
            uk.push_back(un.size());
            upto.push_back(un);
        }
        return HS_OK;
    };
    // scaling rule of hs_spme: |dt| nu / 2^s <= 1/2
    std::vector<double> dmax;
    if (hs_status s = diag_maxima(H, st, dmax)) return s;
    double nu = 0.0;
    for (double v : dmax) nu += v;
    // the SpME stopping rule of each probe, evaluated from the tables, then
    // the offsets of s squarings (S <- S + S; the set only grows, as 0 is in S)
    auto ok = [&](long long r, bool *res) -> hs_status {
        const double dt = t / (double)r;
        int sq = 0;
        while (std::fabs(dt) * nu > 0.5 * std::ldexp(1.0, sq)) ++sq;
        const double h = std::fabs(std::ldexp(dt, -sq));
        double c = 1.0;
        int K = max_iter;
        for (int k = 1; k <= max_iter; ++k) {
            c = c * h / k;
            if (hs_status s = power(k)) return s;
            if (c * mk[k] < tol) { K = k - 1; break; }           // every kept term was within budget
            if (uk[k] > (size_t)budget) { *res = false; return HS_OK; }
        }
        *res = true;
        if (sq == 0) return HS_OK;
        std::set<int64_t> cur = upto[K];
        for (int j = 0; j < sq && *res; ++j) {
            std::set<int64_t> nx;
            for (int64_t a : cur) {
                for (int64_t b : cur)
                    if (a + b > -H->N && a + b < H->N) nx.insert(a + b);
                if (nx.size() > (size_t)budget) break;
            }
            if (nx.size() > (size_t)budget) *res = false;
            cur.swap(nx);
        }
        return HS_OK;
    };
    auto search = [&]() -> hs_status {
        bool f = false;
        long long lo = 1;
        if (hs_status s = ok(lo, &f)) return s;
        if (f) { *steps = 1; return HS_OK; }
        long long u = 2;
        for (;;) {
            if (hs_status s = ok(u, &f)) return s;
            if (f) break;
            lo = u;
            u *= 2;
            if (u > (1ll << 24)) return dfail(HS_EBUDGET, "no step count up to 2^24 meets the budget");
        }
        while (u - lo > 1) {
            const long long mid = (lo + u) / 2;
            if (hs_status s = ok(mid, &f)) return s;
            if (f) u = mid; else lo = mid;
        }
        *steps = (int)u;
        return HS_OK;
    };
    hs_status s = search();
    release();
    if (s == HS_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dhip(e, "hipStreamSynchronize");
    }
    return s;
}

hs_status hs_dia_to_c64(hs_dia A, void *stream, hs_dia *out) {
    if (!A || !out) return dfail(HS_EINVAL, "null argument");
    *out = nullptr;
    if (A->dtype != HS_C128) return dfail(HS_EINVAL, "already complex64");
    hipStream_t st = S(stream);
    hs_dia B = nullptr;
    if (hs_status s = dia_alloc(A->N, HS_C64, A->offs, st, &B)) return s;
    if (hs_status s = dia_tables(A)) { delete B; return s; }
    if (hs_status s = dia_tables(B)) { delete B; return s; }
    int le = hs::launch_dia_to_c64(reinterpret_cast<const double *const *>(A->d_ptrs),
                                   reinterpret_cast<float *const *>(B->d_ptrs), A->d_offs, A->N,
                                   (int)A->offs.size(), st);
    if (le) { delete B; return dhip((hipError_t)le, "convert kernel"); }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) { delete B; return dhip(e, "convert"); }
    *out = B;
    return HS_OK;
}

// Alg. 3's loop: steps applications of U, out of place (U couples rows of
// different tiles in general), ping-ponging with a scratch state.
hs_status hs_dia_evolve(hs_dia U, void *psi, int batch, int steps, void *stream) {
    if (!U || !psi || batch < 1 || steps < 0) return dfail(HS_EINVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(psi) % 16) return dfail(HS_EINVAL, "state pointer must be 16-byte aligned");
    {
        std::string msg;
        if (!hs::device_range_ok(psi, (size_t)batch * U->N * U->elem(), "state", msg)) return dfail(HS_EINVAL, msg);
    }
    if (steps == 0) return HS_OK;
    hipStream_t st = S(stream);
    const int64_t N = U->N;
    const size_t sc = U->elem();
    const int nd = (int)U->offs.size();
    std::vector<long long> offs(U->offs.begin(), U->offs.end());
    std::vector<const void *> ptrs(U->ptr.begin(), U->ptr.end());
    Temps tmp(st);
    const int chunk0 = std::min(HS_MAX_BATCH, batch);
    void *scratch = nullptr;
    DHIP(hipMallocAsync(&scratch, (size_t)chunk0 * N * sc, st), "hipMallocAsync(scratch)");
    tmp.ptrs.push_back(scratch);
    std::map<int, DiagDesc *> descs;
    std::vector<std::vector<DiagDesc>> host_descs;
    for (int c0 = 0; c0 < batch; c0 += HS_MAX_BATCH) {
        const int chunk = std::min(HS_MAX_BATCH, batch - c0);
        const Geo geo = generic_geometry(offs.data(), nd, N, U->dtype, chunk);
        DiagDesc *dd = nullptr;
        auto it = descs.find(chunk);
        if (it == descs.end()) {
            host_descs.emplace_back();
            fill_descs(offs.data(), ptrs.data(), nd, N, geo, host_descs.back());
            DHIP(tmp.up(host_descs.back(), &dd), "descriptors");
            descs[chunk] = dd;
        } else {
            dd = it->second;
        }
        char *cur = static_cast<char *>(psi) + (size_t)c0 * N * sc;
        char *home = cur;
        char *other = static_cast<char *>(scratch);
        for (int s = 0; s < steps; ++s) {
            TileArgs a = open_args(geo, dd, nd, cur, other, N);
            a.stream_out = stream_out(chunk, N, U->dtype);
            int le = hs::launch_tile(a, chunk, U->dtype == HS_C128, false, st);
            if (le) return dhip((hipError_t)le, "tile kernel launch");
            std::swap(cur, other);
        }
        if (cur != home) DHIP(hipMemcpyAsync(home, cur, (size_t)chunk * N * sc, hipMemcpyDeviceToDevice, st), "copy back");
    }
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");   // temporaries are freed on return
    return HS_OK;
}

hs_status hs_dia_norm_bound(hs_dia A, void *stream, double *nu) {
    if (!A || !nu) return dfail(HS_EINVAL, "null argument");
    std::vector<double> mx;
    if (hs_status s = diag_maxima(A, S(stream), mx)) return s;
    double v = 0.0;
    for (double m : mx) v += m;
    *nu = v;
    return HS_OK;
}

hs_status hs_taylor_terms(hs_dia H, double dt, double tol, int max_terms, void *stream, int *K) {
    if (!H || !K || !(tol > 0.0) || max_terms < 1 || max_terms > 64 || !std::isfinite(dt))
        return dfail(HS_EINVAL, "bad arguments");
    double nu = 0.0;
    if (hs_status s = hs_dia_norm_bound(H, stream, &nu)) return s;
    const double x = std::fabs(dt) * nu;
    double b = x;                                   // bound of term k: x^k / k!
    for (int k = 1; k <= max_terms; ++k) {
        b = b * x / (k + 1);
        if (b < tol) {
            *K = k;
            return HS_OK;
        }
    }
    return dfail(HS_EBUDGET, "|dt| nu(H) too large for max_terms Taylor terms; take more steps");
}

hs_status hs_taylor_steps(hs_dia H, double t, double theta, void *stream, int *steps) {
    if (!H || !steps || !(theta > 0.0) || !std::isfinite(t)) return dfail(HS_EINVAL, "bad arguments");
    double nu = 0.0;
    if (hs_status s = hs_dia_norm_bound(H, stream, &nu)) return s;
    const double r0 = std::ceil(std::fabs(t) * nu / theta);
    if (!(r0 <= (double)(1 << 30))) return dfail(HS_EBUDGET, "more than 2^30 steps");
    long long r = std::max(1ll, (long long)r0);
    while (r > 1 && std::fabs(t / (double)(r - 1)) * nu <= theta) --r;   // rounding guards
    while (std::fabs(t / (double)r) * nu > theta) ++r;
    *steps = (int)r;
    return HS_OK;
}

hs_status hs_taylor_evolve(hs_dia H, void *psi, int batch, double dt, int K, int steps, void *stream) {
    if (!H || !psi || batch < 1 || steps < 0 || K < 1 || K > 64 || !std::isfinite(dt))
        return dfail(HS_EINVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(psi) % 16) return dfail(HS_EINVAL, "state pointer must be 16-byte aligned");
    {
        std::string msg;
        if (!hs::device_range_ok(psi, (size_t)batch * H->N * H->elem(), "state", msg)) return dfail(HS_EINVAL, msg);
    }
    if (steps == 0) return HS_OK;
    hipStream_t st = S(stream);
    const int64_t N = H->N;
    const size_t sc = H->elem();
    const bool c128 = H->dtype == HS_C128;
    const int nd = (int)H->offs.size();
    std::vector<long long> offs(H->offs.begin(), H->offs.end());
    std::vector<const void *> ptrs(H->ptr.begin(), H->ptr.end());
    Temps tmp(st);
    const int chunk0 = std::min(HS_MAX_BATCH, batch);
    void *buf[2] = {nullptr, nullptr};
    for (int i = 0; i < (K == 1 ? 1 : 2); ++i) {
        DHIP(hipMallocAsync(&buf[i], (size_t)chunk0 * N * sc, st), "hipMallocAsync(scratch)");
        tmp.ptrs.push_back(buf[i]);
    }
    std::map<int, DiagDesc *> descs;
    std::vector<std::vector<DiagDesc>> host_descs;
    for (int c0 = 0; c0 < batch; c0 += HS_MAX_BATCH) {
        const int chunk = std::min(HS_MAX_BATCH, batch - c0);
        const Geo geo = generic_geometry(offs.data(), nd, N, H->dtype, chunk);
        DiagDesc *dd = nullptr;
        auto it = descs.find(chunk);
        if (it == descs.end()) {
            host_descs.emplace_back();
            fill_descs(offs.data(), ptrs.data(), nd, N, geo, host_descs.back());
            DHIP(tmp.up(host_descs.back(), &dd), "descriptors");
            descs[chunk] = dd;
        } else {
            dd = it->second;
        }
        char *home = static_cast<char *>(psi) + (size_t)c0 * N * sc;
        char *cur = home;
        char *other = static_cast<char *>(buf[0]);
        for (int s = 0; s < steps; ++s) {
            // Horner: w <- x + (-i dt / j) H w for j = K .. 1, starting from w = x.
            // The last stage writes over x itself (each row reads its own x
            // entry only); with K = 1 the only stage reads x as w too, so it
            // writes the other buffer and the roles swap.
            const void *w = cur;
            for (int j = K; j >= 1; --j) {
                void *out = (K == 1) ? other : (j == 1 ? cur : buf[(K - j) & 1]);
                TileArgs a = open_args(geo, dd, nd, w, out, N);
                a.stream_out = stream_out(chunk, N, H->dtype);
                a.x0 = cur;
                a.alpha_re = 0.0;
                a.alpha_im = -dt / j;
                int le = hs::launch_tile_horner(a, chunk, c128, st);
                if (le) return dhip((hipError_t)le, "Horner tile kernel launch");
                w = out;
            }
            if (K == 1) std::swap(cur, other);
        }
        if (cur != home) {
            DHIP(hipMemcpyAsync(home, cur, (size_t)chunk * N * sc, hipMemcpyDeviceToDevice, st), "copy back");
        }
    }
    DHIP(hipStreamSynchronize(st), "hipStreamSynchronize");   // temporaries are freed on return
    return HS_OK;
}

hs_status hs_dia_free(hs_dia A) {
    delete A;
    return HS_OK;
}

}  // extern "C"
