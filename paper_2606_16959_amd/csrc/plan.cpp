// Host planning: Pauli parsing, first-fit grouping under the diagonal budget,
// local unitaries and the structural dry run that fixes each factor's
// diagonal set before any storage exists (paper: Eq. 4 and Eq. 5 applied per
// factor, Section 3.1; Eq. 6 and the "structural dry run", Section 3.2).
//
// Reading of the grouping (the paper does not describe how the H_j of Eq. 4
// are formed): Z-only terms form the diagonal factor; every other term joins
// the first existing group whose members it all commutes with and whose exact
// exponential stays within the budget, else it opens a new group.  Because a
// group's members commute and each Pauli squares to I, the group exponential
// is exactly prod_k (cos(c_k dt) I - i sin(c_k dt) P_k).

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>

#include "hs_internal.h"

namespace hs {
namespace {

int popc(uint64_t v) { return __builtin_popcountll(v); }

bool commute(const Term &a, const Term &b) {
    return ((popc(a.x & b.z) + popc(a.z & b.x)) & 1) == 0;
}

uint64_t pext_bits(uint64_t v, const std::vector<int> &bits) {
    uint64_t o = 0;
    for (size_t j = 0; j < bits.size(); ++j) o |= ((v >> bits[j]) & 1ull) << j;
    return o;
}

int64_t spread_bits(uint64_t a, const std::vector<int> &bits) {
    int64_t o = 0;
    for (size_t j = 0; j < bits.size(); ++j) o |= (int64_t)((a >> j) & 1ull) << bits[j];
    return o;
}

// L = prod over members (first member applied first) of cos(th) I - i sin(th) P,
// restricted to the support bits.  P[y, y^m] = i^ny (-1)^{popcount((y^m) & z)}.
void local_unitary(const std::vector<Term> &terms, const std::vector<int> &members, double dt,
                   std::vector<int> &bits, std::vector<std::complex<double>> &L) {
    uint64_t s = 0;
    for (int k : members) s |= terms[k].x | terms[k].z;
    bits.clear();
    for (int q = 0; q < 64; ++q)
        if ((s >> q) & 1ull) bits.push_back(q);
    const int K = 1 << bits.size();
    L.assign((size_t)K * K, 0.0);
    for (int a = 0; a < K; ++a) L[(size_t)a * K + a] = 1.0;
    std::vector<std::complex<double>> nL((size_t)K * K);
    static const std::complex<double> ipow[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    for (int k : members) {
        const Term &t = terms[k];
        const uint64_t m = pext_bits(t.x, bits), z = pext_bits(t.z, bits);
        const double th = t.c * dt;
        const double c = std::cos(th), sn = std::sin(th);
        const std::complex<double> ph = ipow[t.ny & 3];
        for (int y = 0; y < K; ++y) {
            const uint64_t src = (uint64_t)y ^ m;
            const double sg = (popc(src & z) & 1) ? -1.0 : 1.0;
            // -i sin(th) * (i^ny * sg)
            const std::complex<double> w = std::complex<double>(0.0, -sn) * (ph * sg);
            for (int b = 0; b < K; ++b)
                nL[(size_t)y * K + b] = c * L[(size_t)y * K + b] + w * L[(size_t)src * K + b];
        }
        L.swap(nL);
    }
}

// Offsets spr(b) - spr(a) of the entries above the threshold; zeroes the rest.
std::vector<int64_t> offsets_of(const std::vector<int> &bits, std::vector<std::complex<double>> &L) {
    const int K = 1 << bits.size();
    std::vector<int64_t> spr(K);
    for (int a = 0; a < K; ++a) spr[a] = spread_bits((uint64_t)a, bits);
    std::set<int64_t> offs;
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            std::complex<double> &v = L[(size_t)a * K + b];
            if (std::abs(v) > kTau)
                offs.insert(spr[b] - spr[a]);
            else
                v = 0.0;
        }
    return std::vector<int64_t>(offs.begin(), offs.end());
}

bool support_ok(const std::vector<Term> &terms, const std::vector<int> &members) {
    uint64_t s = 0;
    for (int k : members) s |= terms[k].x | terms[k].z;
    return popc(s) <= HS_MAX_SUPPORT;
}

int count_diags(const std::vector<Term> &terms, const std::vector<int> &members, double dt) {
    std::vector<int> bits;
    std::vector<std::complex<double>> L;
    local_unitary(terms, members, dt, bits, L);
    return (int)offsets_of(bits, L).size();
}

}  // namespace

hs_status parse_terms(int n, int n_terms, const char *const *strings, const double *coeffs,
                      std::vector<Term> &terms, std::string &msg) {
    char buf[256];
    terms.clear();
    double cmax = 0.0;
    for (int k = 0; k < n_terms; ++k) {
        const double re = coeffs[2 * k], im = coeffs[2 * k + 1];
        if (!std::isfinite(re) || !std::isfinite(im)) { msg = "non-finite coefficient"; return HS_EINVAL; }
        cmax = std::max(cmax, std::hypot(re, im));
    }
    for (int k = 0; k < n_terms; ++k) {
        if (std::fabs(coeffs[2 * k + 1]) > 1e-12 * cmax) {
            snprintf(buf, sizeof buf, "term %d has imaginary coefficient %.3g: H is not Hermitian", k,
                     coeffs[2 * k + 1]);
            msg = buf;
            return HS_ENONHERMITIAN;
        }
        const char *s = strings[k];
        if (!s) { msg = "null Pauli string"; return HS_EINVAL; }
        Term tm;
        int len = 0;
        for (; s[len]; ++len) {
            if (len >= n) break;
            const uint64_t bit = 1ull << len;
            switch (s[len]) {
                case 'I': break;
                case 'X': tm.x |= bit; break;
                case 'Z': tm.z |= bit; break;
                case 'Y': tm.x |= bit; tm.z |= bit; ++tm.ny; break;
                default:
                    snprintf(buf, sizeof buf, "term %d: bad Pauli character '%c'", k, s[len]);
                    msg = buf;
                    return HS_EINVAL;
            }
        }
        if (len != n || s[len] != '\0') {
            snprintf(buf, sizeof buf, "term %d: string length differs from n_qubits=%d", k, n);
            msg = buf;
            return HS_EINVAL;
        }
        tm.c = coeffs[2 * k];
        terms.push_back(tm);
    }

    return HS_OK;
}

void layout_factor(Factor &f, int64_t N, size_t elem_bytes) {
    const size_t align = kDiagAlignBytes / elem_bytes;
    size_t pos = 0;
    f.elem_off.clear();
    for (int64_t d : f.offs) {
        f.elem_off.push_back(pos);
        const size_t len = (size_t)(N - (d < 0 ? -d : d));
        pos += (len + align - 1) / align * align;
    }
    f.elems_total = pos;
}

hs_status make_plan(int n, int n_terms, const char *const *strings, const double *coeffs,
                    double t, int steps, int budget, unsigned flags, Plan &P, std::string &msg) {
    char buf[256];
    if (n < 1 || n > HS_MAX_QUBITS) {
        snprintf(buf, sizeof buf, "n_qubits=%d outside [1, %d]", n, HS_MAX_QUBITS);
        msg = buf;
        return n > HS_MAX_QUBITS ? HS_ETOOLARGE : HS_EINVAL;
    }
    if (n_terms < 1 || !strings || !coeffs) { msg = "need n_terms >= 1, strings and coeffs"; return HS_EINVAL; }
    if (steps < 1) { msg = "steps must be >= 1"; return HS_EINVAL; }
    if (budget < 1) { msg = "budget must be >= 1"; return HS_EINVAL; }
    if (!std::isfinite(t)) { msg = "t must be finite"; return HS_EINVAL; }
    if (flags & ~(unsigned)(HS_MERGE_DIAG | HS_ORDER2 | HS_ORDER4)) { msg = "unknown build flag"; return HS_EINVAL; }
    if ((flags & HS_ORDER2) && (flags & HS_ORDER4)) { msg = "choose one product order"; return HS_EINVAL; }

    P = Plan();
    P.n = n;
    P.N = (int64_t)1 << n;
    P.t = t;
    P.steps = steps;
    P.dt = t / steps;
    P.budget = budget;
    P.flags = flags;

    if (hs_status st = parse_terms(n, n_terms, strings, coeffs, P.terms, msg)) return st;

    // first-fit grouping
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < n_terms; ++i) {
        const Term &t = P.terms[i];
        if (t.x == 0) { P.diag.push_back(i); continue; }
        bool placed = false;
        for (auto &g : groups) {
            bool ok = true;
            for (int j : g)
                if (!commute(t, P.terms[j])) { ok = false; break; }
            if (!ok) continue;
            std::vector<int> cand = g;
            cand.push_back(i);
            if (!support_ok(P.terms, cand)) continue;
            if (count_diags(P.terms, cand, P.dt) <= budget) {
                g.push_back(i);
                placed = true;
                break;
            }
        }
        if (!placed) {
            std::vector<int> one{i};
            if (!support_ok(P.terms, one)) {
                snprintf(buf, sizeof buf, "term %d acts on more than %d qubits", i, HS_MAX_SUPPORT);
                msg = buf;
                return HS_ETOOLARGE;
            }
            const int nd = count_diags(P.terms, one, P.dt);
            if (nd > budget) {
                snprintf(buf, sizeof buf, "term %d alone needs %d diagonals > budget %d", i, nd, budget);
                msg = buf;
                return HS_EBUDGET;
            }
            groups.push_back(one);
        }
    }

    auto diag_factor = [&](double h) {
        Factor d;
        d.has_diag = true;
        d.dt = h;
        d.offs = {0};
        for (int k : P.diag) d.smask |= P.terms[k].z;
        return d;
    };
    auto group_factor = [&](const std::vector<int> &g, double h, bool with_diag) {
        Factor f;
        f.has_diag = with_diag;
        f.dt = h;
        f.terms = g;
        local_unitary(P.terms, f.terms, h, f.bits, f.L);
        f.offs = offsets_of(f.bits, f.L);
        for (int q : f.bits) f.smask |= 1ull << q;
        for (int k : f.terms) f.xmask_union |= P.terms[k].x;
        return f;
    };
    P.order = (flags & HS_ORDER4) ? 4 : (flags & HS_ORDER2) ? 2 : 1;
    if (P.order == 1) {
        const bool merge = (flags & HS_MERGE_DIAG) != 0;
        if (!P.diag.empty() && (!merge || groups.empty())) P.factors.push_back(diag_factor(P.dt));
        for (size_t j = 0; j < groups.size(); ++j)
            P.factors.push_back(group_factor(groups[j], P.dt, merge && j == 0 && !P.diag.empty()));
        for (size_t k = 0; k < P.factors.size(); ++k) P.seq.push_back((int)k);
    } else {
        // Symmetric products over F = (D, G_1, ..., G_m): S2(h) applies
        // F_1..F_{L-1} with h/2, F_L with h, then F_{L-1}..F_1 with h/2;
        // S4(dt) = S2(p dt) S2(p dt) S2((1-4p) dt) S2(p dt) S2(p dt),
        // p = 1/(4 - 4^(1/3)).  D stays a factor of its own; every distinct
        // (factor, time step) pair is stored once.
        const int L = (P.diag.empty() ? 0 : 1) + (int)groups.size();
        std::vector<std::pair<int, double>> seq;     // (F index, h); F index 0 = D when present
        auto s2 = [&](double h) {
            if (L == 1) { seq.push_back({0, h}); return; }
            for (int j = 0; j < L - 1; ++j) seq.push_back({j, h / 2});
            seq.push_back({L - 1, h});
            for (int j = L - 2; j >= 0; --j) seq.push_back({j, h / 2});
        };
        if (P.order == 2) {
            s2(P.dt);
        } else {
            const double p = 1.0 / (4.0 - std::pow(4.0, 1.0 / 3.0));
            s2(p * P.dt);
            s2(p * P.dt);
            s2((1 - 4 * p) * P.dt);
            s2(p * P.dt);
            s2(p * P.dt);
        }
        // Neighbours with the same generator combine, exp(-i a G) exp(-i b G) =
        // exp(-i (a + b) G): S4's junctions F_1(p dt/2) F_1(p dt/2) and the
        // like.  Sums are taken left to right.
        std::vector<std::pair<int, double>> merged;
        for (auto &e : seq) {
            if (!merged.empty() && merged.back().first == e.first) merged.back().second += e.second;
            else merged.push_back(e);
        }
        std::map<std::pair<int, double>, int> made;
        auto stored = [&](const std::pair<int, double> &e) {
            auto it = made.find(e);
            if (it == made.end()) {
                const bool is_diag = !P.diag.empty() && e.first == 0;
                const int g = e.first - (P.diag.empty() ? 0 : 1);
                P.factors.push_back(is_diag ? diag_factor(e.second) : group_factor(groups[g], e.second, false));
                it = made.emplace(e, (int)P.factors.size() - 1).first;
            }
            return it->second;
        };
        for (auto &e : merged) P.seq.push_back(stored(e));
        // A symmetric step starts and ends with F_1, so consecutive steps meet
        // in F_1(last h) F_1(first h): stored once as the joint factor.
        if (merged.size() > 1 && merged.front().first == merged.back().first)
            P.joint = stored({merged.front().first, merged.back().second + merged.front().second});
    }
    for (auto &f : P.factors) {
        if (f.xmask_union) {
            f.xlb = __builtin_ctzll(f.xmask_union);
            f.xhb = 64 - __builtin_clzll(f.xmask_union);
        }
    }
    return HS_OK;
}

}  // namespace hs
