// Host planning under AddressSanitizer and UndefinedBehaviorSanitizer: seeded
// random Pauli sums (1..24 qubits, supports anywhere, budgets 3..81, every
// product order, merged or separate diagonal factor) and malformed inputs
// (bad characters, wrong string lengths, null pointers, non-Hermitian
// coefficients, out-of-range sizes and flags) through the planner and the
// storage layout.  Built with g++ and the sanitizers by the CPU test suite;
// exits non-zero on an inconsistent plan, a sanitizer stops it on a fault.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_2606_16959_amd/csrc/hs_internal.h"

static int check_plan(const hs::Plan &P, int n_terms) {
    // every term is in exactly one place: the diagonal factor or one group
    std::vector<int> seen(n_terms, 0);
    for (int k : P.diag) seen[k]++;
    bool diag_carried = false;
    for (const auto &f : P.factors) {
        for (int k : f.terms) seen[k]++;
        diag_carried |= f.has_diag;
        for (size_t j = 1; j < f.offs.size(); ++j)
            if (f.offs[j] <= f.offs[j - 1]) return 1;
        if ((int)f.offs.size() > P.budget && !f.terms.empty()) return 2;
        if (f.elem_off.size() != f.offs.size()) return 3;
    }
    // a first-order product visits every term once per step; higher orders repeat factors
    if (P.order == 1)
        for (int k = 0; k < n_terms; ++k)
            if (seen[k] != 1) return 4;
    if (!P.diag.empty() && !diag_carried) return 5;
    for (int q : P.seq)
        if (q < 0 || q >= (int)P.factors.size()) return 6;
    return 0;
}

int main() {
    std::mt19937_64 rng(20261203);
    const char *paulis = "IXYZ";
    int planned = 0, refused = 0;
    for (int it = 0; it < 400; ++it) {
        const int n = 1 + (int)(rng() % 24);
        const int nt = 1 + (int)(rng() % 40);
        std::vector<std::string> s(nt, std::string(n, 'I'));
        std::vector<double> c(2 * nt, 0.0);
        for (int k = 0; k < nt; ++k) {
            const int w = 1 + (int)(rng() % 3);
            for (int j = 0; j < w; ++j) s[k][rng() % n] = paulis[rng() % 4];
            c[2 * k] = std::uniform_real_distribution<double>(-2.0, 2.0)(rng);
        }
        std::vector<const char *> sp(nt);
        for (int k = 0; k < nt; ++k) sp[k] = s[k].c_str();
        const int budget = 3 + (int)(rng() % 79);
        const unsigned flags = (rng() % 2 ? HS_MERGE_DIAG : 0u) | (unsigned[]){0u, HS_ORDER2, HS_ORDER4}[rng() % 3];
        const int steps = 1 + (int)(rng() % 50);
        hs::Plan P;
        std::string msg;
        const hs_status st = hs::make_plan(n, nt, sp.data(), c.data(), 1.0, steps, budget, flags, P, msg);
        if (st == HS_OK) {
            for (auto &f : P.factors) hs::layout_factor(f, P.N, it % 2 ? 16 : 8);
            if (int e = check_plan(P, nt)) {
                std::printf("inconsistent plan %d at iteration %d\n", e, it);
                return 1;
            }
            ++planned;
        } else {
            if (msg.empty()) return 7;          // a refusal always says why
            ++refused;
        }
    }
    // malformed inputs: each must be refused with a message, never crash
    struct Bad { int n, nt; const char *s0; double re, im; int steps, budget; unsigned flags; };
    const Bad bad[] = {
        {3, 1, "XQZ", 1.0, 0.0, 4, 8, 0},            // bad character
        {3, 1, "XZ", 1.0, 0.0, 4, 8, 0},             // too short
        {3, 1, "XZZI", 1.0, 0.0, 4, 8, 0},           // too long
        {3, 1, "XXX", 1.0, 0.5, 4, 8, 0},            // non-Hermitian
        {0, 1, "", 1.0, 0.0, 4, 8, 0},               // no qubits
        {31, 1, "X", 1.0, 0.0, 4, 8, 0},             // too many qubits
        {3, 1, "XXX", 1.0, 0.0, 0, 8, 0},            // no steps
        {3, 1, "XXX", 1.0, 0.0, 4, 0, 0},            // no budget
        {3, 1, "XXX", 1.0, 0.0, 4, 8, 1u << 9},      // unknown flag
        {3, 1, "XXX", 1.0, 0.0, 4, 8, HS_ORDER2 | HS_ORDER4},
        {3, 1, "XXX", 1.0, 0.0, 4, 3, 0},            // one term over the budget
        {12, 1, "XXXXXXXXXXXX", 1.0, 0.0, 4, 1 << 20, 0},   // support beyond 10 qubits
    };
    for (const Bad &b : bad) {
        const char *sp[1] = {b.s0};
        double c[2] = {b.re, b.im};
        hs::Plan P;
        std::string msg;
        if (hs::make_plan(b.n, b.nt, sp, c, 1.0, b.steps, b.budget, b.flags, P, msg) == HS_OK) {
            std::printf("accepted a malformed input: \"%s\"\n", b.s0);
            return 8;
        }
        if (msg.empty()) return 9;
    }
    {
        hs::Plan P;
        std::string msg;
        if (hs::make_plan(3, 1, nullptr, nullptr, 1.0, 4, 8, 0, P, msg) == HS_OK) return 10;
    }
    std::printf("planned %d, refused %d random sums; %zu malformed inputs refused\n", planned, refused,
                sizeof(bad) / sizeof(bad[0]) + 1);
    return 0;
}
