/* A plain C99 caller of the C ABI (host-side planning only, no device):
 * plans an 8-qubit TFIM chain with budget 8 and prints the factor count,
 * each factor's offsets, and the status of an over-budget plan. */
#include <stdio.h>

#include "hamsim.h"

int main(void) {
    const char *terms[15];
    char buf[15][9];
    double coeffs[30];                          /* (re, im) per term */
    int k = 0;
    for (int i = 0; i < 7; ++i, ++k) {          /* -Z_i Z_{i+1} */
        for (int q = 0; q < 8; ++q) buf[k][q] = (q == i || q == i + 1) ? 'Z' : 'I';
        buf[k][8] = '\0';
        terms[k] = buf[k];
        coeffs[2 * k] = -1.0;
        coeffs[2 * k + 1] = 0.0;
    }
    for (int i = 0; i < 8; ++i, ++k) {          /* -X_i */
        for (int q = 0; q < 8; ++q) buf[k][q] = (q == i) ? 'X' : 'I';
        buf[k][8] = '\0';
        terms[k] = buf[k];
        coeffs[2 * k] = -1.0;
        coeffs[2 * k + 1] = 0.0;
    }
    hs_factors f = NULL;
    hs_status s = hs_plan(8, 15, terms, coeffs, 1.0, 10, 8, HS_MERGE_DIAG, &f);
    if (s != HS_OK) {
        printf("plan failed %d %s\n", (int)s, hs_last_error());
        return 1;
    }
    int nq = 0, nf = 0, nt = 0, nd = 0, dt = 0, steps = 0;
    double h = 0.0;
    hs_factors_info(f, &nq, &nf, &nt, &nd, &dt, &h, &steps);
    printf("qubits %d factors %d terms %d diag_terms %d steps %d\n", nq, nf, nt, nd, steps);
    for (int j = 0; j < nf; ++j) {
        long long offs[64];
        int hd = 0, ng = 0, ndg = 0;
        unsigned long long sm = 0;
        size_t bytes = 0;
        hs_factor_info(f, j, &hd, &ng, &ndg, &sm, &bytes);
        hs_factor_offsets(f, j, offs, 64);
        printf("factor %d diag %d terms %d offsets", j, hd, ng);
        for (int q = 0; q < ndg; ++q) printf(" %lld", offs[q]);
        printf("\n");
    }
    hs_free_factors(f);
    const char *xxx[1] = {"XXXIIIII"};
    double one[2] = {1.0, 0.0};
    hs_factors g = NULL;
    s = hs_plan(8, 1, xxx, one, 1.0, 10, 8, 0, &g);
    printf("over budget status %d handle %s\n", (int)s, g ? "set" : "null");
    return 0;
}
