/*
 * FP64 CPU oracle of Trotterized product formulas -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  It shares no code with the GPU library.
 *
 * Computes psi_r = (U_m ... U_2 U_1 D)^r psi_0 (paper: Eq. 4 with each
 * factor exponentiated exactly, Eq. 2; a diagonal factor is exponentiated
 * elementwise, Section 3.4), or the same factors in any per-step sequence
 * with per-entry time steps (higher-order product formulas), where
 *   D[x]  = exp(-i dt E(x)),  E(x) = sum_{k diag} c_k (-1)^{popcount(x & z_k)}
 *   U_j   = prod_{k in group j} (cos(c_k dt) I - i sin(c_k dt) P_k)
 * and P_k |x> = i^{ny_k} (-1)^{popcount(x & z_k)} |x ^ m_k>.
 * Each rotation is applied to the pair (x, x ^ m) from the old values.
 * All arithmetic is double precision; sin/cos come from libm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double zsign(uint64_t v) { return (__builtin_popcountll(v) & 1) ? -1.0 : 1.0; }

/* psi <- exp(-i th P) psi for one Pauli string (m, z, ny). */
static void rotate(double *psi, int n, uint64_t m, uint64_t z, int ny, double th)
{
    const int64_t N = (int64_t)1 << n;
    const double c = cos(th), s = sin(th);
    /* i^ny */
    static const double PR[4] = {1.0, 0.0, -1.0, 0.0};
    static const double PI_[4] = {0.0, 1.0, 0.0, -1.0};
    const double pr = PR[ny & 3], pi = PI_[ny & 3];
    if (m == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            double sg = zsign((uint64_t)x & z);
            double wr = sg * (pr * psi[2 * x] - pi * psi[2 * x + 1]);
            double wi = sg * (pr * psi[2 * x + 1] + pi * psi[2 * x]);
            /* c*a - i s w */
            psi[2 * x] = c * psi[2 * x] + s * wi;
            psi[2 * x + 1] = c * psi[2 * x + 1] - s * wr;
        }
        return;
    }
    int h = 63 - __builtin_clzll(m);
    const int64_t lowmask = ((int64_t)1 << h) - 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N / 2; ++i) {
        int64_t x = ((i >> h) << (h + 1)) | (i & lowmask); /* bit h of x is 0 */
        int64_t y = x ^ (int64_t)m;
        double ar = psi[2 * x], ai = psi[2 * x + 1];
        double br = psi[2 * y], bi = psi[2 * y + 1];
        /* (P psi)[x] = i^ny sgn(y & z) psi[y];  (P psi)[y] = i^ny sgn(x & z) psi[x] */
        double sx = zsign((uint64_t)y & z), sy = zsign((uint64_t)x & z);
        double wxr = sx * (pr * br - pi * bi), wxi = sx * (pr * bi + pi * br);
        double wyr = sy * (pr * ar - pi * ai), wyi = sy * (pr * ai + pi * ar);
        psi[2 * x] = c * ar + s * wxi;
        psi[2 * x + 1] = c * ai - s * wxr;
        psi[2 * y] = c * br + s * wyi;
        psi[2 * y + 1] = c * bi - s * wyr;
    }
}

/* E(x) = sum_{k diag} c_k (-1)^{popcount(x & z_k)} */
static void energies(int n, int n_diag, const uint64_t *zmask, const double *coeff, const int *diag_idx,
                     double *E)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double e = 0.0;
        for (int j = 0; j < n_diag; ++j) {
            int k = diag_idx[j];
            e += coeff[k] * zsign((uint64_t)x & zmask[k]);
        }
        E[x] = e;
    }
}

/*
 * General product formula: one step applies seq_len entries in order; entry
 * q applies the diagonal factor exp(-i h_q E) when seq_group[q] < 0, else the
 * exact exponential of group seq_group[q], prod_k exp(-i c_k h_q P_k), where
 * h_q = seq_dt[q].  First order is the sequence D, G_1 .. G_m with h = dt.
 */
int oracle_evolve_seq(int n, int batch, double *psi,
                      int n_terms, const uint64_t *xmask, const uint64_t *zmask,
                      const int *ny, const double *coeff,
                      int n_diag, const int *diag_idx,
                      int n_groups, const int *group_ptr, const int *group_idx,
                      int seq_len, const int *seq_group, const double *seq_dt,
                      int steps, int threads)
{
    (void)n_terms;
    (void)n_groups;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    const int64_t N = (int64_t)1 << n;
    double *E = NULL;
    if (n_diag > 0) {
        E = (double *)malloc(sizeof(double) * (size_t)N);
        if (!E) return -1;
        energies(n, n_diag, zmask, coeff, diag_idx, E);
    }
    for (int s = 0; s < steps; ++s) {
        for (int b = 0; b < batch; ++b) {
            double *p = psi + (size_t)b * 2 * (size_t)N;
            for (int q = 0; q < seq_len; ++q) {
                const int g = seq_group[q];
                const double h = seq_dt[q];
                if (g < 0) {
                    if (!E) continue;
#pragma omp parallel for schedule(static)
                    for (int64_t x = 0; x < N; ++x) {
                        double ph = -h * E[x];
                        double cr = cos(ph), ci = sin(ph);
                        double ar = p[2 * x], ai = p[2 * x + 1];
                        p[2 * x] = cr * ar - ci * ai;
                        p[2 * x + 1] = cr * ai + ci * ar;
                    }
                } else {
                    for (int j = group_ptr[g]; j < group_ptr[g + 1]; ++j) {
                        int k = group_idx[j];
                        rotate(p, n, xmask[k], zmask[k], ny[k], coeff[k] * h);
                    }
                }
            }
        }
    }
    free(E);
    return 0;
}

/* first-order product: D, then the groups in order, each with dt */
int oracle_evolve(int n, int batch, double *psi,
                  int n_terms, const uint64_t *xmask, const uint64_t *zmask,
                  const int *ny, const double *coeff,
                  int n_diag, const int *diag_idx,
                  int n_groups, const int *group_ptr, const int *group_idx,
                  double dt, int steps, int threads)
{
    int *sg = (int *)malloc(sizeof(int) * (size_t)(n_groups + 1));
    double *sd = (double *)malloc(sizeof(double) * (size_t)(n_groups + 1));
    if (!sg || !sd) { free(sg); free(sd); return -1; }
    int len = 0;
    if (n_diag > 0) { sg[len] = -1; sd[len] = dt; ++len; }
    for (int g = 0; g < n_groups; ++g) { sg[len] = g; sd[len] = dt; ++len; }
    int rc = oracle_evolve_seq(n, batch, psi, n_terms, xmask, zmask, ny, coeff, n_diag, diag_idx,
                               n_groups, group_ptr, group_idx, len, sg, sd, steps, threads);
    free(sg);
    free(sd);
    return rc;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
