/*
 * hamsim.h -- C ABI of the MI355X (gfx950) library for diagonal-budgeted
 * Trotterized Hamiltonian simulation.
 *
 * The paper's problem statement (Section 3.4): given a Hermitian H, a total
 * time t and an initial state x, approximate e^{-iHt} x without dense
 * matrices.  H arrives as a sum of Pauli strings with coefficients
 * (Section 4.4, "Benchmarks").  The library splits H into factors (the H_j of
 * the Trotter product, Eq. 4), exponentiates each factor exactly, stores each
 * factor exponential in the diagonal layout of Eq. 6 (Section 3.2), and
 * evolves the state by one DIA SpMV per factor per step (Alg. 1 inside the
 * repeat loop of Alg. 3).
 *
 * Conventions
 *  - A Pauli string has n_qubits characters from "IXYZ"; character k acts on
 *    qubit k, which is bit k of the basis index (least-significant first).
 *  - A state is N = 2^n_qubits complex amplitudes, interleaved (re, im), in
 *    the factors' dtype: HS_C64 = 2 x float, HS_C128 = 2 x double.  A batch
 *    of B states is B contiguous states ([B][N]).
 *  - Diagonal d of an N x N operator holds A[r, r+d] at storage index
 *    min(r, r+d) and has N - |d| entries (Section 3.2, Eq. 6; element map of
 *    the DiagonalTimesVector schematic, Section 3.3).
 *  - State and diagonal pointers must be 16-byte aligned (HS_EINVAL otherwise).
 *  - Device pointers are HIP device addresses on the current device; a
 *    stream argument is a hipStream_t (NULL = the default stream).  All device
 *    work is enqueued on that stream.  Every call that takes caller states
 *    or diagonals first checks that each is device (or managed) memory of the
 *    current device and lies inside one allocation, and returns HS_EINVAL
 *    before enqueuing anything otherwise: a host address must never reach a
 *    kernel.
 *  - Every function returns an hs_status.  On failure nothing is left half
 *    built, output handles are set to NULL, and hs_last_error() returns a
 *    message for the calling thread.  No C++ exception crosses this ABI.
 *  - Distinct hs_factors handles may be used concurrently from different
 *    threads on different streams; one handle must not be evolved
 *    concurrently with itself.
 */
#ifndef HAMSIM_H
#define HAMSIM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hs_factors_s *hs_factors;

typedef enum { HS_C64 = 0, HS_C128 = 1 } hs_dtype;

typedef enum {
    HS_OK = 0,
    HS_EINVAL = 1,          /* bad argument (size, pointer, string, flag) */
    HS_ENONHERMITIAN = 2,   /* a coefficient has |Im c| > 1e-12 max|c| */
    HS_EBUDGET = 3,         /* a single term's exponential exceeds the budget */
    HS_ENOMEM = 4,          /* device allocation failed */
    HS_EDEVICE = 5,         /* a HIP call failed */
    HS_ETOOLARGE = 6        /* n_qubits > 30, or a factor support > 10 qubits */
} hs_status;

/* build flags */
#define HS_MERGE_DIAG 1u    /* fold the diagonal factor D into the first group (U_1 D); default in Python */
#define HS_ORDER2 8u        /* symmetric second-order product (future-work section): per step
                               F_1..F_{L-1}(dt/2) F_L(dt) F_{L-1}..F_1(dt/2), F = (D, G_1..G_m) */
#define HS_ORDER4 16u       /* fourth-order Suzuki product: S2(p dt)^2 S2((1-4p) dt) S2(p dt)^2,
                               p = 1/(4 - 4^(1/3)).  Orders 2 and 4 keep D a factor of its own. */
/* evolve flags */
#define HS_RENORM 2u        /* divide each state by its FP64 norm after every step */
#define HS_NO_FUSE 4u       /* one launch per factor instead of fused multi-factor tiles */

#define HS_MAX_QUBITS 30
#define HS_MAX_SUPPORT 10
#define HS_MAX_BATCH 8      /* states per launch; larger batches run in chunks */

/*
 * hs_plan -- group the terms into factors and fix every factor's diagonal
 * set, on the host only (no device memory).  This is the structural dry run
 * of Section 3.2: offsets are known before any storage exists.
 *
 * Grouping (the paper leaves it open; reading used here): Z-only terms
 * (identity included) form the diagonal factor D = exp(-i dt E(x)).  The
 * other terms are placed first-fit in input order: a term joins the first
 * group all of whose members it commutes with and whose exact exponential
 * prod_k (cos(c_k dt) I - i sin(c_k dt) P_k) still has at most `budget`
 * numerically nonzero diagonals (entries with |value| <= 1e-15 count as
 * zero); otherwise it opens a new group.  This applies the diagonal budget
 * of Eq. 5 to each factor.  A step applies D first, then the groups in
 * creation order (first-order product, Eq. 4).
 *
 *   n_qubits     1..30
 *   n_terms      >= 1
 *   pauli_terms  n_terms NUL-terminated strings of exactly n_qubits chars
 *   coeffs       2*n_terms doubles, (re, im) per term; H must be Hermitian
 *   t            total time; steps >= 1 Trotter steps; dt = t / steps
 *   budget       >= 1, maximum diagonals per factor
 *   flags        HS_MERGE_DIAG, HS_ORDER2 or HS_ORDER4 (or 0)
 *   out          receives a handle that only supports the query calls
 *                (describe/footprint/free); hs_evolve rejects it.
 */
hs_status hs_plan(int n_qubits, int n_terms, const char *const *pauli_terms,
                  const double *coeffs, double t, int steps, int budget,
                  unsigned flags, hs_factors *out);

/*
 * hs_build_factors -- hs_plan, then build every factor's coefficient
 * diagonals on the device (Section 3.2 layout; paper's SpME diagonal case,
 * Section 3.3, for D).  Entries are computed in FP64 on the GPU:
 * U[r, r+d] = L[loc(r), loc(r+d)] (times D[r+d] for the factor carrying the
 * diagonal terms) when r and r+d agree outside the factor's support, else 0;
 * they are then stored as complex64 (dtype HS_C64, rounded to nearest) or
 * complex128.  Each diagonal starts on a 256-byte boundary.  The library owns
 * this memory until hs_free_factors.  Device memory is allocated and later
 * released stream-ordered on `stream`, which must stay valid until
 * hs_free_factors.  The call synchronises `stream` before returning.
 */
hs_status hs_build_factors(int n_qubits, int n_terms, const char *const *pauli_terms,
                           const double *coeffs, double t, int steps, int budget,
                           hs_dtype dtype, unsigned flags, void *stream, hs_factors *out);

/*
 * hs_evolve -- the repeat loop of Alg. 3 with the Trotter product of Eq. 4 as
 * the step: psi <- (U_F ... U_1)^steps psi, in place, for `batch` states
 * (device pointer to [batch][N] interleaved complex of the factors' dtype).
 * Enqueues kernels on `stream` and returns; faults surface at the caller's
 * next synchronisation.  May be called repeatedly: for first order,
 * evolve(k) followed by evolve(steps - k) gives bit-identical results to
 * evolve(steps) (orders 2 and 4 join consecutive steps of one call in the
 * joint factor, so a split call differs by rounding only).
 * flags: HS_RENORM (FP64 norm after each step, applied as a scale when the
 * next step loads the state, and once more at the end), HS_NO_FUSE.
 * complex64 states accumulate in FP32 over ascending offsets; complex128 in
 * FP64.  Results do not depend on the batch size or on fusion (with
 * HS_RENORM the FP64 norm sums per tile, and tiles differ between batch
 * sizes, so renormalised complex128 results agree to FP64 rounding).
 * Launch shapes follow four environment variables, read at every call (a
 * handle keeps one launch plan per setting): HAMSIM_WMIN_BYTES (shortest
 * row run of a strided tile, default 256), HAMSIM_MAX_FUSE (factors per
 * launch, 1..8, default 8), HAMSIM_XCD_SWIZZLE (which launches deal
 * contiguous eighths of their tiles to the 8 XCDs: 0 none, 1 all, 2 strided,
 * 3 contiguous, default 3) and HAMSIM_PAIR_LDS (which closed complex64
 * launches whose row pairs read adjacent LDS partners use the pair kernel:
 * 0 none, 1 all except one-state strided launches with row runs under
 * 1 KiB whose factors are stored in natural order, 2 all; odd offsets of
 * contiguous tiles included; default 1).  Results are
 * the same bits for every setting, and for every storage order
 * (hs_factor_storage).
 * A factor whose coupling range fits no tile held in LDS (e.g. X_0 X_{n-1}
 * at large n) is applied out of place into a scratch state (allocated on
 * first use, counted by hs_footprint) and copied back.  Calls that share a
 * handle share its workspace, so they must be ordered on one stream.
 * The state is checked (device memory, batch * N elements inside one
 * allocation) before anything else, also when steps is 0.
 * Small states (N <= 2048 complex64 or 1024 complex128 rows by default; the
 * environment variable HAMSIM_WHOLE_MAX_ROWS sets the cap, at most 8192 /
 * 4096 rows, 0 = never) evolve without HS_RENORM or HS_NO_FUSE in one launch
 * for all steps and states, each state held in LDS by one workgroup (same
 * values as the launch per run and step).
 */
hs_status hs_evolve(hs_factors f, void *psi, int batch, int steps, void *stream,
                    unsigned flags);

/* Description of a planned or built handle. */
hs_status hs_factors_info(hs_factors f, int *n_qubits, int *n_factors, int *n_terms,
                          int *n_diag_terms, int *dtype, double *dt, int *steps);
/* Term indices of the diagonal factor D, in input order (cap entries max). */
hs_status hs_diag_terms(hs_factors f, int *term_idx, int cap);
/* One step applies the stored factors in this order (factor indices; the
 * identity order 0..F-1 for first order).  *len receives the length.  For
 * orders 2 and 4, neighbours that share a generator are already combined
 * (their time steps add), e.g. the junctions F_1(p dt/2) F_1(p dt/2) of the
 * fourth-order product. */
hs_status hs_step_sequence(hs_factors f, int *seq, int cap, int *len);
/* The joint factor of a symmetric product, or -1 (first order, or a step of
 * one factor).  A symmetric step s_0 .. s_{L-1} starts and ends with the same
 * generator, so where two steps meet, hs_evolve applies s_{L-1} s_0 as the
 * one stored factor *factor whose time step is the sum of theirs: `steps`
 * steps apply s_0 .. s_{L-2} J, then (s_1 .. s_{L-2} J) steps-2 times, then
 * s_1 .. s_{L-1}; one step applies the sequence as it is. */
hs_status hs_step_joint(hs_factors f, int *factor);
/* time step h of factor k: its exponential is exp(-i h H_k) */
hs_status hs_factor_step(hs_factors f, int k, double *h);
/* Factor k: whether it carries D, its group size, its number of diagonals,
 * its support bit mask and its stored bytes. */
hs_status hs_factor_info(hs_factors f, int k, int *has_diag, int *n_group_terms,
                         int *n_diags, unsigned long long *support_mask, size_t *bytes);
hs_status hs_factor_terms(hs_factors f, int k, int *term_idx, int cap);
hs_status hs_factor_offsets(hs_factors f, int k, long long *offsets, int cap);
/* Copy entries [start, start + count) of diagonal j (ascending-offset order)
 * of factor k -- a diagonal holds N - |d| entries of the factors' dtype -- to
 * host memory; synchronises `stream`. */
hs_status hs_factor_copy_diagonal(hs_factors f, int k, int j, long long start, long long count,
                                  void *host_dst, void *stream);
/* Storage order of factor k's diagonals in device memory (the values are the
 * same in every order; hs_factor_copy_diagonal always returns natural
 * order).  Eq. 6 stores the coefficient A[r, r + d] of diagonal d at index
 * i = min(r, r + d).  With *split_bit = s > 0 and *chunk_bits = c, entry i
 * sits instead at
 *   ((i mod 2^s) >> c) * ((N - |d|) >> s << c) + (i >> s << c) + (i mod 2^c):
 * runs of 2^c entries, all values of i >> s of one run column one after the
 * other, so that a tile holding every level of bits [s, ...) for a window of
 * low rows reads one short stretch per column instead of one run per level
 * 2^s entries apart.  Each diagonal still holds exactly N - |d| entries.
 * The library chooses it at build for factors applied in strided tiles whose
 * levels lie at least HAMSIM_PERM_MIN_BYTES (default 1 MiB) apart, with
 * runs of four of those tiles' row windows; s = c = 0 is the natural order.
 * Either output may be null. */
hs_status hs_factor_storage(hs_factors f, int k, int *split_bit, int *chunk_bits);
/* Bytes of device memory an evolution of `batch` states needs: the stored
 * diagonals (Eq. 6: N - |d| entries per diagonal, each start aligned to 256
 * bytes), the caller's states and the library's workspace (the scratch state
 * of an open launch, reduction partials).  Used for admission by HBM
 * footprint in a served loop.  Counts the handle's dtype (complex64 for a
 * handle from hs_plan, which has none yet). */
hs_status hs_footprint(hs_factors f, int batch, size_t *bytes);
/* The same figure for the handle built with `dtype`: element size, diagonal
 * alignment and the dtype's own tile limits (a complex128 tile holds half
 * the rows, so a factor closed in complex64 can need the open launch and its
 * scratch state in complex128).  For admission before building. */
hs_status hs_footprint_dtype(hs_factors f, int batch, hs_dtype dtype, size_t *bytes);
/* The launches one Trotter step makes for `batch` states with evolve `flags`:
 * *n_launches receives their count; launch i applies the factors at
 * positions [first_factor[i], first_factor[i] + n_factors[i]) of the part's
 * factor sequence (arrays of `cap` entries, may be NULL to query the count).
 * `part` selects the step: 0 a lone step (the sequence of hs_step_sequence),
 * and of an evolution of several steps 1 the first (s_0 .. s_{L-2} J),
 * 2 a middle one (s_1 .. s_{L-2} J), 3 the last (s_1 .. s_{L-1}), with J the
 * joint factor (hs_step_joint); without a joint all four are the plain step.
 * A launch of several factors is one fused kernel; batches above
 * HS_MAX_BATCH repeat the list per chunk. */
hs_status hs_step_launches(hs_factors f, int batch, unsigned flags, int part, int *n_launches,
                           int *first_factor, int *n_factors, int cap);
/* Sets *violated to 1 if any in-place launch met a nonzero coefficient that
 * couples rows of different tiles (never for factors built here); syncs. */
hs_status hs_check(hs_factors f, void *stream, int *violated);
/* Release a handle.  Device memory is returned stream-ordered on the build
 * stream; work that uses the factors on other streams must have completed. */
hs_status hs_free_factors(hs_factors f);

/*
 * hs_dia_spmv -- y = A x for an arbitrary operator in the diagonal layout
 * (Alg. 1), out of place, for `batch` vectors ([batch][N]).
 *   n_diags     number of stored diagonals (1..65535)
 *   offsets     host array, strictly ascending, each in (-N, N)
 *   diags       host array of n_diags device pointers; diags[j] holds
 *               N - |offsets[j]| entries of `dtype`
 *   x, y        device, [batch][N]; must not overlap; x, y and every
 *               diagonal start on a 16-byte boundary
 *   N           any size in [1, 2^30] (a power of two takes the LDS tiles
 *               with strided shapes; any other N contiguous tiles, the last
 *               one partial)
 * Rows accumulate diagonals in ascending-offset order.
 */
hs_status hs_dia_spmv(int n_diags, const long long *offsets, const void *const *diags,
                      const void *x, void *y, int batch, long long N, hs_dtype dtype,
                      void *stream);

/* FP64 squared norms <psi|psi> of `batch` device states (the norm that the
 * paper's Alg. 2 takes of its Taylor terms, here of states; the per-step
 * renormalisation of hs_evolve uses the same FP64 accumulation); out: host
 * [batch]; syncs. */
hs_status hs_norm2(const void *psi, int batch, long long N, hs_dtype dtype, void *stream,
                   double *out);

/*
 * hs_fidelity -- state fidelity (Section 4.3, "State Fidelity"; the formula
 * is not printed -- reading: F = |<phi|psi>|^2 / (<phi|phi><psi|psi>)),
 * accumulated in FP64 in one pass over both device states.  phi and psi may
 * have different dtypes.  out: host [batch][5] = Re<phi|psi>, Im<phi|psi>,
 * <phi|phi>, <psi|psi>, F.  Syncs.
 */
hs_status hs_fidelity(const void *phi, int phi_dtype, const void *psi, int psi_dtype,
                      int batch, long long N, void *stream, double *out);

/*
 * hs_fidelity_noalloc -- hs_fidelity for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  It allocates nothing (no hipMalloc, no library
 * allocation) and does not synchronise: the same FP64 reduction kernels as
 * hs_fidelity run on `stream` with their partial sums in a static device
 * array of 256.25 KiB per GPU (held until the process ends), and
 * out_dev (device, [batch][5] doubles, the layout of hs_fidelity's output)
 * receives the same values, bit for bit, when the stream reaches it.
 * batch is 1..HS_MAX_BATCH (8); larger batches return HS_EINVAL.  Every call
 * on one GPU shares that array: calls that overlap in time on one GPU (on
 * different streams or threads) race and must be ordered by the caller.
 * Nothing needs clearing between calls (each call writes every partial it
 * reads).
 */
hs_status hs_fidelity_noalloc(const void *phi, int phi_dtype, const void *psi, int psi_dtype,
                              int batch, long long N, void *stream, double *out_dev);

/* ------------------------------------------------------------------------
 * General operators in the diagonal layout, device resident.  These carry
 * the paper's single-propagator pipeline: H is stored by its diagonals, its
 * short-time propagator U ~ exp(-i H dt) is built by a truncated Taylor
 * series of SpGEMM products (Alg. 2), the step count can be chosen as the
 * smallest one whose propagator meets the diagonal budget (Section 3.1
 * flowchart, Eq. 5), and U is applied repeatedly to the state (Alg. 3).
 * Entries are complex128 (FP64) unless converted with hs_dia_to_c64.
 * Memory is allocated and released stream-ordered on the stream given at
 * creation, which must stay valid until hs_dia_free.
 * ------------------------------------------------------------------------ */
typedef struct hs_dia_s *hs_dia;

/* H = sum_k c_k P_k by its diagonals; diagonals whose entries all cancel
 * (e.g. XX + YY on the offsets +-3 of a bond) are not stored.  Same string
 * and coefficient conventions as hs_plan.  Synchronises `stream`. */
hs_status hs_dia_from_pauli(int n_qubits, int n_terms, const char *const *pauli_terms,
                            const double *coeffs, void *stream, hs_dia *out);
/* An operator of any size N in [1, 2^30] from host diagonals: host_diags[j]
 * holds N - |offsets[j]| complex128 entries (interleaved re, im), storage
 * index min(row, col); offsets strictly ascending.  Synchronises `stream`. */
hs_status hs_dia_from_host(long long N, int n_diags, const long long *offsets,
                           const double *const *host_diags, void *stream, hs_dia *out);
hs_status hs_dia_info(hs_dia A, long long *N, int *n_diags, int *dtype);
hs_status hs_dia_offsets(hs_dia A, long long *offsets, int cap);
/* entries [start, start + count) of diagonal j to host memory; syncs */
hs_status hs_dia_copy_diagonal(hs_dia A, int j, long long start, long long count, void *host_dst,
                               void *stream);
/* C = A B (complex128).  C's diagonals are every a + b in (-N, N) of A's and
 * B's offsets (structural: no cancellation check); entry (r, r+c) sums
 * A[r, r+a] B[r+a, r+c] over the pairs a + b = c, in ascending a (the
 * paper's SpGEMM, Section 3.3).  Synchronises `stream`. */
hs_status hs_dia_spgemm(hs_dia A, hs_dia B, void *stream, hs_dia *C);
/* largest entry modulus (FP64); syncs */
hs_status hs_dia_maxabs(hs_dia A, void *stream, double *out);
/* Alg. 2 in its scaling-and-squaring form (SpME subsection):
 * X = -i H dt / 2^s; U = T = I; for k = 1..max_iter: T <- T X / k; stop when
 * max |T_ij| < tol (T not added), else U += T; then s times U <- U U (SpGEMM).
 * squarings: s, or -1 for the smallest s >= 0 with |dt| nu / 2^s <= 1/2,
 * where nu = the sum over H's diagonals (ascending offset) of their largest
 * entry modulus (>= ||H||_1, ||H||_inf, ||H||_2); at most 60.  A diagonal H
 * takes the exact elementwise exponential.  *n_terms = the number of Taylor
 * terms added after I (0 for diagonal H).  Each term's norm is computed
 * before the term is stored, so the dropped term takes no memory.  H must
 * be complex128.  Syncs. */
hs_status hs_spme(hs_dia H, double dt, double tol, int max_iter, int squarings, void *stream,
                  hs_dia *U, int *n_terms);
/* Smallest r such that hs_spme(H, t / r, tol, max_iter, -1) has at most
 * `budget` diagonals (structural count, after squaring: each squaring maps
 * the offset set S to S + S): r = 1 for diagonal H; else r = 1 if it
 * meets the budget, otherwise doubling u = 2, 4, ... until it does, then
 * bisection between the last failing and the first passing value.  A probe
 * stops as soon as a Taylor term above the tolerance would push the count
 * past the budget.  The probes share one sequence of powers of H: term k at
 * step dt has largest entry |dt|^k / k! max|H^k| and H^k's offsets, so each
 * power is formed once (and stored only while its offsets fit the budget).
 * H must be complex128.  HS_EBUDGET above 2^24.  Syncs. */
hs_status hs_estimate_timesteps(hs_dia H, double t, int budget, double tol, int max_iter,
                                void *stream, int *steps);
/* complex64 copy of a complex128 operator (round to nearest); syncs */
hs_status hs_dia_to_c64(hs_dia A, void *stream, hs_dia *out);
/* Alg. 3's loop: psi <- U^steps psi for `batch` device states of U's dtype,
 * by repeated DIA SpMV (out of place with library scratch, result written
 * back to psi).  The state is checked before anything else, also when
 * steps is 0.  Synchronises `stream`. */
hs_status hs_dia_evolve(hs_dia U, void *psi, int batch, int steps, void *stream);
/* nu(A) = sum over A's stored diagonals (ascending offset) of each one's
 * largest entry modulus; bounds ||A||_1, ||A||_inf and ||A||_2.  Syncs. */
hs_status hs_dia_norm_bound(hs_dia A, void *stream, double *nu);

/*
 * The Taylor expansion of exp(-i H dt) fused into the state update (future-
 * work section: no propagator is formed).  One step applies
 *     p_K(X) x = sum_{k=0..K} X^k x / k!,   X = -i dt H,
 * by Horner's rule, K stages w <- x + (-i dt / j) H w for j = K .. 1 from
 * w = x, each stage one DIA SpMV of H (Alg. 1) with the update fused into
 * its epilogue.  H is read once per stage; U is never built, so the memory
 * and traffic of the propagator's diagonals (Alg. 2, Section 3.2) vanish.
 */
/* Smallest K >= 1 (at most max_terms <= 64) with (|dt| nu(H))^(K+1) / (K+1)!
 * < tol: the first dropped term of the series then has 2-norm below tol.
 * HS_EBUDGET when max_terms is not enough.  Syncs. */
hs_status hs_taylor_terms(hs_dia H, double dt, double tol, int max_terms, void *stream, int *K);
/* Smallest r >= 1 with |t / r| nu(H) <= theta (theta > 0), the step count
 * that keeps X small enough for a short series; HS_EBUDGET above 2^30.
 * Syncs. */
hs_status hs_taylor_steps(hs_dia H, double t, double theta, void *stream, int *steps);
/* psi <- p_K(-i dt H)^steps psi for `batch` device states ([batch][N], of
 * H's dtype, 16-byte aligned), 1 <= K <= 64.  In place; library scratch of
 * two states per chunk of HS_MAX_BATCH (one for K = 1), stream-ordered.
 * The state is checked before anything else, also when steps is 0.
 * Synchronises `stream`. */
hs_status hs_taylor_evolve(hs_dia H, void *psi, int batch, double dt, int K, int steps, void *stream);
hs_status hs_dia_free(hs_dia A);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *hs_last_error(void);
int hs_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
