/*
 * tatrg_testing.h - kernel-level entry points of libtatrg for parity tests.
 *
 * These expose the building blocks of the RG step (include/tatrg.h) so that each can be
 * compared with an independent reference: the FP64 MFMA GEMM, the Householder TSQR, the
 * one-sided Jacobi SVD, the shifted Cholesky, the Philox4x32-10 Gaussian sketch, the leg
 * permutation and the gauge rotation of degenerate singular subspaces.  All pointers are
 * device pointers unless stated; matrices are row-major float64; every call is
 * asynchronous on `stream` (a hipStream_t, NULL = default).  Return 0 on success, -1 on
 * invalid arguments, -3 on a HIP launch error.
 */
#ifndef TATRG_TESTING_H
#define TATRG_TESTING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C[b] = alpha op(A[b]) op(B[b]) + beta C[b]; op(A) M x K (A stored K x M when ta),
 * op(B) K x N (B stored N x K when tb); batch strides sA, sB, sC in elements.
 * parts > 1 splits K and sums the parts in order through `partial`
 * (parts * batch * M * N doubles).  parts < 0 selects the skinny-product kernels for batch 1,
 * M, N <= 96: ta = 1, tb = 0 (X^T Y over long columns, one wave per chunk of rows) or
 * ta = 0, tb = 1 (X Y^T over long rows, one wave per chunk of columns; the general 96 x 96
 * case is declined), with `partial` holding -parts * 1024 doubles; returns -1 when the shape
 * does not qualify.  With A == B (same
 * pointer, stride and leading dimension), M == N and ta != tb the product is symmetric and
 * split-K computes only the tiles on and above the diagonal, mirroring the rest. */
int tatrg_test_gemm(const double* A, const double* B, double* C, int64_t M, int64_t N,
                    int64_t K, int64_t lda, int64_t ldb, int64_t ldc, int ta, int tb,
                    double alpha, double beta, int64_t batch, int64_t sA, int64_t sB,
                    int64_t sC, int parts, double* partial, void* stream);

/* Split-bf16 GEMM (three bf16 planes per operand, six products, fp32 accumulation in windows
 * of 128 along K summed in float64).  Same operand conventions as tatrg_test_gemm; ws holds
 * tatrg_test_gemm_bf16x3_ws(...) doubles. */
size_t tatrg_test_gemm_bf16x3_ws(int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb,
                                 int ta, int tb, int64_t batch, int64_t sA, int64_t sB);
int tatrg_test_gemm_bf16x3(const double* A, const double* B, double* C, int64_t M, int64_t N,
                           int64_t K, int64_t lda, int64_t ldb, int64_t ldc, int ta, int tb,
                           double alpha, double beta, int64_t batch, int64_t sA, int64_t sB,
                           int64_t sC, double* ws, void* stream);

/* Accuracy ablation of the split-bf16 engine: every split GEMM launched afterwards, in any
 * handle of the process, runs n = 3 products (i + j <= 1, about 2^-16 of |A||B|) or n = 6
 * (i + j <= 2, the engine's default, about 2^-24).  Returns the previous count, -1 for any
 * other n.  Not for concurrent use with running steps. */
int tatrg_test_split_products(int n);

/* The two contraction GEMMs chained through bf16 planes: P = A1 B1 (A1 row-major
 * [(r1 r2)][K1], B1 row-major [K1][(c1 c2)]) is written by the split GEMM's epilogue as the
 * three bf16 planes of P viewed as [r1][c1][(r2 c2)], and C[r1] = A2^T P[r1] (A2 row-major
 * [(r2 c2)][M2], C row-major [R1][M2][C1]) reads them without splitting P again.  ws: at
 * least tatrg_test_gemm_bf16x3_chain_ws(...) doubles of device memory (0 for a bad shape).
 * Returns 0, -1 for bad arguments, -3 for a launch error. */
size_t tatrg_test_gemm_bf16x3_chain_ws(int64_t R1, int64_t R2, int64_t C1, int64_t C2,
                                       int64_t K1, int64_t M2);
int tatrg_test_gemm_bf16x3_chain(const double* A1, const double* B1, const double* A2,
                                 double* C, int64_t R1, int64_t R2, int64_t C1, int64_t C2,
                                 int64_t K1, int64_t M2, double* ws, size_t ws_doubles,
                                 void* stream);

/* Doubles of workspace tatrg_test_tsqr needs for an m x n panel. */
size_t tatrg_test_tsqr_ws(int64_t m, int n);

/* In-place orthonormal factor of Y (m x n, ld >= n, m >= n, 1 <= n <= 96): Y <- Q with
 * Y_in = Q R; R (n x n) written to R when not NULL. */
int tatrg_test_tsqr(double* Y, int64_t m, int n, int64_t ld, double* R, double* ws,
                    void* stream);

/* One-sided Jacobi SVD of `batch` n x n matrices (n <= 96): A = U diag(S) V^T, S
 * descending. */
int tatrg_test_svd(const double* A, double* U, double* S, double* V, int n, int batch,
                   void* stream);

/* In-place lower Cholesky of `batch` n x n SPD matrices after adding
 * shift_rel * trace to the diagonal; flag[0] set to 1 on a non-positive pivot. */
int tatrg_test_cholesky(double* A, int n, int batch, double shift_rel, int* flag,
                        void* stream);

/* Blocked Cholesky with inverse of `batch` SPD n x n matrices A (stride n*n), the
 * factorisation of the bond swap's panel Grams and of the squeezer Grams: A <- L (lower,
 * zeros above) with A = L L^T; Dinv receives the inverses of L's 64 x 64 diagonal blocks
 * (batch x ceil(n / 64) x 64 x 64 doubles) and Linv (batch x n x n) the full inverse L^{-1};
 * T is scratch of n * n / 2 doubles.  A pivot that is not positive sets flag[0] = 1. */
int tatrg_test_cholesky_blocked_inv(double* A, double* Dinv, double* Linv, double* T, int n,
                                    int batch, int* flag, void* stream);

/* Upper Cholesky factor R (G = R^T R) and its inverse of one n x n Gram (n <= 96), the
 * building block of the CholeskyQR orthonormalisation.  pass 0 factors
 * G + shift_coef * tr(G) * I and fails only on a non-positive or non-finite pivot; pass 1
 * fails when a pivot (of L D L^T) is <= 1e-14 of the largest diagonal entry; pass 2 when a
 * pivot leaves (0.25, 4).  A failure sets *fail = pass + 1 (device int, left untouched
 * otherwise; nothing is computed when it is already set) and R, Rinv are then not written. */
int tatrg_test_chol_inv(const double* G, double* R, double* Rinv, int n, int pass,
                        double shift_coef, int* fail, void* stream);

/* tatrg_test_chol_inv over `batch` Grams at once (G, R, Rinv: batch x n x n, contiguous), as
 * the batched range finders run it: entry b has its own flag fail[b] (device ints), and a
 * failed entry leaves the others unaffected.  Returns 0, -1 for bad arguments, -3 for a
 * launch error. */
int tatrg_test_chol_inv_batched(const double* G, double* R, double* Rinv, int n, int pass,
                                double shift_coef, int* fail, int batch, void* stream);

/* Gaussian sketch: element (i, j) of a rows x cols matrix is Philox4x32-10 draw number
 * i*cols + j of (seed, step, site). */
int tatrg_test_philox(double* out, int64_t rows, int64_t cols, uint64_t seed, uint32_t step,
                      uint32_t site, void* stream);

/* Raw Philox4x32-10 output of the counters the sketches use: for t < npairs, pair
 * p = pair0 + t (elements 2p and 2p + 1 of a sketch) has counter (lo32(p), hi32(p), step,
 * site) and key (lo32(seed), hi32(seed)); its four output words go to out[4t .. 4t + 3].
 * out: device, 4 * npairs uint32, 16-byte aligned.  -1 for pair0 < 0, npairs < 1 or a
 * misaligned out. */
int tatrg_test_philox_words(uint32_t* out, int64_t pair0, int64_t npairs, uint64_t seed,
                            uint32_t step, uint32_t site, void* stream);

/* out = permutation of a rank <= 6 row-major tensor; dims and perm are HOST arrays. */
int tatrg_test_permute(const double* in, double* out, int rank, const int64_t* dims,
                       const int* perm, void* stream);

/* Gauge rotation O (n x n) from singular values s (n) and probe projections P
 * (n_probes x n). */
int tatrg_test_gauge(const double* s, const double* P, double* O, int n, int n_probes,
                     double tau_null, double tau_deg, void* stream);

/* Measurement hooks.  Live timing of the four contraction GEMMs of each step (the
 * dominant kernels, Eqs. (makeMG)/(makeMH)): tatrg_profile_enable reserves event pairs for
 * up to max_launches launches (0 turns timing off) and brackets each launch with HIP events
 * on the handle's stream; tatrg_profile_read synchronises, returns the summed device time
 * of the recorded launches, their count and the algorithmic flops of one launch
 * (2 L^2 chi^5), and clears the record.  `h` is a tatrg_handle*. */
struct tatrg_handle;
int tatrg_profile_enable(struct tatrg_handle* h, int max_launches);
int tatrg_profile_read(struct tatrg_handle* h, double* total_ms, int32_t* launches,
                       double* flops_per_launch);

/* Speculation on the CholeskyQR orthonormalisations of a step: after a step in which no
 * CholeskyQR pass failed, the next step of that temperature does not launch the Householder
 * fallback kernels; a failed pass is caught at the end of the step, whose input was saved,
 * and the step is replayed with the fallback.  Speculation is otherwise limited to steps
 * after one with no failed pass that took the compressed cell middle.  on = 1 makes every
 * following step speculate, on = 0 restores the rule, on < 0 leaves it; *replays (may be
 * NULL) receives the number of replays so far.  Returns 0, -1 for a null handle. */
int tatrg_test_speculation(struct tatrg_handle* h, int on, int64_t* replays);

/* Stage timing of the profiled steps (tatrg_profile_enable also reserves events at the stage
 * boundaries of up to ceil(max_launches / 4) steps, on the handle's stream).  Synchronises; stage_ms[0..5] (host) receives the summed
 * device time of canonical form (S0, Section 2), bond swap (S1, Eq. (1)), isometries (S2,
 * Eqs. (2)-(3)), triad tensors (S3, Eqs. (4)-(11)), squeezers (S4) and contraction with the
 * slot rotation (S5, Eqs. (makeMG)/(makeMH)); *steps the number of steps timed.  Clears the
 * stage record.  Returns 0, -1 for null arguments, -3 on a HIP error. */
int tatrg_profile_read_stages(struct tatrg_handle* h, double* stage_ms, int32_t* steps);

#ifdef __cplusplus
}
#endif

#endif /* TATRG_TESTING_H */
