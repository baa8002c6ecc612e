// Internal declarations shared by the HIP translation units of libtatrg.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace tatrg {

// ---------------------------------------------------------------------------- GEMM
// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], row-major, float64, b < batch.
// op(A) is M x K: A stored M x K (lda) or, with ta, K x M (lda).  op(B) is K x N: B stored
// K x N (ldb) or, with tb, N x K (ldb).  C is M x N (ldc).  Batch strides in elements.
struct GemmArgs {
  int64_t M, N, K;
  const double* A; int64_t lda; int64_t sA; bool ta;
  const double* B; int64_t ldb; int64_t sB; bool tb;
  double* C; int64_t ldc; int64_t sC;
  double alpha, beta;
  int64_t batch;
  // Optional device-side predicate: when `cond` is set the launch does nothing unless
  // (*cond != 0) == cond_when (lets a fallback path be launched without a host sync).  With
  // cond_stride > 0 (gemm_f64 and its split-K form) batch entry b reads cond[b * cond_stride].
  const int* cond = nullptr;
  bool cond_when = false;
  int64_t cond_stride = 0;
  // Symmetric output (op(A) op(B) = X X^T with M = N): split-K computes the tiles on and
  // above the diagonal only and its reduction mirrors them.
  bool sym = false;
};
void gemm_f64(const GemmArgs& g, hipStream_t st);

// Planes of op(B) produced elsewhere (by a Bf16PlanesOut epilogue): p[i] is [batch][N][Kp]
// with Kp = K rounded up to 32, zero for K <= k < Kp; stride is the batch stride in elements.
struct Bf16PlanesIn {
  const uint16_t* p[3];
  int64_t stride;
};
// C written as its three bf16 planes, split exactly as an operand would be, instead of as
// float64.  Element (row, col) of batch entry b, with row = r1 R2 + r2 and col = c1 C2 + c2,
// goes to offset b stride + (r1 C1 + c1) Kp + r2 C2 + c2 of every plane: the planes of a
// following GEMM's op(B) over K = R2 C2 with rows (r1, c1).  Offsets R2 C2 <= k < Kp of
// the M / R2 x C1 rows of every batch entry are zeroed.  cap bounds every plane (elements).
struct Bf16PlanesOut {
  uint16_t* p[3];
  int64_t R2, C1, C2, Kp, stride, cap;
};

// Split-bf16 variant: every operand is split x = x0 + x1 + x2 into bf16 planes and the six
// products with i + j <= 2 are accumulated in fp32 on the bf16 MFMA units.  Same contract.
// ev_after_split (optional) is recorded on st between the plane splitting and the GEMM.
// b_in (optional) supplies op(B) as planes (g.B is then not read); c_out (optional) takes C
// as planes (g.C is then not written; needs beta = 0, M % R2 = 0, N <= C1 C2, N % C2 = 0,
// R2 C2 <= Kp and every offset below cap).  Returns false, launching nothing, when
// planes_ws holds fewer than gemm_bf16x3_ws_doubles(g, b_in != nullptr) doubles or an
// argument of b_in or c_out does not fit.
// group_m: rows of tiles per group of the work-group order (results do not depend on it);
// -1 takes the default (6 with 12 or more rows of tiles, else 0: M fastest throughout).
bool gemm_bf16x3(const GemmArgs& g, double* planes_ws, size_t planes_ws_doubles,
                 hipStream_t st, hipEvent_t ev_after_split = nullptr,
                 const Bf16PlanesIn* b_in = nullptr, const Bf16PlanesOut* c_out = nullptr,
                 int group_m = -1);
// Workspace (in doubles) gemm_bf16x3 needs for the bf16 planes it splits (op(A) always,
// op(B) unless it is given as planes).
size_t gemm_bf16x3_ws_doubles(const GemmArgs& g, bool b_given = false);
// K rounded up to the split GEMM's step of 32 (the row length of its planes).
int64_t bf16x3_kpad(int64_t K);
// The three bf16 planes of the contraction operand FM4[(i4a a)][(g k4 kX)] as op(B) of the
// split GEMM ([N][Kp] with N = (g k4 kX), K = (i4a a) = c^2, zero for K <= k < Kp), read
// straight from tmp[(i4a k4)][(a kX g)] (extents c, c, c, L, c): the planes split3 would make
// of FM4, bit for bit.  planes: 3 N Kp elements (cap); false, launching nothing, when short.
bool fm4_planes(const double* tmp, int c, int L, uint16_t* planes, int64_t cap, hipStream_t st);
// Products every later split GEMM runs: 6 (the engine) or 3 (i + j <= 1, an accuracy
// ablation).  Returns the previous count, -1 for another n.  Process-wide.
int set_split_products(int n);

// C = alpha X^T Y + beta C for the skinny shapes X (K x M), Y (K x N) with M, N <= 96
// (GemmArgs with ta && !tb, batch 1): one wave per chunk of rows writes an M x N partial
// sum to `partial`, summed in a fixed order afterwards.  Also C = X Y^T over long rows
// (!ta && tb, batch 1; the general 96 x 96 case is declined), one wave per chunk of columns.  Returns false (nothing launched)
// when the shape does not qualify or `partial` is too small.
bool gram_tn(const GemmArgs& g, double* partial, size_t partial_doubles, hipStream_t st);

// Long-K GEMM with small M x N: the K range is split into `parts` chunks written to
// `partial` (parts * batch * M * N doubles) and summed in a fixed order (deterministic).
void gemm_f64_splitk(const GemmArgs& g, int parts, double* partial, hipStream_t st);

// ---------------------------------------------------------------------------- TSQR
// Orthonormal basis of a tall panel Y (m x n, row-major, leading dim ld, m >= n, n <= 96),
// computed in place by Householder reflections on row blocks and a reduction tree of the
// R factors.  On return Y holds Q (m x n) with Y_in = Q R; R (n x n) is written to R_out
// when not null.  ws must hold tsqr_ws_doubles(m, n) doubles.
size_t tsqr_ws_doubles(int64_t m, int n);
void tsqr(double* Y, int64_t m, int n, int64_t ld, double* R_out, double* ws, hipStream_t st,
          const int* run_if_set = nullptr);

// Cholesky factor of an n x n Gram G = R^T R (n <= 96, one workgroup) with its inverse.
// pass 0 factors G + shift_coef * tr(G) * I (the shifted first pass of CholeskyQR3) and fails
// only on a non-finite or non-positive pivot; pass 1 fails when a pivot is <= 1e-14 of the
// largest diagonal entry; pass 2 (G close to the identity) when a pivot leaves (0.25, 4).  A
// failure sets *fail = pass + 1 (and, when sticky is given, ORs 1 into *sticky) and leaves
// R, Rinv unwritten.  Does nothing when *fail is already set.
// batch > 1 factors `batch` Grams (strides sG, sR, sRi) with their own flags fail[b * sf].
void chol_inv(const double* G, double* R, double* Rinv, int n, int pass, int* fail,
              hipStream_t st, double shift_coef = 0.0, int* sticky = nullptr, int batch = 1,
              int64_t sG = 0, int64_t sR = 0, int64_t sRi = 0, int sf = 0);

// Solves X L^T = B in place for `batch` tall panels X (m x n, leading dim ldx, stride sX)
// with lower-triangular L (n x n, stride sL): column blocks of 64, each a GEMM update by the
// blocks before it and a forward substitution per row against the diagonal block.
void trsm_right_lower_t(double* X, int64_t ldx, int64_t m, const double* L, int n, int batch,
                        int64_t sX, int64_t sL, hipStream_t st);

// Right-looking blocked Cholesky of `batch` SPD n x n matrices (stride n*n) in place: A <- L
// (lower, zeros above), with the inverses of its 64 x 64 diagonal blocks written to Dinv
// (batch x ceil(n / 64) blocks of 64 x 64).  Per block column: the diagonal block and its
// inverse (one wave), the panel below by a GEMM with that inverse, the trailing update by a
// GEMM.  A non-positive pivot ORs 1 into flag[0].
void cholesky_blocked_inv(double* A, double* Dinv, int n, int batch, int* flag,
                          hipStream_t st);

// cholesky_blocked_inv of A + shift_rel * trace(A) * I (per matrix).
void cholesky_shifted_inv(double* A, double* Dinv, int n, int batch, double shift_rel,
                          int* flag, hipStream_t st);

// Inverse of `batch` lower-triangular n x n matrices L (stride n*n) whose 64 x 64 diagonal
// blocks are already inverted in Dinv (as cholesky_blocked_inv leaves them), by doubling the
// inverted blocks: the off-diagonal block of [[A, 0], [B, C]]^{-1} is -C^{-1} B A^{-1}.
// Linv: batch x n x n; T: scratch of at least n * n / 2 doubles.  With `partial` (device,
// partial_doubles), the products of the upper levels, which have few output tiles, are split
// along K through it.
void tri_inv_lower(const double* L, const double* Dinv, double* Linv, double* T, int n,
                   int batch, hipStream_t st, double* partial = nullptr,
                   size_t partial_doubles = 0);

// Checks the diagonal of `batch` lower Cholesky factors (n x n, stride n*n): ORs `code` into
// *flag when a diagonal entry is not finite or not positive, when the smallest pivot L_ii^2
// is below min_ratio times the largest, or when a pivot leaves (lo, hi).  Leaves *flag alone
// otherwise.
void chol_check(const double* L, int n, int batch, double min_ratio, double lo, double hi,
                int* flag, hipStream_t st, int code = 1);

// ---------------------------------------------------------------------------- small dense
// One-sided Jacobi SVD of `batch` square n x n matrices (n <= 96): A = U diag(S) V^T with S
// descending.  A (read only), U, V row-major n x n, strides n*n; S stride n.  Columns of U
// with S = 0 are returned as zero.
void jacobi_svd(const double* A, double* U, double* S, double* V, int n, int batch,
                hipStream_t st);

// In-place lower Cholesky of `batch` n x n SPD matrices (stride n*n) after adding
// shift_rel * trace(A) to the diagonal; the strict upper triangle is zeroed.  A non-positive
// pivot raises bit 1 of *flag.
void cholesky_shifted(double* A, int n, int batch, double shift_rel, int* flag,
                      hipStream_t st);

// Gauge fixing of an SVD: s (n, descending) and probe projections P (n_probes x n, P[p][j]
// = probe p . singular vector j) give an orthogonal block-diagonal O (n x n) that rotates
// every cluster of (near-)degenerate singular vectors into the canonical basis.
void gauge_rotation(const double* s, const double* P, double* O, int n, int n_probes,
                    double tau_null, double tau_deg, hipStream_t st);

// ---------------------------------------------------------------------------- misc
// Gaussian sketch element (i, j) of a rows x cols matrix is Philox4x32-10 draw number
// e = i * cols + j for (seed, step, site); written to out[i*ld + j] (or out[j*ld + i] when
// transposed).  With row_split = s > 0 (a divisor of rows), row i = u * s + v is stored as row
// v * (rows / s) + u: a sketch whose rows are indexed (u, v) laid out in (v, u) order.
// max_blocks > 0 caps the grid (the kernel strides over the draws), for a draw that runs
// beside latency-bound work and should leave most of the chip to it.
void philox_gaussian(double* out, int64_t rows, int64_t cols, int64_t ld, bool transposed,
                     uint64_t seed, uint32_t step, uint32_t site, hipStream_t st,
                     int64_t row_split = 0, int max_blocks = 0);

// The generator's four 32-bit output words for counter pairs pair0 .. pair0 + npairs - 1 of
// (seed, step, site), pair by pair (out holds 4 * npairs words, 16-byte aligned).
void philox_words(uint32_t* out, int64_t pair0, int64_t npairs, uint64_t seed, uint32_t step,
                  uint32_t site, hipStream_t st);

// out = permutation of a row-major tensor of rank r <= 6 with dims d: out dim k is input
// dim perm[k].
void permute(const double* in, double* out, int rank, const int64_t* dims, const int* perm,
             hipStream_t st);

// y = x diag(s) for a rows x cols row-major x (y, x distinct).
void copy_scale_cols(double* y, const double* x, const double* s, int64_t rows, int64_t cols,
                     hipStream_t st);
// x[i][j] *= s[j] for an rows x cols row-major matrix (ld).
void scale_cols(double* x, const double* s, int64_t rows, int64_t cols, int64_t ld,
                hipStream_t st);

// A factor L (n x n) with L L^T = P of `batch` symmetric positive semidefinite P (n <= 96,
// strides n^2): the Jacobi SVD P = U S V^T, L = U S^{1/2} (U = V on the nonzero singular
// values of a semidefinite P; columns with S = 0 are zero).  S, V: scratch of batch n and
// batch n^2 doubles.
void psd_factor(const double* P, double* L, double* S, double* V, int n, int batch,
                hipStream_t st);

// y = x (n doubles).
// Order parameter X = (Tr A)^2 / Tr A^2 of T = sum_g Phi[., g] Psi[., g] (chi^5 doubles
// each, legs (l1 l2 l3 l4 gamma)), A_kl = T with the legs of the three slots other than
// open_slot (0..3) traced, k and l the forward and backward legs of open_slot.  Writes
// out[0]; part holds order_parameter_ws_doubles(chi) doubles.  chi <= 64.  Deterministic.
constexpr int OP_PARTS = 128;
size_t order_parameter_ws_doubles(int chi);
void order_parameter(const double* phi, const double* psi, int chi, int open_slot,
                     double* part, double* out, hipStream_t st);
void copy(double* y, const double* x, int64_t n, hipStream_t st);

// Fill with zeros / write the identity into an n x n block (ld).
void zero(double* x, int64_t n, hipStream_t st);
void identity(double* x, int n, int64_t ld, hipStream_t st);

// (A + A^T)/2 in place for `batch` n x n matrices (stride n*n).
void symmetrize(double* A, int n, int batch, hipStream_t st);

// Upper factor R = L^T from a lower Cholesky factor (batch, stride n*n), out of place.
void transpose_batched(const double* in, double* out, int rows, int cols, int batch,
                       hipStream_t st);

}  // namespace tatrg
