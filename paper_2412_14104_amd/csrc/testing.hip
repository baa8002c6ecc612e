// Kernel-level entry points for parity tests (include/tatrg_testing.h).
#include "common.h"
#include "../../include/tatrg_testing.h"

using namespace tatrg;

static int launched() { return hipGetLastError() == hipSuccess ? 0 : -3; }

extern "C" {

int tatrg_test_gemm(const double* A, const double* B, double* C, int64_t M, int64_t N,
                    int64_t K, int64_t lda, int64_t ldb, int64_t ldc, int ta, int tb,
                    double alpha, double beta, int64_t batch, int64_t sA, int64_t sB,
                    int64_t sC, int parts, double* partial, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 0 || batch < 1) return -1;
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA; g.ta = ta != 0;
  g.B = B; g.ldb = ldb; g.sB = sB; g.tb = tb != 0;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta; g.batch = batch;
  g.sym = A == B && lda == ldb && g.ta != g.tb && M == N && sA == sB;
  if (parts < 0) {
    if (!partial) return -1;
    if (!gram_tn(g, partial, (size_t)(-(int64_t)parts) * 1024, (hipStream_t)stream)) return -1;
  } else if (parts > 1) {
    if (!partial) return -1;
    gemm_f64_splitk(g, parts, partial, (hipStream_t)stream);
  } else {
    gemm_f64(g, (hipStream_t)stream);
  }
  return launched();
}

static GemmArgs mk(const double* A, const double* B, double* C, int64_t M, int64_t N,
                   int64_t K, int64_t lda, int64_t ldb, int64_t ldc, int ta, int tb,
                   double alpha, double beta, int64_t batch, int64_t sA, int64_t sB,
                   int64_t sC) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA; g.ta = ta != 0;
  g.B = B; g.ldb = ldb; g.sB = sB; g.tb = tb != 0;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta; g.batch = batch;
  return g;
}

size_t tatrg_test_gemm_bf16x3_ws(int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb,
                                 int ta, int tb, int64_t batch, int64_t sA, int64_t sB) {
  return gemm_bf16x3_ws_doubles(
      mk(nullptr, nullptr, nullptr, M, N, K, lda, ldb, 0, ta, tb, 1, 0, batch, sA, sB, 0));
}

int tatrg_test_gemm_bf16x3(const double* A, const double* B, double* C, int64_t M, int64_t N,
                           int64_t K, int64_t lda, int64_t ldb, int64_t ldc, int ta, int tb,
                           double alpha, double beta, int64_t batch, int64_t sA, int64_t sB,
                           int64_t sC, double* ws, void* stream) {
  if (!A || !B || !C || !ws || M < 0 || N < 0 || K < 0 || batch < 1) return -1;
  GemmArgs g = mk(A, B, C, M, N, K, lda, ldb, ldc, ta, tb, alpha, beta, batch, sA, sB, sC);
  if (!gemm_bf16x3(g, ws, gemm_bf16x3_ws_doubles(g), (hipStream_t)stream)) return -1;
  return launched();
}

static bool chain_shapes_ok(int64_t R1, int64_t R2, int64_t C1, int64_t C2, int64_t K1,
                            int64_t M2) {
  return R1 > 0 && R2 > 0 && C1 > 0 && C2 > 0 && K1 > 0 && M2 > 0;
}

static void chain_gemms(const double* A1, const double* B1, const double* A2, double* C,
                        int64_t R1, int64_t R2, int64_t C1, int64_t C2, int64_t K1, int64_t M2,
                        GemmArgs* g1, GemmArgs* g2) {
  *g1 = mk(A1, B1, nullptr, R1 * R2, C1 * C2, K1, K1, C1 * C2, 0, 0, 0, 1.0, 0.0, 1, 0, 0, 0);
  *g2 = mk(A2, nullptr, C, M2, C1, R2 * C2, M2, 0, C1, 1, 0, 1.0, 0.0, R1, 0, 0, M2 * C1);
}

size_t tatrg_test_gemm_bf16x3_chain_ws(int64_t R1, int64_t R2, int64_t C1, int64_t C2,
                                       int64_t K1, int64_t M2) {
  if (!chain_shapes_ok(R1, R2, C1, C2, K1, M2)) return 0;
  GemmArgs g1, g2;
  chain_gemms(nullptr, nullptr, nullptr, nullptr, R1, R2, C1, C2, K1, M2, &g1, &g2);
  const int64_t pn = R1 * C1 * bf16x3_kpad(R2 * C2);
  return (size_t)((3 * pn * 2 + 255) / 256 * 32) +
         std::max(gemm_bf16x3_ws_doubles(g1), gemm_bf16x3_ws_doubles(g2, true));
}

int tatrg_test_gemm_bf16x3_chain(const double* A1, const double* B1, const double* A2,
                                 double* C, int64_t R1, int64_t R2, int64_t C1, int64_t C2,
                                 int64_t K1, int64_t M2, double* ws, size_t ws_doubles,
                                 void* stream) {
  if (!A1 || !B1 || !A2 || !C || !ws || !chain_shapes_ok(R1, R2, C1, C2, K1, M2)) return -1;
  if (ws_doubles < tatrg_test_gemm_bf16x3_chain_ws(R1, R2, C1, C2, K1, M2)) return -1;
  GemmArgs g1, g2;
  chain_gemms(A1, B1, A2, C, R1, R2, C1, C2, K1, M2, &g1, &g2);
  const int64_t Kp = bf16x3_kpad(R2 * C2), pn = R1 * C1 * Kp;
  uint16_t* pp = reinterpret_cast<uint16_t*>(ws);
  const size_t used = (size_t)((3 * pn * 2 + 255) / 256 * 32);
  double* rest = ws + used;
  const size_t rest_n = ws_doubles - used;
  const Bf16PlanesOut po = {{pp, pp + pn, pp + 2 * pn}, R2, C1, C2, Kp, 0, pn};
  const Bf16PlanesIn pi = {{pp, pp + pn, pp + 2 * pn}, C1 * Kp};
  if (!gemm_bf16x3(g1, rest, rest_n, (hipStream_t)stream, nullptr, nullptr, &po)) return -1;
  if (!gemm_bf16x3(g2, rest, rest_n, (hipStream_t)stream, nullptr, &pi, nullptr)) return -1;
  return launched();
}

int tatrg_test_split_products(int n) { return set_split_products(n); }

size_t tatrg_test_tsqr_ws(int64_t m, int n) {
  if (n < 1 || n > 96 || m < n) return 0;
  return tsqr_ws_doubles(m, n);
}

int tatrg_test_tsqr(double* Y, int64_t m, int n, int64_t ld, double* R, double* ws,
                    void* stream) {
  if (!Y || !ws || n < 1 || n > 96 || m < n || ld < n) return -1;
  tsqr(Y, m, n, ld, R, ws, (hipStream_t)stream);
  return launched();
}

int tatrg_test_svd(const double* A, double* U, double* S, double* V, int n, int batch,
                   void* stream) {
  if (!A || !U || !S || !V || n < 1 || n > 96 || batch < 1) return -1;
  jacobi_svd(A, U, S, V, n, batch, (hipStream_t)stream);
  return launched();
}

int tatrg_test_cholesky(double* A, int n, int batch, double shift_rel, int* flag,
                        void* stream) {
  if (!A || !flag || n < 1 || batch < 1) return -1;
  cholesky_shifted(A, n, batch, shift_rel, flag, (hipStream_t)stream);
  return launched();
}

int tatrg_test_cholesky_blocked_inv(double* A, double* Dinv, double* Linv, double* T, int n,
                                    int batch, int* flag, void* stream) {
  if (!A || !Dinv || !Linv || !T || !flag || n < 1 || batch < 1) return -1;
  cholesky_blocked_inv(A, Dinv, n, batch, flag, (hipStream_t)stream);
  tri_inv_lower(A, Dinv, Linv, T, n, batch, (hipStream_t)stream);
  return launched();
}

int tatrg_test_chol_inv(const double* G, double* R, double* Rinv, int n, int pass,
                        double shift_coef, int* fail, void* stream) {
  if (!G || !R || !Rinv || !fail || n < 1 || n > 96 || pass < 0 || pass > 2) return -1;
  chol_inv(G, R, Rinv, n, pass, fail, (hipStream_t)stream, shift_coef);
  return launched();
}

int tatrg_test_chol_inv_batched(const double* G, double* R, double* Rinv, int n, int pass,
                                double shift_coef, int* fail, int batch, void* stream) {
  if (!G || !R || !Rinv || !fail || n < 1 || n > 96 || pass < 0 || pass > 2 || batch < 1)
    return -1;
  const int64_t s = (int64_t)n * n;
  chol_inv(G, R, Rinv, n, pass, fail, (hipStream_t)stream, shift_coef, nullptr, batch, s, s, s,
           1);
  return launched();
}

int tatrg_test_philox(double* out, int64_t rows, int64_t cols, uint64_t seed, uint32_t step,
                      uint32_t site, void* stream) {
  if (!out || rows < 1 || cols < 1) return -1;
  philox_gaussian(out, rows, cols, cols, false, seed, step, site, (hipStream_t)stream);
  return launched();
}

int tatrg_test_philox_words(uint32_t* out, int64_t pair0, int64_t npairs, uint64_t seed,
                            uint32_t step, uint32_t site, void* stream) {
  if (!out || pair0 < 0 || npairs < 1 || ((uintptr_t)out & 15) != 0) return -1;
  philox_words(out, pair0, npairs, seed, step, site, (hipStream_t)stream);
  return launched();
}

int tatrg_test_permute(const double* in, double* out, int rank, const int64_t* dims,
                       const int* perm, void* stream) {
  if (!in || !out || rank < 1 || rank > 6 || !dims || !perm) return -1;
  permute(in, out, rank, dims, perm, (hipStream_t)stream);
  return launched();
}

int tatrg_test_gauge(const double* s, const double* P, double* O, int n, int n_probes,
                     double tau_null, double tau_deg, void* stream) {
  if (!s || !P || !O || n < 1 || n_probes < 1 || n_probes > 8) return -1;
  gauge_rotation(s, P, O, n, n_probes, tau_null, tau_deg, (hipStream_t)stream);
  return launched();
}

}  // extern "C"
