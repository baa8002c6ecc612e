// Dense FP64 factorisations used by the randomized SVDs of the Triad-ATRG step:
//  * TSQR: Householder QR of tall panels (the QR iterations of the RSVD, Table 1 of the
//    paper; the canonical form of Section 2) on row blocks held in LDS, with a reduction tree
//    of the R factors and an explicit Q built by applying the reflectors back down the tree;
//  * one-sided (Hestenes) Jacobi SVD of the small core matrices;
//  * blocked left-looking Cholesky of the squeezer Grams;
//  * gauge rotation fixing the basis of degenerate singular subspaces.
#include "common.h"

#include <vector>

namespace tatrg {

namespace {

constexpr int LDS_DOUBLES = 20224;  // 158 KiB of the 160 KiB a workgroup may allocate

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------------------ TSQR
int leaf_rows(int n) {
  int b = (LDS_DOUBLES - 64) / (n + 2);
  if (b > 1024) b = 1024;
  return b;
}

// Householder QR of row block blockIdx.x (b rows; rows beyond `rows` are zero) of src.
// Output: the block with R on/above the diagonal and the reflector tails below it, written
// to v (may alias src), tau[blk*n + j], and R (n x n, zero below the diagonal) to
// rstack[(blk*n + i)*n + k].
__global__ __launch_bounds__(256) void hh_factor_kernel(const double* src, int64_t rows,
                                                        int64_t lds, int b, int n, double* v,
                                                        int64_t ldv, double* tau,
                                                        double* rstack, const int* run_if) {
  if (run_if && *run_if == 0) return;
  extern __shared__ double sm[];
  const int ld = n + 1;
  double* A = sm;
  double* red = sm + (size_t)b * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int64_t r0 = blk * b;
  const int nb = (int)((rows - r0) < b ? (rows - r0) : b);

  for (int idx = tid; idx < b * n; idx += 256) {
    const int i = idx / n, k = idx - (idx / n) * n;
    A[i * ld + k] = (i < nb) ? src[(r0 + i) * lds + k] : 0.0;
  }
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    double part = 0.0;
    for (int i = j + 1 + tid; i < b; i += 256) part += A[i * ld + j] * A[i * ld + j];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    const double s = red[0] + red[1] + red[2] + red[3];
    const double alpha = A[j * ld + j];
    double t = 0.0, beta = alpha;
    if (s > 0.0) {
      const double nrm = sqrt(alpha * alpha + s);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      t = (beta - alpha) / beta;
      const double scl = 1.0 / (alpha - beta);
      for (int i = j + 1 + tid; i < b; i += 256) A[i * ld + j] *= scl;
    }
    __syncthreads();
    if (tid == 0) {
      A[j * ld + j] = beta;
      tau[blk * n + j] = t;
    }
    if (t != 0.0) {
      for (int k = j + 1 + wave; k < n; k += 4) {
        double w = (lane == 0) ? A[j * ld + k] : 0.0;
        for (int i = j + 1 + lane; i < b; i += 64) w += A[i * ld + j] * A[i * ld + k];
        w = wave_sum(w);
        if (lane == 0) A[j * ld + k] -= t * w;
        for (int i = j + 1 + lane; i < b; i += 64) A[i * ld + k] -= t * A[i * ld + j] * w;
      }
    }
    __syncthreads();
  }

  for (int idx = tid; idx < nb * n; idx += 256) {
    const int i = idx / n, k = idx - (idx / n) * n;
    v[(r0 + i) * ldv + k] = A[i * ld + k];
  }
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx / n, k = idx - (idx / n) * n;
    rstack[(blk * n + i) * n + k] = (k >= i) ? A[i * ld + k] : 0.0;
  }
}

// Q of row block blockIdx.x: H_0 ... H_{n-1} [C; 0] with C = cin rows blk*n .. blk*n+n-1
// (identity when cin is null).  Reflector j is column j of v below the diagonal with an
// implicit unit diagonal.  Rows < `rows` of the result are written to q (may alias v).
__global__ __launch_bounds__(256) void hh_apply_kernel(const double* v, int64_t rows,
                                                       int64_t ldv, int b, int n,
                                                       const double* tau, const double* cin,
                                                       double* q, int64_t ldq,
                                                       const int* run_if) {
  if (run_if && *run_if == 0) return;
  extern __shared__ double sm[];
  const int ld = n + 1;
  double* X = sm;
  double* vc = sm + (size_t)b * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blockIdx.x;
  const int64_t r0 = blk * b;
  const int nb = (int)((rows - r0) < b ? (rows - r0) : b);

  for (int idx = tid; idx < b * n; idx += 256) {
    const int i = idx / n, k = idx - (idx / n) * n;
    double x = 0.0;
    if (i < n) x = cin ? cin[(blk * n + i) * n + k] : (i == k ? 1.0 : 0.0);
    X[i * ld + k] = x;
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double t = tau[blk * n + j];
    if (t == 0.0) continue;
    for (int i = j + tid; i < b; i += 256)
      vc[i] = (i == j) ? 1.0 : ((i < nb) ? v[(r0 + i) * ldv + j] : 0.0);
    __syncthreads();
    for (int k = wave; k < n; k += 4) {
      double w = 0.0;
      for (int i = j + lane; i < b; i += 64) w += vc[i] * X[i * ld + k];
      w = wave_sum(w);
      for (int i = j + lane; i < b; i += 64) X[i * ld + k] -= t * vc[i] * w;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * n; idx += 256) {
    const int i = idx / n, k = idx - (idx / n) * n;
    q[(r0 + i) * ldq + k] = X[i * ld + k];
  }
}

struct TsqrLevel {
  const double* src;
  double* v;
  int64_t rows, ld;
  int b;
  int64_t nblocks;
  double* tau;
  double* rstack;
};

std::vector<TsqrLevel> plan_tsqr(double* Y, int64_t m, int n, int64_t ld, double* ws) {
  std::vector<TsqrLevel> lv;
  const int b0 = leaf_rows(n);
  const int bu = (b0 / n) * n;  // upper levels: whole R blocks
  double* src = Y;
  int64_t rows = m, lds = ld;
  int b = b0;
  for (;;) {
    TsqrLevel L;
    L.src = src;
    L.v = src;
    L.rows = rows;
    L.ld = lds;
    L.b = b;
    L.nblocks = (rows + b - 1) / b;
    L.tau = ws;
    ws += L.nblocks * n;
    L.rstack = ws;
    ws += L.nblocks * n * n;
    lv.push_back(L);
    if (L.nblocks == 1) break;
    src = L.rstack;
    rows = L.nblocks * n;
    lds = n;
    b = bu;
  }
  return lv;
}

void set_lds_attr(const void* fn) {
  static bool done_f = false, done_a = false;
  (void)done_f;
  (void)done_a;
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                      LDS_DOUBLES * (int)sizeof(double));
}

// ------------------------------------------------------------------------------ Jacobi SVD
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(const double* Ain, double* Uo,
                                                          double* So, double* Vo, int n) {
  extern __shared__ double sm[];
  const int ne = n + (n & 1);
  double* W = sm;                         // W[p*n + i] = column p of A (row i)
  double* V = sm + (size_t)ne * n;        // V[p*ne + i]
  __shared__ int rotated;
  __shared__ int order[128];
  __shared__ double norms[128];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const double* A = Ain + (int64_t)blockIdx.x * n * n;

  for (int idx = tid; idx < ne * n; idx += blockDim.x) {
    const int p = idx / n, i = idx - (idx / n) * n;
    W[idx] = (p < n) ? A[i * n + p] : 0.0;
  }
  for (int idx = tid; idx < ne * ne; idx += blockDim.x) {
    const int p = idx / ne, i = idx - (idx / ne) * ne;
    V[idx] = (p == i) ? 1.0 : 0.0;
  }
  __syncthreads();

  const double tol = 1e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < ne - 1; ++r) {
      for (int k = wave; k < ne / 2; k += nw) {
        const int p = (r + k) % (ne - 1);
        const int q = (k == 0) ? (ne - 1) : (r - k + (ne - 1)) % (ne - 1);
        double* wp = W + (size_t)p * n;
        double* wq = W + (size_t)q * n;
        double a = 0.0, bb = 0.0, g = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double x = wp[i], y = wq[i];
          a += x * x;
          bb += y * y;
          g += x * y;
        }
        a = wave_sum(a);
        bb = wave_sum(bb);
        g = wave_sum(g);
        if (a > 0.0 && bb > 0.0 && fabs(g) > tol * sqrt(a * bb)) {
          const double zeta = (bb - a) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int i = lane; i < n; i += 64) {
            const double x = wp[i], y = wq[i];
            wp[i] = c * x - s * y;
            wq[i] = s * x + c * y;
          }
          double* vp = V + (size_t)p * ne;
          double* vq = V + (size_t)q * ne;
          for (int i = lane; i < ne; i += 64) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }

  for (int p = wave; p < ne; p += nw) {
    double a = 0.0;
    for (int i = lane; i < n; i += 64) a += W[(size_t)p * n + i] * W[(size_t)p * n + i];
    a = wave_sum(a);
    if (lane == 0) norms[p] = (p < n) ? sqrt(a) : -1.0;
  }
  __syncthreads();
  if (tid == 0) {
    for (int p = 0; p < ne; ++p) order[p] = p;
    for (int x = 0; x < ne; ++x) {  // selection sort, stable for ties
      int best = x;
      for (int y = x + 1; y < ne; ++y)
        if (norms[order[y]] > norms[order[best]]) best = y;
      const int tmp = order[best];  // move the largest remaining to position x
      for (int y = best; y > x; --y) order[y] = order[y - 1];
      order[x] = tmp;
    }
  }
  __syncthreads();
  double* U = Uo + (int64_t)blockIdx.x * n * n;
  double* Vout = Vo + (int64_t)blockIdx.x * n * n;
  double* S = So + (int64_t)blockIdx.x * n;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, c = idx - (idx / n) * n;
    const int p = order[c];
    const double sv = norms[p];
    U[i * n + c] = (sv > 0.0) ? W[(size_t)p * n + i] / sv : 0.0;
    Vout[i * n + c] = V[(size_t)p * ne + i];
  }
  for (int c = tid; c < n; c += blockDim.x) S[c] = norms[order[c]];
}

// ------------------------------------------------------------------------------ Cholesky
__global__ void add_shift_kernel(double* A, int n, double shift_rel) {
  double* M = A + (int64_t)blockIdx.x * n * n;
  __shared__ double red[16];
  double part = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) part += M[(int64_t)i * n + i];
  part = wave_sum(part);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  double tr = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tr += red[w];
  const double d = shift_rel * tr;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) M[(int64_t)i * n + i] += d;
}

// Factor the diagonal block at (j, j) (jb <= 64, redundantly in every workgroup) and solve
// the panel rows below it: L[i, j:j+jb] = A[i, j:j+jb] L_jj^{-T}.
__global__ __launch_bounds__(256) void chol_panel_kernel(double* Aall, int n, int j, int jb,
                                                         int* flag) {
  __shared__ double D[64][65];
  double* A = Aall + (int64_t)blockIdx.y * n * n;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < jb * jb; idx += 256) {
    const int r = idx / jb, c = idx - (idx / jb) * jb;
    D[r][c] = A[(int64_t)(j + r) * n + j + c];
  }
  __syncthreads();
  __shared__ double dk;
  for (int k = 0; k < jb; ++k) {
    if (tid == 0) {
      const double piv = D[k][k];
      if (!(piv > 0.0)) flag[0] = 1;
      dk = (piv > 0.0) ? sqrt(piv) : __builtin_nan("");
      D[k][k] = dk;
    }
    __syncthreads();
    for (int r = k + 1 + tid; r < jb; r += 256) D[r][k] /= dk;
    __syncthreads();
    for (int idx = tid; idx < jb * jb; idx += 256) {
      const int r = idx / jb, c = idx - (idx / jb) * jb;
      if (r > k && c > k && c <= r) D[r][c] -= D[r][k] * D[c][k];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < jb * jb; idx += 256) {
      const int r = idx / jb, c = idx - (idx / jb) * jb;
      A[(int64_t)(j + r) * n + j + c] = (c <= r) ? D[r][c] : 0.0;
    }
  }
  const int rows_below = n - j - jb;
  const int per = (rows_below + gridDim.x - 1) / gridDim.x;
  const int rb = blockIdx.x * per;
  for (int rr = rb + tid; rr < rb + per && rr < rows_below; rr += 256) {
    double* row = A + (int64_t)(j + jb + rr) * n + j;
    for (int c = 0; c < jb; ++c) {  // forward substitution in place: row <- row L_jj^{-T}
      double s = row[c];
      for (int l = 0; l < c; ++l) s -= row[l] * D[c][l];
      row[c] = s / D[c][c];
    }
  }
}

__global__ void zero_upper_kernel(double* A, int n, int batch) {
  const int64_t per = (int64_t)n * n, total = per * batch;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % per;
    if (r % n > r / n) A[idx] = 0.0;
  }
}

// ------------------------------------------------------------------------------ gauge
__global__ void gauge_kernel(const double* s, const double* P, double* O, int n, int np,
                             double tau_null, double tau_deg) {
  const int inst = blockIdx.x;
  s += (int64_t)inst * n;
  P += (int64_t)inst * np * n;
  O += (int64_t)inst * n * n;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x)
    O[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double smax = n > 0 ? s[0] : 0.0;
  if (!(smax > 0.0)) return;
  int j = 0;
  while (j < n) {
    if (s[j] <= tau_null * smax) break;
    int j1 = j + 1;
    while (j1 < n && s[j1] > tau_null * smax && s[j1 - 1] - s[j1] <= tau_deg * smax) ++j1;
    const int m = j1 - j;
    if (m <= np) {
      // columns of X = P_c^T: X[a][c] = P[c][j + a]; modified Gram-Schmidt (twice) gives the
      // QR with a positive diagonal.
      double X[8][8], Q[8][8];
      for (int a = 0; a < m; ++a)
        for (int c = 0; c < m; ++c) X[a][c] = P[(int64_t)c * n + j + a];
      for (int c = 0; c < m; ++c) {
        double vcol[8];
        for (int a = 0; a < m; ++a) vcol[a] = X[a][c];
        for (int pass = 0; pass < 2; ++pass)
          for (int d = 0; d < c; ++d) {
            double r = 0.0;
            for (int a = 0; a < m; ++a) r += Q[a][d] * vcol[a];
            for (int a = 0; a < m; ++a) vcol[a] -= r * Q[a][d];
          }
        double nr = 0.0;
        for (int a = 0; a < m; ++a) nr += vcol[a] * vcol[a];
        nr = sqrt(nr);
        for (int a = 0; a < m; ++a) Q[a][c] = (nr > 0.0) ? vcol[a] / nr : (a == c ? 1.0 : 0.0);
      }
      for (int a = 0; a < m; ++a)
        for (int c = 0; c < m; ++c) O[(int64_t)(j + a) * n + j + c] = Q[a][c];
    }
    j = j1;
  }
}

}  // namespace

size_t tsqr_ws_doubles(int64_t m, int n) {
  size_t total = 0;
  const int b0 = leaf_rows(n);
  const int bu = (b0 / n) * n;
  int64_t rows = m;
  int b = b0;
  for (;;) {
    const int64_t nb = (rows + b - 1) / b;
    total += (size_t)nb * n + (size_t)nb * n * n;
    if (nb == 1) break;
    rows = nb * n;
    b = bu;
  }
  return total;
}

__global__ void copy_if_kernel(double* y, const double* x, int64_t n, const int* run_if) {
  if (run_if && *run_if == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// G = R^T R (upper R) and R^{-1}, n <= 96, one workgroup; see chol_inv in common.h.
__global__ __launch_bounds__(256) void chol_inv_kernel(const double* G, double* R, double* Ri,
                                                        int n, int pass, int* fail,
                                                        double shift_coef) {
  __shared__ double A[96][97];
  __shared__ double Iv[96][97];
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (*fail) return;  // uniform: read before any write of this launch
  for (int idx = tid; idx < n * n; idx += 256) A[idx / n][idx % n] = G[idx];
  if (tid == 0) bad = 0;
  __syncthreads();
  double dmax = 0.0, tr = 0.0;
  for (int k = 0; k < n; ++k) {
    dmax = fmax(dmax, A[k][k]);
    tr += A[k][k];
  }
  __syncthreads();
  if (pass == 0 && tid < n) A[tid][tid] += shift_coef * tr;  // ||Y||_2^2 <= tr(G)
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = A[k][k];
      bool ok = isfinite(d) && (pass == 0 ? d > 0.0
                                          : pass == 1 ? d > 1e-14 * dmax : (d > 0.25 && d < 4.0));
      if (!ok) bad = 1;
      piv = ok ? sqrt(d) : 1.0;
      A[k][k] = piv;
    }
    __syncthreads();
    for (int j = k + 1 + tid; j < n; j += 256) A[k][j] /= piv;  // row k of R
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx / n, j = idx % n;
      if (i > k && j >= i) A[i][j] -= A[k][i] * A[k][j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) *fail = 1;
    return;
  }
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx / n, j = idx % n;
    R[idx] = (j >= i) ? A[i][j] : 0.0;
  }
  // R^{-1}: column j solves R x = e_j by back substitution (one thread per column, in LDS)
  for (int j = tid; j < n; j += 256) {
    for (int i = n - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int l = i + 1; l <= j; ++l) v -= A[i][l] * Iv[l][j];
      Iv[i][j] = (i <= j) ? v / A[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += 256) Ri[idx] = Iv[idx / n][idx % n];
}

void tsqr(double* Y, int64_t m, int n, int64_t ld, double* R_out, double* ws, hipStream_t st,
          const int* run_if_set) {
  static bool attr = false;
  if (!attr) {
    set_lds_attr((const void*)hh_factor_kernel);
    set_lds_attr((const void*)hh_apply_kernel);
    attr = true;
  }
  std::vector<TsqrLevel> lv = plan_tsqr(Y, m, n, ld, ws);
  for (const TsqrLevel& L : lv) {
    const size_t lds = ((size_t)L.b * (n + 1) + 64) * sizeof(double);
    hipLaunchKernelGGL(hh_factor_kernel, dim3((unsigned)L.nblocks), dim3(256), lds, st, L.src,
                       L.rows, L.ld, L.b, n, L.v, L.ld, L.tau, L.rstack, run_if_set);
  }
  if (R_out)
    hipLaunchKernelGGL(copy_if_kernel, dim3(64), dim3(256), 0, st, R_out, lv.back().rstack,
                       (int64_t)n * n, run_if_set);
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    const TsqrLevel& L = lv[l];
    const double* cin = (l == (int)lv.size() - 1) ? nullptr : lv[l].rstack;
    const size_t lds = ((size_t)L.b * (n + 1) + (size_t)L.b + 64) * sizeof(double);
    hipLaunchKernelGGL(hh_apply_kernel, dim3((unsigned)L.nblocks), dim3(256), lds, st, L.v,
                       L.rows, L.ld, L.b, n, L.tau, cin, L.v, L.ld, run_if_set);
  }
}

void chol_inv(const double* G, double* R, double* Rinv, int n, int pass, int* fail,
              hipStream_t st, double shift_coef) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(256), 0, st, G, R, Rinv, n, pass, fail,
                     shift_coef);
}

void jacobi_svd(const double* A, double* U, double* S, double* V, int n, int batch,
                hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    set_lds_attr((const void*)jacobi_svd_kernel);
    attr = true;
  }
  const int ne = n + (n & 1);
  const size_t lds = ((size_t)ne * n + (size_t)ne * ne) * sizeof(double);
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(batch), dim3(1024), lds, st, A, U, S, V, n);
}

void cholesky_shifted(double* A, int n, int batch, double shift_rel, int* flag,
                      hipStream_t st) {
  hipLaunchKernelGGL(add_shift_kernel, dim3(batch), dim3(1024), 0, st, A, n, shift_rel);
  const int nbk = 64;
  for (int j = 0; j < n; j += nbk) {
    const int jb = (n - j) < nbk ? (n - j) : nbk;
    if (j > 0) {
      GemmArgs g;
      g.M = n - j;
      g.N = jb;
      g.K = j;
      g.A = A + (int64_t)j * n;
      g.lda = n;
      g.sA = (int64_t)n * n;
      g.ta = false;
      g.B = A + (int64_t)j * n;
      g.ldb = n;
      g.sB = (int64_t)n * n;
      g.tb = true;
      g.C = A + (int64_t)j * n + j;
      g.ldc = n;
      g.sC = (int64_t)n * n;
      g.alpha = -1.0;
      g.beta = 1.0;
      g.batch = batch;
      gemm_f64(g, st);
    }
    const int rows_below = n - j - jb;
    int chunks = (rows_below + 255) / 256;
    if (chunks < 1) chunks = 1;
    hipLaunchKernelGGL(chol_panel_kernel, dim3(chunks, batch), dim3(256), 0, st, A, n, j, jb,
                       flag);
  }
  const int64_t total = (int64_t)n * n * batch;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, n, batch);
}

void gauge_rotation(const double* s, const double* P, double* O, int n, int n_probes,
                    double tau_null, double tau_deg, hipStream_t st) {
  hipLaunchKernelGGL(gauge_kernel, dim3(1), dim3(256), 0, st, s, P, O, n, n_probes, tau_null,
                     tau_deg);
}

}  // namespace tatrg
