// Dense FP64 factorisations used by the randomized SVDs of the Triad-ATRG step:
//  * TSQR: Householder QR of tall panels (the QR iterations of the RSVD, Table 1 of the
//    paper; the canonical form of Section 2) on row blocks held in registers, with a
//    reduction tree of the R factors and an explicit Q built by applying the reflectors back
//    down the tree;
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

// v from another lane of the same 16-lane row by a DPP move (CTRL: a quad permutation or a
// row mirror), both 32-bit halves.
template <int CTRL>
__device__ inline double dpp_double(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row, the same value in every lane: pairs (quad permutation
// [1,0,3,2]), quads ([2,3,0,1]), then the two quads of each half row (half-row mirror) and the
// two halves (row mirror) -- the grouping of a butterfly over lane masks 1, 2, 4, 8.
__device__ inline double row16_sum(double v) {
  v += dpp_double<0xB1>(v);
  v += dpp_double<0x4E>(v);
  v += dpp_double<0x141>(v);
  v += dpp_double<0x140>(v);
  return v;
}

// ------------------------------------------------------------------------------ TSQR
// Householder QR of row blocks with the panel held in registers: thread t owns column
// c = t % CW and the rows i = g + RG k (g = t / CW < RG, k < RPG) of its block, so the rank-1
// updates never touch LDS.  Leaf blocks take TsqrShape::leaf rows of the panel; blocks of the
// reduction tree stack whole R factors, up to TsqrShape::up rows (>= 2 R factors).  Block
// heights are chosen so the rows a thread holds fit in registers without spilling.
constexpr int TQ_HV = 8;  // reflector columns staged per chunk in the apply kernel

struct TsqrShape {
  int cw, leaf, up;
};
TsqrShape tsqr_shape(int n) {
  if (n <= 32) return {32, 192, 384};
  if (n <= 64) return {64, 192, 256};
  return {96, 160, 192};
}

// Factor row block blockIdx.x (b rows; rows beyond `rows` are zero) of src.  Output: the block
// with R on/above the diagonal and the reflector tails below it, written to v (may alias src),
// tau[blk*n + j], and R (n x n, zero below the diagonal) to rstack[(blk*n + i)*n + k].  The
// reflector of column j is (1, x_{j+1..} * scl) with tau = (beta - alpha) / beta.
//
// One barrier per column.  At step j every thread holds x = column j (after reflectors
// 0..j-1) in its own rows, zero on and above row j, and computes for its own column c >= j
// the partial dot product sum_{i>j} x_i A[i][c] over its rows (for c = j the squared norm
// below the diagonal); the thread holding row j publishes A[j][c], and the owner of column
// j+1 publishes that column (zero on and above row j+1) as it stands before reflector j.
// After the barrier every thread forms reflector j from the reduced sums, updates its column
// and rebuilds column j+1 in its own rows from the published copy.  The inner loops are plain
// FMAs over all rows a thread holds (rows on and above the diagonal carry zeros in x).  Row j
// is row slot kk = j / RG of group j % RG; the column loop runs as an unrolled loop over kk
// around a loop over the group, so that slot is a compile-time register index.  Scaling of
// the stored reflector and the diagonal beta are applied when the block is written out.
//
// TRI: the block is two stacked upper-triangular n x n factors (a tree level with
// n = RG * RPG / 2).  Then column j of the Householder vector is nonzero only in rows
// n .. n + j, i.e. in register slots RPG/2 .. RPG/2 + j/RG, and the dot, update and rebuild
// loops run over those slots only (the skipped products are with exact zeros).
template <int CW, int RG, int RPG, bool TRI>
__global__ __launch_bounds__(CW * RG) void hh_factor_kernel(const double* src, int64_t rows,
                                                          int64_t lds, int b, int n, double* v,
                                                          int64_t ldv, double* tau,
                                                          double* rstack, const int* run_if) {
  if (run_if && *run_if == 0) return;
  static_assert(RG % 2 == 0 && RPG % 2 == 0, "pairs of doubles are read as one 16-byte word");
  __shared__ double2 xp[2][RG][RPG / 2];  // a column by row group: [g][k] = row g + RG k
  __shared__ double2 pw[2][CW][RG / 2];   // per-column partial dot products of the RG groups
  __shared__ double rj[2][CW];            // row j of the block
  __shared__ double sclv[CW], betav[CW];
  // a wave holds 64 / RG whole columns (all RG row groups); once they are finished the wave
  // only takes part in the barriers
  constexpr int CPW = 64 / RG;
  static_assert(64 % RG == 0 && (CW * RG) % 64 == 0, "waves hold whole columns");
  const int tid = threadIdx.x, lane = tid & 63;
  const int c_lo = __builtin_amdgcn_readfirstlane(tid >> 6) * CPW;  // first column of the wave
  const int g = lane % RG, c = c_lo + lane / RG;
  const int64_t blk = blockIdx.x, r0 = blk * (int64_t)b;
  const int nb = (int)((rows - r0) < b ? (rows - r0) : b);
  double* pws = reinterpret_cast<double*>(pw);

  double a[RPG], x[RPG];
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const int i = g + RG * k;
    a[k] = (i < nb && c < n) ? src[(r0 + i) * lds + c] : 0.0;
  }
  if (c == 0) {
#pragma unroll
    for (int k = 0; k < RPG; k += 2) {
      const int i = g + RG * k;
      xp[0][g][k / 2] = make_double2(i > 0 ? a[k] : 0.0, a[k + 1]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPG; k += 2) {
    const double2 e = xp[0][g][k / 2];
    x[k] = e.x;
    x[k + 1] = e.y;
  }

#pragma unroll
  for (int kk = 0; kk < RPG; ++kk) {
#pragma unroll 1
    for (int jg = 0; jg < RG; ++jg) {
      const int j = kk * RG + jg;
      if (j >= n) break;
      const int bf = j & 1;
      if (c >= j && c < n) {
        double p = 0.0;
#pragma unroll
        for (int k = 0; k < RPG; ++k)
          if (!TRI || (k >= RPG / 2 && k <= RPG / 2 + kk)) p += x[k] * a[k];
        pws[((bf * CW) + c) * RG + g] = p;
        if (g == jg) rj[bf][c] = a[kk];
      }
      if (c == j + 1) {  // column j+1 before reflector j, zero on and above row j+1
#pragma unroll
        for (int k = 0; k < RPG; k += 2) {
          const int i = g + RG * k;
          xp[bf ^ 1][g][k / 2] =
              make_double2(i > j + 1 ? a[k] : 0.0, i + RG > j + 1 ? a[k + 1] : 0.0);
        }
      }
      __syncthreads();
      if (c_lo + CPW <= j || c_lo >= n) continue;  // wave-uniform: all its columns finished

      auto colsum = [&](int cc) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < RG / 2; ++q) {
          const double2 e = pw[bf][cc][q];
          sum += e.x;
          sum += e.y;
        }
        return sum;
      };
      const double s = colsum(j);
      const double alpha = rj[bf][j];
      double t = 0.0, beta = alpha, scl = 0.0;
      if (s > 0.0) {
        const double nrm = sqrt(alpha * alpha + s);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scl = 1.0 / (alpha - beta);
      }
      if (c == j && g == 0) {
        tau[blk * n + j] = t;
        sclv[j] = scl;
        betav[j] = beta;
      }
      if (c > j && c < n) {
        const double tw = t * (rj[bf][c] + scl * colsum(c)), f = tw * scl;
#pragma unroll
        for (int k = 0; k < RPG; ++k)
          if (!TRI || (k >= RPG / 2 && k <= RPG / 2 + kk)) a[k] -= f * x[k];
        if (g == jg) a[kk] -= tw;
      }
      if (j + 1 < n) {
        const double tw = t * (rj[bf][j + 1] + scl * colsum(j + 1)), f = tw * scl;
#pragma unroll
        for (int k = 0; k < RPG; k += 2) {
          if (TRI && (k + 1 < RPG / 2 || k > RPG / 2 + kk + 1)) continue;  // zero rows of x
          const double2 e = xp[bf ^ 1][g][k / 2];
          x[k] = e.x - f * x[k];
          x[k + 1] = e.y - f * x[k + 1];
        }
        // row j+1 leaves x
        if (jg + 1 < RG) {
          if (g == jg + 1) x[kk] = 0.0;
        } else if (kk + 1 < RPG) {
          if (g == 0) x[kk + 1] = 0.0;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const int i = g + RG * k;
    if (c < n) {
      const double e = (i < c) ? a[k] : (i == c ? betav[c] : a[k] * sclv[c]);
      if (i < nb) v[(r0 + i) * ldv + c] = e;
      if (i < n) rstack[(blk * n + i) * n + c] = (c >= i) ? e : 0.0;
    }
  }
}

// Q of row block blockIdx.x: H_0 ... H_{n-1} [C; 0] with C = cin rows blk*n .. blk*n+n-1
// (identity when cin is null).  The block of Q is held in registers like the factor; the
// reflectors are staged TQ_HV columns at a time in LDS, by row group, so a thread reads the
// rows it holds as 16-byte words.  One barrier per reflector (double-buffered partial sums).
// Rows < `rows` of the result are written to q (may alias v).
template <int CW, int RG, int RPG>
__global__ __launch_bounds__(CW * RG) void hh_apply_kernel(const double* v, int64_t rows,
                                                         int64_t ldv, int b, int n,
                                                         const double* tau, const double* cin,
                                                         double* q, int64_t ldq,
                                                         const int* run_if) {
  if (run_if && *run_if == 0) return;
  constexpr int NT = CW * RG, BR = RG * RPG;
  __shared__ double2 vc[TQ_HV][RG][RPG / 2];  // [jj][g][k] = row g + RG k of column j0 + jj
  __shared__ double2 pw[2][CW][RG / 2];
  __shared__ double ts[TQ_HV];
  const int tid = threadIdx.x, c = tid % CW, g = tid / CW;
  const int64_t blk = blockIdx.x, r0 = blk * (int64_t)b;
  const int nb = (int)((rows - r0) < b ? (rows - r0) : b);
  double* vcs = reinterpret_cast<double*>(vc);
  double* pws = reinterpret_cast<double*>(pw);

  double x[RPG];
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const int i = g + RG * k;
    double e = 0.0;
    if (i < n && c < n) e = cin ? cin[(blk * n + i) * n + c] : (i == c ? 1.0 : 0.0);
    x[k] = e;
  }
  int it = 0;
  for (int j0 = ((n - 1) / TQ_HV) * TQ_HV; j0 >= 0; j0 -= TQ_HV) {
    __syncthreads();  // every thread is done with the previous chunk
    for (int idx = tid; idx < TQ_HV * BR; idx += NT) {
      const int i = idx / TQ_HV, jj = idx - (idx / TQ_HV) * TQ_HV, j = j0 + jj;
      double e = 0.0;
      if (j < n && i < nb) e = (i == j) ? 1.0 : (i > j ? v[(r0 + i) * ldv + j] : 0.0);
      vcs[(jj * RG + (i % RG)) * RPG + i / RG] = e;
    }
    if (tid < TQ_HV) ts[tid] = (j0 + tid < n) ? tau[blk * n + j0 + tid] : 0.0;
    __syncthreads();
    for (int jj = TQ_HV - 1; jj >= 0; --jj) {
      const double t = ts[jj];
      if (t == 0.0) continue;  // uniform
      const int bf = it & 1;
      ++it;
      if (c < n) {
        double p = 0.0;
#pragma unroll
        for (int k = 0; k < RPG; k += 2) {
          const double2 e = vc[jj][g][k / 2];
          p += e.x * x[k];
          p += e.y * x[k + 1];
        }
        pws[((bf * CW) + c) * RG + g] = p;
      }
      __syncthreads();
      if (c < n) {
        double w = 0.0;
#pragma unroll
        for (int qq = 0; qq < RG / 2; ++qq) {
          const double2 e = pw[bf][c][qq];
          w += e.x;
          w += e.y;
        }
        const double f = t * w;
#pragma unroll
        for (int k = 0; k < RPG; k += 2) {
          const double2 e = vc[jj][g][k / 2];
          x[k] -= f * e.x;
          x[k + 1] -= f * e.y;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const int i = g + RG * k;
    if (i < nb && c < n) q[(r0 + i) * ldq + c] = x[k];
  }
}

struct TsqrLevel {
  const double* src;
  double* v;
  int64_t rows, ld;
  int b;
  bool leaf;
  int64_t nblocks;
  double* tau;
  double* rstack;
};

// Levels of the reduction tree: level 0 factors the panel in leaf blocks, every later level
// the stacked R factors of the one below in blocks of whole R factors.
std::vector<TsqrLevel> plan_tsqr(double* Y, int64_t m, int n, int64_t ld, double* ws) {
  std::vector<TsqrLevel> lv;
  const TsqrShape sh = tsqr_shape(n);
  const int bu = (sh.up / n) * n;  // >= 2n for n <= 96
  double* src = Y;
  int64_t rows = m, lds = ld;
  int b = sh.leaf;
  for (;;) {
    TsqrLevel L;
    L.src = src;
    L.v = src;
    L.rows = rows;
    L.ld = lds;
    L.b = b;
    L.leaf = lv.empty();
    L.nblocks = (rows + b - 1) / b;
    L.tau = ws;
    if (ws) ws += L.nblocks * n;
    L.rstack = ws;
    if (ws) ws += L.nblocks * n * n;
    lv.push_back(L);
    if (L.nblocks == 1) break;
    src = L.rstack;  // nblocks * n rows; bu >= 2n, so every level at least halves the rows
    rows = L.nblocks * n;
    lds = n;
    b = bu;
  }
  return lv;
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

  {
    // ne n <= 96 x 96 = 9 x 1024 entries (launched with 1024 threads): all loads in flight
    // before the LDS writes
    double v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int idx = tid + t * 1024, p = idx / n, i = idx - (idx / n) * n;
      v[t] = (idx < ne * n && p < n) ? A[i * n + p] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
      if (tid + t * 1024 < ne * n) W[tid + t * 1024] = v[t];
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
    // each rotation pair is handled by 16 lanes (4 pairs per wave); all pairs of a round of
    // the round-robin ordering are disjoint, so they run concurrently
    const int sub = lane & 15, slot = wave * 4 + (lane >> 4), nslots = nw * 4;
    for (int r = 0; r < ne - 1; ++r) {
      for (int k = slot; k < ne / 2; k += nslots) {
        const int p = (r + k) % (ne - 1);
        const int q = (k == 0) ? (ne - 1) : (r - k + (ne - 1)) % (ne - 1);
        double* wp = W + (size_t)p * n;
        double* wq = W + (size_t)q * n;
        // this lane's entries of the two columns (n <= 96: at most six each), kept in
        // registers for the rotation; the padding zeros leave the sums unchanged
        double xr[6], yr[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          const int i = sub + 16 * t;
          xr[t] = (i < n) ? wp[i] : 0.0;
          yr[t] = (i < n) ? wq[i] : 0.0;
        }
        double a = 0.0, bb = 0.0, g = 0.0;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          a += xr[t] * xr[t];
          bb += yr[t] * yr[t];
          g += xr[t] * yr[t];
        }
        a = row16_sum(a);
        bb = row16_sum(bb);
        g = row16_sum(g);
        if (a > 0.0 && bb > 0.0 && fabs(g) > tol * sqrt(a * bb)) {
          const double zeta = (bb - a) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const int i = sub + 16 * t;
            if (i < n) {
              wp[i] = c * xr[t] - s * yr[t];
              wq[i] = s * xr[t] + c * yr[t];
            }
          }
          double* vp = V + (size_t)p * ne;
          double* vq = V + (size_t)q * ne;
          double xv[6], yv[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const int i = sub + 16 * t;
            xv[t] = (i < ne) ? vp[i] : 0.0;
            yv[t] = (i < ne) ? vq[i] : 0.0;
          }
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const int i = sub + 16 * t;
            if (i < ne) {
              vp[i] = c * xv[t] - s * yv[t];
              vq[i] = s * xv[t] + c * yv[t];
            }
          }
          if (sub == 0) rotated = 1;
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

// Factor the diagonal block at (j, j) (jb <= 64) of every matrix of the batch (one wave each)
// and write L_jj back, zero above its diagonal.  Lane r holds row r of the block in registers;
// for column k the pivot comes from lane k, every lane below it scales its entry and publishes
// it through LDS, and each lane updates its own row (right-looking, the same operations in the
// same order as the textbook column algorithm).
__global__ __launch_bounds__(64) void chol_diag_kernel(double* Aall, int n, int j, int jb,
                                                       int* flag) {
  __shared__ double lk[64];
  double* A = Aall + (int64_t)blockIdx.y * n * n;
  const int r = threadIdx.x;
  double row[64];
#pragma unroll
  for (int c = 0; c < 64; ++c)
    row[c] = (r < jb && c < jb) ? A[(int64_t)(j + r) * n + j + c] : 0.0;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    if (k < jb) {
      const double piv = __shfl(row[k], k, 64);
      if (r == 0 && !(piv > 0.0)) flag[0] = 1;
      const double dk = (piv > 0.0) ? sqrt(piv) : __builtin_nan("");
      if (r == k) row[k] = dk;
      if (r > k) row[k] /= dk;
      lk[r] = row[k];
      __syncthreads();
#pragma unroll
      for (int c = k + 1; c < 64; ++c)
        if (c <= r && r < jb) row[c] -= row[k] * lk[c];
      __syncthreads();
    }
  }
  if (r < jb) {
#pragma unroll
    for (int c = 0; c < 64; ++c)
      if (c < jb) A[(int64_t)(j + r) * n + j + c] = (c <= r) ? row[c] : 0.0;
  }
}

// Panel rows below the diagonal block: L[i, j:j+jb] = A[i, j:j+jb] L_jj^{-T} by forward
// substitution, one row per thread held in registers (64 rows per work-group).
__global__ __launch_bounds__(64) void chol_trsm_kernel(double* Aall, int n, int j, int jb) {
  __shared__ double D[64][65];
  double* A = Aall + (int64_t)blockIdx.y * n * n;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < jb * jb; idx += 64) {
    const int r = idx / jb, c = idx - (idx / jb) * jb;
    D[r][c] = A[(int64_t)(j + r) * n + j + c];
  }
  __syncthreads();
  const int rows_below = n - j - jb;
  const int rr = blockIdx.x * 64 + tid;
  if (rr >= rows_below) return;
  double* row = A + (int64_t)(j + jb + rr) * n + j;
  double x[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) x[c] = (c < jb) ? row[c] : 0.0;
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    if (c < jb) {
      double s = x[c];
#pragma unroll
      for (int l = 0; l < c; ++l) s -= x[l] * D[c][l];
      x[c] = s / D[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < 64; ++c)
    if (c < jb) row[c] = x[c];
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
  for (const TsqrLevel& L : plan_tsqr(nullptr, m, n, n, nullptr))
    total += (size_t)L.nblocks * n + (size_t)L.nblocks * n * n;
  return total;
}


__global__ void copy_if_kernel(double* y, const double* x, int64_t n, const int* run_if) {
  if (run_if && *run_if == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// G = R^T R (upper R) and R^{-1}, n <= 96, one workgroup; see chol_inv in common.h.
// Symmetric elimination on the upper triangle: step k subtracts m_i = A[k][i] / d_k times row
// k from every row i > k (d_k = A[k][k], the k-th pivot of G = L D L^T).  The same row
// operations applied to the identity build E = L^{-1}, so R = D^{1/2} L^T and
// R^{-1} = E^T D^{-1/2} come out of one pass.
//
// Thread (q, g) = (tid % 128, tid / 128) keeps column q of A and of E for rows g + 8 s
// (s < 12) in registers.  At step k the threads holding row k publish it (A[k][.] and
// E[k][.]) to a double-buffered LDS vector; after one barrier every thread updates its rows
// below k.  The step loop runs as an unrolled loop over the register slot of row k around a
// loop over its group, so every register index is static.
__global__ __launch_bounds__(1024) void chol_inv_kernel(const double* Gall, double* Rall,
                                                         double* Riall, int n, int pass,
                                                         int* fall, double shift_coef,
                                                         int* sticky, int64_t sG, int64_t sR,
                                                         int64_t sRi, int sf) {
  constexpr int RGP = 8, SL = 12;  // row groups and slots: 96 rows
  __shared__ double ra[2][128], re[2][128], dv[96];
  __shared__ double red[2][2];
  __shared__ int bad;
  const int tid = threadIdx.x, q = tid & 127, g = tid >> 7;
  const int64_t bi = blockIdx.x;  // batch entry
  const double* G = Gall + bi * sG;
  double* R = Rall + bi * sR;
  double* Ri = Riall + bi * sRi;
  int* fail = fall + bi * sf;
  if (*fail) return;  // uniform: read before any write of this launch
  double a[SL], e[SL];
  // the published row entries of columns q >= n stay zero (so are the multipliers of padding
  // rows and the updates of padding columns)
  if (g == 0 && q >= n) {
    ra[0][q] = ra[1][q] = 0.0;
    re[0][q] = re[1][q] = 0.0;
  }
  // diagonal of G: trace and largest entry, reduced over the first two waves
  {
    const double dk = (tid < n) ? G[tid * n + tid] : 0.0;
    double sm = dk, mx = dk;
    for (int o = 32; o > 0; o >>= 1) {
      sm += __shfl_xor(sm, o, 64);
      mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if ((tid & 63) == 0 && tid < 128) {
      red[0][tid >> 6] = sm;
      red[1][tid >> 6] = mx;
    }
    __syncthreads();
  }
  const double tr = red[0][0] + red[0][1], dmax = fmax(red[1][0], red[1][1]);
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int i = g + RGP * s;
    double x = (i < n && q < n) ? G[i * n + q] : 0.0;
    if (pass == 0 && i == q && i < n) x += shift_coef * tr;  // ||Y||_2^2 <= tr(G)
    a[s] = x;
    e[s] = (i == q && i < n) ? 1.0 : 0.0;
  }
  if (tid == 0) bad = 0;
#pragma unroll
  for (int kk = 0; kk < SL; ++kk) {
#pragma unroll 1
    for (int kg = 0; kg < RGP; ++kg) {
      const int k = kk * RGP + kg, bf = k & 1;
      if (k >= n) break;
      if (g == kg && q < n) {  // this thread holds row k of its column
        ra[bf][q] = a[kk];
        re[bf][q] = e[kk];
      }
      __syncthreads();
      const double d = ra[bf][k];
      const bool ok = isfinite(d) && (pass == 0 ? d > 0.0
                                                : pass == 1 ? d > 1e-14 * dmax
                                                            : (d > 0.25 && d < 4.0));
      if (tid == 0) {
        if (!ok) bad = 1;
        dv[k] = d;
      }
      const double rd = 1.0 / (ok ? d : 1.0);
      // rows i > k below the pivot: a -= m_i A[k][.], e -= m_i E[k][.] without a per-column
      // condition.  A's entries left of the diagonal (q < i) are never read back, E[k][q] is
      // zero for q > k, and the multipliers of padding rows (i >= n) are zero; the
      // multipliers are read from LDS in one batch before the updates.
      const double akq = ra[bf][q], ekq = re[bf][q];
      double mrow[SL];
#pragma unroll
      for (int s = kk; s < SL; ++s) mrow[s] = ra[bf][g + RGP * s];
#pragma unroll
      for (int s = kk; s < SL; ++s) {
        if (s == kk && g <= kg) continue;  // rows i <= k are final (wave-uniform)
        const double mi = mrow[s] * rd;
        a[s] -= mi * akq;
        e[s] -= mi * ekq;
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) {
      *fail = pass + 1;  // which pass failed
      if (sticky) atomicOr(sticky, 1);
    }
    return;
  }
  if (q < n) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int i = g + RGP * s;
      if (i >= n) continue;
      // R[i][q] from row i of A; R^{-1}[q][i] = E[i][q] / sqrt(d_i) (E lower triangular)
      R[i * n + q] = (q > i) ? a[s] / sqrt(dv[i]) : (q == i ? sqrt(dv[i]) : 0.0);
      Ri[q * n + i] = (q <= i) ? e[s] / sqrt(dv[i]) : 0.0;
    }
  }
}

template <int CW, int RG, int RPG>
void tsqr_level_launch(bool apply, const TsqrLevel& L, int n, const double* cin,
                       const int* run_if, hipStream_t st) {
  // two stacked triangular factors that fill the slots exactly: structured factorisation
  const bool tri = !L.leaf && L.b == 2 * n && n == RG * RPG / 2;
  if (!apply && tri)
    hipLaunchKernelGGL((hh_factor_kernel<CW, RG, RPG, true>), dim3((unsigned)L.nblocks),
                       dim3(CW * RG), 0, st, L.src, L.rows, L.ld, L.b, n, L.v, L.ld, L.tau,
                       L.rstack, run_if);
  else if (!apply)
    hipLaunchKernelGGL((hh_factor_kernel<CW, RG, RPG, false>), dim3((unsigned)L.nblocks),
                       dim3(CW * RG), 0, st, L.src, L.rows, L.ld, L.b, n, L.v, L.ld, L.tau,
                       L.rstack, run_if);
  else
    hipLaunchKernelGGL((hh_apply_kernel<CW, RG, RPG>), dim3((unsigned)L.nblocks),
                       dim3(CW * RG), 0, st, L.v, L.rows, L.ld, L.b, n, L.tau, cin, L.v, L.ld,
                       run_if);
}

// Rows per thread follow from the block height: RPG = rows / RG (see tsqr_shape).
void tsqr_level(bool apply, const TsqrLevel& L, int n, const double* cin, const int* run_if,
                hipStream_t st) {
  switch (tsqr_shape(n).cw) {
    case 32:
      if (L.leaf) tsqr_level_launch<32, 32, 192 / 32>(apply, L, n, cin, run_if, st);
      else tsqr_level_launch<32, 32, 384 / 32>(apply, L, n, cin, run_if, st);
      break;
    case 64:
      if (L.leaf) tsqr_level_launch<64, 16, 192 / 16>(apply, L, n, cin, run_if, st);
      else tsqr_level_launch<64, 16, 256 / 16>(apply, L, n, cin, run_if, st);
      break;
    default:
      if (L.leaf) tsqr_level_launch<96, 8, 160 / 8>(apply, L, n, cin, run_if, st);
      else tsqr_level_launch<96, 8, 192 / 8>(apply, L, n, cin, run_if, st);
      break;
  }
}

void tsqr(double* Y, int64_t m, int n, int64_t ld, double* R_out, double* ws, hipStream_t st,
          const int* run_if_set) {
  std::vector<TsqrLevel> lv = plan_tsqr(Y, m, n, ld, ws);
  for (const TsqrLevel& L : lv) tsqr_level(false, L, n, nullptr, run_if_set, st);
  if (R_out)
    hipLaunchKernelGGL(copy_if_kernel, dim3(64), dim3(256), 0, st, R_out, lv.back().rstack,
                       (int64_t)n * n, run_if_set);
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    // above the top level Q starts as the identity; below it, as the rows of the level
    // above's Q, which that level wrote over this level's stacked R factors
    const double* cin = (l == (int)lv.size() - 1) ? nullptr : lv[l].rstack;
    tsqr_level(true, lv[l], n, cin, run_if_set, st);
  }
}

void set_lds_attr(const void* fn) {
  hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                      LDS_DOUBLES * (int)sizeof(double));
}

// Rows of X[:, j:j+jb] solved against the diagonal block L_jj: x L_jj^T = b for every row (a
// forward substitution, one row per thread held in registers; the block of L in LDS).
__global__ __launch_bounds__(64) void trsm_diag_kernel(double* Xall, int64_t ldx, int64_t m,
                                                       int64_t sX, const double* Lall, int n,
                                                       int64_t sL, int j, int jb) {
  __shared__ double D[64][65];
  const double* L = Lall + (int64_t)blockIdx.y * sL;
  double* X = Xall + (int64_t)blockIdx.y * sX;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < jb * jb; idx += 64) {
    const int r = idx / jb, c = idx - (idx / jb) * jb;
    D[r][c] = L[(int64_t)(j + r) * n + j + c];
  }
  __syncthreads();
  const int64_t row_i = (int64_t)blockIdx.x * 64 + tid;
  if (row_i >= m) return;
  double* row = X + row_i * ldx + j;
  double x[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) x[c] = (c < jb) ? row[c] : 0.0;
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    if (c < jb) {
      double s = x[c];
#pragma unroll
      for (int l = 0; l < c; ++l) s -= x[l] * D[c][l];
      x[c] = s / D[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < 64; ++c)
    if (c < jb) row[c] = x[c];
}

// Diagonal of each lower factor: raises *flag when an entry is not finite or not positive,
// when min d_i / max d_i < min_ratio (d_i = L_ii^2, the pivots), or when a pivot leaves
// (lo, hi) (lo = 0, hi = inf disable that test).
__global__ __launch_bounds__(256) void chol_check_kernel(const double* Lall, int n, int64_t sL,
                                                         double min_ratio, double lo, double hi,
                                                         int* flag, int code) {
  const double* L = Lall + (int64_t)blockIdx.x * sL;
  __shared__ double mn[256], mx[256];
  __shared__ int bad[256];
  double a = INFINITY, b = 0.0;
  int f = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double l = L[(int64_t)i * n + i];
    const double d = l * l;
    if (!(l > 0.0) || !isfinite(l) || !(d > lo) || !(d < hi)) f = 1;
    a = fmin(a, d);
    b = fmax(b, d);
  }
  mn[threadIdx.x] = a;
  mx[threadIdx.x] = b;
  bad[threadIdx.x] = f;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + o]);
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
      bad[threadIdx.x] |= bad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && (bad[0] || !(mn[0] >= min_ratio * mx[0]))) atomicOr(flag, code);
}

// Factor the (already updated) diagonal block at (j, j), jb <= 64, of every matrix of the
// batch (one wave each) and write L_jj back (zero above its diagonal) and L_jj^{-1} to
// Dinv[b][j / 64] (64 x 64, lower, zero-padded beyond jb).  The block is staged through LDS
// with coalesced loads; lane r then holds row r.  The factorisation is the right-looking
// column algorithm (pivot from lane k, column k published through LDS); the inverse is one
// forward substitution per lane, lane c building column c.  A pivot that is not positive
// ORs 1 into flag[0].
__global__ __launch_bounds__(64) void chol_diag_inv_kernel(double* Aall, double* Dinv, int n,
                                                           int j, int jb, int* flag) {
  __shared__ double blk[64][65];
  __shared__ double lk[64];
  double* A = Aall + (int64_t)blockIdx.y * n * n;
  double* Di = Dinv + ((int64_t)blockIdx.y * ((n + 63) / 64) + j / 64) * 64 * 64;
  const int r = threadIdx.x;
  {
    // all 64 loads in flight before the first LDS write (a load-then-store loop would wait
    // for each row in turn)
    double v[64];
#pragma unroll
    for (int rr = 0; rr < 64; ++rr)
      v[rr] = (rr < jb && r < jb) ? A[(int64_t)(j + rr) * n + j + r] : 0.0;
#pragma unroll
    for (int rr = 0; rr < 64; ++rr) blk[rr][r] = v[rr];
  }
  __syncthreads();
  double row[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) row[c] = (r < jb && c < jb) ? blk[r][c] : 0.0;
  __syncthreads();
  // Column k: every lane scales and publishes its entry, then updates its whole row to the
  // right of k without a per-lane condition: entries above the diagonal (c > r) take values
  // that are never read back, and padding rows (r >= jb) hold zeros throughout.  The
  // multipliers of the row are read from LDS in one batch before the updates.
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    if (k < jb) {
      const double piv = __shfl(row[k], k, 64);
      if (r == 0 && !(piv > 0.0)) atomicOr(flag, 1);
      const double dk = (piv > 0.0) ? sqrt(piv) : __builtin_nan("");
      if (r == k) row[k] = dk;
      if (r > k) row[k] /= dk;
      lk[r] = row[k];
      __syncthreads();
      double l[64];
#pragma unroll
      for (int c = k + 1; c < 64; ++c) l[c] = lk[c];
#pragma unroll
      for (int c = k + 1; c < 64; ++c) row[c] -= row[k] * l[c];
      __syncthreads();
    }
  }
  // L_jj to LDS (lower, zero above) and back to A
#pragma unroll
  for (int c = 0; c < 64; ++c) blk[r][c] = (r < jb && c <= r) ? row[c] : 0.0;
  __syncthreads();
  for (int rr = 0; rr < jb; ++rr)
    if (r < jb) A[(int64_t)(j + rr) * n + j + r] = blk[rr][r];
  // column r of L_jj^{-1}: x_i = (delta_ir - sum_{k < i} L_ik x_k) / L_ii, which is zero for
  // i < r without a condition (x_k = 0 for k < r); four partial sums shorten the chain
  double x[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    double v = 0.0;
    if (i < jb) {
      double p0 = (i == r) ? 1.0 : 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
      for (int k = 0; k + 3 < i; k += 4) {
        p0 -= blk[i][k] * x[k];
        p1 -= blk[i][k + 1] * x[k + 1];
        p2 -= blk[i][k + 2] * x[k + 2];
        p3 -= blk[i][k + 3] * x[k + 3];
      }
#pragma unroll
      for (int k = i & ~3; k < i; ++k) p0 -= blk[i][k] * x[k];
      v = ((p0 + p1) + (p2 + p3)) / blk[i][i];
    }
    x[i] = v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 64; ++i) blk[i][r] = x[i];
  __syncthreads();
  for (int rr = 0; rr < 64; ++rr) Di[rr * 64 + r] = blk[rr][r];
}

// Places the 64 x 64 diagonal-block inverses Dinv of `batch` lower matrices on the diagonal of
// Linv (n x n, zero elsewhere).
__global__ void place_diag_blocks_kernel(const double* Dinv, double* Linv, int n, int batch) {
  const int nb = (n + 63) / 64;
  const int64_t total = (int64_t)batch * n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / ((int64_t)n * n), rem = idx - b * n * n;
    const int i = (int)(rem / n), c = (int)(rem - (rem / n) * n);
    double v = 0.0;
    if (i / 64 == c / 64) v = Dinv[((b * nb + i / 64) * 64 + (i % 64)) * 64 + (c % 64)];
    Linv[idx] = v;
  }
}

namespace {
GemmArgs gemm_args(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, bool ta,
                   const double* B, int64_t ldb, bool tb, double* C, int64_t ldc, double alpha,
                   double beta, int64_t batch, int64_t sA, int64_t sB, int64_t sC) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA; g.ta = ta;
  g.B = B; g.ldb = ldb; g.sB = sB; g.tb = tb;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta; g.batch = batch;
  return g;
}
}  // namespace

void cholesky_blocked_inv(double* A, double* Dinv, int n, int batch, int* flag,
                          hipStream_t st) {
  const int64_t s2 = (int64_t)n * n;
  for (int j = 0; j < n; j += 64) {
    const int jb = (n - j) < 64 ? (n - j) : 64;
    hipLaunchKernelGGL(chol_diag_inv_kernel, dim3(1, batch), dim3(64), 0, st, A, Dinv, n, j, jb,
                       flag);
    const int rest = n - j - jb;
    if (rest <= 0) break;
    const int64_t nb = (n + 63) / 64;
    // panel below the block, in place: L21 = A21 L_jj^{-T} (one column tile, so every
    // work-group reads its rows before writing them)
    double* A21 = A + (int64_t)(j + jb) * n + j;
    gemm_f64(gemm_args(rest, jb, jb, A21, n, false, Dinv + (int64_t)(j / 64) * 64 * 64, 64, true,
                       A21, n, 1.0, 0.0, batch, s2, nb * 64 * 64, s2), st);
    // trailing update A22 -= L21 L21^T
    double* A22 = A + (int64_t)(j + jb) * n + j + jb;
    gemm_f64(gemm_args(rest, rest, jb, A21, n, false, A21, n, true, A22, n, -1.0, 1.0, batch, s2,
                       s2, s2), st);
  }
  const int64_t total = s2 * batch;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, n, batch);
}

void cholesky_shifted_inv(double* A, double* Dinv, int n, int batch, double shift_rel,
                          int* flag, hipStream_t st) {
  hipLaunchKernelGGL(add_shift_kernel, dim3(batch), dim3(1024), 0, st, A, n, shift_rel);
  cholesky_blocked_inv(A, Dinv, n, batch, flag, st);
}

void tri_inv_lower(const double* L, const double* Dinv, double* Linv, double* T, int n,
                   int batch, hipStream_t st, double* partial, size_t partial_doubles) {
  const int64_t s2 = (int64_t)n * n;
  // a product with fewer than 64 output tiles runs split along K (parts of >= 64) when the
  // partial-sum buffer holds them: one work-group per tile would leave most of the chip idle
  auto run = [&](const GemmArgs& g) {
    const int64_t tiles = ((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch;
    const int64_t mn = g.M * g.N * g.batch;
    int64_t parts = std::min<int64_t>(g.K / 64, 8);
    if (partial && mn > 0)
      parts = std::min<int64_t>(parts, (int64_t)(partial_doubles / (size_t)mn));
    if (partial && tiles < 64 && parts >= 2)
      gemm_f64_splitk(g, (int)parts, partial, st);
    else
      gemm_f64(g, st);
  };
  {
    const int64_t total = s2 * batch;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(place_diag_blocks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Dinv,
                       Linv, n, batch);
  }
  // doubling: for a pair of diagonal blocks [[A, 0], [B, C]] whose inverses are in place,
  // the off-diagonal block of the inverse is -C^{-1} (B A^{-1})
  for (int s = 64; s < n; s *= 2) {
    const int pairs_full = n / (2 * s);
    const int64_t stride = 2 * (int64_t)s * (n + 1);
    for (int b = 0; b < batch; ++b) {
      const double* Lb = L + b * s2;
      double* Xb = Linv + b * s2;
      if (pairs_full > 0) {
        // T_i = B_i A_i^{-1}, X21_i = -C_i^{-1} T_i, for the pairs at o = 2 s i
        run(gemm_args(s, s, s, Lb + (int64_t)s * n, n, false, Xb, n, false, T, s, 1.0, 0.0,
                           pairs_full, stride, stride, (int64_t)s * s));
        run(gemm_args(s, s, s, Xb + (int64_t)s * n + s, n, false, T, s, false,
                           Xb + (int64_t)s * n, n, -1.0, 0.0, pairs_full, stride,
                           (int64_t)s * s, stride));
      }
      const int o = pairs_full * 2 * s;
      const int sc = n - o - s;  // a last, partial pair: A of size s, C of size sc < s
      if (sc > 0) {
        run(gemm_args(sc, s, s, Lb + (int64_t)(o + s) * n + o, n, false,
                           Xb + (int64_t)o * n + o, n, false, T, s, 1.0, 0.0, 1, 0, 0, 0));
        run(gemm_args(sc, s, sc, Xb + (int64_t)(o + s) * n + o + s, n, false, T, s, false,
                           Xb + (int64_t)(o + s) * n + o, n, -1.0, 0.0, 1, 0, 0, 0));
      }
    }
  }
}

void trsm_right_lower_t(double* X, int64_t ldx, int64_t m, const double* L, int n, int batch,
                        int64_t sX, int64_t sL, hipStream_t st) {
  const int nbk = 64;
  for (int j = 0; j < n; j += nbk) {
    const int jb = (n - j) < nbk ? (n - j) : nbk;
    if (j > 0) {
      // X[:, j:j+jb] -= X[:, 0:j] L[j:j+jb, 0:j]^T
      GemmArgs g;
      g.M = m;
      g.N = jb;
      g.K = j;
      g.A = X;
      g.lda = ldx;
      g.sA = sX;
      g.ta = false;
      g.B = L + (int64_t)j * n;
      g.ldb = n;
      g.sB = sL;
      g.tb = true;
      g.C = X + j;
      g.ldc = ldx;
      g.sC = sX;
      g.alpha = -1.0;
      g.beta = 1.0;
      g.batch = batch;
      gemm_f64(g, st);
    }
    hipLaunchKernelGGL(trsm_diag_kernel, dim3((unsigned)((m + 63) / 64), batch), dim3(64), 0,
                       st, X, ldx, m, sX, L, n, sL, j, jb);
  }
}

void chol_check(const double* L, int n, int batch, double min_ratio, double lo, double hi,
                int* flag, hipStream_t st, int code) {
  hipLaunchKernelGGL(chol_check_kernel, dim3(batch), dim3(256), 0, st, L, n, (int64_t)n * n,
                     min_ratio, lo, hi, flag, code);
}

void chol_inv(const double* G, double* R, double* Rinv, int n, int pass, int* fail,
              hipStream_t st, double shift_coef, int* sticky, int batch, int64_t sG,
              int64_t sR, int64_t sRi, int sf) {
  if (batch < 1) return;
  hipLaunchKernelGGL(chol_inv_kernel, dim3((unsigned)batch), dim3(1024), 0, st, G, R, Rinv, n,
                     pass, fail, shift_coef, sticky, sG, sR, sRi, sf);
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
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1, batch), dim3(64), 0, st, A, n, j, jb, flag);
    const int rows_below = n - j - jb;
    if (rows_below > 0)
      hipLaunchKernelGGL(chol_trsm_kernel, dim3((rows_below + 63) / 64, batch), dim3(64), 0, st,
                         A, n, j, jb);
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
