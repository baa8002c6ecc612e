// FP64 GEMM on the CDNA4 FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Every contraction of the Triad-ATRG step (Section 2: bond swap products, Grams of the
// isometries and squeezers, triad tensors and the O(r^2 chi^7) contraction of Eqs. (makeMG),
// (makeMH)) is issued as a strided-batched row-major GEMM after leg reordering.
//
// Tiling: a 256-thread workgroup (4 wave64s in a 2 x 2 grid) computes a 128 x 128 tile of C;
// each wave owns 64 x 64 = 4 x 4 MFMA blocks of 16 x 16 held in 64 accumulator doubles per
// lane.  Products with N <= 96 (a tall panel times a small matrix) use tiles 32, 64 or 96
// wide, so the matrix cores do no work on padding columns.  K advances in steps of BK = 8 through a double-buffered LDS stage (A as [k][m], B as
// [k][n], so MFMA fragments are read with unit stride); the next stage's global loads are
// issued before the MFMAs of the current one.  Global loads are mapped so that consecutive
// lanes read consecutive addresses of whichever dimension is contiguous in memory (the
// transposes are template parameters).  Optional split-K: blockIdx.z enumerates (batch, K part)
// and parts are summed afterwards in a fixed order.
#include "common.h"

#include <algorithm>

namespace tatrg {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 128, BK = 8, PAD = 4, NT = 256;
constexpr int EA = BM * BK / NT;  // staged A elements per thread

struct KArgs {
  GemmArgs g;
  int kparts;       // 1 = no split
  int64_t kchunk;   // K elements per part
  double* partial;  // kparts > 1: output [batch][kparts][M][N]
};

// PLAIN: C = op(A) op(B) (alpha = 1, beta = 0, or a split-K partial).  The accumulators are
// then stored straight from the accumulation registers; the general epilogue (scaling by
// alpha, adding beta C) moves them to vector registers first and halves the occupancy.
// TN: MFMA blocks per wave along N (tile width 32 TN): narrower tiles for products with
// N <= 96 (panel times a small matrix) so that no matrix-core work is spent on padding.
template <bool TA, bool TB, bool PLAIN, int TN>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(KArgs ka) {
  constexpr int BNT = 32 * TN, EB = BNT * BK / NT;
  const GemmArgs& g = ka.g;
  if (g.cond && ((g.cond[(int64_t)(blockIdx.z / ka.kparts) * g.cond_stride] != 0) !=
                 g.cond_when))
    return;
  // tile: blockIdx.(x, y) = (N tile, M tile); for a symmetric split-K product blockIdx.x
  // enumerates the tiles on and above the diagonal column by column, t = tn (tn + 1) / 2 + tm,
  // so consecutive work-groups (which the dispatcher spreads over the XCDs) share the load
  int tile_m = blockIdx.y, tile_n = blockIdx.x;
  if (g.sym && ka.kparts > 1) {
    const int t = blockIdx.x;
    int tn = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((tn + 1) * (tn + 2) / 2 <= t) ++tn;
    while (tn * (tn + 1) / 2 > t) --tn;
    tile_n = tn;
    tile_m = t - tn * (tn + 1) / 2;
  }
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BNT + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t z = blockIdx.z;
  const int64_t b = z / ka.kparts;
  const int64_t p = z - b * ka.kparts;
  const int64_t kb = p * ka.kchunk;
  const int64_t K = (ka.kparts > 1) ? ((g.K - kb) < ka.kchunk ? (g.K - kb) : ka.kchunk) : g.K;

  const double* A = g.A + b * g.sA + (TA ? kb * g.lda : kb);
  const double* B = g.B + b * g.sB + (TB ? kb : kb * g.ldb);
  const int64_t m0 = (int64_t)tile_m * BM;
  const int64_t n0 = (int64_t)tile_n * BNT;
  const int64_t M = g.M, N = g.N;

  // element e of a stage: A tile row/k and B tile column/k
  auto a_rk = [&](int e, int& r, int& kk) {
    if (TA) { r = e % BM; kk = e / BM; } else { r = e / BK; kk = e % BK; }
  };
  auto b_ck = [&](int e, int& c, int& kk) {
    if (TB) { c = e / BK; kk = e % BK; } else { c = e % BNT; kk = e / BNT; }
  };
  double ra[EA], rb[EB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      int r, kk;
      a_rk(tid + i * NT, r, kk);
      const int64_t m = m0 + r, k = k0 + kk;
      ra[i] = (m < M && k < K) ? (TA ? A[k * g.lda + m] : A[m * g.lda + k]) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      int c, kk;
      b_ck(tid + i * NT, c, kk);
      const int64_t n = n0 + c, k = k0 + kk;
      rb[i] = (n < N && k < K) ? (TB ? B[n * g.ldb + k] : B[k * g.ldb + n]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < EA; ++i) {
      int r, kk;
      a_rk(tid + i * NT, r, kk);
      As[buf][kk][r] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < EB; ++i) {
      int c, kk;
      b_ck(tid + i * NT, c, kk);
      Bs[buf][kk][c] = rb[i];
    }
  };

  d4 acc[4][TN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[4], bb[TN];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        a[t] = As[cur][kk + (lane >> 4)][wm * 64 + t * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < TN; ++t)
        bb[t] = Bs[cur][kk + (lane >> 4)][wn * TN * 16 + t * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // D fragment of v_mfma_f64_16x16x4: lane l, element v holds row (l/16) + 4v, column l%16
  // of the 16 x 16 block (checked against a host reference by the GEMM tests).
  double* C;
  int64_t ldc;
  double alpha, beta;
  if (ka.kparts > 1) {
    C = ka.partial + (b * ka.kparts + p) * M * N;
    ldc = N;
    alpha = 1.0;
    beta = 0.0;
  } else {
    C = g.C + b * g.sC;
    ldc = g.ldc;
    alpha = g.alpha;
    beta = g.beta;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // the old C of a row block is loaded before any of its stores, so the loads are in flight
    // together (interleaved, each store would wait for its own load); out-of-range entries read
    // the nearest in-range one (unused), so the loads need no per-entry branch
    double cold[TN][4];
    if (!PLAIN && beta != 0.0) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * v;
          const int64_t col = n0 + wn * TN * 16 + j * 16 + (lane & 15);
          const int64_t rc = row < M ? row : M - 1, cc = col < N ? col : N - 1;
          cold[j][v] = C[rc * ldc + cc];
        }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + (lane >> 4) + 4 * v;
        const int64_t col = n0 + wn * TN * 16 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          if (PLAIN) {
            C[row * ldc + col] = acc[i][j][v];
          } else {
            double val = alpha * acc[i][j][v];
            if (beta != 0.0) val += beta * cold[j][v];
            C[row * ldc + col] = val;
          }
        }
      }
  }
}

// C[b] = alpha * sum_p partial[b][p] + beta * C[b], parts summed in increasing p.  With sym,
// the partial sums exist for the 128 x 128 tiles on and above the diagonal only, and element
// (i, j) of a tile below it is read from (j, i).
__global__ void splitk_reduce(const double* partial, double* C, int64_t M, int64_t N,
                              int64_t ldc, int64_t sC, int kparts, int64_t batch, double alpha,
                              double beta, const int* cond, int cond_when, int sym,
                              int64_t cond_stride) {
  if (cond && cond_stride == 0 && ((*cond != 0) != (cond_when != 0))) return;
  const int64_t total = batch * M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / (M * N);
    if (cond && cond_stride > 0 && ((cond[b * cond_stride] != 0) != (cond_when != 0))) continue;
    const int64_t r = idx - b * M * N;
    const int64_t i = r / N, j = r - (r / N) * N;
    const int64_t src = (sym && i / BM > j / BN) ? j * N + i : r;
    const double* pp = partial + b * kparts * M * N + src;
    // parts added in increasing order, eight loads in flight at a time
    double s = 0.0;
    int p = 0;
    for (; p + 8 <= kparts; p += 8) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = pp[(int64_t)(p + t) * M * N];
#pragma unroll
      for (int t = 0; t < 8; ++t) s += v[t];
    }
    for (; p < kparts; ++p) s += pp[(int64_t)p * M * N];
    double* c = C + b * sC + i * ldc + j;
    double val = alpha * s;
    if (beta != 0.0) val += beta * *c;
    *c = val;
  }
}

// C = alpha * sum_p partial[p] + beta * C for many parts p of a small M x N output (one
// batch): 64 outputs per work-group, 16 groups of threads each summing every 16th part in
// increasing order, then the 16 group sums added in a fixed order (deterministic).
__global__ __launch_bounds__(1024) void parts_reduce_kernel(const double* partial, double* C,
                                                            int64_t M, int64_t N, int64_t ldc,
                                                            int64_t parts, double alpha,
                                                            double beta, const int* cond,
                                                            int cond_when) {
  if (cond && ((*cond != 0) != (cond_when != 0))) return;
  __shared__ double acc[16][64];
  const int tid = threadIdx.x, ol = tid & 63, pg = tid >> 6;
  const int64_t mn = M * N, o = (int64_t)blockIdx.x * 64 + ol;
  double sum = 0.0;
  if (o < mn) {
    // every 16th part in increasing order, eight loads in flight at a time
    int64_t p = pg;
    for (; p + 7 * 16 < parts; p += 8 * 16) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = partial[(p + 16 * t) * mn + o];
#pragma unroll
      for (int t = 0; t < 8; ++t) sum += v[t];
    }
    for (; p < parts; p += 16) sum += partial[p * mn + o];
  }
  acc[pg][ol] = sum;
  __syncthreads();
  if (pg == 0 && o < mn) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += acc[q][ol];
    const int64_t i = o / N, j = o - (o / N) * N;
    double* c = C + i * ldc + j;
    double val = alpha * t;
    if (beta != 0.0) val += beta * *c;
    *c = val;
  }
}

// Skinny products C = X^T Y with X (m x M), Y (m x N) row-major, M, N <= 16 NB, m long.
// Every wave sums its own chunk of rows into partial[wave] (M x N); no LDS: a lane loads
// its MFMA fragments straight from the rows (four rows per step, lane l reading row l/16,
// column 16 b + l%16), so each step reads four contiguous rows.  SYM (X = Y, M = N): only
// the 16 x 16 blocks on and above the diagonal are accumulated and each is also written
// transposed below it.
template <int NB, bool SYM>
__global__ __launch_bounds__(256) void gram_tn_kernel(const double* X, int64_t ldx,
                                                      const double* Y, int64_t ldy, int64_t m,
                                                      int M, int N, int64_t rows_per_wave,
                                                      int64_t nwaves, double* partial,
                                                      const int* cond, int cond_when) {
  if (cond && ((*cond != 0) != (cond_when != 0))) return;
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= nwaves) return;
  const int64_t r0 = wid * rows_per_wave;
  const int64_t r1 = (r0 + rows_per_wave < m) ? r0 + rows_per_wave : m;
  const int kr = lane >> 4, cl = lane & 15;
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // Rows go in batches of PF steps of four; the loads of the next batch are issued before the
  // products of the current one, so a wave keeps 6 PF (or 12 PF) loads in flight.  Rows are
  // accumulated in increasing order, one step at a time, as without the batching.
  constexpr int PF = SYM ? 4 : (NB >= 5 ? 1 : (NB == 4 ? 2 : 4));
  constexpr int PY = SYM ? 1 : PF;
  auto load = [&](double (&x)[PF][NB], double (&y)[PY][NB], int64_t rb) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int64_t row = rb + 4 * p + kr;
      const bool ok = row < r1;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = b * 16 + cl;
        x[p][b] = (ok && col < M) ? X[row * ldx + col] : 0.0;
        if (!SYM) y[SYM ? 0 : p][b] = (ok && col < N) ? Y[row * ldy + col] : 0.0;
      }
    }
  };
  auto compute = [&](double (&x)[PF][NB], double (&y)[PY][NB]) {
#pragma unroll
    for (int p = 0; p < PF; ++p)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (!SYM || i <= j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                x[p][i], SYM ? x[p][j] : y[SYM ? 0 : p][j], acc[i][j], 0, 0, 0);
  };
  double xa[PF][NB], ya[PY][NB], xb[PF][NB], yb[PY][NB];
  load(xa, ya, r0);
  for (int64_t r = r0; r < r1; r += 8 * PF) {
    load(xb, yb, r + 4 * PF);
    compute(xa, ya);
    load(xa, ya, r + 8 * PF);
    compute(xb, yb);
  }
  double* out = partial + wid * (int64_t)M * N;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (SYM && i > j) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + (lane >> 4) + 4 * v, col = j * 16 + cl;
        if (row < M && col < N) {
          out[row * N + col] = acc[i][j][v];
          if (SYM && i < j) out[col * N + row] = acc[i][j][v];
        }
      }
    }
}

// Skinny products C = X Y^T with X (M x k), Y (N x k) row-major, M, N <= 16 NB, k long (the
// rows are long).  Every wave sums its own chunk of k into partial[wave] (M x N).  Per step of
// 16 along k, lane l reads four consecutive values k0 + 4 (l/16) + 0..3 of row 16 b + l%16, so
// the 64 lanes of a block read 16 contiguous 128-byte row segments; MFMA j of the step then
// pairs the j-th of those four values of X and of Y (each lane supplies the same k to both
// operands, which is all the product needs).  SYM (X = Y, M = N): upper blocks only, mirrored.
template <int NB, bool SYM>
__global__ __launch_bounds__(256) void gram_nt_kernel(const double* X, int64_t ldx,
                                                      const double* Y, int64_t ldy, int64_t k,
                                                      int M, int N, int64_t cols_per_wave,
                                                      int64_t nwaves, double* partial,
                                                      const int* cond, int cond_when) {
  if (cond && ((*cond != 0) != (cond_when != 0))) return;
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= nwaves) return;
  const int64_t c0 = wid * cols_per_wave;
  const int64_t c1 = (c0 + cols_per_wave < k) ? c0 + cols_per_wave : k;
  const int kq = 4 * (lane >> 4), rl = lane & 15;
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t c = c0; c < c1; c += 16) {
    double xa[NB][4], yb[SYM ? 1 : NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int row = b * 16 + rl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = c + kq + q;
        xa[b][q] = (row < M && col < c1) ? X[row * ldx + col] : 0.0;
        if (!SYM) yb[SYM ? 0 : b][q] = (row < N && col < c1) ? Y[row * ldy + col] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (!SYM || i <= j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                xa[i][q], SYM ? xa[j][q] : yb[SYM ? 0 : j][q], acc[i][j], 0, 0, 0);
  }
  double* out = partial + wid * (int64_t)M * N;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (SYM && i > j) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i * 16 + (lane >> 4) + 4 * v, col = j * 16 + rl;
        if (row < M && col < N) {
          out[row * N + col] = acc[i][j][v];
          if (SYM && i < j) out[col * N + row] = acc[i][j][v];
        }
      }
    }
}

template <bool TA, bool TB, int TN>
void launch_t(const KArgs& ka, hipStream_t st) {
  const GemmArgs& g = ka.g;
  const int64_t tn = (g.N + 32 * TN - 1) / (32 * TN), tm = (g.M + BM - 1) / BM;
  dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)(g.batch * ka.kparts));
  if (g.sym && ka.kparts > 1) grid = dim3((unsigned)(tn * (tn + 1) / 2), 1u,
                                          (unsigned)(g.batch * ka.kparts));
  const bool plain = ka.kparts > 1 || (g.alpha == 1.0 && g.beta == 0.0);
  if (plain)
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, true, TN>), grid, dim3(NT), 0, st, ka);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, false, TN>), grid, dim3(NT), 0, st, ka);
}

template <bool TA, bool TB>
void launch_b(const KArgs& ka, hipStream_t st) {
  // the triangular tile order of symmetric split-K products needs square tiles
  const int64_t N = ka.g.N;
  if ((ka.g.sym && ka.kparts > 1) || N > 96) launch_t<TA, TB, 4>(ka, st);
  else if (N > 64) launch_t<TA, TB, 3>(ka, st);
  else if (N > 32) launch_t<TA, TB, 2>(ka, st);
  else launch_t<TA, TB, 1>(ka, st);
}

void launch(const KArgs& ka, hipStream_t st) {
  const GemmArgs& g = ka.g;
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (g.ta) {
    if (g.tb) launch_b<true, true>(ka, st);
    else launch_b<true, false>(ka, st);
  } else {
    if (g.tb) launch_b<false, true>(ka, st);
    else launch_b<false, false>(ka, st);
  }
}

}  // namespace

void gemm_f64(const GemmArgs& g, hipStream_t st) {
  KArgs ka{g, 1, g.K, nullptr};
  launch(ka, st);
}

namespace {

// C = alpha X Y^T + beta C for long rows (M, N <= 96): gram_nt_kernel, then the parts.
bool gram_nt(const GemmArgs& g, double* partial, size_t partial_doubles, hipStream_t st) {
  const int64_t mn = g.M * g.N;
  int64_t nw = std::min<int64_t>(2048, (g.K + 255) / 256);   // >= 256 of k per wave
  nw = std::min<int64_t>(nw, (int64_t)(partial_doubles / (size_t)mn));
  if (nw < 1) return false;
  int64_t cpw = (g.K + nw - 1) / nw;
  cpw = ((cpw + 15) / 16) * 16;
  nw = (g.K + cpw - 1) / cpw;
  const int nbk = (int)((std::max(g.M, g.N) + 15) / 16);
  const dim3 grid((unsigned)((nw + 3) / 4));
  const int cw = g.cond_when ? 1 : 0;
  const bool sym = g.A == g.B && g.lda == g.ldb && g.M == g.N;
  switch (nbk) {
#define GRAM_NT_CASE(NB)                                                                      \
  case NB:                                                                                    \
    if (sym)                                                                                  \
      hipLaunchKernelGGL((gram_nt_kernel<NB, true>), grid, dim3(256), 0, st, g.A, g.lda, g.B, \
                         g.ldb, g.K, (int)g.M, (int)g.N, cpw, nw, partial, g.cond, cw);       \
    else                                                                                      \
      hipLaunchKernelGGL((gram_nt_kernel<NB, false>), grid, dim3(256), 0, st, g.A, g.lda,     \
                         g.B, g.ldb, g.K, (int)g.M, (int)g.N, cpw, nw, partial, g.cond, cw);  \
    break;
    GRAM_NT_CASE(1)
    GRAM_NT_CASE(2)
    GRAM_NT_CASE(3)
    GRAM_NT_CASE(4)
    GRAM_NT_CASE(5)
#undef GRAM_NT_CASE
    case 6:  // the general 96 x 96 product does not fit the registers: GEMM path
      if (!sym) return false;
      hipLaunchKernelGGL((gram_nt_kernel<6, true>), grid, dim3(256), 0, st, g.A, g.lda, g.B,
                         g.ldb, g.K, (int)g.M, (int)g.N, cpw, nw, partial, g.cond, cw);
      break;
    default:
      return false;
  }
  hipLaunchKernelGGL(parts_reduce_kernel, dim3((unsigned)((mn + 63) / 64)), dim3(1024), 0, st,
                     partial, g.C, g.M, g.N, g.ldc, nw, g.alpha, g.beta, g.cond, cw);
  return true;
}

}  // namespace

bool gram_tn(const GemmArgs& g, double* partial, size_t partial_doubles, hipStream_t st) {
  if (g.batch != 1 || g.M > 96 || g.N > 96 || g.M < 1 || g.N < 1) return false;
  if (!g.ta && g.tb) return gram_nt(g, partial, partial_doubles, st);
  if (!(g.ta && !g.tb)) return false;
  const int64_t mn = g.M * g.N;
  int64_t nw = std::min<int64_t>(2048, (g.K + 63) / 64);   // >= 64 rows per wave
  nw = std::min<int64_t>(nw, (int64_t)(partial_doubles / (size_t)mn));
  if (nw < 1) return false;
  int64_t rpw = (g.K + nw - 1) / nw;
  rpw = ((rpw + 3) / 4) * 4;
  nw = (g.K + rpw - 1) / rpw;
  const int nbk = (int)((std::max(g.M, g.N) + 15) / 16);
  const dim3 grid((unsigned)((nw + 3) / 4));
  const int cw = g.cond_when ? 1 : 0;
  const bool sym = g.A == g.B && g.lda == g.ldb && g.M == g.N;
  switch (nbk) {
#define GRAM_CASE(NB)                                                                         \
  case NB:                                                                                    \
    if (sym)                                                                                  \
      hipLaunchKernelGGL((gram_tn_kernel<NB, true>), grid, dim3(256), 0, st, g.A, g.lda, g.B, \
                         g.ldb, g.K, (int)g.M, (int)g.N, rpw, nw, partial, g.cond, cw);       \
    else                                                                                      \
      hipLaunchKernelGGL((gram_tn_kernel<NB, false>), grid, dim3(256), 0, st, g.A, g.lda,     \
                         g.B, g.ldb, g.K, (int)g.M, (int)g.N, rpw, nw, partial, g.cond, cw);  \
    break;
    GRAM_CASE(1) GRAM_CASE(2) GRAM_CASE(3) GRAM_CASE(4) GRAM_CASE(5) GRAM_CASE(6)
#undef GRAM_CASE
    default:
      return false;
  }
  hipLaunchKernelGGL(parts_reduce_kernel, dim3((unsigned)((mn + 63) / 64)), dim3(1024), 0, st,
                     partial, g.C, g.M, g.N, g.ldc, nw, g.alpha, g.beta, g.cond, cw);
  return true;
}

void gemm_f64_splitk(const GemmArgs& g, int parts, double* partial, hipStream_t st) {
  if (parts <= 1 || g.K <= BK) {
    gemm_f64(g, st);
    return;
  }
  int64_t chunk = (g.K + parts - 1) / parts;
  chunk = ((chunk + BK - 1) / BK) * BK;
  const int used = (int)((g.K + chunk - 1) / chunk);
  KArgs ka{g, used, chunk, partial};
  launch(ka, st);
  const int64_t total = g.batch * g.M * g.N;
  const int threads = 256;
  int64_t blocks = (total + threads - 1) / threads;
  if (blocks > 65535) blocks = 65535;
  const int sym = (g.sym && g.M == g.N) ? 1 : 0;
  hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)blocks), dim3(threads), 0, st, partial, g.C,
                     g.M, g.N, g.ldc, g.sC, used, g.batch, g.alpha, g.beta, g.cond,
                     g.cond_when ? 1 : 0, sym, g.cond_stride);
}

}  // namespace tatrg
