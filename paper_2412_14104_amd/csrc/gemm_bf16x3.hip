// Split-precision GEMM on the CDNA4 bf16 matrix cores for the contraction of Eqs. (makeMG),
// (makeMH) (the O(r^2 chi^7) part of the step, Table 1).
//
// Every float64 operand x is split into three bf16 planes x = x0 + x1 + x2 (each residual is
// formed exactly in float64 before rounding to bf16), so the planes hold ~24 significant
// bits.  C = sum_{i+j<=2} A_i B_j: six bf16 x bf16 products on v_mfma_f32_16x16x32_bf16.  The
// leading product A_0 B_0 has float32 accumulators of its own that are added into float64
// accumulators after every 32-wide step of K (one MFMA per block), so its float32 rounding is
// that of a single 32-term dot product; the five smaller products (2^-8 of its size and less)
// share a second set flushed every LO_FLUSH_TILES steps.
//
// Layout: the split kernel writes every operand's planes k-contiguous -- A as [M][Kp], B as
// [N][Kp], Kp = K rounded up to 8 and zero padded -- transposing through an LDS tile where the
// float64 operand is stored the other way, so the GEMM reads 16-byte vectors of 8 bf16 along
// K for both operands and stores them to LDS unchanged; an MFMA fragment is then one 16-byte
// LDS read.  Tiling: 512 threads (8 wave64 in a 2 x 4 grid), 128 x 128 tile of C, 64 x 32 per
// wave as 4 x 2 MFMA blocks; K advances by 32 through double-buffered LDS holding all six
// planes of the stage; each plane's fragments are read once and serve every product they
// enter.  Work-groups are ordered so that the tiles sharing a B tile run on one XCD.
#include "common.h"

namespace tatrg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8, NT = 512;
constexpr int LO_FLUSH_TILES = 4;  // float32 window of the small products: 4 x 32 values of K
constexpr int ST = 64;             // split kernel tile (rows x K)

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

// Planes of a float64 operand viewed as R x K per batch entry b: element (r, k) is
// x[b*sx + k*ld + r] (trans) or x[b*sx + r*ld + k].  Output plane p: out_p[(b*R + r)*Kp + k],
// zero for K <= k < Kp.  One 64 x 64 tile per work-group, staged through LDS so that both the
// float64 reads and the bf16 writes are contiguous.
__global__ __launch_bounds__(256) void split3_kernel(const double* __restrict__ x, int64_t R,
                                                     int64_t K, int64_t ld, int64_t sx,
                                                     int trans, int64_t Kp,
                                                     uint16_t* __restrict__ p0,
                                                     uint16_t* __restrict__ p1,
                                                     uint16_t* __restrict__ p2) {
  __shared__ double tile[ST][ST + 1];  // [r][k]
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.z;
  const int64_t r0 = (int64_t)blockIdx.y * ST, k0 = (int64_t)blockIdx.x * ST;
  const double* xb = x + b * sx;
  for (int idx = tid; idx < ST * ST; idx += 256) {
    int rr, kk;
    if (trans) {
      kk = idx / ST;
      rr = idx % ST;
    } else {
      rr = idx / ST;
      kk = idx % ST;
    }
    const int64_t r = r0 + rr, k = k0 + kk;
    tile[rr][kk] = (r < R && k < K) ? (trans ? xb[k * ld + r] : xb[r * ld + k]) : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < ST * ST; idx += 256) {
    const int rr = idx / ST, kk = idx % ST;
    const int64_t r = r0 + rr, k = k0 + kk;
    if (r < R && k < Kp) {
      const double v = tile[rr][kk];
      const uint16_t a = bf16_rne((float)v);
      const double r1 = v - bf16_to_double(a);
      const uint16_t c = bf16_rne((float)r1);
      const double r2 = r1 - bf16_to_double(c);
      const int64_t o = (b * R + r) * Kp + k;
      p0[o] = a;
      p1[o] = c;
      p2[o] = bf16_rne((float)r2);
    }
  }
}

struct BArgs {
  GemmArgs g;
  const uint16_t* a[3];  // [batchA][M][Kp]
  const uint16_t* b[3];  // [batchB][N][Kp]
  int64_t Kp, sAp, sBp;  // plane batch strides (0 for an operand shared by the batch)
  int tiles_m, tiles_n;
};

__global__ __launch_bounds__(NT, 1) void gemm_bf16x3_kernel(BArgs ba) {
  const GemmArgs& g = ba.g;
  __shared__ uint16_t As[2][3][BM][KP];
  __shared__ uint16_t Bs[2][3][BN][KP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int64_t b = blockIdx.z;
  // XCD-aware order: work-group w runs on XCD w % 8; tiles are numbered so that each XCD
  // gets a contiguous range, M fastest, i.e. the tiles that share a B tile.
  const int nt = ba.tiles_m * ba.tiles_n;
  int w = blockIdx.x;
  if (nt % 8 == 0) w = (w % 8) * (nt / 8) + w / 8;
  const int tm = w % ba.tiles_m, tn = w / ba.tiles_m;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = g.M, N = g.N, Kp = ba.Kp;

  // A stage: 3 planes x 128 rows x 4 chunks of 8 bf16; B likewise: 3072 chunks, 6 per thread
  uint4 stg[6];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int e = tid + i * NT;
      const int op = e / 1536, rem = e - op * 1536;
      const int p = rem >> 9, row = (rem & 511) >> 2, kc = rem & 3;
      const int64_t k = k0 + kc * 8;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (op == 0) {
        const int64_t m = m0 + row;
        if (m < M && k < Kp)
          v = *reinterpret_cast<const uint4*>(ba.a[p] + b * ba.sAp + m * Kp + k);
      } else {
        const int64_t n = n0 + row;
        if (n < N && k < Kp)
          v = *reinterpret_cast<const uint4*>(ba.b[p] + b * ba.sBp + n * Kp + k);
      }
      stg[i] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int e = tid + i * NT;
      const int op = e / 1536, rem = e - op * 1536;
      const int p = rem >> 9, row = (rem & 511) >> 2, kc = rem & 3;
      uint16_t* dst = (op == 0) ? &As[buf][p][row][kc * 8] : &Bs[buf][p][row][kc * 8];
      *reinterpret_cast<uint4*>(dst) = stg[i];
    }
  };

  f4 hi[4][2], lo[4][2];
  double dacc[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      hi[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      lo[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
    }

  const int64_t nk = (Kp + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int kg = 8 * (lane >> 4), rl = lane & 15;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
    bf16x8 fa[3][4], fb[3][2];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        fa[p][t] = *reinterpret_cast<const bf16x8*>(&As[cur][p][wm * 64 + t * 16 + rl][kg]);
#pragma unroll
      for (int t = 0; t < 2; ++t)
        fb[p][t] = *reinterpret_cast<const bf16x8*>(&Bs[cur][p][wn * 32 + t * 16 + rl][kg]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        hi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[0][j], hi[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[1][j], lo[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[0][j], lo[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[1][j], lo[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[2][j], lo[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[0][j], lo[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)hi[i][j][v];
        hi[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    if ((kt + 1) % LO_FLUSH_TILES == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)lo[i][j][v];
          lo[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  // D fragment of v_mfma_f32_16x16x32_bf16: lane l, element v holds row 4*(l/16) + v,
  // column l%16 of the 16 x 16 block.
  double* C = g.C + b * g.sC;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn * 32 + j * 16 + rl;
        if (row < M && col < N) {
          double val = g.alpha * dacc[i][j][v];
          if (g.beta != 0.0) val += g.beta * C[row * g.ldc + col];
          C[row * g.ldc + col] = val;
        }
      }
}

// Plane batch entries of an operand: 1 when it is shared by the batch (stride 0).
int64_t plane_batches(const GemmArgs& g, bool a_side) {
  const int64_t s = a_side ? g.sA : g.sB;
  return s == 0 ? 1 : g.batch;
}

int64_t kpad(int64_t K) { return ((K + 7) / 8) * 8; }

}  // namespace

size_t gemm_bf16x3_ws_doubles(const GemmArgs& g) {
  const int64_t Kp = kpad(g.K);
  const int64_t na = plane_batches(g, true) * g.M * Kp;
  const int64_t nb = plane_batches(g, false) * g.N * Kp;
  return (size_t)((3 * (na + nb) * 2 + 7) / 8 + 64);
}

void gemm_bf16x3(const GemmArgs& g, double* planes_ws, size_t planes_ws_doubles,
                 hipStream_t st, hipEvent_t ev_after_split) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  (void)planes_ws_doubles;
  const int64_t Kp = kpad(g.K);
  const int64_t ba_n = plane_batches(g, true), bb_n = plane_batches(g, false);
  const int64_t na = ba_n * g.M * Kp, nb = bb_n * g.N * Kp;
  // plane starts stay 16-byte aligned: na and nb are multiples of 8 elements
  uint16_t* w = reinterpret_cast<uint16_t*>(planes_ws);
  BArgs ba;
  ba.g = g;
  for (int p = 0; p < 3; ++p) {
    ba.a[p] = w + p * na;
    ba.b[p] = w + 3 * na + p * nb;
  }
  ba.Kp = Kp;
  ba.sAp = (ba_n == 1) ? 0 : g.M * Kp;
  ba.sBp = (bb_n == 1) ? 0 : g.N * Kp;
  ba.tiles_m = (int)((g.M + BM - 1) / BM);
  ba.tiles_n = (int)((g.N + BN - 1) / BN);
  // op(A) is M x K, stored K x M when ta.  op(B) is K x N and its planes are N x K, so the
  // float64 B is read transposed unless it is stored N x K (tb).
  {
    dim3 grid((unsigned)((Kp + ST - 1) / ST), (unsigned)((g.M + ST - 1) / ST), (unsigned)ba_n);
    hipLaunchKernelGGL(split3_kernel, grid, dim3(256), 0, st, g.A, g.M, g.K, g.lda, g.sA,
                       g.ta ? 1 : 0, Kp, w, w + na, w + 2 * na);
  }
  {
    dim3 grid((unsigned)((Kp + ST - 1) / ST), (unsigned)((g.N + ST - 1) / ST), (unsigned)bb_n);
    hipLaunchKernelGGL(split3_kernel, grid, dim3(256), 0, st, g.B, g.N, g.K, g.ldb, g.sB,
                       g.tb ? 0 : 1, Kp, w + 3 * na, w + 3 * na + nb, w + 3 * na + 2 * nb);
  }
  if (ev_after_split) (void)hipEventRecord(ev_after_split, st);
  dim3 grid((unsigned)(ba.tiles_m * ba.tiles_n), 1u, (unsigned)g.batch);
  hipLaunchKernelGGL(gemm_bf16x3_kernel, grid, dim3(NT), 0, st, ba);
}

}  // namespace tatrg
