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
// Tiling: 256 threads (4 wave64 in a 2 x 2 grid), 128 x 128 tile of C, 64 x 64 per wave as 4 x 4
// MFMA blocks; K advances by 32 through double-buffered LDS holding all six planes of the
// stage, stored k-contiguous ([m][k] for A, [n][k] for B) so that every MFMA fragment is one
// 16-byte LDS read.
#include "common.h"

namespace tatrg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8, NT = 256;
constexpr int LO_FLUSH_TILES = 4;  // float32 window of the small products: 4 x 32 values of K

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

__global__ void split3_kernel(const double* __restrict__ x, int64_t n, uint16_t* __restrict__ p0,
                              uint16_t* __restrict__ p1, uint16_t* __restrict__ p2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    const uint16_t a = bf16_rne((float)v);
    const double r1 = v - bf16_to_double(a);
    const uint16_t b = bf16_rne((float)r1);
    const double r2 = r1 - bf16_to_double(b);
    p0[i] = a;
    p1[i] = b;
    p2[i] = bf16_rne((float)r2);
  }
}

struct Planes {
  const uint16_t* a[3];
  const uint16_t* b[3];
};

struct BArgs {
  GemmArgs g;
  Planes pl;
};

__global__ __launch_bounds__(NT) void gemm_bf16x3_kernel(BArgs ba) {
  const GemmArgs& g = ba.g;
  __shared__ uint16_t As[2][3][BM][KP];
  __shared__ uint16_t Bs[2][3][BN][KP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t b = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t M = g.M, N = g.N, K = g.K;

  // staging registers: 16 values per plane per operand
  uint16_t ra[3][16], rb[3][16];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const uint16_t* A = ba.pl.a[p] + b * g.sA;
      const uint16_t* B = ba.pl.b[p] + b * g.sB;
      if (!g.ta) {  // A[m][k]: row r = tid/2, k half = (tid&1)*16
        const int r = tid >> 1, kc = (tid & 1) * 16;
        const int64_t m = m0 + r;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t k = k0 + kc + i;
          ra[p][i] = (m < M && k < K) ? A[m * g.lda + k] : (uint16_t)0;
        }
      } else {      // A stored K x M: k = tid/8, m chunk = (tid&7)*16
        const int kk = tid >> 3, mc = (tid & 7) * 16;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t m = m0 + mc + i;
          ra[p][i] = (m < M && k < K) ? A[k * g.lda + m] : (uint16_t)0;
        }
      }
      if (!g.tb) {  // B stored K x N: k = tid/8, n chunk = (tid&7)*16
        const int kk = tid >> 3, nc = (tid & 7) * 16;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t n = n0 + nc + i;
          rb[p][i] = (n < N && k < K) ? B[k * g.ldb + n] : (uint16_t)0;
        }
      } else {      // B stored N x K
        const int r = tid >> 1, kc = (tid & 1) * 16;
        const int64_t n = n0 + r;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t k = k0 + kc + i;
          rb[p][i] = (n < N && k < K) ? B[n * g.ldb + k] : (uint16_t)0;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      if (!g.ta) {
        const int r = tid >> 1, kc = (tid & 1) * 16;
#pragma unroll
        for (int i = 0; i < 16; ++i) As[buf][p][r][kc + i] = ra[p][i];
      } else {
        const int kk = tid >> 3, mc = (tid & 7) * 16;
#pragma unroll
        for (int i = 0; i < 16; ++i) As[buf][p][mc + i][kk] = ra[p][i];
      }
      if (!g.tb) {
        const int kk = tid >> 3, nc = (tid & 7) * 16;
#pragma unroll
        for (int i = 0; i < 16; ++i) Bs[buf][p][nc + i][kk] = rb[p][i];
      } else {
        const int r = tid >> 1, kc = (tid & 1) * 16;
#pragma unroll
        for (int i = 0; i < 16; ++i) Bs[buf][p][r][kc + i] = rb[p][i];
      }
    }
  };

  f4 hi[4][4], lo[4][4];
  double dacc[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      hi[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      lo[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
    }

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int pa[6] = {0, 0, 1, 1, 0, 2};
  const int pb[6] = {0, 1, 0, 1, 2, 0};
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
    const int kg = 8 * (lane >> 4);
#pragma unroll
    for (int pr = 0; pr < 6; ++pr) {
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fa[t] = *reinterpret_cast<const bf16x8*>(
            &As[cur][pa[pr]][wm * 64 + t * 16 + (lane & 15)][kg]);
        fb[t] = *reinterpret_cast<const bf16x8*>(
            &Bs[cur][pb[pr]][wn * 64 + t * 16 + (lane & 15)][kg]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (pr == 0)
            hi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], hi[i][j], 0, 0, 0);
          else
            lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], lo[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)hi[i][j][v];
        hi[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
    if ((kt + 1) % LO_FLUSH_TILES == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
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
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double val = g.alpha * dacc[i][j][v];
          if (g.beta != 0.0) val += g.beta * C[row * g.ldc + col];
          C[row * g.ldc + col] = val;
        }
      }
}

// Number of elements spanned by a (possibly batched) operand: (batch-1)*stride + rows*ld.
int64_t span(int64_t rows, int64_t ld, int64_t batch, int64_t stride) {
  return (batch - 1) * stride + rows * ld;
}

}  // namespace

size_t gemm_bf16x3_ws_doubles(const GemmArgs& g) {
  const int64_t ra = g.ta ? g.K : g.M, rb = g.tb ? g.N : g.K;
  const int64_t na = span(ra, g.lda, g.batch, g.sA), nb = span(rb, g.ldb, g.batch, g.sB);
  return (size_t)((3 * (na + nb) * 2 + 7) / 8 + 64);
}

void gemm_bf16x3(const GemmArgs& g, double* planes_ws, size_t planes_ws_doubles,
                 hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  const int64_t ra = g.ta ? g.K : g.M, rb = g.tb ? g.N : g.K;
  const int64_t na = span(ra, g.lda, g.batch, g.sA), nb = span(rb, g.ldb, g.batch, g.sB);
  (void)planes_ws_doubles;
  uint16_t* w = reinterpret_cast<uint16_t*>(planes_ws);
  Planes pl;
  uint16_t* pa[3] = {w, w + na, w + 2 * na};
  uint16_t* pbp[3] = {w + 3 * na, w + 3 * na + nb, w + 3 * na + 2 * nb};
  auto blocks = [](int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b > 1048576 ? 1048576 : (b < 1 ? 1 : b));
  };
  hipLaunchKernelGGL(split3_kernel, dim3(blocks(na)), dim3(256), 0, st, g.A, na, pa[0], pa[1],
                     pa[2]);
  hipLaunchKernelGGL(split3_kernel, dim3(blocks(nb)), dim3(256), 0, st, g.B, nb, pbp[0], pbp[1],
                     pbp[2]);
  for (int p = 0; p < 3; ++p) {
    pl.a[p] = pa[p];
    pl.b[p] = pbp[p];
  }
  BArgs ba{g, pl};
  dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM), (unsigned)g.batch);
  hipLaunchKernelGGL(gemm_bf16x3_kernel, grid, dim3(NT), 0, st, ba);
}

}  // namespace tatrg
