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
// [N][Kp], Kp = K rounded up to 32 and zero padded -- transposing through an LDS tile where the
// float64 operand is stored the other way, so the GEMM moves 16-byte vectors of 8 bf16 along
// K for both operands and an MFMA fragment is one 16-byte LDS read.  Tiling: 512 threads
// (8 wave64 in a 2 x 4 grid), 128 x 128 tile of C, 64 x 32 per wave as 4 x 2 MFMA blocks; K
// advances by 32 through two LDS stages filled by direct global-to-LDS loads, so the loads of
// the next stage overlap the products of the current one (a third stage measured 2-3 %
// slower on both contraction shapes, and two leave the LDS for staging C's planes); each
// plane's fragments are read once and serve every product they enter.  C is written either
// in float64 or, for a GEMM whose product is the next GEMM's op(B), directly as that
// operand's bf16 planes (Bf16PlanesOut), so it is never stored in float64 and split again.  Work-groups are ordered so
// that the tiles sharing a B tile run on one XCD.
#include <atomic>

#include "common.h"

namespace tatrg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 128, BK = 32, NT = 512;
constexpr int NSTAGE = 2;                    // LDS stages: 2 x 48 KB
constexpr int STAGE_UNITS = 2 * 3 * 8 * 64;  // 16-byte units per stage
// s_waitcnt immediate (vmcnt in bits 3:0 and 15:14, expcnt and lgkmcnt left at their
// maxima): wait until no vector-memory operation is outstanding
constexpr unsigned WAIT_VM0 = 0x0F70u;
typedef __attribute__((address_space(3))) void* lds_ptr;
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
  // four consecutive k per thread: one 8-byte store per plane (Kp is a multiple of 4 and the
  // tile starts at a multiple of 64, so a group of four is either wholly inside or outside)
  for (int idx = tid; idx < ST * ST / 4; idx += 256) {
    const int rr = idx / (ST / 4), kk = 4 * (idx % (ST / 4));
    const int64_t r = r0 + rr, k = k0 + kk;
    if (r < R && k < Kp) {
      uint16_t a[4], c[4], e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double v = tile[rr][kk + q];
        a[q] = bf16_rne((float)v);
        const double r1 = v - bf16_to_double(a[q]);
        c[q] = bf16_rne((float)r1);
        const double r2 = r1 - bf16_to_double(c[q]);
        e[q] = bf16_rne((float)r2);
      }
      const int64_t o = (b * R + r) * Kp + k;
      *reinterpret_cast<ushort4*>(p0 + o) = make_ushort4(a[0], a[1], a[2], a[3]);
      *reinterpret_cast<ushort4*>(p1 + o) = make_ushort4(c[0], c[1], c[2], c[3]);
      *reinterpret_cast<ushort4*>(p2 + o) = make_ushort4(e[0], e[1], e[2], e[3]);
    }
  }
}

struct BArgs {
  GemmArgs g;
  const uint16_t* a[3];  // [batchA][M][Kp]
  const uint16_t* b[3];  // [batchB][N][Kp]
  int64_t Kp, sAp, sBp;  // plane batch strides (0 for an operand shared by the batch)
  int tiles_m, tiles_n;
  int group_m;           // rows of tiles per group of the tile order (0: M fastest throughout)
  uint16_t* cp[3];       // C as planes (Bf16PlanesOut) when cp[0] is set
  int64_t cR2, cC1, cC2, cKp, cstride;
};

// Zero offsets [k0, Kp) of `rows` plane rows of every batch entry (the K padding of planes
// written by a Bf16PlanesOut epilogue).
__global__ void zero_plane_tail_kernel(uint16_t* p0, uint16_t* p1, uint16_t* p2, int64_t rows,
                                       int64_t k0, int64_t Kp, int64_t stride) {
  const int64_t w = Kp - k0, n = rows * w;
  const int64_t b = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = b * stride + (i / w) * Kp + k0 + i % w;
    p0[o] = 0;
    p1[o] = 0;
    p2[o] = 0;
  }
}

// One 128 x 128 tile of C per work-group.  Operand tiles move from global memory straight
// into LDS (global_load_lds_dwordx4, no staging registers) through NSTAGE = 2 stages of
// BK = 32: the loads for step kt + 1 are in flight while stage kt is multiplied.  A stage is
// 48 blocks of 1 KB (2 operands x 3 planes x 8 row blocks of 16 rows x 32 k); lane l of the
// wave that fills a block writes unit l = 4 r + (c ^ (r / 4 % 4)) with the 16-byte chunk c
// of row r, a swizzle under which the 16 lanes of each fragment read hit distinct banks.
// NPROD = 6 is the engine (all products with i + j <= 2); NPROD = 3 keeps only i + j <= 1,
// an ablation of the split's accuracy (about 2^-16 of |A||B| instead of 2^-24).
template <int NPROD>
__global__ __launch_bounds__(NT, 1) void gemm_bf16x3_kernel(BArgs ba) {
  const GemmArgs& g = ba.g;
  __shared__ __attribute__((aligned(1024))) uint4 lds[NSTAGE][STAGE_UNITS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int64_t b = blockIdx.z;
  // XCD-aware order: work-group w runs on XCD w % 8; tiles are numbered so that each XCD
  // gets a contiguous range.  Within it the tiles run M fastest (those that share a B tile),
  // in groups of group_m rows of tiles when there are many: the ~32 tiles an XCD runs at once
  // then share A tiles as well as B tiles in its L2 (6 x 5 rather than 24 x 1 for P = E.FM4,
  // measured 5 % faster there).
  const int nt = ba.tiles_m * ba.tiles_n;
  int w = blockIdx.x;
  if (nt % 8 == 0) w = (w % 8) * (nt / 8) + w / 8;
  int tm, tn;
  if (ba.group_m > 0) {
    const int per = ba.group_m * ba.tiles_n, grp = w / per, fm = grp * ba.group_m;
    const int gs = min(ba.tiles_m - fm, ba.group_m), r = w - grp * per;
    tm = fm + r % gs;
    tn = r / gs;
  } else {
    tm = w % ba.tiles_m;
    tn = w / ba.tiles_m;
  }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = g.M, N = g.N, Kp = ba.Kp;

  // Source of this lane's unit in each of the wave's six blocks (block wave + 8 i).  Rows past
  // M or N read the last valid row: they only feed rows and columns of C that are not stored.
  const int ur = lane >> 2, uc = (lane & 3) ^ ((ur >> 2) & 3);
  const uint16_t* src[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int bi = wave + 8 * i;
    const int op = bi / 24, p = (bi % 24) / 8, rb = bi % 8;
    const int64_t lim = (op == 0 ? M : N) - 1;
    int64_t row = (op == 0 ? m0 : n0) + rb * 16 + ur;
    if (row > lim) row = lim;
    src[i] = (op == 0 ? ba.a[p] + b * ba.sAp : ba.b[p] + b * ba.sBp) + row * Kp + uc * 8;
  }
  auto issue = [&](int stage, int64_t k0) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
      __builtin_amdgcn_global_load_lds((const void*)(src[i] + k0),
                                       (lds_ptr)&lds[stage][(wave + 8 * i) * 64], 16, 0, 0);
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

  const int64_t nk = Kp / BK;
  if (nk > 0) issue(0, 0);
  // fragment unit of this lane: row l % 16 of a block, 16-byte chunk l / 16
  const int rl = lane & 15, fpos = rl * 4 + ((lane >> 4) ^ ((rl >> 2) & 3));
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    // This wave's loads of stage kt have landed; the barrier makes every wave's blocks
    // visible and ends all reads of stage kt - 1, whose buffer the loads of step kt + 1 then
    // refill.
    __builtin_amdgcn_s_waitcnt(WAIT_VM0);
    __builtin_amdgcn_s_barrier();
    if (kt + 1 < nk) issue((int)((kt + 1) & 1), (kt + 1) * BK);
    bf16x8 fa[3][4], fb[3][2];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        fa[p][t] = *reinterpret_cast<const bf16x8*>(&lds[cur][(p * 8 + wm * 4 + t) * 64 + fpos]);
#pragma unroll
      for (int t = 0; t < 2; ++t)
        fb[p][t] =
            *reinterpret_cast<const bf16x8*>(&lds[cur][((3 + p) * 8 + wn * 2 + t) * 64 + fpos]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        hi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[0][j], hi[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[1][j], lo[i][j], 0, 0, 0);
        lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[0][j], lo[i][j], 0, 0, 0);
        if (NPROD == 6) {
          lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[1][j], lo[i][j], 0, 0, 0);
          lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[2][j], lo[i][j], 0, 0, 0);
          lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[2][i], fb[0][j], lo[i][j], 0, 0, 0);
        }
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
  }

  // D fragment of v_mfma_f32_16x16x32_bf16: lane l, element v holds row 4*(l/16) + v,
  // column l%16 of the 16 x 16 block.
  if (ba.cp[0]) {
    // C as planes, staged through LDS (the two operand stages are free once every wave has
    // done its last products): each wave writes its fragments as [plane][row][col] bf16,
    // then the work-group stores 16-byte chunks of 8 consecutive columns, which for a chunk
    // inside one c1 group are 8 consecutive plane elements.
    uint16_t* st16 = reinterpret_cast<uint16_t*>(&lds[0][0]);  // [3][BM][BN]
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = wm * 64 + i * 16 + 4 * (lane >> 4) + v, cc = wn * 32 + j * 16 + rl;
          const double x = g.alpha * dacc[i][j][v];
          const uint16_t h0 = bf16_rne((float)x);
          const double x1 = x - bf16_to_double(h0);
          const uint16_t h1 = bf16_rne((float)x1);
          const double x2 = x1 - bf16_to_double(h1);
          st16[(0 * BM + rr) * BN + cc] = h0;
          st16[(1 * BM + rr) * BN + cc] = h1;
          st16[(2 * BM + rr) * BN + cc] = bf16_rne((float)x2);
        }
    __syncthreads();
    const int64_t base = b * ba.cstride;
    for (int q = tid; q < BM * BN / 8; q += NT) {
      const int rr = q / (BN / 8), cc = 8 * (q % (BN / 8));
      const int64_t row = m0 + rr, col = n0 + cc;
      if (row >= M) continue;
      const int64_t r1 = row / ba.cR2, r2 = row - r1 * ba.cR2;
      const int64_t c1 = col / ba.cC2, c2 = col - c1 * ba.cC2;
      const int64_t o = base + (r1 * ba.cC1 + c1) * ba.cKp + r2 * ba.cC2 + c2;
      if (col + 8 <= N && c2 + 8 <= ba.cC2 && (o & 7) == 0) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
          *reinterpret_cast<uint4*>(ba.cp[p] + o) =
              *reinterpret_cast<const uint4*>(&st16[(p * BM + rr) * BN + cc]);
      } else {
        for (int t = 0; t < 8 && col + t < N; ++t) {
          const int64_t ct1 = (col + t) / ba.cC2, ct2 = (col + t) - ct1 * ba.cC2;
          const int64_t ot = base + (r1 * ba.cC1 + ct1) * ba.cKp + r2 * ba.cC2 + ct2;
#pragma unroll
          for (int p = 0; p < 3; ++p) ba.cp[p][ot] = st16[(p * BM + rr) * BN + cc + t];
        }
      }
    }
    return;
  }
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

// The planes of the contraction's FM4 operand straight from tmp[(i4a k4)][(a kX g)] (leg
// extents c, c, c, L, c): plane row n = (g, k4, kX), column k = (i4a, a), i.e. FM4 with kX
// innermost, transposed to the k-contiguous layout the split GEMM reads, without storing FM4
// in float64.  One work-group per (k4, kX), group of FM4_I consecutive i4a and 32 x 32 tile of
// (a, g), transposed through LDS: the reads run along g, and each plane row takes FM4_I
// consecutive runs of a, contiguous when the a tile is whole.  Every value is split exactly as
// split3_kernel splits it.
constexpr int FM4_I = 4;

__global__ __launch_bounds__(256) void fm4_planes_kernel(const double* __restrict__ tmp, int c,
                                                         int L, int64_t Kp,
                                                         uint16_t* __restrict__ p0,
                                                         uint16_t* __restrict__ p1,
                                                         uint16_t* __restrict__ p2) {
  __shared__ double tile[FM4_I][32][33];  // [i4a - i0][a][g]
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;  // (i4a group, k4, kX)
  const int kX = (int)(blk % L);
  const int k4 = (int)((blk / L) % c);
  const int i0 = FM4_I * (int)(blk / ((int64_t)L * c));
  const int a0 = 32 * (int)blockIdx.y, g0 = 32 * (int)blockIdx.z;
  // tmp row (i4a k4), column (a kX g): contiguous in g; all of a thread's loads in flight
  // before the LDS writes
  double v[FM4_I * 32 * 32 / 256];
#pragma unroll
  for (int q = 0; q < FM4_I * 4; ++q) {
    const int idx = tid + 256 * q, ii = idx / 1024, aa = (idx / 32) % 32, gg = idx % 32;
    const int i4a = i0 + ii, a = a0 + aa, g = g0 + gg;
    v[q] = (i4a < c && a < c && g < c)
               ? tmp[(((int64_t)i4a * c + k4) * c + a) * ((int64_t)L * c) + (int64_t)kX * c + g]
               : 0.0;
  }
#pragma unroll
  for (int q = 0; q < FM4_I * 4; ++q) {
    const int idx = tid + 256 * q;
    tile[idx / 1024][(idx / 32) % 32][idx % 32] = v[q];
  }
  __syncthreads();
  // plane row (g k4 kX), columns i4a c + a: consecutive threads take consecutive a, then i4a
#pragma unroll 4
  for (int q = 0; q < FM4_I * 4; ++q) {
    const int idx = tid + 256 * q, gg = idx / (32 * FM4_I), ii = (idx / 32) % FM4_I,
              aa = idx % 32;
    const int i4a = i0 + ii, a = a0 + aa, g = g0 + gg;
    if (i4a < c && a < c && g < c) {
      const double x = tile[ii][aa][gg];
      const uint16_t h0 = bf16_rne((float)x);
      const double r1 = x - bf16_to_double(h0);
      const uint16_t h1 = bf16_rne((float)r1);
      const double r2 = r1 - bf16_to_double(h1);
      const int64_t row = ((int64_t)g * c + k4) * L + kX;
      const int64_t o = row * Kp + (int64_t)i4a * c + a;
      p0[o] = h0;
      p1[o] = h1;
      p2[o] = bf16_rne((float)r2);
    }
  }
}

}  // namespace

// Products per split GEMM (6; 3 for the accuracy ablation), process-wide.
static std::atomic<int> g_split_products{6};

int set_split_products(int n) {
  if (n != 3 && n != 6) return -1;
  return g_split_products.exchange(n);
}

int64_t bf16x3_kpad(int64_t K) { return ((K + BK - 1) / BK) * BK; }

bool fm4_planes(const double* tmp, int c, int L, uint16_t* planes, int64_t cap,
                hipStream_t st) {
  const int64_t n2 = (int64_t)c * c, Kp = bf16x3_kpad(n2), rows = (int64_t)L * n2;
  if (!tmp || !planes || c < 1 || L < 1 || 3 * rows * Kp > cap) return false;
  uint16_t* p0 = planes;
  uint16_t* p1 = planes + rows * Kp;
  uint16_t* p2 = planes + 2 * rows * Kp;
  if (Kp > n2) {
    const int64_t n = rows * (Kp - n2);
    dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 4096), 1u);
    hipLaunchKernelGGL(zero_plane_tail_kernel, grid, dim3(256), 0, st, p0, p1, p2, rows, n2, Kp,
                       (int64_t)0);
  }
  dim3 grid((unsigned)((int64_t)((c + FM4_I - 1) / FM4_I) * c * L), (unsigned)((c + 31) / 32),
            (unsigned)((c + 31) / 32));
  hipLaunchKernelGGL(fm4_planes_kernel, grid, dim3(256), 0, st, tmp, c, L, Kp, p0, p1, p2);
  return true;
}

size_t gemm_bf16x3_ws_doubles(const GemmArgs& g, bool b_given) {
  const int64_t Kp = bf16x3_kpad(g.K);
  const int64_t na = plane_batches(g, true) * g.M * Kp;
  const int64_t nb = b_given ? 0 : plane_batches(g, false) * g.N * Kp;
  return (size_t)((3 * (na + nb) * 2 + 7) / 8 + 64);
}

bool gemm_bf16x3(const GemmArgs& g, double* planes_ws, size_t planes_ws_doubles,
                 hipStream_t st, hipEvent_t ev_after_split, const Bf16PlanesIn* b_in,
                 const Bf16PlanesOut* c_out, int group_m) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return true;
  // the planes of the split operands must fit the workspace: launch nothing otherwise
  if (!planes_ws || planes_ws_doubles < gemm_bf16x3_ws_doubles(g, b_in != nullptr))
    return false;
  const int64_t Kp = bf16x3_kpad(g.K);
  if (b_in && (!b_in->p[0] || !b_in->p[1] || !b_in->p[2] || b_in->stride < 0 ||
               (g.batch > 1 && b_in->stride > 0 && b_in->stride < g.N * Kp)))
    return false;
  if (c_out) {
    const Bf16PlanesOut& o = *c_out;
    if (!o.p[0] || !o.p[1] || !o.p[2] || g.beta != 0.0 || o.R2 < 1 || o.C2 < 1 ||
        g.M % o.R2 != 0 || g.N % o.C2 != 0 || g.N / o.C2 > o.C1 || o.R2 * o.C2 > o.Kp ||
        o.Kp % 8 != 0 || o.stride < 0)
      return false;
    // the last element of every batch entry's last plane row
    const int64_t last = (g.batch - 1) * o.stride + ((g.M / o.R2 - 1) * o.C1 + o.C1 - 1) * o.Kp +
                         o.Kp;
    if (last > o.cap || (g.batch > 1 && o.stride < (g.M / o.R2) * o.C1 * o.Kp)) return false;
  }
  const int64_t ba_n = plane_batches(g, true), bb_n = plane_batches(g, false);
  const int64_t na = ba_n * g.M * Kp, nb = b_in ? 0 : bb_n * g.N * Kp;
  // plane starts stay 16-byte aligned: na and nb are multiples of 8 elements
  uint16_t* w = reinterpret_cast<uint16_t*>(planes_ws);
  BArgs ba;
  ba.g = g;
  for (int p = 0; p < 3; ++p) {
    ba.a[p] = w + p * na;
    ba.b[p] = b_in ? b_in->p[p] : w + 3 * na + p * nb;
    ba.cp[p] = c_out ? c_out->p[p] : nullptr;
  }
  ba.Kp = Kp;
  ba.sAp = (ba_n == 1) ? 0 : g.M * Kp;
  ba.sBp = b_in ? b_in->stride : (bb_n == 1) ? 0 : g.N * Kp;
  ba.tiles_m = (int)((g.M + BM - 1) / BM);
  ba.tiles_n = (int)((g.N + BN - 1) / BN);
  ba.group_m = group_m >= 0 ? group_m : (ba.tiles_m >= 12 ? 6 : 0);
  ba.cR2 = c_out ? c_out->R2 : 1;
  ba.cC1 = c_out ? c_out->C1 : 1;
  ba.cC2 = c_out ? c_out->C2 : 1;
  ba.cKp = c_out ? c_out->Kp : 0;
  ba.cstride = c_out ? c_out->stride : 0;
  if (c_out && c_out->R2 * c_out->C2 < c_out->Kp) {
    const int64_t rows = (g.M / c_out->R2) * c_out->C1;
    const int64_t n = rows * (c_out->Kp - c_out->R2 * c_out->C2);
    dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 4096), (unsigned)g.batch);
    hipLaunchKernelGGL(zero_plane_tail_kernel, grid, dim3(256), 0, st, c_out->p[0],
                       c_out->p[1], c_out->p[2], rows, c_out->R2 * c_out->C2, c_out->Kp,
                       c_out->stride);
  }
  // op(A) is M x K, stored K x M when ta.  op(B) is K x N and its planes are N x K, so the
  // float64 B is read transposed unless it is stored N x K (tb).
  {
    dim3 grid((unsigned)((Kp + ST - 1) / ST), (unsigned)((g.M + ST - 1) / ST), (unsigned)ba_n);
    hipLaunchKernelGGL(split3_kernel, grid, dim3(256), 0, st, g.A, g.M, g.K, g.lda, g.sA,
                       g.ta ? 1 : 0, Kp, w, w + na, w + 2 * na);
  }
  if (!b_in) {
    dim3 grid((unsigned)((Kp + ST - 1) / ST), (unsigned)((g.N + ST - 1) / ST), (unsigned)bb_n);
    hipLaunchKernelGGL(split3_kernel, grid, dim3(256), 0, st, g.B, g.N, g.K, g.ldb, g.sB,
                       g.tb ? 0 : 1, Kp, w + 3 * na, w + 3 * na + nb, w + 3 * na + 2 * nb);
  }
  if (ev_after_split) (void)hipEventRecord(ev_after_split, st);
  dim3 grid((unsigned)(ba.tiles_m * ba.tiles_n), 1u, (unsigned)g.batch);
  if (g_split_products == 3)
    hipLaunchKernelGGL(gemm_bf16x3_kernel<3>, grid, dim3(NT), 0, st, ba);
  else
    hipLaunchKernelGGL(gemm_bf16x3_kernel<6>, grid, dim3(NT), 0, st, ba);
  return true;
}

}  // namespace tatrg
