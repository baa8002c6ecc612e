// Memory-bound helper kernels: Philox Gaussian sketches, leg permutations, scaling, copies.
#include "common.h"

namespace tatrg {

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(int64_t n, int tpb = TPB) {
  int64_t b = (n + tpb - 1) / tpb;
  if (b < 1) b = 1;
  if (b > 1048576) b = 1048576;
  return (unsigned)b;
}

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round
// (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2, c = (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is
// advanced by the Weyl increments between rounds.
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Element pair p = e >> 1 of stream (seed, step, site): counter (lo(p), hi(p), step, site),
// key (lo(seed), hi(seed)); two 53-bit uniforms, Box-Muller (cos for even e, sin for odd e).
__global__ void philox_gauss_kernel(double* out, int64_t rows, int64_t cols, int64_t ld,
                                    int transposed, int64_t row_split, uint32_t k0,
                                    uint32_t k1, uint32_t step, uint32_t site) {
  const int64_t total = rows * cols;
  const int64_t npairs = (total + 1) >> 1;
  for (int64_t pr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pr < npairs;
       pr += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)pr, (uint32_t)((uint64_t)pr >> 32), step, site};
    philox10(c, k0, k1);
    const double two26 = 67108864.0;
    const double scale = 1.1102230246251565e-16;  // 2^-53
    const double u1 = ((double)(c[0] >> 5) * two26 + (double)(c[1] >> 6) + 1.0) * scale;
    const double u2 = ((double)(c[2] >> 5) * two26 + (double)(c[3] >> 6)) * scale;
    const double r = sqrt(-2.0 * log(u1));
    const double th = 6.283185307179586 * u2;
    const double g[2] = {r * cos(th), r * sin(th)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t e = 2 * pr + h;
      if (e < total) {
        int64_t i = e / cols;
        const int64_t j = e - i * cols;
        if (row_split > 0) i = (i % row_split) * (rows / row_split) + i / row_split;
        if (transposed)
          out[j * ld + i] = g[h];
        else
          out[i * ld + j] = g[h];
      }
    }
  }
}

// Raw output words of the generator for counter pairs pair0 .. pair0 + npairs - 1 (the same
// counters and key the sketches use): out[4 t + w] = word w of pair pair0 + t.
__global__ void philox_words_kernel(uint32_t* out, int64_t pair0, int64_t npairs, uint32_t k0,
                                    uint32_t k1, uint32_t step, uint32_t site) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npairs;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pr = pair0 + t;
    uint32_t c[4] = {(uint32_t)pr, (uint32_t)((uint64_t)pr >> 32), step, site};
    philox10(c, k0, k1);
    uint4 v;
    v.x = c[0];
    v.y = c[1];
    v.z = c[2];
    v.w = c[3];
    reinterpret_cast<uint4*>(out)[t] = v;
  }
}

struct PermArgs {
  int rank;
  int64_t out_dims[6];
  int64_t in_stride_for_out[6];  // input stride of output dimension k
};

__global__ void permute_kernel(const double* __restrict__ in, double* __restrict__ out,
                               PermArgs pa, int64_t total) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, off = 0;
    for (int k = pa.rank - 1; k >= 0; --k) {
      const int64_t d = pa.out_dims[k];
      const int64_t q = rem / d;
      off += (rem - q * d) * pa.in_stride_for_out[k];
      rem = q;
    }
    out[idx] = in[off];
  }
}

// A permutation that keeps the innermost leg (its length a multiple of 4): each thread moves
// four consecutive doubles of it, so the index arithmetic is paid once per 32 bytes.
__global__ void permute_vec4_kernel(const double* __restrict__ in, double* __restrict__ out,
                                   PermArgs pa, int64_t total4) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total4;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx * 4, off = 0;
    for (int k = pa.rank - 1; k >= 0; --k) {
      const int64_t d = pa.out_dims[k];
      const int64_t q = rem / d;
      off += (rem - q * d) * pa.in_stride_for_out[k];
      rem = q;
    }
    const double2 v0 = *reinterpret_cast<const double2*>(in + off);
    const double2 v1 = *reinterpret_cast<const double2*>(in + off + 2);
    *reinterpret_cast<double2*>(out + idx * 4) = v0;
    *reinterpret_cast<double2*>(out + idx * 4 + 2) = v1;
  }
}

// A permutation whose output-innermost leg is not the input-innermost leg, as 32 x 32 tiles
// of those two legs staged through LDS: reads run along the input-innermost leg and writes
// along the output-innermost leg, so both are contiguous.  Work-group w takes tiles w, w + G,
// ...; tile index = (tile along la) + ta (tile along lb + tb (the other output legs, last
// fastest)).
struct TileArgs {
  int rank;
  int la, lb;  // output positions: la = rank - 1, lb = the leg that is innermost in the input
  int64_t out_dims[6], in_stride_for_out[6], out_stride[6];
  int64_t ta, tb;  // tiles along la and lb
};

__global__ __launch_bounds__(256) void permute_tiled_kernel(const double* __restrict__ in,
                                                            double* __restrict__ out,
                                                            TileArgs t, int64_t ntiles) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t sa_in = t.in_stride_for_out[t.la], sb_out = t.out_stride[t.lb];
  for (int64_t w = blockIdx.x; w < ntiles; w += gridDim.x) {
    int64_t rem = w;
    const int64_t ia = rem % t.ta;
    rem /= t.ta;
    const int64_t ib = rem % t.tb;
    rem /= t.tb;
    int64_t in_base = 0, out_base = 0;
    for (int k = t.rank - 1; k >= 0; --k) {
      if (k == t.la || k == t.lb) continue;
      const int64_t d = t.out_dims[k];
      const int64_t q = rem / d, i = rem - q * d;
      in_base += i * t.in_stride_for_out[k];
      out_base += i * t.out_stride[k];
      rem = q;
    }
    const int64_t a0 = ia * 32, b0 = ib * 32;
    const int na = (int)(t.out_dims[t.la] - a0 < 32 ? t.out_dims[t.la] - a0 : 32);
    const int nb = (int)(t.out_dims[t.lb] - b0 < 32 ? t.out_dims[t.lb] - b0 : 32);
    __syncthreads();  // the previous tile has been written out
    if (tx < nb) {
      // the four loads of a thread are in flight together (na <= 32 = 4 x 8)
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = ty + 8 * q;
        v[q] = (a < na) ? in[in_base + (a0 + a) * sa_in + b0 + tx] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (ty + 8 * q < na) tile[ty + 8 * q][tx] = v[q];
    }
    __syncthreads();
    if (tx < na)
      for (int b = ty; b < nb; b += 8) out[out_base + (b0 + b) * sb_out + a0 + tx] = tile[tx][b];
  }
}

__global__ void scale_cols_kernel(double* x, const double* s, int64_t rows, int64_t cols,
                                  int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / cols, j = idx - (idx / cols) * cols;
    x[i * ld + j] *= s[j];
  }
}

// y = x diag(s) for a rows x cols row-major x (one pass instead of a copy and a scaling).
__global__ void copy_scale_cols_kernel(double* __restrict__ y, const double* __restrict__ x,
                                       const double* __restrict__ s, int64_t rows,
                                       int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    y[idx] = x[idx] * s[idx % cols];
}

// U[b] <- U[b] diag(sqrt(S[b])) for `batch` n x n matrices (strides n^2 and n).
__global__ void sqrt_scale_cols_kernel(double* U, const double* S, int n, int batch) {
  const int64_t total = (int64_t)batch * n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / ((int64_t)n * n);
    const int j = (int)(idx % n);
    U[idx] *= sqrt(S[b * n + j]);
  }
}

__global__ void copy_kernel(double* y, const double* x, int64_t n) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x)
    y[idx] = x[idx];
}

__global__ void zero_kernel(double* y, int64_t n) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x)
    y[idx] = 0.0;
}

__global__ void identity_kernel(double* x, int n, int64_t ld) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx - (idx / n) * n;
    x[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
}

__global__ void symmetrize_kernel(double* A, int n, int batch) {
  const int64_t per = (int64_t)n * n;
  const int64_t total = per * batch;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / per, r = idx - b * per;
    const int64_t i = r / n, j = r - (r / n) * n;
    if (j > i) {
      double* M = A + b * per;
      const double v = 0.5 * (M[i * n + j] + M[j * n + i]);
      M[i * n + j] = v;
      M[j * n + i] = v;
    }
  }
}

__global__ void transpose_batched_kernel(const double* in, double* out, int rows, int cols,
                                         int batch) {
  const int64_t per = (int64_t)rows * cols;
  const int64_t total = per * batch;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / per, r = idx - b * per;
    const int64_t i = r / cols, j = r - (r / cols) * cols;
    out[b * per + j * rows + i] = in[idx];
  }
}

// Order parameter X = (Tr A)^2 / Tr A^2 of T = sum_g Phi[f, g] Psi[b, g], with
// A_kl = sum over the three other directions of T with forward and backward legs identified
// (Section 3, the order parameter of the transition).  With the open leg in slot j, Phi is
// [pre][k][post] (pre = chi^j, post = chi^(4-j), gamma included) and
// A_kl = sum_{p, q} Phi[p][k][q] Psi[p][l][q].
constexpr int OP_QC = 32;    // trailing-leg chunk staged in LDS
constexpr int OP_MAXK = 16;  // outputs per thread: l = tid % chi, k = tid / chi + (256 / chi) i

// Work-group g sums the (p, q-chunk) units g, g + G, ... into part[g][k][l].
__global__ __launch_bounds__(TPB) void order_param_partial_kernel(
    const double* __restrict__ phi, const double* __restrict__ psi, int chi, int64_t pre,
    int64_t post, double* __restrict__ part) {
  __shared__ double sa[64][OP_QC + 1], sb[64][OP_QC + 1];
  const int tid = threadIdx.x;
  const int kgn = TPB / chi, l = tid % chi, kg = tid / chi;
  const bool act = kg < kgn;
  double acc[OP_MAXK];
#pragma unroll
  for (int i = 0; i < OP_MAXK; ++i) acc[i] = 0.0;
  const int64_t nq = (post + OP_QC - 1) / OP_QC, units = pre * nq;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const int64_t p = u / nq, q0 = (u - p * nq) * OP_QC;
    const int64_t qn = post - q0 < OP_QC ? post - q0 : OP_QC;
    __syncthreads();
    for (int e = tid; e < chi * OP_QC; e += TPB) {
      const int k = e / OP_QC, q = e - (e / OP_QC) * OP_QC;
      const int64_t off = (p * chi + k) * post + q0 + q;
      sa[k][q] = q < qn ? phi[off] : 0.0;
      sb[k][q] = q < qn ? psi[off] : 0.0;
    }
    __syncthreads();
    if (act) {
      for (int q = 0; q < OP_QC; ++q) {
        const double bv = sb[l][q];
#pragma unroll
        for (int i = 0; i < OP_MAXK; ++i) {
          const int k = kg + kgn * i;
          if (k < chi) acc[i] += sa[k][q] * bv;
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < OP_MAXK; ++i) {
      const int k = kg + kgn * i;
      if (k < chi) part[(int64_t)blockIdx.x * chi * chi + k * chi + l] = acc[i];
    }
  }
}

// One work-group: A = sum of the parts in order, then Tr A, Tr A^2 and X.
__global__ __launch_bounds__(TPB) void order_param_final_kernel(const double* __restrict__ part,
                                                                int nparts, int chi,
                                                                double* __restrict__ out) {
  __shared__ double a[64 * 64];
  __shared__ double red[TPB];
  const int tid = threadIdx.x, n = chi * chi;
  for (int e = tid; e < n; e += TPB) {
    double s = 0.0;
    for (int g = 0; g < nparts; ++g) s += part[(int64_t)g * n + e];
    a[e] = s;
  }
  __syncthreads();
  double t2 = 0.0;
  for (int e = tid; e < n; e += TPB) {
    const int k = e / chi, l = e - (e / chi) * chi;
    t2 += a[k * chi + l] * a[l * chi + k];
  }
  red[tid] = t2;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    double tr = 0.0;
    for (int k = 0; k < chi; ++k) tr += a[k * chi + k];
    out[0] = tr * tr / red[0];
  }
}

}  // namespace

void philox_gaussian(double* out, int64_t rows, int64_t cols, int64_t ld, bool transposed,
                     uint64_t seed, uint32_t step, uint32_t site, hipStream_t st,
                     int64_t row_split, int max_blocks) {
  const int64_t npairs = (rows * cols + 1) / 2;
  if (row_split > 0 && rows % row_split != 0) row_split = 0;  // callers pass a divisor
  unsigned blocks = grid_for(npairs);
  if (max_blocks > 0 && blocks > (unsigned)max_blocks) blocks = (unsigned)max_blocks;
  hipLaunchKernelGGL(philox_gauss_kernel, dim3(blocks), dim3(TPB), 0, st, out, rows,
                     cols, ld, transposed ? 1 : 0, row_split, (uint32_t)seed,
                     (uint32_t)(seed >> 32), step, site);
}

void philox_words(uint32_t* out, int64_t pair0, int64_t npairs, uint64_t seed, uint32_t step,
                  uint32_t site, hipStream_t st) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(philox_words_kernel, dim3(grid_for(npairs)), dim3(TPB), 0, st, out, pair0,
                     npairs, (uint32_t)seed, (uint32_t)(seed >> 32), step, site);
}

void permute(const double* in, double* out, int rank, const int64_t* dims, const int* perm,
             hipStream_t st) {
  PermArgs pa;
  pa.rank = rank;
  int64_t in_stride[6];
  int64_t s = 1;
  for (int k = rank - 1; k >= 0; --k) {
    in_stride[k] = s;
    s *= dims[k];
  }
  int lb = rank - 1;
  for (int k = 0; k < rank; ++k) {
    pa.out_dims[k] = dims[perm[k]];
    pa.in_stride_for_out[k] = in_stride[perm[k]];
    if (perm[k] == rank - 1) lb = k;
  }
  const int la = rank - 1;
  if (lb != la && pa.out_dims[la] >= 8 && pa.out_dims[lb] >= 8) {
    TileArgs t;
    t.rank = rank;
    t.la = la;
    t.lb = lb;
    int64_t os = 1;
    for (int k = rank - 1; k >= 0; --k) {
      t.out_dims[k] = pa.out_dims[k];
      t.in_stride_for_out[k] = pa.in_stride_for_out[k];
      t.out_stride[k] = os;
      os *= pa.out_dims[k];
    }
    t.ta = (pa.out_dims[la] + 31) / 32;
    t.tb = (pa.out_dims[lb] + 31) / 32;
    const int64_t ntiles = s / (pa.out_dims[la] * pa.out_dims[lb]) * t.ta * t.tb;
    const int64_t g = ntiles < 1048576 ? ntiles : 1048576;
    hipLaunchKernelGGL(permute_tiled_kernel, dim3((unsigned)g), dim3(256), 0, st, in, out, t,
                       ntiles);
    return;
  }
  if (lb == la && pa.out_dims[la] % 4 == 0 && ((uintptr_t)in % 16) == 0 &&
      ((uintptr_t)out % 16) == 0) {
    hipLaunchKernelGGL(permute_vec4_kernel, dim3(grid_for(s / 4)), dim3(TPB), 0, st, in, out,
                       pa, s / 4);
    return;
  }
  hipLaunchKernelGGL(permute_kernel, dim3(grid_for(s)), dim3(TPB), 0, st, in, out, pa, s);
}

void copy_scale_cols(double* y, const double* x, const double* s, int64_t rows, int64_t cols,
                     hipStream_t st) {
  hipLaunchKernelGGL(copy_scale_cols_kernel, dim3(grid_for(rows * cols)), dim3(TPB), 0, st, y, x,
                     s, rows, cols);
}

void scale_cols(double* x, const double* s, int64_t rows, int64_t cols, int64_t ld,
                hipStream_t st) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(rows * cols)), dim3(TPB), 0, st, x, s,
                     rows, cols, ld);
}

void psd_factor(const double* P, double* L, double* S, double* V, int n, int batch,
                hipStream_t st) {
  jacobi_svd(P, L, S, V, n, batch, st);
  const int64_t total = (int64_t)batch * n * n;
  hipLaunchKernelGGL(sqrt_scale_cols_kernel, dim3(grid_for(total)), dim3(TPB), 0, st, L, S, n,
                     batch);
}

void copy(double* y, const double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(TPB), 0, st, y, x, n);
}

void zero(double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(TPB), 0, st, x, n);
}

void identity(double* x, int n, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(identity_kernel, dim3(grid_for((int64_t)n * n)), dim3(TPB), 0, st, x, n,
                     ld);
}

void symmetrize(double* A, int n, int batch, hipStream_t st) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(grid_for((int64_t)n * n * batch)), dim3(TPB), 0,
                     st, A, n, batch);
}

void transpose_batched(const double* in, double* out, int rows, int cols, int batch,
                       hipStream_t st) {
  hipLaunchKernelGGL(transpose_batched_kernel, dim3(grid_for((int64_t)rows * cols * batch)),
                     dim3(TPB), 0, st, in, out, rows, cols, batch);
}

size_t order_parameter_ws_doubles(int chi) { return (size_t)OP_PARTS * chi * chi; }

void order_parameter(const double* phi, const double* psi, int chi, int open_slot,
                     double* part, double* out, hipStream_t st) {
  int64_t pre = 1, post = 1;
  for (int j = 0; j < open_slot; ++j) pre *= chi;
  for (int j = open_slot + 1; j < 5; ++j) post *= chi;  // legs after the open one, and gamma
  hipLaunchKernelGGL(order_param_partial_kernel, dim3(OP_PARTS), dim3(TPB), 0, st, phi, psi,
                     chi, pre, post, part);
  hipLaunchKernelGGL(order_param_final_kernel, dim3(1), dim3(TPB), 0, st, part, OP_PARTS, chi,
                     out);
}

}  // namespace tatrg
