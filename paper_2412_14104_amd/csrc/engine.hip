// Triad-ATRG RG step engine and C ABI (include/tatrg.h).
//
// One call of tatrg_step runs the whole coarse-graining step of Section 2 of Sugimoto &
// Sasaki (arXiv:2412.14104) on the device, on the caller's stream, with no host
// synchronisation and no allocation: canonical form and normalisation (S0), bond swap by a
// randomized SVD of the cell middle (S1, Eq. (1)), oversampled isometries from the Grams of
// A X sigma and sigma Y D (S2, Eqs. (2)-(3)), triad tensors E..L (S3, Eqs. (4)-(11)),
// squeezers (S4, the squeezer cost function), the contraction of Eqs. (makeMG), (makeMH)
// (S5) and the slot rotation that brings the next direction to slot 1 (S6).
#include "common.h"
#include "../../include/tatrg.h"
#include "../../include/tatrg_testing.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <memory>
#include <mutex>
#include <vector>

namespace tatrg {

// Philox call sites (must match the method's definition of the sketches).
enum : uint32_t {
  SITE_SWAP = 0,
  SITE_ISO_A = 1, SITE_ISO_X = 2, SITE_ISO_Y = 3, SITE_ISO_D = 4,
  SITE_SQZ_2 = 5, SITE_SQZ_3 = 6, SITE_SQZ_4 = 7,
  SITE_PROBE_CANON = 8,
  SITE_PROBE_SQZ_2 = 9, SITE_PROBE_SQZ_3 = 10, SITE_PROBE_SQZ_4 = 11,
};
constexpr int N_PROBES = 8;
constexpr double TAU_NULL = 1e-11;
constexpr double TAU_DEG = 1e-6;
constexpr double SQZ_CUTOFF = 1e-10;
constexpr double CHOL_SHIFT = 1e-13;
constexpr int MAX_W = 96;

namespace {

constexpr int TPB = 256;
inline unsigned grid_for(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > 1048576) b = 1048576;
  return (unsigned)b;
}

// ---------------------------------------------------------------------------- small kernels
__global__ void init_tensor_kernel(double* phi, double* psi, int chi, double w00, double w01,
                                   double w10, double w11) {
  const int t = threadIdx.x;  // 32 entries: a (2) x f1..f4 (16)
  if (t >= 32) return;
  const int a = t >> 4, f = t & 15;
  const double w[2][2] = {{w00, w01}, {w10, w11}};
  const int f1 = (f >> 3) & 1, f2 = (f >> 2) & 1, f3 = (f >> 1) & 1, f4 = f & 1;
  const double u = w[a][f1] * w[a][f2] * w[a][f3] * w[a][f4];
  const int64_t c = chi;
  const int64_t idx = (((((int64_t)f1 * c + f2) * c + f3) * c + f4) * c) + a;
  phi[idx] = u;
  psi[idx] = u;
}

// c = |s|, s /= c, acc += 2^-k ln c, spectra record; flags non-finite or zero c.
__global__ void normalize_kernel(double* s, int n, int k, double* acc, double* lnc_out,
                                 double* rec, int* flag) {
  if (threadIdx.x != 0) return;
  double ss = 0.0;
  for (int i = 0; i < n; ++i) ss += s[i] * s[i];
  const double c = sqrt(ss);
  if (!(c > 0.0) || !isfinite(c)) flag[0] = 1;
  for (int i = 0; i < n; ++i) s[i] /= c;
  const double l = log(c);
  if (lnc_out) lnc_out[k] = l;
  acc[0] += ldexp(l, -k);
  if (rec)
    for (int i = 0; i < n; ++i) rec[i] = s[i];
}

// Weight matrix of the gauge-rotated canonical form: S[i][j] = sum_k O[k][i] s[k] O[k][j].
__global__ void smat_kernel(const double* O, const double* s, double* S, int n) {
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - (idx / n) * n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += O[k * n + i] * s[k] * O[k * n + j];
    S[idx] = acc;
  }
}

// d_k = S_k^-1/2 for S_k > cutoff * S_0, else 0.
__global__ void mask_kernel(const double* S, double* D, int n, double cutoff) {
  const int i = threadIdx.x;
  if (i >= n) return;
  const double smax = S[0];
  D[i] = (S[i] > cutoff * smax) ? 1.0 / sqrt(S[i]) : 0.0;
}

__global__ void zero_int_kernel(int* x) {
  if (threadIdx.x == 0) x[0] = 0;
}

__global__ void copy_small_kernel(double* dst, const double* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// partial sums of sum_{f,g} A[f,g] s_g B[f,g] per block; final reduction by one block.
__global__ void trace_partial_kernel(const double* A, const double* s, const double* B,
                                     int64_t rows, int chi, double* part) {
  __shared__ double red[TPB];
  double acc = 0.0;
  const int64_t total = rows * chi;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    acc += A[idx] * (s ? s[idx % chi] : 1.0) * B[idx];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void trace_final_kernel(const double* part, int nparts, double* out, int* flag) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += part[i];
  out[0] = s;
  if (!(s > 0.0)) flag[0] = 1;
}

// ---------------------------------------------------------------------------- helpers
struct Dims {
  int c;
  int64_t n2, n3, n4, n5;
  int L, Ls;
};

GemmArgs G(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, bool ta,
           const double* B, int64_t ldb, bool tb, double* C, int64_t ldc, double alpha = 1.0,
           double beta = 0.0) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = 0; g.ta = ta;
  g.B = B; g.ldb = ldb; g.sB = 0; g.tb = tb;
  g.C = C; g.ldc = ldc; g.sC = 0;
  g.alpha = alpha; g.beta = beta; g.batch = 1;
  return g;
}
GemmArgs Gb(GemmArgs g, int64_t batch, int64_t sA, int64_t sB, int64_t sC) {
  g.batch = batch; g.sA = sA; g.sB = sB; g.sC = sC;
  return g;
}

}  // namespace
}  // namespace tatrg

using namespace tatrg;

struct tatrg_handle {
  tatrg_config cfg;
  Dims d;
  hipStream_t st;
  // Side stream of the compressed bond swap: the swap's sketch and its map through the first
  // orthonormal factor are independent of the panels' Cholesky chains (latency bound, two
  // work-groups), so they run beside them (fork events on st, a join event on st2).
  hipStream_t st2 = nullptr;  // created at the first step (st itself if that fails)
  bool st2_tried = false;
  bool side_off = false;  // tatrg_set_side_stream(h, 0): the side work runs in order on st
  hipEvent_t fork_ev[2] = {nullptr, nullptr}, join_ev = nullptr;
  bool side_ok = false;  // t1 holds the sketch map of the current step (Q1B of the first pass)
  double* partial2 = nullptr;  // split-K partial sums of the side stream (FP64 path)
  std::string err;
  int step = 0;
  bool initialized = false;
  bool host_fault = false;  // a stage could not be enqueued (reported by tatrg_step)
  int64_t replays = 0;      // steps replayed after a speculation on the CholeskyQR passes failed
  bool force_speculation = false;  // testing: speculate on every step
  // work-group grouping of the split GEMMs chosen by tatrg_autotune (-1: the default rule):
  // [0] P = E.FM4, [1] Phi = Qt^T.P, [2] the swap's sketch map
  int tuned_group[3] = {-1, -1, -1};
  std::vector<double> betas;
  // buffers
  double *phi, *psi, *A, *B, *X, *Y, *atf, *btx, *P1, *P2, *P3, *Gq, *t1, *t2, *tsqr_ws;
  double *Xs, *Ys, *AP, *Ap, *APp, *rho, *UZ, *E, *F, *Gt, *H;
  double *Ah, *Xh, *Yh, *Dh, *XA, *xg, *yg, *pm1, *pm3, *sq1, *sq2, *sq3, *sq4;
  double *chol, *Cm, *Msq, *Nsq, *Fp, *tmp5, *FM4, *P, *q1, *q2, *Qt, *phin;
  double *partial, *probe, *small, *planes;
  // compressed cell middle of the bond swap: the two panels [f'][(x beta)], [b'][(x alpha)]
  // (cp, stride n5), their orthonormal factors (cq), the Cholesky factors of the two passes
  // (cg, cg2), T = L1 L2 = R^T (ct) and R_A (cra); cflag carries the conditioning verdict
  double *cp, *cq, *cg, *cg2, *ctt, *ct, *cra, *cdi, *cli1, *cli2, *ctmp, *cg3;
  double* cqx = nullptr;  // the explicit orthonormal-up-to-the-last-pass panels (cq or cp)
  double* sqdi;  // inverses of the diagonal blocks of the six squeezer Cholesky factors
  int* cflag = nullptr;
  int* vflags = nullptr;  // device: [0] compression verdict, [2 + slot] CholeskyQR verdicts
  // Householder fallback of the CholeskyQR orthonormalisations: while `speculate` is set the
  // fallback kernels are not launched; every failed CholeskyQR pass ORs into orth_sticky, which
  // the end of the step reads, replaying the step with the fallback from the saved state
  // (save_phi, save_psi, save_small) when a pass did fail
  bool speculate = false;
  int* orth_sticky = nullptr;
  // the inputs of the last two temperature-steps (alternating slots): phi, psi, and acc with
  // the fault flag
  double *save_phi[2] = {nullptr, nullptr}, *save_psi[2] = {nullptr, nullptr};
  double *save_small[2] = {nullptr, nullptr};
  int64_t seq = 0;  // temperature-steps enqueued (selects the save slot)
  // the last temperature-step: its CholeskyQR verdict (vflags[2 + slot]) is read at the next
  // synchronisation point; when it ran speculatively and a pass failed it is replayed
  struct Pending {
    bool active = false, spec = false;
    int b = 0, k = 0, slot = 0;
  } pending;
  size_t planes_doubles;
  int* flag;
  double* acc;
  double* lnc;
  double* spectra;
  double* xrec;  // order parameter X^(m), m = 0..n_steps
  double* ttr;   // trace of the last normalised tensor
  double* trace_part;
  size_t partial_doubles;
  // small buffers (carved from `small`)
  size_t tsqr_cap;
  // live timing of the contraction GEMMs (the dominant kernels): event pairs on st
  bool profile = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  // stage boundaries of each profiled step: STAGE_EVENTS events per step on st
  static constexpr int STAGE_EVENTS = 7;
  std::vector<hipEvent_t> sev;
  int sev_used = 0;
  double flops_per_launch = 0.0;
  double *Smat;
  double *s, *sig, *Rp, *Rs, *Cc, *Uc, *Vc, *Oc, *Pm, *Pm0, *RbT, *Rb, *Uh, *Sh, *Vh, *Dm;
  double *Ssq, *Usq, *Vsq, *Umat, *Vmat;
  // Batched randomized SVDs of up to MAX_RB dense chi^2 x chi^2 operators (the four isometry
  // Grams, the three squeezer cores) as one chain of launches: per-entry CholeskyQR flags
  // (bflag), the scratch of the passes (Gqb: six roles x MAX_RB x MAX_W^2) and the core SVDs.
  static constexpr int MAX_RB = 4;
  int* bflag = nullptr;
  double *Gqb = nullptr, *Rbb = nullptr, *RbTb = nullptr, *Uhb = nullptr, *Shb = nullptr;
  double *Vhb = nullptr;
  // One RG state per temperature of the batch; the step runs them in turn through the shared
  // scratch, with phi, psi, flag, acc, lnc, spectra, xrec and ttr pointing at the selected one.
  struct State {
    double *phi = nullptr, *psi = nullptr, *acc = nullptr, *lnc = nullptr;
    double *spectra = nullptr, *xrec = nullptr, *ttr = nullptr;
    int* flag = nullptr;
    std::vector<signed char> swap_compressed;  // per step: 1 compressed middle, 0 full, -1 not run
    bool need_fallback = true;  // a CholeskyQR pass failed in this temperature's last step
  };
  std::vector<State> states;
};

namespace {

constexpr int MAX_BATCH = 1024;

void zero_int(int* x, hipStream_t st) { hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, st, x); }

void select_state(tatrg_handle* h, int b) {
  const tatrg_handle::State& s = h->states[b];
  h->phi = s.phi; h->psi = s.psi; h->acc = s.acc; h->lnc = s.lnc;
  h->spectra = s.spectra; h->xrec = s.xrec; h->ttr = s.ttr; h->flag = s.flag;
}

int open_slot(int m) { return ((3 - m) % 4 + 4) % 4; }

bool valid(const tatrg_config* c) {
  if (!c) return false;
  if (c->chi < 2 || c->chi > 64) return false;
  if (c->r < 1 || c->q < 0 || c->q > 16) return false;
  if (c->n_steps < 1 || c->n_steps > 64) return false;
  if (c->batch < 1 || c->batch > MAX_BATCH) return false;
  if (c->precision != TATRG_FP64 && c->precision != TATRG_BF16X3) return false;
  if (c->swap_mode != 0 && c->swap_mode != 1) return false;
  const int64_t L = std::min<int64_t>((int64_t)c->r * c->chi, (int64_t)c->chi * c->chi);
  if (L > MAX_W) return false;
  return true;
}

Dims dims_of(const tatrg_config* c) {
  Dims d;
  d.c = c->chi;
  d.n2 = (int64_t)d.c * d.c;
  d.n3 = d.n2 * d.c;
  d.n4 = d.n3 * d.c;
  d.n5 = d.n4 * d.c;
  d.L = (int)std::min<int64_t>((int64_t)c->r * d.c, d.n2);
  d.Ls = (int)std::min<int64_t>((int64_t)c->r * d.c, d.n4);
  return d;
}

// Bump allocator: sizes everything when base == nullptr.
struct Carver {
  char* base;
  size_t off = 0;
  double* take(size_t doubles) {
    off = (off + 255) & ~(size_t)255;
    double* p = base ? (double*)(base + off) : nullptr;
    off += doubles * sizeof(double);
    return p;
  }
};

// The three bf16 planes of FM4, [(g k4 kX)][Kp] each with Kp = chi^2 rounded up to 32, in
// doubles.
int64_t fm4_planes_doubles(const Dims& d) {
  return (3 * d.L * d.n2 * bf16x3_kpad(d.n2) * 2 + 7) / 8;
}

// The three bf16 planes of P, [i1][(g k4)][Kp] each with Kp = L^2 rounded up to 32, in
// doubles.
int64_t p_planes_doubles(const Dims& d) {
  return (3 * d.c * d.n2 * bf16x3_kpad(d.L * d.L) * 2 + 7) / 8;
}

size_t splitk_partial_doubles(const Dims& d) {
  // Grams: up to 16 parts of n2 x n2, or 256 parts of c x c
  size_t a = 16 * (size_t)d.n2 * d.n2;
  size_t b = 256 * (size_t)d.c * d.c;
  size_t cbig = 64 * (size_t)N_PROBES * d.c;
  return std::max(a, std::max(b, cbig));
}

void carve(tatrg_handle* h, Carver& cv) {
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2, n3 = d.n3, n4 = d.n4, n5 = d.n5, L = d.L, Ls = d.Ls;
  h->states.assign(h->cfg.batch, tatrg_handle::State());
  for (tatrg_handle::State& st : h->states) {
    st.phi = cv.take(n5);
    st.psi = cv.take(n5);
    st.flag = (int*)cv.take(8);
    st.acc = cv.take(8);
    st.lnc = cv.take(72);
    st.spectra = cv.take((size_t)(h->cfg.n_steps + 1) * 5 * c);
    st.xrec = cv.take((size_t)h->cfg.n_steps + 1);
    st.ttr = cv.take(8);
    if (cv.base) st.swap_compressed.assign((size_t)h->cfg.n_steps + 1, -1);
  }
  select_state(h, 0);
  h->A = cv.take(n5); h->B = cv.take(n5);
  h->X = cv.take(n5); h->Y = cv.take(n5);
  h->cp = cv.take(2 * n5);
  h->atf = cv.take(n5);
  h->btx = cv.take(n5);
  h->cq = cv.take(2 * n5);
  h->cg = cv.take(2 * n2 * n2); h->cg2 = cv.take(2 * n2 * n2); h->ct = cv.take(2 * n2 * n2);
  h->ctt = cv.take(2 * n2 * n2);
  h->cdi = cv.take(2 * (size_t)((n2 + 63) / 64) * 64 * 64);
  h->cli1 = cv.take(2 * n2 * n2); h->cli2 = cv.take(2 * n2 * n2);
  h->ctmp = cv.take(n2 * n2);
  h->cg3 = cv.take(2 * n2 * n2);
  h->sqdi = cv.take(6 * (size_t)((n2 + 63) / 64) * 64 * 64);
  h->cra = cv.take(n2 * n2);
  h->vflags = (int*)cv.take(8);
  h->cflag = h->vflags;            // vflags[0]: compression verdict
  h->orth_sticky = h->vflags + 2;  // vflags[2 + slot]: CholeskyQR verdict of a step
  for (int sl = 0; sl < 2; ++sl) {
    h->save_phi[sl] = cv.take(n5); h->save_psi[sl] = cv.take(n5);
    h->save_small[sl] = cv.take(8);
  }
  h->P1 = cv.take(n4 * Ls); h->P2 = cv.take(n4 * Ls);
  h->P3 = cv.take(n4 * std::max(Ls, c));
  h->Gq = cv.take(6 * (int64_t)MAX_W * MAX_W);
  h->t1 = cv.take(n3 * Ls); h->t2 = cv.take(n3 * Ls);
  const size_t tq = std::max(tsqr_ws_doubles(n4, (int)Ls),
                             std::max(tsqr_ws_doubles(n4, (int)c), tsqr_ws_doubles(n2, (int)L)));
  h->tsqr_ws = cv.take(tq);
  h->tsqr_cap = tq;
  h->Xs = cv.take(n5); h->Ys = cv.take(n5);
  h->AP = cv.take(n5); h->Ap = cv.take(n5); h->APp = cv.take(n5);
  h->rho = cv.take(6 * n2 * n2);
  h->UZ = cv.take(4 * n2 * L);
  h->E = cv.take(L * n3); h->F = cv.take(L * n3); h->Gt = cv.take(L * n3); h->H = cv.take(L * n3);
  h->Ah = cv.take(n5); h->Xh = cv.take(n5); h->Yh = cv.take(n5); h->Dh = cv.take(n5);
  h->XA = cv.take(n5); h->xg = cv.take(n5); h->yg = cv.take(n5);
  h->pm1 = cv.take(n5); h->pm3 = cv.take(n5);
  h->sq1 = cv.take(n2 * n2); h->sq2 = cv.take(n2 * n2); h->sq3 = cv.take(n2 * n2);
  h->sq4 = cv.take(n2 * n2);
  h->chol = cv.take(6 * n2 * n2);
  h->Cm = cv.take(n2 * n2);
  h->Msq = cv.take(3 * n2 * c); h->Nsq = cv.take(3 * n2 * c);
  h->Fp = cv.take(L * n3);
  h->tmp5 = cv.take(L * n4);
  // FM4 in float64 on the FP64 path, its three bf16 planes on the split path
  h->FM4 = cv.take(std::max(L * n4, fm4_planes_doubles(d)));
  // P in float64; on the split path the P GEMM writes P's bf16 planes here instead
  h->P = cv.take(std::max(L * L * n3, p_planes_doubles(d)));
  h->q1 = cv.take(std::max(L * n3, L * L * n2));  // [(i3a kA),(i2b k2)] then [(kA k2 k3), kX]
  // the factors of Qt and their permuted copies (3 c^3 L + c^3 + n2 L)
  h->q2 = cv.take(3 * c * c * c * L + c * c * c + n2 * L);
  h->Qt = cv.take(L * L * n2);
  h->phin = cv.take(n5);
  h->planes_doubles = 0;
  h->planes = nullptr;
  if (h->cfg.precision == TATRG_BF16X3) {
    // bf16 planes the two contraction GEMMs split: E and FM4 for P = E.FM4, Qt for
    // Qt^T.P (whose P planes come from the first GEMM's epilogue)
    GemmArgs g1 = G(c * L, L * n2, n2, nullptr, n2, false, nullptr, L * n2, false, nullptr, 0);
    GemmArgs g2 = Gb(G(n2, n2, L * L, nullptr, n2, true, nullptr, n2, false, nullptr, 0), c, 0,
                     L * L * n2, n4);
    // and the swap's sketch map (Q1B^T Omega)
    GemmArgs g3 = G(n2, c * d.Ls, n3, nullptr, n2, true, nullptr, c * d.Ls, false, nullptr, 0);
    h->planes_doubles = std::max(std::max(gemm_bf16x3_ws_doubles(g1),
                                          gemm_bf16x3_ws_doubles(g2, true)),
                                 gemm_bf16x3_ws_doubles(g3));
    h->planes = cv.take(h->planes_doubles);
  }
  h->partial_doubles = splitk_partial_doubles(d);
  h->partial = cv.take(h->partial_doubles);
  h->partial2 = cv.take(h->partial_doubles);
  h->probe = cv.take((size_t)N_PROBES * n4);
  h->trace_part = cv.take(4096);
  // core factors of an RSVD of any width up to MAX_W (the step's widths are L and Ls; the
  // standalone tatrg_rsvd accepts up to MAX_W)
  const int64_t w = MAX_W;
  h->s = cv.take(c); h->sig = cv.take(c);
  h->Smat = cv.take(c * c);
  h->Rp = cv.take(c * c); h->Rs = cv.take(c * c); h->Cc = cv.take(c * c);
  h->Uc = cv.take(c * c); h->Vc = cv.take(c * c); h->Oc = cv.take(w * w);
  h->Pm = cv.take(N_PROBES * w);
  h->Pm0 = cv.take(N_PROBES * c);
  h->RbT = cv.take(w * w); h->Rb = cv.take(w * w);
  h->Uh = cv.take(w * w); h->Sh = cv.take(w); h->Vh = cv.take(w * w);
  h->Dm = cv.take(w);
  h->Ssq = cv.take(3 * c);
  h->Usq = cv.take(n2 * c); h->Vsq = cv.take(n2 * c);
  h->Umat = cv.take(n2 * c); h->Vmat = cv.take(n2 * c);
  h->small = nullptr;
  // batched RSVDs (the pass-0 panels of orth_b go to P3, the panels themselves to P1, P2)
  const int64_t rb = tatrg_handle::MAX_RB;
  h->bflag = (int*)cv.take(8);
  h->Gqb = cv.take(6 * rb * w * w);
  h->Rbb = cv.take(rb * w * w); h->RbTb = cv.take(rb * w * w);
  h->Uhb = cv.take(rb * w * w); h->Vhb = cv.take(rb * w * w); h->Shb = cv.take(rb * w);
}

bool hip_ok(tatrg_handle* h, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    h->err = std::string(where) + ": " + hipGetErrorString(e);
    return false;
  }
  return true;
}

void gemm(tatrg_handle* h, const GemmArgs& g) { gemm_f64(g, h->st); }

// The contraction GEMMs, bracketed by events when live timing is on (on the split path the
// bracket starts after the plane splitting, so it times the GEMM kernel alone).  b_in and
// c_out (split path only) pass op(B) and C as bf16 planes.
void gemm_timed(tatrg_handle* h, const GemmArgs& g, const Bf16PlanesIn* b_in = nullptr,
                const Bf16PlanesOut* c_out = nullptr, int group_m = -1) {
  const bool on = h->profile && h->ev_used + 2 <= (int)h->ev.size();
  hipEvent_t e0 = on ? h->ev[h->ev_used] : nullptr;
  if (h->cfg.precision == TATRG_BF16X3) {
    if (!gemm_bf16x3(g, h->planes, h->planes_doubles, h->st, e0, b_in, c_out, group_m)) {
      h->err = "split-bf16 plane workspace too small for a contraction GEMM";
      h->host_fault = true;
    }
  } else {
    if (on) hipEventRecord(e0, h->st);
    gemm_f64(g, h->st);
  }
  if (on) {
    hipEventRecord(h->ev[h->ev_used + 1], h->st);
    h->ev_used += 2;
  }
}

// Deterministic split-K for products with a small output and a long K.  The part count fills
// whole rounds of the chip (256 CUs x 2 resident GEMM work-groups) with the tiles that run
// -- for a symmetric product only those on and above the diagonal -- keeping at least 128
// values of K per part and within the partial-sum buffer `partial` of the stream st (partial on
// the handle's stream, partial2 on its side stream).
void gemm_long_k_on(tatrg_handle* h, const GemmArgs& g, double* partial, hipStream_t st) {
  if (g.K >= 4096 && gram_tn(g, partial, h->partial_doubles, st)) return;
  constexpr int64_t SLOTS = 512;
  const int64_t mn = g.M * g.N * g.batch;
  const int64_t tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
  const int64_t tiles = tm * tn * g.batch;
  if (tiles >= 256) {
    gemm_f64(g, st);
    return;
  }
  GemmArgs gs = g;
  gs.sym = g.A == g.B && g.lda == g.ldb && g.ta != g.tb && g.M == g.N && g.sA == g.sB;
  const int64_t active = gs.sym ? tm * (tm + 1) / 2 * g.batch : tiles;
  const int64_t cap = std::min<int64_t>(
      std::min<int64_t>(g.K / 128, (int64_t)(h->partial_doubles / (size_t)mn)), 2048);
  int64_t rounds = (active * ((1024 + tiles - 1) / tiles) + SLOTS - 1) / SLOTS;
  int64_t parts = rounds * SLOTS / active;
  while (parts > cap && rounds > 1) parts = --rounds * SLOTS / active;
  parts = std::min(parts, cap);
  if (parts < 2) {
    gemm_f64(g, st);
    return;
  }
  gemm_f64_splitk(gs, (int)parts, partial, st);
}

void gemm_long_k(tatrg_handle* h, const GemmArgs& g) { gemm_long_k_on(h, g, h->partial, h->st); }

// dst <- src (m x n panels) when lo <= *flag <= hi.
__global__ void copy_panel_when_kernel(const double* src, int64_t lds, double* dst, int64_t ldd,
                                       int64_t m, int n, const int* flag, int lo, int hi) {
  const int f = *flag;
  if (f < lo || f > hi) return;
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / n, j = idx - (idx / n) * n;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

// Orthonormal basis of a tall panel Y (m x n, ld, n <= 96), in place: Y <- Q with Y_in = Q R.
// Shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SISC 2020): a first
// Cholesky pass on the Gram plus the shift 11 (mn + n(n+1)) u ||Y||^2 makes the panel
// well conditioned, two plain passes make it orthonormal; Grams and products run on the
// FP64 MFMA.  A pivot check that fails (the panel is numerically rank deficient) hands the
// panel to the Householder TSQR instead.  The choice is a device flag: both paths are
// launched and each kernel of the unused one returns at once.  Both give the same span up to
// rounding.
//   pass 0: P3 = Y R0^-1        pass 1: Y = P3 R1^-1        pass 2: Y = Y R2^-1 (in place:
//   with n <= 128 each GEMM work-group reads its whole row block before writing it).
// The flag records the failing pass (chol_inv sets pass + 1): after a failure in pass 0 Y
// still holds the input and R = R_tsqr; after one in pass 1 or 2 the pass-0 panel P3 is
// copied back and R = R_tsqr R0.
void orth(tatrg_handle* h, double* Y, int64_t m, int n, int64_t ld, double* R_out,
          bool try_cholqr) {
  hipStream_t st = h->st;
  if (!try_cholqr) {
    tsqr(Y, m, n, ld, R_out, h->tsqr_ws, st, nullptr);
    return;
  }
  int* fail = h->flag + 4;
  const int64_t sq = (int64_t)MAX_W * MAX_W;
  double* G1 = h->Gq;
  double* R0 = h->Gq + sq;
  double* R1 = h->Gq + 2 * sq;
  double* R2 = h->Gq + 3 * sq;
  double* Ri = h->Gq + 4 * sq;
  double* Rt = h->Gq + 5 * sq;
  const double shift = 11.0 * ((double)m * n + (double)n * (n + 1)) * 1.1102230246251565e-16;
  zero((double*)fail, 1, st);
  auto when_ok = [&](GemmArgs g) {
    g.cond = fail;
    g.cond_when = false;
    return g;
  };
  int* sticky = h->speculate ? h->orth_sticky : nullptr;
  // pass 0 (shifted)
  gemm_long_k(h, G(n, n, m, Y, ld, true, Y, ld, false, G1, n));
  chol_inv(G1, R0, Ri, n, 0, fail, st, shift, sticky);
  gemm(h, when_ok(G(m, n, n, Y, ld, false, Ri, n, false, h->P3, n)));
  // pass 1
  gemm_long_k(h, when_ok(G(n, n, m, h->P3, n, true, h->P3, n, false, G1, n)));
  chol_inv(G1, R1, Ri, n, 1, fail, st, 0.0, sticky);
  gemm(h, when_ok(G(m, n, n, h->P3, n, false, Ri, n, false, Y, ld)));
  // pass 2, in place
  gemm_long_k(h, when_ok(G(n, n, m, Y, ld, true, Y, ld, false, G1, n)));
  chol_inv(G1, R2, Ri, n, 2, fail, st, 0.0, sticky);
  gemm(h, when_ok(G(m, n, n, Y, ld, false, Ri, n, false, Y, ld)));
  if (R_out) {  // success: R = R2 R1 R0
    gemm(h, when_ok(G(n, n, n, R2, n, false, R1, n, false, Rt, n)));
    gemm(h, when_ok(G(n, n, n, Rt, n, false, R0, n, false, R_out, n)));
  }
  // speculating that no pass fails: the fallback is not launched (a failure is caught at the
  // end of the step through the sticky flag, and the step is replayed)
  if (h->speculate) return;
  // failure in pass 1 or 2: factorise the pass-0 panel
  hipLaunchKernelGGL(copy_panel_when_kernel, dim3(grid_for(m * n)), dim3(TPB), 0, st, h->P3,
                     (int64_t)n, Y, ld, m, n, fail, 2, 3);
  tsqr(Y, m, n, ld, R_out ? Rt : nullptr, h->tsqr_ws, st, fail);
  if (R_out) {
    GemmArgs a3 = G(n, n, n, Rt, n, false, R0, n, false, R_out, n);
    a3.cond = fail;
    a3.cond_when = true;
    gemm(h, a3);  // R = R_tsqr R0 (overwritten below when pass 0 failed)
    hipLaunchKernelGGL(copy_panel_when_kernel, dim3(grid_for((int64_t)n * n)), dim3(TPB), 0, st,
                       Rt, (int64_t)n, R_out, (int64_t)n, (int64_t)n, n, fail, 1, 1);
  }
}

void perm(tatrg_handle* h, const double* in, double* out, std::vector<int64_t> dims,
          std::vector<int> p) {
  permute(in, out, (int)dims.size(), dims.data(), p.data(), h->st);
}

// ---------------------------------------------------------------------------- RSVD
// Operator interface: apply(in, out, w) computes out = Op * in (rows m), apply_t the
// transpose (rows n); panels are row-major with w columns.
struct Op {
  // Row order of the right-space panels: 0 = the sketch's own order; s > 0 = rows (u, v),
  // u < n / s, v < s, stored in (v, u) order (see philox_gaussian).
  int64_t right_split = 0;
  virtual void apply(const double* in, double* out, int w) = 0;
  virtual void apply_t(const double* in, double* out, int w) = 0;
  virtual ~Op() {}
};

// Randomized SVD (Gaussian sketch, q QR iterations): on return Pa (m x w) holds Q and Pb
// (n x w) holds Qb; Uh, S, Vh (w x w) are the core SVD of Rb^T, so that
// Op ~= (Q Uh) S (Qb Vh)^T.  range_only stops after the last orthonormalisation of Pa.
// sketch_given: Pb already holds the sketch (n x w) instead of a fresh Philox draw.
void rsvd(tatrg_handle* h, Op& op, int64_t m, int64_t n, int w, int q, uint32_t site,
          double* Pa, double* Pb, bool range_only, bool try_cholqr, bool sketch_given = false) {
  hipStream_t st = h->st;
  if (!sketch_given)
    philox_gaussian(Pb, n, w, w, false, h->cfg.seed, (uint32_t)h->step, site, st,
                    op.right_split);
  op.apply(Pb, Pa, w);
  orth(h, Pa, m, w, w, nullptr, try_cholqr);
  for (int it = 0; it < h->cfg.q; ++it) {
    op.apply_t(Pa, Pb, w);
    orth(h, Pb, n, w, w, nullptr, try_cholqr);
    op.apply(Pb, Pa, w);
    orth(h, Pa, m, w, w, nullptr, try_cholqr);
  }
  (void)q;
  (void)st;
  if (range_only) return;
  op.apply_t(Pa, Pb, w);
  orth(h, Pb, n, w, w, h->Rb, try_cholqr);
  transpose_batched(h->Rb, h->RbT, w, w, 1, st);
  jacobi_svd(h->RbT, h->Uh, h->Sh, h->Vh, w, 1, st);
}

// Cell middle of the swap as a product of two factors over the inner bond x:
//   M[(p,alpha),(p',beta)] = sum_x fa[p, (x beta)] fb[(x alpha), p'],
// fa: na x chi^2, fb: chi^2 x nb.  The full middle has fa = A~ as [f'][(x beta)] and
// fb = B~ as [(x alpha)][b'] (na = nb = chi^3); the compressed one has fa = R_A and fb = R_B^T
// (na = nb = chi^2).  Rows of the left-space panels are (p, alpha), those of the right-space
// panels (p', beta), p-major, so that every product is one GEMM with N = chi * w.
struct SwapOp : Op {
  tatrg_handle* h;
  const double* fa = nullptr;
  const double* fb = nullptr;
  int64_t na = 0, nb = 0;
  void apply(const double* om, double* y, int w) override {
    const Dims& d = h->d;
    // t1[(x alpha), (beta j)] = fb[(x alpha), p'] om[p', (beta j)]
    gemm_long_k(h, G(d.n2, d.c * w, nb, fb, nb, false, om, d.c * w, false, h->t1, d.c * w));
    perm(h, h->t1, h->t2, {d.c, d.c, d.c, w}, {0, 2, 1, 3});  // [x, beta, alpha, j]
    // y[p, (alpha j)] = fa[p, (x beta)] t2[(x beta), (alpha j)]
    gemm_long_k(h, G(na, d.c * w, d.n2, fa, d.n2, false, h->t2, d.c * w, false, y, d.c * w));
  }
  void apply_t(const double* qm, double* z, int w) override {
    const Dims& d = h->d;
    // t1[(x beta), (alpha j)] = fa^T qm[p, (alpha j)]
    gemm_long_k(h, G(d.n2, d.c * w, na, fa, d.n2, true, qm, d.c * w, false, h->t1, d.c * w));
    perm(h, h->t1, h->t2, {d.c, d.c, d.c, w}, {0, 2, 1, 3});  // [x, alpha, beta, j]
    // z[p', (beta j)] = fb^T[p', (x alpha)] t2[(x alpha), (beta j)]
    gemm_long_k(h, G(nb, d.c * w, d.n2, fb, nb, true, h->t2, d.c * w, false, z, d.c * w));
  }
};

struct DenseOp : Op {
  tatrg_handle* h;
  const double* M;
  int64_t n;
  void apply(const double* in, double* out, int w) override {
    gemm_long_k(h, G(n, w, n, M, n, false, in, w, false, out, w));
  }
  void apply_t(const double* in, double* out, int w) override {
    gemm_long_k(h, G(n, w, n, M, n, true, in, w, false, out, w));
  }
};

// CholeskyQR3 of nb dense panels Y[e] (m x n, leading dimension n, stride sY, nb <= MAX_RB)
// as one chain of batched launches, with per-panel flags (bflag) and the Householder fallback
// per panel (the steps of orth).  R_out (stride sR) receives each R when given.
void orth_b(tatrg_handle* h, double* Y, int64_t m, int n, int nb, int64_t sY, double* R_out,
            int64_t sR) {
  hipStream_t st = h->st;
  int* fail = h->bflag;
  const int64_t sq = (int64_t)MAX_W * MAX_W, rl = tatrg_handle::MAX_RB * sq, mn = m * n;
  double* G1 = h->Gqb;
  double* R0 = h->Gqb + rl;
  double* R1 = h->Gqb + 2 * rl;
  double* R2 = h->Gqb + 3 * rl;
  double* Ri = h->Gqb + 4 * rl;
  double* Rt = h->Gqb + 5 * rl;
  const double shift = 11.0 * ((double)m * n + (double)n * (n + 1)) * 1.1102230246251565e-16;
  zero((double*)fail, (nb + 1) / 2, st);
  auto when_ok = [&](GemmArgs g) {
    g.cond = fail;
    g.cond_when = false;
    g.cond_stride = 1;
    return g;
  };
  int* sticky = h->speculate ? h->orth_sticky : nullptr;
  // pass 0 (shifted)
  gemm_long_k(h, Gb(G(n, n, m, Y, n, true, Y, n, false, G1, n), nb, sY, sY, sq));
  chol_inv(G1, R0, Ri, n, 0, fail, st, shift, sticky, nb, sq, sq, sq, 1);
  gemm(h, when_ok(Gb(G(m, n, n, Y, n, false, Ri, n, false, h->P3, n), nb, sY, sq, mn)));
  // pass 1
  gemm_long_k(h, when_ok(Gb(G(n, n, m, h->P3, n, true, h->P3, n, false, G1, n), nb, mn, mn,
                            sq)));
  chol_inv(G1, R1, Ri, n, 1, fail, st, 0.0, sticky, nb, sq, sq, sq, 1);
  gemm(h, when_ok(Gb(G(m, n, n, h->P3, n, false, Ri, n, false, Y, n), nb, mn, sq, sY)));
  // pass 2, in place (one tile column: every work-group reads only the rows it writes)
  gemm_long_k(h, when_ok(Gb(G(n, n, m, Y, n, true, Y, n, false, G1, n), nb, sY, sY, sq)));
  chol_inv(G1, R2, Ri, n, 2, fail, st, 0.0, sticky, nb, sq, sq, sq, 1);
  gemm(h, when_ok(Gb(G(m, n, n, Y, n, false, Ri, n, false, Y, n), nb, sY, sq, sY)));
  if (R_out) {  // success: R = R2 R1 R0
    gemm(h, when_ok(Gb(G(n, n, n, R2, n, false, R1, n, false, Rt, n), nb, sq, sq, sq)));
    gemm(h, when_ok(Gb(G(n, n, n, Rt, n, false, R0, n, false, R_out, n), nb, sq, sq, sR)));
  }
  if (h->speculate) return;  // see orth
  for (int e = 0; e < nb; ++e) {
    double* Ye = Y + e * sY;
    hipLaunchKernelGGL(copy_panel_when_kernel, dim3(grid_for(mn)), dim3(TPB), 0, st,
                       h->P3 + e * mn, (int64_t)n, Ye, (int64_t)n, m, n, fail + e, 2, 3);
    tsqr(Ye, m, n, n, R_out ? Rt + e * sq : nullptr, h->tsqr_ws, st, fail + e);
    if (R_out) {
      GemmArgs a3 = G(n, n, n, Rt + e * sq, n, false, R0 + e * sq, n, false, R_out + e * sR, n);
      a3.cond = fail + e;
      a3.cond_when = true;
      gemm(h, a3);
      hipLaunchKernelGGL(copy_panel_when_kernel, dim3(grid_for((int64_t)n * n)), dim3(TPB), 0,
                         st, Rt + e * sq, (int64_t)n, R_out + e * sR, (int64_t)n, (int64_t)n, n,
                         fail + e, 1, 1);
    }
  }
}

// Randomized SVD of nb dense n x n operators M[e] (stride sM, nb <= MAX_RB) as one chain of
// batched launches -- the steps of rsvd, with sketch site sites[e] for entry e.  Pa, Pb: nb
// panels of n x w (stride n w); Pa ends as Q, Pb as Qb.  Unless range_only, the core SVDs of
// Rb^T land in Uhb, Shb, Vhb (strides w^2, w).
void rsvd_b(tatrg_handle* h, const double* M, int64_t sM, int nb, int64_t n, int w,
            const uint32_t* sites, double* Pa, double* Pb, bool range_only) {
  hipStream_t st = h->st;
  const int64_t pw = n * w;
  for (int e = 0; e < nb; ++e)
    philox_gaussian(Pb + e * pw, n, w, w, false, h->cfg.seed, (uint32_t)h->step, sites[e], st);
  auto apply = [&](const double* in, double* out) {
    gemm_long_k(h, Gb(G(n, w, n, M, n, false, in, w, false, out, w), nb, sM, pw, pw));
  };
  auto apply_t = [&](const double* in, double* out) {
    gemm_long_k(h, Gb(G(n, w, n, M, n, true, in, w, false, out, w), nb, sM, pw, pw));
  };
  apply(Pb, Pa);
  orth_b(h, Pa, n, w, nb, pw, nullptr, 0);
  for (int it = 0; it < h->cfg.q; ++it) {
    apply_t(Pa, Pb);
    orth_b(h, Pb, n, w, nb, pw, nullptr, 0);
    apply(Pb, Pa);
    orth_b(h, Pa, n, w, nb, pw, nullptr, 0);
  }
  if (range_only) return;
  apply_t(Pa, Pb);
  orth_b(h, Pb, n, w, nb, pw, h->Rbb, (int64_t)w * w);
  transpose_batched(h->Rbb, h->RbTb, w, w, nb, st);
  jacobi_svd(h->RbTb, h->Uhb, h->Shb, h->Vhb, w, nb, st);
}

// ---------------------------------------------------------------------------- step stages
// S0: T = Phi Psi^T = A s B^T, gauge fixed, normalised.  rec: spectra slot or null.
void canonicalize(tatrg_handle* h, int k, double* rec) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int c = d.c;
  orth(h, h->phi, d.n4, c, c, h->Rp, true);
  orth(h, h->psi, d.n4, c, c, h->Rs, true);
  gemm(h, G(c, c, c, h->Rp, c, false, h->Rs, c, true, h->Cc, c));
  jacobi_svd(h->Cc, h->Uc, h->s, h->Vc, c, 1, st);
  // probes against A = Q_Phi U
  philox_gaussian(h->probe, N_PROBES, d.n4, d.n4, false, h->cfg.seed, (uint32_t)k,
                  SITE_PROBE_CANON, st);
  gemm_long_k(h, G(N_PROBES, c, d.n4, h->probe, d.n4, false, h->phi, c, false, h->Pm0, c));
  gemm(h, G(N_PROBES, c, c, h->Pm0, c, false, h->Uc, c, false, h->Pm, c));
  gauge_rotation(h->s, h->Pm, h->Oc, c, N_PROBES, TAU_NULL, TAU_DEG, st);
  gemm(h, G(c, c, c, h->Uc, c, false, h->Oc, c, false, h->Rb, c));
  gemm(h, G(c, c, c, h->Vc, c, false, h->Oc, c, false, h->Uh, c));
  gemm(h, G(d.n4, c, c, h->phi, c, false, h->Rb, c, false, h->A, c));
  gemm(h, G(d.n4, c, c, h->psi, c, false, h->Uh, c, false, h->B, c));
  hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(64), 0, st, h->s, c, k, h->acc, h->lnc,
                     rec, h->flag);
  // T = c A' S' B'^T with S' = O^T diag(s) O (exact for any gauge rotation O)
  hipLaunchKernelGGL(smat_kernel, dim3(1), dim3(256), 0, st, h->Oc, h->s, h->Smat, c);
}

// Orthonormal factors of the two swap panels, the canonical isometries reshaped as
// P_A[f', (x g)] = A'[x, f', g] and P_B[b', (x g)] = B'[x, b', g] (chi^3 x chi^2 each, stored
// in cp with stride n5, batched): CholeskyQR2, P = Q R^ with Q = Q1 L2^{-T}, Q1 = P L1^{-T}
// (L1, L2 the Cholesky factors of P^T P and Q1^T Q1) and R^ = L2^T L1^T.  Q1 is formed (cq)
// because the second Gram must be taken of it; Q itself is only ever applied, as
// Q1 L2^{-T}, so L2^{-1} is kept (cli2).  The cell middle's panels are P (1 x S'), with the
// gauge-rotated weights S' of the canonical form on the g index, so its factors are
// R = R^ (1 x S'); the isometries are far better conditioned than the weighted panels, whose
// condition grows like 1 / s_min.  Writes R_A to cra and R_B^T = (1 x S') L1 L2 to
// ct + chi^4.  cflag is raised when a pivot of the first pass is below 1e-15 of the largest
// (condition beyond ~3e7, where two passes no longer give an orthonormal Q to rounding; also
// every rank-deficient panel, as in the first steps or at beta = 0) or a pivot of the second
// pass leaves (0.5, 2).
void weights_into_r(tatrg_handle* h);

// The side stream, created at first use (default priority) with its fork and join events; the
// handle's own stream when that fails (the side work then runs in order).
hipStream_t side_stream(tatrg_handle* h) {
  if (h->side_off) return h->st;
  if (!h->st2_tried) {
    h->st2_tried = true;
    if (hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->fork_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->fork_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (h->st2) hipStreamDestroy(h->st2);
      h->st2 = nullptr;
    }
  }
  return h->st2 ? h->st2 : h->st;
}

// Orders the side stream after the work enqueued on st so far (fork event i).
void side_fork(tatrg_handle* h, int i) {
  if (!h->st2 || h->side_off) return;
  hipEventRecord(h->fork_ev[i], h->st);
  hipStreamWaitEvent(h->st2, h->fork_ev[i], 0);
}

// Marks the end of the side stream's work enqueued so far (join event).
void side_join(tatrg_handle* h) {
  if (h->st2 && !h->side_off) hipEventRecord(h->join_ev, h->st2);
}

// Orders st after the side stream's work (no-op without a side stream or before any join).
void side_join_wait(tatrg_handle* h) {
  if (h->st2 && h->join_ev) hipStreamWaitEvent(h->st, h->join_ev, 0);
}

// The swap's Gaussian sketch (rows (beta, b') stored in (b', beta) order) into P2, on stream st;
// on the side stream with a grid of one work-group per CU, so that the Cholesky chain it runs
// beside keeps its CUs.
void swap_sketch(tatrg_handle* h, hipStream_t st) {
  const Dims& d = h->d;
  philox_gaussian(h->P2, d.n4, d.Ls, d.Ls, false, h->cfg.seed, (uint32_t)h->step, SITE_SWAP, st,
                  d.n3, st == h->st ? 0 : 256);
}

// The sketch mapped through the first-pass orthonormal factor of the B panel,
// t1 = Q1B^T Omega (rows (p', beta)), on stream st with the split-K buffer `partial`.  On the
// split path it runs on the split-bf16 engine: it only maps a Gaussian sketch, whose rounding
// at 2^-24 moves the randomized SVD's result far below the split path's error.
void swap_sketch_map(tatrg_handle* h, const double* Q1B, hipStream_t st, double* partial) {
  const Dims& d = h->d;
  const int64_t c = d.c, w = d.Ls;
  const GemmArgs gs = G(d.n2, c * w, d.n3, Q1B, d.n2, true, h->P2, c * w, false, h->t1, c * w);
  if (h->cfg.precision == TATRG_BF16X3) {
    if (!gemm_bf16x3(gs, h->planes, h->planes_doubles, st, nullptr, nullptr, nullptr,
                     h->tuned_group[2])) {
      h->err = "split-bf16 plane workspace too small for the swap sketch map";
      h->host_fault = true;
    }
  } else {
    gemm_long_k_on(h, gs, partial, st);
  }
}

void compress_swap_panels(tatrg_handle* h) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int64_t c = d.c, n2 = d.n2, n3 = d.n3, n5 = d.n5, s2 = n2 * n2;
  zero((double*)h->cflag, 1, st);
  gemm_long_k(h, Gb(G(n2, n2, n3, h->cp, n2, true, h->cp, n2, false, h->cg, n2), 2, n5, n5, s2));
  // side stream: the sketch is drawn while the Cholesky chain below runs (every earlier use of
  // P2 is ordered before the fork)
  const hipStream_t side = side_stream(h);
  side_fork(h, 0);
  swap_sketch(h, side);
  // a zero column of a panel (a zero diagonal entry of its Gram) is structural rank deficiency
  chol_check(h->cg, (int)n2, 2, 0.0, 0.0, INFINITY, h->cflag, st, 8);
  cholesky_blocked_inv(h->cg, h->cdi, (int)n2, 2, h->cflag, st);
  chol_check(h->cg, (int)n2, 2, 1e-15, 0.0, INFINITY, h->cflag, st, 2);
  tri_inv_lower(h->cg, h->cdi, h->cli1, h->ctmp, (int)n2, 2, st, h->partial,
                h->partial_doubles);
  // Q1 = P L1^{-T}
  gemm(h, Gb(G(n3, n2, n2, h->cp, n2, false, h->cli1, n2, true, h->cq, n2), 2, n5, s2, n5));
  // side stream: the sketch map through Q1B runs while the second pass factors its Gram (the
  // bond swap uses it when the verdict is a compressed middle from these panels)
  side_fork(h, 1);
  swap_sketch_map(h, h->cq + n5, side, h->partial2);
  side_join(h);
  h->side_ok = true;
  gemm_long_k(h, Gb(G(n2, n2, n3, h->cq, n2, true, h->cq, n2, false, h->cg2, n2), 2, n5, n5, s2));
  cholesky_blocked_inv(h->cg2, h->cdi, (int)n2, 2, h->cflag, st);
  chol_check(h->cg2, (int)n2, 2, 0.0, 0.5, 2.0, h->cflag, st, 4);
  tri_inv_lower(h->cg2, h->cdi, h->cli2, h->ctmp, (int)n2, 2, st, h->partial,
                h->partial_doubles);
  h->cqx = h->cq;
  // ctt = L1 L2 = R^^T, rows (x g); ct[(x b)] = sum_g S'[b, g] ctt[(x g)] (S' is symmetric)
  gemm_long_k(h, Gb(G(n2, n2, n2, h->cg, n2, false, h->cg2, n2, false, h->ctt, n2), 2, s2, s2, s2));
  weights_into_r(h);
}

// ct[(x b)] = sum_g S'[b, g] ctt[(x g)] for both panels (S' is symmetric), and R_A = ct[0]^T.
void weights_into_r(tatrg_handle* h) {
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2;
  gemm(h, Gb(G(c, n2, c, h->Smat, c, false, h->ctt, n2, false, h->ct, n2), 2 * c, 0, c * n2,
             c * n2));
  transpose_batched(h->ct, h->cra, (int)n2, (int)n2, 1, h->st);
}

// Second attempt, for panels without a zero column that were too ill-conditioned for two
// passes: shifted CholeskyQR3 (Fukaya,
// Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SISC 2020).  Pass 1 factors P^T P + s I with
// s = 11 (m n + n (n + 1)) u tr(P^T P), which bounds the condition of Q1 = P L1^{-T}; passes
// 2 and 3 are plain, Q2 = Q1 L2^{-T} is formed (in cp) and Q = Q2 L3^{-T} is applied
// implicitly.  R^ = L3^T L2^T L1^T.  cflag as in the first attempt.
void compress_swap_panels_shifted(tatrg_handle* h) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int64_t n2 = d.n2, n3 = d.n3, n5 = d.n5, s2 = n2 * n2;
  const double shift = 11.0 * ((double)n3 * n2 + (double)n2 * (n2 + 1)) * 1.1102230246251565e-16;
  h->side_ok = false;  // the sketch map of the side stream used the first attempt's factor
  zero((double*)h->cflag, 1, st);
  gemm_long_k(h, Gb(G(n2, n2, n3, h->cp, n2, true, h->cp, n2, false, h->cg, n2), 2, n5, n5, s2));
  cholesky_shifted_inv(h->cg, h->cdi, (int)n2, 2, shift, h->cflag, st);
  tri_inv_lower(h->cg, h->cdi, h->cli1, h->ctmp, (int)n2, 2, st, h->partial,
                h->partial_doubles);
  gemm(h, Gb(G(n3, n2, n2, h->cp, n2, false, h->cli1, n2, true, h->cq, n2), 2, n5, s2, n5));
  gemm_long_k(h, Gb(G(n2, n2, n3, h->cq, n2, true, h->cq, n2, false, h->cg2, n2), 2, n5, n5, s2));
  cholesky_blocked_inv(h->cg2, h->cdi, (int)n2, 2, h->cflag, st);
  chol_check(h->cg2, (int)n2, 2, 1e-15, 0.0, INFINITY, h->cflag, st, 2);
  tri_inv_lower(h->cg2, h->cdi, h->cli1, h->ctmp, (int)n2, 2, st, h->partial,
                h->partial_doubles);
  // Q2 = Q1 L2^{-T} into cp (the panels are no longer needed)
  gemm(h, Gb(G(n3, n2, n2, h->cq, n2, false, h->cli1, n2, true, h->cp, n2), 2, n5, s2, n5));
  gemm_long_k(h, Gb(G(n2, n2, n3, h->cp, n2, true, h->cp, n2, false, h->cg3, n2), 2, n5, n5, s2));
  cholesky_blocked_inv(h->cg3, h->cdi, (int)n2, 2, h->cflag, st);
  chol_check(h->cg3, (int)n2, 2, 0.0, 0.5, 2.0, h->cflag, st, 4);
  tri_inv_lower(h->cg3, h->cdi, h->cli2, h->ctmp, (int)n2, 2, st, h->partial,
                h->partial_doubles);
  h->cqx = h->cp;
  // ctt = L1 L2 L3
  gemm_long_k(h, Gb(G(n2, n2, n2, h->cg, n2, false, h->cg2, n2, false, h->ct, n2), 2, s2, s2, s2));
  gemm_long_k(h, Gb(G(n2, n2, n2, h->ct, n2, false, h->cg3, n2, false, h->ctt, n2), 2, s2, s2, s2));
  weights_into_r(h);
}

// Bond swap (Section 2, Eq. (1)): rank-chi randomized SVD of the cell middle M, which gives
// X, sigma, Y.  M = (Q_A x 1)(K)(Q_B x 1)^T with the panels' QR factors P = Q R and
// K[(p,alpha),(p',beta)] = sum_x R_A[p,(x beta)] R_B[p',(x alpha)] (chi^3 x chi^3): with Q_A,
// Q_B orthonormal, the randomized SVD of M with the sketch Omega is the one of K with the
// sketch (Q_B x 1)^T Omega, lifted back by Q_A and Q_B, and each product with K costs
// 4 chi^5 Ls instead of 4 chi^6 Ls (Table 1 prices bond swapping at O(q r chi^6)).  When the
// panels are too ill-conditioned for that (compress_swap_panels, verdict read by the caller),
// or with swap_mode = 1, the products run on the full middle instead; both give the same X,
// sigma, Y up to rounding.  Returns whether the compressed middle was used.
// The compression of the swap panels (enqueued; its verdict is read at the step's
// synchronisation point).
void swap_prepare(tatrg_handle* h) {
  const Dims& d = h->d;
  const int c = d.c;
  // P_A = [f', (x g)] and P_B = [b', (x g)] from A' and B'
  perm(h, h->A, h->cp, {c, d.n3, c}, {1, 0, 2});
  perm(h, h->B, h->cp + d.n5, {c, d.n3, c}, {1, 0, 2});
  compress_swap_panels(h);
}

bool bond_swap(tatrg_handle* h, double* rec, bool compressed) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int c = d.c;
  const int w = d.Ls;
  SwapOp op;
  op.h = h;
  if (compressed) {
    const double* Q1A = h->cqx;
    const double* Q1B = h->cqx + d.n5;
    const double* L2iA = h->cli2;
    const double* L2iB = h->cli2 + d.n2 * d.n2;
    // the sketch of M, rows (beta, b') stored in (b', beta) order, then
    // (Q_B x 1)^T Omega = L2B^{-1} Q1B^T Omega: rows (p', beta).  Q1B^T Omega was formed on the
    // side stream during the compression, unless the shifted second attempt replaced Q1B.
    side_join_wait(h);
    if (!h->side_ok) {
      swap_sketch(h, st);
      swap_sketch_map(h, Q1B, st, h->partial);
    }
    h->side_ok = false;
    gemm(h, G(d.n2, c * w, d.n2, L2iB, d.n2, false, h->t1, c * w, false, h->P1, c * w));
    op.fa = h->cra;               // R_A
    op.na = d.n2;
    op.fb = h->ct + d.n2 * d.n2;  // R_B^T
    op.nb = d.n2;
    rsvd(h, op, d.n3, d.n3, w, h->cfg.q, SITE_SWAP, h->P2, h->P1, false, true, true);
    // U~ = Q Uh[:, :c] as [p][(alpha g)]; X rows (f', alpha) = Q_A U~ = Q1A (L2A^{-T} U~)
    gemm(h, G(d.n3, c, w, h->P2, w, false, h->Uh, w, false, h->t1, c));
    gemm_long_k(h, G(d.n2, d.n2, d.n2, L2iA, d.n2, true, h->t1, d.n2, false, h->t2, d.n2));
    gemm(h, G(d.n3, d.n2, d.n2, Q1A, d.n2, false, h->t2, d.n2, false, h->Xs, d.n2));
    perm(h, h->Xs, h->X, {d.n3, c, c}, {1, 0, 2});
    gemm(h, G(d.n3, c, w, h->P1, w, false, h->Vh, w, false, h->t1, c));
    gemm_long_k(h, G(d.n2, d.n2, d.n2, L2iB, d.n2, true, h->t1, d.n2, false, h->t2, d.n2));
    gemm(h, G(d.n3, d.n2, d.n2, Q1B, d.n2, false, h->t2, d.n2, false, h->Xs, d.n2));
    perm(h, h->Xs, h->Y, {d.n3, c, c}, {1, 0, 2});
  } else {
    // the side stream's sketch work of the compression (if any) has to end before P2 and t1
    // are reused (a wait on an event never recorded returns at once)
    side_join_wait(h);
    h->side_ok = false;
    // A~ = A' S', B~ = B' S'; atf = [f', (x beta)], btx = [(x alpha), b']
    gemm(h, G(d.n4, c, c, h->A, c, false, h->Smat, c, false, h->Xs, c));
    gemm(h, G(d.n4, c, c, h->B, c, false, h->Smat, c, false, h->Ys, c));
    perm(h, h->Xs, h->atf, {c, d.n3, c}, {1, 0, 2});
    perm(h, h->Ys, h->btx, {c, d.n3, c}, {0, 2, 1});
    op.fa = h->atf;
    op.na = d.n3;
    op.fb = h->btx;
    op.nb = d.n3;
    op.right_split = d.n3;  // sketch rows (beta, b') stored in (b', beta) order
    rsvd(h, op, d.n4, d.n4, w, h->cfg.q, SITE_SWAP, h->P2, h->P1, false, true);
    // X rows (f', alpha) = Q Uh[:, :c]; Y rows (beta, b') = Qb Vh[:, :c] (Qb rows in (b', beta))
    gemm(h, G(d.n4, c, w, h->P2, w, false, h->Uh, w, false, h->Xs, c));
    perm(h, h->Xs, h->X, {d.n3, c, c}, {1, 0, 2});
    gemm(h, G(d.n4, c, w, h->P1, w, false, h->Vh, w, false, h->Xs, c));
    perm(h, h->Xs, h->Y, {d.n3, c, c}, {1, 0, 2});
  }
  hipLaunchKernelGGL(copy_small_kernel, dim3(1), dim3(64), 0, st, h->sig, h->Sh, c);
  if (rec) hipLaunchKernelGGL(copy_small_kernel, dim3(1), dim3(64), 0, st, rec, h->Sh, c);
  return compressed;
}

// Gram of the (l2 l3) pair: rho[(l2 l3),(l2' l3')] = sum over the other legs of T T' for
// 5-leg tensors T, T' laid out [l1,l2,l3,l4,l5] with the pair at positions (p, p+1) = (1,2)
// (A-type, [f1,f2,f3,f4,a]) -- both operands are permuted to [(l2 l3), rest].
void pair_gram(tatrg_handle* h, const double* T1, const double* T2, double* out) {
  const Dims& d = h->d;
  const int64_t c = d.c;
  perm(h, T1, h->Ap, {c, c, c, c, c}, {1, 2, 0, 3, 4});
  const double* rhs = h->Ap;
  if (T2 != T1) {
    perm(h, T2, h->APp, {c, c, c, c, c}, {1, 2, 0, 3, 4});
    rhs = h->APp;
  }
  gemm_long_k(h, G(d.n2, d.n2, d.n3, h->Ap, d.n3, false, rhs, d.n3, true, out, d.n2));
}

void isometries(tatrg_handle* h) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int64_t c = d.c, n2 = d.n2;
  copy_scale_cols(h->Xs, h->X, h->sig, d.n4, c, st);
  copy_scale_cols(h->Ys, h->Y, h->sig, d.n4, c, st);
  // P_X = (X sigma)(X sigma)^T and P_Y alike (c x c, semidefinite), side by side in the
  // batched scratch, and factors L L^T = P: rho_A = sum A P_X A^T = (A L_X)(A L_X)^T is then a
  // symmetric Gram (half the tiles of the product), and rho_D alike
  double* px = h->Gqb;
  double* py = h->Gqb + c * c;
  double* lx = h->Uhb;
  double* ly = h->Uhb + c * c;
  gemm_long_k(h, G(c, c, d.n4, h->Xs, d.n4, false, h->Xs, d.n4, true, px, c));
  gemm_long_k(h, G(c, c, d.n4, h->Ys, d.n4, false, h->Ys, d.n4, true, py, c));
  // the factors (a latency-bound Jacobi SVD) on the side stream while the X- and Y-type Grams,
  // which do not need them, run here
  const hipStream_t side = side_stream(h);
  side_fork(h, 0);
  psd_factor(px, lx, h->Shb, h->Vhb, (int)c, 2, side);
  side_join(h);
  double* rA = h->rho;
  double* rX = h->rho + n2 * n2;
  double* rY = h->rho + 2 * n2 * n2;
  double* rD = h->rho + 3 * n2 * n2;
  // X-type: [alpha, f2, f3, f4, g] -> [(f2 f3), alpha, f4, g]
  perm(h, h->Xs, h->Ap, {c, c, c, c, c}, {1, 2, 0, 3, 4});
  gemm_long_k(h, G(n2, n2, d.n3, h->Ap, d.n3, false, h->Ap, d.n3, true, rX, n2));
  perm(h, h->Ys, h->Ap, {c, c, c, c, c}, {1, 2, 0, 3, 4});
  gemm_long_k(h, G(n2, n2, d.n3, h->Ap, d.n3, false, h->Ap, d.n3, true, rY, n2));
  side_join_wait(h);
  gemm(h, G(d.n4, c, c, h->A, c, false, lx, c, false, h->AP, c));
  pair_gram(h, h->AP, h->AP, rA);
  gemm(h, G(d.n4, c, c, h->B, c, false, ly, c, false, h->AP, c));
  pair_gram(h, h->AP, h->AP, rD);
  // the four range finders as one batched chain: U^Z lands in UZ + z n2 L
  const uint32_t sites[4] = {SITE_ISO_A, SITE_ISO_X, SITE_ISO_Y, SITE_ISO_D};
  rsvd_b(h, h->rho, n2 * n2, 4, n2, d.L, sites, h->UZ, h->P1, true);
}

void triad(tatrg_handle* h) {
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2, L = d.L;
  // c products of L x n2 x n2: one row of output tiles each, so in two halves of K (two
  // resident work-groups per CU instead of one) when the partial sums fit
  auto gemm = [&](tatrg_handle* hh, const GemmArgs& g) {
    if ((size_t)(2 * g.batch * g.M * g.N) <= hh->partial_doubles)
      gemm_f64_splitk(g, 2, hh->partial, hh->st);
    else
      gemm_f64(g, hh->st);
  };
  const double* UA = h->UZ;
  const double* UX = h->UZ + n2 * L;
  const double* UY = h->UZ + 2 * n2 * L;
  const double* UD = h->UZ + 3 * n2 * L;
  // E[f1][kA][(f4 a)] = UA^T A[f1][(f2 f3)][(f4 a)]   (and F, G, H alike)
  gemm(h, Gb(G(L, n2, n2, UA, L, true, h->A, n2, false, h->E, n2), c, 0, d.n4, L * n2));
  gemm(h, Gb(G(L, n2, n2, UX, L, true, h->X, n2, false, h->F, n2), c, 0, d.n4, L * n2));
  scale_cols(h->F, h->sig, c * L * c, c, c, h->st);
  gemm(h, Gb(G(L, n2, n2, UY, L, true, h->Y, n2, false, h->Gt, n2), c, 0, d.n4, L * n2));
  gemm(h, Gb(G(L, n2, n2, UD, L, true, h->B, n2, false, h->H, n2), c, 0, d.n4, L * n2));
}

void squeezers(tatrg_handle* h, double* rec) {
  const Dims& d = h->d;
  hipStream_t st = h->st;
  const int64_t c = d.c, n2 = d.n2, n3 = d.n3, n4 = d.n4, L = d.L;
  const double* UA = h->UZ;
  const double* UX = h->UZ + n2 * L;
  const double* UY = h->UZ + 2 * n2 * L;
  const double* UD = h->UZ + 3 * n2 * L;
  // projected fundamental tensors
  gemm(h, Gb(G(n2, n2, L, UA, L, false, h->E, n2, false, h->Ah, n2), c, 0, L * n2, n4));
  gemm(h, Gb(G(n2, n2, L, UX, L, false, h->F, n2, false, h->Xh, n2), c, 0, L * n2, n4));
  gemm(h, Gb(G(n2, n2, L, UY, L, false, h->Gt, n2, false, h->Yh, n2), c, 0, L * n2, n4));
  gemm(h, Gb(G(n2, n2, L, UD, L, false, h->H, n2, false, h->Dh, n2), c, 0, L * n2, n4));
  double* aag = h->Cc;
  double* ddg = h->Uc;
  // g_f, g_b side by side in the batched scratch, their factors L L^T = g in Uhb
  double* gf = h->Gqb;
  double* gb = h->Gqb + c * c;
  double* lf = h->Uhb;
  double* lb = h->Uhb + c * c;
  gemm_long_k(h, G(c, c, n4, h->Ah, c, true, h->Ah, c, false, aag, c));
  gemm_long_k(h, G(c, c, n4, h->Dh, c, true, h->Dh, c, false, ddg, c));
  // g_f = Xh^T (aag^T Xh), g_b = Yh^T (ddg^T Yh) with Xh viewed (c x n4) / (n4 x c): Grams of
  // Ah Xh and Dh Yh, so semidefinite
  gemm(h, G(c, n4, c, aag, c, true, h->Xh, n4, false, h->XA, n4));
  gemm_long_k(h, G(c, c, n4, h->Xh, c, true, h->XA, c, false, gf, c));
  gemm(h, G(c, n4, c, ddg, c, true, h->Yh, n4, false, h->XA, n4));
  gemm_long_k(h, G(c, c, n4, h->Yh, c, true, h->XA, c, false, gb, c));
  const std::vector<int> a_perm[3] = {{1, 4, 0, 2, 3}, {2, 4, 0, 1, 3}, {3, 4, 0, 1, 2}};
  const std::vector<int> x_perm[3] = {{0, 1, 2, 3, 4}, {0, 2, 1, 3, 4}, {0, 3, 1, 2, 4}};
  const std::vector<int64_t> d5 = {c, c, c, c, c};
  const std::vector<int64_t> d4 = {c, c, c, c};
  // the factors (a latency-bound Jacobi SVD) on the side stream while the first Gram of Ah
  // alone, which does not need them, runs here
  const hipStream_t side = side_stream(h);
  side_fork(h, 0);
  psd_factor(gf, lf, h->Shb, h->Vhb, (int)c, 2, side);
  side_join(h);
  perm(h, h->Ah, h->pm1, d5, a_perm[0]);
  gemm_long_k(h, G(n2, n2, n3, h->pm1, n3, false, h->pm1, n3, true, h->sq1, n2));
  side_join_wait(h);
  // xg = Xh L_b, yg = Yh L_f: the Grams of the forward and backward pairs below are then
  // symmetric products of one operand (sum Xh g_b Xh^T = (Xh L_b)(Xh L_b)^T)
  gemm(h, G(n4, c, c, h->Xh, c, false, lb, c, false, h->xg, c));
  gemm(h, G(n4, c, c, h->Yh, c, false, lf, c, false, h->yg, c));

  for (int mi = 0; mi < 3; ++mi) {
    double* rl = h->rho + mi * n2 * n2;
    double* rr = h->rho + (3 + mi) * n2 * n2;
    // rho_L = sum_{a a'} aa[u1 a u1' a'] xx[a u2 a' u2'] (aa of mi = 0 is formed above)
    if (mi > 0) {
      perm(h, h->Ah, h->pm1, d5, a_perm[mi]);
      gemm_long_k(h, G(n2, n2, n3, h->pm1, n3, false, h->pm1, n3, true, h->sq1, n2));
    }
    // (x_perm[0] is the identity: xg is used as it is)
    const double* xs = h->xg;
    if (mi > 0) {
      perm(h, h->xg, h->pm3, d5, x_perm[mi]);
      xs = h->pm3;
    }
    gemm_long_k(h, G(n2, n2, n3, xs, n3, false, xs, n3, true, h->sq2, n2));
    perm(h, h->sq1, h->sq3, d4, {0, 2, 1, 3});
    perm(h, h->sq2, h->sq4, d4, {0, 2, 1, 3});
    gemm_long_k(h, G(n2, n2, n2, h->sq3, n2, false, h->sq4, n2, false, h->sq1, n2));
    perm(h, h->sq1, rl, d4, {0, 2, 1, 3});
    // rho_R = sum_{b b'} yy[b v1 b' v1'] dd[v2 b v2' b']
    const double* ys = h->yg;
    if (mi > 0) {
      perm(h, h->yg, h->pm3, d5, x_perm[mi]);
      ys = h->pm3;
    }
    gemm_long_k(h, G(n2, n2, n3, ys, n3, false, ys, n3, true, h->sq2, n2));
    perm(h, h->Dh, h->pm1, d5, a_perm[mi]);
    gemm_long_k(h, G(n2, n2, n3, h->pm1, n3, false, h->pm1, n3, true, h->sq1, n2));
    perm(h, h->sq2, h->sq3, d4, {1, 3, 0, 2});
    perm(h, h->sq1, h->sq4, d4, {1, 3, 0, 2});
    gemm_long_k(h, G(n2, n2, n2, h->sq3, n2, false, h->sq4, n2, false, h->sq1, n2));
    perm(h, h->sq1, rr, d4, {0, 2, 1, 3});
  }
  symmetrize(h->rho, (int)n2, 6, st);
  copy(h->chol, h->rho, 6 * n2 * n2, st);
  cholesky_shifted_inv(h->chol, h->sqdi, (int)n2, 6, CHOL_SHIFT, h->flag, st);
  const uint32_t sq_sites[3] = {SITE_SQZ_2, SITE_SQZ_3, SITE_SQZ_4};
  const uint32_t pr_sites[3] = {SITE_PROBE_SQZ_2, SITE_PROBE_SQZ_3, SITE_PROBE_SQZ_4};
  // the three squeezer pairs after the shared Cholesky: C = R_L R_R^T = Ll^T Lr for each
  // (rho_L + shift = Ll Ll^T, R_L = Ll^T; R_R = Lr^T), into the Grams' space, then one batched
  // randomized SVD of the three (Q in P2, Qb in P1, cores in Uhb, Shb, Vhb)
  const int w = d.L;
  gemm_long_k(h, Gb(G(n2, n2, n2, h->chol, n2, true, h->chol + 3 * n2 * n2, n2, false, h->rho, n2),
                    3, n2 * n2, n2 * n2, n2 * n2));
  rsvd_b(h, h->rho, n2 * n2, 3, n2, w, sq_sites, h->P2, h->P1, false);
  for (int mi = 0; mi < 3; ++mi) {
    const double* Ll = h->chol + mi * n2 * n2;
    const double* Lr = h->chol + (3 + mi) * n2 * n2;
    const double* Q = h->P2 + mi * n2 * w;
    const double* Qb = h->P1 + mi * n2 * w;
    const double* Uh = h->Uhb + (int64_t)mi * w * w;
    const double* Vh = h->Vhb + (int64_t)mi * w * w;
    const double* Sh = h->Shb + mi * w;
    // U = Q Uh[:, :c], V = Qb Vh[:, :c]
    gemm(h, G(n2, c, w, Q, w, false, Uh, w, false, h->Usq, c));
    gemm(h, G(n2, c, w, Qb, w, false, Vh, w, false, h->Vsq, c));
    double* S = h->Ssq + mi * c;
    hipLaunchKernelGGL(copy_small_kernel, dim3(1), dim3(64), 0, st, S, Sh, (int)c);
    if (rec)
      hipLaunchKernelGGL(copy_small_kernel, dim3(1), dim3(64), 0, st, rec + mi * c, Sh, (int)c);
    philox_gaussian(h->probe, N_PROBES, n2, n2, false, h->cfg.seed, (uint32_t)h->step,
                    pr_sites[mi], st);
    gemm(h, G(N_PROBES, c, n2, h->probe, n2, false, h->Vsq, c, false, h->Pm, c));
    gauge_rotation(S, h->Pm, h->Oc, (int)c, N_PROBES, TAU_NULL, TAU_DEG, st);
    hipLaunchKernelGGL(mask_kernel, dim3(1), dim3(128), 0, st, S, h->Dm, (int)c, SQZ_CUTOFF);
    // M = (R_R^T V D) O = (Lr V D) O  (n2 x c), stored [u1][u2][k]; rotating after the
    // S^-1/2 weights keeps M N = R_R^T V S^-1 U^T R_L for any O.
    double* M = h->Msq + mi * n2 * c;
    gemm_long_k(h, G(n2, c, n2, Lr, n2, false, h->Vsq, c, false, h->Vmat, c));
    scale_cols(h->Vmat, h->Dm, n2, c, c, st);
    gemm(h, G(n2, c, c, h->Vmat, c, false, h->Oc, c, false, M, c));
    // N = O^T (D U^T R_L) = ((Ll U D) O)^T  (c x n2), stored [k][v1][v2]
    gemm_long_k(h, G(n2, c, n2, Ll, n2, false, h->Usq, c, false, h->Umat, c));
    scale_cols(h->Umat, h->Dm, n2, c, c, st);
    gemm(h, G(n2, c, c, h->Umat, c, false, h->Oc, c, false, h->Vsq, c));
    transpose_batched(h->Vsq, h->Nsq + mi * n2 * c, (int)n2, (int)c, 1, st);
  }
}

// One half of the contraction (Eqs. (makeMG) / (makeMH)):
//   out[k2,k3,k4,l1,g] = sum (E F S4)(I J S2 S3), rotated.
// E: [l1][kA][(l4a a)], F: [a][kX][(l4b g)], I/J: [(l2 l3)][k], S4p: [l4b][l4a][k4],
// S2, S3: [l_a][l_b][k].
void contract_half(tatrg_handle* h, const double* E, const double* F, const double* I,
                   const double* J, const double* S4p, const double* S2, const double* S3,
                   double* out) {
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2, L = d.L;
  // Fp[i4b][(a kX g)]
  perm(h, F, h->Fp, {c, L, c, c}, {2, 0, 1, 3});
  // tmp[(i4a k4)][(a kX g)] = S4p^T Fp
  gemm(h, G(n2, c * L * c, c, S4p, n2, true, h->Fp, c * L * c, false, h->tmp5, c * L * c));
  const bool split = h->cfg.precision == TATRG_BF16X3;
  const int64_t Kp = bf16x3_kpad(L * L);
  uint16_t* pp = reinterpret_cast<uint16_t*>(h->P);
  const int64_t pn = c * n2 * Kp;  // elements per plane of P
  if (split) {
    // FM4[i4a][a][g][k4][kX], kX innermost, goes straight from tmp5 into the bf16 planes the
    // P GEMM reads (it is never stored in float64); the P GEMM's columns are (g k4, kX) and
    // its epilogue writes P's planes [i1][(g k4)][(kA kX)], K-contiguous for Qt^T.P
    uint16_t* fp = reinterpret_cast<uint16_t*>(h->FM4);
    const int64_t fn = L * n2 * bf16x3_kpad(n2);
    if (!fm4_planes(h->tmp5, (int)c, (int)L, fp, 4 * fm4_planes_doubles(d), h->st)) {
      h->err = "FM4 plane workspace too small";
      h->host_fault = true;
    }
    const Bf16PlanesIn fi = {{fp, fp + fn, fp + 2 * fn}, 0};
    const Bf16PlanesOut po = {{pp, pp + pn, pp + 2 * pn}, L, n2, L, Kp, 0, pn};
    gemm_timed(h, G(c * L, L * n2, n2, E, n2, false, nullptr, L * n2, false, nullptr, 0), &fi,
               &po, h->tuned_group[0]);
  } else {
    // FM4[i4a][a][kX][g][k4]
    perm(h, h->tmp5, h->FM4, {c, c, c, L, c}, {0, 2, 3, 4, 1});
    // P[(i1 kA)][(kX g k4)] = E[(i1 kA)][(i4a a)] FM4[(i4a a)][(kX g k4)]
    gemm_timed(h, G(c * L, L * n2, n2, E, n2, false, h->FM4, L * n2, false, h->P, L * n2));
  }
  // Qt[kA][kX][k2][k3] = sum I[(i2a i3a)][kA] S2[i2a][i2b][k2] S3[i3a][i3b][k3] J[(i2b i3b)][kX],
  // as (I S2)(S3 J) contracted over (i3a, i2b): both factors have c^3 L entries, so no
  // intermediate of L chi^4 entries is formed
  double* fap = h->q2;                   // [kA][k2][i3a][i2b]
  double* s3p = fap + c * c * c * L;     // [i3a][k3][i3b]
  double* jp = s3p + c * c * c;          // [i3b][i2b][kX]
  double* fb = jp + n2 * L;              // [i3a][k3][i2b][kX]
  double* fbp = fb + c * c * c * L;      // [i3a][i2b][k3][kX]
  gemm(h, G(c * L, n2, c, I, c * L, true, S2, n2, false, h->q1, n2));        // [(i3a kA),(i2b k2)]
  perm(h, h->q1, fap, {c, L, c, c}, {1, 3, 0, 2});
  perm(h, S3, s3p, {c, c, c}, {0, 2, 1});
  perm(h, J, jp, {c, c, L}, {1, 0, 2});
  gemm(h, G(n2, c * L, c, s3p, c, false, jp, c * L, false, fb, c * L));     // [(i3a k3),(i2b kX)]
  perm(h, fb, fbp, {c, c, c, L}, {0, 2, 1, 3});
  gemm(h, G(c * L, c * L, n2, fap, n2, false, fbp, c * L, false, h->q1, c * L));  // [(kA k2),(k3 kX)]
  perm(h, h->q1, h->Qt, {L, c, c, L}, {0, 3, 1, 2});                        // [kA,kX,k2,k3]
  // phin[i1][(k2 k3)][(g k4)] = Qt^T P[i1]
  if (split) {
    const Bf16PlanesIn pi = {{pp, pp + pn, pp + 2 * pn}, n2 * Kp};
    gemm_timed(h, Gb(G(n2, n2, L * L, h->Qt, n2, true, nullptr, 0, false, h->phin, n2), c, 0,
                     0, d.n4), &pi, nullptr, h->tuned_group[1]);
  } else {
    gemm_timed(h, Gb(G(n2, n2, L * L, h->Qt, n2, true, h->P, n2, false, h->phin, n2), c, 0,
                     L * L * n2, d.n4));
  }
  // rotate: [i1,k2,k3,g,k4] -> [k2,k3,k4,i1,g]
  perm(h, h->phin, out, {c, c, c, c, c}, {1, 2, 4, 0, 3});
}

void contraction(tatrg_handle* h) {
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2, L = d.L;
  const double* UA = h->UZ;
  const double* UX = h->UZ + n2 * L;
  const double* UY = h->UZ + 2 * n2 * L;
  const double* UD = h->UZ + 3 * n2 * L;
  const double* M2 = h->Msq;
  const double* M3 = h->Msq + n2 * c;
  const double* M4 = h->Msq + 2 * n2 * c;
  const double* N2 = h->Nsq;
  const double* N3 = h->Nsq + n2 * c;
  const double* N4 = h->Nsq + 2 * n2 * c;
  const std::vector<int64_t> d3 = {c, c, c};
  // Phi: S4p = M4 [i4a,i4b,k4] -> [i4b,i4a,k4]
  double* s4p = h->sq1;
  double* s2 = h->sq2;
  double* s3 = h->sq3;
  perm(h, M4, s4p, d3, {1, 0, 2});
  contract_half(h, h->E, h->F, UA, UX, s4p, M2, M3, h->phi);
  // Psi: roles E<-H (site n), F<-G; N stored [k][j_a][j_b]:
  // S4p[j4a][j4b][k] = N4 perm (1,2,0); S2[j2b][j2a][k] = N2 perm (2,1,0)
  perm(h, N4, s4p, d3, {1, 2, 0});
  perm(h, N2, s2, d3, {2, 1, 0});
  perm(h, N3, s3, d3, {2, 1, 0});
  contract_half(h, h->H, h->Gt, UD, UY, s4p, s2, s3, h->psi);
}

}  // namespace

// ============================================================================== C ABI
extern "C" {

size_t tatrg_workspace_bytes(const tatrg_config* cfg) {
  if (!valid(cfg)) return 0;
  tatrg_handle tmp;
  tmp.cfg = *cfg;
  tmp.d = dims_of(cfg);
  Carver cv{nullptr};
  carve(&tmp, cv);
  return cv.off + 256;
}

tatrg_status tatrg_create(const tatrg_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                          tatrg_handle** out) {
  if (!out) return TATRG_EINVAL;
  *out = nullptr;
  if (!valid(cfg)) return TATRG_EINVAL;
  const size_t need = tatrg_workspace_bytes(cfg);
  if (!d_ws || ws_bytes < need) return TATRG_ENOMEM;
  tatrg_handle* h = new tatrg_handle();
  h->cfg = *cfg;
  h->d = dims_of(cfg);
  h->st = (hipStream_t)stream;
  char* base = (char*)(((uintptr_t)d_ws + 255) & ~(uintptr_t)255);
  Carver cv{base};
  carve(h, cv);
  (void)hipGetLastError();
  *out = h;
  return TATRG_OK;
}

tatrg_status tatrg_init_tensor(tatrg_handle* h, const double* h_betas) {
  if (!h || !h_betas) return TATRG_EINVAL;
  const int nb = h->cfg.batch;
  for (int b = 0; b < nb; ++b) {
    if (!std::isfinite(h_betas[b]) || h_betas[b] < 0.0) {
      h->err = "every beta must be finite and >= 0";
      return TATRG_EINVAL;
    }
  }
  h->betas.assign(h_betas, h_betas + nb);
  const Dims& d = h->d;
  hipStream_t st = h->st;
  for (int b = 0; b < nb; ++b) {
    select_state(h, b);
    zero(h->phi, d.n5, st);
    zero(h->psi, d.n5, st);
    // W = element-wise square root of [[cosh b, sinh b], [cosh b, -sinh b]]
    const double sc = std::sqrt(std::cosh(h_betas[b])), ss = std::sqrt(std::sinh(h_betas[b]));
    hipLaunchKernelGGL(init_tensor_kernel, dim3(1), dim3(64), 0, st, h->phi, h->psi, d.c, sc,
                       ss, sc, -ss);
    zero((double*)h->flag, 4, st);
    zero(h->acc, 8, st);
    zero(h->lnc, 72, st);
    zero(h->spectra, (int64_t)(h->cfg.n_steps + 1) * 5 * d.c, st);
    zero(h->xrec, h->cfg.n_steps + 1, st);
    zero(h->ttr, 8, st);
  }
  for (tatrg_handle::State& sta : h->states) sta.need_fallback = true;
  h->pending.active = false;
  select_state(h, 0);
  h->step = 0;
  h->initialized = true;
  if (!hip_ok(h, "init_tensor")) return TATRG_EHIP;
  return TATRG_OK;
}

}  // extern "C"

namespace {

// Phase A of a temperature-step: the order parameter record, the canonical form and the
// compression of the swap panels (up to the step's synchronisation point).
void step_phase_a(tatrg_handle* h, int b, double* rec, bool timed) {
  auto mark = [&](int i) {
    if (timed) hipEventRecord(h->sev[h->sev_used + i], h->st);
  };
  if (rec)
    order_parameter(h->phi, h->psi, h->d.c, open_slot(h->step), h->partial, h->xrec + h->step,
                    h->st);
  mark(0);
  canonicalize(h, h->step, rec);
  mark(1);
  if (h->cfg.swap_mode == 0) swap_prepare(h);
  (void)b;
}

// Phase B: bond swap, isometries, triad, squeezers, contraction and rotation.
void step_phase_b(tatrg_handle* h, int b, double* rec, bool timed, bool compressed) {
  auto mark = [&](int i) {
    if (timed) hipEventRecord(h->sev[h->sev_used + i], h->st);
  };
  const bool comp = bond_swap(h, rec ? rec + h->d.c : nullptr, compressed);
  if (h->step < (int)h->states[b].swap_compressed.size())
    h->states[b].swap_compressed[h->step] = comp ? 1 : 0;
  mark(2);
  isometries(h);
  mark(3);
  triad(h);
  mark(4);
  squeezers(h, rec ? rec + 2 * h->d.c : nullptr);
  mark(5);
  contraction(h);
  mark(6);
  if (timed) h->sev_used += tatrg_handle::STAGE_EVENTS;
}

// The step's synchronisation point: waits for the stream and reads the compression verdict
// (vflags[0]) and, when one is pending, the previous temperature-step's CholeskyQR verdict
// (vflags[2 + slot]).  Returns false on a HIP error.
bool sync_point(tatrg_handle* h, bool want_compression, bool* compressed, bool* prev_failed,
                int* verdict = nullptr) {
  *compressed = false;
  *prev_failed = false;
  // wait for the streams, then read the verdicts (one small copy from an idle device)
  if (hipStreamSynchronize(h->st) != hipSuccess) return false;
  if (h->st2 && hipStreamSynchronize(h->st2) != hipSuccess) return false;
  int v[4] = {1, 0, 1, 1};
  if (hipMemcpy(v, h->vflags, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return false;
  *compressed = want_compression && v[0] == 0;
  if (verdict) *verdict = v[0];
  if (h->pending.active) {
    // the last temperature-step's CholeskyQR verdict: whether its temperature still needs the
    // fallback, and whether it has to be replayed (it ran without the fallback)
    const bool failed = v[2 + h->pending.slot] != 0;
    h->states[h->pending.b].need_fallback = failed;
    *prev_failed = failed && h->pending.spec;
    if (!*prev_failed) h->pending.active = false;
  }
  return true;
}

// Phase A, the synchronisation point and -- when the compression failed with every pivot
// positive -- the shifted three-pass compression with a second synchronisation.  Returns
// false on a HIP error.
bool phase_a_and_sync(tatrg_handle* h, int b, double* rec, bool timed, bool* compressed,
                      bool* prev_failed) {
  step_phase_a(h, b, rec, timed);
  *compressed = false;
  *prev_failed = false;
  int verdict = 0;
  if (h->cfg.swap_mode == 0 || h->pending.active)
    if (!sync_point(h, h->cfg.swap_mode == 0, compressed, prev_failed, &verdict)) return false;
  if (!*prev_failed && h->cfg.swap_mode == 0 && !*compressed && !(verdict & 8)) {
    // no zero column: ill-conditioned rather than structurally rank deficient, so the shifted
    // three-pass factorisation may still compress the middle
    compress_swap_panels_shifted(h);
    bool dummy = false;
    if (!sync_point(h, true, compressed, &dummy)) return false;
  }
  return true;
}

void restore_state(tatrg_handle* h, int b, int slot) {
  select_state(h, b);
  copy(h->phi, h->save_phi[slot], h->d.n5, h->st);
  copy(h->psi, h->save_psi[slot], h->d.n5, h->st);
  copy(h->acc, h->save_small[slot], 1, h->st);
  copy((double*)h->flag, h->save_small[slot] + 1, 1, h->st);
}

// One temperature-step of state b at step index h->step.  Saves the input, enqueues phase A,
// synchronises (verifying a pending speculative step and replaying it when its CholeskyQR
// passes failed without the fallback), then phase B.  Speculating (when the last step of b
// had no failed pass), the Householder fallbacks are not launched; the step is then left
// pending until the next synchronisation point.
bool temperature_step(tatrg_handle* h, int b) {
  for (;;) {
    select_state(h, b);
    tatrg_handle::State& state = h->states[b];
    const int slot = (int)(h->seq & 1);
    copy(h->save_phi[slot], h->phi, h->d.n5, h->st);
    copy(h->save_psi[slot], h->psi, h->d.n5, h->st);
    copy(h->save_small[slot], h->acc, 1, h->st);
    copy(h->save_small[slot] + 1, (const double*)h->flag, 1, h->st);
    h->orth_sticky = h->vflags + 2 + slot;
    zero_int(h->orth_sticky, h->st);
    // speculate once this temperature's last step had no failed CholeskyQR pass and took the
    // compressed cell middle (the panels of the full middle come with rank-deficient steps)
    h->speculate = h->force_speculation ||
                   (!state.need_fallback && h->step > 0 &&
                    state.swap_compressed[h->step - 1] == 1);
    const bool spec_a = h->speculate;
    double* rec = h->cfg.record_spectra ? h->spectra + (int64_t)h->step * 5 * h->d.c : nullptr;
    const bool timed =
        h->profile && h->sev_used + tatrg_handle::STAGE_EVENTS <= (int)h->sev.size();
    bool compressed = false, prev_failed = false;
    if (!phase_a_and_sync(h, b, rec, timed, &compressed, &prev_failed)) {
      h->err = "step: synchronisation failed";
      h->host_fault = true;
      return false;
    }
    if (prev_failed) {
      // the previous temperature-step ran without the fallback and a CholeskyQR pass failed:
      // restore this step's input, replay that step with the fallback, then start over
      const tatrg_handle::Pending p = h->pending;
      h->pending.active = false;
      h->replays += 1;
      restore_state(h, b, slot);
      const int save_step = h->step;
      h->step = p.k;
      h->states[p.b].need_fallback = true;
      restore_state(h, p.b, p.slot);
      h->speculate = false;
      double* prec = h->cfg.record_spectra ? h->spectra + (int64_t)h->step * 5 * h->d.c
                                           : nullptr;
      bool pcomp = false, dummy = false;
      if (!phase_a_and_sync(h, p.b, prec, false, &pcomp, &dummy)) {
        h->err = "step: synchronisation failed";
        h->host_fault = true;
        return false;
      }
      step_phase_b(h, p.b, prec, false, pcomp);
      h->step = save_step;
      continue;  // this temperature-step from its (restored) input
    }
    // a cell middle too ill-conditioned to compress goes with sketch panels that CholeskyQR may
    // not orthonormalise: no speculation for the rest of this step
    if (h->cfg.swap_mode == 0 && !compressed) h->speculate = false;
    step_phase_b(h, b, rec, timed, compressed);
    // the verdict of this step's CholeskyQR passes (vflags[2 + slot]) is read at the next
    // synchronisation point
    h->pending.active = true;
    h->pending.spec = spec_a || h->speculate;
    h->pending.b = b;
    h->pending.k = h->step;
    h->pending.slot = slot;
    h->speculate = false;
    h->seq += 1;
    return true;
  }
}

}  // namespace

extern "C" {

tatrg_status tatrg_step(tatrg_handle* h) {
  if (!h) return TATRG_EINVAL;
  if (!h->initialized || h->step >= h->cfg.n_steps) {
    h->err = "step called before init_tensor or after n_steps steps";
    return TATRG_ESTATE;
  }
  // the temperatures of the batch in turn, each through the whole step
  for (int b = 0; b < h->cfg.batch; ++b)
    if (!temperature_step(h, b)) break;
  select_state(h, 0);
  if (!hip_ok(h, "step")) return TATRG_EHIP;
  if (h->host_fault) return TATRG_EHIP;
  h->step += 1;
  return TATRG_OK;
}

}  // extern "C"

namespace tatrg {
// Scratch of tatrg_rsvd_noalloc: a file-scope device array, one copy per device, held until
// the process ends.  Host code never passes its name to a kernel: the device address comes
// from hipGetSymbolAddress, once per device, and is cached (noalloc_scratch).
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)36 << 17;  // 36 MiB
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
}  // namespace tatrg

namespace {

// The standalone randomized SVD on the scratch of h (P1, P2, P3, Gq, tsqr_ws, partial, flag and
// the core factors), shared by tatrg_rsvd and tatrg_rsvd_noalloc.  Arguments are validated by
// the callers.
tatrg_status standalone_rsvd(tatrg_handle* h, const double* d_A, int64_t m, int64_t n,
                             int64_t lda, int32_t k, int32_t w, int32_t q, uint64_t seed,
                             uint32_t site, double* d_U, double* d_S, double* d_Vt) {
  struct MOp : Op {
    tatrg_handle* h;
    const double* A;
    int64_t m, n, lda;
    void apply(const double* in, double* out, int w) override {
      gemm_f64(G(m, w, n, A, lda, false, in, w, false, out, w), h->st);
    }
    void apply_t(const double* in, double* out, int w) override {
      gemm_f64(G(n, w, m, A, lda, true, in, w, false, out, w), h->st);
    }
  } op;
  op.h = h;
  op.A = d_A;
  op.m = m;
  op.n = n;
  op.lda = lda;
  const uint64_t save_seed = h->cfg.seed;
  const int save_q = h->cfg.q, save_step = h->step;
  h->cfg.seed = seed;
  h->cfg.q = q;
  h->step = 0;
  rsvd(h, op, m, n, w, q, site, h->P2, h->P1, false, true);
  h->cfg.seed = save_seed;
  h->cfg.q = save_q;
  h->step = save_step;
  gemm_f64(G(m, k, w, h->P2, w, false, h->Uh, w, false, d_U, k), h->st);
  // Vt = (Qb Vh[:, :k])^T = Vh[:, :k]^T Qb^T
  gemm_f64(G(k, n, w, h->Vh, w, true, h->P1, w, true, d_Vt, n), h->st);
  hipLaunchKernelGGL(copy_small_kernel, dim3(1), dim3(64), 0, h->st, d_S, h->Sh, k);
  if (!hip_ok(h, "rsvd")) return TATRG_EHIP;
  return TATRG_OK;
}

// ---------------------------------------------------------------------------- no-alloc RSVD
constexpr int64_t NOALLOC_MAX_DIM = 8192;

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
double* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's scratch (nullptr on a HIP error).
double* noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    noalloc_ptr[dev] = static_cast<double*>(p);
  }
  return noalloc_ptr[dev];
}

// Carves the scratch for an m x n problem of width w into a handle that lives on the caller's
// stack; returns false when it does not fit.
bool carve_noalloc(tatrg_handle* h, double* base, int64_t m, int64_t n, int w) {
  Carver cv{reinterpret_cast<char*>(base)};
  const int64_t mx = std::max(m, n);
  h->P1 = cv.take((size_t)n * w);
  h->P2 = cv.take((size_t)m * w);
  h->P3 = cv.take((size_t)mx * w);
  h->Gq = cv.take(6 * (size_t)MAX_W * MAX_W);
  const size_t tq = std::max(tsqr_ws_doubles(m, w), tsqr_ws_doubles(n, w));
  h->tsqr_ws = cv.take(tq);
  h->tsqr_cap = tq;
  h->partial_doubles = 64 * (size_t)MAX_W * MAX_W;
  h->partial = cv.take(h->partial_doubles);
  h->flag = reinterpret_cast<int*>(cv.take(8));
  h->RbT = cv.take((size_t)MAX_W * MAX_W);
  h->Rb = cv.take((size_t)MAX_W * MAX_W);
  h->Uh = cv.take((size_t)MAX_W * MAX_W);
  h->Vh = cv.take((size_t)MAX_W * MAX_W);
  h->Sh = cv.take(MAX_W);
  return cv.off <= NOALLOC_SCRATCH_DOUBLES * sizeof(double);
}

}  // namespace

extern "C" {

tatrg_status tatrg_rsvd(tatrg_handle* h, const double* d_A, int64_t m, int64_t n, int64_t lda,
                        int32_t k, int32_t w, int32_t q, uint64_t seed, uint32_t site,
                        double* d_U, double* d_S, double* d_Vt) {
  if (!h || !d_A || !d_U || !d_S || !d_Vt) return TATRG_EINVAL;
  if (k < 1 || w < k || w > MAX_W || m < w || n < w || lda < n || q < 0) return TATRG_EINVAL;
  const int64_t cap = h->d.n4 * h->d.Ls;
  if (m * w > cap || n * w > cap) return TATRG_EINVAL;
  if (tsqr_ws_doubles(m, w) > h->tsqr_cap || tsqr_ws_doubles(n, w) > h->tsqr_cap)
    return TATRG_EINVAL;
  return standalone_rsvd(h, d_A, m, n, lda, k, w, q, seed, site, d_U, d_S, d_Vt);
}

tatrg_status tatrg_rsvd_noalloc(const double* d_A, int64_t m, int64_t n, int64_t lda,
                                int32_t k, int32_t w, int32_t q, uint64_t seed, uint32_t site,
                                double* d_U, double* d_S, double* d_Vt, void* stream) {
  if (!d_A || !d_U || !d_S || !d_Vt) return TATRG_EINVAL;
  if (k < 1 || w < k || w > MAX_W || m < w || n < w || lda < n || q < 0 || q > 16)
    return TATRG_EINVAL;
  if (m > NOALLOC_MAX_DIM || n > NOALLOC_MAX_DIM) return TATRG_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TATRG_EHIP;
  if (dev >= NOALLOC_MAX_DEVICES) return TATRG_EINVAL;
  double* base = noalloc_scratch(dev);
  if (!base) return TATRG_EHIP;
  // a handle on the stack: its strings and vectors stay empty, so nothing is allocated
  tatrg_handle h;
  h.cfg = tatrg_config{};
  h.st = (hipStream_t)stream;
  if (!carve_noalloc(&h, base, m, n, w)) return TATRG_EINVAL;
  return standalone_rsvd(&h, d_A, m, n, lda, k, w, q, seed, site, d_U, d_S, d_Vt);
}

namespace {
// Verifies the last temperature-step when it ran speculatively, replaying it with the
// Householder fallback when one of its CholeskyQR passes failed (see temperature_step).
bool settle(tatrg_handle* h) {
  if (!h->pending.active) return true;
  bool comp = false, failed = false;
  if (!sync_point(h, false, &comp, &failed)) return false;
  if (!failed) return true;
  const tatrg_handle::Pending p = h->pending;
  h->pending.active = false;
  h->replays += 1;
  const int save_step = h->step;
  h->step = p.k;
  h->states[p.b].need_fallback = true;
  restore_state(h, p.b, p.slot);
  h->speculate = false;
  double* rec = h->cfg.record_spectra ? h->spectra + (int64_t)h->step * 5 * h->d.c : nullptr;
  bool pcomp = false, dummy = false;
  if (!phase_a_and_sync(h, p.b, rec, false, &pcomp, &dummy)) return false;
  step_phase_b(h, p.b, rec, false, pcomp);
  h->step = save_step;
  select_state(h, 0);
  return hipStreamSynchronize(h->st) == hipSuccess;
}
}  // namespace

static tatrg_status sync_check(tatrg_handle* h) {
  if (!settle(h)) {
    h->err = "verification of the last step failed";
    return TATRG_EHIP;
  }
  if (hipStreamSynchronize(h->st) != hipSuccess) {
    h->err = "stream synchronisation failed";
    return TATRG_EHIP;
  }
  int flag = 0;
  for (const tatrg_handle::State& s : h->states) {
    int f = 0;
    if (hipMemcpy(&f, s.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      h->err = "flag readback failed";
      return TATRG_EHIP;
    }
    flag |= f;
  }
  if (flag) {
    h->err = "numerical fault on the device (non-finite norm, Cholesky pivot or trace)";
    return TATRG_ENUMERIC;
  }
  return TATRG_OK;
}

tatrg_status tatrg_lognorm(tatrg_handle* h, double* h_acc) {
  if (!h || !h_acc) return TATRG_EINVAL;
  tatrg_status s = sync_check(h);
  for (int b = 0; b < h->cfg.batch; ++b)
    if (hipMemcpy(h_acc + b, h->states[b].acc, sizeof(double), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return TATRG_EHIP;
  return s;
}

tatrg_status tatrg_free_energy(tatrg_handle* h, double* h_f, double* h_lnzv) {
  if (!h) return TATRG_EINVAL;
  if (!h->initialized || h->step != h->cfg.n_steps) {
    h->err = "free_energy needs exactly n_steps completed steps";
    return TATRG_ESTATE;
  }
  if (!settle(h)) {
    h->err = "verification of the last step failed";
    return TATRG_EHIP;
  }
  const Dims& d = h->d;
  const int nparts = 1024;
  // The last canonical form runs on copies of Phi and Psi and into a copy of the log-norm
  // accumulator (ttr[1]), so the state is left as it was: a repeated call returns the same
  // values and get_state still returns the tensor after n_steps steps.
  for (int b = 0; b < h->cfg.batch; ++b) {
    select_state(h, b);
    double* rec = h->cfg.record_spectra ? h->spectra + (int64_t)h->step * 5 * d.c : nullptr;
    if (rec)
      order_parameter(h->phi, h->psi, d.c, open_slot(h->step), h->partial, h->xrec + h->step,
                      h->st);
    copy(h->Xs, h->phi, d.n5, h->st);
    copy(h->Ys, h->psi, d.n5, h->st);
    copy(h->ttr + 1, h->acc, 1, h->st);
    double* const phi = h->phi;
    double* const psi = h->psi;
    double* const acc = h->acc;
    h->phi = h->Xs;
    h->psi = h->Ys;
    h->acc = h->ttr + 1;
    canonicalize(h, h->step, rec);
    h->phi = phi;
    h->psi = psi;
    h->acc = acc;
    // tTr = sum_f (A' S' B'^T)[f, f]
    gemm(h, G(d.n4, d.c, d.c, h->A, d.c, false, h->Smat, d.c, false, h->atf, d.c));
    hipLaunchKernelGGL(trace_partial_kernel, dim3(nparts), dim3(TPB), 0, h->st, h->atf,
                       (const double*)nullptr, h->B, d.n4, d.c, h->trace_part);
    hipLaunchKernelGGL(trace_final_kernel, dim3(1), dim3(64), 0, h->st, h->trace_part, nparts,
                       h->ttr, h->flag);
  }
  select_state(h, 0);
  if (!hip_ok(h, "free_energy")) return TATRG_EHIP;
  tatrg_status s = sync_check(h);
  const int N = h->cfg.n_steps;
  for (int b = 0; b < h->cfg.batch; ++b) {
    double t[2] = {0.0, 0.0};
    if (hipMemcpy(t, h->states[b].ttr, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess) {
      h->err = "free_energy readback failed";
      return TATRG_EHIP;
    }
    // t[1] = sum_{k=0}^{N} 2^-k ln c_k (the last canonical form added c_N), t[0] = tTr
    const double lnzv = t[1] + std::ldexp(std::log(t[0]), -N);
    const double beta = h->betas[b];
    if (h_lnzv) h_lnzv[b] = lnzv;
    if (h_f) h_f[b] = (beta > 0.0) ? -lnzv / beta : std::nan("");
  }
  return s;
}

tatrg_status tatrg_lnz_derivatives(tatrg_handle* h, double* h_lnzv, double* h_d1,
                                   double* h_d2) {
  if (!h) return TATRG_EINVAL;
  const int nb = h->cfg.batch;
  if (nb % 3 != 0) {
    h->err = "lnz_derivatives needs the batch as triples (beta - d, beta, beta + d)";
    return TATRG_EINVAL;
  }
  if (h->initialized) {
    for (int i = 0; i < nb / 3; ++i) {
      const double bm = h->betas[3 * i], b0 = h->betas[3 * i + 1], bp = h->betas[3 * i + 2];
      const double dm = b0 - bm, dp = bp - b0;
      // a symmetric triple: the central differences below are then second-order accurate
      if (!(dm > 0.0 && dp > 0.0) || std::fabs(dp - dm) > 1e-9 * (dp + dm)) {
        h->err = "lnz_derivatives: temperatures 3i, 3i+1, 3i+2 must be beta - d, beta, beta + d";
        return TATRG_EINVAL;
      }
    }
  }
  std::vector<double> l(nb);
  const tatrg_status s = tatrg_free_energy(h, nullptr, l.data());
  if (s != TATRG_OK && s != TATRG_ENUMERIC) return s;
  for (int i = 0; i < nb / 3; ++i) {
    const double bm = h->betas[3 * i], b0 = h->betas[3 * i + 1], bp = h->betas[3 * i + 2];
    const double lm = l[3 * i], l0 = l[3 * i + 1], lp = l[3 * i + 2];
    if (h_lnzv) h_lnzv[i] = l0;
    if (h_d1) h_d1[i] = (lp - lm) / (bp - bm);
    if (h_d2) h_d2[i] = 2.0 * ((lp - l0) / (bp - b0) - (l0 - lm) / (b0 - bm)) / (bp - bm);
  }
  return s;
}

tatrg_status tatrg_set_side_stream(tatrg_handle* h, int32_t on) {
  if (!h) return TATRG_EINVAL;
  if (!settle(h)) {
    h->err = "verification of the last step failed";
    return TATRG_EHIP;
  }
  h->side_off = on == 0;
  return TATRG_OK;
}

tatrg_status tatrg_autotune(tatrg_handle* h, int32_t* h_choice) {
  if (!h) return TATRG_EINVAL;
  if (h->cfg.precision != TATRG_BF16X3) {
    if (h_choice)
      for (int t = 0; t < 3; ++t) h_choice[t] = -1;
    return TATRG_OK;
  }
  if (!settle(h)) {
    h->err = "verification of the last step failed";
    return TATRG_EHIP;
  }
  // the three split GEMMs of a step at their real shapes, on the handle's scratch (their
  // inputs' values do not matter for the timing; no RG state is touched)
  const Dims& d = h->d;
  const int64_t c = d.c, n2 = d.n2, n3 = d.n3, L = d.L, w = d.Ls;
  const int64_t Kp = bf16x3_kpad(L * L), pn = c * n2 * Kp;
  uint16_t* pp = reinterpret_cast<uint16_t*>(h->P);
  const Bf16PlanesOut po = {{pp, pp + pn, pp + 2 * pn}, L, n2, L, Kp, 0, pn};
  const Bf16PlanesIn pi = {{pp, pp + pn, pp + 2 * pn}, n2 * Kp};
  uint16_t* fp = reinterpret_cast<uint16_t*>(h->FM4);
  const int64_t fn = L * n2 * bf16x3_kpad(n2);
  const Bf16PlanesIn fi = {{fp, fp + fn, fp + 2 * fn}, 0};
  const GemmArgs gP = G(c * L, L * n2, n2, h->E, n2, false, nullptr, L * n2, false, nullptr, 0);
  const GemmArgs gPhi =
      Gb(G(n2, n2, L * L, h->Qt, n2, true, nullptr, 0, false, h->phin, n2), c, 0, 0, d.n4);
  const GemmArgs gS = G(n2, c * w, n3, h->cp, n2, true, h->P2, c * w, false, h->t1, c * w);
  const int cand[6] = {0, 2, 4, 6, 8, 12};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    h->err = "autotune: event creation failed";
    return TATRG_EHIP;
  }
  bool ok = true;
  for (int t = 0; t < 3 && ok; ++t) {
    float best = 0.0f;
    int best_g = -1;
    for (int ci = 0; ci < 6 && ok; ++ci) {
      auto run = [&]() {
        if (t == 0)
          ok = ok && gemm_bf16x3(gP, h->planes, h->planes_doubles, h->st, nullptr, &fi, &po,
                                 cand[ci]);
        else if (t == 1)
          ok = ok && gemm_bf16x3(gPhi, h->planes, h->planes_doubles, h->st, nullptr, &pi,
                                 nullptr, cand[ci]);
        else
          ok = ok && gemm_bf16x3(gS, h->planes, h->planes_doubles, h->st, nullptr, nullptr,
                                 nullptr, cand[ci]);
      };
      run();  // warm-up
      hipEventRecord(e0, h->st);
      run();
      run();
      hipEventRecord(e1, h->st);
      float ms = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        ok = false;
      if (ok && (best_g < 0 || ms < best)) {
        best = ms;
        best_g = cand[ci];
      }
    }
    h->tuned_group[t] = best_g;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok || !hip_ok(h, "autotune")) {
    for (int t = 0; t < 3; ++t) h->tuned_group[t] = -1;
    if (h->err.empty()) h->err = "autotune: a split GEMM could not be launched";
    return TATRG_EHIP;
  }
  if (h_choice)
    for (int t = 0; t < 3; ++t) h_choice[t] = h->tuned_group[t];
  return TATRG_OK;
}

tatrg_status tatrg_get_record(tatrg_handle* h, int32_t b, int32_t step, int32_t which,
                              double* h_out, int32_t cap, int32_t* n_out) {
  if (!h || !h_out || !n_out || cap < 1) return TATRG_EINVAL;
  if (b < 0 || b >= h->cfg.batch || step < 0 || step > h->cfg.n_steps || which < 0 ||
      which > 6 || (which < 6 && !h->cfg.record_spectra))
    return TATRG_EINVAL;
  const tatrg_handle::State& st = h->states[b];
  if (which == 6) {  // host-side record, no synchronisation
    const int v = step < (int)st.swap_compressed.size() ? st.swap_compressed[step] : -1;
    h_out[0] = (double)v;
    *n_out = 1;
    return TATRG_OK;
  }
  tatrg_status s = sync_check(h);
  int n = 1;
  if (which == 5) {
    hipMemcpy(h_out, st.xrec + step, sizeof(double), hipMemcpyDeviceToHost);
  } else {
    n = std::min<int>(cap, h->d.c);
    hipMemcpy(h_out, st.spectra + ((int64_t)step * 5 + which) * h->d.c, sizeof(double) * n,
              hipMemcpyDeviceToHost);
  }
  *n_out = n;
  return s == TATRG_ENUMERIC ? TATRG_OK : s;
}

tatrg_status tatrg_get_spectra(tatrg_handle* h, int32_t step, int32_t which, double* h_out,
                               int32_t cap, int32_t* n_out) {
  return tatrg_get_record(h, 0, step, which, h_out, cap, n_out);
}

tatrg_status tatrg_get_state(tatrg_handle* h, double* d_phi, double* d_psi, int32_t* step,
                             double* acc) {
  if (!h || !d_phi || !d_psi) return TATRG_EINVAL;
  if (h->cfg.batch != 1) {
    h->err = "get_state / set_state need batch = 1";
    return TATRG_EINVAL;
  }
  if (!settle(h)) {
    h->err = "verification of the last step failed";
    return TATRG_EHIP;
  }
  copy(d_phi, h->phi, h->d.n5, h->st);
  copy(d_psi, h->psi, h->d.n5, h->st);
  if (step) *step = h->step;
  if (acc) {
    if (hipStreamSynchronize(h->st) != hipSuccess) return TATRG_EHIP;
    hipMemcpy(acc, h->acc, sizeof(double), hipMemcpyDeviceToHost);
  }
  if (!hip_ok(h, "get_state")) return TATRG_EHIP;
  return TATRG_OK;
}

tatrg_status tatrg_set_state(tatrg_handle* h, const double* d_phi, const double* d_psi,
                             int32_t step, double acc) {
  if (!h || !d_phi || !d_psi || step < 0 || step > h->cfg.n_steps) return TATRG_EINVAL;
  if (h->cfg.batch != 1) {
    h->err = "get_state / set_state need batch = 1";
    return TATRG_EINVAL;
  }
  if (!h->initialized) {
    h->err = "set_state needs a prior init_tensor (for beta)";
    return TATRG_ESTATE;
  }
  copy(h->phi, d_phi, h->d.n5, h->st);
  copy(h->psi, d_psi, h->d.n5, h->st);
  zero((double*)h->flag, 4, h->st);
  h->states[0].need_fallback = true;
  h->pending.active = false;
  if (hipStreamSynchronize(h->st) != hipSuccess) return TATRG_EHIP;
  hipMemcpy(h->acc, &acc, sizeof(double), hipMemcpyHostToDevice);
  h->step = step;
  if (!hip_ok(h, "set_state")) return TATRG_EHIP;
  return TATRG_OK;
}

const char* tatrg_last_error(const tatrg_handle* h) { return h ? h->err.c_str() : "null handle"; }

int tatrg_profile_enable(tatrg_handle* h, int max_launches) {
  if (!h || max_launches < 0) return -1;
  for (hipEvent_t e : h->ev) hipEventDestroy(e);
  for (hipEvent_t e : h->sev) hipEventDestroy(e);
  h->ev.clear();
  h->sev.clear();
  h->ev_used = 0;
  h->sev_used = 0;
  h->profile = max_launches > 0;
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -3;
    h->ev.push_back(e);
  }
  // stage boundaries for the steps those launches belong to (four contraction GEMMs each)
  const int steps = (max_launches + 3) / 4;
  for (int i = 0; i < steps * tatrg_handle::STAGE_EVENTS; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -3;
    h->sev.push_back(e);
  }
  const double L = h->d.L, c5 = (double)h->d.n5;
  h->flops_per_launch = 2.0 * L * L * c5;  // each of the four contraction GEMMs
  return 0;
}

int tatrg_profile_read(tatrg_handle* h, double* total_ms, int32_t* launches,
                       double* flops_per_launch) {
  if (!h || !total_ms || !launches || !flops_per_launch) return -1;
  if (hipStreamSynchronize(h->st) != hipSuccess) return -3;
  double t = 0.0;
  for (int i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) != hipSuccess) return -3;
    t += ms;
  }
  *total_ms = t;
  *launches = h->ev_used / 2;
  *flops_per_launch = h->flops_per_launch;
  h->ev_used = 0;
  return 0;
}

int tatrg_test_speculation(tatrg_handle* h, int on, int64_t* replays) {
  if (!h) return -1;
  if (on >= 0) h->force_speculation = on != 0;
  if (replays) *replays = h->replays;
  return 0;
}

int tatrg_profile_read_stages(tatrg_handle* h, double* stage_ms, int32_t* steps) {
  if (!h || !stage_ms || !steps) return -1;
  if (hipStreamSynchronize(h->st) != hipSuccess) return -3;
  constexpr int NS = tatrg_handle::STAGE_EVENTS - 1;
  for (int j = 0; j < NS; ++j) stage_ms[j] = 0.0;
  for (int i = 0; i + NS < h->sev_used; i += tatrg_handle::STAGE_EVENTS) {
    for (int j = 0; j < NS; ++j) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h->sev[i + j], h->sev[i + j + 1]) != hipSuccess) return -3;
      stage_ms[j] += ms;
    }
  }
  *steps = h->sev_used / tatrg_handle::STAGE_EVENTS;
  h->sev_used = 0;
  return 0;
}

void tatrg_destroy(tatrg_handle* h) {
  if (!h) return;
  for (hipEvent_t e : h->ev) hipEventDestroy(e);
  for (hipEvent_t e : h->sev) hipEventDestroy(e);
  if (h->st2) {
    hipStreamSynchronize(h->st2);
    hipStreamDestroy(h->st2);
  }
  for (hipEvent_t e : {h->fork_ev[0], h->fork_ev[1], h->join_ev})
    if (e) hipEventDestroy(e);
  delete h;
}

}  // extern "C"
