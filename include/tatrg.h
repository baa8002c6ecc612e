/*
 * tatrg.h - C ABI of the MI355X (gfx950) Triad-ATRG coarse-graining library.
 *
 * Method: Sugimoto & Sasaki, "Applying the Triad network representation to four-dimensional
 * ATRG method", LATTICE2024, arXiv:2412.14104.  One RG step coarse-grains the 4D Ising
 * tensor network along one direction: canonical form and bond swap of the unit cell
 * (Section 2, Eq. (1)), oversampled isometries (Eqs. (2)-(3)), triad tensors (Eqs. (4)-(11)),
 * squeezers (the squeezer cost function of Section 2) and the O(r^2 chi^7) contraction
 * (Eqs. (makeMG), (makeMH)).  Every randomized SVD uses a Gaussian sketch with q QR
 * (power) iterations (Table 1).  The partition function is Z = tTr prod T (Section 3).
 *
 * Conventions
 *  - All device pointers are HIP device memory on the device that is current when
 *    tatrg_create is called; all host pointers are ordinary host memory.
 *  - Matrices are row-major float64.  The caller owns every buffer passed in, including the
 *    workspace; the library never allocates device memory after tatrg_create returns.
 *  - Calls are asynchronous on the stream given to tatrg_create unless documented as
 *    synchronising (a step also runs work on a second stream of the handle, ordered by
 *    events, so that all of it is complete wherever the caller's stream is; see
 *    tatrg_set_side_stream).  A handle must not be used from two threads at once.
 *  - Errors: invalid arguments are reported synchronously (TATRG_EINVAL); HIP launch
 *    errors as TATRG_EHIP; numerical faults detected on the device (non-finite c_k,
 *    non-positive Cholesky pivot, non-positive final trace) set a sticky device flag that
 *    the next synchronising call reports as TATRG_ENUMERIC.  tatrg_last_error returns a
 *    message for the last failure of a handle.
 *  - Fixed thresholds of the step (not configurable; part of what a run computes, and the
 *    same in the independent CPU reference): singular values below 1e-11 s_max carry no
 *    gauge; neighbouring singular values closer than 1e-6 s_max form one degenerate cluster
 *    (at most 8 vectors), rotated to a basis fixed by 8 Philox probe vectors; squeezer modes
 *    with S < 1e-10 S_max are masked; the squeezer Grams get 1e-13 tr(rho) added to the
 *    diagonal before their Cholesky factorisation.
 */
#ifndef TATRG_H
#define TATRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TATRG_OK = 0,
  TATRG_EINVAL = -1,   /* invalid configuration or argument                         */
  TATRG_ENOMEM = -2,   /* workspace smaller than tatrg_workspace_bytes()            */
  TATRG_EHIP = -3,     /* a HIP runtime call or kernel launch failed                */
  TATRG_ENUMERIC = -4, /* device-side numerical fault (sticky until tatrg_init_tensor) */
  TATRG_ESTATE = -5    /* call out of order (e.g. step before init, past n_steps)    */
} tatrg_status;

typedef enum {
  TATRG_FP64 = 0,   /* every contraction in float64 on the FP64 MFMA units           */
  TATRG_BF16X3 = 1  /* contraction GEMMs as three-way split bf16 products with fp32
                       accumulation; QR, SVD, Cholesky and log-norms stay float64    */
} tatrg_precision;

typedef struct {
  int32_t chi;            /* bond dimension chi >= 2                                  */
  int32_t r;              /* internal-line oversampling r >= 1: L = min(r chi, chi^2)  */
  int32_t q;              /* QR (power) iterations of every randomized SVD, q >= 0     */
  int32_t n_steps;        /* RG steps N, 1 <= N <= 64; lattice of 2^N sites            */
  int32_t batch;          /* number of temperatures B, 1 <= B <= 1024 (a beta scan)    */
  int32_t precision;      /* tatrg_precision                                          */
  uint64_t seed;          /* Philox4x32-10 key for every Gaussian sketch               */
  int32_t record_spectra; /* nonzero: keep per-step singular spectra and the order
                             parameter X^(m) for readback                               */
  int32_t swap_mode;      /* bond swap: 0 = run the randomized SVD on the compressed cell
                             middle (QR factors of its two chi^3 x chi^2 panels) whenever
                             those panels are well enough conditioned, else on the full
                             middle; 1 = always on the full middle.  Both give the same
                             result up to rounding (see tatrg_step)                     */
} tatrg_config;

typedef struct tatrg_handle tatrg_handle;

/* Bytes of device workspace the configuration needs; 0 for an invalid configuration. */
size_t tatrg_workspace_bytes(const tatrg_config* cfg);

/* Validate cfg, carve the caller's workspace d_ws (>= tatrg_workspace_bytes bytes, 256-byte
 * aligned) and bind the HIP stream `stream` (a hipStream_t; NULL = default stream).
 * Returns EINVAL for a bad configuration, ENOMEM for a short workspace.  *out receives the
 * handle; release it with tatrg_destroy (which does not free d_ws). */
tatrg_status tatrg_create(const tatrg_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                          tatrg_handle** out);

/* Build the initial tensor T = sum_a prod W[a,i] prod W[a,j] from beta (Section 3, the
 * definitions of T and W; W is the element-wise square root of the printed matrix so that
 * W W^T is the bond Boltzmann weight) and reset the step counter and log-norm accumulator.
 * h_betas: host array of `batch` values, each finite and >= 0.  Asynchronous. */
tatrg_status tatrg_init_tensor(tatrg_handle* h, const double* h_betas);

/* One RG step on the device: canonical form and normalisation c_k = |T|_F, bond swap by
 * randomized SVD, isometries, triad tensors, squeezers, contraction and slot rotation
 * (Section 2).  With swap_mode = 0 the bond swap factors the two panels of the cell middle
 * M = sum_x A~_x B~_x^T by a two-pass Cholesky QR and runs the randomized SVD on the
 * chi^3 x chi^3 middle K between their triangular factors, with the sketch mapped through
 * the orthonormal factor; the one host synchronisation of the step reads the device's
 * verdict on the panels' conditioning, and ill-conditioned panels (the first steps, beta = 0)
 * take the full middle instead.  With swap_mode = 1 no host synchronisation happens.  With batch = B the step runs for every
 * temperature in turn; all temperatures share the same Gaussian sketches (common random
 * numbers), so entry b of a batch equals a batch-1 run at beta_b bit for bit.  With
 * record_spectra it first records X^(k) of the incoming tensor (see tatrg_get_record).
 * ESTATE before init or after n_steps steps. */
tatrg_status tatrg_step(tatrg_handle* h);

/* Standalone randomized SVD A ~= U diag(S) V^T of a device matrix (Introduction, Table 1):
 * Gaussian sketch of width w drawn from (seed, step = 0, site), q QR iterations, rank k.
 * d_A: m x n row-major with leading dimension lda >= n (read only).  Outputs (device):
 * d_U m x k, d_S k, d_Vt k x n (all row-major, dense).  Requires 1 <= k <= w <= min(m, n),
 * w <= 96.  Uses the handle's workspace, so m*w and n*w must not exceed chi^4 * Ls of the
 * handle's configuration (Ls = min(r chi, chi^4), the swap sketch width), and the panel
 * workspace of the Householder fallback must fit (EINVAL otherwise).  Asynchronous. */
tatrg_status tatrg_rsvd(tatrg_handle* h, const double* d_A, int64_t m, int64_t n, int64_t lda,
                        int32_t k, int32_t w, int32_t q, uint64_t seed, uint32_t site,
                        double* d_U, double* d_S, double* d_Vt);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): tatrg_rsvd without a handle.  Same operation,
 * arguments and outputs as tatrg_rsvd (with q <= 16), on the stream `stream` (a hipStream_t,
 * NULL = default), for m, n <= 8192.  Its scratch (panels, factor workspace, partial sums,
 * flags; 36 MiB) is a static device array of the library, one per device, held until the
 * process ends; no device or host memory is allocated.  Every call on a device shares that
 * device's scratch: calls that overlap on one device (two streams, two threads) race, so
 * order them.  EINVAL for sizes beyond the limits or invalid arguments (nothing launched),
 * EHIP when the scratch's device address cannot be obtained.  Asynchronous. */
tatrg_status tatrg_rsvd_noalloc(const double* d_A, int64_t m, int64_t n, int64_t lda,
                                int32_t k, int32_t w, int32_t q, uint64_t seed, uint32_t site,
                                double* d_U, double* d_S, double* d_Vt, void* stream);

/* Synchronising.  h_acc[b], b < batch, receives the log-norm accumulator
 * sum_{j<k} 2^-j ln c_j after k steps, where c_j = |T_j|_F is the norm taken out of the
 * tensor at the canonical form of step j (Section 2, canonical form; Section 3, Z = tTr prod T
 * on a lattice of 2^k sites, each normalisation of T_j counting for 2^-j of a site).
 * Returns ENUMERIC when a device-side numerical fault has been flagged (the values are still
 * copied out). */
tatrg_status tatrg_lognorm(tatrg_handle* h, double* h_acc);

/* Synchronising; valid after n_steps steps (ESTATE otherwise).  The partition function of
 * the periodic lattice is Z = tTr prod T (Section 3): the last tensor is normalised once more
 * (c_N) and traced on the 1x1x1x1 periodic lattice, so
 *   ln Z / V = sum_{k=0}^{N} 2^-k ln c_k + 2^-N ln tTr,    f = -(ln Z / V) / beta
 * (the free energy per site of Table 2).  The final normalisation works on copies, so the
 * RG state is left unchanged: a repeated call returns the same values and get_state still
 * returns the tensor after n_steps steps.  h_f and h_lnzv (host, `batch` entries each;
 * either may be NULL).  f is NaN at beta = 0.  ENUMERIC when a fault has been flagged
 * (including a non-positive final trace). */
tatrg_status tatrg_free_energy(tatrg_handle* h, double* h_f, double* h_lnzv);

/* Synchronising; valid after n_steps steps (ESTATE otherwise), on a handle whose batch holds
 * triples of temperatures (beta_i - d_i, beta_i, beta_i + d_i), i = 0 .. batch/3 - 1, in
 * that order (tatrg_init_tensor; EINVAL for a batch that is not a multiple of 3 or a triple
 * that is not symmetric to 1e-9 of its spacing).  The derivatives of ln Z / V (Section 3,
 * Z = tTr prod T with the bond weight e^{beta s s'} of W) in beta by central differences:
 *   h_d1[i] = (L+ - L-) / (2 d_i)                      u = -h_d1 is the internal energy per site
 *   h_d2[i] = (L+ - 2 L0 + L-) / d_i^2 (nonuniform form)  c = beta^2 h_d2 is the specific heat
 * with L = ln Z / V of the three runs, and h_lnzv[i] = L0.  The Gaussian sketches do not
 * depend on beta, so the three runs share them and ln Z / V of the truncated RG is a smooth
 * function of beta between changes of the truncation; with d ~ 1e-4 the difference error
 * is ~d^2 of the third derivative and the rounding error ~1e-15 / d.  Output arrays (host,
 * batch / 3 entries each) may be NULL.  Leaves the state unchanged (as tatrg_free_energy);
 * ENUMERIC when a fault has been flagged. */
tatrg_status tatrg_lnz_derivatives(tatrg_handle* h, double* h_lnzv, double* h_d1,
                                   double* h_d2);

/* Between steps (verifies a pending step first).  The step puts work that does not depend on
 * the latency-bound factorisations around it on a second stream of the handle (created at the
 * first step, default priority, ordered by events): the bond swap's sketch and its map through
 * the first orthonormal factor of the panels, Eq. (1), beside their Cholesky chains, and the
 * semidefinite factors of the isometries and squeezers beside Grams that do not need them.
 * on = 0 runs that work in order on the handle's own stream instead (for a process that
 * already runs several handles at once, where the extra streams only compete for hardware
 * queues), on != 0 restores the default.  Results are the same bit for bit either way.
 * EINVAL for a null handle, EHIP on a HIP error. */
tatrg_status tatrg_set_side_stream(tatrg_handle* h, int32_t on);

/* Synchronising; between steps.  A measured table for the split-bf16 GEMMs of the step (the
 * contraction of Eqs. (makeMG)/(makeMH): P = E.FM4 and Phi = Qt^T.P, and the bond swap's
 * sketch map, Eq. (1)): each is timed at its real shape on the handle's scratch for
 * work-group orders grouping 0, 2, 4, 6, 8 or 12 rows of tiles (which of the tiles run
 * together, and so share operand tiles in an XCD's L2), and the fastest is kept for the
 * following steps.  The order does not change any result: runs are bit for bit those without
 * tuning.  No RG state is touched.  h_choice (host, 3 ints, may be NULL) receives the chosen
 * groupings of the three GEMMs in that order (-1 each on the FP64 path, where the call does
 * nothing).  EHIP on a HIP error, the defaults then stay in use. */
tatrg_status tatrg_autotune(tatrg_handle* h, int32_t* h_choice);

/* Synchronising.  Per-step records of temperature b (0 <= b < batch), kept when
 * record_spectra != 0, for step = 0..n_steps (step n_steps is recorded by
 * tatrg_free_energy):
 *   which = 0: canonical s (chi values), 1: swap sigma (chi), 2/3/4: squeezer S of
 *   direction mu = 2/3/4 (chi);
 *   which = 6: the bond swap's path at that step: 1 (compressed middle), 0 (full middle),
 *   -1 (not run yet); available without record_spectra, no synchronisation;
 *   which = 5: the order parameter X^(step) = (Tr A)^2 / Tr A^2 of the incoming tensor, with
 *   A_kl = T summed over the forward = backward legs of three directions and the legs k, l
 *   of lattice direction 4 open (Section 3, the order parameter of the transition point;
 *   one value).
 * Copies min(cap, chi) values (one for which = 5, 6) to h_out and the count to *n_out.
 * EINVAL without record_spectra (which < 6), for b, step or which out of range, or cap < 1.  A flagged
 * numerical fault is NOT reported here (the call returns OK and copies the records as they
 * are, so the steps before a fault can be inspected); tatrg_lognorm and tatrg_free_energy
 * report it. */
tatrg_status tatrg_get_record(tatrg_handle* h, int32_t b, int32_t step, int32_t which,
                              double* h_out, int32_t cap, int32_t* n_out);

/* tatrg_get_record of temperature 0. */
tatrg_status tatrg_get_spectra(tatrg_handle* h, int32_t step, int32_t which, double* h_out,
                               int32_t cap, int32_t* n_out);

/* Checkpoint / resume of the RG state (Phi, Psi, step index, log-norm accumulator); batch = 1
 * only (EINVAL otherwise).
 * d_phi, d_psi: device buffers of chi^5 doubles each, legs (l1,l2,l3,l4,gamma) row-major with
 * T = sum_g Phi[..,g] Psi[..,g].  get copies out, set copies in (asynchronous).  set also
 * clears the sticky numerical flag. */
tatrg_status tatrg_get_state(tatrg_handle* h, double* d_phi, double* d_psi, int32_t* step,
                             double* acc);
tatrg_status tatrg_set_state(tatrg_handle* h, const double* d_phi, const double* d_psi,
                             int32_t step, double acc);

/* Message describing the last failure on h (never NULL; "" when none). */
const char* tatrg_last_error(const tatrg_handle* h);

/* Release the handle (not the workspace). */
void tatrg_destroy(tatrg_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* TATRG_H */
