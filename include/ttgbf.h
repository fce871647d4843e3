/*
 * ttgbf.h -- C ABI of the MI355X (gfx950) tensor-train grid-based filter.
 *
 * The library implements one Bayesian recursion step of the point-mass
 * filter with every density held in tensor-train (TT) format:
 *   prediction  = per-core convolution of the PMD TT with a TT transition
 *                 kernel (Sec. 2.1 "Tensor Form", eq. tpmconvFFT; Sec. 4.2
 *                 "FFT Convolution in Tensor Train"),
 *   update      = Hadamard product with a TT likelihood and the normaliser
 *                 c_k (Sec. 2.2, eqs. pmf_filtrace_a/b; Sec. 4.1 'times'),
 *   rounding    = orthogonalisation sweep + truncated-SVD sweep capping the
 *                 ranks (Sec. 3.2, Sec. 4.1 'round'),
 *   moments     = full TT contractions (Sec. 4.1 'sum', 'power', 'dot').
 * The step order is that of Alg. 2 with the convolution prediction of
 * Alg. 3 (fixed grid, f = identity).
 *
 * Conventions shared by every entry point
 *   - All pointers named *_dev and every pointer inside tt_train point to
 *     device memory owned by the caller.  The library never allocates device
 *     memory; scratch comes from the caller's workspace (ws, ws_bytes), whose
 *     required size the matching *_workspace query returns.  Host pointers
 *     (descriptors, q, halfwidths) are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is enqueued asynchronously; results are valid after the stream
 *     is synchronised.  Calls are reentrant given distinct workspaces.
 *     Descriptor tables reach the device through a page-locked ring the
 *     library keeps per process (64 MB, allocated on the first call that
 *     uploads; its regions are reused only after their copies completed),
 *     so the uploads do not wait on the stream; the calls marked
 *     synchronous below wait for their own reasons (host reads of ranks or
 *     boxes).
 *   - Return value: TT_OK, or an argument/shape/workspace/HIP error detected
 *     on the host BEFORE anything is enqueued (TT_ERR_HIP is returned when a
 *     launch fails; tt_last_error() then holds the message).
 *   - Numerical failures are reported per TT in its device status word
 *     (sticky bit flags TT_STATUS_*); a failed filter's later outputs are NaN
 *     and other filters in a batch are unaffected.
 */
#ifndef TTGBF_H
#define TTGBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAXD 16

typedef int32_t tt_status;
#define TT_OK 0
#define TT_ERR_ARG 1        /* null pointer, non-positive size, bad enum */
#define TT_ERR_SHAPE 2      /* inconsistent d, n, capacities */
#define TT_ERR_WORKSPACE 3  /* workspace smaller than the query returns */
#define TT_ERR_HIP 4        /* a HIP call failed; see tt_last_error() */

/* Per-TT device status bits (sticky; OR-ed by the kernels). */
#define TT_STATUS_NONPOSITIVE 1  /* mass or c_k <= 0 */
#define TT_STATUS_NONFINITE 2    /* NaN/Inf met */
#define TT_STATUS_CAPACITY 4     /* a rank needed more room than reserved */

typedef enum { TT_F64 = 0, TT_F32 = 1 } tt_dtype;

/* Equidistant grid (Sec. 2 eq. pdf_pm; Sec. 4 grid bullet): axis l holds
 * n[l] points lo[l] + i*(hi[l]-lo[l])/(n[l]-1), i = 0..n[l]-1. */
typedef struct {
  int32_t d;
  int32_t n[TT_MAXD];
  double lo[TT_MAXD];
  double hi[TT_MAXD];
} tt_grid;

/* One tensor train on the device (Sec. 3.1 eq. ttd_exact):
 *   A(i_1..i_d) = exp(*log_scale) * G_1(:,i_1,:) ... G_d(:,i_d,:).
 * Core k is stored at element offset off_k = sum_{j<k} cap[j]*n[j]*cap[j+1]
 * of `cores` (elements of `dtype`), packed with the CURRENT ranks r = ranks[]
 * in row-major layout [r_{k-1}][n_k][r_k]; cap[] reserves the room
 * (cap[0] = cap[d] = 1).  ranks, log_scale and status live on the device and
 * are updated by the kernels without host synchronisation. */
typedef struct {
  int32_t d;
  int32_t n[TT_MAXD];
  int32_t cap[TT_MAXD + 1];
  int32_t dtype;            /* tt_dtype */
  void* cores;              /* device, tt_train_elems(...) elements */
  int32_t* ranks;           /* device int32[d+1] */
  double* log_scale;        /* device double[1] */
  int32_t* status;          /* device int32[1] */
} tt_train;

/* Measurement model (Sec. 1 eq. asz with Gaussian v):
 *   kind 0: z_l = x_l + v_l on every axis, v ~ N(0, sigma_lin^2 I);
 *   kind 1: z_0 = ||(x_1,x_2) - sensor|| + v_0 (v_0 ~ N(0, sigma_r^2)) and
 *           z_j = x_{j+1} + v_j for j = 1..d-2 (v_j ~ N(0, sigma_lin^2)).
 * The likelihood tensor (Sec. 2.2 L^v, Sec. 4 tensor bullet) is held as a
 * TT: rank one on the linear axes; the (x_1,x_2) block is a dense matrix
 * truncated by SVD at relative Frobenius tolerance lik_tol (and to at most
 * lik_max_rank terms when that is > 0). */
typedef struct {
  int32_t kind;
  double sensor[2];
  double sigma_r;
  double sigma_lin;
  double lik_tol;
  int32_t lik_max_rank;
} tt_meas;

/* Number of elements a TT with these capacities needs. */
size_t tt_train_elems(int32_t d, const int32_t* n, const int32_t* cap);

/* Message of the last host-side error in this thread (never NULL). */
const char* tt_last_error(void);

/* Static description of a tt_status return code (never NULL). */
const char* tt_status_string(int32_t code);

/* Static description of a combination of TT_STATUS_* device bits (never NULL). */
const char* tt_device_status_string(int32_t bits);

/* Library version string. */
const char* tt_version(void);

/* ---------------------------------------------------------------------
 * tt_kernel_build -- TT transition kernel (Sec. 2.1 eq. TPMmat and the
 * middle-row tensor of eq. tpmconvFFT; Sec. 3.1 TT decomposition).
 *   K(m) = N(Delta o m; 0, Q) * delta   for |m_l| <= halfwidths[l],
 * Delta_l = (hi_l-lo_l)/(n_l-1), delta = prod Delta_l, evaluated densely on
 * the device in FP64 and decomposed by TT-SVD (sequential truncated SVDs,
 * per-bond threshold svd_tol*||K||_F/sqrt(d-1)).
 *   grid        host; d <= 8 and prod(2h_l+1) <= 2^28 (dense build)
 *   q           host, d*d row-major, symmetric positive definite
 *   halfwidths  host, d entries h_l >= 0
 *   out         TT with n[l] = 2*h_l+1 and rank capacities cap[]; dtype
 *               TT_F64 or TT_F32 (the decomposition is FP64 either way).
 *               On return (after sync) out->ranks holds the kernel ranks;
 *               TT_STATUS_CAPACITY is set if a rank exceeded cap.
 * --------------------------------------------------------------------- */
size_t tt_kernel_build_workspace(const tt_grid* grid, const int32_t* halfwidths,
                                 const int32_t* cap);
tt_status tt_kernel_build(const tt_grid* grid, const double* q, const int32_t* halfwidths,
                          double svd_tol, const tt_train* out, void* ws, size_t ws_bytes,
                          void* stream);
/* tt_kernel_build_batch -- the same build for `batch` kernels at once (one
 * launch per step for all of them).  grids[batch] and q[batch*d*d] may
 * differ per kernel; d and the offset box (halfwidths, d entries) are
 * shared; out[batch] may have different capacities but one dtype.
 * Workspace: tt_kernel_build_batch_workspace(batch, grids, halfwidths,
 * caps) with caps[b*(d+1) + j] = out[b].cap[j]; it holds two dense kernels
 * per filter (batch * prod(2h_l+1) doubles each). */
size_t tt_kernel_build_batch_workspace(int32_t batch, const tt_grid* grids, const int32_t* halfwidths,
                                       const int32_t* caps);
tt_status tt_kernel_build_batch(int32_t batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                double svd_tol, const tt_train* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_kernel_build_cross -- the transition kernel of tt_kernel_build without
 * the dense tensor, for any d (the d = 10, 41-tap kernel has 1.3e16
 * entries): K(m) is evaluated point by point and approximated by a
 * deterministic TT-cross (Sec. 3.3 cross approximation; maxvol pivots in
 * place of the paper's randomised greedy cross): alternating sweeps over
 * the cores, each fibre matrix f(I_{<k}, i_k, J_{>k}) reduced to an
 * orthonormal basis of its range (the library's rounding of a two-core
 * train; only exactly dependent columns are dropped), maxvol rows of that
 * basis as the next index set, the cores in interpolation form; at each
 * rank level sweeps until the rounded result's ranks stop moving (two to
 * six), the rank starting at 8 and doubling up to max_rank (and to at most
 * 4096 / the largest mode size) until the rounded ranks have room (2 below
 * the rank used, or the bond's full rank) and equal those of the previous
 * level.  The result is rounded
 * (Sec. 4.1 'round') at svd_tol into out.  Synchronous (reads ranks after
 * each level).
 *   grids, q, halfwidths, out  as tt_kernel_build_batch (d <= TT_MAXD,
 *              2 h_l + 1 <= 4096 taps); out FP64 or FP32, its capacities
 *              bound the result's ranks (TT_STATUS_CAPACITY when a rank
 *              needs more).
 *   max_rank   in [1, 64]: the working rank of the cross, not the result's
 *              cap; a search stopped by it before the ranks have room is
 *              not converged, so it should exceed the expected ranks by 2.
 * Workspace: tt_kernel_build_cross_workspace(batch, grids, halfwidths, out).
 * Errors: TT_ERR_ARG (null, svd_tol <= 0, max_rank out of range, Q not
 * positive definite), TT_ERR_SHAPE, TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_kernel_build_cross_workspace(int32_t batch, const tt_grid* grids, const int32_t* halfwidths,
                                       const tt_train* out);
tt_status tt_kernel_build_cross(int32_t batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                double svd_tol, int32_t max_rank, const tt_train* out, void* ws, size_t ws_bytes,
                                void* stream);

/* ---------------------------------------------------------------------
 * tt_interpolate_lattice -- the second interpolation of Alg. 3: for linear
 * dynamics the temporary predictive lives on the lattice x(j) = F xi(j) of
 * an axis-aligned grid `lattice` (the time update's convolution grid); it
 * is interpolated onto the axis-aligned grid `to` (the smallest box holding
 * the lattice's corners, Alg. 3 and Alg. 4):
 *   out(i) = sum over the 2^d lattice neighbours j of u of
 *            prod_l (1 - |u_l - j_l|) in(j),   u = (F diag dx)^{-1} (x(i) - F lo)
 * with dx, lo the lattice grid's spacing and lower corner, x(i) the point i
 * of `to`, and zero for a neighbour off the lattice.  The result couples
 * the axes, so it is built by the TT-cross of tt_kernel_build_cross from
 * point values of the interpolant (each a sum of 2^d point values of `in`)
 * and rounded at tol with out's capacities; out's log_scale is in's plus
 * the rounding's.
 *   f          d x d row-major, host, shared by the batch (invertible)
 *   lattice[b], to[b]  host grids of filter b (2 <= d <= 6; every `to`
 *              grid has the same point counts)
 *   in[b]      FP64 on lattice's modes, rank capacities <= 32
 *   out[b]     FP64 or FP32 on to's modes; max_rank in [1, 64] bounds the
 *              cross (and 4096 / the largest point count)
 * Synchronous.  Workspace: tt_interpolate_lattice_workspace(batch, to, out,
 * max_rank).  Errors: TT_ERR_ARG (null, tol <= 0, F singular),
 * TT_ERR_SHAPE, TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_interpolate_lattice_workspace(int32_t batch, const tt_grid* to, const tt_train* out, int32_t max_rank);
tt_status tt_interpolate_lattice(int32_t batch, const double* f, const tt_grid* lattice, const tt_grid* to,
                                 const tt_train* in, double tol, int32_t max_rank, const tt_train* out, void* ws,
                                 size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_predict -- Chapman-Kolmogorov prediction for x_{k+1} = x_k + w_k as
 * the linear convolution of the PMD with the kernel, cropped to the grid
 * (Sec. 2.1 eq. tpmconvFFT; Sec. 4.2: the cores of a TT convolution are the
 * convolutions of the cores).  For every filter b and core k:
 *   C_k(a*rp+b', i, a'*rp'+b'') = sum_{m=-h_k}^{h_k} K_k(a, m+h_k, a') P_k(b', i-m, b'')
 * with P = 0 off the grid and h_k = (kernel n_k - 1)/2.  The product is NOT
 * rounded: out ranks are r_K * r_P; out->cap must be >= kernel cap * in cap.
 * log_scale(out) = log_scale(kernel) + log_scale(in).
 *   batch      number of filters; kernels[b], p_in[b], p_out[b] describe
 *              filter b (kernels[] entries may describe the same TT).
 * --------------------------------------------------------------------- */
size_t tt_predict_workspace(int32_t batch);
tt_status tt_predict(int32_t batch, const tt_train* kernels, const tt_train* p_in,
                     const tt_train* p_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_predict_einsum -- Chapman-Kolmogorov prediction with a general
 * transition tensor by Einstein summation (Sec. 4.2, eqs. ttConvolutionP,
 * ttConvolutionZ, ttConvolutionM, ttConvolutionZrecursion; Alg. 1):
 *   P'(i_1..i_d) = sum_{j_1..j_d} T(i_1..i_d, j_1..j_d) P(j_1..j_d)
 * with T a TT of 2d cores (cores 0..d-1 over the predicted grid, cores
 * d..2d-1 over the current grid, mode sizes n[k] = n[d+k] = the density's)
 * and P a d-core TT.  P' keeps T's first d-1 cores; its core d-1 is
 * T_{d-1} x_3 Z with Z built backwards over T's second half from Z = 1:
 *   Z'(a, c) = sum_{i, b, e} T_{d+k}(a, i, b) P_k(c, i, e) Z(b, e).
 * Out ranks are T's ranks 0..d-1 and 1; log_scale(out) = log_scale(tpm) +
 * log_scale(in); status(out) = status(in).  Sums in FP64 whatever the
 * storage type; all trains of a call share one dtype and one d (2d <= 16).
 *   tpm[b], p_in[b], p_out[b]  filter b (tpm entries may describe one TT);
 *              p_out->cap[k] >= tpm->cap[k] for k < d.
 * Workspace: tt_predict_einsum_workspace(batch, tpm, p_in) bytes (per
 * filter max_k cap'_k n_k cap_{d+k+1} + 2 max_k cap_{d+k} cap'_k doubles).
 * Errors: TT_ERR_ARG (null), TT_ERR_SHAPE (d, modes or capacities
 * inconsistent), TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_predict_einsum_workspace(int32_t batch, const tt_train* tpm, const tt_train* p_in);
tt_status tt_predict_einsum(int32_t batch, const tt_train* tpm, const tt_train* p_in, const tt_train* p_out,
                            void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_grid_redesign -- the grid re-design of Alg. 4 (used twice by Alg. 3):
 * per filter, the local Kalman prediction of the filtering moments
 * m' = F m, P' = F P F^T + Q, the predictive box m' +- nsigma sqrt(P'_ll),
 * and the new filtering grid: the smallest axis-aligned box holding the
 * box's 2^d corners mapped by F^{-1} (computed as F^{-1} m' +- |F^{-1}| h),
 * with the old grid's number of points per axis.
 *   f, q       d x d row-major, host, shared by the batch (F invertible)
 *   mean_dev   device [batch*d], cov_dev device [batch*d*d] (the outputs of
 *              tt_normalize_moments)
 *   old_grids  host [batch]; new_grids host [batch], written (n copied)
 * Synchronous (returns after the boxes are on the host).  Workspace:
 * tt_grid_redesign_workspace(batch, d).  Errors: TT_ERR_ARG (null, nsigma
 * <= 0, F singular, a degenerate or non-finite box), TT_ERR_SHAPE (a grid's
 * d differs), TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_grid_redesign_workspace(int32_t batch, int32_t d);
tt_status tt_grid_redesign(int32_t batch, int32_t d, const double* f, const double* q, double nsigma,
                           const double* mean_dev, const double* cov_dev, const tt_grid* old_grids,
                           tt_grid* new_grids, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_interpolate -- multilinear interpolation of a TT density onto a new
 * axis-aligned grid (Sec. 4.2, interpolation on the level of the cores;
 * Alg. 3 and Alg. 4): every core is contracted with its axis' two-tap
 * linear interpolation operator,
 *   out_k(a, i', b) = (1 - t) in_k(a, j, b) + t in_k(a, j + 1, b)
 * where x_j <= x'_{i'} <= x_{j+1} on the old axis, and zero where x'_{i'}
 * is off the old grid.  Grid points are lo + (hi - lo) i / (n - 1).  Out
 * ranks, log_scale and status are in's; mass is not renormalised.
 *   from[b], to[b]  host grids of filter b (from = in's grid, to = out's;
 *              n >= 2 per axis); in[b], out[b] one dtype, out->cap >= in's.
 * Workspace: tt_interpolate_workspace(batch).  Errors: TT_ERR_ARG,
 * TT_ERR_SHAPE (grids, modes or capacities inconsistent),
 * TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_interpolate_workspace(int32_t batch);
tt_status tt_interpolate(int32_t batch, const tt_grid* from, const tt_grid* to, const tt_train* in,
                         const tt_train* out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_update -- Bayes update (Sec. 2.2 eqs. pmf_filtrace_a/b; the update of Alg. 2):
 * builds the likelihood TT for measurement z (FP64, max-shifted, its log
 * shift added to the log-scale), forms H = L o P_pred as the Kronecker
 * product of the core slices (Sec. 4.1 'times'; ranks multiply) and
 *   log_c_dev[b] = log( sum_i L(i) P_pred(i) * delta )
 * on the unrounded product.  H is not rounded or normalised.
 *   grids[b], meas[b]  host descriptors per filter
 *   z_dev              device FP64, filter b's measurement at z_dev + b*z_stride
 *   h_out              capacity >= (likelihood rank cap) * p_pred cap on bond 1,
 *                      >= p_pred cap elsewhere; lik_rank_cap bounds r_L.
 * --------------------------------------------------------------------- */
size_t tt_update_workspace(int32_t batch, const tt_grid* grids, const tt_meas* meas,
                           const tt_train* p_pred, const tt_train* h_out, int32_t lik_rank_cap);
tt_status tt_update(int32_t batch, const tt_grid* grids, const tt_meas* meas,
                    const double* z_dev, int32_t z_stride, const tt_train* p_pred,
                    const tt_train* h_out, int32_t lik_rank_cap, double* log_c_dev,
                    void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_round -- TT rounding (Sec. 3.2 maximum rank; Sec. 4.1 'round'):
 * in exact arithmetic the result is that of a right-to-left orthogonalisation
 * followed by a left-to-right sweep of truncated SVDs keeping at bond k the
 * smallest r whose discarded tail sqrt(sum_{j>r} s_j^2) <= eps*||A||_F/sqrt(d-1),
 * then r = min(max(r,1), max_rank).  The orthogonalisation is computed from
 * Gram matrices accumulated in double-double (FP64 TTs) or FP64 (FP32 TTs)
 * with pivoted Cholesky factors that drop directions below a relative
 * pre-truncation threshold (1e-15 for FP64, 1e-7 for FP32 TTs); the small
 * SVDs are one-sided Jacobi in FP64.  After rounding the last core is scaled
 * to unit Frobenius norm and its norm moved into log_scale.
 *   t_in, t_out  may be the same TT (in place); t_out->cap bounds the ranks
 *                (capacity overflow sets TT_STATUS_CAPACITY).
 * --------------------------------------------------------------------- */
size_t tt_round_workspace(int32_t batch, const tt_train* t_in, const tt_train* t_out);
tt_status tt_round(int32_t batch, const tt_train* t_in, const tt_train* t_out, double eps,
                   int32_t max_rank, void* ws, size_t ws_bytes, void* stream);

/* tt_round_taped -- tt_round (FP64 trains only) that also records, per
 * filter, the products of its two sweeps that tt_round_adjoint would
 * otherwise recompute.  valid[j] is a bit set per bond j = 1..d-1:
 *   1: g[j] = the Gram matrix G of the right part of the input at bond j
 *      (r_j x r_j, r_j = the input's rank there, row-major, leading
 *      dimension r_j) and f[j] = its pivoted Cholesky factor F (G ~ F F^T,
 *      rows in the original order, r_j x r_j, columns beyond its rank zero),
 *      rank[j] = the factor's rank;
 *   2: bond 1 wider than n[0], which the sweep folds with core 0: g[1], f[1]
 *      = the Gram of the folded n[0] x (n[1] r_2) unfolding (n[0] x n[0],
 *      leading dimension n[0]) and its factor, rank[1] its rank (not
 *      recorded when n[0] exceeds 256);
 *   4: v[j], s[j] = the singular vectors and values of the left-to-right
 *      step that ends at bond j (the unfolding of output core j-1 in the
 *      coordinates of F at bond j): vector c in column c of v[j] (r_j x r_j,
 *      column-major, leading dimension r_j), s[j] descending, zeros beyond
 *      the rank (not recorded for the folded bond 1).
 * Caller-owned device buffers: g[j], f[j], v[j] of c_j^2 doubles and s[j]
 * of c_j doubles with c_j = in->cap[j] (c_1 = min(in->cap[1], n[0]): a
 * bond 1 of rank above n[0] is folded), valid and rank of d+1 int32 each. */
typedef struct {
  double* g[TT_MAXD];
  double* f[TT_MAXD];
  double* v[TT_MAXD];
  double* s[TT_MAXD];
  int32_t* valid;
  int32_t* rank;
} tt_round_tape;
tt_status tt_round_taped(int32_t batch, const tt_train* t_in, const tt_train* t_out, double eps,
                         int32_t max_rank, const tt_round_tape* tape, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_normalize_moments -- mass, normalisation and moments (Sec. 4.1 'sum',
 * 'mrdivide', 'power', 'dot'; the normalisation of Alg. 2), for rank capacities <= 64:
 *   mass = sum_i A(i) * delta,  log_mass_dev[b] = log(mass) (before),
 *   log_scale -= log(mass)  (A now integrates to one),
 *   mean_dev[b*d + l]       = sum_i xi_l(i_l) A(i) delta,
 *   cov_dev[b*d*d + l*d + j] = sum_i xi_l xi_j A(i) delta - mean_l mean_j.
 * mean_dev and cov_dev may be NULL.  Contractions accumulate in FP64.
 * --------------------------------------------------------------------- */
tt_status tt_normalize_moments(int32_t batch, const tt_grid* grids, const tt_train* t,
                               double* log_mass_dev, double* mean_dev, double* cov_dev,
                               void* ws, size_t ws_bytes, void* stream);
size_t tt_normalize_moments_workspace(int32_t batch, const tt_train* t);

/* ---------------------------------------------------------------------
 * tt_normalize_moments_noalloc -- tt_normalize_moments for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, bitwise, with the workspace replaced by a static device array of
 * TT_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  The caller still owns t and the outputs.
 * The call allocates nothing (no hipMalloc/hipFree, no allocating library
 * routine); its first call on a device looks the array's address up with
 * that device current.  Every call on a device shares that device's array
 * and leaves its contents behind: calls that overlap on one device (several
 * streams or host threads) race and must be serialised by the caller.  The
 * descriptor upload does not use the library's upload ring: it copies from
 * the call's own host memory and synchronises `stream`.
 * Errors: as tt_normalize_moments; TT_ERR_WORKSPACE when batch, d and the
 * rank capacities need more than TT_NOALLOC_SCRATCH_BYTES (the message
 * gives both sizes), TT_ERR_HIP when the device or the array's address
 * cannot be queried.
 * --------------------------------------------------------------------- */
#define TT_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
tt_status tt_normalize_moments_noalloc(int32_t batch, const tt_grid* grids, const tt_train* t,
                                       double* log_mass_dev, double* mean_dev, double* cov_dev, void* stream);

/* ---------------------------------------------------------------------
 * Adjoints (reverse-mode derivatives) of the linear steps.
 *
 * Convention: a TT is its stored cores times exp(log_scale).  An adjoint
 * train has its primal's modes and ranks (the library sets its ranks from
 * the primal); its cores hold the derivative of the caller's scalar with
 * respect to the primal's stored cores and its log_scale field holds the
 * derivative with respect to the primal's log-scale.  Its status word is
 * set to TT_STATUS_CAPACITY when a rank does not fit its capacity or the
 * incoming adjoint's ranks do not match (the cores are then not written),
 * else 0.  All sums are FP64 in a fixed order.  Workspace:
 * tt_adjoint_workspace(batch, d, largest rank capacity) bytes, used for the
 * uploaded descriptors (and the sum environments of tt_normalize_adjoint);
 * the calls are asynchronous on stream, like the forward calls.
 *
 * tt_predict_adjoint: for the prediction C = K (*) P of tt_predict (Sec.
 * 4.2: C_k(a rp0 + c, i, b rp1 + e) = sum_m K_k(a, m+h, b) P_k(c, i-m, e),
 * P = 0 off the grid; log_scale(C) = log_scale(K) + log_scale(P)), given
 * c_bar (ranks must be the product ranks), writes
 *   p_bar_k(c, j, e) = sum_{m,a,b} K_k(a, m+h, b) c_bar_k(a rp0 + c, j+m, b rp1 + e)
 *   k_bar_k(a, m+h, b) = sum_{c,i,e} c_bar_k(a rp0 + c, i, b rp1 + e) P_k(c, i-m, e)
 * and copies c_bar's log_scale into both.
 *
 * tt_hadamard_adjoint: for H = A o B (Sec. 4.1 'times': H_k(a rb0 + c, i,
 * b rb1 + e) = A_k(a,i,b) B_k(c,i,e)), A in FP64 (the likelihood of
 * tt_update), given h_bar writes
 *   a_bar_k(a,i,b) = sum_{c,e} h_bar_k(a rb0 + c, i, b rb1 + e) B_k(c,i,e)
 *   b_bar_k(c,i,e) = sum_{a,b} h_bar_k(a rb0 + c, i, b rb1 + e) A_k(a,i,b)
 * (either output may be null) and copies h_bar's log_scale into both.
 *
 * tt_normalize_adjoint: the normalisation of tt_normalize_moments (Alg. 2,
 * the normaliser of eq. pmf_filtrace_b) keeps the cores of X and
 * sets log_scale(P) = -log(S delta), S = sum of the stored entries of X,
 * with log-mass log m = log_scale(X) + log(S delta).  Given p_bar (its
 * log_scale = the derivative with respect to log_scale(P)) and the
 * derivative mbar of log m (log_mass_bar_dev[b], nullable: 0), writes
 *   x_bar cores = p_bar cores + (mbar - p_bar.log_scale) / S * dS/dX,
 *   x_bar.log_scale = mbar.
 * --------------------------------------------------------------------- */
/* ---------------------------------------------------------------------
 * tt_update_adjoint: the adjoint of tt_update (Sec. 2.2 eqs.
 * pmf_filtrace_a/b: the likelihood TT L built from z, H = L o P_pred,
 * log c_k = log(sum(H) delta) + log-scales), FP64.  Given the forward's
 * p_pred and its output h (same grids, meas, z, lik_rank_cap as that
 * tt_update call), the adjoint h_bar of H (cores and log-scale, H's ranks;
 * nullable: 0) and log_c_bar_dev[b] (nullable: 0), it rebuilds L and the
 * dense likelihood input, and writes
 *   p_pred_bar   the adjoint of P_pred (cores; log_scale = that of H's
 *                total adjoint), TT_STATUS_CAPACITY on its status word when a
 *                rank or capacity does not match;
 *   theta_bar_dev[b * n_theta + d + j] += the derivative with respect to the
 *                measurement parameters (sigma_r, sigma_lin, s_1, s_2 for the
 *                range model, n_theta = d + 4; sigma_lin for the linear one,
 *                n_theta = d + 1), analytic in the dense likelihood through
 *                the adjoint of its truncated SVD (tt_likelihood_adjoint);
 *                entries 0..d-1 are not touched (the caller zeroes or
 *                accumulates).
 * z_dev[b * z_stride + j] as for tt_update.  Workspace:
 * tt_update_adjoint_workspace(...) bytes.  Asynchronous after its descriptor
 * uploads.  Errors: TT_ERR_ARG, TT_ERR_SHAPE, TT_ERR_WORKSPACE and those of
 * the composed calls.
 * --------------------------------------------------------------------- */
size_t tt_update_adjoint_workspace(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                                   const tt_train* h, int32_t lik_rank_cap);
tt_status tt_update_adjoint(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                            int32_t z_stride, const tt_train* p_pred, const tt_train* h, const tt_train* h_bar,
                            const double* log_c_bar_dev, int32_t lik_rank_cap, const tt_train* p_pred_bar,
                            double* theta_bar_dev, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_normalize_moments_adjoint: the adjoint of tt_normalize_moments with
 * its moments (the moments of Alg. 2; Sec. 4.1 'dot', 'power'): given p_bar
 * and log_mass_bar_dev as for tt_normalize_adjoint, and the adjoints of the
 * moments of the normalised density, mean_bar_dev[b * d + l] and
 * cov_bar_dev[b * d * d + l * d + j] (each nullable: 0; both entries of a
 * symmetric pair count), writes x_bar = tt_normalize_adjoint's result plus
 * the moments' term: with M_w = sum_i w(i) X(i) for the rank-one weights
 * 1, x_l, x_l^2 and x_l x_j on the grid points of grids[b] (the cell volume
 * and the log-scale cancel), mean_l = M_{x_l} / M_1 and cov_lj =
 * M_{x_l x_j} / M_1 - mean_l mean_j, the term is sum_w c_w dM_w / dX with
 * the coefficients of the quotient and product rules.  x, p_bar, x_bar as
 * for tt_normalize_adjoint (FP64 or FP32, x_bar with x's layout); grids[b]
 * has x[b]'s modes.  Workspace: tt_normalize_moments_adjoint_workspace(
 * batch, x) bytes.  Asynchronous after its descriptor uploads.  Errors:
 * TT_ERR_ARG, TT_ERR_SHAPE, TT_ERR_WORKSPACE.
 * --------------------------------------------------------------------- */
size_t tt_normalize_moments_adjoint_workspace(int32_t batch, const tt_train* x);
tt_status tt_normalize_moments_adjoint(int32_t batch, const tt_grid* grids, const tt_train* x,
                                       const tt_train* p_bar, const double* log_mass_bar_dev,
                                       const double* mean_bar_dev, const double* cov_bar_dev,
                                       const tt_train* x_bar, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_round_adjoint: adjoint of the rounding of Sec. 4.1 'round' (the
 * right-to-left orthogonalisation and the left-to-right truncated SVDs of
 * tt_round) at the ranks it produced, FP64.
 *
 * a: the input train of tt_round; y: its output (the output's cores define
 * the basis in which y_bar is expressed); y_bar: adjoint of y (same
 * capacities and ranks); a_bar: written with a's ranks, the derivative with
 * respect to a's stored cores, log_scale = y_bar's log_scale.  The rounding
 * is differentiated as a function of the input cores with every output rank
 * held fixed: Gram matrices of the right parts, leading eigenvectors of the
 * projected unfoldings (their adjoint couples kept and discarded singular
 * directions; the vectors and singular values come from the adjoint's own
 * SVD of each projected unfolding, and y and y_bar are sign-matched to it
 * bond by bond), then both sweeps backwards.  Kept singular values below
 * 6e-6 of the largest at a bond are left out of the eigenvector adjoint
 * (rounding noise there exceeds their signal) and discarded ones below 1e-9
 * count as null space.  The call reads the ranks to the host once and is
 * synchronous (it returns after the work is done); its job tables go
 * through one page-locked host staging area per process (allocated on
 * first use, at least 8 MB, grown when needed; calls from several threads
 * take turns on it).  tape (nullable): the
 * record tt_round_taped wrote for this rounding, read only; its Grams,
 * factors and the singular vectors of the tall unfoldings whose right
 * factor it holds are used instead of being recomputed.  Workspace:
 * tt_round_adjoint_workspace(batch, a, y) bytes (from the capacities).
 * Errors: TT_ERR_ARG (null, non-FP64, a recorded bond whose buffers are
 * null), TT_ERR_SHAPE (modes, capacities or ranks inconsistent, y_bar ranks
 * differ from y, a rank above 1024),
 * TT_ERR_WORKSPACE, TT_ERR_HIP.
 * --------------------------------------------------------------------- */
size_t tt_round_adjoint_workspace(int32_t batch, const tt_train* a, const tt_train* y);
tt_status tt_round_adjoint(int32_t batch, const tt_train* a, const tt_train* y, const tt_train* y_bar,
                           const tt_train* a_bar, const tt_round_tape* tape, void* ws, size_t ws_bytes,
                           void* stream);

/* ---------------------------------------------------------------------
 * Pieces for a composed reverse-mode gradient (all FP64 trains):
 *
 * tt_prior: the rank-one Gaussian prior of Sec. 2 (eq. pdf_pm with a
 * diagonal Gaussian p(x_0)), per axis exp(-(xi - m0)^2 / (2 p0)) shifted by
 * its maximum, the shifts and Gaussian constants in log_scale (the density
 * is not normalised here).  m0, p0_diag: host arrays [batch*d].
 *
 * tt_likelihood: the likelihood TT that tt_update multiplies with (Sec.
 * 2.2; the range block by truncated SVD at meas.lik_tol, linear axes rank
 * one, each factor max-shifted into log_scale), written to l_out (FP64;
 * capacities 1 except cap[1] = min(lik_rank_cap, n[1]) for the range
 * model).  Workspace: tt_update_workspace with p_pred = h_out = l_out.
 *
 * tt_likelihood_dense: the likelihood before the range block's truncation
 * (p_out, FP64): core 0 = the max-shifted (x_1, x_2) block M (n[0] x n[1]),
 * core 1 = the identity (capacities 1 except cap[1] = n[1] for the range
 * model), linear-axis factors and log_scale as tt_likelihood writes them.
 * Workspace: tt_update_workspace(batch, grids, meas, p_out, p_out, 1).
 *
 * tt_likelihood_adjoint: adjoint of the build l = tt_likelihood(...) with
 * respect to its dense input p = tt_likelihood_dense(...) of the same
 * measurement: given l_bar (the adjoint of l, l's capacities and ranks),
 * writes p_bar (p's capacities): core 0 = the adjoint of M through the
 * truncated SVD at l's rank (Sec. 3.1 truncation, differentiated as the
 * rounding adjoint of the two-core train (M^T, I), tt_round_adjoint), core 1
 * zero, linear factors and the log-scale adjoint copied from l_bar.  For
 * the linear model p_bar = l_bar.  <p_bar, dp> is then the derivative of the
 * scalar l_bar belongs to along a parameter tangent dp of the dense
 * likelihood.  TT_STATUS_CAPACITY on p_bar if l_bar's ranks differ from l's.
 * Workspace: tt_likelihood_adjoint_workspace(batch, meas, p, l).
 *
 * tt_adjoint_axpy: y += alpha x (cores and log_scale) for adjoint trains of
 * equal ranks (TT_STATUS_CAPACITY on y otherwise).
 *
 * tt_adjoint_inner: out_dev[b] = sum of the stored core entries of a_bar
 * times those of b over the ranks both share, plus the product of their
 * log_scale fields: the derivative <a_bar, db> of the scalar that a_bar is
 * the adjoint of, for a tangent db of the train b.
 *
 * tt_align_signs: rotates each bond basis of t (in both adjacent cores, so
 * the tensor is unchanged) by the orthogonal polar factor of its cosine
 * matrix with ref's, bond by bond from the left (sign flips, and rotations
 * among nearly equal singular values; a bond with a cosine singular value
 * below 1e-6 is left as is): puts a truncated-SVD build at perturbed
 * parameters into the basis of the build at the base parameters.
 * Workspace for the last three: tt_adjoint_workspace.
 * --------------------------------------------------------------------- */
tt_status tt_prior(int32_t batch, const tt_grid* grids, const double* m0, const double* p0_diag, const tt_train* out,
                   void* ws, size_t ws_bytes, void* stream);
tt_status tt_likelihood(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                        int32_t z_stride, const tt_train* l_out, int32_t lik_rank_cap, void* ws, size_t ws_bytes,
                        void* stream);
tt_status tt_likelihood_dense(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                              int32_t z_stride, const tt_train* p_out, void* ws, size_t ws_bytes, void* stream);
size_t tt_likelihood_adjoint_workspace(int32_t batch, const tt_meas* meas, const tt_train* p, const tt_train* l);
tt_status tt_likelihood_adjoint(int32_t batch, const tt_meas* meas, const tt_train* p, const tt_train* l,
                                const tt_train* l_bar, const tt_train* p_bar, void* ws, size_t ws_bytes,
                                void* stream);
tt_status tt_adjoint_axpy(int32_t batch, double alpha, const tt_train* x, const tt_train* y, void* ws,
                          size_t ws_bytes, void* stream);
tt_status tt_adjoint_inner(int32_t batch, const tt_train* a_bar, const tt_train* b, double* out_dev, void* ws,
                           size_t ws_bytes, void* stream);
tt_status tt_align_signs(int32_t batch, const tt_train* ref, const tt_train* t, void* ws, size_t ws_bytes,
                         void* stream);

size_t tt_adjoint_workspace(int32_t batch, int32_t d, int32_t rank_cap);
tt_status tt_predict_adjoint(int32_t batch, const tt_train* kernels, const tt_train* p_in, const tt_train* c_bar,
                             const tt_train* p_bar, const tt_train* k_bar, void* ws, size_t ws_bytes,
                             void* stream);
tt_status tt_hadamard_adjoint(int32_t batch, const tt_train* a, const tt_train* b, const tt_train* h_bar,
                              const tt_train* a_bar, const tt_train* b_bar, void* ws, size_t ws_bytes,
                              void* stream);
tt_status tt_normalize_adjoint(int32_t batch, const tt_train* x, const tt_train* p_bar,
                               const double* log_mass_bar_dev, const tt_train* x_bar, void* ws, size_t ws_bytes,
                               void* stream);

/* ---------------------------------------------------------------------
 * tt_filter_run -- the whole recursion for a batch of independent filters
 * (Alg. 2 loop order with the convolution prediction; step 0 is an update
 * only; steps k >= 1 predict, round, normalise, update, round, normalise).
 * All filters share d and the rounding tolerance eps; N, rank cap and model
 * may differ per filter (ragged batch: each filter's rank rule is capped at
 * its own spec.cap).  Outputs (device, FP64):
 *   loglik_dev[b]          = sum_k log c_k
 *   log_c_dev[b*K + k]     = log c_k
 *   log_mpred_dev[b*K + k] = log predictive mass before normalisation
 *                            (mass leaving the grid; 0 at k = 0)
 *   mean_dev[(b*K + k)*d + l], cov_dev[((b*K + k)*d + l)*d + j]  (nullable)
 *   ranks_dev[(b*K + k)*(d+1) + j]  filtering ranks per step (nullable)
 *   status_dev[b]          sticky TT_STATUS_* bits
 *   ranks_pred_dev[(b*K + k)*(d+1) + j]  ranks of the predictive after its
 *                          rounding (the prior's at k = 0) (nullable)
 * Rank replay (nullable inputs, same layout as ranks_pred_dev / ranks_dev):
 * replay_pred_dev and replay_filt_dev give the ranks the prediction and the
 * update rounding of every step must take instead of the rank rule (clamped
 * to at least 1, the available singular values and the capacity).  A run
 * replaying the ranks recorded by a base run computes the log-likelihood
 * with its rank pattern frozen, whose central differences in the model
 * parameters are the derivative of the computed sum of log c_k.
 * Inputs: z_dev[(b*K + k)*zdim + j] with zdim = max over filters of b
 * (d for kind 0, d-1 for kind 1); kernels[spec.kernel_index] is the filter's
 * transition kernel TT (built by tt_kernel_build on the filter's grid).
 * Steps k_begin .. k_begin+k_count-1 of a K-step horizon are run (outputs
 * and z are always laid out for K steps).  k_begin = 0 starts from the
 * prior; k_begin > 0 resumes from the filter state that the previous call
 * left in the same workspace (same specs, kernels and ws), so a run split
 * into several calls gives bitwise the same results as one call.
 * loglik_dev sums log c_k over steps 0 .. k_begin+k_count-1.
 * precision: TT_F64 (plain FP64 path) or TT_F32 (FP32 bulk cores and
 * contractions, FP64 Gram/pivoted-Cholesky/Jacobi factorisations and FP64
 * log-normaliser).  The kernels[] cores must have the same dtype.
 * --------------------------------------------------------------------- */
typedef struct {
  tt_grid grid;
  tt_meas meas;
  double m0[TT_MAXD];       /* Gaussian prior mean */
  double p0_diag[TT_MAXD];  /* Gaussian prior variances (diagonal) */
  int32_t cap;              /* rank cap of the PMD */
  double eps;               /* rounding tolerance */
  int32_t kernel_index;
  int32_t kernel_cap;       /* largest kernel TT rank reserved for */
  int32_t lik_rank_cap;     /* largest likelihood rank reserved for */
} tt_filter_spec;

size_t tt_filter_run_workspace(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                               int32_t n_kernels, int32_t precision);
tt_status tt_filter_run(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                        int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K,
                        int32_t k_begin, int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                        double* log_mpred_dev, double* mean_dev, double* cov_dev,
                        int32_t* ranks_dev, int32_t* status_dev, int32_t* ranks_pred_dev,
                        const int32_t* replay_pred_dev, const int32_t* replay_filt_dev, void* ws, size_t ws_bytes,
                        void* stream);

/* ---------------------------------------------------------------------
 * tt_filter_run_monitored -- tt_filter_run with per-step records of two
 * quantities the paper's filter leaves unchecked: the negativity of the TT
 * density (Sec. 5.1 and Sec. 6 report negative PMD values for d >= 3) and
 * the error of each rounding (Sec. 3.2: the TT-SVD truncation error is at
 * most the square root of the sum of the squared discarded tails).  Every
 * argument but monitor is that of tt_filter_run (same workspace query);
 * monitor (host struct, nullable) holds device pointers, each nullable:
 *   marg_min_dev[b * K + k]      smallest value over every 1-D marginal of
 *                                the filtering density P_{k|k} (the sums of
 *                                its point values over all axes but one)
 *   tail_dev[(b * K + k) * 2]    sqrt(sum over the bonds of the discarded
 *                                tail^2) / ||A|| of the prediction's
 *                                rounding at step k (0 at k = 0), and at
 *                                + 1 the same for the update's rounding
 * Records of steps outside [k_begin, k_begin + k_count) are not written.
 *
 * tt_marginal_min: out_dev[b] = the smallest 1-D marginal value of the TT
 * t[b] as above (log_scale included), any dtype, ragged ranks.  Workspace:
 * tt_marginal_min_workspace(batch, t) bytes.  Asynchronous.  Errors:
 * TT_ERR_ARG, TT_ERR_SHAPE, TT_ERR_WORKSPACE.
 * --------------------------------------------------------------------- */
typedef struct {
  double* marg_min_dev;
  double* tail_dev;
} tt_monitor;

tt_status tt_filter_run_monitored(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                  int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin,
                                  int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                                  double* log_mpred_dev, double* mean_dev, double* cov_dev, int32_t* ranks_dev,
                                  int32_t* status_dev, int32_t* ranks_pred_dev, const int32_t* replay_pred_dev,
                                  const int32_t* replay_filt_dev, const tt_monitor* monitor, void* ws,
                                  size_t ws_bytes, void* stream);
size_t tt_marginal_min_workspace(int32_t batch, const tt_train* t);
tt_status tt_marginal_min(int32_t batch, const tt_train* t, double* out_dev, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------------------
 * The differentiated recursion: LL = sum_k log c_k (Sec. 2.2, eq.
 * pmf_filtrace_b) of every filter of a batch and its gradient with respect
 * to theta = (sigma_w[0..d-1], sigma_r, sigma_lin, s_1, s_2) for the range
 * model (n_theta = d + 4) or (sigma_w[0..d-1], sigma_lin) for the all-linear
 * one (n_theta = d + 1), where Q = D C D with D = diag(sigma_w) and C the
 * correlation of spec.q.  FP64 throughout.
 *
 * tt_grad_spec: a filter (grid, measurement model with sigma_r, sigma_lin and
 * sensor, prior, rank cap, eps, lik_rank_cap; kernel_cap = the largest kernel
 * TT rank reserved for; kernel_index unused), its process-noise covariance q
 * (d x d row-major, sigma_w = sqrt(diag q)), the kernel offset box and the
 * kernel's TT-SVD tolerance.  All filters of a batch share d, the
 * measurement kind, eps, cap, kernel_cap, lik_rank_cap and the box.
 *
 * tt_filter_run_taped runs the recursion of tt_filter_run (Alg. 2 order,
 * materialised prediction) from the prior: it builds each filter's kernel
 * TT (tt_kernel_build_batch), writes loglik_dev[b] and keeps in ws what the
 * reverse sweep needs: with ckpt_every = 1 every step's rounded predictive,
 * likelihood TT, update product, filtering density and the records of both
 * roundings (tt_round_taped); with ckpt_every = C > 1 only the filtering
 * density that starts each segment of C steps.
 * tt_filter_run_adjoint then runs the reverse sweep on the same ws (same
 * batch, specs, z_dev, K and ckpt_every, nothing else written to ws in
 * between): segments from the last, each recomputed from its checkpoint,
 * steps backwards through tt_normalize_adjoint, tt_round_adjoint (ranks of
 * the forward held fixed), tt_hadamard_adjoint, tt_likelihood_adjoint and
 * tt_predict_adjoint, the adjoint of every log c_k seeded with
 * loglik_bar_dev[b].  It writes
 *   theta_bar_dev[b * n_theta + j] = loglik_bar[b] * dLL_b / dtheta_j.
 * The measurement parameters enter through the dense likelihood, whose
 * theta-derivative is analytic (the log-derivatives of the range and linear
 * Gaussian factors, evaluated on the device); sigma_w enters through the
 * kernel TT, whose tangent is the central difference of two device builds at
 * sigma_w[j] +- h_j (h_j = 1e-5 max(1, sigma_w[j])) put into the base
 * build's bond bases (tt_align_signs), the quotient taken on the device.
 * The builds are the dense TT-SVD up to d = 8 and 2^28 taps; beyond, the
 * base kernel is a TT-cross (as tt_kernel_build_cross, working rank 64)
 * whose index sets, row choices and ranks are kept, and the 2d perturbed
 * kernels (built in one batched call) are the same cross replayed on those
 * index sets and rounded to the base ranks, so that they change smoothly
 * with sigma_w.
 * status_dev[b] (both calls) receives the OR of the filter's TT_STATUS_*
 * bits (TT_STATUS_CAPACITY also when a perturbed kernel build changes a
 * rank); the caller clears it before the taped run.  Both calls synchronise
 * the stream before they return.  Workspace: tt_filter_grad_workspace bytes
 * (device memory for the kernels, the tape or checkpoints, one step's
 * temporaries and the sub-calls' workspaces).  Errors: TT_ERR_ARG (null,
 * ckpt_every < 1, K < 1, a parameter <= 0 where positive is required),
 * TT_ERR_SHAPE (the shared fields differ, d < 2), TT_ERR_WORKSPACE,
 * TT_ERR_HIP, and those of the sub-calls.
 * --------------------------------------------------------------------- */
typedef struct {
  tt_filter_spec f;
  double q[TT_MAXD * TT_MAXD];
  int32_t halfwidths[TT_MAXD];
  double kernel_tol;
} tt_grad_spec;

size_t tt_filter_grad_workspace(int32_t batch, const tt_grad_spec* specs, int32_t K, int32_t ckpt_every);
tt_status tt_filter_run_taped(int32_t batch, const tt_grad_spec* specs, const double* z_dev, int32_t zdim,
                              int32_t K, int32_t ckpt_every, double* loglik_dev, int32_t* status_dev, void* ws,
                              size_t ws_bytes, void* stream);
tt_status tt_filter_run_adjoint(int32_t batch, const tt_grad_spec* specs, const double* z_dev, int32_t zdim,
                                int32_t K, int32_t ckpt_every, const double* loglik_bar_dev, double* theta_bar_dev,
                                int32_t* status_dev, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_filter_run_linear -- the point-mass filter for linear dynamics
 * x_{k+1} = F x_k + w_k (w ~ N(0, Q)) on grids that follow the density
 * (Alg. 3 with the grid re-design of Alg. 4), FP64.  Step 0 updates the
 * prior on spec.grid; every later step
 *   re-designs the grid (tt_normalize_moments, tt_grid_redesign with
 *     nsigma: the predictive moments' sigma box mapped back by F^{-1}) and
 *     interpolates the density onto it (tt_interpolate);
 *   predicts on the lattice F xi of that grid: the convolution (tt_predict)
 *     with the kernel N(F (dx o m); 0, Q) dx^d = N(dx o m; 0, F^{-1} Q F^{-T})
 *     dx^d / |det F| on the box |m_l| <= floor(kernel_nsigma
 *     sqrt((F^{-1} Q F^{-T})_ll) / dx_l) (the smallest spacing over the
 *     batch, capped at N - 1), built by tt_kernel_build_cross at kernel_tol,
 *     then rounds (eps, cap);
 *   re-designs again: the smallest box holding the lattice's corners, onto
 *     which the prediction is interpolated (tt_interpolate_lattice at
 *     kernel_tol), rounded and normalised (log_mpred);
 * then updates as tt_filter_run does (likelihood, c_k, rounding,
 * normalisation, moments).  Outputs as tt_filter_run (log_c_dev,
 * log_mpred_dev [B*K], mean_dev [B*K*d], cov_dev [B*K*d*d], nullable
 * moments) plus grids_out (host, nullable) [B*K*2d]: lo then hi of each
 * step's filtering grid.  specs: grid (N points on every axis), meas,
 * prior, cap and kernel_cap in [1, 32], eps, lik_rank_cap, all but the
 * grid box, prior and measurement values shared by the batch; f, q: d x d
 * host (shared), 2 <= d <= 6.  Synchronous.  Workspace:
 * tt_filter_run_linear_workspace(batch, specs, K).  Errors: TT_ERR_ARG,
 * TT_ERR_SHAPE, TT_ERR_WORKSPACE, TT_ERR_HIP and those of the sub-calls.
 * --------------------------------------------------------------------- */
size_t tt_filter_run_linear_workspace(int32_t batch, const tt_filter_spec* specs, int32_t K);
tt_status tt_filter_run_linear(int32_t batch, const tt_filter_spec* specs, const double* f, const double* q,
                               double nsigma, double kernel_nsigma, double kernel_tol, const double* z_dev,
                               int32_t zdim, int32_t K, double* loglik_dev, double* log_c_dev, double* log_mpred_dev,
                               double* mean_dev, double* cov_dev, double* grids_out, int32_t* status_dev, void* ws,
                               size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * tt_filter_graph_* -- the steps of tt_filter_run recorded once as a HIP
 * graph and replayed (one graph per time step when k_count = 1; the
 * recursion of Alg. 2 repeated without host launch work).
 *
 * tt_filter_graph_create takes exactly the arguments of tt_filter_run.  It
 * validates them, uploads the batch descriptors into ws (on stream, then
 * waits for them), records the launches of steps k_begin .. k_begin+k_count-1 on a
 * capture stream of its own and instantiates the graph; nothing runs.
 * k_begin must be >= 1: step 0 starts from the prior and is run once with
 * tt_filter_run.  Every tt_filter_graph_launch then executes those steps on
 * stream, continuing from whatever filter state the workspace holds, reading
 * z_dev at the rows of those steps and writing the outputs of those steps
 * (a streaming filter: write the next measurement into z_dev's row k_begin,
 * launch, read log_c / mean at k_begin).  Every pointer is baked into the
 * graph: z_dev, the outputs and ws must stay allocated and unchanged in
 * layout until tt_filter_graph_destroy, and the specs/kernels arrays are not
 * read again.  Results are bitwise those of tt_filter_run on the same state.
 * Errors: as tt_filter_run; TT_ERR_ARG for k_begin < 1, a null handle or
 * active profiling (tt_profile_begin); TT_ERR_HIP when capture or
 * instantiation fails.  The handle is owned by the caller.
 * --------------------------------------------------------------------- */
typedef struct tt_graph_s tt_graph;

tt_status tt_filter_graph_create(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                 int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin,
                                 int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                                 double* log_mpred_dev, double* mean_dev, double* cov_dev, int32_t* ranks_dev,
                                 int32_t* status_dev, int32_t* ranks_pred_dev, const int32_t* replay_pred_dev,
                                 const int32_t* replay_filt_dev, void* ws, size_t ws_bytes, void* stream,
                                 tt_graph** out);
tt_status tt_filter_graph_launch(tt_graph* graph, void* stream);
void tt_filter_graph_destroy(tt_graph* graph);

/* ---------------------------------------------------------------------
 * tt_filter_state -- save or restore the filtering densities that a
 * tt_filter_run workspace carries from one call to the next: after steps
 * 0..k of the recursion (Alg. 2), filter b's state is its filtering density
 * P_{k|k} as a TT (ranks, FP64 log-scale and cores); nothing else persists
 * between calls.
 *   direction TT_STATE_SAVE: ws -> trains[b]; TT_STATE_LOAD: trains[b] -> ws.
 *   specs, kernels, n_kernels, precision: exactly those of the tt_filter_run
 *              calls the workspace serves (they fix its layout); ws, ws_bytes
 *              that workspace (tt_filter_run_workspace bytes).
 *   trains[b]  caller-owned device TT of dtype `precision`, d and modes of
 *              filter b's grid, capacities >= 1 (cap[j] >= spec.cap suffices).
 * A load followed by tt_filter_run with k_begin = k+1 continues the
 * recursion bitwise as an uninterrupted run would, in the same or in a fresh
 * workspace (log_c of steps 0..k must then already be in log_c_dev for the
 * log-likelihood sum).  Save clears the train's status word; a rank that does
 * not fit the destination's capacity copies nothing and sets
 * TT_STATUS_CAPACITY on the train's status word (both directions).  The
 * caller's status_dev of the run is not part of the state.  Asynchronous on
 * stream.  Errors: TT_ERR_ARG,
 * TT_ERR_SHAPE (d or modes differ from the grids), TT_ERR_WORKSPACE,
 * TT_ERR_HIP.
 * --------------------------------------------------------------------- */
#define TT_STATE_SAVE 0
#define TT_STATE_LOAD 1
tt_status tt_filter_state(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels, int32_t n_kernels,
                          int32_t precision, int32_t direction, const tt_train* trains, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------------------
 * tt_autotune_prediction -- time the launch shapes of the matrix-core
 * prediction on the caller's own batch and keep the fastest.
 *
 * The prediction (the per-core convolution of Sec. 4.2, fused with the
 * first rounding sweep) gives each workgroup one kernel row block and BB
 * density fibres; BB trades LDS reuse of the kernel block against the
 * number of workgroups.  The tuner runs step 0 and warmup_steps steps, then
 * `rounds` rounds of one step per candidate BB in {2, 4, 8, 16}, continuing
 * the recursion in ws and timing every step with HIP events on stream (it
 * synchronises).  Each candidate keeps its fastest step; the fastest
 * candidate is recorded for this launch shape (precision, batch size,
 * largest kernel half-width, grid size, PMD and kernel rank capacities) and
 * used by later tt_filter_run calls with the same shape.  BB does not change
 * any result bit.  Arguments are those of tt_filter_run (moments and rank
 * records are not written); K >= 1 + warmup_steps + 4 * rounds.  Outputs:
 * *best_bb (0 when the batch does not use the matrix-core prediction) and
 * ms_per_candidate[4] (ms of the candidate's fastest step).  The filter
 * state and outputs left in ws are those of the tuning steps: start the
 * real run at k_begin = 0.  Errors: TT_ERR_ARG for bad sizes, null outputs
 * or active profiling; as tt_filter_run otherwise.
 * --------------------------------------------------------------------- */
#define TT_TUNE_CANDIDATES 4
tt_status tt_autotune_prediction(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                 int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K,
                                 int32_t precision, double* loglik_dev, double* log_c_dev, double* log_mpred_dev,
                                 int32_t* status_dev, void* ws, size_t ws_bytes, void* stream,
                                 int32_t warmup_steps, int32_t rounds, int32_t* best_bb, float* ms_per_candidate);

/* tt_autotune_save / tt_autotune_load -- persist the tuned launch shapes.
 * save writes every shape tt_autotune_prediction has decided in this
 * process to `path` as a JSON array, one object per shape:
 *   {"arch": "gfx950", "knob": "prediction_fibres_per_workgroup",
 *    "dtype": "f32", "batch": 256, "halfwidth": 12, "n": 128,
 *    "rank_cap": 16, "kernel_rank_cap": 16, "value": 16}
 * (arch = the current device's architecture name).  load reads such a
 * file (the format save writes, objects in any order) and adopts the
 * entries whose arch is the current device's, replacing decisions for the
 * same shape; *n_loaded (nullable) receives their number.  Host-only file
 * I/O, no device work.  Errors: TT_ERR_ARG (null path, unreadable or
 * unwritable file, an entry that does not parse), TT_ERR_HIP (device
 * properties unavailable). */
tt_status tt_autotune_save(const char* path);
tt_status tt_autotune_load(const char* path, int32_t* n_loaded);

/* ---------------------------------------------------------------------
 * How tt_filter_run evaluates the prediction for d >= 3 (process-wide
 * setting; all modes compute the same Z_k = conv(K_k, P_k) x_3 L_{k+1} that
 * the rounding's right-to-left sweep consumes, Sec. 2.1 eq. tpmconvFFT and
 * Sec. 4.2):
 *   0 (default) direct fused: the convolution and the absorption of L in
 *     one time-domain kernel; the product TT is never materialised.  FP32
 *     runs it on the matrix cores (v_mfma_f32_16x16x4f32) when its LDS
 *     tiles fit, FP64 on the vector ALUs;
 *   1 FFT fused: kernel-fibre spectra (computed once per kernel TT) times the
 *     spectra of P x_3 L, inverse FFT and crop, per output column in LDS;
 *   2 unfused: materialise the product (tt_predict's kernel) and absorb L
 *     with a tall GEMM;
 *   3 direct fused on the vector ALUs for both precisions (mode 0 without
 *     the matrix cores).
 * A batch whose fused prediction would need more than the 160 KB of LDS of
 * a compute unit (FP64 at rank cap 24 and N = 128, say) runs mode 2.
 * tt_predict always materialises the product.
 * --------------------------------------------------------------------- */
tt_status tt_set_predict_mode(int32_t mode);
int32_t tt_get_predict_mode(void);

/* ---------------------------------------------------------------------
 * Optional timing of kernel classes (measurement support, not part of the
 * method).  tt_profile_begin(mask) makes the library record a pair of HIP
 * events on the launch stream around every launch of each class c with bit
 * (1 << c) set in mask:
 *   0 convolution, 1 Hadamard, 2 Gram, 3 pivoted Cholesky, 4 Jacobi,
 *   5 triangular solve, 6 GEMM, 7 likelihood build, 8 sum/moments,
 *   9 fused prediction (convolution and absorption of the next factor),
 *   10 Einstein-summation prediction (all passes of one call),
 *   11 interpolation onto a new grid.
 * For classes with a work model (9; direct prediction mode only) a
 * one-workgroup kernel after each launch adds the launch's algorithmic
 * flops and HBM bytes, computed from the device-resident ranks, to a small
 * device buffer that tt_profile_begin allocates once and clears.
 * tt_profile_end waits for the recorded events, writes the summed
 * milliseconds, launch counts, algorithmic flops and bytes of classes
 * 0..nclass-1 (any array may be NULL; classes without a work model report
 * 0), stops recording and returns the number of classes (or -1).  The state
 * is per process; do not profile from several threads at once.
 * --------------------------------------------------------------------- */
void tt_profile_begin(int32_t class_mask);
int32_t tt_profile_end(double* ms, int32_t* launches, double* flops, double* bytes, int32_t nclass);

#ifdef __cplusplus
}
#endif

#endif /* TTGBF_H */
