/*
 * rfi.h -- C ABI of librfi: multi-beam RFI identification by eigenvalue
 * decomposition of per-cell cross-correlation matrices, on one MI355X (gfx950).
 *
 * Method: Bai et al., "Radio frequency interference identification using
 * eigenvalue decomposition for multi-beam observations" (arXiv 2512.16278).
 * A cell is one (sub-interval k, frequency channel j). For every cell the
 * library forms the nbeam x nbeam cross-correlation matrix of the beams'
 * total power (Sec. 3.2, Eq. 1), eigendecomposes it (Sec. 3.3, Eq. 2), forms
 * the normalised dominant eigenvalue lambda_1^2 / sum_i lambda_i^2 (Sec. 3.3),
 * and turns it into an RFI mask by iterative Gaussian clipping (Sec. 3.3,
 * threshold multiple kappa of Sec. 4.5), optionally refined per beam with the
 * dominant eigenvector (Sec. 3.3 last paragraph, kappa_v of Sec. 4.5).
 *
 * Conventions for every call:
 *  - Every array argument is a DEVICE pointer unless marked "host". The
 *    caller owns all of them; the library never frees caller memory.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    rfi_stream_t; NULL is the null stream). Argument errors are returned
 *    synchronously and nothing is launched; rfi_last_error() then holds a
 *    message for the calling thread. Device-side conditions are reported
 *    through per-cell status bits and the stats structs.
 *  - ncell = nsub * nchan and cell = k * nchan + j. Per-cell arrays are
 *    "structure of arrays": element e of cell c is at [e * ncell + c].
 *  - Packed upper triangle of an nbeam x nbeam symmetric matrix, a <= b:
 *        pair(a, b) = a * nbeam - a * (a - 1) / 2 + (b - a),
 *    npair = nbeam * (nbeam + 1) / 2.
 */
#ifndef RFI_H
#define RFI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rfi_status;
enum {
  RFI_OK = 0,
  RFI_E_INVALID = -1,    /* bad argument (message in rfi_last_error) */
  RFI_E_OVERFLOW = -2,   /* sums would leave the exact int32 range */
  RFI_E_NOMEM = -3,      /* device or host allocation failed */
  RFI_E_BUDGET = -4,     /* block larger than the session's HBM budget */
  RFI_E_DEVICE = -5,     /* HIP runtime error */
  RFI_E_NOT_READY = -6,  /* result not yet available */
  RFI_E_CANCELLED = -7,  /* request cancelled before it ran */
  RFI_E_TIMEOUT = -8     /* wait timed out */
};

/* per-cell status bits (uint8) */
enum {
  RFI_CELL_DEGENERATE = 1,     /* a beam has zero variance in the cell */
  RFI_CELL_NOT_CONVERGED = 2,  /* Jacobi still rotating after max_sweeps */
  RFI_CELL_PROTECTED = 4,      /* channel preserved by the caller */
  RFI_CELL_REFINE_FAILED = 8,  /* FP64 refinement fell back to the FP32 value */
  RFI_CELL_BAD_COUNT = 16      /* fewer than 2 or more than RFI_MAX_COUNT samples */
};

typedef void* rfi_stream_t;            /* hipStream_t */

#define RFI_MAX_BEAMS 79
/* Largest number of samples a cell may accumulate in the int32 sums:
 * 255^2 * count < 2^31. */
#define RFI_MAX_COUNT 33025
/* Largest sub-interval of the int64 (long sub-interval) path: with
 * count < 2^18 every covariance numerator count S_ab - S_a S_b stays below
 * 2^50, exact in int64 and in FP64. 10 s of 49.152 us samples is 203,450. */
#define RFI_MAX_COUNT_LONG 262143

/* One observation block (Sec. 2 data layout): per beam, a time-major
 * filterbank of uint8 total power, channels contiguous within a time row.
 * beam[b] points to beam b's [nsamp][row_stride] bytes. row_stride >= nchan
 * and a multiple of 16; every beam[b] 16-byte aligned. Bytes of a row past
 * nchan are read but never used. Pointers are device pointers held in this
 * host struct. */
typedef struct {
  int32_t nbeam;                 /* 2 .. RFI_MAX_BEAMS */
  int32_t nchan;                 /* >= 1 */
  int64_t nsamp;                 /* time rows in the block */
  int64_t row_stride;            /* bytes between consecutive time rows */
  const uint8_t* beam[RFI_MAX_BEAMS];
} rfi_block;

/* Placement of the beams (a speed matter only; any placement meeting the
 * rules above gives the same results). The sums kernels read the same time
 * row of every beam at once. When every beam[b] has the same address modulo
 * 4 KB and row_stride is a multiple of 4 KB, those reads land on the same
 * memory channels: on a 19-beam, 4096-channel block of 2048-sample cells the
 * sums then take about 9 % longer. rfi_beam_offsets lays out nbeam beams of
 * nsamp rows of row_stride bytes in one allocation, beam b starting
 * 64 (b mod 64) bytes past a 4 KB boundary: offsets[b] is beam b's byte
 * offset from a 4 KB-aligned base, *total the bytes to allocate from that
 * base. Host arithmetic only (offsets and total are host pointers).
 * Errors: RFI_E_INVALID for nbeam outside 1..RFI_MAX_BEAMS, nsamp < 0,
 * row_stride < 1 or not a multiple of 16, null pointers; RFI_E_OVERFLOW if
 * the total exceeds 2^62 bytes. */
rfi_status rfi_beam_offsets(int32_t nbeam, int64_t nsamp, int64_t row_stride,
                            int64_t* offsets /* host, nbeam */, int64_t* total /* host */);

enum { RFI_CCM_AUTO = 0, RFI_CCM_MFMA = 1, RFI_CCM_VALU = 2 };

/* Per-cell sums of Eq. 1 (Sec. 3.2) for sub-intervals [t0 + kL, t0 + (k+1)L),
 * k < nsub, of every channel:
 *     sum_x [b][cell]        = sum_t x_b(t)                (nbeam rows)
 *     sum_xy[pair(a,b)][cell] = sum_t x_a(t) x_b(t), a <= b (npair rows)
 *     count [k]              = samples accumulated into sub-interval k
 * exact in int32. accumulate = 0 overwrites the outputs; 1 adds into them
 * (a sub-interval spanning two blocks is accumulated in two calls; the
 * caller keeps the accumulated count <= RFI_MAX_COUNT). variant selects the
 * engine: int8 MFMA on x - 128 (exact: the offset is removed again in
 * integer arithmetic) or plain VALU dot products (nbeam <= 20 only).
 * Errors: RFI_E_INVALID for bad shapes or alignment, t0 + nsub*L > nsamp,
 * L < 1; RFI_E_OVERFLOW for L > RFI_MAX_COUNT. */
rfi_status rfi_ccm_accumulate(const rfi_block* blk /* host */, int64_t t0, int32_t L,
                              int32_t nsub, int32_t* sum_x, int32_t* sum_xy,
                              int32_t* count, int32_t accumulate, int32_t variant,
                              rfi_stream_t stream);

/* Sums of Eq. 1 (Sec. 3.2) for long sub-intervals, RFI_MAX_COUNT < L <=
 * RFI_MAX_COUNT_LONG (Table 1 runs sub-intervals up to 10 s, 203,450 samples of
 * 49.152 us; any L >= 1 is accepted): the same sums as rfi_ccm_accumulate, as
 * exact int64 in one record per cell,
 *     sums[cell * (nbeam + npair) + b]          = sum_t x_b(t)
 *     sums[cell * (nbeam + npair) + nbeam + p]  = sum_t x_a(t) x_b(t), p = pair(a, b)
 * and count[k] = L. Each sub-interval is summed in time chunks of at most
 * RFI_MAX_COUNT samples by the int32 engine and the chunks are added exactly
 * in int64. workspace: rfi_ccm_long_workspace_size(nbeam, nchan, nsub) bytes
 * of device scratch, 256-byte aligned, caller-owned, one call at a time.
 * Outputs are overwritten (no accumulate mode). Errors: as
 * rfi_ccm_accumulate with the bound RFI_MAX_COUNT_LONG; RFI_E_INVALID for a
 * NULL or misaligned workspace. */
size_t rfi_ccm_long_workspace_size(int32_t nbeam, int32_t nchan, int32_t nsub);
rfi_status rfi_ccm_accumulate_long(const rfi_block* blk /* host */, int64_t t0, int32_t L,
                                   int32_t nsub, int64_t* sums, int32_t* count, void* workspace,
                                   rfi_stream_t stream);

/* Eigen solver selection:
 *  RFI_EIG_LANE    cyclic Jacobi, FP32, one cell per lane in registers, nbeam <= 20;
 *  RFI_EIG_WAVE    cyclic Jacobi (round-robin parallel ordering), one cell per
 *                  wavefront in LDS, FP32 or FP64, any nbeam;
 *  RFI_EIG_TRIDIAG Householder reduction to tridiagonal form and Sturm
 *                  bisection (Golub & Van Loan Sec. 8.3-8.4), FP64, one cell per
 *                  wavefront with the matrix in registers, any nbeam: about
 *                  (4/3) n^3 flops per cell instead of 6 n^3 per Jacobi sweep.
 *  RFI_EIG_LANE_TRI Householder reduction and Sturm bisection in FP32, one
 *                  cell per lane in registers, nbeam <= 20 (about (4/3) n^3 flops
 *                  instead of the Jacobi's 6 n^3 per sweep), one launch: the
 *                  two-vector block inverse iteration runs on the tridiagonal
 *                  (the vectors go back through the stored reflectors), then
 *                  the FP64 Ritz value as for LANE.
 *  RFI_EIG_AUTO    LANE_TRI for FP32 and nbeam <= 20, TRIDIAG for FP32 and
 *                  more beams, WAVE for FP64 (FP64 Jacobi).
 * The per-lane solvers refine lambda_1 in FP64 by two-vector block inverse
 * iteration on the FP32 matrix (LANE) or on its FP32 tridiagonal form
 * (LANE_TRI) and the Ritz value of the FP64 matrix on that subspace, also when
 * lambda_2 is close to lambda_1; the statistic is then within about 1e-13
 * (LANE) and 3e-12 (LANE_TRI) of its FP64 value. */
enum {
  RFI_EIG_AUTO = 0, RFI_EIG_LANE = 1, RFI_EIG_WAVE = 2, RFI_EIG_TRIDIAG = 3,
  RFI_EIG_LANE_TRI = 4
};

typedef struct {
  int32_t precision;     /* 32: FP32 Jacobi (default); 64: FP64 Jacobi */
  int32_t max_sweeps;    /* cyclic Jacobi sweep cap, 1..30 (default 12) */
  int32_t refine;        /* 1: lambda_1 refined in FP64 (default) */
  int32_t solver;        /* RFI_EIG_AUTO | _LANE, _LANE_TRI (nbeam <= 20, FP32) | _WAVE |
                            _TRIDIAG */
} rfi_eig_params;

/* Per cell (Sec. 3.2-3.3): the Pearson correlation matrix
 *     r_ab = N_ab / sqrt(N_aa N_bb),  N_ab = count * S_ab - S_a S_b
 * (N exact in int64, r in FP64; a beam with N_aa = 0 gets r_ab = 0 off the
 * diagonal and the cell RFI_CELL_DEGENERATE), its eigenvalues by the
 * selected solver (Jacobi: eps-relative skip rule, stop after a sweep without
 * rotations or max_sweeps), and
 *     stat[cell] = lambda_1^2 / ||r||_F^2         (FP64)
 * with lambda_1 the eigenvalue of largest magnitude, refined in FP64 when
 * p->refine (FP32 solvers: Ritz value of the FP64 matrix on two vectors of
 * block inverse iteration; FP64 solvers need none). Optional outputs
 * (NULL = not computed): eigvals[i][cell] (FP32, |lambda| descending) and
 * v1[b][cell] (FP32 unit dominant eigenvector, sign: sum_b v1_b >= 0).
 * status[cell] gets RFI_CELL_* bits. Inputs are the outputs of
 * rfi_ccm_accumulate for the same nbeam, nsub, nchan. p may be NULL
 * (defaults). */
rfi_status rfi_eig_batched(int32_t nbeam, int32_t nsub, int32_t nchan,
                           const int32_t* sum_x, const int32_t* sum_xy,
                           const int32_t* count, const rfi_eig_params* p /* host */,
                           float* eigvals, double* stat, float* v1, uint8_t* status,
                           rfi_stream_t stream);

/* The eigen stage of rfi_eig_batched (Sec. 3.2-3.3, Eq. 2) on the int64 sums
 * of rfi_ccm_accumulate_long (count[k] <= RFI_MAX_COUNT_LONG): the FP64
 * Householder-tridiagonal solver (RFI_EIG_TRIDIAG) for every beam count, the
 * covariance numerators formed exactly in int64. Outputs as rfi_eig_batched
 * (eigvals and v1 nullable). */
rfi_status rfi_eig_batched_long(int32_t nbeam, int32_t nsub, int32_t nchan, const int64_t* sums,
                                const int32_t* count, float* eigvals, double* stat, float* v1,
                                uint8_t* status, rfi_stream_t stream);

/* ArPLS bandpass (Sec. 3.1; lam, ratio, itermax of Sec. 4.5): for every beam
 * b and sub-interval k, the channel means y_j = sum_x[b][k nchan + j] /
 * count[k] are fitted by asymmetrically reweighted penalised least squares
 * (Baek et al. 2015): with D the second-difference operator over channels,
 * solve (W + lam D^T D) z = W y (W = diag(w), w = 1 at first), d = y - z,
 * m and s the mean and sample standard deviation (ddof 1) of the negative d,
 * w' = 1 / (1 + exp(2 (d - (2 s - m)) / s)); stop when ||w - w'|| / ||w|| <
 * ratio (keeping this pass's z), when fewer than two residuals are negative
 * or s = 0, or after itermax passes. z[b][k nchan + j] (FP64) receives the
 * baseline, the bandpass to subtract from every sample of the channel;
 * passes[k nbeam + b] (nullable) the passes taken. Inputs in the rows layout
 * of rfi_ccm_accumulate. workspace: rfi_bandpass_workspace_size bytes
 * (caller-owned, one call at a time). One thread per (beam, sub-interval):
 * the solve is sequential over the channels.
 * Errors: RFI_E_INVALID for bad sizes, lam <= 0, ratio < 0, itermax < 1 or
 * NULL pointers. */
size_t rfi_bandpass_workspace_size(int32_t nbeam, int32_t nchan, int32_t nsub);
rfi_status rfi_bandpass_arpls(int32_t nbeam, int32_t nsub, int32_t nchan, const int32_t* sum_x,
                              const int32_t* count, double lam, double ratio, int32_t itermax,
                              double* z, int32_t* passes, void* workspace, rfi_stream_t stream);

/* The non-centred reading of Eq. 1's <B_a B_b> (Sec. 3.2) on the
 * bandpass-subtracted power of Sec. 3.1: per cell the raw second-moment
 * matrix
 *     M_ab = (S_ab - z_b S_a - z_a S_b + count z_a z_b) / count
 * of x - z (z[b][cell] from rfi_bandpass_arpls, or NULL for z = 0), each
 * entry formed in FP64 in that order, then its eigenvalues by the FP64
 * Householder-tridiagonal solver and stat = lambda_1^2 / ||M||_F^2 (Sec. 3.3).
 * Sums in the rows layout of rfi_ccm_accumulate; outputs as rfi_eig_batched
 * (eigvals, v1 nullable; status RFI_CELL_DEGENERATE where M = 0,
 * RFI_CELL_BAD_COUNT where count < 2). */
rfi_status rfi_eig_noncentred(int32_t nbeam, int32_t nsub, int32_t nchan, const int32_t* sum_x,
                              const int32_t* sum_xy, const int32_t* count, const double* z,
                              float* eigvals, double* stat, float* v1, uint8_t* status,
                              rfi_stream_t stream);

/* Clip summary written by rfi_flag (device struct). */
typedef struct {
  double mu, sigma, thr;   /* last fit: mean, population sigma, mu + kappa sigma */
  int32_t iterations;      /* fits computed */
  int32_t converged;       /* 1 if the last fit masked nothing new */
  int64_t nflag;           /* cells masked */
  int64_t nfit;            /* eligible cells left unmasked (this block) */
} rfi_flag_stats;

#define RFI_HIST_CAP 1024
typedef struct {
  double mu, sigma, thr;
  int32_t iterations, converged;
} rfi_hist_entry;

/* Per-stream pooled clip state (device struct, zero-initialise to start a
 * stream). Exact sums over every unmasked cell of the stream's earlier
 * blocks: n, q1 = sum q, q2 = sum q^2 with q = rint(stat * 2^40), 128-bit
 * little-endian limbs; and the ring of the last RFI_HIST_CAP fits. */
typedef struct {
  int64_t n;
  uint64_t q1[2];
  uint64_t q2[2];
  int64_t nblocks;
  rfi_hist_entry hist[RFI_HIST_CAP];
} rfi_stream_state;

/* Iterative one-sided Gaussian clip of stat over the nsub x nchan cells
 * (Sec. 3.3; kappa of Sec. 4.5; preserved ranges of Sec. 4.3). Eligible
 * cells: status without RFI_CELL_DEGENERATE / RFI_CELL_BAD_COUNT and channel
 * not protected (protect_chan[j] != 0; NULL = none). On the statistic
 * quantised to q = rint(stat * 2^40): mu = Q1 / (N 2^40) and
 * sigma^2 = (N Q2 - Q1^2) / (N^2 2^80), each the exact rational of the integer
 * sums over the eligible unmasked cells (pooled with *state when state !=
 * NULL) rounded once to FP64, sigma its correctly rounded square root,
 * thr = mu + kappa sigma (FP64 product and sum, no fused multiply-add); mask
 * every such cell with q * 2^-40 > thr, repeat until a fit masks nothing new
 * or max_iter fits. mask[cell] = 1 for masked cells, else 0. If state != NULL
 * the block's final unmasked sums are folded into it and the fit appended to
 * its history. out (nullable) receives the summary.
 * workspace: device scratch of rfi_flag_workspace_size(nsub, nchan) bytes,
 * 256-byte aligned, owned by the caller and used by one call at a time (it
 * holds per-workgroup partial sums and the list of tail cells; the library
 * allocates nothing). nsub = 0 runs an empty clip (no fit; a history entry
 * with iterations 0 is still appended to *state).
 * Errors: RFI_E_INVALID for bad sizes, kappa < 0, max_iter < 1, or a NULL or
 * misaligned workspace. */
size_t rfi_flag_workspace_size(int32_t nsub, int32_t nchan);
rfi_status rfi_flag(int32_t nsub, int32_t nchan, const double* stat, const uint8_t* status,
                    const uint8_t* protect_chan, double kappa, int32_t max_iter,
                    rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out,
                    void* workspace, rfi_stream_t stream);

/* rfi_flag without a workspace argument, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Arguments, results and errors as rfi_flag; the workspace is a
 * fixed array of about 8.1 MiB of device memory inside this library, one per
 * GPU, set aside when the library loads and held until the process ends (its
 * address is looked up on the first call on each device). Blocks of at most
 * RFI_FLAG_NOALLOC_MAX_CELLS cells (nsub * nchan); larger ones return
 * RFI_E_INVALID. The call allocates nothing. Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (on different streams, or
 * from different threads) race; calls in one stream order are safe. */
#define RFI_FLAG_NOALLOC_MAX_CELLS 1048576
rfi_status rfi_flag_noalloc(int32_t nsub, int32_t nchan, const double* stat,
                            const uint8_t* status, const uint8_t* protect_chan, double kappa,
                            int32_t max_iter, rfi_stream_state* state, uint8_t* mask,
                            rfi_flag_stats* out, rfi_stream_t stream);

/* Clip scopes and fits (Sec. 3.3: outliers are masked as a function of
 * frequency and time; the mean and standard deviation come from a Gaussian
 * fitted to the distribution, Fig. 1). scopes is a bit set:
 *   RFI_SCOPE_GLOBAL   one clip over every cell (as rfi_flag, state-free);
 *   RFI_SCOPE_CHANNEL  one clip per channel over its nsub sub-intervals;
 *   RFI_SCOPE_SUBINT   one clip per sub-interval over its nchan channels;
 * mask[cell] = 1 where any requested scope masks the cell (the combined
 * mask). Each clip iterates as rfi_flag (same eligibility, kappa, max_iter,
 * quantised statistic). fit: RFI_FIT_MOMENTS is rfi_flag's exact moment fit
 * (every reported fit bit-equal to it); RFI_FIT_HISTOGRAM fits a Gaussian to
 * the histogram of the live values: 64 bins of width sigma_m / 8 over
 * mu_m +- 4 sigma_m of the exact moment fit, then a least-squares parabola
 * a + b z + c z^2 through ln(count) at the standardised bin centres
 * z = (i + 1/2) / 8 - 4 with weights count^2 over the non-empty bins
 * (Cramer's rule), mu = mu_m - b / (2c) sigma_m, sigma = sqrt(-1 / (2c))
 * sigma_m; fewer than 8 live values, sigma_m = 0, fewer than 3 non-empty
 * bins or c >= 0 keep the moment fit. Summaries (nullable): out for the
 * global scope, chan_out[nchan] per channel, sub_out[nsub] per sub-interval.
 * workspace: rfi_flag_workspace_size bytes (256-byte aligned) when the global
 * scope uses the moment fit, else unused (may be NULL).
 * Errors: RFI_E_INVALID for bad sizes, scopes outside 1..7, an unknown fit,
 * kappa < 0, max_iter < 1 or a missing workspace. */
enum { RFI_SCOPE_GLOBAL = 1, RFI_SCOPE_CHANNEL = 2, RFI_SCOPE_SUBINT = 4 };
enum { RFI_FIT_MOMENTS = 0, RFI_FIT_HISTOGRAM = 1 };
rfi_status rfi_flag_scoped(int32_t nsub, int32_t nchan, const double* stat, const uint8_t* status,
                           const uint8_t* protect_chan, double kappa, int32_t max_iter,
                           int32_t scopes, int32_t fit, uint8_t* mask, rfi_flag_stats* out,
                           rfi_flag_stats* chan_out, rfi_flag_stats* sub_out, void* workspace,
                           rfi_stream_t stream);

/* The clip's moment fit on its own (Sec. 3.3 Gaussian fit; the arithmetic
 * rfi_flag applies at every iteration), for checking its rounding: for each
 * i < n, from N[i] > 0 and the 128-bit sums Q1 = (Q1[2i], Q1[2i+1]) and
 * Q2 = (Q2[2i], Q2[2i+1]) (little-endian 64-bit limbs, N Q2 >= Q1^2):
 * mu[i] = Q1 / (N 2^40) and var = (N Q2 - Q1^2) / (N^2 2^80) rounded once to
 * FP64, sigma[i] = sqrt(var) correctly rounded, thr[i] = mu + kappa sigma.
 * N[i] <= 0 gives NaN. All arrays are device arrays of n entries.
 * Errors: RFI_E_INVALID for n < 0, NULL arrays or kappa < 0. */
rfi_status rfi_clip_fit(int32_t n, const int64_t* N, const uint64_t* Q1, const uint64_t* Q2,
                        double kappa, double* mu, double* sigma, double* thr,
                        rfi_stream_t stream);

/* Per-beam eigenvector stage (Sec. 3.3 last paragraph; kappa_v of Sec. 4.5):
 * for each beam b, mu_b and sigma_b (population) of |v1_b| over eligible
 * unmasked cells; beam_mask[b][cell] = mask[cell] && |v1_b| > mu_b +
 * kappa_v sigma_b. Eligibility as in rfi_flag. beam_mu / beam_sigma
 * (nullable, [nbeam] FP64) receive the fits (FP64 sums of |v1_b| and
 * |v1_b|^2 over the cells, sigma^2 = (sum x^2 - mu sum x) / n; NaN with no
 * cell). workspace: rfi_eigvec_workspace_size bytes of device memory,
 * 8-byte aligned, owned by the caller, one call at a time (at most 485 KB).
 * Errors: RFI_E_INVALID for bad sizes, NULL pointers, kappa_v < 0. */
size_t rfi_eigvec_workspace_size(int32_t nbeam, int32_t nsub, int32_t nchan);
rfi_status rfi_eigvec_flag(int32_t nbeam, int32_t nsub, int32_t nchan, const float* v1,
                           const uint8_t* mask, const uint8_t* status,
                           const uint8_t* protect_chan, double kappa_v,
                           uint8_t* beam_mask, double* beam_mu, double* beam_sigma,
                           void* workspace, rfi_stream_t stream);

/* The whole per-block path in one call: the sums of Eq. 1, the eigen stage
 * of Eq. 2 and the statistic (as rfi_eig_batched, FP32 Jacobi unless
 * eig_precision = 64), then the clip (as rfi_flag), for the nsub full
 * sub-intervals of L samples that start at sample t0 of blk. Sub-intervals
 * are processed in groups of `group`: the sums of group g are formed on
 * `stream` while earlier groups are eigendecomposed on a library-owned
 * helper stream, and the sums of at most three groups live in the workspace
 * at once, so the workspace stays bounded for any block length. group = 0
 * takes the whole block as one group while its sums fit in 1 GiB (the
 * fastest schedule measured: the two stages contend for the same vector ALU
 * when they overlap), else the largest group that keeps the ring within
 * 1 GiB. The results equal those of the three separate calls bit for bit
 * (same arithmetic, whatever the grouping).
 * Outputs: stat, status, mask [ncell] as in rfi_eig_batched / rfi_flag;
 * eigvals [nbeam][ncell] and v1 [nbeam][ncell] are optional (NULL); with
 * p->beam_mask the per-beam stage runs after the clip (the paper's final
 * output: which beams of a masked cell carry the interference). state,
 * protect_chan and out as in rfi_flag. The call is asynchronous on `stream`
 * (all work, including the helper stream's, completes before later work on
 * `stream` starts). Calls that run concurrently from several host threads
 * are serialised while they enqueue. workspace: rfi_process_workspace_size()
 * bytes of device memory, 256-byte aligned, owned by the caller and used by
 * one call at a time.
 * nsub = 0 launches nothing and accepts NULL outputs and workspace.
 * Errors: as rfi_ccm_accumulate, rfi_eig_batched and rfi_flag;
 * RFI_E_INVALID if workspace is NULL or misaligned, or group < 0. */
typedef struct {
  int64_t t0;            /* first sample of the first sub-interval */
  int32_t L;             /* samples per sub-interval, 1..RFI_MAX_COUNT_LONG; above
                            RFI_MAX_COUNT the sums are int64 (as
                            rfi_ccm_accumulate_long) and the eigen stage is the
                            FP64 tridiagonal solver */
  int32_t nsub;          /* full sub-intervals to process */
  int32_t group;         /* sub-intervals per pipeline group; 0 = automatic */
  int32_t eig_precision; /* 32 (default) or 64 */
  int32_t max_sweeps;    /* 0 = 12 */
  int32_t max_iter;      /* clip fits, 0 = 50 */
  double kappa;          /* clip multiple (Sec. 4.5), >= 0 */
  double kappa_v;        /* per-beam eigenvector multiple (Sec. 4.5), >= 0; read only when
                            beam_mask is given */
  uint8_t* beam_mask;    /* NULL, or a device [nbeam][ncell] output: the per-beam mask of
                            the eigenvector stage (Sec. 3.3 last paragraph) on this call's
                            mask and v1, exactly as rfi_eigvec_flag; then v1 must be given */
  int32_t scopes;        /* clip scopes as rfi_flag_scoped (RFI_SCOPE_* bits); 0 = the global
                            clip */
  int32_t fit;           /* RFI_FIT_MOMENTS (0) or RFI_FIT_HISTOGRAM; with scopes or the
                            histogram fit the clip is rfi_flag_scoped's (no pooled state:
                            state must be NULL) and out gets the global scope's summary */
} rfi_process_params;

size_t rfi_process_workspace_size(int32_t nbeam, int32_t nchan,
                                  const rfi_process_params* p /* host */);
rfi_status rfi_process_block(const rfi_block* blk /* host */,
                             const rfi_process_params* p /* host */,
                             const uint8_t* protect_chan, rfi_stream_state* state,
                             double* stat, uint8_t* status, uint8_t* mask, float* eigvals,
                             float* v1, rfi_flag_stats* out, void* workspace,
                             rfi_stream_t stream);

/* ---------------------------------------------------------------------------
 * Batched uneven blocks: many blocks of different beam counts, channel counts
 * and sub-interval lengths through the whole path (as rfi_process_block for
 * each) with one launch per kernel class instead of one per block:
 *  - one sums launch per instance class of the sums engine (beam-count
 *    range), whose workgroups cover the tiles of all blocks of the class;
 *  - one eigen launch (or two: Jacobi, then refinement) per solver class
 *    (beam-count template of the per-lane solver, or the per-wavefront
 *    solver) over all cells of its blocks;
 *  - one clip launch, one workgroup per block.
 * The sums of every block live in the workspace at once. Outputs per block as
 * rfi_process_block (stat, status, mask; out and state nullable), every one
 * equal to what rfi_process_block computes for that block alone, bit for bit.
 * The clip of a batch runs one workgroup per block: it suits blocks of up to
 * a few hundred thousand cells; larger blocks are better served by
 * rfi_process_block. rfi_batch_graph_* capture the same launches once into a
 * HIP graph that is replayed with one call (the descriptors and pointers are
 * fixed at capture: replays reprocess the same buffers). */
typedef struct {
  const rfi_block* blk;          /* host pointer to the block description */
  int64_t t0;                    /* first sample of the first sub-interval */
  int32_t L;                     /* samples per sub-interval, 1..RFI_MAX_COUNT_LONG;
                                    above RFI_MAX_COUNT the item takes the long route of
                                    rfi_process_block (int64 sums of time chunks, FP64
                                    tridiagonal solver) with launches of its own, and
                                    the batched clip */
  int32_t nsub;                  /* full sub-intervals (0: the block is skipped) */
  const uint8_t* protect_chan;   /* device [nchan] or NULL */
  rfi_stream_state* state;       /* device or NULL: pooled clip state */
  double* stat;                  /* device [nsub * nchan] */
  uint8_t* status;               /* device [nsub * nchan] */
  uint8_t* mask;                 /* device [nsub * nchan] */
  rfi_flag_stats* out;           /* device or NULL */
  float* v1;                     /* device [nbeam][nsub * nchan] or NULL: dominant eigenvectors */
  uint8_t* beam_mask;            /* device [nbeam][nsub * nchan] or NULL: the per-beam mask
                                    (Sec. 3.3 last paragraph), as rfi_eigvec_flag on this
                                    block's v1 and mask; needs v1 */
} rfi_batch_item;

/* Launch configuration of one shape class of the batched path. A class is
 * the range of beam counts [nbeam_lo, nbeam_hi] that one sums-engine tile
 * family serves (2-15, 16-31, 32-47, 48-63, 64-79); 0 in a choice field
 * means the library default:
 *  ccm_tile        sums tile variant, 0 .. rfi_ccm_tile_variants(nbeam) - 1
 *                  (16-31 beams: 0 = 64 channels on 16 waves, 1 = 64
 *                  channels on 8 waves, 2 = 32 channels on 8 waves; others:
 *                  0 only);
 *  ccm_stages      cap of the global-to-LDS load ring depth, 2..4;
 *  ccm_group_bytes contiguous row bytes of the tiles one XCD takes in turn
 *                  (16 .. 16384; default 1024);
 *  eig_solver      RFI_EIG_* for the class (AUTO: the default rule; LANE and
 *                  LANE_TRI need FP32 and nbeam <= 20);
 *  eig_wg          cells per workgroup of the per-lane solver: 64, 128, 256.
 * ms_default / ms_tuned: class time (sums + eigen launches, ms) with the
 * defaults and with the entry's choices, as measured by rfi_tune_batch. */
typedef struct {
  int32_t nbeam_lo, nbeam_hi;
  int32_t ccm_tile, ccm_stages, ccm_group_bytes;
  int32_t eig_solver, eig_wg, pad;
  double ms_default, ms_tuned;
} rfi_tune_entry;

#define RFI_TUNE_MAX 8
typedef struct {
  int32_t n;                     /* entries in use */
  int32_t pad;
  rfi_tune_entry e[RFI_TUNE_MAX];
} rfi_tune_table;

/* Tile variants of the sums engine for a beam count (0 if unsupported). */
int32_t rfi_ccm_tile_variants(int32_t nbeam);

typedef struct {
  int32_t eig_precision;         /* 32 (0 = 32) or 64 */
  int32_t max_sweeps;            /* 0 = 12 */
  int32_t max_iter;              /* clip fits, 0 = 50 */
  int32_t pad;
  double kappa;                  /* clip multiple, >= 0 */
  const rfi_tune_table* tune;    /* host, nullable: per-class launch choices
                                    (read when the call plans the batch) */
  double kappa_v;                /* per-beam multiple (Sec. 4.5), >= 0; read for items
                                    with a beam_mask */
} rfi_batch_params;

/* Workspace bytes for the batch (0 on invalid arguments; rfi_last_error). */
size_t rfi_batch_workspace_size(int32_t nitem, const rfi_batch_item* items /* host */,
                                const rfi_batch_params* p /* host */);
/* Asynchronous on stream. workspace: device, 256-byte aligned, caller-owned,
 * used by one call (or graph) at a time. */
rfi_status rfi_process_batch(int32_t nitem, const rfi_batch_item* items /* host */,
                             const rfi_batch_params* p /* host */, void* workspace,
                             rfi_stream_t stream);

/* Autotuner (batched path): for every shape class of the batch, times the
 * class's sums launch for each tile variant and ring depth, then for each
 * XCD group size, and its eigen launch for each applicable solver (and
 * per-lane workgroup size), on the caller's blocks, and writes the fastest
 * choices to *table (host), one entry per class, ordered by beam count (a
 * choice replaces the default only when it is more than 2 % faster).
 * Every candidate computes the same sums (exact integers) and, per solver,
 * the same statistic bits, so only time differs. Synchronous: it runs the
 * candidates on stream and waits for them (a warm-up and three timed runs
 * each). workspace as for rfi_process_batch (rfi_batch_workspace_size of the
 * same items); the items' stat/status buffers are written as scratch, the
 * masks are not. p->tune is ignored. */
rfi_status rfi_tune_batch(int32_t nitem, const rfi_batch_item* items /* host */,
                          const rfi_batch_params* p /* host */, void* workspace,
                          rfi_tune_table* table /* host */, rfi_stream_t stream);

typedef struct rfi_batch_graph rfi_batch_graph;
rfi_status rfi_batch_graph_create(int32_t nitem, const rfi_batch_item* items /* host */,
                                  const rfi_batch_params* p /* host */, void* workspace,
                                  rfi_batch_graph** g);
rfi_status rfi_batch_graph_launch(rfi_batch_graph* g, rfi_stream_t stream);
void rfi_batch_graph_destroy(rfi_batch_graph* g);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of observation blocks from many streams.
 *
 * A session owns one device, a set of execution slots (each a HIP stream with
 * its own workspace) and a scheduler thread. rfi_submit queues a block of a
 * stream and returns at once with a ticket. The scheduler admits queued
 * blocks in submission order while a slot is free and the session's HBM
 * budget (block input + result buffers + workspace, charged from admission to
 * rfi_result_release) allows, so blocks that arrive while others run are
 * taken as soon as slots and memory free up, and blocks of different streams
 * run concurrently on the device. Blocks of one stream run in submission
 * order, since each updates that stream's state:
 *  - the pooled clip state and fit history (rfi_stream_state, the streaming
 *    reading of the Sec. 3.3 clip: each fit pools the exact moment sums of
 *    the stream's earlier unmasked cells);
 *  - the partial sub-interval: samples after a block's last full
 *    sub-interval are summed into the stream's carry and completed by the
 *    next block, so sub-intervals span block boundaries.
 * A block's cells are: the completed carry sub-interval (if any) followed by
 * its full sub-intervals, nsub x nchan in all. The result of every block is
 * the same whether it runs alone or among other streams' blocks.
 *
 * Threading: every call is thread-safe. Block input buffers are zero-copy
 * and must stay valid and unchanged until the ticket is done. Result device
 * buffers belong to the session until rfi_result_release. */
typedef struct rfi_session rfi_session;

typedef struct {
  int32_t device;        /* HIP device ordinal */
  int32_t max_inflight;  /* execution slots, 1..64 (0 = 8); 1 = one block at a time */
  int64_t hbm_budget;    /* bytes admitted at once (0 = 64 GiB) */
  /* HOST table from rfi_tune_batch, or NULL (defaults). Copied at create;
   * each stream takes the entry whose beam range holds its nbeam when it
   * opens and uses its solver, sums tile, ring depth, XCD grouping and
   * per-lane workgroup for every block. Results do not depend on it (the
   * sums choices are bit-exact with the defaults; another solver gives the
   * same masks with statistics within its accuracy, 1e-12 for the solvers
   * rfi_tune_batch picks). Entries out of range fail rfi_stream_open with
   * RFI_E_INVALID. */
  const rfi_tune_table* tune;
} rfi_session_config;

typedef struct {
  int32_t nbeam, nchan;  /* block shape of this stream */
  int32_t L;             /* samples per sub-interval, 1..RFI_MAX_COUNT_LONG; above
                            RFI_MAX_COUNT the sums (the carry's too) are int64 and the
                            eigen stage is the FP64 tridiagonal solver, as in
                            rfi_process_block */
  int32_t eig_precision; /* 32 (0 = 32) or 64 */
  int32_t max_sweeps;    /* 0 = 12 */
  int32_t max_iter;      /* clip fits, 0 = 50 */
  double kappa;          /* clip multiple (Sec. 4.5), >= 0 */
  const uint8_t* protect_chan; /* HOST [nchan] (1 = preserved channel) or NULL; copied */
  int32_t beam_stage;    /* 1: every block also yields v1 and the per-beam mask of the
                            eigenvector stage (Sec. 3.3 last paragraph; as rfi_eigvec_flag
                            on the block's mask); 0: not */
  int32_t pad;
  double kappa_v;        /* per-beam multiple (Sec. 4.5), >= 0, read when beam_stage = 1 */
} rfi_stream_config;

typedef struct {
  uint64_t ticket, user_tag;
  int32_t stream_id;
  rfi_status status;     /* RFI_OK, or the error that ended this block */
  int32_t nsub, nchan;   /* cells of this block: nsub x nchan */
  int32_t carried;       /* 1 if row 0 is the sub-interval completed from the carry */
  int64_t carry_samples; /* samples of the stream's partial sub-interval after this block */
  const double* stat;    /* DEVICE [nsub * nchan] statistic, session-owned */
  const uint8_t* cell_status; /* DEVICE [nsub * nchan] RFI_CELL_* bits */
  const uint8_t* mask;   /* DEVICE [nsub * nchan] 1 = masked */
  rfi_flag_stats flag;   /* host copy of the block's clip summary */
  double t_submit_us, t_admit_us, t_done_us; /* host clock, microseconds since session start */
  const float* v1;       /* DEVICE [nbeam][nsub * nchan] dominant eigenvectors, or NULL
                            (stream without beam_stage) */
  const uint8_t* beam_mask; /* DEVICE [nbeam][nsub * nchan] per-beam mask, or NULL */
} rfi_result;

rfi_status rfi_session_create(const rfi_session_config* cfg /* host, nullable */,
                              rfi_session** s);
/* Waits for all admitted work, cancels queued blocks (RFI_E_CANCELLED) and
 * frees everything, including unreleased results. */
void rfi_session_destroy(rfi_session* s);
rfi_status rfi_stream_open(rfi_session* s, const rfi_stream_config* c /* host */,
                           int32_t* stream_id);
/* Waits for the stream's blocks, then frees its state. */
rfi_status rfi_stream_close(rfi_session* s, int32_t stream_id);
/* Queue one block (beam pointers and shape as for rfi_ccm_accumulate; nbeam
 * and nchan must match the stream). Errors (synchronous): RFI_E_INVALID,
 * RFI_E_BUDGET if the block alone exceeds the budget. */
rfi_status rfi_submit(rfi_session* s, int32_t stream_id, const rfi_block* blk /* host */,
                      uint64_t user_tag, uint64_t* ticket);
/* RFI_OK and *r filled when the ticket is done (r->status tells how it
 * ended); RFI_E_NOT_READY while queued or running; RFI_E_INVALID for an
 * unknown or released ticket. */
rfi_status rfi_poll(rfi_session* s, uint64_t ticket, rfi_result* r);
/* As rfi_poll, blocking up to timeout_us (< 0: no limit); RFI_E_TIMEOUT. */
rfi_status rfi_wait(rfi_session* s, uint64_t ticket, int64_t timeout_us, rfi_result* r);
/* Cancel a block that has not been admitted yet (RFI_E_NOT_READY if it is
 * already running or done). Later blocks of the stream still run. */
rfi_status rfi_cancel(rfi_session* s, uint64_t ticket);
/* Copy a done ticket's per-cell results into HOST buffers of nsub * nchan
 * elements (each pointer nullable). Synchronous. */
rfi_status rfi_result_copy(rfi_session* s, uint64_t ticket, double* stat, uint8_t* cell_status,
                           uint8_t* mask);
/* Copy a done ticket's v1 and per-beam mask ([nbeam][nsub * nchan] each,
 * HOST, nullable) of a stream opened with beam_stage = 1. Synchronous.
 * RFI_E_INVALID for a stream without the stage. */
rfi_status rfi_result_copy_beams(rfi_session* s, uint64_t ticket, float* v1,
                                 uint8_t* beam_mask);
/* Free a done ticket's result buffers and budget. */
rfi_status rfi_result_release(rfi_session* s, uint64_t ticket);
/* Checkpoint / resume of a stream (clip state, fit history, partial
 * sub-interval). Export waits for the stream's blocks; *nbytes is in/out
 * (host_buf NULL: query the size). Import needs an open stream of the same
 * nbeam, nchan and L with no block in flight. */
rfi_status rfi_stream_export(rfi_session* s, int32_t stream_id, void* host_buf, size_t* nbytes);
rfi_status rfi_stream_import(rfi_session* s, int32_t stream_id, const void* host_buf,
                             size_t nbytes);

/* Message for the last error returned on the calling thread ("" if none). */
const char* rfi_last_error(void);

/* Library version string. */
const char* rfi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RFI_H */
