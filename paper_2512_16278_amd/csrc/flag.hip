// Iterative Gaussian clipping of the statistic into the RFI mask (Sec. 3.3:
// the mean and standard deviation of the dominant eigenvalues are fitted, the
// cells above a dynamic threshold are masked, and this repeats until
// convergence; the threshold multiple kappa is the eigenvalue threshold
// parameter of Sec. 4.5; preserved channels of Sec. 4.3 are excluded), and
// the per-beam eigenvector threshold (Sec. 3.3 last paragraph; kappa_v of
// Sec. 4.5).
//
// The clip works on the statistic quantised to q = rint(s 2^40). Its moment
// sums N, Q1 = sum q and Q2 = sum q^2 are exact integers (64/128-bit), so every
// reduction order gives the same fit; mu and sigma are formed from them once
// in FP64. The masked set is always {q > T} for the running minimum T of the
// thresholds (in units of 2^-40), so an iteration is one pass that sums the
// eligible cells with q <= T; the pass after a fit tells whether that fit
// masked anything new (the count dropped). One workgroup of 1024 threads does
// all passes, so no grid-wide synchronisation is needed.
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

typedef unsigned __int128 u128;
constexpr double TWO40 = 1099511627776.0;   // 2^40
constexpr int FT = 1024;

__device__ __forceinline__ u128 mk128(uint64_t lo, uint64_t hi) {
  return ((u128)hi << 64) | (u128)lo;
}

// FP64 value of a 256-bit unsigned integer given as 4 little-endian limbs.
__device__ double u256_to_double(const uint64_t w[4]) {
  double r = 0.0;
  for (int i = 3; i >= 0; --i) r = r * 18446744073709551616.0 + (double)w[i];
  return r;
}

// w = a * b for 128-bit a, b (256-bit result)
__device__ void mul128(u128 a, u128 b, uint64_t w[4]) {
  const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
  const uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  const u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  w[0] = (uint64_t)p00;
  w[1] = (uint64_t)mid;
  const u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
  w[2] = (uint64_t)hi;
  w[3] = (uint64_t)(hi >> 64) + (uint64_t)(p11 >> 64);
}

__device__ void sub256(uint64_t a[4], const uint64_t b[4]) {
  uint64_t borrow = 0;
  for (int i = 0; i < 4; ++i) {
    const uint64_t x = a[i] - b[i] - borrow;
    borrow = (a[i] < b[i] || (a[i] == b[i] && borrow)) ? 1 : 0;
    a[i] = x;
  }
}

// mu = Q1 / (N 2^40); sigma^2 = (N Q2 - Q1^2) / (N^2 2^80)
__device__ void fit(int64_t N, u128 Q1, u128 Q2, double& mu, double& sigma) {
  const double dN = (double)N;
  mu = ((double)Q1 / dN) / TWO40;
  uint64_t a[4], b[4];
  mul128((u128)(uint64_t)N, Q2, a);
  mul128(Q1, Q1, b);
  sub256(a, b);
  const double var = (u256_to_double(a) / (dN * dN)) / (TWO40 * TWO40);
  sigma = sqrt(var);
}

__device__ __forceinline__ bool eligible(const uint8_t* status, const uint8_t* protect,
                                         int64_t c, int nchan) {
  if (status[c] & (RFI_CELL_DEGENERATE | RFI_CELL_BAD_COUNT)) return false;
  if (protect && protect[c % nchan]) return false;
  return true;
}

struct Shared {
  int64_t n[FT / 64];
  u128 q1[FT / 64];
  u128 q2[FT / 64];
  int64_t T;        // live cells: q <= T
  int stop;
};

// Sum (count, q, q^2) over eligible cells with q <= T; result valid in thread 0.
__device__ void pass_sums(const double* stat, const uint8_t* status, const uint8_t* protect,
                          int64_t ncell, int nchan, int64_t T, Shared& sh, int64_t& N,
                          u128& Q1, u128& Q2) {
  int64_t n = 0;
  u128 q1 = 0, q2 = 0;
  for (int64_t c = threadIdx.x; c < ncell; c += FT) {
    if (!eligible(status, protect, c, nchan)) continue;
    const int64_t q = __double2ll_rn(stat[c] * TWO40);
    if (q > T) continue;
    n += 1;
    q1 += (u128)(uint64_t)q;
    q2 += (u128)(uint64_t)q * (u128)(uint64_t)q;
  }
  // wave partials in a fixed order (integer sums: order is irrelevant anyway)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    n += __shfl_down(n, off);
    const uint64_t a0 = __shfl_down((uint64_t)q1, off), a1 = __shfl_down((uint64_t)(q1 >> 64), off);
    const uint64_t b0 = __shfl_down((uint64_t)q2, off), b1 = __shfl_down((uint64_t)(q2 >> 64), off);
    if (lane + off < 64) {
      q1 += mk128(a0, a1);
      q2 += mk128(b0, b1);
    }
  }
  if (lane == 0) {
    sh.n[wave] = n;
    sh.q1[wave] = q1;
    sh.q2[wave] = q2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    N = 0;
    Q1 = 0;
    Q2 = 0;
    for (int w = 0; w < FT / 64; ++w) {
      N += sh.n[w];
      Q1 += sh.q1[w];
      Q2 += sh.q2[w];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(FT) void flag_kernel(int nsub, int nchan, const double* __restrict__ stat,
                                                  const uint8_t* __restrict__ status,
                                                  const uint8_t* __restrict__ protect, double kappa,
                                                  int max_iter, rfi_stream_state* state,
                                                  uint8_t* __restrict__ mask,
                                                  rfi_flag_stats* out) {
  __shared__ Shared sh;
  const int64_t ncell = (int64_t)nsub * nchan;
  // pooled history (thread 0 only uses it)
  int64_t Nh = 0;
  u128 Q1h = 0, Q2h = 0;
  if (state && threadIdx.x == 0) {
    Nh = state->n;
    Q1h = mk128(state->q1[0], state->q1[1]);
    Q2h = mk128(state->q2[0], state->q2[1]);
  }
  if (threadIdx.x == 0) {
    sh.T = INT64_MAX;
    sh.stop = 0;
  }
  __syncthreads();

  int64_t prevN = -1, N = 0, Nelig = 0;
  u128 Q1 = 0, Q2 = 0;
  int it = 0, converged = 1;
  double mu = NAN, sigma = NAN, thr = NAN;
  for (int guard = 0; guard <= max_iter + 1; ++guard) {
    pass_sums(stat, status, protect, ncell, nchan, sh.T, sh, N, Q1, Q2);
    if (threadIdx.x == 0) {
      if (guard == 0) Nelig = N;
      int stop = 0;
      if (it > 0 && N == prevN) {
        stop = 1;                       // the last fit masked nothing new
      } else if (it > 0 && it >= max_iter) {
        stop = 1;                       // capped while still masking
        converged = 0;
      } else if (N + Nh == 0) {
        stop = 1;                       // nothing left to fit
      } else {
        ++it;
        fit(N + Nh, Q1 + Q1h, Q2 + Q2h, mu, sigma);
        thr = mu + kappa * sigma;
        // s_q > thr  <=>  q > thr 2^40  <=>  q > floor(thr 2^40)
        const double tq = floor(thr * TWO40);
        const int64_t Tnew = tq >= 9.2e18 ? INT64_MAX : (tq < -9.2e18 ? INT64_MIN : (int64_t)tq);
        if (Tnew < sh.T) sh.T = Tnew;
        prevN = N;
      }
      sh.stop = stop;
    }
    __syncthreads();
    if (sh.stop) break;
  }
  const int64_t T = sh.T;
  for (int64_t c = threadIdx.x; c < ncell; c += FT) {
    uint8_t mval = 0;
    if (eligible(status, protect, c, nchan)) {
      const int64_t q = __double2ll_rn(stat[c] * TWO40);
      mval = q > T ? 1 : 0;
    }
    mask[c] = mval;
  }
  if (threadIdx.x == 0) {
    if (out) {
      out->mu = mu;
      out->sigma = sigma;
      out->thr = thr;
      out->iterations = it;
      out->converged = converged;
      out->nflag = Nelig - N;
      out->nfit = N;
    }
    if (state) {
      const u128 a = Q1h + Q1, b = Q2h + Q2;
      state->n = Nh + N;
      state->q1[0] = (uint64_t)a;
      state->q1[1] = (uint64_t)(a >> 64);
      state->q2[0] = (uint64_t)b;
      state->q2[1] = (uint64_t)(b >> 64);
      rfi_hist_entry& h = state->hist[state->nblocks % RFI_HIST_CAP];
      h.mu = mu;
      h.sigma = sigma;
      h.thr = thr;
      h.iterations = it;
      h.converged = converged;
      state->nblocks += 1;
    }
  }
}

// Per-beam eigenvector threshold: one workgroup per beam.
__global__ __launch_bounds__(FT) void eigvec_kernel(int nbeam, int nsub, int nchan,
                                                    const float* __restrict__ v1,
                                                    const uint8_t* __restrict__ mask,
                                                    const uint8_t* __restrict__ status,
                                                    const uint8_t* __restrict__ protect,
                                                    double kappa_v, uint8_t* __restrict__ beam_mask,
                                                    double* beam_mu, double* beam_sigma) {
  __shared__ double s1[FT / 64], s2[FT / 64];
  __shared__ int64_t sn[FT / 64];
  __shared__ double fit_thr;
  const int b = blockIdx.x;
  const int64_t ncell = (int64_t)nsub * nchan;
  const float* vb = v1 + (int64_t)b * ncell;
  // pass 1: mean of |v_b| over eligible unmasked cells
  double a1 = 0.0;
  int64_t n = 0;
  for (int64_t c = threadIdx.x; c < ncell; c += FT) {
    if (!eligible(status, protect, c, nchan) || mask[c]) continue;
    a1 += fabs((double)vb[c]);
    n += 1;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    a1 += __shfl_down(a1, off);
    n += __shfl_down(n, off);
  }
  if (lane == 0) { s1[wave] = a1; sn[wave] = n; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    int64_t nn = 0;
    for (int w = 0; w < FT / 64; ++w) { t += s1[w]; nn += sn[w]; }
    s1[0] = nn > 0 ? t / (double)nn : NAN;
    sn[0] = nn;
  }
  __syncthreads();
  const double mu = s1[0];
  const int64_t ntot = sn[0];
  __syncthreads();
  // pass 2: population variance about mu
  double a2 = 0.0;
  for (int64_t c = threadIdx.x; c < ncell; c += FT) {
    if (!eligible(status, protect, c, nchan) || mask[c]) continue;
    const double dv = fabs((double)vb[c]) - mu;
    a2 += dv * dv;
  }
  for (int off = 32; off > 0; off >>= 1) a2 += __shfl_down(a2, off);
  if (lane == 0) s2[wave] = a2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < FT / 64; ++w) t += s2[w];
    const double sd = ntot > 0 ? sqrt(t / (double)ntot) : NAN;
    fit_thr = mu + kappa_v * sd;
    if (beam_mu) beam_mu[b] = mu;
    if (beam_sigma) beam_sigma[b] = sd;
  }
  __syncthreads();
  const double thr = fit_thr;
  uint8_t* out = beam_mask + (int64_t)b * ncell;
  for (int64_t c = threadIdx.x; c < ncell; c += FT)
    out[c] = (mask[c] && fabs((double)vb[c]) > thr) ? 1 : 0;
}

}  // namespace

hipError_t launch_flag(int nsub, int nchan, const double* stat, const uint8_t* status,
                       const uint8_t* protect_chan, double kappa, int max_iter,
                       rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(flag_kernel, dim3(1), dim3(FT), 0, s, nsub, nchan, stat, status,
                     protect_chan, kappa, max_iter, state, mask, out);
  return hipGetLastError();
}

hipError_t launch_eigvec_flag(int nbeam, int nsub, int nchan, const float* v1,
                              const uint8_t* mask, const uint8_t* status,
                              const uint8_t* protect_chan, double kappa_v,
                              uint8_t* beam_mask, double* beam_mu, double* beam_sigma,
                              hipStream_t s) {
  hipLaunchKernelGGL(eigvec_kernel, dim3(nbeam), dim3(FT), 0, s, nbeam, nsub, nchan, v1, mask,
                     status, protect_chan, kappa_v, beam_mask, beam_mu, beam_sigma);
  return hipGetLastError();
}

}  // namespace rfi
