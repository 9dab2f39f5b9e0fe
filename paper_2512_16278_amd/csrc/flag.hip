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
// masked anything new (the count dropped). The main kernel spreads the cells
// over one co-resident workgroup per CU (below); a single-workgroup kernel
// that re-reads the statistic every pass covers very large blocks.
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

typedef unsigned __int128 u128;
constexpr double TWO40 = 1099511627776.0;   // 2^40
constexpr int FT = 1024;
constexpr int kMaxFlagWg = 1024;     // workgroups of the grid-wide clip

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

__device__ __forceinline__ void flag_body(int nsub, int nchan, const double* __restrict__ stat,
                                          const uint8_t* __restrict__ status,
                                          const uint8_t* __restrict__ protect, double kappa,
                                          int max_iter, rfi_stream_state* state,
                                          uint8_t* __restrict__ mask, rfi_flag_stats* out) {
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

__global__ __launch_bounds__(FT) void flag_kernel(int nsub, int nchan, const double* __restrict__ stat,
                                                  const uint8_t* __restrict__ status,
                                                  const uint8_t* __restrict__ protect, double kappa,
                                                  int max_iter, rfi_stream_state* state,
                                                  uint8_t* __restrict__ mask,
                                                  rfi_flag_stats* out) {
  flag_body(nsub, nchan, stat, status, protect, kappa, max_iter, state, mask, out);
}

// Batched: one workgroup per block, each clipping its own cells.
__global__ __launch_bounds__(FT) void flag_batch_kernel(const FlagItem* __restrict__ items) {
  const FlagItem& it = items[blockIdx.x];
  flag_body(it.nsub, it.nchan, it.stat, it.status, it.protect, it.kappa, it.max_iter, it.state,
            it.mask, it.out);
}

// ---------------------------------------------------------------------------
// Grid-wide version: one workgroup per CU, co-resident (cooperative launch).
// Each workgroup keeps the quantised statistic of its contiguous slice of
// cells in LDS, so only the first pass reads HBM. Per iteration every
// workgroup publishes its exact partial sums, meets the others at a bounded
// grid barrier, and sums all partials itself (integer sums: every workgroup
// gets the identical totals and takes the identical decision).
constexpr int CT = 1024;                 // threads per workgroup
constexpr int SLICE_MAX = 8192;          // cells per workgroup kept in LDS (64 KB)
constexpr unsigned SPIN_LIMIT = 1u << 26; // bounded wait: ~ seconds, never a hang

struct Part {
  int64_t n;
  uint64_t q1[2];
  uint64_t q2[2];
};

struct CoopWs {
  unsigned arrive;          // grid barrier counter (zeroed before launch)
  unsigned timeout;         // set if a barrier wait gave up
  unsigned pad[2];
  Part part[2][1];          // [2][nwg], double-buffered by iteration parity
};

__global__ void coop_ws_reset(CoopWs* ws) {
  ws->arrive = 0;
  ws->timeout = 0;
}

__device__ __forceinline__ void grid_barrier(CoopWs* ws, unsigned target) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&ws->arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(&ws->arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > SPIN_LIMIT) {
        __hip_atomic_store(&ws->timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(CT) void flag_coop_kernel(int nsub, int nchan,
                                                       const double* __restrict__ stat,
                                                       const uint8_t* __restrict__ status,
                                                       const uint8_t* __restrict__ protect,
                                                       double kappa, int max_iter,
                                                       rfi_stream_state* state,
                                                       uint8_t* __restrict__ mask,
                                                       rfi_flag_stats* out, CoopWs* ws) {
  __shared__ int64_t qs[SLICE_MAX];
  __shared__ int64_t wn[CT / 64];
  __shared__ u128 wq1[CT / 64], wq2[CT / 64];
  __shared__ int64_t sT;
  __shared__ int sstop;
  const int nwg = gridDim.x, wg = blockIdx.x;
  const int64_t ncell = (int64_t)nsub * nchan;
  const int64_t per = (ncell + nwg - 1) / nwg;
  const int64_t c0 = (int64_t)wg * per;
  const int64_t c1 = c0 + per < ncell ? c0 + per : ncell;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Part* parts = ws->part[0];

  // pass 0: quantise the slice into LDS (INT64_MIN marks ineligible cells)
  for (int64_t c = c0 + threadIdx.x; c < c1; c += CT)
    qs[c - c0] = eligible(status, protect, c, nchan) ? __double2ll_rn(stat[c] * TWO40) : INT64_MIN;
  int64_t Nh = 0;
  u128 Q1h = 0, Q2h = 0;
  if (state) {
    Nh = state->n;
    Q1h = mk128(state->q1[0], state->q1[1]);
    Q2h = mk128(state->q2[0], state->q2[1]);
  }
  if (threadIdx.x == 0) { sT = INT64_MAX; sstop = 0; }
  __syncthreads();

  int64_t prevN = -1, N = 0, Nelig = 0;
  u128 Q1 = 0, Q2 = 0;
  int it = 0, converged = 1;
  double mu = NAN, sigma = NAN, thr = NAN;
  for (int pass = 0; pass <= max_iter + 1; ++pass) {
    const int64_t T = sT;
    int64_t n = 0;
    u128 q1 = 0, q2 = 0;
    for (int64_t i = threadIdx.x; i < c1 - c0; i += CT) {
      const int64_t q = qs[i];
      if (q == INT64_MIN || q > T) continue;
      n += 1;
      q1 += (u128)(uint64_t)q;
      q2 += (u128)(uint64_t)q * (u128)(uint64_t)q;
    }
    for (int off = 32; off > 0; off >>= 1) {
      n += __shfl_down(n, off);
      const uint64_t a0 = __shfl_down((uint64_t)q1, off), a1 = __shfl_down((uint64_t)(q1 >> 64), off);
      const uint64_t b0 = __shfl_down((uint64_t)q2, off), b1 = __shfl_down((uint64_t)(q2 >> 64), off);
      if (lane + off < 64) { q1 += mk128(a0, a1); q2 += mk128(b0, b1); }
    }
    if (lane == 0) { wn[wave] = n; wq1[wave] = q1; wq2[wave] = q2; }
    __syncthreads();
    Part* slot = parts + (pass & 1) * nwg;
    if (threadIdx.x == 0) {
      int64_t tn = 0;
      u128 t1 = 0, t2 = 0;
      for (int w = 0; w < CT / 64; ++w) { tn += wn[w]; t1 += wq1[w]; t2 += wq2[w]; }
      Part pr;
      pr.n = tn;
      pr.q1[0] = (uint64_t)t1; pr.q1[1] = (uint64_t)(t1 >> 64);
      pr.q2[0] = (uint64_t)t2; pr.q2[1] = (uint64_t)(t2 >> 64);
      slot[wg] = pr;
    }
    grid_barrier(ws, (unsigned)(pass + 1) * (unsigned)nwg);
    if (__hip_atomic_load(&ws->timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    // every workgroup sums all partials (exact, so identical everywhere)
    n = 0; q1 = 0; q2 = 0;
    for (int w = threadIdx.x; w < nwg; w += CT) {
      const Part pr = slot[w];
      n += pr.n;
      q1 += mk128(pr.q1[0], pr.q1[1]);
      q2 += mk128(pr.q2[0], pr.q2[1]);
    }
    for (int off = 32; off > 0; off >>= 1) {
      n += __shfl_down(n, off);
      const uint64_t a0 = __shfl_down((uint64_t)q1, off), a1 = __shfl_down((uint64_t)(q1 >> 64), off);
      const uint64_t b0 = __shfl_down((uint64_t)q2, off), b1 = __shfl_down((uint64_t)(q2 >> 64), off);
      if (lane + off < 64) { q1 += mk128(a0, a1); q2 += mk128(b0, b1); }
    }
    __syncthreads();
    if (lane == 0) { wn[wave] = n; wq1[wave] = q1; wq2[wave] = q2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      N = 0; Q1 = 0; Q2 = 0;
      for (int w = 0; w < CT / 64; ++w) { N += wn[w]; Q1 += wq1[w]; Q2 += wq2[w]; }
      if (pass == 0) Nelig = N;
      int stop = 0;
      if (it > 0 && N == prevN) {
        stop = 1;
      } else if (it > 0 && it >= max_iter) {
        stop = 1;
        converged = 0;
      } else if (N + Nh == 0) {
        stop = 1;
      } else {
        ++it;
        fit(N + Nh, Q1 + Q1h, Q2 + Q2h, mu, sigma);
        thr = mu + kappa * sigma;
        const double tq = floor(thr * TWO40);
        const int64_t Tnew = tq >= 9.2e18 ? INT64_MAX : (tq < -9.2e18 ? INT64_MIN : (int64_t)tq);
        if (Tnew < sT) sT = Tnew;
        prevN = N;
      }
      sstop = stop;
    }
    __syncthreads();
    if (sstop) break;
  }
  const int64_t T = sT;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += CT) {
    const int64_t q = qs[c - c0];
    mask[c] = (q != INT64_MIN && q > T) ? 1 : 0;
  }
  if (wg == 0 && threadIdx.x == 0) {
    const bool tmo = __hip_atomic_load(&ws->timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (out) {
      out->mu = mu;
      out->sigma = sigma;
      out->thr = thr;
      out->iterations = tmo ? -1 : it;
      out->converged = tmo ? 0 : converged;
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

size_t flag_workspace_size(int nsub, int nchan) {
  (void)nsub; (void)nchan;
  return sizeof(CoopWs) + 2 * (size_t)kMaxFlagWg * sizeof(Part);
}

hipError_t launch_flag(int nsub, int nchan, const double* stat, const uint8_t* status,
                       const uint8_t* protect_chan, double kappa, int max_iter,
                       rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out,
                       void* workspace, hipStream_t s) {
  const int64_t ncell = (int64_t)nsub * nchan;
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)flag_coop_kernel, CT, 0);
  if (e != hipSuccess) return e;
  int nwg = ncu;                       // one co-resident workgroup per CU
  if (nwg > kMaxFlagWg) nwg = kMaxFlagWg;
  // small problems: fewer workgroups (at least 256 cells each)
  const int64_t want = (ncell + 255) / 256;
  if (want < nwg) nwg = (int)(want < 1 ? 1 : want);
  if (per_cu < 1 || ncell > (int64_t)nwg * SLICE_MAX || workspace == nullptr) {
    // one workgroup re-reading the statistic every pass
    hipLaunchKernelGGL(flag_kernel, dim3(1), dim3(FT), 0, s, nsub, nchan, stat, status,
                       protect_chan, kappa, max_iter, state, mask, out);
    return hipGetLastError();
  }
  CoopWs* ws = (CoopWs*)workspace;
  hipLaunchKernelGGL(coop_ws_reset, dim3(1), dim3(1), 0, s, ws);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&nsub, &nchan, &stat, &status, &protect_chan, &kappa, &max_iter,
                  &state, &mask, &out, &ws};
  return hipLaunchCooperativeKernel((const void*)flag_coop_kernel, dim3(nwg), dim3(CT), args, 0, s);
}

hipError_t launch_flag_batch(const FlagItem* items, int nitem, hipStream_t s) {
  hipLaunchKernelGGL(flag_batch_kernel, dim3((unsigned)nitem), dim3(FT), 0, s, items);
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
