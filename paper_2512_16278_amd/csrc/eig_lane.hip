// Per-cell correlation matrix, eigenvalues and statistic, one cell per LANE
// (nbeam <= 20). Sec. 3.2-3.3 of the paper: C_jk is the correlation matrix of
// the cell's beams (Eq. 1); C = Q Lambda Q^-1 (Eq. 2); the statistic is the
// dominant eigenvalue normalised as lambda_1^2 / sum_i lambda_i^2.
//
// Each lane holds its cell's symmetric matrix (packed upper triangle, N(N+1)/2
// floats) entirely in registers; every index is a compile-time constant, so
// the cyclic-by-row Jacobi sweep (Golub & Van Loan, Sec. 8.5) is straight-line
// FP32 code with no LDS traffic and no cross-lane communication. Rotations
// whose |a_pq| <= eps sqrt(|a_pp a_qq|) (eps = 2^-23) are skipped (relative
// criterion of Demmel & Veselic); a lane stops after a sweep without rotations
// or after max_sweeps.
//
// The dominant eigenvalue is then refined in FP64, since the clip compares the
// statistic against a threshold at FP64 resolution: the eigenvector v1 comes
// from inverse iteration with an FP32 Cholesky factor of (sigma I - C),
// sigma just above the FP32 lambda_1, and lambda_1 is replaced by the FP64
// Rayleigh quotient v1^T C v1 / v1^T v1 on the FP64 correlation matrix (error
// of order ||dC||^2 / gap for an FP32 v1).
#include <float.h>
#include <math.h>

#include <type_traits>

#include "internal.h"

namespace rfi {
namespace {

// Compile-time loop: every index into the register-resident matrix must be a
// constant, which this guarantees independently of the loop unroller.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
#define RFI_CI(v) decltype(v)::value

template <int N>
struct Sym {
  static constexpr int NP = N * (N + 1) / 2;
  __device__ __forceinline__ static constexpr int idx(int i, int j) {
    return i <= j ? i * N - i * (i - 1) / 2 + (j - i) : j * N - j * (j - 1) / 2 + (i - j);
  }
};

__device__ __forceinline__ int64_t pidx(int a, int b, int n) {
  return (int64_t)a * n - (int64_t)a * (a - 1) / 2 + (b - a);
}

// Build the FP32 correlation matrix of one cell from its exact sums:
// N_ab = cnt S_ab - S_a S_b in int64, r_ab = N_ab / sqrt(N_aa N_bb).
// Padding indices (>= n) get an identity row and column.
template <int N>
__device__ __forceinline__ void load_corr32(const EigArgs& g, int64_t ncell, int64_t cell,
                                            int n, int64_t cnt, float (&A)[Sym<N>::NP],
                                            bool& degenerate) {
  // N_ab = cnt S_ab - S_a S_b is formed exactly in FP64: cnt S_ab < 2^47 and
  // S_a S_b < 2^48 are integers held exactly, and the FMA's one rounding is
  // exact too (|N_ab| < 2^48 < 2^53) -- cheaper than int64 arithmetic.
  double Sd[N];
  float dinv[N];
  degenerate = false;
  const double cd = (double)cnt;
  static_for<0, N>([&](auto Ai) {
    constexpr int a = RFI_CI(Ai);
    const int aa = a < n ? a : 0;                    // clamped: always a valid address
    Sd[a] = (double)g.sum_x[aa * ncell + cell];
    const double Saa = (double)g.sum_xy[pidx(aa, aa, n) * ncell + cell];
    const double Naa = fma(cd, Saa, -Sd[a] * Sd[a]);
    dinv[a] = (a < n && Naa > 0.0) ? __builtin_amdgcn_rsqf((float)Naa) : 0.f;
    degenerate |= (a < n && Naa <= 0.0);
    A[Sym<N>::idx(a, a)] = 1.0f;
  });
  // one row at a time, so that only a row's raw sums are in flight at once
  static_for<0, N>([&](auto Ai) {
    constexpr int a = RFI_CI(Ai);
    __builtin_amdgcn_sched_barrier(0);
    static_for<a + 1, N>([&](auto Bi) {
      constexpr int b = RFI_CI(Bi);
      const int64_t p = b < n ? pidx(a, b, n) : 0;   // b < n implies a < n
      const double Sab = (double)g.sum_xy[p * ncell + cell];
      const double Nab = fma(cd, Sab, -Sd[a] * Sd[b]);
      A[Sym<N>::idx(a, b)] = b < n ? (float)Nab * dinv[a] * dinv[b] : 0.f;
    });
  });
}

template <int N>
__device__ __forceinline__ bool jacobi_sweep(float (&A)[Sym<N>::NP]) {
  constexpr float EPS = 1.1920928955078125e-07f;   // 2^-23
  bool rotated = false;
  static_for<0, N - 1>([&](auto P) {
    constexpr int p = RFI_CI(P);
    static_for<p + 1, N>([&](auto Q) {
      constexpr int q = RFI_CI(Q);
      const float apq = A[Sym<N>::idx(p, q)];
      const float app = A[Sym<N>::idx(p, p)];
      const float aqq = A[Sym<N>::idx(q, q)];
      if (apq * apq > EPS * EPS * fabsf(app * aqq)) {
        rotated = true;
        // symmetric 2x2 Schur: theta = (a_qq - a_pp) / (2 a_pq); hardware
        // rcp / sqrt / rsq (about 1 ulp) are ample: c^2 + s^2 = 1 to a few ulp
        const float theta = (aqq - app) * __builtin_amdgcn_rcpf(2.0f * apq);
        // |theta| clamped so theta^2 cannot overflow (t is then ~1/(2|theta|),
        // a rotation that is the identity to working precision)
        const float at = fminf(fabsf(theta), 1e18f);
        float t = __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.0f)));
        t = theta < 0.f ? -t : t;
        const float c = __builtin_amdgcn_rsqf(1.0f + t * t);
        const float s = t * c;
        A[Sym<N>::idx(p, p)] = app - t * apq;
        A[Sym<N>::idx(q, q)] = aqq + t * apq;
        A[Sym<N>::idx(p, q)] = 0.f;
        static_for<0, N>([&](auto K) {
          constexpr int k = RFI_CI(K);
          if constexpr (k != p && k != q) {
            const float akp = A[Sym<N>::idx(k, p)];
            const float akq = A[Sym<N>::idx(k, q)];
            A[Sym<N>::idx(k, p)] = c * akp - s * akq;
            A[Sym<N>::idx(k, q)] = s * akp + c * akq;
          }
        });
      }
    });
  });
  return rotated;
}

// Kernel 1: correlation matrix and cyclic Jacobi. Writes the FP32 dominant
// eigenvalue into stat[] (consumed by kernel 2), the optional sorted
// eigenvalues, and the status bits of this stage.
template <int N>
__device__ __forceinline__ void jacobi_cell(const EigArgs& g, int64_t cell) {
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int n = g.nbeam;
  const int64_t cnt = g.count[cell / g.nchan];
  if (cnt < 2 || cnt > RFI_MAX_COUNT) {
    g.stat[cell] = 1.0;
    g.status[cell] = RFI_CELL_BAD_COUNT | RFI_CELL_DEGENERATE;
    if (g.eigvals)
      for (int i = 0; i < n; ++i) g.eigvals[i * g.out_stride + cell] = 0.f;
    return;
  }
  uint8_t st = 0;
  float A[Sym<N>::NP];
  bool degenerate;
  load_corr32<N>(g, ncell, cell, n, cnt, A, degenerate);
  if (degenerate) st |= RFI_CELL_DEGENERATE;

  int sweep = 0;
  bool last = false;
  for (; sweep < g.max_sweeps; ++sweep) {
    last = jacobi_sweep<N>(A);
    if (!last) break;
  }
  if (last && sweep == g.max_sweeps) st |= RFI_CELL_NOT_CONVERGED;

  // dominant eigenvalue by magnitude
  float lam1 = A[Sym<N>::idx(0, 0)];
  static_for<1, N>([&](auto I) {
    constexpr int i = RFI_CI(I);
    const float v = A[Sym<N>::idx(i, i)];
    if (i < n && fabsf(v) > fabsf(lam1)) lam1 = v;
  });
  g.stat[cell] = (double)lam1;
  g.status[cell] = st;

  if (g.eigvals) {
    // all eigenvalues, |lambda| descending (odd-even transposition sort)
    float ev[N], key[N];
    static_for<0, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      ev[i] = A[Sym<N>::idx(i, i)];
      key[i] = i < n ? fabsf(ev[i]) : -1.0f;
    });
#pragma unroll
    for (int pass = 0; pass < N; ++pass) {
#pragma unroll
      for (int i = pass & 1; i + 1 < N; i += 2) {
        const bool sw = key[i + 1] > key[i];
        const float k0 = sw ? key[i + 1] : key[i], k1 = sw ? key[i] : key[i + 1];
        const float e0 = sw ? ev[i + 1] : ev[i], e1 = sw ? ev[i] : ev[i + 1];
        key[i] = k0; key[i + 1] = k1; ev[i] = e0; ev[i + 1] = e1;
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i < n) g.eigvals[i * g.out_stride + cell] = ev[i];
  }
}

// Kernel 2: eigenvector by inverse iteration and FP64 Rayleigh quotient;
// writes the statistic lambda_1^2 / ||C||_F^2, v1 and the remaining status bits.
template <int N>
__device__ __forceinline__ void refine_cell(const EigArgs& g, int64_t cell) {
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int n = g.nbeam;
  const int64_t cnt = g.count[cell / g.nchan];
  uint8_t st = g.status[cell];
  if (st & RFI_CELL_BAD_COUNT) {
    g.stat[cell] = 0.0;
    if (g.v1)
      for (int i = 0; i < n; ++i) g.v1[i * g.out_stride + cell] = 0.f;
    return;
  }
  const float lam1 = (float)g.stat[cell];

  float v[N];
  bool have_v = false;
  if (g.refine || g.v1) {
    float A[Sym<N>::NP];
    bool dg;
    load_corr32<N>(g, ncell, cell, n, cnt, A, dg);
    const float sigma = lam1 * (1.0f + 2e-5f) + 1e-6f;
    bool ok = true;
    float rinv[N];
    static_for<0, N>([&](auto J) {
      constexpr int j = RFI_CI(J);
      // column j of the factor R (B = R R^T, R lower), B = sigma I - C
      float d = sigma - A[Sym<N>::idx(j, j)];
      static_for<0, j>([&](auto K) {
        constexpr int k = RFI_CI(K);
        d -= A[Sym<N>::idx(j, k)] * A[Sym<N>::idx(j, k)];
      });
      ok = ok && d > 0.f;
      rinv[j] = 1.0f / sqrtf(fmaxf(d, 1e-30f));
      static_for<j + 1, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        float x = -A[Sym<N>::idx(i, j)];
        static_for<0, j>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(i, k)] * A[Sym<N>::idx(j, k)];
        });
        A[Sym<N>::idx(i, j)] = x * rinv[j];
      });
    });
    // start vector with no exact linear relation to any eigenvector that a
    // correlation matrix can have (all-ones is orthogonal to (1, -1) for two
    // anticorrelated beams): components 0.5 + frac(0.5 + i g), g = 0.7548...
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float f = 0.5f + 0.7548776662466927f * (float)i;
      v[i] = i < n ? 0.5f + (f - floorf(f)) : 0.0f;
    }
    for (int it = 0; it < 3; ++it) {
      // R y = v (forward), then R^T w = y (backward), in place
      static_for<0, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        float x = v[i];
        static_for<0, i>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(i, k)] * v[k];
        });
        v[i] = x * rinv[i];
      });
      static_for<0, N>([&](auto II) {
        constexpr int i = N - 1 - RFI_CI(II);
        float x = v[i];
        static_for<i + 1, N>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(k, i)] * v[k];
        });
        v[i] = x * rinv[i];
      });
      float nrm = 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) nrm += v[i] * v[i];
      const float sc = 1.0f / sqrtf(nrm);
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] *= sc;
    }
    have_v = ok;
    if (!ok) st |= RFI_CELL_REFINE_FAILED;
  }

  // FP64 pass over the exact sums: ||C||_F^2 and the Rayleigh quotient
  double num = 0.0, vv = 0.0, f2 = 0.0;
  {
    int32_t S[N];
    double d[N];
    double vd[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      S[a] = 0;
      d[a] = 0.0;
      vd[a] = have_v ? (double)v[a] : 0.0;
      if (a < n) {
        S[a] = g.sum_x[a * ncell + cell];
        const int64_t Saa = g.sum_xy[pidx(a, a, n) * ncell + cell];
        const int64_t Naa = cnt * Saa - (int64_t)S[a] * S[a];
        d[a] = Naa > 0 ? 1.0 / sqrt((double)Naa) : 0.0;
        num += vd[a] * vd[a];
        vv += vd[a] * vd[a];
        f2 += 1.0;
      }
    }
    double off = 0.0, offv = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = a + 1; b < N; ++b) {
        if (b < n) {
          const int64_t Sab = g.sum_xy[pidx(a, b, n) * ncell + cell];
          const int64_t Nab = cnt * Sab - (int64_t)S[a] * S[b];
          const double r = (double)Nab * d[a] * d[b];
          off += r * r;
          offv += r * vd[a] * vd[b];
        }
      }
    f2 += 2.0 * off;
    num += 2.0 * offv;
  }
  const double lam = (g.refine && have_v) ? num / vv : (double)lam1;
  g.stat[cell] = lam * lam / f2;
  g.status[cell] = st;

  if (g.v1) {
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) sum += v[i];
    float first = 0.f;
#pragma unroll
    for (int i = N - 1; i >= 0; --i)
      if (i < n && v[i] != 0.f) first = v[i];
    const float sgn = (sum < 0.f || (sum == 0.f && first < 0.f)) ? -1.0f : 1.0f;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i < n) g.v1[i * g.out_stride + cell] = have_v ? sgn * v[i] : 0.f;
  }
}

template <int N>
__global__ __launch_bounds__(256) void eig_lane_jacobi(EigArgs g) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < (int64_t)g.nsub * g.nchan) jacobi_cell<N>(g, cell);
}

template <int N>
__global__ __launch_bounds__(256) void eig_lane_refine(EigArgs g) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < (int64_t)g.nsub * g.nchan) refine_cell<N>(g, cell);
}

// Batched: the cells of several blocks (one EigArgs each, in device memory)
// as one index space; cell0[i] = first global cell of item i (ascending).
__device__ __forceinline__ int find_item(const int64_t* cell0, int nitem, int64_t c) {
  int lo = 0, hi = nitem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell0[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int N>
__global__ __launch_bounds__(256) void eig_lane_jacobi_batch(const EigArgs* items,
                                                             const int64_t* cell0, int nitem,
                                                             int64_t total) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  const int i = find_item(cell0, nitem, c);
  const EigArgs g = items[i];
  jacobi_cell<N>(g, c - cell0[i]);
}

template <int N>
__global__ __launch_bounds__(256) void eig_lane_refine_batch(const EigArgs* items,
                                                             const int64_t* cell0, int nitem,
                                                             int64_t total) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  const int i = find_item(cell0, nitem, c);
  const EigArgs g = items[i];
  refine_cell<N>(g, c - cell0[i]);
}

template <int N>
hipError_t launch_batch_n(const EigArgs* items, const int64_t* cell0, int nitem, int64_t total,
                          int wg, hipStream_t s) {
  const dim3 grid((unsigned)((total + wg - 1) / wg));
  hipLaunchKernelGGL(eig_lane_jacobi_batch<N>, grid, dim3(wg), 0, s, items, cell0, nitem, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_lane_refine_batch<N>, grid, dim3(wg), 0, s, items, cell0, nitem, total);
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const EigArgs& a, int wg, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  const dim3 grid((unsigned)((ncell + wg - 1) / wg));
  hipLaunchKernelGGL(eig_lane_jacobi<N>, grid, dim3(wg), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_lane_refine<N>, grid, dim3(wg), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int eig_lane_class(int n) {
  if (n <= 4) return 4;
  if (n <= 8) return 8;
  if (n <= 12) return 12;
  if (n <= 16) return 16;
  if (n == 19) return 19;
  if (n <= 20) return 20;
  return 0;
}

hipError_t launch_eig_lane_batch(int cls, const EigArgs* items, const int64_t* cell0, int nitem,
                                 int64_t total, hipStream_t s, int wg) {
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  switch (cls) {
    case 4: return launch_batch_n<4>(items, cell0, nitem, total, wg, s);
    case 8: return launch_batch_n<8>(items, cell0, nitem, total, wg, s);
    case 12: return launch_batch_n<12>(items, cell0, nitem, total, wg, s);
    case 16: return launch_batch_n<16>(items, cell0, nitem, total, wg, s);
    case 19: return launch_batch_n<19>(items, cell0, nitem, total, wg, s);
    case 20: return launch_batch_n<20>(items, cell0, nitem, total, wg, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eig_lane(const EigArgs& a, hipStream_t s, int wg) {
  const int n = a.nbeam;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  if (n <= 4) return launch_n<4>(a, wg, s);
  if (n <= 8) return launch_n<8>(a, wg, s);
  if (n <= 12) return launch_n<12>(a, wg, s);
  if (n <= 16) return launch_n<16>(a, wg, s);
  if (n == 19) return launch_n<19>(a, wg, s);
  if (n <= 20) return launch_n<20>(a, wg, s);
  return hipErrorInvalidValue;
}

}  // namespace rfi
