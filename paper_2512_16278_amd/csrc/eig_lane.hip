// Per-cell correlation matrix, eigenvalues and statistic, one cell per LANE
// (nbeam <= 20). Sec. 3.2-3.3 of the paper: C_jk is the correlation matrix of
// the cell's beams (Eq. 1); C = Q Lambda Q^-1 (Eq. 2); the statistic is the
// dominant eigenvalue normalised as lambda_1^2 / sum_i lambda_i^2.
//
// Each lane holds its cell's symmetric matrix (packed upper triangle, N(N+1)/2
// floats) entirely in registers; every index is a compile-time constant, so
// the solvers are straight-line FP32 code with no LDS traffic and no
// cross-lane communication. Two solvers for the first kernel:
//  - cyclic-by-row Jacobi (Golub & Van Loan, Sec. 8.5). Rotations whose
//    |a_pq| <= eps sqrt(|a_pp a_qq|) (eps = 2^-23) are skipped (relative
//    criterion of Demmel & Veselic); a lane stops after a sweep without
//    rotations or after max_sweeps;
//  - Householder reduction to tridiagonal form (Sec. 8.3) and Sturm
//    bisection (Sec. 8.4): about (4/3) n^3 flops instead of 6 n^3 per sweep.
//
// The dominant eigenvalue is then refined in FP64, since the clip compares the
// statistic against a threshold at FP64 resolution: two vectors of block
// inverse iteration with an FP32 Cholesky factor of (sigma I - C), sigma just
// above the FP32 lambda_1, span (nearly) the eigenvectors of lambda_1 and
// lambda_2; lambda_1 is replaced by the largest Ritz value of the FP64
// correlation matrix on that span. The subspace converges at the rate
// (sigma - lambda_2) / (sigma - lambda_3), so a lambda_2 within the shift
// distance of lambda_1 (where one vector of inverse iteration would stall and
// its Rayleigh quotient miss lambda_1 by up to the gap) costs nothing.
//
// The kernels are bound by the latency of reading the cell's raw sums, not by
// arithmetic: loads are unconditional (padding reads a clamped valid address
// and is zeroed by its scale factor, so the compiler cannot sink a load into
// a branch that waits for it alone) and issued in large groups, and the
// Householder and refinement kernels run one wave per SIMD so that their
// register overflow goes to AGPRs: a scratch reload would wait for every
// load in flight.
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

// Rows of the strict upper triangle are read in groups of about G loads: row a
// opens a group when the rows since the last group start hold >= G entries.
// A fence at each group start bounds the raw sums in flight, while the loads
// of one group overlap a single memory round trip.
template <int N, int G>
__device__ __forceinline__ constexpr bool row_group_start(int a) {
  int acc = 0;
  for (int k = 0; k < a; ++k) {
    acc += N - 1 - k;
    if (acc >= G) acc = 0;
  }
  return acc == 0;
}
constexpr int kRowGroup = 48;

// Entry of this lane's cell in row `row` of a [rows][ncell] int32 array: a
// wave-uniform row address plus the lane's 32-bit byte offset off4 = 4 cell,
// which the load takes as a scalar base and one offset register (the launch
// checks ncell <= 2^30). A 64-bit per-lane address would hold two more
// registers for every load in flight.
// The pointer is taken as global memory: the batched kernels read it from
// their item table, where the compiler cannot tell the address space, and
// a flat load would also count against the LDS/scalar counter, so every wait
// for a scalar load would wait for the sums in flight as well.
__device__ __forceinline__ int32_t lane_row(const int32_t* base, int64_t row, int64_t ncell,
                                            uint32_t off4) {
  typedef const __attribute__((address_space(1))) int32_t gint32;
  return *(gint32*)((const char*)(base + row * ncell) + off4);
}

// Entry k of the strict upper triangle of an N x N matrix in row order:
// (0,1), (0,2), ..., (0,N-1), (1,2), ...
template <int N>
struct UpperPair {
  static constexpr int row(int k) {
    int a = 0;
    while (k >= N - 1 - a) {
      k -= N - 1 - a;
      ++a;
    }
    return a;
  }
  static constexpr int col(int k) {
    int a = 0;
    while (k >= N - 1 - a) {
      k -= N - 1 - a;
      ++a;
    }
    return a + 1 + k;
  }
};

__device__ __forceinline__ int64_t pidx(int a, int b, int n) {
  return (int64_t)a * n - (int64_t)a * (a - 1) / 2 + (b - a);
}

// Where a lane finds the raw sums of its cell: S_a (row a of sum_x), S_aa and
// S_ab (rows of sum_xy); pair k is (a, b) = UpperPair<N>(k). Padding indices
// (>= n) read a clamped valid row. RowsDirect forms each row's address from
// the arrays; RowsTable reads it from a per-workgroup table in LDS, filled
// once, which spares every load the 64-bit scalar address arithmetic (about
// ten scalar instructions each, 2 n + n (n - 1) / 2 loads per pass).
template <int N>
struct RowsDirect {
  const int32_t* sx;
  const int32_t* sxy;
  int64_t ncell;
  int n;
  __device__ __forceinline__ int32_t S(int a, uint32_t off4) const {
    return lane_row(sx, a < n ? a : 0, ncell, off4);
  }
  __device__ __forceinline__ int32_t Sdg(int a, uint32_t off4) const {
    const int aa = a < n ? a : 0;
    return lane_row(sxy, pidx(aa, aa, n), ncell, off4);
  }
  __device__ __forceinline__ int32_t pair(int a, int b, int, uint32_t off4) const {
    return lane_row(sxy, b < n ? pidx(a, b, n) : 0, ncell, off4);   // b < n implies a < n
  }
};

template <int N>
struct RowTab {
  static constexpr int K = 2 * N + N * (N - 1) / 2;   // S rows, S_aa rows, pairs
};

__device__ __forceinline__ int32_t lane_at(uint64_t row, uint32_t off4) {
  typedef const __attribute__((address_space(1))) int32_t gint32;
  return *(gint32*)((const char*)(uintptr_t)row + off4);
}

template <int N>
struct RowsTable {
  const uint64_t* tab;   // LDS, RowTab<N>::K row addresses
  __device__ __forceinline__ int32_t S(int a, uint32_t off4) const { return lane_at(tab[a], off4); }
  __device__ __forceinline__ int32_t Sdg(int a, uint32_t off4) const {
    return lane_at(tab[N + a], off4);
  }
  __device__ __forceinline__ int32_t pair(int, int, int k, uint32_t off4) const {
    return lane_at(tab[2 * N + k], off4);
  }
};

// The table of a launch over one block (the same rows as RowsDirect reads),
// filled by the workgroup's threads; the caller synchronises.
template <int N>
__device__ __forceinline__ void fill_rows(const EigArgs& g, uint64_t* tab) {
  const int n = g.nbeam;
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  for (int e = threadIdx.x; e < RowTab<N>::K; e += blockDim.x) {
    const int32_t* base;
    int64_t row;
    if (e < N) {
      base = g.sum_x;
      row = e < n ? e : 0;
    } else if (e < 2 * N) {
      const int aa = e - N < n ? e - N : 0;
      base = g.sum_xy;
      row = pidx(aa, aa, n);
    } else {
      const int k = e - 2 * N;
      const int a = UpperPair<N>::row(k), b = UpperPair<N>::col(k);
      base = g.sum_xy;
      row = b < n ? pidx(a, b, n) : 0;
    }
    tab[e] = (uint64_t)(uintptr_t)(base + row * ncell);
  }
}

// 1 / sqrt(x) for x > 0 to about 1 ulp: the hardware estimate and one Newton
// step, r (3 - x r^2) / 2 (the correctly rounded division and square root
// cost tens of instructions each, 2 n of them per cell).
__device__ __forceinline__ double rsqrt64(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  return r * fma(-0.5 * x * r, r, 1.5);
}

// Build the FP32 correlation matrix of one cell from its exact sums:
// N_ab = cnt S_ab - S_a S_b in int64, r_ab = N_ab / sqrt(N_aa N_bb).
// Padding indices (>= n) get an identity row and column.
template <int N, class Rows>
__device__ __forceinline__ void load_corr32(const Rows& rows, int64_t cell, int n, int64_t cnt,
                                            float (&A)[Sym<N>::NP], bool& degenerate) {
  // N_ab = cnt S_ab - S_a S_b is formed exactly in FP64: cnt S_ab < 2^47 and
  // S_a S_b < 2^48 are integers held exactly, and the FMA's one rounding is
  // exact too (|N_ab| < 2^48 < 2^53) -- cheaper than int64 arithmetic.
  int32_t S[N];
  float dinv[N];
  degenerate = false;
  const double cd = (double)cnt;
  const uint32_t off4 = (uint32_t)cell * 4u;
  static_for<0, N>([&](auto Ai) {
    constexpr int a = RFI_CI(Ai);
    S[a] = rows.S(a, off4);                          // clamped: always a valid address
    const double Sa = (double)S[a];
    const double Saa = (double)rows.Sdg(a, off4);
    const double Naa = fma(cd, Saa, -Sa * Sa);
    dinv[a] = (a < n && Naa > 0.0) ? __builtin_amdgcn_rsqf((float)Naa) : 0.f;
    degenerate |= (a < n && Naa <= 0.0);
    A[Sym<N>::idx(a, a)] = 1.0f;
  });
  static_for<0, N>([&](auto Ai) {
    constexpr int a = RFI_CI(Ai);
    if constexpr (row_group_start<N, kRowGroup>(a)) __builtin_amdgcn_sched_barrier(0);
    static_for<a + 1, N>([&](auto Bi) {
      constexpr int b = RFI_CI(Bi);
      constexpr int k = a * N - a * (a + 1) / 2 + (b - a - 1);   // pair index in row order
      const double Sab = (double)rows.pair(a, b, k, off4);
      const double Nab = fma(cd, Sab, -(double)S[a] * (double)S[b]);
      // no select on b < n: padding has dinv[b] = 0, and + 0 turns its -0
      // into +0, so the load stays unconditional and is issued with its group
      A[Sym<N>::idx(a, b)] = (float)Nab * dinv[a] * dinv[b] + 0.0f;
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
template <int N, class Rows>
__device__ __forceinline__ void jacobi_cell(const EigArgs& g, int64_t cell, const Rows& rows) {
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
  load_corr32<N>(rows, cell, n, cnt, A, degenerate);
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

// Sturm count of the lane's tridiagonal below x (FP32: negative pivots of the
// LDL^T factorisation of T - x I; a zero pivot counts as negative). Only the
// first n entries take part (the padding of a smaller beam count is a
// decoupled identity block).
template <int N>
__device__ __forceinline__ int lane_sturm(const float (&dg)[N], const float (&e2)[N], int n,
                                          float x) {
  float q = 1.0f;
  int c = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float t = fmaf(-e2[i], __builtin_amdgcn_rcpf(q), dg[i] - x);
    if (fabsf(t) < 1e-30f) t = -1e-30f;
    if (i < n) {
      q = t;
      c += t < 0.f;
    }
  }
  return c;
}

// The same count when every index is a beam (n == N): no padding selects.
template <int N>
__device__ __forceinline__ int lane_sturm_full(const float (&dg)[N], const float (&e2)[N],
                                               float x) {
  float q = 1.0f;
  int c = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float t = fmaf(-e2[i], __builtin_amdgcn_rcpf(q), dg[i] - x);
    if (fabsf(t) < 1e-30f) t = -1e-30f;
    q = t;
    c += t < 0.f;
  }
  return c;
}

// Halvings of the Sturm bracket of lambda_1: the FP32 value to working
// precision, or, when the FP64 refinement follows, only far enough to place
// the inverse iteration's shift just above lambda_1 (2^-12 of the bracket;
// the shift adds 2e-5 lambda_1 to its upper end).
constexpr int kPassFull = 26;
constexpr int kPassShift = 12;

template <int N>
__device__ __forceinline__ void bisect_lam1(const float (&dg)[N], const float (&e2)[N], int n,
                                            int it0, int it1, float& lo, float& hi) {
  if (n == N) {
    for (int it = it0; it < it1; ++it) {
      const float mid = 0.5f * (lo + hi);
      if (lane_sturm_full<N>(dg, e2, mid) >= N) hi = mid; else lo = mid;
    }
  } else {
    for (int it = it0; it < it1; ++it) {
      const float mid = 0.5f * (lo + hi);
      if (lane_sturm<N>(dg, e2, n, mid) >= n) hi = mid; else lo = mid;
    }
  }
}

template <int N, class Rows>
__device__ __forceinline__ void ritz_fp64(const EigArgs& g, const Rows& rows, int64_t cell, int n,
                                          int64_t cnt, float lam1, bool have_v, float (&v)[N],
                                          float (&u)[N], uint8_t st);

// Start vectors of the block inverse iteration: components with no exact
// linear relation to any eigenvector that a correlation matrix can have
// (all-ones is orthogonal to (1, -1) for two anticorrelated beams):
// 0.5 + frac(0.5 + i g), g = 0.7548..., and frac(0.5 + i h) - 0.5,
// h = 0.3819... (mixed signs); zero at padding indices.
template <int N>
__device__ __forceinline__ void start_vectors(int n, float (&v)[N], float (&u)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float f = 0.5f + 0.7548776662466927f * (float)i;
    const float h = 0.5f + 0.3819660112501051f * (float)i;
    v[i] = i < n ? 0.5f + (f - floorf(f)) : 0.0f;
    u[i] = i < n ? (h - floorf(h)) - 0.5f : 0.0f;
  }
}

// v unit, u unit and orthogonal to v
template <int N>
__device__ __forceinline__ void orthonormalise(float (&v)[N], float (&u)[N]) {
  float nv = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) nv += v[i] * v[i];
  const float sv = __builtin_amdgcn_rsqf(nv);
  float vu = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    v[i] *= sv;
    vu += v[i] * u[i];
  }
  float nu = 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    u[i] -= vu * v[i];
    nu += u[i] * u[i];
  }
  const float su = nu > 0.f ? __builtin_amdgcn_rsqf(nu) : 0.f;
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] *= su;
}

// Householder + Sturm solver with its own FP64 refinement, one kernel:
// reduction of the FP32 correlation matrix to tridiagonal form T = Q^T C Q in
// the lane's registers (Golub & Van Loan Sec. 8.3: about (4/3) n^3 flops
// instead of 6 n^3 per Jacobi sweep), the FP32 lambda_1 by Sturm bisection on
// T (Sec. 8.4), optional sorted eigenvalues (one bisection each); then the
// two-vector block inverse iteration of the refinement runs on T itself
// (sigma I - T is tridiagonal and positive definite for sigma above lambda_1:
// an O(n) LDL^T factor and O(n) solves), the two vectors go back to C's basis
// through the stored reflectors, Q y = H_0 H_1 ... y, and the FP64 Ritz pass
// over the exact sums gives lambda_1 and the statistic (ritz_fp64).
template <int N, class Rows>
__device__ __forceinline__ void lanetri_cell(const EigArgs& g, int64_t cell, const Rows& rows) {
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int n = g.nbeam;
  const int64_t cnt = g.count[cell / g.nchan];
  if (cnt < 2 || cnt > RFI_MAX_COUNT) {
    g.stat[cell] = 0.0;
    g.status[cell] = RFI_CELL_BAD_COUNT | RFI_CELL_DEGENERATE;
    if (g.eigvals)
      for (int i = 0; i < n; ++i) g.eigvals[i * g.out_stride + cell] = 0.f;
    if (g.v1)
      for (int i = 0; i < n; ++i) g.v1[i * g.out_stride + cell] = 0.f;
    return;
  }
  float A[Sym<N>::NP];
  bool degenerate;
  load_corr32<N>(rows, cell, n, cnt, A, degenerate);

  // The tridiagonal T stays in the matrix's own registers: its diagonal in
  // A(i, i) (final once step i - 1 is done) and its squared couplings in
  // A(i, i - 1) (the reduced column's head, dead after its step). The
  // reflector of step k (v_{k+1} = 1 implied) is kept below it, in
  // A(i, k), i > k + 1, and its beta in tau[k]; off[k] is the signed coupling
  // T(k + 1, k).
  float tau[N], off[N];
  static_for<0, N - 2>([&](auto K) {
    constexpr int k = RFI_CI(K);
    // reflector of (x0, x_{k+2}, ...) onto (mu, 0, ...): v0 = x0 - mu without
    // cancellation, beta = 2 v0^2 / (s2 + v0^2) = -v0 / mu; nothing to do
    // (beta = 0, v = e_{k+1}) when the column is already reduced
    float s2 = 0.f;
    static_for<k + 2, N>([&](auto I) {
      const float x = A[Sym<N>::idx(RFI_CI(I), k)];
      s2 = fmaf(x, x, s2);
    });
    const float x0 = A[Sym<N>::idx(k + 1, k)];
    const float mu2 = fmaf(x0, x0, s2);
    // hardware square root and reciprocals (about 1 ulp): the FP32 reduction
    // only has to span the subspace the FP64 Ritz pass refines
    const float mu = __builtin_amdgcn_sqrtf(mu2);
    const bool refl = s2 > 0.f;
    const float v0 = x0 <= 0.f ? x0 - mu : -s2 * __builtin_amdgcn_rcpf(x0 + mu);
    const float beta = refl ? -v0 * __builtin_amdgcn_rcpf(mu) : 0.f;
    const float iv0 = refl ? __builtin_amdgcn_rcpf(v0) : 0.f;
    float v[N], w[N];
    static_for<k + 1, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      v[i] = i == k + 1 ? 1.0f : A[Sym<N>::idx(i, k)] * iv0;
      if constexpr (i > k + 1) A[Sym<N>::idx(i, k)] = v[i];
    });
    A[Sym<N>::idx(k + 1, k)] = mu2;
    tau[k] = beta;
    off[k] = refl ? mu : x0;
    // p = beta A22 v, K = beta p.v / 2, w = p - K v
    float pv = 0.f;
    static_for<k + 1, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      float acc = 0.f;
      static_for<k + 1, N>([&](auto J) {
        constexpr int j = RFI_CI(J);
        acc = fmaf(A[Sym<N>::idx(i, j)], v[j], acc);
      });
      w[i] = beta * acc;
      pv = fmaf(w[i], v[i], pv);
    });
    const float Kf = 0.5f * beta * pv;
    static_for<k + 1, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      w[i] = fmaf(-Kf, v[i], w[i]);
    });
    // A22 -= v w^T + w v^T (upper triangle)
    static_for<k + 1, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      static_for<i, N>([&](auto J) {
        constexpr int j = RFI_CI(J);
        A[Sym<N>::idx(i, j)] =
            fmaf(-v[i], w[j], fmaf(-w[i], v[j], A[Sym<N>::idx(i, j)]));
      });
    });
  });
  {
    const float x = A[Sym<N>::idx(N - 1, N - 2)];
    off[N - 2] = x;
    A[Sym<N>::idx(N - 1, N - 2)] = x * x;
  }
  float dg[N], e2[N];
  static_for<0, N>([&](auto I) {
    constexpr int i = RFI_CI(I);
    dg[i] = A[Sym<N>::idx(i, i)];
    e2[i] = i > 0 ? A[Sym<N>::idx(i, i > 0 ? i - 1 : 0)] : 0.f;
  });

  // Gershgorin bracket of T; lambda_1 (the largest: a correlation matrix is
  // positive semidefinite) is at least every diagonal entry
  float glo = 3.0e38f, ghi = -3.0e38f, dmax = -3.0e38f;
  static_for<0, N>([&](auto I) {
    constexpr int i = RFI_CI(I);
    if (i < n) {
      const float rad = __builtin_amdgcn_sqrtf(e2[i]) +
                        (i + 1 < N ? __builtin_amdgcn_sqrtf(e2[(i + 1) % N]) : 0.f);
      glo = fminf(glo, dg[i] - rad);
      ghi = fmaxf(ghi, dg[i] + rad);
      dmax = fmaxf(dmax, dg[i]);
    }
  });
  // padding of a smaller beam count is decoupled only below n - 1
  const float span = fmaxf(ghi - glo, 1e-30f);
  glo -= 1e-6f * span;
  ghi += 1e-6f * span;
  float lo = fmaxf(glo, dmax - 1e-6f * span), hi = ghi;
  const int npass = g.refine ? kPassShift : kPassFull;
  bisect_lam1<N>(dg, e2, n, 0, npass, lo, hi);
  float lam1 = 0.5f * (lo + hi);
  uint8_t st = degenerate ? RFI_CELL_DEGENERATE : 0;

  if (g.eigvals) {
    // eigenvalue j (ascending) by bisection, then |lambda| descending
    float ev[N], key[N];
    // (the count without padding selects when the beams fill the instance)
    auto bisect_all = [&](auto full) {
      static_for<0, N>([&](auto J) {
        constexpr int j = RFI_CI(J);
        float a = glo, b = ghi;
        if (j < n) {
          for (int it = 0; it < 28; ++it) {
            const float mid = 0.5f * (a + b);
            const int c = decltype(full)::value ? lane_sturm_full<N>(dg, e2, mid)
                                                : lane_sturm<N>(dg, e2, n, mid);
            if (c > j) b = mid; else a = mid;
          }
        }
        ev[j] = 0.5f * (a + b);
        key[j] = j < n ? fabsf(ev[j]) : -1.0f;
      });
    };
    if (n == N)
      bisect_all(std::integral_constant<bool, true>{});
    else
      bisect_all(std::integral_constant<bool, false>{});
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

  // Two vectors of block inverse iteration on T (the same shift, start vectors
  // and three iterations as the Jacobi path's refinement on C): the subspace
  // converges to that of lambda_1 and lambda_2 at the rate
  // (sigma - lambda_2) / (sigma - lambda_3).
  float v[N], u[N];
  bool have_v = false;
  if (g.refine || g.v1) {
    // hi bounds lambda_1 from above (Sturm count n there)
    const float sigma = hi * (1.0f + 2e-5f) + 1e-6f;
    // B = sigma I - T = L D L^T: pivots d_i (kept as 1 / d_i) and multipliers
    // l_i = B(i, i - 1) / d_{i-1} = -off_{i-1} / d_{i-1}; indices >= n (the
    // decoupled padding) get l = 1 / d = 0, so their components stay zero
    float l[N], id[N];
    bool ok = true;
    static_for<0, N>([&](auto I) {
      constexpr int i = RFI_CI(I);
      float d = sigma - dg[i];
      float li = 0.f;
      if constexpr (i > 0) {
        li = i < n ? -off[i - 1] * id[i - 1] : 0.f;
        d = fmaf(li, off[i - 1], d);
      }
      ok = ok && (i >= n || d > 0.f);
      l[i] = li;
      id[i] = i < n ? __builtin_amdgcn_rcpf(fmaxf(d, 1e-30f)) : 0.f;
    });
    if (!ok && g.refine) {
      // no refinement for this cell: its lambda_1 is the FP32 one, to
      // working precision
      bisect_lam1<N>(dg, e2, n, kPassShift, kPassFull, lo, hi);
      lam1 = 0.5f * (lo + hi);
    }
    start_vectors<N>(n, v, u);
    for (int it = 0; it < 3; ++it) {
      // L y = x (forward), y / d, then L^T z = y (backward), in place
      static_for<1, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        v[i] = fmaf(-l[i], v[i - 1], v[i]);
        u[i] = fmaf(-l[i], u[i - 1], u[i]);
      });
      static_for<0, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        v[i] *= id[i];
        u[i] *= id[i];
      });
      static_for<1, N>([&](auto II) {
        constexpr int i = N - 1 - RFI_CI(II);
        v[i] = fmaf(-l[i + 1], v[i + 1], v[i]);
        u[i] = fmaf(-l[i + 1], u[i + 1], u[i]);
      });
      orthonormalise<N>(v, u);
    }
    // back to C's basis: x <- H_k x for k = N - 3 .. 0,
    // H_k = I - tau_k w w^T, w = (0 .. 0, 1, A(k + 2, k), ...)
    static_for<0, N - 2>([&](auto KK) {
      constexpr int k = N - 3 - RFI_CI(KK);
      float dv = v[k + 1], du = u[k + 1];
      static_for<k + 2, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        dv = fmaf(A[Sym<N>::idx(i, k)], v[i], dv);
        du = fmaf(A[Sym<N>::idx(i, k)], u[i], du);
      });
      dv *= tau[k];
      du *= tau[k];
      v[k + 1] -= dv;
      u[k + 1] -= du;
      static_for<k + 2, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        v[i] = fmaf(-dv, A[Sym<N>::idx(i, k)], v[i]);
        u[i] = fmaf(-du, A[Sym<N>::idx(i, k)], u[i]);
      });
    });
    have_v = ok;
    if (!ok) st |= RFI_CELL_REFINE_FAILED;
  }
  ritz_fp64<N>(g, rows, cell, n, cnt, lam1, have_v, v, u, st);
}

// Kernel 2 of the Jacobi path: block inverse iteration and the FP64 Ritz value
// of lambda_1; writes the statistic lambda_1^2 / ||C||_F^2, v1 and the
// remaining status bits.
template <int N, class Rows>
__device__ __forceinline__ void refine_cell(const EigArgs& g, int64_t cell, const Rows& rows) {
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

  // Two vectors of block inverse iteration (v, u): the subspace converges to
  // that of lambda_1 and lambda_2 at the rate (sigma - lambda_2) /
  // (sigma - lambda_3), so the Ritz value below is exact to FP64 rounding
  // even when lambda_2 is within the shift distance of lambda_1.
  float v[N], u[N];
  bool have_v = false;
  if (g.refine || g.v1) {
    float A[Sym<N>::NP];
    bool dg;
    load_corr32<N>(rows, cell, n, cnt, A, dg);
    const float sigma = lam1 * (1.0f + 2e-5f) + 1e-6f;
    bool ok = true;
    static_for<0, N>([&](auto J) {
      constexpr int j = RFI_CI(J);
      // column j of the factor R (B = R R^T, R lower), B = sigma I - C
      float d = sigma - A[Sym<N>::idx(j, j)];
      static_for<0, j>([&](auto K) {
        constexpr int k = RFI_CI(K);
        d -= A[Sym<N>::idx(j, k)] * A[Sym<N>::idx(j, k)];
      });
      ok = ok && d > 0.f;
      // the diagonal of B is not read again: it keeps 1 / R_jj
      const float rj = __builtin_amdgcn_rsqf(fmaxf(d, 1e-30f));
      A[Sym<N>::idx(j, j)] = rj;
      static_for<j + 1, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        float x = -A[Sym<N>::idx(i, j)];
        static_for<0, j>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(i, k)] * A[Sym<N>::idx(j, k)];
        });
        A[Sym<N>::idx(i, j)] = x * rj;
      });
    });
    start_vectors<N>(n, v, u);
    for (int it = 0; it < 3; ++it) {
      // R y = x (forward), then R^T z = y (backward), in place, for x = v, u
      static_for<0, N>([&](auto I) {
        constexpr int i = RFI_CI(I);
        float x = v[i], y = u[i];
        static_for<0, i>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(i, k)] * v[k];
          y -= A[Sym<N>::idx(i, k)] * u[k];
        });
        v[i] = x * A[Sym<N>::idx(i, i)];
        u[i] = y * A[Sym<N>::idx(i, i)];
      });
      static_for<0, N>([&](auto II) {
        constexpr int i = N - 1 - RFI_CI(II);
        float x = v[i], y = u[i];
        static_for<i + 1, N>([&](auto K) {
          constexpr int k = RFI_CI(K);
          x -= A[Sym<N>::idx(k, i)] * v[k];
          y -= A[Sym<N>::idx(k, i)] * u[k];
        });
        v[i] = x * A[Sym<N>::idx(i, i)];
        u[i] = y * A[Sym<N>::idx(i, i)];
      });
      orthonormalise<N>(v, u);
    }
    have_v = ok;
    if (!ok) st |= RFI_CELL_REFINE_FAILED;
  }
  ritz_fp64<N>(g, rows, cell, n, cnt, lam1, have_v, v, u, st);
}

// The FP64 part of the refinement: ||C||_F^2 from the exact sums and the
// largest Ritz value of the FP64 correlation matrix on span(v, u) (v, u: FP32
// vectors spanning nearly the eigenvectors of lambda_1 and lambda_2; unused
// when !have_v, and then lambda_1 stays the FP32 lam1). Writes stat, status
// and v1 (the Ritz vector).
template <int N, class Rows>
__device__ __forceinline__ void ritz_fp64(const EigArgs& g, const Rows& rows, int64_t cell, int n,
                                          int64_t cnt, float lam1, bool have_v, float (&v)[N],
                                          float (&u)[N], uint8_t st) {
  // FP64 pass over the exact sums: ||C||_F^2 and the projections of C on
  // span(v, u): H = [v u]^T C [v u] and the Gram matrix of (v, u)
  double f2 = 0.0, h11 = 0.0, h12 = 0.0, h22 = 0.0, gvv = 0.0, gvu = 0.0, guu = 0.0;
  {
    // an opaque copy of the lane's offset: the per-lane addresses of this
    // pass are formed anew instead of being kept (spilled) from the first
    // read of the same sums
    uint32_t off4 = (uint32_t)cell * 4u;
    asm volatile("" : "+v"(off4));
    // Branch-free, and the loads of each group are issued together before
    // any is used: padding indices (>= n) read a clamped valid address and
    // get d = 0 (v = u = 0 there too), which zeroes their terms. N_ab =
    // cnt S_ab - S_a S_b is exact in FP64 (as in load_corr32).
    const double cd = (double)cnt;
    int32_t S[N], Sdg[N];
    // v and u are widened to FP64 where they are used (exact conversions):
    // FP64 copies of both would hold 4 N more registers through the pass
    double d[N];
    if (!have_v) {
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = u[i] = 0.f;
    }
    static_for<0, N>([&](auto Ai) {
      constexpr int a = RFI_CI(Ai);
      S[a] = rows.S(a, off4);
      Sdg[a] = rows.Sdg(a, off4);
    });
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, N>([&](auto Ai) {
      constexpr int a = RFI_CI(Ai);
      const double Sa = (double)S[a];
      const double Naa = fma(cd, (double)Sdg[a], -Sa * Sa);
      d[a] = (a < n && Naa > 0.0) ? rsqrt64(Naa) : 0.0;
      const double va = (double)v[a], ua = (double)u[a];
      h11 += va * va;
      h12 += va * ua;
      h22 += ua * ua;
      f2 += a < n ? 1.0 : 0.0;
    });
    gvv = h11;
    gvu = h12;
    guu = h22;
    double off = 0.0, o11 = 0.0, o12 = 0.0, o22 = 0.0;
    // strict upper triangle in row order, in groups of kGroup entries
    constexpr int kPairs = N * (N - 1) / 2;
    constexpr int kGroup = kRowGroup;
    static_for<0, (kPairs + kGroup - 1) / kGroup>([&](auto Ci) {
      constexpr int k0 = RFI_CI(Ci) * kGroup;
      constexpr int k1 = k0 + kGroup < kPairs ? k0 + kGroup : kPairs;
      int32_t R[kGroup];
      static_for<k0, k1>([&](auto Ki) {
        constexpr int k = RFI_CI(Ki);
        constexpr int a = UpperPair<N>::row(k), b = UpperPair<N>::col(k);
        R[k - k0] = rows.pair(a, b, k, off4);
      });
      __builtin_amdgcn_sched_barrier(0);
      static_for<k0, k1>([&](auto Ki) {
        constexpr int k = RFI_CI(Ki);
        constexpr int a = UpperPair<N>::row(k), b = UpperPair<N>::col(k);
        const double Nab = fma(cd, (double)R[k - k0], -(double)S[a] * (double)S[b]);
        const double r = Nab * d[a] * d[b];
        off += r * r;
        const double va = (double)v[a], vb = (double)v[b];
        const double ua = (double)u[a], ub = (double)u[b];
        o11 += r * (va * vb);
        o12 += r * (va * ub + ua * vb);
        o22 += r * (ua * ub);
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    f2 += 2.0 * off;
    h11 += 2.0 * o11;
    h12 += o12;
    h22 += 2.0 * o22;
  }
  // Ritz values of C on span(v, u) in FP64: with v' = v / |v| and
  // u' = (u - al v) / |u - al v|, al = (v.u) / (v.v), the projected matrix is
  // [[p, q], [q, r]]; lambda_1 = (p + r) / 2 + sqrt(((p - r) / 2)^2 + q^2)
  double lam = (double)lam1;
  double cv = 1.0, cu = 0.0;   // Ritz vector = cv v' + cu u'
  double sv = 1.0, su = 0.0, al = 0.0;
  if (have_v && gvv > 0.0) {
    al = gvu / gvv;
    const double nu2 = guu - al * gvu;
    const double pp = h11 / gvv;
    lam = pp;
    sv = 1.0 / sqrt(gvv);
    if (nu2 > 1e-12 * guu) {
      su = 1.0 / sqrt(nu2);
      const double qq = (h12 - al * h11) * sv * su;
      const double rr = (h22 - 2.0 * al * h12 + al * al * h11) * su * su;
      const double hd = 0.5 * (pp - rr);
      const double rt = sqrt(hd * hd + qq * qq);
      lam = 0.5 * (pp + rr) + rt;
      // eigenvector of the 2 x 2 matrix for lam, from the better conditioned
      // of its two expressions
      if (hd >= 0.0) {
        cv = hd + rt;
        cu = qq;
      } else {
        cv = qq;
        cu = rt - hd;
      }
      const double nc = sqrt(cv * cv + cu * cu);
      if (nc > 0.0) {
        cv /= nc;
        cu /= nc;
      } else {
        cv = 1.0;
        cu = 0.0;
      }
    }
  }
  if (!g.refine || !have_v) lam = (double)lam1;
  if (have_v) {
    // v1 = cv v' + cu u' in the original basis
#pragma unroll
    for (int i = 0; i < N; ++i)
      v[i] = (float)(cv * sv * v[i] + cu * su * ((double)u[i] - al * (double)v[i]));
  }
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

// The single-block kernels read their sums through the workgroup's table of
// row addresses (RowsTable); the batched ones, whose workgroups can hold cells
// of several blocks, form the addresses per lane (RowsDirect).
template <int N>
__global__ __launch_bounds__(256, 2) void eig_lane_jacobi(EigArgs g) {
  __shared__ uint64_t tab[RowTab<N>::K];
  fill_rows<N>(g, tab);
  __syncthreads();
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < (int64_t)g.nsub * g.nchan) jacobi_cell<N>(g, cell, RowsTable<N>{tab});
}

template <int N>
__global__ __launch_bounds__(256, 1) void eig_lane_tri(EigArgs g) {
  __shared__ uint64_t tab[RowTab<N>::K];
  fill_rows<N>(g, tab);
  __syncthreads();
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < (int64_t)g.nsub * g.nchan) lanetri_cell<N>(g, cell, RowsTable<N>{tab});
}

template <int N>
__global__ __launch_bounds__(256, 1) void eig_lane_refine(EigArgs g) {
  __shared__ uint64_t tab[RowTab<N>::K];
  fill_rows<N>(g, tab);
  __syncthreads();
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell < (int64_t)g.nsub * g.nchan) refine_cell<N>(g, cell, RowsTable<N>{tab});
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
__global__ __launch_bounds__(256, 2) void eig_lane_jacobi_batch(const EigArgs* items,
                                                             const int64_t* cell0, int nitem,
                                                             int64_t total) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  const int i = find_item(cell0, nitem, c);
  const EigArgs g = items[i];
  jacobi_cell<N>(g, c - cell0[i],
                 RowsDirect<N>{g.sum_x, g.sum_xy, (int64_t)g.nsub * g.nchan, g.nbeam});
}

template <int N>
__global__ __launch_bounds__(256, 1) void eig_lane_tri_batch(const EigArgs* items,
                                                          const int64_t* cell0, int nitem,
                                                          int64_t total) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  const int i = find_item(cell0, nitem, c);
  const EigArgs g = items[i];
  lanetri_cell<N>(g, c - cell0[i],
                  RowsDirect<N>{g.sum_x, g.sum_xy, (int64_t)g.nsub * g.nchan, g.nbeam});
}

template <int N>
__global__ __launch_bounds__(256, 1) void eig_lane_refine_batch(const EigArgs* items,
                                                             const int64_t* cell0, int nitem,
                                                             int64_t total) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= total) return;
  const int i = find_item(cell0, nitem, c);
  const EigArgs g = items[i];
  refine_cell<N>(g, c - cell0[i],
                 RowsDirect<N>{g.sum_x, g.sum_xy, (int64_t)g.nsub * g.nchan, g.nbeam});
}

template <int N>
hipError_t launch_batch_n(const EigArgs* items, const int64_t* cell0, int nitem, int64_t total,
                          int wg, bool tri, hipStream_t s) {
  const dim3 grid((unsigned)((total + wg - 1) / wg));
  if (tri) {   // Householder, Sturm and the FP64 refinement in one kernel
    hipLaunchKernelGGL(eig_lane_tri_batch<N>, grid, dim3(wg), 0, s, items, cell0, nitem, total);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(eig_lane_jacobi_batch<N>, grid, dim3(wg), 0, s, items, cell0, nitem, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_lane_refine_batch<N>, grid, dim3(wg), 0, s, items, cell0, nitem, total);
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const EigArgs& a, int wg, bool tri, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  const dim3 grid((unsigned)((ncell + wg - 1) / wg));
  if (tri) {   // Householder, Sturm and the FP64 refinement in one kernel
    hipLaunchKernelGGL(eig_lane_tri<N>, grid, dim3(wg), 0, s, a);
    return hipGetLastError();
  }
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
                                 int64_t total, hipStream_t s, int wg, bool tri) {
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  switch (cls) {
    case 4: return launch_batch_n<4>(items, cell0, nitem, total, wg, tri, s);
    case 8: return launch_batch_n<8>(items, cell0, nitem, total, wg, tri, s);
    case 12: return launch_batch_n<12>(items, cell0, nitem, total, wg, tri, s);
    case 16: return launch_batch_n<16>(items, cell0, nitem, total, wg, tri, s);
    case 19: return launch_batch_n<19>(items, cell0, nitem, total, wg, tri, s);
    case 20: return launch_batch_n<20>(items, cell0, nitem, total, wg, tri, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eig_lane(const EigArgs& a, hipStream_t s, int wg, bool tri) {
  const int n = a.nbeam;
  if (wg != 64 && wg != 128 && wg != 256) return hipErrorInvalidValue;
  if (n <= 4) return launch_n<4>(a, wg, tri, s);
  if (n <= 8) return launch_n<8>(a, wg, tri, s);
  if (n <= 12) return launch_n<12>(a, wg, tri, s);
  if (n <= 16) return launch_n<16>(a, wg, tri, s);
  if (n == 19) return launch_n<19>(a, wg, tri, s);
  if (n <= 20) return launch_n<20>(a, wg, tri, s);
  return hipErrorInvalidValue;
}

}  // namespace rfi
