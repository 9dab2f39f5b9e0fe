// Per-cell eigen stage for larger beam counts, one cell per WAVEFRONT, in
// FP64 (Sec. 3.2-3.3, Eq. 1-2): Householder reduction of the correlation
// matrix to tridiagonal form, then Sturm-sequence bisection on the tridiagonal
// (Golub & Van Loan, Matrix Computations, Sec. 8.3 and 8.4).
//
// Work per cell is about (4/3) n^3 flops for the reduction instead of the
// 6 n^3 per sweep of cyclic Jacobi, and it runs in FP64 at the full vector
// rate of the chip, so lambda_1 needs no separate refinement.
//
// Register-resident layout: the cell's matrix (padded to 8 NL x 8 NL with
// zeros) lives in the registers of one wave as an 8 x 8 grid of lanes, lane
// 8 r + c holding the entries (r + 8 ii, c + 8 jj), ii, jj < NL (a cyclic 2-D
// distribution, so the shrinking active block stays spread over all lanes).
// Step k of the reduction:
//  - row k (= column k) is broadcast through LDS by the 8 lanes that hold it;
//  - the reflector v (v_{k+1} = 1, zero at indices <= k) and beta;
//  - p = A v: each lane sums its partial rows; the 8 partials of each row go
//    through LDS and one lane per row adds them, so beta p is in LDS for the
//    lanes that hold its entries as rows and as columns;
//  - w = beta p - (beta^2 p.v / 2) v and A -= v w^T + w v^T.
// The update is the full two-sided product H A H on the whole padded matrix:
// rows and columns already reduced are only multiplied by the orthogonal H
// (v vanishes there), so their leftover entries stay bounded and never reach
// the active block; local rows / columns whose every index is reduced are
// skipped at compile time (the loop over blocks of 8 steps is unrolled). The
// diagonal is read back at the end of each block of 8 steps; the
// sub-diagonal is the reflected column norm of each step (the last step, a
// single entry, needs no reflection).
//
// Then:
//  - lambda_1 = largest eigenvalue (a correlation matrix is positive
//    semidefinite, so it is also the largest in magnitude): multisection, the
//    64 lanes each evaluating the Sturm count at one point of the bracket;
//  - all eigenvalues (optional): bisection, one eigenvalue index per lane;
//  - v1 (optional): inverse iteration on the tridiagonal with the shift
//    lambda_1, then the reflectors (kept in LDS) applied in reverse order.
#include <math.h>

#include <type_traits>

#include "internal.h"

namespace rfi {
namespace {

// Compile-time loop: every index into the register-resident matrix must be a
// constant.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
#define RFI_CI(v) decltype(v)::value

__device__ __forceinline__ int64_t pidx(int a, int b, int n) {
  return (int64_t)a * n - (int64_t)a * (a - 1) / 2 + (b - a);
}


// DPP move of a double (two 32-bit halves); every source lane is valid for
// the patterns used here, so no old value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 8 consecutive lanes of a lane row (lanes 8 r .. 8 r + 7):
// lane ^ 1, lane ^ 2 (quad permutations), then the mirror within the 8
// lanes, which pairs each lane with one of the other quad. Every lane of the
// row ends with the same bits (each stage adds the same two operands).
__device__ __forceinline__ double sum8(double x) {
  x += dpp_mov<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_mov<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_mov<0x141>(x);  // row_half_mirror
  return x;
}

__device__ __forceinline__ double lane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wavefront reductions without LDS-routed lane permutes: the 8-lane stages
// above, then the mirror within each 16-lane row, then the four row results
// read as scalars and combined in a fixed order (every lane gets the same
// bits). A permute address held across the long reduction would cost
// registers the kernel does not have.
__device__ __forceinline__ double wave_sum(double x) {
  x = sum8(x);
  x += dpp_mov<0x140>(x);  // row_mirror
  return (lane_f64(x, 0) + lane_f64(x, 16)) + (lane_f64(x, 32) + lane_f64(x, 48));
}
__device__ __forceinline__ double wave_min(double x) {
  x = fmin(x, dpp_mov<0xB1>(x));
  x = fmin(x, dpp_mov<0x4E>(x));
  x = fmin(x, dpp_mov<0x141>(x));
  x = fmin(x, dpp_mov<0x140>(x));
  return fmin(fmin(lane_f64(x, 0), lane_f64(x, 16)), fmin(lane_f64(x, 32), lane_f64(x, 48)));
}
__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_mov<0xB1>(x));
  x = fmax(x, dpp_mov<0x4E>(x));
  x = fmax(x, dpp_mov<0x141>(x));
  x = fmax(x, dpp_mov<0x140>(x));
  return fmax(fmax(lane_f64(x, 0), lane_f64(x, 16)), fmax(lane_f64(x, 32), lane_f64(x, 48)));
}

// Reciprocal of q to about full FP64 precision: the hardware estimate and one
// Newton step (a Sturm count needs each pivot to a few ulps only: the count
// is then exact for a tridiagonal within a few ulps of this one).
__device__ __forceinline__ double rcp1(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

// Number of eigenvalues of the tridiagonal below x (Sturm count: negative
// pivots of the LDL^T factorisation of T - x I), for P points at once (P
// independent recurrences per lane). ae[i] = (alpha_i, off_{i-1}^2),
// off_{-1} = 0. A pivot that is zero (or nearly) is replaced by a tiny
// negative one, which keeps the count exact for x on an eigenvalue of a
// leading block.
template <int P>
__device__ __forceinline__ void sturm_below_p(const double2* ae, int n, const double (&x)[P],
                                              int (&cnt)[P]) {
  constexpr double PIV = 1e-290;
  double q[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    q[j] = 1.0;   // with off_{-1}^2 = 0 the first step is alpha_0 - x
    cnt[j] = 0;
  }
  for (int i = 0; i < n; ++i) {
    const double2 v = ae[i];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      q[j] = fma(-v.y, rcp1(q[j]), v.x - x[j]);
      if (fabs(q[j]) < PIV) q[j] = -PIV;
      cnt[j] += q[j] < 0.0;
    }
  }
}

__device__ __forceinline__ int sturm_below(const double2* ae, int n, double x) {
  const double xs[1] = {x};
  int c[1];
  sturm_below_p<1>(ae, n, xs, c);
  return c[0];
}

// Inverse iteration for the eigenvector of the tridiagonal (alpha, off)
// nearest sigma; ud, ue, uf: scratch [n]; x: result [n], unit norm.
__device__ void tri_inverse_iteration(const double* alpha, const double* off, int n, double sigma,
                                      double* ud, double* ue, double* uf, double* x) {
  for (int i = 0; i < n; ++i) x[i] = 1.0;
  for (int iter = 0; iter < 3; ++iter) {
    double d = alpha[0] - sigma, e = n > 1 ? off[0] : 0.0, r = x[0];
    for (int i = 0; i + 1 < n; ++i) {
      const double s = off[i];
      const double dn = alpha[i + 1] - sigma;
      const double en = i + 2 < n ? off[i + 1] : 0.0;
      const double rn = x[i + 1];
      if (fabs(s) > fabs(d)) {
        // pivot on row i + 1: U row i = (s, dn, en); the old row is eliminated
        const double m = d / s;
        ud[i] = s;
        ue[i] = dn;
        uf[i] = en;
        x[i] = rn;
        d = e - m * dn;
        e = -m * en;
        r = r - m * rn;
      } else {
        const double m = s / (d != 0.0 ? d : 1e-300);
        ud[i] = d;
        ue[i] = e;
        uf[i] = 0.0;
        x[i] = r;
        d = dn - m * e;
        e = en;
        r = rn - m * r;
      }
    }
    ud[n - 1] = d;
    x[n - 1] = r;
    double nrm = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      double t = x[i];
      if (i + 1 < n) t -= ue[i] * x[i + 1];
      if (i + 2 < n) t -= uf[i] * x[i + 2];
      x[i] = t / (ud[i] != 0.0 ? ud[i] : 1e-300);
      nrm += x[i] * x[i];
    }
    const double sc = 1.0 / sqrt(nrm);
    for (int i = 0; i < n; ++i) x[i] *= sc;
  }
}

// Workgroup b runs on XCD b mod 8; give each XCD a contiguous run of cells
// (a bijection of [0, total)), so the cells that share the cache lines of the
// structure-of-arrays sums are read through one L2 at about the same time.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t total) {
  const int64_t q = total >> 3, rem = total & 7, x = b & 7;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

__device__ __forceinline__ int find_item_t(const int64_t* cell0, int nitem, int64_t c) {
  int lo = 0, hi = nitem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell0[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// vcap: doubles of dynamic LDS for the reflectors ((n - 1) 8 NL are needed
// when v1 is requested; 0 in launches that never ask for v1).
// Two waves per SIMD up to NL = 9 (72 beams: a few spilled registers cost less
// than the latency one wave per SIMD leaves exposed); one beyond.
// W: the sums are int64 cell records (sub-intervals longer than the int32
// bound, summed in time chunks and widened); such cells read n L >= 66,050
// bytes each, so their eigen stage is never the bound and one wave per SIMD
// (room for the wider LDS copy of the sums) costs nothing.
// NC: the non-centred matrix of the bandpass-subtracted power instead of the
// correlation matrix: M_ab = (S_ab - z_b S_a - z_a S_b + L z_a z_b) / L from
// the exact sums and the baseline zb [nbeam][ncell] (NULL: 0), every entry
// formed in that operation order (no fused multiply-add), ||M||_F^2 over all
// entries.
template <int NL, bool W = false, bool NC = false>
__global__ __launch_bounds__(64, (NL <= 9 && !W && !NC) ? 2 : 1) void eig_tri_kernel(
    EigArgs g, const EigArgs* items, const int64_t* cell0, int nitem, int vcap,
    const double* zb) {
  constexpr int NN = 8 * NL;
  using ST = std::conditional_t<W, int64_t, int32_t>;
  // the sums are global memory (batched launches read their pointers from the
  // item table, where the compiler cannot tell the address space)
  typedef const __attribute__((address_space(1))) int32_t gint32;
  typedef const __attribute__((address_space(1))) int64_t gint64;
  __shared__ double X[NN], P[NN], alpha[NN], offd[NN], tau[NN], dinv[NN], z[NN];
  __shared__ double2 ae[NN];
  // values needed only at the end, kept in LDS instead of registers through
  // the reduction (registers are what bounds this kernel's occupancy)
  __shared__ double s_frob2;
  __shared__ int s_degen;
  __shared__ ST S[NN];
  __shared__ __attribute__((aligned(16))) ST SP[NN * (NN + 1) / 2];
  // partial row sums of p = A v, [lane column][row] with an odd row stride;
  // they live in the staged sums' space (dead once the matrix is formed)
  // where it is large enough
  constexpr int kPPS = NN + 1;
  constexpr bool kPPAlias = sizeof(ST) * (NN * (NN + 1) / 2) >= sizeof(double) * 8 * kPPS;
  __shared__ double PPown[kPPAlias ? 1 : 8 * kPPS];
  double* const PP = kPPAlias ? reinterpret_cast<double*>(SP) : PPown;
  extern __shared__ __attribute__((aligned(16))) double vst[];
  int64_t cell = xcd_order(blockIdx.x, gridDim.x);
  if (items) {
    const int i = find_item_t(cell0, nitem, cell);
    g = items[i];
    cell -= cell0[i];
  }
  const int n = g.nbeam;
  const int lane = threadIdx.x, r = lane >> 3, c = lane & 7;
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int64_t cnt = g.count[cell / g.nchan];
  if (cnt < 2 || cnt > (W ? RFI_MAX_COUNT_LONG : RFI_MAX_COUNT)) {
    for (int i = lane; i < n; i += 64) {
      if (g.eigvals) g.eigvals[i * g.out_stride + cell] = 0.f;
      if (g.v1) g.v1[i * g.out_stride + cell] = 0.f;
    }
    if (lane == 0) {
      g.stat[cell] = 0.0;
      g.status[cell] = RFI_CELL_BAD_COUNT | RFI_CELL_DEGENERATE;
    }
    return;
  }
  const bool want_v1 = g.v1 && (int64_t)(n - 1) * NN <= vcap;

  // correlation matrix in FP64 and ||C||_F^2 (the cell's sums first go to
  // LDS, one pair per lane)
  // The loads of kLd rows per lane are issued before any is stored (indices
  // clamped into the record, so every load is unconditional): one memory
  // round trip per kLd x 64 sums instead of one per 64.
  const int np = n * (n + 1) / 2;
  constexpr int kLd = 16;
  auto stage = [&](auto load) {
    for (int q0 = lane; q0 < n + np; q0 += 64 * kLd) {
      decltype(load(0)) v[kLd];
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int q = q0 + 64 * u;
        v[u] = load(q < n + np ? q : n + np - 1);
      }
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int q = q0 + 64 * u;
        if (q < n) S[q] = v[u];
        else if (q < n + np) SP[q - n] = v[u];
      }
    }
  };
  if constexpr (W) {
    // one contiguous int64 record per cell
    const gint64* rec = (const gint64*)g.sum_x + cell * (int64_t)(n + np);
    stage([&](int q) { return rec[q]; });
  } else if (g.layout) {
    // one contiguous record per cell: coalesced
    const gint32* rec = (const gint32*)g.sum_x + cell * (int64_t)(n + np);
    stage([&](int q) { return rec[q]; });
  } else {
    // rows layout: row q of the record is sum_x[q] (q < n) or sum_xy[q - n]
    stage([&](int q) {
      const gint32* row = (const gint32*)(q < n ? g.sum_x + (int64_t)q * ncell
                                                : g.sum_xy + (int64_t)(q - n) * ncell);
      return row[cell];
    });
  }
  __syncthreads();
  int dead = 0;
  for (int a = lane; a < n; a += 64) {
    if constexpr (NC) {
      dinv[a] = zb ? zb[(int64_t)a * ncell + cell] : 0.0;     // the baseline z_a
    } else {
      const int64_t Naa = cnt * (int64_t)SP[pidx(a, a, n)] - (int64_t)S[a] * S[a];
      dinv[a] = Naa > 0 ? 1.0 / sqrt((double)Naa) : 0.0;
      dead |= Naa <= 0;
    }
  }
  int degenerate = __syncthreads_or(dead);
  double A[NL][NL];
  double offsq = 0.0;
  // this lane's row and column values of S and 1 / sqrt(N_aa) (0 at padding
  // indices), read once
  [[maybe_unused]] double Srow[NL], Scol[NL], drow[NL], dcol[NL];
  if constexpr (!NC) {
    static_for<0, NL>([&](auto II) {
      constexpr int ii = RFI_CI(II);
      const int gi = r + 8 * ii, gj = c + 8 * ii;
      Srow[ii] = (double)S[gi < n ? gi : 0];
      Scol[ii] = (double)S[gj < n ? gj : 0];
      drow[ii] = gi < n ? dinv[gi] : 0.0;
      dcol[ii] = gj < n ? dinv[gj] : 0.0;
    });
  }
  const double cd = (double)cnt;
  static_for<0, NL>([&](auto II) {
    constexpr int ii = RFI_CI(II);
    static_for<0, NL>([&](auto JJ) {
      constexpr int jj = RFI_CI(JJ);
      const int gi = r + 8 * ii, gj = c + 8 * jj;
      double val = 0.0;
      if constexpr (NC) {
        if (gi < n && gj < n) {
#pragma clang fp contract(off)
          const int a = gi < gj ? gi : gj, b = gi < gj ? gj : gi;
          const double Lc = (double)cnt, za = dinv[a], zbv = dinv[b];
          const double Sa = (double)S[a], Sb = (double)S[b];
          val = ((((double)SP[pidx(a, b, n)] - zbv * Sa) - za * Sb) + (Lc * za) * zbv) / Lc;
          offsq += gi == gj ? val * val : (gi < gj ? 2.0 * val * val : 0.0);
        }
      } else {
        // N_ab = cnt S_ab - S_a S_b is exact in FP64: both products and the
        // difference are integers below 2^53 (S_ab <= 255^2 L, L <= 262,143);
        // branch-free, padding indices read a valid entry and get d = 0. The
        // product d_a d_b keeps both triangles bit-identical.
        const int ga = gi < n ? gi : 0, gb = gj < n ? gj : 0;
        const int a = ga < gb ? ga : gb, b = ga < gb ? gb : ga;
        const double Nab = fma(cd, (double)SP[pidx(a, b, n)], -Srow[ii] * Scol[jj]);
        val = gi == gj ? (gi < n ? 1.0 : 0.0) : Nab * (drow[ii] * dcol[jj]);
        offsq += gi < gj ? val * val : 0.0;
      }
      A[ii][jj] = val;
    });
  });
  {
    const double frob2 = NC ? wave_sum(offsq) : (double)n + 2.0 * wave_sum(offsq);
    if constexpr (NC) degenerate = !(frob2 > 0.0);
    if (lane == 0) {
      s_frob2 = frob2;
      s_degen = degenerate;
    }
  }

  // Householder reduction: steps k = 0 .. n - 2 (the last one only records
  // the final sub-diagonal entry)
  static_for<0, NL>([&](auto IKc) {
    constexpr int IK = RFI_CI(IKc);
    const int nk = min(8, n - 1 - 8 * IK);   // steps of this block (may be <= 0)
#pragma unroll 1
    for (int rk = 0; rk < nk; ++rk) {
      const int k = 8 * IK + rk;
      __syncthreads();
      if (r == rk) {
        // this lane row holds row k (= column k) of A, at local row IK: it
        // forms the reflector of (x0, x_{k+2}, ...) onto (mu, 0, ...) with
        // v0 = x0 - mu (without cancellation), beta = 2 v0^2 / (s2 + v0^2)
        // = -v0 / mu, and publishes v (v_{k+1} = 1) and beta
        double s2 = 0.0, x0 = 0.0;
        static_for<IK, NL>([&](auto JJ) {
          constexpr int jj = RFI_CI(JJ);
          const int gj = c + 8 * jj;
          const double x = A[IK][jj];
          s2 += gj > k + 1 ? x * x : 0.0;
          x0 += gj == k + 1 ? x : 0.0;
        });
        s2 = sum8(s2);
        // one non-zero term, on the lane that holds column k + 1 of row k
        x0 = lane_f64(x0, 8 * rk + ((k + 1) & 7));
        double beta = 0.0, sub = x0, iv0 = 0.0;
        if (s2 > 0.0) {
          const double mu = sqrt(fma(x0, x0, s2));
          const double v0 = x0 <= 0.0 ? x0 - mu : -s2 * rcp1(x0 + mu);
          beta = -v0 * rcp1(mu);
          iv0 = rcp1(v0);
          sub = mu;
        }
        static_for<IK, NL>([&](auto JJ) {
          constexpr int jj = RFI_CI(JJ);
          const int gj = c + 8 * jj;
          const double v = gj > k + 1 ? A[IK][jj] * iv0 : (gj == k + 1 ? 1.0 : 0.0);
          X[gj] = v;
          if (want_v1 && gj < n) vst[k * NN + gj] = v;
        });
        if (c == 0) {
          offd[k] = sub;
          tau[k] = beta;
        }
      }
      __syncthreads();
      // with beta = 0 (nothing below the sub-diagonal) v = e_{k+1} and w = 0:
      // the update below leaves A unchanged, so it runs without a branch
      const double beta = tau[k];
      // p = A v (unscaled) for this lane's rows; v is read from LDS per column
      double pr[NL];
      static_for<IK, NL>([&](auto II) { pr[RFI_CI(II)] = 0.0; });
      static_for<IK, NL>([&](auto JJ) {
        constexpr int jj = RFI_CI(JJ);
        const double vcj = X[c + 8 * jj];
        static_for<IK, NL>([&](auto II) {
          constexpr int ii = RFI_CI(II);
          pr[ii] = fma(A[ii][jj], vcj, pr[ii]);
        });
      });
      // the row sums over the 8 lanes of a lane row go through LDS: every
      // lane stores its partials, then lane (r, c) adds the eight partials of
      // local row IK + c (and IK + c + 8) in a fixed order and stores beta
      // times the sum in P (fewer instructions than an 8-lane DPP sum per row)
      static_for<IK, NL>([&](auto II) {
        constexpr int ii = RFI_CI(II);
        PP[c * kPPS + r + 8 * ii] = pr[ii];
      });
      __syncthreads();
      for (int jj = IK + c; jj < NL; jj += 8) {
        const int i = r + 8 * jj;
        const double s01 = PP[i] + PP[kPPS + i], s23 = PP[2 * kPPS + i] + PP[3 * kPPS + i];
        const double s45 = PP[4 * kPPS + i] + PP[5 * kPPS + i];
        const double s67 = PP[6 * kPPS + i] + PP[7 * kPPS + i];
        P[i] = beta * ((s01 + s23) + (s45 + s67));
      }
      __syncthreads();
      // with P = beta p: K = beta^2 (p.v) / 2 = beta (P.v) / 2
      double pv = 0.0;
      static_for<IK, NL>([&](auto JJ) {
        pv = fma(P[c + 8 * RFI_CI(JJ)], X[c + 8 * RFI_CI(JJ)], pv);
      });
      pv = sum8(pv);
      const double K = 0.5 * beta * pv;
      // w = beta p - K v; A -= v w^T + w v^T
      double vr[NL];
      static_for<IK, NL>([&](auto II) {
        constexpr int ii = RFI_CI(II);
        vr[ii] = X[r + 8 * ii];
        pr[ii] = fma(-K, vr[ii], P[r + 8 * ii]);
      });
      static_for<IK, NL>([&](auto JJ) {
        constexpr int jj = RFI_CI(JJ);
        const double vcj = X[c + 8 * jj];
        const double wcj = fma(-K, vcj, P[c + 8 * jj]);
        static_for<IK, NL>([&](auto II) {
          constexpr int ii = RFI_CI(II);
          A[ii][jj] = fma(-vr[ii], wcj, fma(-pr[ii], vcj, A[ii][jj]));
        });
      });
    }
    // diagonal entries of block IK are final
    if (r == c && r + 8 * IK < n) alpha[r + 8 * IK] = A[IK][IK];
  });
  __syncthreads();

  for (int i = lane; i < n; i += 64) ae[i] = make_double2(alpha[i], i ? offd[i - 1] * offd[i - 1] : 0.0);
  // Gershgorin bracket of the spectrum; lambda_1 is at least the largest
  // eigenvalue of every 2 x 2 principal block (Cauchy interlacing)
  double glo = 1e300, ghi = -1e300, lb = -1e300;
  for (int i = lane; i < n; i += 64) {
    const double rad = (i > 0 ? fabs(offd[i - 1]) : 0.0) + (i + 1 < n ? fabs(offd[i]) : 0.0);
    glo = fmin(glo, alpha[i] - rad);
    ghi = fmax(ghi, alpha[i] + rad);
    double m = alpha[i];
    if (i + 1 < n) {
      const double h = 0.5 * (alpha[i] - alpha[i + 1]);
      m = 0.5 * (alpha[i] + alpha[i + 1]) + sqrt(h * h + offd[i] * offd[i]);
    }
    lb = fmax(lb, m);
  }
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  lb = wave_max(lb);
  const double span = fmax(ghi - glo, 1e-300);
  glo -= 1e-12 * span;
  ghi += 1e-12 * span;
  __syncthreads();

  // lambda_1 = the largest eigenvalue: multisection. The bracket [lo, hi]
  // always holds exactly one crossing of count n-1 -> n (count(lo) <= n-1,
  // count(hi) = n); lane l tests the points l + 1 + 64 j (j < NP) of the
  // 64 NP + 1 equal parts of the bracket. One point per lane: the counts are
  // issue-bound, so more points per pass cost more than the passes they save.
  // The bracket stops at 2e-14 relative width, the order of the backward
  // error of the FP64 reduction itself.
  constexpr int NP = 1;
  // a correlation matrix has lambda_1 >= 1; the non-centred matrix has the
  // scale of the data, so its stop is relative only
  constexpr double kFloor = NC ? 1e-300 : 1.0;
  double lo = fmax(glo, lb - 1e-12 * span), hi = ghi;
  for (int it = 0; it < 16 && hi - lo > 2e-14 * fmax(fabs(hi), kFloor); ++it) {
    const double h = (hi - lo) * (1.0 / (64 * NP + 1));
    double xs[NP];
    int cn[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) xs[j] = lo + (lane + 1 + 64 * j) * h;
    sturm_below_p<NP>(ae, n, xs, cn);
    // the first point with all n eigenvalues below it
    int first = 64 * NP + 1;
#pragma unroll
    for (int j = NP - 1; j >= 0; --j) {
      const unsigned long long bj = __ballot(cn[j] >= n);
      if (bj) first = __builtin_ctzll(bj) + 1 + 64 * j;
    }
    const double nlo = lo + (first - 1) * h;
    const double nhi = first == 64 * NP + 1 ? hi : lo + first * h;
    lo = nlo;
    hi = nhi;
  }
  const double lam1 = 0.5 * (lo + hi);

  if (lane == 0) {
    const double frob2 = s_frob2;
    const int degenerate = s_degen;
    g.stat[cell] = (NC && degenerate) ? 0.0 : lam1 * lam1 / frob2;
    g.status[cell] = degenerate ? RFI_CELL_DEGENERATE : 0;
  }

  if (g.eigvals) {
    // eigenvalue index i (ascending) by bisection on lane i mod 64; the
    // matrix is positive semidefinite up to rounding, so |lambda| descending
    // is index n - 1 - i
    for (int i = lane; i < n; i += 64) {
      double a = glo, b = ghi;
      for (int it = 0; it < 64 && b - a > 2e-16 * fmax(fabs(b), kFloor); ++it) {
        const double mid = 0.5 * (a + b);
        if (sturm_below(ae, n, mid) > i) b = mid; else a = mid;
      }
      z[i] = 0.5 * (a + b);
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
      const double li = fabs(z[i]);
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const double lj = fabs(z[j]);
        rank += (lj > li) || (lj == li && j > i);
      }
      g.eigvals[rank * g.out_stride + cell] = (float)z[i];
    }
    __syncthreads();
  }

  if (g.v1) {
    if (!want_v1) {
      // no room for the reflectors in this launch (the launchers below always
      // give it when v1 is asked for): NaN rather than a wrong vector
      for (int i = lane; i < n; i += 64) g.v1[i * g.out_stride + cell] = __builtin_nanf("");
      return;
    }
    // inverse iteration on T - sigma I, sigma just above lambda_1 (lane 0):
    // Gaussian elimination with partial pivoting of the tridiagonal into
    // U = (ud, ue, uf) (diagonal and two upper diagonals), then back
    // substitution; three iterations from the all-ones vector
    if (lane == 0) tri_inverse_iteration(alpha, offd, n, lam1 + 1e-13 * fmax(fabs(lam1), kFloor),
                                         X, P, dinv, z);
    __syncthreads();
    // back-transform: v1 = H_0 H_1 ... H_{n-3} z, applied from the last
    for (int k = n - 3; k >= 0; --k) {
      const double beta = tau[k];
      if (beta == 0.0) continue;
      const double* vk = vst + (size_t)k * NN;
      double dot = 0.0;
      for (int i = k + 1 + lane; i < n; i += 64) dot += vk[i] * z[i];
      dot = beta * wave_sum(dot);
      for (int i = k + 1 + lane; i < n; i += 64) z[i] -= dot * vk[i];
      __syncthreads();
    }
    // sign: sum_b v_b >= 0, else first non-zero component positive
    double sum = 0.0;
    for (int i = lane; i < n; i += 64) sum += z[i];
    sum = wave_sum(sum);
    double first = 0.0;
    for (int i = 0; i < n; ++i)
      if (z[i] != 0.0) { first = z[i]; break; }
    const double sgn = (sum < 0.0 || (sum == 0.0 && first < 0.0)) ? -1.0 : 1.0;
    for (int i = lane; i < n; i += 64) g.v1[i * g.out_stride + cell] = (float)(sgn * z[i]);
  }
}

template <int NL, bool W, bool NC>
hipError_t launch_nl(int nbeam, const EigArgs& a, const EigArgs* items, const int64_t* cell0,
                     int nitem, int64_t total, bool v1, const double* zb, hipStream_t s) {
  const int vcap = v1 ? (nbeam - 1) * 8 * NL : 0;
  const size_t shm = (size_t)vcap * sizeof(double);
  if (shm > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)eig_tri_kernel<NL, W, NC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((eig_tri_kernel<NL, W, NC>), dim3((unsigned)total), dim3(64), shm, s, a,
                     items, cell0, nitem, vcap, zb);
  return hipGetLastError();
}

template <bool W, bool NC = false>
hipError_t launch_cls(int cls, int nbeam, const EigArgs& a, const EigArgs* items,
                      const int64_t* cell0, int nitem, int64_t total, bool v1, hipStream_t s,
                      const double* zb = nullptr) {
  switch (cls) {
    case 3: return launch_nl<3, W, NC>(nbeam, a, items, cell0, nitem, total, v1, zb, s);
    case 5: return launch_nl<5, W, NC>(nbeam, a, items, cell0, nitem, total, v1, zb, s);
    case 8: return launch_nl<8, W, NC>(nbeam, a, items, cell0, nitem, total, v1, zb, s);
    case 9: return launch_nl<9, W, NC>(nbeam, a, items, cell0, nitem, total, v1, zb, s);
    case 10: return launch_nl<10, W, NC>(nbeam, a, items, cell0, nitem, total, v1, zb, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int eig_tri_class(int n) {
  if (n < 2) return 0;
  if (n <= 24) return 3;
  if (n <= 40) return 5;
  if (n <= 64) return 8;
  if (n <= 72) return 9;
  if (n <= 80) return 10;
  return 0;
}

hipError_t launch_eig_tri(const EigArgs& a, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  if (ncell == 0) return hipSuccess;
  if (a.layout == 2)
    return launch_cls<true>(eig_tri_class(a.nbeam), a.nbeam, a, nullptr, nullptr, 0, ncell,
                            a.v1 != nullptr, s);
  return launch_cls<false>(eig_tri_class(a.nbeam), a.nbeam, a, nullptr, nullptr, 0, ncell,
                           a.v1 != nullptr, s);
}

hipError_t launch_eig_tri_nc(const EigArgs& a, const double* zb, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  if (ncell == 0) return hipSuccess;
  return launch_cls<false, true>(eig_tri_class(a.nbeam), a.nbeam, a, nullptr, nullptr, 0, ncell,
                                 a.v1 != nullptr, s, zb);
}

hipError_t launch_eig_tri_batch(int cls, const EigArgs* items, const int64_t* cell0, int nitem,
                                int64_t total, hipStream_t s, bool v1) {
  if (total == 0) return hipSuccess;
  EigArgs none{};
  // with v1, LDS for the reflectors of the class's largest matrix (8 cls rows)
  return launch_cls<false>(cls, v1 ? 8 * cls : 0, none, items, cell0, nitem, total, v1, s);
}

}  // namespace rfi
