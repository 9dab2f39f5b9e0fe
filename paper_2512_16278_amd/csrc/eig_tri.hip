// Per-cell eigen stage for larger beam counts, one cell per WAVEFRONT, in
// FP64 (Sec. 3.2-3.3, Eq. 1-2): Householder reduction of the correlation
// matrix to tridiagonal form, then Sturm-sequence bisection on the tridiagonal
// (Golub & Van Loan, Matrix Computations, Sec. 8.3 and 8.4).
//
// Work per cell is about (4/3) n^3 flops for the reduction instead of the
// 6 n^3 per sweep of cyclic Jacobi, and it runs in FP64 at the full vector
// rate of the chip, so lambda_1 needs no separate refinement:
//  - reduction: for k = 0 .. n-3 the reflector of column k below the diagonal
//    (v, beta with v_0 = 1), p = beta A22 v, w = p - (beta p.v / 2) v and
//    A22 -= v w^T + w v^T; rows are spread over the lanes;
//  - lambda_1 = largest eigenvalue (a correlation matrix is positive
//    semidefinite, so it is also the largest in magnitude): multisection, the
//    64 lanes each evaluating the Sturm count at one point of the bracket;
//  - all eigenvalues (optional): bisection, one eigenvalue index per lane;
//  - v1 (optional): inverse iteration on the tridiagonal with the shift
//    lambda_1, then the reflectors applied in reverse order.
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

__device__ __forceinline__ int64_t pidx(int a, int b, int n) {
  return (int64_t)a * n - (int64_t)a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// LDS layout for an n-beam cell (doubles unless noted): A [n][ld] with the
// odd row stride ld = n | 1 (rows of one column fall in different banks),
// then v, w, dinv, alpha (diagonal of T), beta_off (sub-diagonal of T),
// tau (reflector scales), z, then S (int32).
struct TriLds {
  static __host__ __device__ int ld(int n) { return n | 1; }
  static __host__ __device__ size_t bytes(int n) {
    return ((size_t)n * ld(n) + 7 * (size_t)n + 64) * sizeof(double) + (size_t)n * 4;
  }
};

// Number of eigenvalues of the tridiagonal (alpha, off) below x (Sturm
// count: negative pivots of the LDL^T factorisation of T - x I). A pivot
// that is zero (or nearly) is replaced by a tiny negative one, which keeps
// the count exact for x on an eigenvalue of a leading block.
__device__ __forceinline__ int sturm_below(const double* alpha, const double* off, int n,
                                           double x) {
  constexpr double PIV = 1e-290;
  double q = alpha[0] - x;
  if (fabs(q) < PIV) q = -PIV;
  int c = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (alpha[i] - x) - off[i - 1] * off[i - 1] / q;
    if (fabs(q) < PIV) q = -PIV;
    c += q < 0.0;
  }
  return c;
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

__device__ __forceinline__ int find_item_t(const int64_t* cell0, int nitem, int64_t c) {
  int lo = 0, hi = nitem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell0[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(64) void eig_tri_kernel(EigArgs g, const EigArgs* items,
                                                     const int64_t* cell0, int nitem) {
  extern __shared__ __attribute__((aligned(16))) double tsm[];
  int64_t cell = blockIdx.x;
  if (items) {
    const int i = find_item_t(cell0, nitem, cell);
    g = items[i];
    cell -= cell0[i];
  }
  const int n = g.nbeam;
  const int ld = TriLds::ld(n);
  double* A = tsm;
  double* v = A + (size_t)n * ld;
  double* w = v + n;
  double* dinv = w + n;
  double* alpha = dinv + n;
  double* off = alpha + n;
  double* tau = off + n;
  double* z = tau + n;
  int32_t* S = (int32_t*)(z + n + 64);
  const int lane = threadIdx.x;
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int64_t cnt = g.count[cell / g.nchan];
  if (cnt < 2 || cnt > RFI_MAX_COUNT) {
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

  // correlation matrix in FP64 (full, both triangles) and ||C||_F^2
  int dead = 0;
  for (int a = lane; a < n; a += 64) {
    S[a] = g.sum_x[a * ncell + cell];
    const int64_t Saa = g.sum_xy[pidx(a, a, n) * ncell + cell];
    const int64_t Naa = cnt * Saa - (int64_t)S[a] * S[a];
    dinv[a] = Naa > 0 ? 1.0 / sqrt((double)Naa) : 0.0;
    dead |= Naa <= 0;
  }
  const int degenerate = __syncthreads_or(dead);
  double offsq = 0.0;
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e - (e / n) * n;
    double r = 1.0;
    if (i != j) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      const int64_t Sab = g.sum_xy[pidx(a, b, n) * ncell + cell];
      const int64_t Nab = cnt * Sab - (int64_t)S[a] * S[b];
      r = (double)Nab * dinv[a] * dinv[b];
      if (i < j) offsq += r * r;
    }
    A[i * ld + j] = r;
  }
  const double frob2 = (double)n + 2.0 * wave_sum(offsq);
  __syncthreads();

  // Householder reduction to tridiagonal form
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;                 // length of the column below the diagonal
    const int r0 = k + 1;
    double s2 = 0.0;
    for (int i = lane + 1; i < m; i += 64) {
      const double x = A[(r0 + i) * ld + k];
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    const double x0 = A[r0 * ld + k];
    double beta = 0.0, sub = x0, v0 = 1.0;
    if (s2 > 0.0) {
      const double mu = sqrt(x0 * x0 + s2);
      v0 = x0 <= 0.0 ? x0 - mu : -s2 / (x0 + mu);
      beta = 2.0 * v0 * v0 / (s2 + v0 * v0);
      sub = mu;
    }
    for (int i = lane; i < m; i += 64) v[i] = i == 0 ? 1.0 : A[(r0 + i) * ld + k] / v0;
    if (lane == 0) {
      off[k] = sub;
      tau[k] = beta;
    }
    __syncthreads();
    if (beta != 0.0) {
      // p = beta A22 v (rows over lanes); K = beta p.v / 2; w = p - K v
      double pv = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double* row = A + (r0 + i) * ld + r0;
        double p = 0.0;
        for (int j = 0; j < m; ++j) p += row[j] * v[j];
        p *= beta;
        w[i] = p;
        pv += p * v[i];
      }
      const double K = 0.5 * beta * wave_sum(pv);
      __syncthreads();
      for (int i = lane; i < m; i += 64) w[i] -= K * v[i];
      __syncthreads();
      // A22 -= v w^T + w v^T
      for (int i = lane; i < m; i += 64) {
        double* row = A + (r0 + i) * ld + r0;
        const double vi = v[i], wi = w[i];
        for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
      }
    }
    // keep the reflector (v_1.. below the sub-diagonal) for the eigenvector
    for (int i = lane; i < m; i += 64) A[(r0 + i) * ld + k] = v[i];
    __syncthreads();
  }
  for (int i = lane; i < n; i += 64) alpha[i] = A[i * ld + i];
  if (lane == 0 && n >= 2) off[n - 2] = A[(n - 1) * ld + (n - 2)];
  __syncthreads();

  // Gershgorin bracket of the spectrum
  double glo = 1e300, ghi = -1e300;
  for (int i = lane; i < n; i += 64) {
    const double rad = (i > 0 ? fabs(off[i - 1]) : 0.0) + (i + 1 < n ? fabs(off[i]) : 0.0);
    glo = fmin(glo, alpha[i] - rad);
    ghi = fmax(ghi, alpha[i] + rad);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o));
    ghi = fmax(ghi, __shfl_xor(ghi, o));
  }
  const double span = fmax(ghi - glo, 1e-300);
  glo -= 1e-12 * span;
  ghi += 1e-12 * span;

  // lambda_1 = the largest eigenvalue: multisection. The bracket [lo, hi]
  // always holds exactly one crossing of count n-1 -> n (count(lo) <= n-1,
  // count(hi) = n); lane l tests lo + (l + 1) (hi - lo) / 65.
  double lo = glo, hi = ghi;
  for (int it = 0; it < 12 && hi - lo > 4e-16 * fmax(fabs(hi), 1.0); ++it) {
    const double h = (hi - lo) / 65.0;
    const double x = lo + (lane + 1) * h;
    const int c = sturm_below(alpha, off, n, x);
    // the first lane whose point has all n eigenvalues below it
    const unsigned long long ball = __ballot(c >= n);
    const int first = ball ? __builtin_ctzll(ball) : 64;
    const double nlo = first == 0 ? lo : lo + first * h;
    const double nhi = first == 64 ? hi : lo + (first + 1) * h;
    lo = nlo;
    hi = nhi;
  }
  const double lam1 = 0.5 * (lo + hi);

  if (lane == 0) {
    g.stat[cell] = lam1 * lam1 / frob2;
    g.status[cell] = degenerate ? RFI_CELL_DEGENERATE : 0;
  }

  if (g.eigvals) {
    // eigenvalue index i (ascending) by bisection on lane i mod 64; the
    // matrix is positive semidefinite up to rounding, so |lambda| descending
    // is index n - 1 - i
    for (int i = lane; i < n; i += 64) {
      double a = glo, b = ghi;
      for (int it = 0; it < 64 && b - a > 2e-16 * fmax(fabs(b), 1.0); ++it) {
        const double mid = 0.5 * (a + b);
        if (sturm_below(alpha, off, n, mid) > i) b = mid; else a = mid;
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
    // inverse iteration on T - sigma I, sigma just above lambda_1 (lane 0):
    // Gaussian elimination with partial pivoting of the tridiagonal into
    // U = (ud, ue, uf) (diagonal and two upper diagonals), then back
    // substitution; three iterations from the all-ones vector
    if (lane == 0) tri_inverse_iteration(alpha, off, n, lam1 + 1e-13 * fmax(fabs(lam1), 1.0),
                                         v, w, dinv, z);
    __syncthreads();
    // back-transform: v1 = H_0 H_1 ... H_{n-3} z, applied from the last
    for (int k = n - 3; k >= 0; --k) {
      const int m = n - k - 1, r0 = k + 1;
      const double beta = tau[k];
      if (beta == 0.0) continue;
      double dot = 0.0;
      for (int i = lane; i < m; i += 64) dot += A[(r0 + i) * ld + k] * z[r0 + i];
      dot = beta * wave_sum(dot);
      for (int i = lane; i < m; i += 64) z[r0 + i] -= dot * A[(r0 + i) * ld + k];
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

}  // namespace

size_t eig_tri_lds(int nbeam) { return TriLds::bytes(nbeam); }

hipError_t launch_eig_tri(const EigArgs& a, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  const size_t shm = TriLds::bytes(a.nbeam);
  hipError_t e = hipFuncSetAttribute((const void*)eig_tri_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_tri_kernel, dim3((unsigned)ncell), dim3(64), shm, s, a,
                     (const EigArgs*)nullptr, (const int64_t*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_eig_tri_batch(int max_nbeam, const EigArgs* items, const int64_t* cell0,
                                int nitem, int64_t total, hipStream_t s) {
  const size_t shm = TriLds::bytes(max_nbeam);
  hipError_t e = hipFuncSetAttribute((const void*)eig_tri_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  EigArgs none{};
  hipLaunchKernelGGL(eig_tri_kernel, dim3((unsigned)total), dim3(64), shm, s, none, items, cell0,
                     nitem);
  return hipGetLastError();
}

}  // namespace rfi
