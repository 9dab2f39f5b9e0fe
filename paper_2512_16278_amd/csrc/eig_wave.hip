// Per-cell eigendecomposition, one cell per WAVEFRONT, matrix in LDS; any
// nbeam <= RFI_MAX_BEAMS, in FP32 or FP64 (Sec. 3.2-3.3, Eq. 1-2).
//
// Two-sided Jacobi in the parallel round-robin ordering (Brent & Luk; the
// "circle" tournament): a sweep is m - 1 rounds (m = nbeam rounded up to
// even) of m/2 disjoint rotations, so the m/2 rotation angles of a round are
// computed by m/2 lanes at once and the whole wave then applies them: A <- A J
// and V <- V J column pairs in place, then A <- J^T A row pairs in place. The
// same skip rule as the per-lane solver is used (|a_pq| <= eps sqrt(|a_pp
// a_qq|), eps the unit of the working precision), sweeps stop after one
// without rotations or at max_sweeps. The dominant eigenvector is a column of
// the accumulated V, and lambda_1 is refined by its FP64 Rayleigh quotient;
// when all eigenvalues are requested each is refined the same way.
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr float v = 1.1920928955078125e-07f; };
template <> struct Eps<double> { static constexpr double v = 2.220446049250313e-16; };

__device__ __forceinline__ int64_t pidx(int a, int b, int n) {
  return (int64_t)a * n - (int64_t)a * (a - 1) / 2 + (b - a);
}

template <typename T>
struct WaveLds {
  // byte offsets of the LDS regions for an n-beam cell
  static __host__ __device__ size_t a_off(int) { return 0; }
  static __host__ __device__ size_t v_off(int n) { return (size_t)n * n * sizeof(T); }
  static __host__ __device__ size_t pair_off(int n) { return 2 * (size_t)n * n * sizeof(T); }
  // per pair k < m/2: P, Q (int), C, S (T)
  static __host__ __device__ size_t d_off(int n) {
    const int m = n + (n & 1);
    size_t o = pair_off(n) + (size_t)(m / 2) * (2 * sizeof(int) + 2 * sizeof(T));
    return (o + 7) & ~(size_t)7;
  }
  static __host__ __device__ size_t s_off(int n) { return d_off(n) + (size_t)n * sizeof(double); }
  static __host__ __device__ size_t red_off(int n) {
    return (s_off(n) + (size_t)n * sizeof(int32_t) + 7) & ~(size_t)7;
  }
  static __host__ __device__ size_t bytes(int n) { return red_off(n) + 2 * 64 * sizeof(double); }
};

__device__ __forceinline__ int find_item_w(const int64_t* cell0, int nitem, int64_t c) {
  int lo = 0, hi = nitem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell0[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// items == nullptr: the cells of g; else the cells of several blocks as one
// index space (cell0[i] = first global cell of items[i], ascending).
template <typename T>
__global__ __launch_bounds__(64) void eig_wave_kernel(EigArgs g, const EigArgs* items,
                                                      const int64_t* cell0, int nitem) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  int64_t cell = blockIdx.x;
  if (items) {
    const int i = find_item_w(cell0, nitem, cell);
    g = items[i];
    cell -= cell0[i];
  }
  using L = WaveLds<T>;
  const int n = g.nbeam;
  const int m = n + (n & 1);
  const int h = m / 2;
  T* A = (T*)(smem + L::a_off(n));
  T* V = (T*)(smem + L::v_off(n));
  int* P = (int*)(smem + L::pair_off(n));
  int* Q = P + h;
  T* Cc = (T*)(Q + h);
  T* Ss = Cc + h;
  double* d = (double*)(smem + L::d_off(n));
  int32_t* S = (int32_t*)(smem + L::s_off(n));
  double* red = (double*)(smem + L::red_off(n));

  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  const int lane = threadIdx.x;
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

  int dead = 0;
  for (int a = lane; a < n; a += 64) {
    S[a] = g.sum_x[a * ncell + cell];
    const int64_t Saa = g.sum_xy[pidx(a, a, n) * ncell + cell];
    const int64_t Naa = cnt * Saa - (int64_t)S[a] * S[a];
    d[a] = Naa > 0 ? 1.0 / sqrt((double)Naa) : 0.0;
    dead |= Naa <= 0;
  }
  const int degenerate = __syncthreads_or(dead);
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    T r = (T)1;
    if (i != j) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      const int64_t Sab = g.sum_xy[pidx(a, b, n) * ncell + cell];
      const int64_t Nab = cnt * Sab - (int64_t)S[a] * S[b];
      r = (T)((double)Nab * d[a] * d[b]);
    }
    A[e] = r;
    V[e] = i == j ? (T)1 : (T)0;
  }
  __syncthreads();

  const T eps = Eps<T>::v;
  int sweep = 0, last = 0;
  for (; sweep < g.max_sweeps; ++sweep) {
    int rot_sweep = 0;
    for (int r = 0; r < m - 1; ++r) {
      int rotated = 0;
      if (lane < h) {
        int p, q;
        if (lane == 0) {
          p = m - 1; q = r;
        } else {
          p = (r + lane) % (m - 1);
          q = (r - lane + m - 1) % (m - 1);
        }
        if (p > q) { const int t = p; p = q; q = t; }
        T c = (T)1, s = (T)0;
        if (q < n) {
          const T apq = A[p * n + q], app = A[p * n + p], aqq = A[q * n + q];
          if (apq * apq > eps * eps * fabs(app * aqq)) {
            const T theta = (aqq - app) / ((T)2 * apq);
            const T at = fabs(theta);
            T t = at > (T)1e15 ? (T)0.5 / at : (T)1 / (at + sqrt((T)1 + at * at));
            t = theta < (T)0 ? -t : t;
            c = (T)1 / sqrt((T)1 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        P[lane] = p; Q[lane] = q; Cc[lane] = c; Ss[lane] = s;
      }
      if (!__syncthreads_or(rotated)) continue;
      rot_sweep = 1;
      // A <- A J, V <- V J: column pairs (p, q) of every row i
      for (int w = lane; w < n * h; w += 64) {
        const int k = w % h, i = w / h;
        const T s = Ss[k];
        if (s == (T)0) continue;
        const int p = P[k], q = Q[k];
        const T c = Cc[k];
        const T aip = A[i * n + p], aiq = A[i * n + q];
        A[i * n + p] = c * aip - s * aiq;
        A[i * n + q] = s * aip + c * aiq;
        const T vip = V[i * n + p], viq = V[i * n + q];
        V[i * n + p] = c * vip - s * viq;
        V[i * n + q] = s * vip + c * viq;
      }
      __syncthreads();
      // A <- J^T A: row pairs (p, q) of every column j
      for (int w = lane; w < n * h; w += 64) {
        const int k = w % h, j = w / h;
        const T s = Ss[k];
        if (s == (T)0) continue;
        const int p = P[k], q = Q[k];
        const T c = Cc[k];
        const T apj = A[p * n + j], aqj = A[q * n + j];
        A[p * n + j] = c * apj - s * aqj;
        A[q * n + j] = s * apj + c * aqj;
      }
      __syncthreads();
      if (lane < h && Ss[lane] != (T)0) {
        A[P[lane] * n + Q[lane]] = (T)0;
        A[Q[lane] * n + P[lane]] = (T)0;
      }
      __syncthreads();
    }
    last = rot_sweep;
    if (!rot_sweep) break;
  }

  if (g.eigvals) {
    // every eigenvalue as the FP64 Rayleigh quotient of its column of V on the
    // FP64 correlation matrix: the error becomes second order in the
    // eigenvector error, instead of the O(n eps) of the FP32 sweeps. Rows of C
    // are formed one at a time in LDS and shared by all lanes.
    double* row = red;                          // n <= 79 <= 128 doubles
    double lam[2] = {0.0, 0.0};
    for (int a = 0; a < n; ++a) {
      __syncthreads();
      for (int b = lane; b < n; b += 64) {
        double cab = 1.0;
        if (b != a) {
          const int lo = a < b ? a : b, hi = a < b ? b : a;
          const int64_t Sab = g.sum_xy[pidx(lo, hi, n) * ncell + cell];
          const int64_t Nab = cnt * Sab - (int64_t)S[lo] * S[hi];
          cab = (double)Nab * d[lo] * d[hi];
        }
        row[b] = cab;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int i = lane + 64 * k;
        if (i >= n) continue;
        double tsum = 0.0;
        for (int b = 0; b < n; ++b) tsum += row[b] * (double)V[b * n + i];
        lam[k] += (double)V[a * n + i] * tsum;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int i = lane + 64 * k;
      if (i >= n) continue;
      double nrm = 0.0;
      for (int a = 0; a < n; ++a) nrm += (double)V[a * n + i] * (double)V[a * n + i];
      A[i * n + i] = (T)(lam[k] / nrm);
    }
    __syncthreads();
  }

  // dominant eigenvalue (largest |lambda|, lowest index on ties)
  if (lane == 0) {
    int i1 = 0;
    for (int i = 1; i < n; ++i)
      if (fabs(A[i * n + i]) > fabs(A[i1 * n + i1])) i1 = i;
    P[0] = i1;
  }
  __syncthreads();
  const int i1 = P[0];
  const double lam1 = (double)A[i1 * n + i1];
  if (g.eigvals) {
    for (int i = lane; i < n; i += 64) {
      const T li = fabs(A[i * n + i]);
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const T lj = fabs(A[j * n + j]);
        rank += (lj > li) || (lj == li && j < i);
      }
      g.eigvals[rank * g.out_stride + cell] = (float)A[i * n + i];
    }
  }

  // FP64 pass: ||C||_F^2, and the Rayleigh quotient of v = V[:, i1]
  double off = 0.0, num = 0.0, vv = 0.0;
  for (int a = lane; a < n; a += 64) {
    const double va = (double)V[a * n + i1];
    num += va * va;
    vv += va * va;
  }
  for (int e = lane; e < n * n; e += 64) {
    const int a = e / n, b = e % n;
    if (b <= a) continue;
    const int64_t Sab = g.sum_xy[pidx(a, b, n) * ncell + cell];
    const int64_t Nab = cnt * Sab - (int64_t)S[a] * S[b];
    const double rab = (double)Nab * d[a] * d[b];
    off += rab * rab;
    num += 2.0 * rab * (double)V[a * n + i1] * (double)V[b * n + i1];
  }
  // deterministic reductions: per-lane partials, summed in lane order
  red[lane] = off;
  red[64 + lane] = num;
  __syncthreads();
  double vsum = 0.0;
  if (lane == 0) {
    double so = 0.0, sn = 0.0;
    for (int i = 0; i < 64; ++i) { so += red[i]; sn += red[64 + i]; }
    red[0] = so;
    red[64] = sn;
  }
  __syncthreads();
  off = red[0];
  num = red[64];
  __syncthreads();
  red[lane] = vv;
  __syncthreads();
  if (lane == 0) {
    for (int i = 0; i < 64; ++i) vsum += red[i];
    const double f2 = (double)n + 2.0 * off;
    const double lam = g.refine ? num / vsum : lam1;
    g.stat[cell] = lam * lam / f2;
    uint8_t st = 0;
    if (degenerate) st |= RFI_CELL_DEGENERATE;
    if (last && sweep == g.max_sweeps) st |= RFI_CELL_NOT_CONVERGED;
    g.status[cell] = st;
    // sign convention: sum_b v_b >= 0, else first non-zero component positive
    double sum = 0.0, first = 0.0;
    for (int a = 0; a < n; ++a) {
      const double va = (double)V[a * n + i1];
      sum += va;
      if (first == 0.0) first = va;
    }
    red[0] = (sum < 0.0 || (sum == 0.0 && first < 0.0)) ? -1.0 : 1.0;
  }
  __syncthreads();
  if (g.v1) {
    const double sgn = red[0];   // columns of V are unit vectors
    for (int a = lane; a < n; a += 64) g.v1[a * g.out_stride + cell] = (float)(sgn * (double)V[a * n + i1]);
  }
}

template <typename T>
hipError_t launch_t(const EigArgs& a, hipStream_t s) {
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  const size_t shm = WaveLds<T>::bytes(a.nbeam);
  const auto kern = eig_wave_kernel<T>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)ncell), dim3(64), shm, s, a, (const EigArgs*)nullptr,
                     (const int64_t*)nullptr, 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_t(int max_nbeam, const EigArgs* items, const int64_t* cell0, int nitem,
                          int64_t total, hipStream_t s) {
  const size_t shm = WaveLds<T>::bytes(max_nbeam);
  const auto kern = eig_wave_kernel<T>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  EigArgs none{};
  hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(64), shm, s, none, items, cell0, nitem);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eig_wave(const EigArgs& a, int precision, hipStream_t s) {
  return precision == 64 ? launch_t<double>(a, s) : launch_t<float>(a, s);
}

hipError_t launch_eig_wave_batch(int precision, int max_nbeam, const EigArgs* items,
                                 const int64_t* cell0, int nitem, int64_t total, hipStream_t s) {
  return precision == 64 ? launch_batch_t<double>(max_nbeam, items, cell0, nitem, total, s)
                         : launch_batch_t<float>(max_nbeam, items, cell0, nitem, total, s);
}

}  // namespace rfi
