// ArPLS bandpass normalisation (Sec. 3.1; its parameters lam, ratio and
// itermax are those of Sec. 4.5): for each beam and sub-interval, the channel
// means y_j = S_b(k, j) / L (the sums of Eq. 1 over the sub-interval) are
// fitted by asymmetrically reweighted penalised least squares (Baek et al.
// 2015): with D the second-difference operator, solve (W + lam D^T D) z = W y,
// take the residuals d = y - z, the mean m and sample standard deviation s
// (ddof 1) of the negative ones, the weights w' = 1 / (1 + exp(2 (d - (2 s -
// m)) / s)), and repeat with W = diag(w') until ||w - w'|| / ||w|| < ratio
// (that pass's z is kept) or itermax passes. The baseline z is the bandpass
// that Sec. 3.1 subtracts from every sample of the channel.
//
// One thread per (beam, sub-interval) system: the solve is a sequential
// recurrence along the channels (banded Cholesky of the pentadiagonal
// matrix, then the two triangular sweeps), so the parallelism is across
// systems; the per-system vectors live in a workspace laid out
// [channel][system], so that neighbouring threads touch neighbouring words
// at every step.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

constexpr int kBpThreads = 64;

struct BpArgs {
  int nbeam, nsub, nchan, itermax;
  double lam, ratio;
  const int32_t* sum_x;   // rows layout: sum_x[b][k * nchan + j]
  const int32_t* count;   // [nsub]
  double* z;              // out [nbeam][ncell]
  int32_t* passes;        // out [nsub][nbeam] or NULL
  double* ws;             // 6 vectors of nchan * nsys doubles
};

// (D^T D) entries of row i: diagonal, first and second super-diagonal (D has
// rows r = 0 .. F - 3 with 1, -2, 1 at columns r, r + 1, r + 2).
__device__ __forceinline__ double dcoef(int o) { return o == 1 ? -2.0 : 1.0; }
__device__ __forceinline__ void dtd_row(int i, int F, double& d0, double& d1, double& d2) {
  d0 = d1 = d2 = 0.0;
  for (int r = i - 2; r <= i; ++r) {
    if (r < 0 || r > F - 3) continue;
    const int o = i - r;                         // position of i in row r
    d0 += dcoef(o) * dcoef(o);
    if (o + 1 <= 2) d1 += dcoef(o) * dcoef(o + 1);
    if (o + 2 <= 2) d2 += dcoef(o) * dcoef(o + 2);
  }
}

__global__ __launch_bounds__(kBpThreads) void arpls_kernel(BpArgs a) {
#pragma clang fp contract(off)
  const int nsys = a.nbeam * a.nsub;
  const int sys = blockIdx.x * kBpThreads + threadIdx.x;
  if (sys >= nsys) return;
  const int b = sys % a.nbeam, k = sys / a.nbeam;
  const int F = a.nchan;
  const int64_t ncell = (int64_t)a.nsub * F;
  const double L = (double)a.count[k];
  const int32_t* sx = a.sum_x + (int64_t)b * ncell + (int64_t)k * F;
  double* zo = a.z + (int64_t)b * ncell + (int64_t)k * F;
  // workspace vectors, element j of this system at [j * nsys + sys]
  double* w = a.ws;
  double* r0 = w + (size_t)F * nsys;
  double* r1 = r0 + (size_t)F * nsys;
  double* r2 = r1 + (size_t)F * nsys;
  double* u = r2 + (size_t)F * nsys;
  double* z = u + (size_t)F * nsys;
  auto at = [&](double* v, int j) -> double& { return v[(size_t)j * nsys + sys]; };
  auto yv = [&](int j) { return (double)sx[j] / L; };
  if (F < 3) {
    for (int j = 0; j < F; ++j) zo[j] = yv(j);
    if (a.passes) a.passes[k * a.nbeam + b] = 0;
    return;
  }
  for (int j = 0; j < F; ++j) at(w, j) = 1.0;
  int passes = 0;
  for (int it = 0; it < a.itermax; ++it) {
    ++passes;
    // Cholesky A = R^T R of A = W + lam D^T D (R upper, bandwidth 2), then
    // R^T u = W y and R z = u
    for (int j = 0; j < F; ++j) {
      double d0, d1, d2;
      dtd_row(j, F, d0, d1, d2);
      const double p1 = j >= 1 ? at(r1, j - 1) : 0.0;   // R_{j-1, j}
      const double p2 = j >= 2 ? at(r2, j - 2) : 0.0;   // R_{j-2, j}
      const double q1 = j >= 1 ? at(r2, j - 1) : 0.0;   // R_{j-1, j+1}
      const double rjj = sqrt(at(w, j) + a.lam * d0 - p1 * p1 - p2 * p2);
      at(r0, j) = rjj;
      at(r1, j) = (a.lam * d1 - p1 * q1) / rjj;
      at(r2, j) = a.lam * d2 / rjj;
      const double u1 = j >= 1 ? at(u, j - 1) : 0.0;
      const double u2 = j >= 2 ? at(u, j - 2) : 0.0;
      at(u, j) = (at(w, j) * yv(j) - p1 * u1 - p2 * u2) / rjj;
    }
    for (int j = F - 1; j >= 0; --j) {
      const double z1 = j + 1 < F ? at(z, j + 1) : 0.0;
      const double z2 = j + 2 < F ? at(z, j + 2) : 0.0;
      at(z, j) = (at(u, j) - at(r1, j) * z1 - at(r2, j) * z2) / at(r0, j);
    }
    // negative residuals: mean and sample standard deviation
    double sn = 0.0;
    int nn = 0;
    for (int j = 0; j < F; ++j) {
      const double d = yv(j) - at(z, j);
      if (d < 0.0) { sn += d; ++nn; }
    }
    if (nn < 2) break;
    const double m = sn / nn;
    double ss = 0.0;
    for (int j = 0; j < F; ++j) {
      const double d = yv(j) - at(z, j);
      if (d < 0.0) ss += (d - m) * (d - m);
    }
    const double s = sqrt(ss / (nn - 1));
    if (!(s > 0.0)) break;
    double dw = 0.0, nw = 0.0;
    for (int j = 0; j < F; ++j) {
      const double d = yv(j) - at(z, j);
      const double wt = 1.0 / (1.0 + exp(2.0 * (d - (2.0 * s - m)) / s));
      const double wj = at(w, j);
      dw += (wj - wt) * (wj - wt);
      nw += wj * wj;
      at(u, j) = wt;                               // new weights, kept until the test
    }
    if (sqrt(dw) / sqrt(nw) < a.ratio) break;
    for (int j = 0; j < F; ++j) at(w, j) = at(u, j);
  }
  for (int j = 0; j < F; ++j) zo[j] = at(z, j);
  if (a.passes) a.passes[k * a.nbeam + b] = passes;
}

}  // namespace

size_t bandpass_workspace_size(int nbeam, int nchan, int nsub) {
  return (size_t)6 * nchan * nbeam * nsub * sizeof(double);
}

hipError_t launch_arpls(int nbeam, int nsub, int nchan, const int32_t* sum_x,
                        const int32_t* count, double lam, double ratio, int itermax, double* z,
                        int32_t* passes, void* ws, hipStream_t s) {
  const int nsys = nbeam * nsub;
  if (nsys == 0) return hipSuccess;
  BpArgs a{nbeam, nsub, nchan, itermax, lam, ratio, sum_x, count, z, passes, (double*)ws};
  hipLaunchKernelGGL(arpls_kernel, dim3((unsigned)((nsys + kBpThreads - 1) / kBpThreads)),
                     dim3(kBpThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rfi
