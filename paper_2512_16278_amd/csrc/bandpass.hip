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
// systems. The per-system vectors live in a workspace laid out
// [channel][system], so that neighbouring threads touch neighbouring words
// at every step; the spectrum y is staged there once per call. Every sweep
// walks the channels in blocks of kBlk: the loads of a block are issued
// together before its steps run, so a step never waits on memory alone.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

namespace rfi {
namespace {

constexpr int kBpThreads = 64;
constexpr int kBlk = 16;
constexpr int kVecs = 7;          // w, 1/R_jj, R_{j,j+1}, R_{j,j+2}, u, z, y

struct BpArgs {
  int nbeam, nsub, nchan, itermax;
  double lam, ratio;
  const int32_t* sum_x;   // rows layout: sum_x[b][k * nchan + j]
  const int32_t* count;   // [nsub]
  double* z;              // out [nbeam][ncell]
  int32_t* passes;        // out [nsub][nbeam] or NULL
  double* ws;             // kVecs vectors of nchan * nsys doubles
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
  const size_t vs = (size_t)F * nsys;
  double* w = a.ws;
  double* r0 = w + vs;            // 1 / R_jj
  double* r1 = r0 + vs;
  double* r2 = r1 + vs;
  double* u = r2 + vs;
  double* z = u + vs;
  double* y = z + vs;
  auto at = [&](double* v, int j) -> double& { return v[(size_t)j * nsys + sys]; };
  if (F < 3) {
    for (int j = 0; j < F; ++j) zo[j] = (double)sx[j] / L;
    if (a.passes) a.passes[k * a.nbeam + b] = 0;
    return;
  }
  // stage the spectrum (channel means) and the first weights
  for (int j0 = 0; j0 < F; j0 += kBlk) {
    int32_t v[kBlk];
#pragma unroll
    for (int t = 0; t < kBlk; ++t) v[t] = sx[j0 + t < F ? j0 + t : F - 1];
#pragma unroll
    for (int t = 0; t < kBlk; ++t)
      if (j0 + t < F) {
        at(y, j0 + t) = (double)v[t] / L;
        at(w, j0 + t) = 1.0;
      }
  }
  int passes = 0;
  for (int it = 0; it < a.itermax; ++it) {
    ++passes;
    // Cholesky A = R^T R of A = W + lam D^T D (R upper, bandwidth 2), then
    // R^T u = W y and R z = u. The recurrences carry the previous two rows in
    // registers (p1 = R_{j-1,j}, p2 = R_{j-2,j}, q1 = R_{j-1,j+1}, u1, u2);
    // R and u go to the workspace for the backward sweep only.
    double p1 = 0.0, p2 = 0.0, q1 = 0.0, u1 = 0.0, u2 = 0.0;
    for (int j0 = 0; j0 < F; j0 += kBlk) {
      double wb[kBlk], yb[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j0 + t < F ? j0 + t : F - 1;
        wb[t] = at(w, j);
        yb[t] = at(y, j);
      }
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j0 + t;
        if (j >= F) break;
        double d0, d1, d2;
        dtd_row(j, F, d0, d1, d2);
        // one division per row: the row is scaled by 1 / R_jj
        const double ir = 1.0 / sqrt(wb[t] + a.lam * d0 - p1 * p1 - p2 * p2);
        const double r1j = (a.lam * d1 - p1 * q1) * ir;
        const double r2j = a.lam * d2 * ir;
        const double uj = (wb[t] * yb[t] - p1 * u1 - p2 * u2) * ir;
        at(r0, j) = ir;
        at(r1, j) = r1j;
        at(r2, j) = r2j;
        at(u, j) = uj;
        p2 = q1;        // R_{j-1, j+1} is R_{(j+1)-2, j+1}
        p1 = r1j;       // R_{j, j+1}
        q1 = r2j;       // R_{j, j+2}
        u2 = u1;
        u1 = uj;
      }
    }
    double z1 = 0.0, z2 = 0.0;
    for (int j1 = F - 1; j1 >= 0; j1 -= kBlk) {
      double ub[kBlk], ab[kBlk], bb[kBlk], cb[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j1 - t >= 0 ? j1 - t : 0;
        ub[t] = at(u, j);
        ab[t] = at(r1, j);
        bb[t] = at(r2, j);
        cb[t] = at(r0, j);
      }
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j1 - t;
        if (j < 0) break;
        const double zj = (ub[t] - ab[t] * z1 - bb[t] * z2) * cb[t];
        at(z, j) = zj;
        z2 = z1;
        z1 = zj;
      }
    }
    // negative residuals: mean and sample standard deviation
    double sn = 0.0;
    int nn = 0;
    for (int j0 = 0; j0 < F; j0 += kBlk) {
      double d[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j0 + t < F ? j0 + t : F - 1;
        d[t] = at(y, j) - at(z, j);
      }
#pragma unroll
      for (int t = 0; t < kBlk; ++t)
        if (j0 + t < F && d[t] < 0.0) { sn += d[t]; ++nn; }
    }
    if (nn < 2) break;
    const double m = sn / nn;
    double ss = 0.0;
    for (int j0 = 0; j0 < F; j0 += kBlk) {
      double d[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j0 + t < F ? j0 + t : F - 1;
        d[t] = at(y, j) - at(z, j);
      }
#pragma unroll
      for (int t = 0; t < kBlk; ++t)
        if (j0 + t < F && d[t] < 0.0) ss += (d[t] - m) * (d[t] - m);
    }
    const double sd = sqrt(ss / (nn - 1));
    if (!(sd > 0.0)) break;
    // new weights into u (free until the next pass), kept until the test
    double dw = 0.0, nw = 0.0;
    for (int j0 = 0; j0 < F; j0 += kBlk) {
      double d[kBlk], wo[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        const int j = j0 + t < F ? j0 + t : F - 1;
        d[t] = at(y, j) - at(z, j);
        wo[t] = at(w, j);
      }
#pragma unroll
      for (int t = 0; t < kBlk; ++t) {
        if (j0 + t >= F) break;
        const double wt = 1.0 / (1.0 + exp(2.0 * (d[t] - (2.0 * sd - m)) / sd));
        dw += (wo[t] - wt) * (wo[t] - wt);
        nw += wo[t] * wo[t];
        at(u, j0 + t) = wt;
      }
    }
    if (sqrt(dw) / sqrt(nw) < a.ratio) break;
    for (int j0 = 0; j0 < F; j0 += kBlk) {
      double v[kBlk];
#pragma unroll
      for (int t = 0; t < kBlk; ++t) v[t] = at(u, j0 + t < F ? j0 + t : F - 1);
#pragma unroll
      for (int t = 0; t < kBlk; ++t)
        if (j0 + t < F) at(w, j0 + t) = v[t];
    }
  }
  for (int j0 = 0; j0 < F; j0 += kBlk) {
    double v[kBlk];
#pragma unroll
    for (int t = 0; t < kBlk; ++t) v[t] = at(z, j0 + t < F ? j0 + t : F - 1);
#pragma unroll
    for (int t = 0; t < kBlk; ++t)
      if (j0 + t < F) zo[j0 + t] = v[t];
  }
  if (a.passes) a.passes[k * a.nbeam + b] = passes;
}

}  // namespace

size_t bandpass_workspace_size(int nbeam, int nchan, int nsub) {
  return (size_t)kVecs * nchan * nbeam * nsub * sizeof(double);
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
