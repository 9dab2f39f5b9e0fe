// Sums of Eq. 1 (Sec. 3.2) for sub-intervals longer than the int32 bound
// (Table 1 runs sub-intervals up to 10 s = 203,450 samples of 49.152 us):
// each sub-interval's time range is cut into chunks of at most RFI_MAX_COUNT
// samples, the sums engine forms the exact int32 sums of one chunk of every
// sub-interval in one launch (sub-interval starts L apart, chunk length c),
// and a widening pass adds them into int64 cell records
//     rec[cell][b]          = sum_t x_b(t)
//     rec[cell][n + pair]   = sum_t x_a(t) x_b(t)
// exact for any L <= RFI_MAX_COUNT_LONG (|sums| < 255^2 2^18 < 2^34).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace rfi {
namespace {

constexpr int kWidenThreads = 256;

// rec64[i] = (first ? 0 : rec64[i]) + rec32[i]; count[k] = L on the last chunk
__global__ __launch_bounds__(kWidenThreads) void widen_kernel(const int32_t* __restrict__ rec32,
                                                              int64_t* __restrict__ rec64,
                                                              int64_t n, int first,
                                                              int32_t* __restrict__ count,
                                                              int nsub, int L) {
  const int64_t i0 = ((int64_t)blockIdx.x * kWidenThreads + threadIdx.x) * 4;
  if (i0 + 3 < n) {
    const int4 v = *(const int4*)(rec32 + i0);
    if (first) {
      rec64[i0] = v.x; rec64[i0 + 1] = v.y; rec64[i0 + 2] = v.z; rec64[i0 + 3] = v.w;
    } else {
      rec64[i0] += v.x; rec64[i0 + 1] += v.y; rec64[i0 + 2] += v.z; rec64[i0 + 3] += v.w;
    }
  } else {
    for (int64_t i = i0; i < n; ++i) rec64[i] = (first ? 0 : rec64[i]) + rec32[i];
  }
  if (count && blockIdx.x == 0)
    for (int k = threadIdx.x; k < nsub; k += kWidenThreads) count[k] = L;
}

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

size_t ccm_long_tmp_bytes(int nbeam, int nchan, int nsub) {
  const size_t ncell = (size_t)nsub * nchan;
  return up256(ncell * (size_t)(nbeam + npair_of(nbeam)) * 4) + up256((size_t)nsub * 4);
}

hipError_t launch_ccm_long(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int64_t* rec, int32_t* count, void* tmp,
                           hipStream_t s, const CcmTune* t) {
  if (nsub == 0) return hipSuccess;
  const int nrow = nbeam + npair_of(nbeam);
  const int64_t nval = (int64_t)nsub * nchan * nrow;
  int32_t* rec32 = (int32_t*)tmp;
  int32_t* cnt32 = (int32_t*)((char*)tmp + up256((size_t)nval * 4));
  const int nch = (L + RFI_MAX_COUNT - 1) / RFI_MAX_COUNT;
  const int c = (L + nch - 1) / nch;
  const unsigned grid = (unsigned)((nval + 4 * kWidenThreads - 1) / (4 * kWidenThreads));
  for (int j = 0; j < nch; ++j) {
    const int Lj = L - j * c < c ? L - j * c : c;
    hipError_t e = launch_ccm_mfma(bp, nbeam, nchan, row_stride, t0 + (int64_t)j * c, Lj, nsub,
                                   rec32, nullptr, cnt32, 0, 0, s, t, 1, (int64_t)L);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(widen_kernel, dim3(grid), dim3(kWidenThreads), 0, s, rec32, rec, nval,
                       j == 0 ? 1 : 0, j == nch - 1 ? count : (int32_t*)nullptr, nsub, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rfi
