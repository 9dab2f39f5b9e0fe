// Sums of Eq. 1 (Sec. 3.2) for sub-intervals longer than the int32 bound
// (Table 1 runs sub-intervals up to 10 s = 203,450 samples of 49.152 us).
//
// Each sub-interval's time range is cut into P chunks of c = floor(L / P)
// samples plus a remainder of L - P c < P samples. One launch of the sums
// engine forms the exact int32 sums of every (sub-interval, chunk) pair at
// once, as if each chunk were a sub-interval of its own (ksplit = P), and a
// second, small launch those of the remainders; a widening pass then adds the
// P (+ 1) int32 records of each cell into its int64 record
//     rec[cell][b]          = sum_t x_b(t)
//     rec[cell][n + pair]   = sum_t x_a(t) x_b(t)
// exact for any L <= RFI_MAX_COUNT_LONG (|sums| < 255^2 2^18 < 2^34).
//
// P is at least ceil(L / RFI_MAX_COUNT) (each chunk within the int32 bound)
// and large enough that the chunk launch has about 2048 workgroups of 64
// channels: a single 10 s sub-interval of 4096 channels is only 64 tiles,
// which as one launch per chunk would leave three quarters of the CUs idle.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace rfi {
namespace {

constexpr int kWidenThreads = 256;
constexpr int kMaxSplit = 64;
constexpr int64_t kTargetTileChannels = (int64_t)2048 * 64;

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// chunks per sub-interval for n sub-intervals of F channels (at most
// kMaxSplit beyond what exactness needs)
int split_for(int L, int nsub, int nchan) {
  const int need = (L + RFI_MAX_COUNT - 1) / RFI_MAX_COUNT;
  int64_t want = (kTargetTileChannels + (int64_t)nsub * nchan - 1) / ((int64_t)nsub * nchan);
  if (want > kMaxSplit) want = kMaxSplit;
  if (want > L / 64) want = L / 64 > 0 ? L / 64 : 1;   // chunks of at least 64 samples
  return need > (int)want ? need : (int)want;
}

// largest split any L <= RFI_MAX_COUNT_LONG can take (sizes the scratch)
int max_split(int nsub, int nchan) {
  const int need = (RFI_MAX_COUNT_LONG + RFI_MAX_COUNT - 1) / RFI_MAX_COUNT;
  int64_t want = (kTargetTileChannels + (int64_t)nsub * nchan - 1) / ((int64_t)nsub * nchan);
  if (want > kMaxSplit) want = kMaxSplit;
  return need > (int)want ? need : (int)want;
}

// rec64[cell][row] = sum over the P chunk records (and the remainder record
// when rem) of that cell; count[k] = L. With accumulate the sums and counts
// are added to what the records and counts hold.
__global__ __launch_bounds__(kWidenThreads) void widen_kernel(const int32_t* __restrict__ rec32,
                                                              int64_t* __restrict__ rec64,
                                                              int nsub, int nchan, int nrow,
                                                              int P, int rem,
                                                              int32_t* __restrict__ count,
                                                              int L, int accumulate) {
  const int64_t per_sub = (int64_t)nchan * nrow;         // values of one sub-interval
  const int64_t n = (int64_t)nsub * per_sub;
  const int64_t i = (int64_t)blockIdx.x * kWidenThreads + threadIdx.x;
  if (count && blockIdx.x == 0)
    for (int k = threadIdx.x; k < nsub; k += kWidenThreads)
      count[k] = accumulate ? count[k] + L : L;
  if (i >= n) return;
  const int64_t k = i / per_sub, w = i % per_sub;
  const int32_t* src = rec32 + k * P * per_sub + w;
  int64_t acc = 0;
  for (int j = 0; j < P; ++j) acc += src[(int64_t)j * per_sub];
  if (rem) acc += rec32[(int64_t)nsub * P * per_sub + i];
  rec64[i] = accumulate ? rec64[i] + acc : acc;
}

}  // namespace

size_t ccm_long_tmp_bytes(int nbeam, int nchan, int nsub) {
  const size_t per_sub = (size_t)nchan * (nbeam + npair_of(nbeam));
  const size_t P = (size_t)max_split(nsub, nchan);
  return up256((size_t)nsub * (P + 1) * per_sub * 4) + up256((size_t)nsub * (P + 1) * 4);
}

hipError_t launch_ccm_long(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int64_t* rec, int32_t* count, void* tmp,
                           hipStream_t s, const CcmTune* t, int accumulate) {
  if (nsub == 0) return hipSuccess;
  const int nrow = nbeam + npair_of(nbeam);
  const int P = split_for(L, nsub, nchan);
  const int c = L / P, rem = L - P * c;
  const size_t per_sub = (size_t)nchan * nrow;
  const int Pmax = max_split(nsub, nchan);
  int32_t* rec32 = (int32_t*)tmp;
  int32_t* cnt32 = (int32_t*)((char*)tmp + up256((size_t)nsub * (Pmax + 1) * per_sub * 4));
  // every chunk of every sub-interval: launch sub-interval k P + j is chunk j
  // of sub-interval k, records [k P + j][channel][row]
  hipError_t e = launch_ccm_mfma(bp, nbeam, nchan, row_stride, t0, c, nsub * P, rec32, nullptr,
                                 cnt32, 0, 0, s, t, 1, (int64_t)L, P);
  if (e != hipSuccess) return e;
  if (rem) {
    // the last rem samples of each sub-interval, records after the chunks'
    e = launch_ccm_mfma(bp, nbeam, nchan, row_stride, t0 + (int64_t)P * c, rem, nsub,
                        rec32 + (size_t)nsub * P * per_sub, nullptr, cnt32 + (size_t)nsub * P, 0,
                        0, s, t, 1, (int64_t)L, 1);
    if (e != hipSuccess) return e;
  }
  const int64_t nval = (int64_t)nsub * (int64_t)per_sub;
  const unsigned grid = (unsigned)((nval + kWidenThreads - 1) / kWidenThreads);
  hipLaunchKernelGGL(widen_kernel, dim3(grid), dim3(kWidenThreads), 0, s, rec32, rec, nsub, nchan,
                     nrow, P, rem, count, L, accumulate);
  return hipGetLastError();
}

}  // namespace rfi
