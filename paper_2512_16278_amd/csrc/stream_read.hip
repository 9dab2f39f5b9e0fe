// Streaming-read reference kernel for the HBM roofline: every byte of a
// buffer is loaded once, in 16-byte vector loads with several in flight per
// lane, and folded into a per-thread XOR so that the loads are live.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfi_synth.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 256 * 8;        // 8 workgroups per CU
constexpr int kUnroll = 8;              // 16-byte loads in flight per lane

typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void stream_read_kernel(const u4* __restrict__ src,
                                                               int64_t nvec,
                                                               uint32_t* __restrict__ sink) {
  const int64_t nthr = (int64_t)gridDim.x * kThreads;
  const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  uint32_t acc = 0;
  int64_t i = tid;
  // main part: kUnroll independent loads per iteration, consecutive lanes on
  // consecutive 16-byte vectors
  for (; i + (kUnroll - 1) * nthr < nvec; i += kUnroll * nthr) {
    u4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * nthr);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < nvec; i += nthr) {
    const u4 v = src[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  sink[tid] = acc;
}

}  // namespace

extern "C" int32_t rfi_stream_read_sink_words(void) { return kThreads * kBlocks; }

extern "C" int32_t rfi_stream_read(const void* src, int64_t nbytes, uint32_t* sink,
                                   void* stream) {
  if (!src || !sink || nbytes < 0 || nbytes % 16 != 0 || ((uintptr_t)src) % 16 != 0) return -1;
  hipLaunchKernelGGL(stream_read_kernel, dim3(kBlocks), dim3(kThreads), 0, (hipStream_t)stream,
                     (const u4*)src, nbytes / 16, sink);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}
