// GPU twin of the seeded input generator (paper_2512_16278_amd/synth.py).
// Input generation only: none of the method's arithmetic lives here. The
// bytes are the same integer function of (seed, beam, time, channel) as the
// NumPy generator, from the same integer tables; see that module for the
// sample model. Philox4x32-10: Salmon, Moraes, Dror & Shaw, SC 2011.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfi_synth.h"

namespace {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ __launch_bounds__(256) void synth_kernel(rfi_synth_spec sp, int beam, int64_t t_lo,
                                                    int64_t nt, uint8_t* __restrict__ dst) {
  __shared__ uint32_t cdf[255];
  for (int i = threadIdx.x; i < 255; i += 256) cdf[i] = sp.cdf[beam * 255 + i];
  __syncthreads();
  const int ngrp = (sp.nchan + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= nt * ngrp) return;
  const int64_t t = t_lo + gid / ngrp;
  const int g = (int)(gid % ngrp);
  uint32_t c[4] = {(uint32_t)t, (uint32_t)g, (uint32_t)beam, (uint32_t)(t >> 32)};
  philox10(c, sp.key0, sp.key1);
  uint32_t word = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int ch = 4 * g + w;
    if (ch >= sp.nchan) break;
    // base = #{k : cdf[k] <= u}, by binary search on the monotone table
    const uint32_t u = c[w];
    int lo = 0, hi = 255;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cdf[mid] <= u) lo = mid + 1; else hi = mid;
    }
    int v = lo;
    const int si = sp.sin_of_chan[ch];
    if (si >= 0) {
      const int64_t* m = sp.sin_meta + 4 * si;
      if (t >= m[0] && t < m[1]) {
        const int64_t ph = (t + m[3]) % m[2];
        v += (sp.sin_tab[(int64_t)si * sp.pmax + ph] * sp.sin_gain[si * sp.nbeam + beam] + (1 << 15)) >> 16;
      }
    }
    for (int i = 0; i < sp.nburst; ++i)
      if (t >= sp.burst_meta[2 * i] && t < sp.burst_meta[2 * i + 1]) v += sp.burst_amp[i * sp.nbeam + beam];
    for (int i = 0; i < sp.npulse; ++i) {
      const int64_t* m = sp.pulse_meta + 5 * i;
      if (m[0] != beam) continue;
      const int64_t d = t - m[1] - sp.pulse_delay[(int64_t)i * sp.nchan + ch];
      if (d >= 0 && d % m[2] < m[3]) v += (int)m[4];
    }
    v = v < 0 ? 0 : (v > 255 ? 255 : v);
    word |= (uint32_t)v << (8 * w);
  }
  uint8_t* row = dst + (t - t_lo) * sp.row_stride + 4 * g;
  if (4 * g + 4 <= sp.row_stride) {
    *(uint32_t*)row = word;
  } else {
    for (int w = 0; w < 4 && 4 * g + w < sp.row_stride; ++w) row[w] = (uint8_t)(word >> (8 * w));
  }
}

}  // namespace

extern "C" int32_t rfi_synth_fill(const rfi_synth_spec* spec, int32_t beam, int64_t t_lo,
                                  int64_t t_hi, uint8_t* dst, void* stream) {
  if (!spec || !dst || beam < 0 || beam >= spec->nbeam || t_lo < 0 || t_hi < t_lo ||
      t_hi > spec->nsamp || spec->row_stride < spec->nchan || spec->row_stride % 4 != 0)
    return -1;
  const int64_t nt = t_hi - t_lo;
  if (nt == 0) return 0;
  const int64_t nthr = nt * ((spec->nchan + 3) / 4);
  const int64_t nblk = (nthr + 255) / 256;
  if (nblk > 0x7fffffff) return -1;
  hipLaunchKernelGGL(synth_kernel, dim3((unsigned)nblk), dim3(256), 0, (hipStream_t)stream, *spec,
                     beam, t_lo, nt, dst);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}
