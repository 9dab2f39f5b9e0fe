// Per-cell exact sums of Eq. 1 (Sec. 3.2): S_a = sum_t x_a(t) and
// S_ab = sum_t x_a(t) x_b(t), a <= b, for every (sub-interval, channel) cell.
//
// Main engine (ccm_mfma_kernel): the cell's beams x time samples form a small
// integer matrix X and the sums are X X^T, a dense contraction over time. The
// kernel feeds it to the int8 matrix cores (v_mfma_i32_16x16x32_i8) on
// x' = x - 128 (a byte XOR with 0x80), which is exact; the offset is removed
// again in integer arithmetic:
//     S_a  = S'_a + 128 L
//     S_ab = S'_ab + 128 (S'_a + S'_b) + 16384 L.
// S'_a comes out of the same products: one padding row of X is all ones.
//
// Data path: a workgroup owns CW consecutive channels of one sub-interval and
// walks its L samples in chunks of 32 rows. A chunk of every beam (32 rows x
// CW channel bytes) goes from HBM straight into LDS with the direct
// global-to-LDS loads (global_load_lds_dwordx4: lane l of a wave instruction
// fills bytes [16 l, 16 l + 16) of a 1 KB LDS window), into a ring of NST
// chunk buffers, so NST - 1 chunks are in flight while one is consumed and no
// registers hold staged data. The 16-byte units of a chunk are XOR-swizzled
// (unit ^= (beam + 2 (row / 8)) mod 8) so that the 64 lanes reading one row
// dword of 16 beams x 4 row groups hit every LDS bank group equally. A wave
// reads the rows of its channels back as dwords (4 channels x 1 time),
// transposes 4x4 bytes in registers (v_perm) to time-packed operands, and
// issues one MFMA per (channel, 16x16 beam block pair). Waits on the DMA use
// explicit vmcnt counts (every wave issues the same number of loads per
// chunk), not the workgroup fence, so later chunks stay in flight across the
// per-chunk barrier. The workgroups of 1 KB of adjacent channels are
// dispatched back to back on one XCD, so the rows are fetched in long runs.
//
// Comparison engine (ccm_valu_kernel, nbeam <= 20): one lane per channel, all
// pair accumulators in registers, four samples per v_dot4_u32_u8.
#include <stdlib.h>

#include "internal.h"

namespace rfi {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int TC = 32;              // rows per chunk = K of one MFMA
constexpr uint32_t OFFSET_XOR = 0x80808080u;

__device__ __forceinline__ void transpose4x4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                             uint32_t& o0, uint32_t& o1, uint32_t& o2,
                                             uint32_t& o3) {
  // rows r_i hold bytes (channel 0..3) of time i; o_c holds bytes (time 0..3)
  // of channel c.
  uint32_t t0 = __builtin_amdgcn_perm(r1, r0, 0x05010400u);
  uint32_t t1 = __builtin_amdgcn_perm(r3, r2, 0x05010400u);
  uint32_t t2 = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
  uint32_t t3 = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
  o0 = __builtin_amdgcn_perm(t1, t0, 0x05040100u);
  o1 = __builtin_amdgcn_perm(t1, t0, 0x07060302u);
  o2 = __builtin_amdgcn_perm(t3, t2, 0x05040100u);
  o3 = __builtin_amdgcn_perm(t3, t2, 0x07060302u);
}

__device__ __forceinline__ int block_pair(int b1, int b2, int nb) {
  // index of (b1 <= b2) in row-major upper-triangle order of nb blocks
  return b1 * nb - b1 * (b1 - 1) / 2 + (b2 - b1);
}

template <int NB, int CW, int CPW, int IPW, int NST>
struct MfmaCfg {
  static constexpr int NBP = NB * (NB + 1) / 2;        // 16x16 block pairs
  static constexpr int NWAVE = CW / CPW;
  static constexpr int NTHR = 64 * NWAVE;
  static constexpr int SEGS = CW / 16;                 // 16-byte units per row
  static constexpr int UPB = TC * SEGS;                // units per beam per chunk
  static constexpr int STAGE = IPW * NWAVE * 1024;     // bytes per chunk buffer
  static constexpr int NGRP = CPW >= 4 ? CPW / 4 : 1;  // dword groups of 4 channels
};

// LDS unit (16 bytes) of (beam, row, segment) inside a chunk buffer
template <int UPB, int SEGS>
__device__ __forceinline__ int unit_of(int beam, int row, int seg) {
  const int lin = beam * UPB + row * SEGS + seg;
  return lin ^ ((beam + 2 * (row >> 3)) & 7);
}

// wait until at most N vector-memory operations of this wave are in flight,
// then meet the workgroup; the memory clobber keeps LDS accesses on their side
template <int N>
__device__ __forceinline__ void vm_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

template <int IPW, int NST>
__device__ __forceinline__ void wait_chunk(int ahead) {
  // 'ahead' chunks were requested after the one about to be consumed
  if constexpr (NST >= 4) {
    if (ahead >= 2) { vm_wait_barrier<2 * IPW>(); return; }
  }
  if constexpr (NST >= 3) {
    if (ahead >= 1) { vm_wait_barrier<IPW>(); return; }
  }
  vm_wait_barrier<0>();
}

template <int NB, int CW, int CPW, int IPW, int NST>
__global__ __launch_bounds__((MfmaCfg<NB, CW, CPW, IPW, NST>::NTHR), 1) void ccm_mfma_kernel(
    BeamPtrs bp, int nbeam, int nchan, int64_t row_stride, int64_t t0, int L, int nsub,
    int nct, int32_t* __restrict__ sum_x, int32_t* __restrict__ sum_xy,
    int32_t* __restrict__ count, int accumulate, int remap) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  // workgroup -> tile: G consecutive channel tiles of a sub-interval (G CW
  // contiguous bytes of every row) go to G workgroups that are dispatched
  // back to back on the same XCD (workgroup ids w, w + 8, w + 16, ...), so
  // each row is fetched as one long run per XCD (DRAM page locality, shared L2)
  const int ntiles = nsub * nct;
  const int w = blockIdx.x;
  const int G = remap;
  const int full = G > 1 ? (ntiles / (8 * G)) * (8 * G) : 0;
  int tile = w;
  if (w < full) {
    const int u = w / (8 * G), rem = w % (8 * G);
    tile = G * (8 * u + rem % 8) + rem / 8;
  }
  const int k = tile / nct;
  const int c0 = (tile % nct) * CW;
  const int64_t ncell = (int64_t)nsub * nchan;
  const int64_t row0 = t0 + (int64_t)k * L;
  const int nchunk = (L + TC - 1) / TC;

  // the beam pointer table is the first kernel argument: index it in place
  const uint8_t* const* beam_tab = (const uint8_t* const*)__builtin_amdgcn_kernarg_segment_ptr();

  // Per chunk this thread's lane fills unit (64 q + lane) of the buffer for
  // q = wave + NWAVE i, i < IPW; decode which (beam, row, seg) lands there.
  // Units past the beams, rows past the sub-interval and segments past the
  // row read a valid dummy address (never consumed), so every wave issues
  // exactly IPW loads per chunk and vmcnt counts stay uniform.
  int64_t src_off[IPW];
  const uint8_t* src_base[IPW];
  int src_row[IPW];
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    const int s = 64 * (wave + C::NWAVE * i) + lane;
    const int hi = s & ~7;
    const int bh = hi / C::UPB, rh = (hi % C::UPB) / C::SEGS;
    const int lin = s ^ ((bh + 2 * (rh >> 3)) & 7);
    const int b = lin / C::UPB, r = (lin % C::UPB) / C::SEGS, g = lin % C::SEGS;
    const int64_t col = c0 + 16 * g;
    const bool ok = b < nbeam && col < row_stride;
    src_base[i] = beam_tab[ok ? b : 0];
    src_off[i] = ok ? col : 0;
    src_row[i] = ok ? r : -1;
  }
  auto issue = [&](int chunk) {
    uint8_t* buf = lds + (chunk % NST) * C::STAGE;
    const int rows = min(TC, L - chunk * TC);
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int r = (src_row[i] >= 0 && src_row[i] < rows) ? src_row[i] : 0;
      const uint8_t* src = src_base[i] + (row0 + (int64_t)chunk * TC + r) * row_stride + src_off[i];
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)src,
          (__attribute__((address_space(3))) void*)(buf + 1024 * (wave + C::NWAVE * i)), 16, 0, 0);
    }
  };

  v4i acc[CPW][C::NBP];
#pragma unroll
  for (int c = 0; c < CPW; ++c)
#pragma unroll
    for (int p = 0; p < C::NBP; ++p) acc[c][p] = v4i{0, 0, 0, 0};

  const int li = lane & 15;     // row (beam) within a 16-row block
  const int kg = lane >> 4;     // which 8 of the chunk's 32 rows this lane supplies
  const int cb = wave * CPW;    // first channel of this wave within the tile

  auto compute_chunk = [&](int chunk) {
    const uint8_t* src = lds + (chunk % NST) * C::STAGE;
    const int rows = min(TC, L - chunk * TC);
#pragma unroll
    for (int grp = 0; grp < C::NGRP; ++grp) {
      const int ch4 = (CPW >= 4) ? (cb + 4 * grp) : (cb & ~3);
      const int seg = ch4 >> 4, wrd = (ch4 & 15) >> 2;
      long op[NB][4];
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int beam = 16 * bb + li;
        uint32_t r[8];
        if (beam < nbeam) {
          // rows 8 kg + j: the swizzle only permutes units within aligned
          // groups of 8, so unit(j) = unit(j mod P) + 8 (j / P), P = 8 / SEGS,
          // and the 8 reads need P base addresses plus immediate offsets
          constexpr int P = 8 / C::SEGS;
          const uint8_t* basep[P];
#pragma unroll
          for (int m = 0; m < P; ++m)
            basep[m] = src + 16 * unit_of<C::UPB, C::SEGS>(beam, 8 * kg + m, seg) + 4 * wrd;
#pragma unroll
          for (int j = 0; j < 8; ++j)
            r[j] = *(const uint32_t*)(basep[j % P] + 128 * (j / P)) ^ OFFSET_XOR;
        } else {
          const uint32_t v = (beam == nbeam) ? 0x01010101u : 0u;
#pragma unroll
          for (int j = 0; j < 8; ++j) r[j] = v;
        }
        if (rows < TC) {
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (8 * kg + j >= rows) r[j] = 0;
        }
        uint32_t o[8];
        transpose4x4(r[0], r[1], r[2], r[3], o[0], o[1], o[2], o[3]);
        transpose4x4(r[4], r[5], r[6], r[7], o[4], o[5], o[6], o[7]);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          op[bb][c] = (long)(((uint64_t)o[4 + c] << 32) | (uint64_t)o[c]);
      }
      if constexpr (CPW >= 4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int slot = 4 * grp + c;
#pragma unroll
          for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
            for (int b2 = b1; b2 < NB; ++b2) {
              const int p = block_pair(b1, b2, NB);
              acc[slot][p] = __builtin_amdgcn_mfma_i32_16x16x32_i8(op[b1][c], op[b2][c],
                                                                   acc[slot][p], 0, 0, 0);
            }
        }
      } else {
        // this wave owns channels (cb & 3) .. (cb & 3) + CPW - 1 of the dword
        const int coff = cb & 3;
#pragma unroll
        for (int slot = 0; slot < CPW; ++slot) {
          const int c = coff + slot;                 // wave-uniform
          long sel[NB];
#pragma unroll
          for (int bb = 0; bb < NB; ++bb)
            sel[bb] = c == 0 ? op[bb][0] : c == 1 ? op[bb][1] : c == 2 ? op[bb][2] : op[bb][3];
#pragma unroll
          for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
            for (int b2 = b1; b2 < NB; ++b2) {
              const int p = block_pair(b1, b2, NB);
              acc[slot][p] = __builtin_amdgcn_mfma_i32_16x16x32_i8(sel[b1], sel[b2],
                                                                   acc[slot][p], 0, 0, 0);
            }
        }
      }
    }
  };

  // ring of NST buffers: chunks c+1 .. c+NST-2 (and c+NST-1 once issued) are
  // in flight while chunk c is consumed
  for (int c = 0; c < NST - 1 && c < nchunk; ++c) issue(c);
  for (int c = 0; c < nchunk; ++c) {
    const int last_issued = min(c + NST - 2, nchunk - 1);
    wait_chunk<IPW, NST>(last_issued - c);           // chunk c complete in LDS
    if (c + NST - 1 < nchunk) issue(c + NST - 1);     // reuses the buffer of chunk c - 1
    compute_chunk(c);
  }
  __syncthreads();

  // Epilogue: offset sums S'_a sit in the ones column; share them through LDS,
  // then every lane converts its entries to raw sums and stores them.
  int32_t* sxl = (int32_t*)lds;                      // [nbeam][CW]
  const int jn = nbeam & 15, bn = nbeam >> 4;
  if (li == jn) {
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
        for (int b2 = b1; b2 < NB; ++b2) {
          if (b2 != bn) continue;
          const int p = block_pair(b1, b2, NB);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = 16 * b1 + 4 * kg + r;
            if (a < nbeam) sxl[a * CW + cb + c] = acc[c][p][r];
          }
        }
  }
  __syncthreads();
  const uint32_t cnt = (uint32_t)L;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int chl = cb + c;
    const int chan = c0 + chl;
    if (chan >= nchan) continue;
    const int64_t cell = (int64_t)k * nchan + chan;
#pragma unroll
    for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
      for (int b2 = b1; b2 < NB; ++b2) {
        const int p = block_pair(b1, b2, NB);
        const int b = 16 * b2 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * b1 + 4 * kg + r;
          const uint32_t v = (uint32_t)acc[c][p][r];
          if (a <= b && b < nbeam) {
            const uint32_t raw = v + 128u * ((uint32_t)sxl[a * CW + chl] + (uint32_t)sxl[b * CW + chl]) +
                                 16384u * cnt;
            const int64_t idx = (int64_t)a * nbeam - (int64_t)a * (a - 1) / 2 + (b - a);
            int32_t* dst = sum_xy + idx * ncell + cell;
            *dst = accumulate ? (int32_t)((uint32_t)*dst + raw) : (int32_t)raw;
          } else if (b == nbeam && a < nbeam) {
            const uint32_t raw = v + 128u * cnt;
            int32_t* dst = sum_x + (int64_t)a * ncell + cell;
            *dst = accumulate ? (int32_t)((uint32_t)*dst + raw) : (int32_t)raw;
          }
        }
      }
  }
  if (c0 == 0 && tid == 0) count[k] = accumulate ? count[k] + L : L;
}

template <int NB, int CW, int CPW, int IPW, int NST>
hipError_t launch_mfma_cfg(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, hipStream_t s) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  if ((int64_t)nbeam * C::UPB > (int64_t)64 * IPW * C::NWAVE) return hipErrorInvalidValue;
  const int nct = (nchan + CW - 1) / CW;
  const size_t ring = (size_t)NST * C::STAGE;
  const size_t epi = (size_t)nbeam * CW * 4;
  const size_t shm = ring > epi ? ring : epi;
  const auto kern = ccm_mfma_kernel<NB, CW, CPW, IPW, NST>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  const int64_t ntiles = (int64_t)nsub * nct;
  // tiles per XCD group: 1 KB of contiguous row bytes by default (measured
  // best for the 4 KB-row FAST layout); RFI_CCM_GROUP_BYTES overrides
  static const int group_bytes = [] {
    const char* e = getenv("RFI_CCM_GROUP_BYTES");
    const int v = e ? atoi(e) : 1024;
    return v < 16 ? 16 : v;
  }();
  const int remap = group_bytes / CW > 1 ? group_bytes / CW : 1;
  hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(C::NTHR), shm, s, bp, nbeam, nchan,
                     row_stride, t0, L, nsub, nct, sum_x, sum_xy, count, accumulate, remap);
  return hipGetLastError();
}

// Largest ring (<= 4 buffers) of IPW KB-per-wave chunk buffers within 160 KB.
template <int NB, int CW, int CPW, int IPW>
hipError_t launch_ipw(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride, int64_t t0,
                      int L, int nsub, int32_t* sum_x, int32_t* sum_xy, int32_t* count,
                      int accumulate, int max_stages, hipStream_t s) {
  constexpr int stage_kb = IPW * (CW / CPW);
  constexpr int NST = (4 * stage_kb <= 160) ? 4 : (3 * stage_kb <= 160) ? 3 : 2;
  if (NST >= 4 && max_stages >= 4)
    return launch_mfma_cfg<NB, CW, CPW, IPW, (NST >= 4 ? 4 : 2)>(bp, nbeam, nchan, row_stride, t0,
                                                                  L, nsub, sum_x, sum_xy, count,
                                                                  accumulate, s);
  if (NST >= 3 && max_stages >= 3)
    return launch_mfma_cfg<NB, CW, CPW, IPW, (NST >= 3 ? 3 : 2)>(bp, nbeam, nchan, row_stride, t0,
                                                                  L, nsub, sum_x, sum_xy, count,
                                                                  accumulate, s);
  return launch_mfma_cfg<NB, CW, CPW, IPW, 2>(bp, nbeam, nchan, row_stride, t0, L, nsub, sum_x,
                                              sum_xy, count, accumulate, s);
}

// ---------------------------------------------------------------------------
// VALU comparison engine: one lane per channel, nbeam <= 20.
constexpr int VN = 20;
constexpr int VNP = VN * (VN + 1) / 2;

__global__ __launch_bounds__(256) void ccm_valu_kernel(BeamPtrs bp, int nbeam, int nchan,
                                                       int64_t row_stride, int64_t t0, int L,
                                                       int nsub, int32_t* __restrict__ sum_x,
                                                       int32_t* __restrict__ sum_xy,
                                                       int32_t* __restrict__ count,
                                                       int accumulate) {
  const int chan = blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) count[k] = accumulate ? count[k] + L : L;
  if (chan >= nchan) return;
  const int64_t row0 = t0 + (int64_t)k * L;
  uint32_t acc[VNP];
  uint32_t sx[VN];
#pragma unroll
  for (int i = 0; i < VNP; ++i) acc[i] = 0;
#pragma unroll
  for (int i = 0; i < VN; ++i) sx[i] = 0;
  for (int t = 0; t < L; t += 4) {
    uint32_t x[VN];
#pragma unroll
    for (int b = 0; b < VN; ++b) {
      uint32_t v = 0;
      if (b < nbeam) {
        const uint8_t* p = bp.p[b] + (row0 + t) * row_stride + chan;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < L) v |= (uint32_t)p[i * row_stride] << (8 * i);
      }
      x[b] = v;
    }
#pragma unroll
    for (int a = 0; a < VN; ++a) {
      sx[a] = __builtin_amdgcn_udot4(x[a], 0x01010101u, sx[a], false);
#pragma unroll
      for (int b = a; b < VN; ++b) {
        const int idx = a * VN - a * (a - 1) / 2 + (b - a);
        acc[idx] = __builtin_amdgcn_udot4(x[a], x[b], acc[idx], false);
      }
    }
  }
  const int64_t ncell = (int64_t)nsub * nchan;
  const int64_t cell = (int64_t)k * nchan + chan;
#pragma unroll
  for (int a = 0; a < VN; ++a) {
    if (a >= nbeam) continue;
    int32_t* d = sum_x + a * ncell + cell;
    *d = accumulate ? (int32_t)((uint32_t)*d + sx[a]) : (int32_t)sx[a];
#pragma unroll
    for (int b = a; b < VN; ++b) {
      if (b >= nbeam) continue;
      const int idx = a * VN - a * (a - 1) / 2 + (b - a);
      const int64_t out = (int64_t)a * nbeam - (int64_t)a * (a - 1) / 2 + (b - a);
      int32_t* q = sum_xy + out * ncell + cell;
      *q = accumulate ? (int32_t)((uint32_t)*q + acc[idx]) : (int32_t)acc[idx];
    }
  }
}

}  // namespace

hipError_t launch_ccm_mfma(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, int shared_cu, hipStream_t s) {
  const int nb = (nbeam + 1 + 15) / 16;   // 16-row blocks incl. the ones row
  // tile shape per block count: (CW channels, CPW channels per wave). With
  // shared_cu the tile is 32 channels on 8 waves of ~120 VGPRs, which leaves
  // every SIMD room for one wave of the register-resident eigensolver, so the
  // two kernels run side by side on each CU.
  int cw, cpw;
  static const int cpw2 = [] {
    const char* e = getenv("RFI_CCM_CPW");
    return e && atoi(e) == 4 ? 4 : 8;
  }();
  switch (nb) {
    case 1: cw = 64; cpw = 8; break;
    case 2:
      if (shared_cu) { cw = 32; cpw = 4; } else { cw = 64; cpw = cpw2; }
      break;
    case 3: cw = 32; cpw = 4; break;
    case 4: case 5: cw = 16; cpw = 2; break;
    default: return hipErrorInvalidValue;
  }
  // ring depth cap (tuning knob; default: the largest ring that fits)
  static const int max_stages = [] {
    const char* e = getenv("RFI_CCM_STAGES");
    const int v = e ? atoi(e) : 4;
    return v < 2 ? 2 : v;
  }();
  const int nwave = cw / cpw;
  const int units = nbeam * 32 * (cw / 16);        // 16-byte units per chunk
  const int ipw = (units + 64 * nwave - 1) / (64 * nwave);  // loads per wave per chunk
#define RFI_CCM(NB, CW, CPW, IPW)                                                          \
  if (nb == NB && cw == CW && cpw == CPW && ipw == IPW)                                \
    return launch_ipw<NB, CW, CPW, IPW>(bp, nbeam, nchan, row_stride, t0, L, nsub, sum_x, \
                                        sum_xy, count, accumulate, max_stages, s);
  RFI_CCM(1, 64, 8, 1) RFI_CCM(1, 64, 8, 2) RFI_CCM(1, 64, 8, 3) RFI_CCM(1, 64, 8, 4)
  RFI_CCM(2, 64, 8, 4) RFI_CCM(2, 64, 8, 5) RFI_CCM(2, 64, 8, 6) RFI_CCM(2, 64, 8, 7)
  RFI_CCM(2, 64, 8, 8)
  RFI_CCM(2, 64, 4, 2) RFI_CCM(2, 64, 4, 3) RFI_CCM(2, 64, 4, 4)
  RFI_CCM(2, 32, 4, 2) RFI_CCM(2, 32, 4, 3) RFI_CCM(2, 32, 4, 4)
  RFI_CCM(3, 32, 4, 4) RFI_CCM(3, 32, 4, 5) RFI_CCM(3, 32, 4, 6)
  RFI_CCM(4, 16, 2, 3) RFI_CCM(4, 16, 2, 4)
  RFI_CCM(5, 16, 2, 4) RFI_CCM(5, 16, 2, 5)
#undef RFI_CCM
  return hipErrorInvalidValue;
}

hipError_t launch_ccm_valu(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, hipStream_t s) {
  if (nbeam > VN) return hipErrorInvalidValue;
  dim3 grid((nchan + 255) / 256, nsub);
  hipLaunchKernelGGL(ccm_valu_kernel, grid, dim3(256), 0, s, bp, nbeam, nchan, row_stride, t0,
                     L, nsub, sum_x, sum_xy, count, accumulate);
  return hipGetLastError();
}

}  // namespace rfi
