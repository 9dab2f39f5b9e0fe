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
#include <string.h>

#include <type_traits>

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
  // LDS: the ring of NST chunk buffers. After the last chunk the same space
  // holds the epilogue's offset sums [MAXB][CW], its row table [MAXROW]
  // (uint16) and its staging rows.
  static constexpr int MAXB = 16 * NB - 1;             // beams (plus the ones row)
  static constexpr int MAXROW = MAXB + MAXB * (MAXB + 1) / 2;
  static constexpr int LDS_MAX = 160 * 1024;
  static constexpr int RING = NST * STAGE;
  static constexpr int SXL_OFF = 0;
  static constexpr int TAB_OFF = SXL_OFF + MAXB * CW * 4;
  static constexpr int STG_OFF = (TAB_OFF + MAXROW * 2 + 15) / 16 * 16;
  // worst case of the staging: one wave's channels per pass at the largest
  // beam count
  static constexpr int STG_MIN = MAXROW * (CPW + 1) * 4;
  // the workgroup's LDS: the ring, or the epilogue's minimum if larger (more
  // epilogue passes in less space), 1 KB granules. A tile whose ring is at
  // most half the CU's LDS leaves room for a second workgroup, whose loads
  // then stream during this one's epilogue.
  static constexpr int NEED = RING > STG_OFF + STG_MIN ? RING : STG_OFF + STG_MIN;
  static constexpr int LDS = (NEED + 1023) / 1024 * 1024 < LDS_MAX
                                 ? (NEED + 1023) / 1024 * 1024
                                 : LDS_MAX;
  static constexpr int STG_BYTES = LDS - STG_OFF;
  static constexpr bool FITS = RING <= LDS_MAX && STG_BYTES >= STG_MIN;
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
  // 'ahead' chunks (IPW loads each) were requested after the one about to be
  // consumed; at most NST - 1
  if constexpr (NST >= 4) {
    if (ahead >= 3) { vm_wait_barrier<3 * IPW>(); return; }
  }
  if constexpr (NST >= 3) {
    if (ahead >= 2) { vm_wait_barrier<2 * IPW>(); return; }
  }
  if (ahead >= 1) { vm_wait_barrier<IPW>(); return; }
  vm_wait_barrier<0>();
}

// Tiles per XCD group: 1 KB of contiguous row bytes by default (measured best
// for the 4 KB-row FAST layout); a tune entry may choose another size.
int group_tiles(int cw, int group_bytes_override = 0) {
  const int gb = group_bytes_override > 0 ? group_bytes_override : 1024;
  return gb / cw > 1 ? gb / cw : 1;
}

template <int NB, int CW, int CPW, int IPW, int NST>
__global__ __launch_bounds__((MfmaCfg<NB, CW, CPW, IPW, NST>::NTHR), 1) void ccm_mfma_kernel(
    BeamPtrs bp, int nbeam, int nchan, int64_t row_stride, int64_t t0, int L, int nsub,
    int nct, int32_t* __restrict__ sum_x, int32_t* __restrict__ sum_xy,
    int32_t* __restrict__ count, int accumulate, int G, int nh, int prio, int layout,
    int64_t kstride, int ksplit, const CcmItem* __restrict__ items, int nitem) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  // the beam pointer table is the first kernel argument: index it in place
  const uint8_t* const* beam_tab = (const uint8_t* const*)__builtin_amdgcn_kernarg_segment_ptr();
  int w = blockIdx.x;
  if (items) {
    // batched launch: workgroups [wg0, wg0 + 8 ceil(tiles / 8)) belong to one
    // block (its own shape, beams, sub-intervals and sum buffers); find it
    int lo = 0, hi = nitem - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].wg0 <= w) lo = mid; else hi = mid - 1;
    }
    const CcmItem& it = items[lo];
    beam_tab = it.beams;
    nbeam = it.nbeam;
    nchan = it.nchan;
    row_stride = it.row_stride;
    t0 = it.t0;
    L = it.L;
    nsub = it.nsub;
    nct = it.nct;
    nh = it.nh;
    sum_x = it.sum_x;
    sum_xy = it.sum_xy;
    count = it.count;
    layout = it.layout;
    w -= it.wg0;
    if (w >= nsub * nct) return;      // padding to a multiple of 8 workgroups
    kstride = 0;
    ksplit = 1;
  }
  // sub-interval k of the launch starts at t0 + (k / ksplit) kstride +
  // (k mod ksplit) L: with ksplit = 1 and kstride = L they are back to back; a
  // longer stride sums one time chunk of each of several long sub-intervals,
  // and ksplit > 1 cuts each of those into ksplit consecutive chunks of L
  if (kstride == 0) kstride = L;
  // optional issue priority over waves of other kernels on the same SIMD
  if (prio) __builtin_amdgcn_s_setprio(2);
  extern __shared__ __attribute__((aligned(1024))) uint8_t lds[];
  // epilogue areas, over the drained ring
  int32_t* sxl = (int32_t*)(lds + C::SXL_OFF);       // [nbeam][CW] offset sums S'_a
  uint16_t* rowab = (uint16_t*)(lds + C::TAB_OFF);   // [nrow] (a, b) of each output row
  int32_t* stg = (int32_t*)(lds + C::STG_OFF);       // [nrow][CW / nh + 1] output staging
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ntiles = nsub * nct;
  const int nchunk = (L + TC - 1) / TC;
  const int64_t ncell = (int64_t)nsub * nchan;
  const int nrow = nbeam + nbeam * (nbeam + 1) / 2;

  // workgroup -> tile: G consecutive channel tiles of a sub-interval (G CW
  // contiguous bytes of every row) go to G workgroups that are dispatched
  // back to back on the same XCD (workgroup ids w, w + 8, w + 16, ...): the
  // hardware dispatcher then keeps adjacent tiles in step, and each row is
  // fetched in long runs through one L2
  const int full = G > 1 ? (ntiles / (8 * G)) * (8 * G) : 0;
  int tile = w;
  if (w < full) {
    const int u = w / (8 * G), rem = w % (8 * G);
    tile = G * (8 * u + rem % 8) + rem / 8;
  }

  // Per chunk this thread's lane fills unit (64 q + lane) of the buffer for
  // q = wave + NWAVE i, i < IPW; decode which (beam, row, seg) lands there.
  // Units past the beams, rows past the sub-interval and segments past the
  // row read a valid dummy address (never consumed), so every wave issues
  // exactly IPW loads per chunk and vmcnt counts stay uniform.
  const uint8_t* src_base[IPW];
  int src_row[IPW], src_col[IPW];
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    const int s = 64 * (wave + C::NWAVE * i) + lane;
    const int hi = s & ~7;
    const int bh = hi / C::UPB, rh = (hi % C::UPB) / C::SEGS;
    const int lin = s ^ ((bh + 2 * (rh >> 3)) & 7);
    const int b = lin / C::UPB, r = (lin % C::UPB) / C::SEGS, g = lin % C::SEGS;
    src_base[i] = beam_tab[b < nbeam ? b : 0];
    src_row[i] = b < nbeam ? r : -1;
    src_col[i] = 16 * g;
  }
  // DMA of chunk `chunk` of tile T into ring buffer `slot`
  auto issue = [&](int T, int chunk, int slot) {
    const int k = T / nct;
    const int c0 = (T % nct) * CW;
    uint8_t* buf = lds + slot * C::STAGE;
    const int rows = min(TC, L - chunk * TC);
    const int64_t row = t0 + (int64_t)(k / ksplit) * kstride + (int64_t)(k % ksplit) * L +
                        (int64_t)chunk * TC;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int64_t col = c0 + src_col[i];
      const bool ok = src_row[i] >= 0 && col < row_stride;
      const int r = (ok && src_row[i] < rows) ? src_row[i] : 0;
      const uint8_t* src = src_base[i] + (row + r) * row_stride + (ok ? col : 0);
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)src,
          (__attribute__((address_space(3))) void*)(buf + 1024 * (wave + C::NWAVE * i)), 16, 0, 0);
    }
  };

  v4i acc[CPW][C::NBP];
  auto zero_acc = [&]() {
#pragma unroll
    for (int c = 0; c < CPW; ++c)
#pragma unroll
      for (int p = 0; p < C::NBP; ++p) acc[c][p] = v4i{0, 0, 0, 0};
  };
  zero_acc();

  const int li = lane & 15;     // row (beam) within a 16-row block
  const int kg = lane >> 4;     // which 8 of the chunk's 32 rows this lane supplies
  const int cb = wave * CPW;    // first channel of this wave within the tile

  auto compute_chunk = [&](int slot) {
    const uint8_t* src = lds + slot * C::STAGE;
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

  // Epilogue of one tile. Output rows: r < nbeam is sum_x of beam r, r =
  // nbeam + pair(a, b) is sum_xy of (a, b); rowab[r] = a | b << 8 (b = 255
  // for sum_x rows). The offset sums S'_a (ones column) go to LDS first.
  // Then, in nh passes over the tile's channels (whole waves per pass), the
  // waves of the pass write their raw offset sums to the staging rows
  // [row][CW / nh + 1] (the pad keeps the scattered writes of one
  // instruction in distinct banks), and the whole workgroup converts them to
  // raw sums
  //     S_a = S'_a + 128 L,   S_ab = S'_ab + 128 (S'_a + S'_b) + 16384 L
  // and stores each row as CW / nh consecutive cells: coalesced runs. The
  // epilogue runs over the drained ring; its barriers wait for LDS only.
  auto lds_barrier = []() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };
  const int cwp = CW / nh;
  const int ch_st = tid % cwp, row_st = tid / cwp, rstep = C::NTHR / cwp;
  auto epilogue = [&](int T) {
    const int k = T / nct;
    const int c0 = (T % nct) * CW;
    for (int r = tid; r < nrow; r += C::NTHR) {
      int a = r, b = 255;
      if (r >= nbeam) {
        int q = r - nbeam;
        a = 0;
        while (q >= nbeam - a) { q -= nbeam - a; ++a; }
        b = a + q;
      }
      rowab[r] = (uint16_t)(a | (b << 8));
    }
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
    const uint32_t cnt = (uint32_t)L;
    const int mypass = cb / cwp;
    for (int h = 0; h < nh; ++h) {
      if (mypass == h) {
#pragma unroll
        for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
          for (int b2 = b1; b2 < NB; ++b2) {
            const int p = block_pair(b1, b2, NB);
            const int b = 16 * b2 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int a = 16 * b1 + 4 * kg + r;
              int row = -1;
              if (a <= b && b < nbeam) row = nbeam + a * nbeam - a * (a - 1) / 2 + (b - a);
              else if (b == nbeam && a < nbeam) row = a;
              if (row >= 0) {
                int32_t* dst = stg + row * (cwp + 1) + (cb - h * cwp);
#pragma unroll
                for (int c = 0; c < CPW; ++c) dst[c] = acc[c][p][r];
              }
            }
          }
      }
      lds_barrier();
      // rows layout: thread t stores channel t mod cwp of rows t / cwp,
      // t / cwp + rstep, ... (runs of consecutive cells); cell records:
      // thread t stores rows t mod rstep, + rstep, ... of channel t / rstep
      // (runs of consecutive rows of one cell)
      const int ch = layout ? tid / rstep : ch_st;
      const int row0 = layout ? tid % rstep : row_st;
      const int chl = h * cwp + ch;
      const int chan = c0 + chl;
      if (chan < nchan) {
        const int64_t cell = (int64_t)k * nchan + chan;
        int32_t* rec = sum_x + cell * nrow;
        for (int row = row0; row < nrow; row += rstep) {
          const uint32_t v = (uint32_t)stg[row * (cwp + 1) + ch];
          const int ab = rowab[row];
          const int a = ab & 255, b = ab >> 8;
          const uint32_t raw = b == 255 ? v + 128u * cnt
                                        : v + 128u * ((uint32_t)sxl[a * CW + chl] +
                                                      (uint32_t)sxl[b * CW + chl]) + 16384u * cnt;
          int32_t* dst = layout ? rec + row
                                : (row < nbeam ? sum_x + (int64_t)row * ncell
                                               : sum_xy + (int64_t)(row - nbeam) * ncell) + cell;
          *dst = accumulate ? (int32_t)((uint32_t)*dst + raw) : (int32_t)raw;
        }
      }
      lds_barrier();
    }
    if (c0 == 0 && tid == 0) count[k] = accumulate ? count[k] + L : L;
  };

  // ring of NST buffers: chunks c+1 .. c+NST-2 (and c+NST-1 once issued) are
  // in flight while chunk c is consumed
  for (int c = 0; c < NST - 1 && c < nchunk; ++c) issue(tile, c, c);
  for (int c = 0; c < nchunk; ++c) {
    const int last_issued = min(c + NST - 2, nchunk - 1);
    const int slot = c % NST;
    wait_chunk<IPW, NST>(last_issued - c);          // chunk c complete in LDS
    if (c + NST - 1 < nchunk) issue(tile, c + NST - 1, (c + NST - 1) % NST);  // buffer of c - 1
    if (c == nchunk - 1 && L % TC != 0) {
      // short last chunk: its rows past L hold dummy data; overwrite them
      // with 0x80 bytes (0 after the offset XOR)
      const int rows = L - c * TC;
      uint8_t* buf = lds + slot * C::STAGE;
      const int nu = nbeam * (TC - rows) * C::SEGS;
      for (int u = tid; u < nu; u += C::NTHR) {
        const int b = u / ((TC - rows) * C::SEGS);
        const int rr = rows + (u / C::SEGS) % (TC - rows);
        const int sg = u % C::SEGS;
        *(uint4*)(buf + 16 * unit_of<C::UPB, C::SEGS>(b, rr, sg)) =
            make_uint4(OFFSET_XOR, OFFSET_XOR, OFFSET_XOR, OFFSET_XOR);
      }
      lds_barrier();
    }
    compute_chunk(slot);
  }
  // every wave is past its last read of the ring before the epilogue reuses it
  lds_barrier();
  epilogue(tile);
}

// Epilogue passes: the fewest (power of two, whole waves each) whose staging
// rows fit; 0 if none does.
template <int NB, int CW, int CPW, int IPW, int NST>
int epilogue_passes(int nbeam) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  const int nrow = nbeam + nbeam * (nbeam + 1) / 2;
  int nh = 1;
  while (nh < C::NWAVE && nrow * (CW / nh + 1) * 4 > C::STG_BYTES) nh *= 2;
  return nrow * (CW / nh + 1) * 4 > C::STG_BYTES ? 0 : nh;
}

template <int NB, int CW, int CPW, int IPW, int NST>
hipError_t launch_mfma_cfg(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, int group_bytes, int layout,
                           int64_t kstride, int ksplit, hipStream_t s) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  if ((int64_t)nbeam * C::UPB > (int64_t)64 * IPW * C::NWAVE) return hipErrorInvalidValue;
  if (nbeam > C::MAXB) return hipErrorInvalidValue;
  const int nh = epilogue_passes<NB, CW, CPW, IPW, NST>(nbeam);
  if (nh == 0) return hipErrorInvalidValue;
  const int nct = (nchan + CW - 1) / CW;
  const auto kern = ccm_mfma_kernel<NB, CW, CPW, IPW, NST>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
  if (e != hipSuccess) return e;
  const int64_t ntiles = (int64_t)nsub * nct;
  const int G = group_tiles(CW, group_bytes);
  const int prio = 0;   // raised issue priority of the streaming waves measured no gain
  hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(C::NTHR), C::LDS, s, bp, nbeam, nchan,
                     row_stride, t0, L, nsub, nct, sum_x, sum_xy, count, accumulate, G, nh, prio,
                     layout, kstride, ksplit, (const CcmItem*)nullptr, 0);
  return hipGetLastError();
}

template <int NB, int CW, int CPW, int IPW, int NST>
hipError_t launch_batch_cfg(const CcmItem* items, int nitem, int total_wg, int group_bytes,
                            hipStream_t s) {
  using C = MfmaCfg<NB, CW, CPW, IPW, NST>;
  const auto kern = ccm_mfma_kernel<NB, CW, CPW, IPW, NST>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
  if (e != hipSuccess) return e;
  const int G = group_tiles(CW, group_bytes);
  BeamPtrs none;
  memset(&none, 0, sizeof(none));
  hipLaunchKernelGGL(kern, dim3((unsigned)total_wg), dim3(C::NTHR), C::LDS, s, none, 0, 0,
                     (int64_t)0, (int64_t)0, 0, 0, 0, (int32_t*)nullptr, (int32_t*)nullptr,
                     (int32_t*)nullptr, 0, G, 1, 0, 0, (int64_t)0, 1, items, nitem);
  return hipGetLastError();
}

// Largest ring (<= 4 buffers) of IPW KB-per-wave chunk buffers within 160 KB;
// calls op.run<NB, CW, CPW, IPW, NST>().
template <int NB, int CW, int CPW, int IPW, class Op>
hipError_t dispatch_nst(int max_stages, Op& op) {
  if constexpr (MfmaCfg<NB, CW, CPW, IPW, 4>::FITS) {
    if (max_stages >= 4) return op.template run<NB, CW, CPW, IPW, 4>();
  }
  if constexpr (MfmaCfg<NB, CW, CPW, IPW, 3>::FITS) {
    if (max_stages >= 3) return op.template run<NB, CW, CPW, IPW, 3>();
  }
  if constexpr (MfmaCfg<NB, CW, CPW, IPW, 2>::FITS) return op.template run<NB, CW, CPW, IPW, 2>();
  return hipErrorInvalidValue;
}

// The MFMA engine's instance for a beam count: 16-row blocks NB (including
// the ones row), tile width CW channels, CPW channels per wave, IPW loads per
// wave per chunk, ring depth NST. t (nullable) selects another tile variant
// of the beam count and caps the ring depth.
template <class Op>
hipError_t ccm_dispatch(int nbeam, int shared_cu, Op& op, const CcmTune* t = nullptr) {
  const int nb = (nbeam + 1 + 15) / 16;
  // tile shape per block count: (CW channels, CPW channels per wave). The
  // 16-31-beam default is 64 channels on 16 waves of 4 channels (a 3-deep
  // ring of 48 KB chunks): on the 19-beam FAST block it beats 8 waves of 8
  // channels (4-deep ring), variant 1, by about 3 % once the beams are
  // staggered across the memory channels. With shared_cu the tile is 32
  // channels on 8 waves of ~120 VGPRs.
  int cw, cpw;
  const int tile = t ? t->tile : 0;
  if (tile < 0 || tile >= ccm_tile_variants(nbeam)) return hipErrorInvalidValue;
  switch (nb) {
    case 1: cw = 64; cpw = 8; break;
    case 2:
      if (tile == 1) { cw = 64; cpw = 8; }
      else if (tile == 2 || shared_cu) { cw = 32; cpw = 4; }
      else { cw = 64; cpw = 4; }
      break;
    case 3: cw = 32; cpw = 4; break;
    case 4: case 5: cw = 16; cpw = 2; break;
    default: return hipErrorInvalidValue;
  }
  // ring depth cap (a tune entry's choice; default: the largest ring that fits)
  const int max_stages = t && t->stages >= 2 ? t->stages : 4;
  const int nwave = cw / cpw;
  const int units = nbeam * 32 * (cw / 16);        // 16-byte units per chunk
  const int ipw = (units + 64 * nwave - 1) / (64 * nwave);  // loads per wave per chunk
#define RFI_CCM(NB, CW, CPW, IPW)                         \
  if (nb == NB && cw == CW && cpw == CPW && ipw == IPW) \
    return dispatch_nst<NB, CW, CPW, IPW>(max_stages, op);
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

struct LaunchOne {
  const BeamPtrs& bp;
  int nbeam, nchan;
  int64_t row_stride, t0;
  int L, nsub;
  int32_t *sum_x, *sum_xy, *count;
  int accumulate, group_bytes, layout;
  int64_t kstride;
  int ksplit;
  hipStream_t s;
  template <int NB, int CW, int CPW, int IPW, int NST>
  hipError_t run() {
    return launch_mfma_cfg<NB, CW, CPW, IPW, NST>(bp, nbeam, nchan, row_stride, t0, L, nsub, sum_x,
                                                  sum_xy, count, accumulate, group_bytes, layout,
                                                  kstride, ksplit, s);
  }
};

struct Describe {
  int nbeam;
  CcmClass* out;
  template <int NB, int CW, int CPW, int IPW, int NST>
  hipError_t run() {
    out->key = ((NB * 128 + CW) * 16 + CPW) * 16 * 8 + IPW * 8 + NST;
    out->cw = CW;
    out->nh = epilogue_passes<NB, CW, CPW, IPW, NST>(nbeam);
    return out->nh > 0 ? hipSuccess : hipErrorInvalidValue;
  }
};

struct LaunchBatch {
  const CcmItem* items;
  int nitem, total_wg, group_bytes;
  hipStream_t s;
  template <int NB, int CW, int CPW, int IPW, int NST>
  hipError_t run() {
    return launch_batch_cfg<NB, CW, CPW, IPW, NST>(items, nitem, total_wg, group_bytes, s);
  }
};

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

int ccm_tile_variants(int nbeam) {
  const int nb = (nbeam + 1 + 15) / 16;
  return nb == 2 ? 3 : (nb >= 1 && nb <= 5 ? 1 : 0);
}

hipError_t launch_ccm_mfma(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, int shared_cu, hipStream_t s,
                           const CcmTune* t, int layout, int64_t kstride, int ksplit) {
  LaunchOne op{bp, nbeam, nchan, row_stride, t0, L, nsub, sum_x, sum_xy, count, accumulate,
               t ? t->group_bytes : 0, layout, kstride, ksplit < 1 ? 1 : ksplit, s};
  return ccm_dispatch(nbeam, shared_cu, op, t);
}

hipError_t ccm_class(int nbeam, CcmClass* c, const CcmTune* t) {
  Describe op{nbeam, c};
  hipError_t e = ccm_dispatch(nbeam, 0, op, t);
  // the tile group size is a launch argument: part of the class
  c->group_bytes = t ? t->group_bytes : 0;
  c->key = c->key * 65536 + (c->group_bytes & 0xFFFF);
  return e;
}

hipError_t launch_ccm_batch(int nbeam_of_class, const CcmTune* t, const CcmItem* items,
                            int nitem, int total_wg, hipStream_t s) {
  LaunchBatch op{items, nitem, total_wg, t ? t->group_bytes : 0, s};
  return ccm_dispatch(nbeam_of_class, 0, op, t);
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
