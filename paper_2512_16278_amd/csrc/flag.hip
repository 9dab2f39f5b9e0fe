// Iterative Gaussian clipping of the statistic into the RFI mask (Sec. 3.3:
// the mean and standard deviation of the dominant eigenvalues are fitted, the
// cells above a dynamic threshold are masked, and this repeats until
// convergence; the threshold multiple kappa is the eigenvalue threshold
// parameter of Sec. 4.5; preserved channels of Sec. 4.3 are excluded), and
// the per-beam eigenvector threshold (Sec. 3.3 last paragraph; kappa_v of
// Sec. 4.5).
//
// The clip works on the statistic quantised to q = rint(s 2^40). Its moment
// sums N, Q1 = sum q and Q2 = sum q^2 are exact integers (64/128-bit), so every
// reduction order gives the same fit; mu = Q1 / (N 2^40) and
// sigma^2 = (N Q2 - Q1^2) / (N^2 2^80) are each rounded once from the exact
// rationals (integer long-division checks around an FP64 estimate), sigma is
// the correctly rounded square root, thr = mu + kappa sigma with two FP64
// roundings and no fused multiply-add. The masked set is always {q > T} for
// the running minimum T of the thresholds (in units of 2^-40), so a fit needs
// the sums over the eligible cells with q <= T, i.e. the block's totals minus
// the sums over the tail q > T.
//
// Four launches per block, no grid-wide barrier:
//  1. plan (one workgroup): the clip run in plain FP64 on a strided sample of
//     at most 4096 cells predicts its first threshold and where it will end;
//     a band (L, H] is placed from half a predicted sigma below the end to one
//     predicted sigma above the first threshold;
//  2. scan (many workgroups): exact per-workgroup sums over all eligible cells
//     and over those above the band (q > H), and every eligible cell inside
//     the band appended to a list;
//  3. iterate (one workgroup): the exact iteration. The sums at a threshold T
//     inside the band are the totals minus the sums above H minus the listed
//     cells above T (the list is held in LDS). Each fit is first formed in
//     FP64 from the exact integers with a proven error bound; when that bound
//     shows floor(thr 2^40) unambiguously, it is the exact fit's, otherwise the
//     exact fit is formed, and the reported (last) fit is always the exact one.
//     A T outside the band (the prediction was off) or a list that overflowed
//     its capacity falls back to a pass over every cell, so the result never
//     depends on the prediction, only the time does;
//  4. mask (many workgroups): mask = eligible and q > T.
// A batched form runs the same four launches over many blocks at once.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace rfi {
namespace {

typedef unsigned __int128 u128;
constexpr double TWO40 = 1099511627776.0;   // 2^40
constexpr int kPlanThreads = 64;               // one wavefront: no barriers
constexpr int kPlanPer = 16;                 // sample cells per plan thread
constexpr int kSample = kPlanThreads * kPlanPer;
constexpr int kIterThreads = 512;
constexpr int kIterLoad = 16;                // tail entries per iterate thread and load batch
constexpr int kNearMax = 16384;              // near-threshold tail entries kept in LDS
constexpr int kGridThreads = 256;
constexpr int kChunkPer = 4;                 // cells per thread and chunk (scan, mask)
constexpr int kChunk = kGridThreads * kChunkPer;
constexpr int kMaxParts = 2048;              // scan workgroups (grid-stride over chunks)
constexpr int64_t kTailMax = (int64_t)1 << 22;  // tail list capacity cap (entries)

__device__ __forceinline__ u128 mk128(uint64_t lo, uint64_t hi) {
  return ((u128)hi << 64) | (u128)lo;
}

// ---------------------------------------------------------------------------
// Exact arithmetic of the fit.

// Unsigned integer of 5 little-endian 64-bit limbs (320 bits).
struct U320 {
  uint64_t w[5];
};

__device__ __forceinline__ int clz64(uint64_t x) { return x ? __clzll((long long)x) : 64; }

// All limb loops below are unrolled with constant indices: a runtime index
// into the limb array would place it in scratch memory.
__device__ __forceinline__ int bitlen(const U320& a) {
  int r = 0;
#pragma unroll
  for (int i = 4; i >= 0; --i)
    if (r == 0 && a.w[i]) r = 64 * i + 64 - clz64(a.w[i]);
  return r;
}

__device__ __forceinline__ int cmp320(const U320& a, const U320& b) {
  int r = 0;
#pragma unroll
  for (int i = 4; i >= 0; --i)
    if (r == 0 && a.w[i] != b.w[i]) r = a.w[i] < b.w[i] ? -1 : 1;
  return r;
}

// a << s for 0 <= s < 320 (bits shifted past 320 are dropped; callers keep
// the result below 2^320): whole limbs by a select per limb, then bits.
__device__ __forceinline__ U320 shl320(const U320& a, int s) {
  const int q = s >> 6, b = s & 63;
  U320 r;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    uint64_t v = 0;
#pragma unroll
    for (int k = 0; k <= i; ++k)
      if (q == i - k) v = a.w[k];
    r.w[i] = v;
  }
  if (b) {
#pragma unroll
    for (int i = 4; i > 0; --i) r.w[i] = (r.w[i] << b) | (r.w[i - 1] >> (64 - b));
    r.w[0] <<= b;
  }
  return r;
}

// d * m for a 128-bit d and a 64-bit m (192-bit product)
__device__ U320 mul128x64(u128 d, uint64_t m) {
  const u128 lo = (u128)(uint64_t)d * m;
  const u128 hi = (u128)(uint64_t)(d >> 64) * m + (uint64_t)(lo >> 64);
  U320 r{};
  r.w[0] = (uint64_t)lo;
  r.w[1] = (uint64_t)hi;
  r.w[2] = (uint64_t)(hi >> 64);
  return r;
}

// w = a * b for 128-bit a, b (256-bit result, limbs 0..3)
__device__ U320 mul128x128(u128 a, u128 b) {
  const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
  const uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  const u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  U320 w{};
  w.w[0] = (uint64_t)p00;
  w.w[1] = (uint64_t)mid;
  const u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
  w.w[2] = (uint64_t)hi;
  w.w[3] = (uint64_t)(hi >> 64) + (uint64_t)(p11 >> 64);
  return w;
}

// a -= b (a >= b)
__device__ __forceinline__ void sub320(U320& a, const U320& b) {
  uint64_t borrow = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const uint64_t x = a.w[i] - b.w[i] - borrow;
    borrow = (a.w[i] < b.w[i] || (a.w[i] == b.w[i] && borrow)) ? 1 : 0;
    a.w[i] = x;
  }
}

// FP64 estimate of an integer (a few ulps; only seeds the exact search)
__device__ __forceinline__ double approx(const U320& a) {
  double r = 0.0;
#pragma unroll
  for (int i = 4; i >= 0; --i) r = r * 18446744073709551616.0 + (double)a.w[i];
  return r;
}

// sign(A - D * M * 2^e), A > 0, D > 0, M > 0
__device__ int cmp_scaled(const U320& A, u128 D, uint64_t M, int e) {
  const U320 R = mul128x64(D, M);
  const int la = bitlen(A), lr = bitlen(R);
  if (e >= 0) {
    if (la != lr + e) return la < lr + e ? -1 : 1;
    return cmp320(A, shl320(R, e));
  }
  if (la - e != lr) return la - e < lr ? -1 : 1;
  return cmp320(shl320(A, -e), R);
}

// A / D rounded to the nearest FP64 value (ties to even), for integers
// 0 <= A < 2^256 and 0 < D < 2^128 whose quotient is 0 or a normal number.
// The FP64 estimate is within a few ulps; the candidate m 2^e is moved until
// A / D lies between its two rounding midpoints, each compared exactly.
__device__ __noinline__ double div_rn(const U320& A, u128 D) {
  if (bitlen(A) == 0) return 0.0;
  U320 Dw{};
  Dw.w[0] = (uint64_t)D;
  Dw.w[1] = (uint64_t)(D >> 64);
  const double y = approx(A) / approx(Dw);
  int E;
  const double f = frexp(y, &E);                  // y = f 2^E, f in [0.5, 1)
  const uint64_t lo = (uint64_t)1 << 52, top = (uint64_t)1 << 53;
  uint64_t m = (uint64_t)ldexp(f, 53);            // [2^52, 2^53)
  int e = E - 53;
  for (int guard = 0; guard < 64; ++guard) {
    const int cu = cmp_scaled(A, D, 2 * m + 1, e - 1);   // upper midpoint
    if (cu > 0 || (cu == 0 && (m & 1))) {
      m += 1;
      if (m == top) { m = lo; e += 1; }
      if (cu == 0) break;                            // tie: the even neighbour
      continue;
    }
    if (cu == 0) break;                              // tie, m even
    // lower midpoint; at the bottom of a binade the neighbour below is
    // (2^53 - 1) 2^(e - 1)
    const int cl = m == lo ? cmp_scaled(A, D, 2 * top - 1, e - 2)
                           : cmp_scaled(A, D, 2 * m - 1, e - 1);
    if (cl < 0 || (cl == 0 && (m & 1))) {
      if (m == lo) { m = top - 1; e -= 1; } else { m -= 1; }
      if (cl == 0) break;
      continue;
    }
    break;
  }
  return ldexp((double)m, e);
}

// Correctly rounded square root of a non-negative normal (or zero) FP64 value:
// the hardware estimate, then exact integer checks of the two midpoints.
// (A midpoint's square is never a double, so there are no ties.)
__device__ __noinline__ double sqrt_rn(double v) {
  if (!(v > 0.0)) return v == 0.0 ? 0.0 : NAN;
  double r = sqrt(v);
  int ev;
  const double fv = frexp(v, &ev);
  const uint64_t mv = (uint64_t)ldexp(fv, 53);   // v = mv 2^(ev - 53)
  const int xv = ev - 53;
  const uint64_t lo = (uint64_t)1 << 52, top = (uint64_t)1 << 53;
  int er;
  const double fr = frexp(r, &er);
  uint64_t mr = (uint64_t)ldexp(fr, 53);          // r = mr 2^(er - 53)
  int xr = er - 53;
  // sign((M 2^x)^2 - mv 2^xv) for an odd M < 2^55 at exponent x
  auto cmp_sq = [&](uint64_t M, int x) -> int {
    const u128 lhs = (u128)M * M;                  // < 2^110
    const int d = xv - 2 * x;                      // compare lhs with mv 2^d
    const uint64_t lh = (uint64_t)(lhs >> 64);
    const int ll = lh ? 128 - clz64(lh) : 64 - clz64((uint64_t)lhs);
    const int lr = 64 - clz64(mv) + d;
    if (ll != lr) return ll < lr ? -1 : 1;         // equal lengths: both below 2^110
    if (d >= 0) {
      const u128 rhs = (u128)mv << d;
      return lhs < rhs ? -1 : (lhs > rhs ? 1 : 0);
    }
    const u128 l2 = lhs << (-d);                   // below 2^53
    return l2 < (u128)mv ? -1 : (l2 > (u128)mv ? 1 : 0);
  };
  for (int guard = 0; guard < 8; ++guard) {
    if (cmp_sq(2 * mr + 1, xr - 1) < 0) {          // (upper midpoint)^2 < v
      mr += 1;
      if (mr == top) { mr = lo; xr += 1; }
      continue;
    }
    const int cl = mr == lo ? cmp_sq(2 * top - 1, xr - 2) : cmp_sq(2 * mr - 1, xr - 1);
    if (cl > 0) {                                  // (lower midpoint)^2 > v
      if (mr == lo) { mr = top - 1; xr -= 1; } else { mr -= 1; }
      continue;
    }
    break;
  }
  return ldexp((double)mr, xr);
}

// sign(mid^2 - v) for mid = M 2^x (odd M < 2^55) and v = mv 2^xv
__device__ int cmp_sq(uint64_t M, int x, uint64_t mv, int xv) {
  const u128 lhs = (u128)M * M;                    // < 2^110
  const int d = xv - 2 * x;                        // compare lhs with mv 2^d
  const uint64_t lh = (uint64_t)(lhs >> 64);
  const int ll = lh ? 128 - clz64(lh) : 64 - clz64((uint64_t)lhs);
  const int lr = 64 - clz64(mv) + d;
  if (ll != lr) return ll < lr ? -1 : 1;           // equal lengths: both below 2^110
  if (d >= 0) {
    const u128 rhs = (u128)mv << d;
    return lhs < rhs ? -1 : (lhs > rhs ? 1 : 0);
  }
  const u128 l2 = lhs << (-d);                     // below 2^53
  return l2 < (u128)mv ? -1 : (l2 > (u128)mv ? 1 : 0);
}

// mu = Q1 / (N 2^40), sigma = sqrt((N Q2 - Q1^2) / (N^2 2^80)), thr = mu +
// kappa sigma, as the exact rationals rounded once each (N > 0), computed by
// the 64 lanes of one wavefront at once: lanes 0-15 place Q1 / N and lanes
// 16-31 (N Q2 - Q1^2) / N^2 between 16 consecutive rounding midpoints around
// their FP64 estimates in one round of exact comparisons, then lanes 0-15 do
// the same for the square root. A quotient whose 17 candidates straddle a
// power of two (or fall outside the window) is finished by the sequential
// search. Every lane gets the results.
__device__ __noinline__ void fit_wave(int64_t N, u128 Q1, u128 Q2, double kappa, double& mu, double& sigma,
                         double& thr) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int grp = (lane >> 4) & 1, j = lane & 15;
  const uint64_t lo = (uint64_t)1 << 52, top = (uint64_t)1 << 53;
  U320 A{};
  u128 D;
  if (grp == 0) {
    A.w[0] = (uint64_t)Q1;
    A.w[1] = (uint64_t)(Q1 >> 64);
    D = (u128)(uint64_t)N;
  } else {
    A = mul128x128((u128)(uint64_t)N, Q2);
    sub320(A, mul128x128(Q1, Q1));
    D = (u128)(uint64_t)N * (uint64_t)N;
  }
  const bool zero = bitlen(A) == 0;
  U320 Dw{};
  Dw.w[0] = (uint64_t)D;
  Dw.w[1] = (uint64_t)(D >> 64);
  int E = 0;
  const double f = zero ? 0.5 : frexp(approx(A) / approx(Dw), &E);
  const uint64_t m = (uint64_t)ldexp(f, 53);
  const int e = E - 53;
  const bool inside = m >= lo + 8 && m + 9 <= top;   // candidates m-8 .. m+8 in one binade
  // t = sign(x - mid_i), mid_i the midpoint above candidate m + i, i = j - 8
  const int t = (!zero && inside) ? cmp_scaled(A, D, 2 * (m + j - 8) + 1, e - 1) : 0;
  const unsigned long long pos = __ballot(t > 0), tie = __ballot(t == 0);
  const int sh = grp * 16;
  const unsigned gpos = (unsigned)(pos >> sh) & 0xffffu, gtie = (unsigned)(tie >> sh) & 0xffffu;
  const int cnt = __popc(gpos);
  double val;
  if (zero) {
    val = 0.0;
  } else if (!inside || cnt == 0 || cnt == 16 || (gtie & 1u) || ((gtie >> 15) & 1u)) {
    val = div_rn(A, D);                             // rare: the sequential search
  } else {
    // x lies above the midpoints i < cnt - 8, at or below mid_(cnt - 8)
    uint64_t c = m + cnt - 8;
    if ((gtie >> cnt) & 1u) c += (c & 1);           // exactly on a midpoint: the even one
    val = ldexp((double)c, e);
  }
  mu = ldexp(__shfl(val, 0), -40);
  const double var = ldexp(__shfl(val, 16), -80);
  // sigma: the correctly rounded square root of var
  double sg;
  if (!(var > 0.0)) {
    sg = 0.0;
  } else {
    int ev, er;
    const double fv = frexp(var, &ev);
    const uint64_t mv = (uint64_t)ldexp(fv, 53);
    const int xv = ev - 53;
    const double fr = frexp(sqrt(var), &er);
    const uint64_t mr = (uint64_t)ldexp(fr, 53);
    const int xr = er - 53;
    const bool in2 = mr >= lo + 8 && mr + 9 <= top;
    // u = sign(v - mid_i^2)
    const int u = in2 ? -cmp_sq(2 * (mr + j - 8) + 1, xr - 1, mv, xv) : 0;
    const unsigned long long p2 = __ballot(u > 0 && lane < 16);
    const int c2 = __popcll(p2);
    if (!in2 || c2 == 0 || c2 == 16) sg = sqrt_rn(var);
    else sg = ldexp((double)(mr + c2 - 8), xr);
  }
  sigma = sg;
  const double ks = kappa * sigma;     // two roundings: no fused multiply-add here
  thr = mu + ks;
}

__device__ __forceinline__ int64_t thr_to_T(double thr) {
  // s_q > thr  <=>  q > thr 2^40  <=>  q > floor(thr 2^40)  (exact scaling)
  const double tq = floor(thr * TWO40);
  return tq >= 9.2e18 ? INT64_MAX : (tq < -9.2e18 ? INT64_MIN : (int64_t)tq);
}

// ---------------------------------------------------------------------------
// Cells.

__device__ __forceinline__ int64_t quant(double s) { return __double2ll_rn(s * TWO40); }

// Cell c's statistic and eligibility (status without DEGENERATE / BAD_COUNT,
// channel not protected), loaded together so that a thread issues all its
// loads before it waits for any: c is clamped into the block (the caller
// drops clamped cells).
struct CellLd {
  double s;
  uint8_t st, pr;
};
__device__ __forceinline__ CellLd load_cell(const ClipJob& J, int64_t c, int64_t ncell) {
  const int64_t cc = c < ncell ? c : ncell - 1;
  CellLd r;
  r.s = J.stat[cc];
  r.st = J.status[cc];
  r.pr = J.protect ? J.protect[(uint32_t)cc % (uint32_t)J.nchan] : 0;
  return r;
}
__device__ __forceinline__ bool elig(const CellLd& x) {
  return !(x.st & (RFI_CELL_DEGENERATE | RFI_CELL_BAD_COUNT)) && !x.pr;
}

// Workspace of one clip: control words, the scan's per-workgroup partial
// sums, then the list of band cells.
struct Part {
  int64_t n, nf;              // all eligible cells; those above the band
  uint64_t q1[2], q2[2];
  uint64_t f1[2], f2[2];
  int64_t pad[6];
};
struct Ctrl {
  int64_t L, H;               // band (L, H]: eligible cells with L < q <= H are listed
  int64_t T;                  // final threshold for the mask pass
  unsigned long long count;   // band entries appended (may exceed the capacity)
  int64_t pad[4];
};
constexpr size_t kPartsOff = 256;
constexpr size_t kTailOff = kPartsOff + (size_t)kMaxParts * sizeof(Part);

__device__ __forceinline__ Ctrl* ctrl_of(const ClipJob& j) { return (Ctrl*)j.ws; }
__device__ __forceinline__ Part* parts_of(const ClipJob& j) {
  return (Part*)((char*)j.ws + kPartsOff);
}
__device__ __forceinline__ int64_t* tail_of(const ClipJob& j) {
  return (int64_t*)((char*)j.ws + kTailOff);
}

// Block-wide exact sum of (n, a, b); every thread gets the totals.
template <int NT>
struct Red3 {
  int64_t n[NT / 64];
  uint64_t a[NT / 64][2];
  uint64_t b[NT / 64][2];
};

// Wavefront sums by DPP row shifts (an inclusive scan within each 16-lane
// row; the four row totals are read from lanes 15, 31, 47 and 63): plain
// ALU operations instead of LDS-routed lane permutes. The results are
// wave-uniform.
template <int SHIFT>
__device__ __forceinline__ uint64_t dpp_shr(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x110 + SHIFT, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x110 + SHIFT, 0xf, 0xf, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  v += dpp_shr<1>(v);
  v += dpp_shr<2>(v);
  v += dpp_shr<4>(v);
  v += dpp_shr<8>(v);
  return lane_u64(v, 15) + lane_u64(v, 31) + lane_u64(v, 47) + lane_u64(v, 63);
}
__device__ __forceinline__ double wave_sum_f64(double x) {
  uint64_t v = __double_as_longlong(x);
  x += __longlong_as_double(dpp_shr<1>(v)); v = __double_as_longlong(x);
  x += __longlong_as_double(dpp_shr<2>(v)); v = __double_as_longlong(x);
  x += __longlong_as_double(dpp_shr<4>(v)); v = __double_as_longlong(x);
  x += __longlong_as_double(dpp_shr<8>(v)); v = __double_as_longlong(x);
  return __longlong_as_double(lane_u64(v, 15)) + __longlong_as_double(lane_u64(v, 31)) +
         __longlong_as_double(lane_u64(v, 47)) + __longlong_as_double(lane_u64(v, 63));
}
// exact wave sum of a u128 (32-bit limbs summed separately cannot overflow)
__device__ __forceinline__ u128 wave_sum_u128(u128 x) {
  const uint64_t l0 = wave_sum_u64((uint32_t)x), l1 = wave_sum_u64((uint32_t)(x >> 32));
  const uint64_t l2 = wave_sum_u64((uint32_t)(x >> 64)), l3 = wave_sum_u64((uint32_t)(x >> 96));
  return (u128)l0 + ((u128)l1 << 32) + ((u128)l2 << 64) + ((u128)l3 << 96);
}
__device__ __forceinline__ void wave_sum3(int64_t& n, u128& a, u128& b) {
  n = (int64_t)wave_sum_u64((uint64_t)n);
  a = wave_sum_u128(a);
  b = wave_sum_u128(b);
}

template <int NT>
__device__ void block_sum3(int64_t& n, u128& a, u128& b, Red3<NT>& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  wave_sum3(n, a, b);
  __syncthreads();                        // sh may still be read by an earlier call
  if (lane == 0) {
    sh.n[wave] = n;
    sh.a[wave][0] = (uint64_t)a; sh.a[wave][1] = (uint64_t)(a >> 64);
    sh.b[wave][0] = (uint64_t)b; sh.b[wave][1] = (uint64_t)(b >> 64);
  }
  __syncthreads();
  n = 0; a = 0; b = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    n += sh.n[w];
    a += mk128(sh.a[w][0], sh.a[w][1]);
    b += mk128(sh.b[w][0], sh.b[w][1]);
  }
}

// The band cells' moments with 64-bit partials: for 0 <= q < 2^42 split
// q = qh 2^21 + ql (qh, ql < 2^21), so that q^2 = qh^2 2^42 + qh ql 2^22 +
// ql^2 and every partial sum over at most 2^14 cells stays below 2^64; four
// 64-bit wave sums and one 32-bit instead of the nine 64-bit ones of the
// 128-bit sums. The totals are rebuilt exactly in 128 bits.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 15) + (uint32_t)__builtin_amdgcn_readlane((int)v, 31) +
         (uint32_t)__builtin_amdgcn_readlane((int)v, 47) + (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
struct SplitSums {
  uint32_t n;
  uint64_t a, h2, hl, l2;
};
template <int NT>
struct RedSplit {
  uint32_t n[NT / 64];
  uint64_t a[NT / 64], h2[NT / 64], hl[NT / 64], l2[NT / 64];
};
__device__ __forceinline__ void acc_split(int64_t q, SplitSums& t) {
  const uint64_t qh = (uint64_t)q >> 21, ql = (uint64_t)q & ((1u << 21) - 1);
  t.n += 1;
  t.a += (uint64_t)q;
  t.h2 += qh * qh;
  t.hl += qh * ql;
  t.l2 += ql * ql;
}
template <int NT>
__device__ void block_sum_split(SplitSums& t, int64_t& n, u128& a, u128& b, RedSplit<NT>& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  t.n = wave_sum_u32(t.n);
  t.a = wave_sum_u64(t.a);
  t.h2 = wave_sum_u64(t.h2);
  t.hl = wave_sum_u64(t.hl);
  t.l2 = wave_sum_u64(t.l2);
  __syncthreads();                        // sh may still be read by an earlier call
  if (lane == 0) {
    sh.n[wave] = t.n;
    sh.a[wave] = t.a;
    sh.h2[wave] = t.h2;
    sh.hl[wave] = t.hl;
    sh.l2[wave] = t.l2;
  }
  __syncthreads();
  uint64_t nn = 0, aa = 0, h2 = 0, hl = 0, l2 = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    nn += sh.n[w];
    aa += sh.a[w];
    h2 += sh.h2[w];
    hl += sh.hl[w];
    l2 += sh.l2[w];
  }
  n = (int64_t)nn;
  a = (u128)aa;
  b = ((u128)h2 << 42) + ((u128)hl << 22) + (u128)l2;
}

__device__ __forceinline__ void acc(int64_t q, int64_t& n, u128& a, u128& b) {
  n += 1;
  a += (u128)(uint64_t)q;
  b += (u128)(uint64_t)q * (uint64_t)q;
}

template <bool kBatch>
__device__ __forceinline__ ClipJob job_of(const ClipJob& j, const ClipJob* jobs, int idx) {
  if constexpr (kBatch) return jobs[idx];
  else return j;
}

__device__ __forceinline__ int64_t to_q(double x) {
  return x >= 9.2e18 ? INT64_MAX : (x < -9.2e18 ? INT64_MIN : (int64_t)x);
}

// Threshold of the FP64 fit from the exact sums when it provably equals the
// exact fit's: ok = 0 when floor(thr 2^40) could differ. The FP64 thr differs
// from the exactly rounded one by at most 10 u thr (u = 2^-53: Q1, N, the
// exact N Q2 - Q1^2 and N^2 each rounded once or, for the 256-bit value,
// accumulated over its limbs, then a division, a square root, a product and a
// sum, against mu, var, sigma, kappa sigma and thr of the exact fit each
// rounded once); the test keeps a margin of 64 u thr 2^40.
__device__ __forceinline__ int64_t fit_T_fast(int64_t N, u128 Q1, u128 Q2, double kappa, bool& ok) {
  U320 X = mul128x128((u128)(uint64_t)N, Q2);
  sub320(X, mul128x128(Q1, Q1));
  const double dN = (double)N;
  const double mu = (double)Q1 / dN;                       // in units of 2^-40
  const double var = approx(X) / (dN * dN);                 // in units of 2^-80
  const double t = mu + kappa * sqrt(var);                  // thr 2^40
  const double fl = floor(t);
  const double margin = 64.0 * 1.1102230246251565e-16 * t + 1e-300;
  ok = (t - fl) > margin && (fl + 1.0 - t) > margin && t < 9.0e18;
  return to_q(fl);
}

// 1. plan: the band (L, H] from a strided sample (FP64, inexact on purpose:
// it only places the band).
template <bool kBatch>
__global__ __launch_bounds__(kPlanThreads) void clip_plan_kernel(ClipJob job0, const ClipJob* jobs) {
  const ClipJob J = job_of<kBatch>(job0, jobs, blockIdx.x);
  const int64_t ncell = (int64_t)J.nsub * J.nchan;
  const int64_t ns = ncell < kSample ? ncell : kSample;
  const double stride = ns > 0 ? (double)ncell / (double)ns : 0.0;
  double v[kPlanPer];
  if (ns > 0) {
    CellLd x[kPlanPer];
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) {
      const int64_t k = threadIdx.x + (int64_t)i * kPlanThreads;
      x[i] = load_cell(J, k < ns ? (int64_t)((double)k * stride) : ncell, ncell);
    }
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) {
      const int64_t k = threadIdx.x + (int64_t)i * kPlanThreads;
      v[i] = (k < ns && elig(x[i])) ? (double)quant(x[i].s) / TWO40 : NAN;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) v[i] = NAN;
  }
  double Nh = 0.0, Q1h = 0.0, Q2h = 0.0;
  if (J.state) {
    Nh = (double)J.state->n;
    Q1h = (double)mk128(J.state->q1[0], J.state->q1[1]) / TWO40;
    Q2h = (double)mk128(J.state->q2[0], J.state->q2[1]) / (TWO40 * TWO40);
  }
  double T = INFINITY, sig = 0.0, prev = -1.0, T1 = INFINITY, sig1 = 0.0;
  for (int it = 0; it < J.max_iter + 1; ++it) {
    double n = 0, a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i)
      if (v[i] <= T) { n += 1; a += v[i]; b += v[i] * v[i]; }
    n = wave_sum_f64(n);
    a = wave_sum_f64(a);
    b = wave_sum_f64(b);
    if (n == prev) break;                      // the last fit masked nothing new
    prev = n;
    const double N = stride * n + Nh;
    if (!(N > 0)) break;
    const double mu = (stride * a + Q1h) / N;
    const double var = (stride * b + Q2h) / N - mu * mu;
    sig = var > 0 ? sqrt(var) : 0.0;
    const double thr = mu + J.kappa * sig;
    if (it == 0) { T1 = thr; sig1 = sig; }
    if (!(thr < T)) break;
    T = thr;
  }
  if (threadIdx.x == 0) {
    Ctrl* ct = ctrl_of(J);
    int64_t L = INT64_MIN, H = INT64_MAX;
    if (isfinite(T)) L = to_q(floor((T - 0.5 * sig) * TWO40) - 1.0);
    if (isfinite(T1)) H = to_q(floor((T1 + (1.0 + J.kappa) * 0.25 * sig1) * TWO40) + 1.0);
    if (H < L) H = L;
    ct->L = L;
    ct->H = H;
    ct->count = 0;
  }
}

// 2. scan: exact partial sums (all eligible cells, and those above the band)
// and the list of band cells. A workgroup reserves room for all its band cells
// of a chunk with one atomic.
template <bool kBatch>
__global__ __launch_bounds__(kGridThreads) void clip_scan_kernel(ClipJob job0, const ClipJob* jobs) {
  const ClipJob J = job_of<kBatch>(job0, jobs, blockIdx.y);
  if ((int)blockIdx.x >= J.nparts) return;
  __shared__ Red3<kGridThreads> red;
  __shared__ unsigned wcnt[kGridThreads / 64];
  __shared__ unsigned long long wbase[kGridThreads / 64];
  const int64_t ncell = (int64_t)J.nsub * J.nchan;
  Ctrl* ct = ctrl_of(J);
  const int64_t L = ct->L, H = ct->H;
  int64_t* tail = tail_of(J);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long below = lane ? ((~0ull) >> (64 - lane)) : 0ull;
  int64_t n = 0, nf = 0;
  u128 q1 = 0, q2 = 0, f1 = 0, f2 = 0;
  for (int64_t ch = blockIdx.x; ch * kChunk < ncell; ch += J.nparts) {
    CellLd x[kChunkPer];
#pragma unroll
    for (int i = 0; i < kChunkPer; ++i)
      x[i] = load_cell(J, ch * kChunk + i * kGridThreads + threadIdx.x, ncell);
    int64_t q[kChunkPer];
    unsigned off[kChunkPer];
    bool hit[kChunkPer];
    unsigned wtot = 0;
#pragma unroll
    for (int i = 0; i < kChunkPer; ++i) {
      const int64_t c = ch * kChunk + i * kGridThreads + threadIdx.x;
      const bool ok = c < ncell && elig(x[i]);
      q[i] = quant(x[i].s);
      if (ok) acc(q[i], n, q1, q2);
      if (ok && q[i] > H) acc(q[i], nf, f1, f2);
      hit[i] = ok && q[i] > L && q[i] <= H;
      const unsigned long long m = __ballot(hit[i]);
      off[i] = wtot + (unsigned)__popcll(m & below);
      wtot += (unsigned)__popcll(m);
    }
    if (lane == 0) wcnt[wave] = wtot;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned tot = 0;
      for (int w = 0; w < kGridThreads / 64; ++w) tot += wcnt[w];
      unsigned long long base = tot ? atomicAdd(&ct->count, (unsigned long long)tot) : 0ull;
      for (int w = 0; w < kGridThreads / 64; ++w) { wbase[w] = base; base += wcnt[w]; }
    }
    __syncthreads();
    const unsigned long long base = wbase[wave];
#pragma unroll
    for (int i = 0; i < kChunkPer; ++i) {
      const unsigned long long idx = base + off[i];
      if (hit[i] && idx < (unsigned long long)J.tail_cap) tail[idx] = q[i];
    }
  }
  block_sum3<kGridThreads>(n, q1, q2, red);
  block_sum3<kGridThreads>(nf, f1, f2, red);
  if (threadIdx.x == 0) {
    Part p{};
    p.n = n;
    p.q1[0] = (uint64_t)q1; p.q1[1] = (uint64_t)(q1 >> 64);
    p.q2[0] = (uint64_t)q2; p.q2[1] = (uint64_t)(q2 >> 64);
    p.nf = nf;
    p.f1[0] = (uint64_t)f1; p.f1[1] = (uint64_t)(f1 >> 64);
    p.f2[0] = (uint64_t)f2; p.f2[1] = (uint64_t)(f2 >> 64);
    parts_of(J)[blockIdx.x] = p;
  }
}

// 3. iterate: the exact clip (one workgroup per block).
template <bool kBatch>
__global__ __launch_bounds__(kIterThreads) void clip_iter_kernel(ClipJob job0, const ClipJob* jobs) {
  const ClipJob J = job_of<kBatch>(job0, jobs, blockIdx.x);
  __shared__ Red3<kIterThreads> red;
  __shared__ RedSplit<kIterThreads> reds;
  __shared__ int64_t near[kNearMax];
  __shared__ int64_t sT;
  __shared__ double sfit[3];
  const int64_t ncell = (int64_t)J.nsub * J.nchan;
  Ctrl* ct = ctrl_of(J);
  // totals and the sums above the band, from the scan's partials
  int64_t Nt = 0, Nf = 0;
  u128 Q1t = 0, Q2t = 0, F1 = 0, F2 = 0;
  for (int w = threadIdx.x; w < J.nparts; w += kIterThreads) {
    const Part p = parts_of(J)[w];
    Nt += p.n;
    Q1t += mk128(p.q1[0], p.q1[1]);
    Q2t += mk128(p.q2[0], p.q2[1]);
    Nf += p.nf;
    F1 += mk128(p.f1[0], p.f1[1]);
    F2 += mk128(p.f2[0], p.f2[1]);
  }
  block_sum3<kIterThreads>(Nt, Q1t, Q2t, red);
  block_sum3<kIterThreads>(Nf, F1, F2, red);
  const int64_t L = ct->L, H = ct->H;
  const unsigned long long cnt = ct->count;
  const bool complete = cnt <= (unsigned long long)J.tail_cap;
  const int64_t M = complete ? (int64_t)cnt : 0;
  const bool in_lds = M <= kNearMax;
  // every listed q lies in (L, H]: the 64-bit split sums are exact when
  // 0 <= q < 2^42 and at most 2^14 cells are summed
  const bool split = L >= -1 && H < ((int64_t)1 << 42) && kNearMax <= (1 << 14);
  const int64_t* tail = tail_of(J);
  if (complete && in_lds) {
    for (int64_t k0 = 0; k0 < M; k0 += (int64_t)kIterThreads * kIterLoad) {
      int64_t v[kIterLoad];
#pragma unroll
      for (int i = 0; i < kIterLoad; ++i) {
        const int64_t k = k0 + threadIdx.x + (int64_t)i * kIterThreads;
        v[i] = tail[k < M ? k : 0];
      }
#pragma unroll
      for (int i = 0; i < kIterLoad; ++i) {
        const int64_t k = k0 + threadIdx.x + (int64_t)i * kIterThreads;
        if (k < M) near[k] = v[i];
      }
    }
  }
  int64_t Nh = 0;
  u128 Q1h = 0, Q2h = 0;
  if (J.state) {
    Nh = J.state->n;
    Q1h = mk128(J.state->q1[0], J.state->q1[1]);
    Q2h = mk128(J.state->q2[0], J.state->q2[1]);
  }
  if (threadIdx.x == 0) sT = INT64_MAX;
  __syncthreads();

  int64_t prevN = -1, N = 0, Nelig = Nt;
  u128 Q1 = 0, Q2 = 0;
  int it = 0, converged = 1;
  bool last_exact = true;
  int64_t Nl = 0;                        // sums of the last fit (pooled)
  u128 Q1l = 0, Q2l = 0;
  double mu = NAN, sigma = NAN, thr = NAN;
  for (int guard = 0; guard <= J.max_iter + 1; ++guard) {
    __syncthreads();                      // thread 0's update of sT is visible
    const int64_t T = sT;
    __syncthreads();                      // every thread has read T before it changes
    if (T == INT64_MAX) {
      N = Nt; Q1 = Q1t; Q2 = Q2t;
    } else if (complete && T >= L && T <= H) {
      // band cells above T (LDS, or the list itself when it is too long)
      int64_t n = 0;
      u128 a = 0, b = 0;
      if (in_lds && split) {
        SplitSums t{0, 0, 0, 0, 0};
        for (int64_t k = threadIdx.x; k < M; k += kIterThreads) {
          const int64_t q = near[k];
          if (q > T) acc_split(q, t);
        }
        block_sum_split<kIterThreads>(t, n, a, b, reds);
      } else if (in_lds) {
        for (int64_t k = threadIdx.x; k < M; k += kIterThreads) {
          const int64_t q = near[k];
          if (q > T) acc(q, n, a, b);
        }
      } else {
        for (int64_t k0 = 0; k0 < M; k0 += (int64_t)kIterThreads * kIterLoad) {
          int64_t v[kIterLoad];
#pragma unroll
          for (int i = 0; i < kIterLoad; ++i) {
            const int64_t k = k0 + threadIdx.x + (int64_t)i * kIterThreads;
            v[i] = tail[k < M ? k : 0];
          }
#pragma unroll
          for (int i = 0; i < kIterLoad; ++i) {
            const int64_t k = k0 + threadIdx.x + (int64_t)i * kIterThreads;
            if (k < M && v[i] > T) acc(v[i], n, a, b);
          }
        }
      }
      if (!(in_lds && split)) block_sum3<kIterThreads>(n, a, b, red);
      N = Nt - Nf - n; Q1 = Q1t - F1 - a; Q2 = Q2t - F2 - b;
    } else {
      // fallback: a pass over every cell
      int64_t n = 0;
      u128 a = 0, b = 0;
      for (int64_t c = threadIdx.x; c < ncell; c += kIterThreads) {
        const CellLd x = load_cell(J, c, ncell);
        if (!elig(x)) continue;
        const int64_t q = quant(x.s);
        if (q <= T) acc(q, n, a, b);
      }
      block_sum3<kIterThreads>(n, a, b, red);
      N = n; Q1 = a; Q2 = b;
    }
    // decision (uniform: every thread holds the same N, prevN, it)
    if (it > 0 && N == prevN) break;      // the last fit masked nothing new
    if (it > 0 && it >= J.max_iter) {     // capped while still masking
      converged = 0;
      break;
    }
    if (N + Nh == 0) break;               // nothing left to fit
    Nl = N + Nh; Q1l = Q1 + Q1h; Q2l = Q2 + Q2h;
    bool ok;
    int64_t Tn = fit_T_fast(Nl, Q1l, Q2l, J.kappa, ok);
    last_exact = !ok;
    if (!ok) {
      if (threadIdx.x < 64) {
        double m_, s_, t_;
        fit_wave(Nl, Q1l, Q2l, J.kappa, m_, s_, t_);
        if (threadIdx.x == 0) { sfit[0] = m_; sfit[1] = s_; sfit[2] = t_; }
      }
      __syncthreads();
      mu = sfit[0]; sigma = sfit[1]; thr = sfit[2];
      Tn = thr_to_T(thr);
    }
    if (threadIdx.x == 0 && Tn < sT) sT = Tn;
    ++it;
    prevN = N;
  }
  if (it > 0 && !last_exact) {            // the reported fit is the exact one
    if (threadIdx.x < 64) {
      double m_, s_, t_;
      fit_wave(Nl, Q1l, Q2l, J.kappa, m_, s_, t_);
      if (threadIdx.x == 0) { sfit[0] = m_; sfit[1] = s_; sfit[2] = t_; }
    }
    __syncthreads();
    mu = sfit[0]; sigma = sfit[1]; thr = sfit[2];
  }
  if (threadIdx.x == 0) {
    ct->T = sT;
    if (J.out) {
      J.out->mu = mu;
      J.out->sigma = sigma;
      J.out->thr = thr;
      J.out->iterations = it;
      J.out->converged = converged;
      J.out->nflag = Nelig - N;
      J.out->nfit = N;
    }
    if (J.state) {
      const u128 a = Q1h + Q1, b = Q2h + Q2;
      J.state->n = Nh + N;
      J.state->q1[0] = (uint64_t)a;
      J.state->q1[1] = (uint64_t)(a >> 64);
      J.state->q2[0] = (uint64_t)b;
      J.state->q2[1] = (uint64_t)(b >> 64);
      rfi_hist_entry& h = J.state->hist[J.state->nblocks % RFI_HIST_CAP];
      h.mu = mu;
      h.sigma = sigma;
      h.thr = thr;
      h.iterations = it;
      h.converged = converged;
      J.state->nblocks += 1;
    }
  }
}

// 4. mask = eligible and q > T.
template <bool kBatch>
__global__ __launch_bounds__(kGridThreads) void clip_mask_kernel(ClipJob job0, const ClipJob* jobs) {
  const ClipJob J = job_of<kBatch>(job0, jobs, blockIdx.y);
  const int64_t ncell = (int64_t)J.nsub * J.nchan;
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  if (c0 >= ncell) return;
  const int64_t T = ctrl_of(J)->T;
  CellLd x[kChunkPer];
#pragma unroll
  for (int i = 0; i < kChunkPer; ++i) x[i] = load_cell(J, c0 + i * kGridThreads + threadIdx.x, ncell);
#pragma unroll
  for (int i = 0; i < kChunkPer; ++i) {
    const int64_t c = c0 + i * kGridThreads + threadIdx.x;
    if (c < ncell) J.mask[c] = (elig(x[i]) && quant(x[i].s) > T) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Clip scopes (Sec. 3.3: outliers are masked as a function of frequency and
// time): one workgroup clips one segment of cells -- a channel over its
// sub-intervals, a sub-interval over its channels, or the whole block -- with
// the same exact iteration, re-reading its cells every pass; the masks of the
// requested scopes are OR-ed into one. The fit is the exact moment fit, or the
// histogram Gaussian fit: 64 bins of width sigma_m / 8 over +-4 sigma_m of
// the exact moment fit, a least-squares parabola through the log counts with
// weights c^2 (one thread, bins in index order, the operation order of the
// definition, no fused multiply-add), falling back to the moments where the
// parabola is undefined.
constexpr int kSegThreads = 256;      // channel and sub-interval segments
constexpr int kSegThreadsAll = 1024;  // the whole block as one segment
constexpr int kSegUnroll = 4;         // cells per thread whose loads are issued together
constexpr int kBins = 64;

struct SegArgs {
  int nsub, nchan, max_iter, fit;
  double kappa;
  const double* stat;
  const uint8_t* status;
  const uint8_t* protect;
  uint8_t* mask;
  rfi_flag_stats* out;   // [segments] or NULL
  int write;             // 1: store the mask, 0: OR it in
};

// the segment's i-th cell (MODE 0: channel blockIdx.x over sub-intervals;
// 1: sub-interval blockIdx.x over channels; 2: every cell)
template <int MODE>
__device__ __forceinline__ int64_t seg_cell(const SegArgs& a, int64_t i) {
  if constexpr (MODE == 0) return i * a.nchan + blockIdx.x;
  else if constexpr (MODE == 1) return (int64_t)blockIdx.x * a.nchan + i;
  else return i;
}

// mu, sigma of the histogram fit (thread 0; cnt: the 64 bin counts)
__device__ void hist_fit(const unsigned* cnt, int64_t N, double mu_m, double sg_m, double& mu,
                         double& sg) {
#pragma clang fp contract(off)
  mu = mu_m;
  sg = sg_m;
  if (N < 8 || !(sg_m > 0.0)) return;
  int nz = 0;
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
  for (int i = 0; i < kBins; ++i) {
    const unsigned c = cnt[i];
    if (c == 0) continue;
    ++nz;
    const double z = ((double)i + 0.5) * 0.125 - 4.0;
    const double y = log((double)c);
    const double wt = (double)c * (double)c;
    const double z2 = z * z;
    S0 += wt;
    S1 += wt * z;
    S2 += wt * z2;
    S3 += wt * (z2 * z);
    S4 += wt * (z2 * z2);
    T0 += wt * y;
    T1 += wt * (z * y);
    T2 += wt * (z2 * y);
  }
  if (nz < 3) return;
  const double m0 = S2 * S4 - S3 * S3;
  const double m1 = S1 * S4 - S3 * S2;
  const double m2 = S1 * S3 - S2 * S2;
  const double det = S0 * m0 - S1 * m1 + S2 * m2;
  if (!(det != 0.0)) return;
  const double db = S0 * (T1 * S4 - S3 * T2) - T0 * m1 + S2 * (S1 * T2 - T1 * S2);
  const double dc = S0 * (S2 * T2 - T1 * S3) - S1 * (S1 * T2 - T1 * S2) + T0 * m2;
  const double b = db / det;
  const double c2 = dc / det;
  if (!(c2 < 0.0)) return;
  const double mu_z = -b / (2.0 * c2);
  const double sg_z = sqrt(-1.0 / (2.0 * c2));
  mu = mu_m + mu_z * sg_m;
  sg = sg_z * sg_m;
}

template <int MODE, int NT>
__global__ __launch_bounds__(NT) void segclip_kernel(SegArgs a) {
  __shared__ Red3<NT> red;
  __shared__ unsigned hcnt[kBins];
  __shared__ int64_t sT;
  __shared__ double sfit[3];
  const int64_t m = MODE == 0 ? a.nsub : (MODE == 1 ? a.nchan : (int64_t)a.nsub * a.nchan);
  const ClipJob J{a.nsub, a.nchan, a.max_iter, 0, a.kappa, a.stat, a.status, a.protect,
                  nullptr, a.mask, nullptr, nullptr, 0};
  const int64_t ncell = (int64_t)a.nsub * a.nchan;
  if (threadIdx.x == 0) sT = INT64_MAX;
  int64_t prevN = -1, N = 0, Nelig = -1;
  u128 Q1 = 0, Q2 = 0;
  int it = 0, converged = 1;
  bool last_exact = true;
  int64_t Nl = 0;                        // sums of the last fit
  u128 Q1l = 0, Q2l = 0;
  double mu = NAN, sigma = NAN, thr = NAN;
  for (int guard = 0; guard <= a.max_iter + 1; ++guard) {
    __syncthreads();
    const int64_t T = sT;
    __syncthreads();
    int64_t n = 0;
    u128 q1 = 0, q2 = 0;
    for (int64_t i0 = threadIdx.x; i0 < m; i0 += (int64_t)NT * kSegUnroll) {
      CellLd x[kSegUnroll];
#pragma unroll
      for (int u = 0; u < kSegUnroll; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        x[u] = load_cell(J, seg_cell<MODE>(a, i < m ? i : 0), ncell);
      }
#pragma unroll
      for (int u = 0; u < kSegUnroll; ++u) {
        if (i0 + (int64_t)u * NT >= m || !elig(x[u])) continue;
        const int64_t q = quant(x[u].s);
        if (q <= T) acc(q, n, q1, q2);
      }
    }
    block_sum3<NT>(n, q1, q2, red);
    N = n; Q1 = q1; Q2 = q2;
    if (Nelig < 0) Nelig = N;
    if (it > 0 && N == prevN) break;
    if (it > 0 && it >= a.max_iter) { converged = 0; break; }
    if (N == 0) break;
    Nl = N; Q1l = Q1; Q2l = Q2;
    int64_t Tn;
    if (a.fit == 0) {
      bool ok;
      Tn = fit_T_fast(N, Q1, Q2, a.kappa, ok);
      last_exact = !ok;
      if (!ok) {
        if (threadIdx.x < 64) {
          double m_, s_, t_;
          fit_wave(N, Q1, Q2, a.kappa, m_, s_, t_);
          if (threadIdx.x == 0) { sfit[0] = m_; sfit[1] = s_; sfit[2] = t_; }
        }
        __syncthreads();
        mu = sfit[0]; sigma = sfit[1]; thr = sfit[2];
        Tn = thr_to_T(thr);
      }
    } else {
      // histogram fit: exact moments, the 64 bin counts of the live values, the parabola
      if (threadIdx.x < 64) {
        double m_, s_, t_;
        fit_wave(N, Q1, Q2, a.kappa, m_, s_, t_);
        if (threadIdx.x == 0) { sfit[0] = m_; sfit[1] = s_; }
      }
      for (int i = threadIdx.x; i < kBins; i += NT) hcnt[i] = 0;
      __syncthreads();
      const double mu_m = sfit[0], sg_m = sfit[1];
      {
#pragma clang fp contract(off)
        const double lo = mu_m - 4.0 * sg_m;
        const double w = sg_m * 0.125;
        for (int64_t i0 = threadIdx.x; i0 < m; i0 += (int64_t)NT * kSegUnroll) {
          CellLd x[kSegUnroll];
#pragma unroll
          for (int u = 0; u < kSegUnroll; ++u) {
            const int64_t i = i0 + (int64_t)u * NT;
            x[u] = load_cell(J, seg_cell<MODE>(a, i < m ? i : 0), ncell);
          }
#pragma unroll
          for (int u = 0; u < kSegUnroll; ++u) {
            if (i0 + (int64_t)u * NT >= m || !elig(x[u])) continue;
            const int64_t q = quant(x[u].s);
            if (q > T) continue;
            const double v = (double)q / TWO40;
            const double f = floor((v - lo) / w);
            if (f >= 0.0 && f < (double)kBins) atomicAdd(&hcnt[(int)f], 1u);
          }
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        double hm, hs;
        hist_fit(hcnt, N, mu_m, sg_m, hm, hs);
        const double ks = a.kappa * hs;
        sfit[0] = hm; sfit[1] = hs; sfit[2] = hm + ks;
      }
      __syncthreads();
      mu = sfit[0]; sigma = sfit[1]; thr = sfit[2];
      Tn = thr_to_T(thr);
      last_exact = true;
    }
    if (threadIdx.x == 0 && Tn < sT) sT = Tn;
    ++it;
    prevN = N;
  }
  if (a.fit == 0 && it > 0 && !last_exact) {
    // the reported fit is the exact one, from the last fit's sums
    if (threadIdx.x < 64) {
      double m_, s_, t_;
      fit_wave(Nl, Q1l, Q2l, a.kappa, m_, s_, t_);
      if (threadIdx.x == 0) { sfit[0] = m_; sfit[1] = s_; sfit[2] = t_; }
    }
    __syncthreads();
    mu = sfit[0]; sigma = sfit[1]; thr = sfit[2];
  }
  __syncthreads();
  const int64_t T = sT;
  for (int64_t i = threadIdx.x; i < m; i += NT) {
    const int64_t c = seg_cell<MODE>(a, i);
    const CellLd x = load_cell(J, c, ncell);
    const uint8_t hit = (elig(x) && quant(x.s) > T) ? 1 : 0;
    if (a.write) a.mask[c] = hit;
    else if (hit) a.mask[c] = 1;
  }
  if (threadIdx.x == 0 && a.out) {
    rfi_flag_stats& o = a.out[blockIdx.x];
    o.mu = mu;
    o.sigma = sigma;
    o.thr = thr;
    o.iterations = it;
    o.converged = converged;
    o.nflag = (Nelig < 0 ? 0 : Nelig) - N;
    o.nfit = N;
  }
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Exact fit of given moment sums (the clip's arithmetic, for checking it):
// one wavefront per entry.
__global__ __launch_bounds__(256) void fit_kernel(int n, const int64_t* N, const uint64_t* Q1,
                                                  const uint64_t* Q2, double kappa, double* mu,
                                                  double* sigma, double* thr) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;                     // whole wavefronts leave together
  double m = NAN, s = NAN, t = NAN;
  if (N[i] > 0)
    fit_wave(N[i], mk128(Q1[2 * i], Q1[2 * i + 1]), mk128(Q2[2 * i], Q2[2 * i + 1]), kappa, m, s, t);
  if ((threadIdx.x & 63) == 0) {
    mu[i] = m;
    sigma[i] = s;
    thr[i] = t;
  }
}

// Per-beam eigenvector threshold, two launches over (beam, cell range)
// workgroups: (1) each workgroup's (n, sum |v|, sum |v|^2) over the eligible
// unmasked cells of its range, in FP64; (2) every workgroup of a beam sums its
// beam's partials in one fixed order (so all of them get the same fit), forms
// mu, sigma (population) and thr = mu + kappa_v sigma, and writes the beam
// mask of its range. Loads are issued four cells at a time, unconditionally.
constexpr int kVT = 256;                // threads per workgroup
constexpr int kVPer = 4;                // cells per thread and step
constexpr int kVCells = 16384;          // cells per workgroup and beam (at least)
constexpr int kVMaxBlk = 256;           // workgroups per beam (at most)

int eigvec_blocks(int64_t ncell) {
  int64_t nb = (ncell + kVCells - 1) / kVCells;
  return nb < 1 ? 1 : (nb > kVMaxBlk ? kVMaxBlk : (int)nb);
}

__device__ __forceinline__ void eigvec_range(int64_t ncell, int nblk, int blk, int64_t& c0,
                                             int64_t& c1) {
  const int64_t per = (ncell + nblk - 1) / nblk;
  c0 = (int64_t)blk * per;
  c1 = c0 + per < ncell ? c0 + per : ncell;
}

__global__ __launch_bounds__(kVT) void eigvec_stats_kernel(int nsub, int nchan, int nblk,
                                                           const float* __restrict__ v1,
                                                           const uint8_t* __restrict__ mask,
                                                           const uint8_t* __restrict__ status,
                                                           const uint8_t* __restrict__ protect,
                                                           double* __restrict__ part) {
  const int blk = blockIdx.x, b = blockIdx.y;
  const int64_t ncell = (int64_t)nsub * nchan;
  int64_t c0, c1;
  eigvec_range(ncell, nblk, blk, c0, c1);
  const float* vb = v1 + (int64_t)b * ncell;
  double n = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t base = c0 + threadIdx.x; base < c1; base += (int64_t)kVT * kVPer) {
    float v[kVPer];
    uint8_t m[kVPer], st[kVPer], pr[kVPer];
#pragma unroll
    for (int i = 0; i < kVPer; ++i) {
      const int64_t c = base + (int64_t)i * kVT;
      const int64_t cc = c < c1 ? c : c0;
      v[i] = vb[cc];
      m[i] = mask[cc];
      st[i] = status[cc];
      pr[i] = protect ? protect[cc % nchan] : 0;
    }
#pragma unroll
    for (int i = 0; i < kVPer; ++i) {
      const int64_t c = base + (int64_t)i * kVT;
      const bool use = c < c1 && !(st[i] & (RFI_CELL_DEGENERATE | RFI_CELL_BAD_COUNT)) &&
                       !pr[i] && !m[i];
      const double x = fabs((double)v[i]);
      n += use ? 1.0 : 0.0;
      a1 += use ? x : 0.0;
      a2 += use ? x * x : 0.0;
    }
  }
  __shared__ double sh[3][kVT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    n += __shfl_down(n, off);
    a1 += __shfl_down(a1, off);
    a2 += __shfl_down(a2, off);
  }
  if (lane == 0) {
    sh[0][wave] = n;
    sh[1][wave] = a1;
    sh[2][wave] = a2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kVT / 64; ++w) {
      t0 += sh[0][w];
      t1 += sh[1][w];
      t2 += sh[2][w];
    }
    double* o = part + ((int64_t)b * nblk + blk) * 3;
    o[0] = t0;
    o[1] = t1;
    o[2] = t2;
  }
}

__global__ __launch_bounds__(kVT) void eigvec_mask_kernel(int nsub, int nchan, int nblk,
                                                          const float* __restrict__ v1,
                                                          const uint8_t* __restrict__ mask,
                                                          const double* __restrict__ part,
                                                          double kappa_v,
                                                          uint8_t* __restrict__ beam_mask,
                                                          double* beam_mu, double* beam_sigma) {
  const int blk = blockIdx.x, b = blockIdx.y;
  const int64_t ncell = (int64_t)nsub * nchan;
  // the beam's fit from its partials: thread t takes partial t (nblk <= kVT),
  // then a fixed tree, so every workgroup of the beam gets the same bits
  __shared__ double sh[3][kVT];
  const double* pb = part + (int64_t)b * nblk * 3;
  const int t = threadIdx.x;
  sh[0][t] = t < nblk ? pb[3 * t] : 0.0;
  sh[1][t] = t < nblk ? pb[3 * t + 1] : 0.0;
  sh[2][t] = t < nblk ? pb[3 * t + 2] : 0.0;
  __syncthreads();
  for (int h = kVT / 2; h > 0; h >>= 1) {
    if (t < h) {
      sh[0][t] += sh[0][t + h];
      sh[1][t] += sh[1][t + h];
      sh[2][t] += sh[2][t + h];
    }
    __syncthreads();
  }
  const double n = sh[0][0], s1 = sh[1][0], s2 = sh[2][0];
  const double mu = n > 0.0 ? s1 / n : NAN;
  const double var = n > 0.0 ? (s2 - s1 * mu) / n : NAN;
  const double sd = n > 0.0 ? sqrt(var > 0.0 ? var : 0.0) : NAN;
  const double thr = mu + kappa_v * sd;
  if (blk == 0 && t == 0) {
    if (beam_mu) beam_mu[b] = mu;
    if (beam_sigma) beam_sigma[b] = sd;
  }
  int64_t c0, c1;
  eigvec_range(ncell, nblk, blk, c0, c1);
  const float* vb = v1 + (int64_t)b * ncell;
  uint8_t* out = beam_mask + (int64_t)b * ncell;
  for (int64_t c = c0 + t; c < c1; c += kVT)
    out[c] = (mask[c] && fabs((double)vb[c]) > thr) ? 1 : 0;
}

}  // namespace

int64_t clip_tail_cap(int64_t ncell) { return ncell < kTailMax ? (ncell < 1 ? 1 : ncell) : kTailMax; }

size_t clip_workspace_size(int64_t ncell) {
  return kTailOff + (size_t)clip_tail_cap(ncell) * sizeof(int64_t);
}

size_t clip_workspace_size_for_cap(int64_t tail_cap) {
  return kTailOff + (size_t)tail_cap * sizeof(int64_t);
}

ClipJob make_clip_job(int nsub, int nchan, const double* stat, const uint8_t* status,
                      const uint8_t* protect_chan, double kappa, int max_iter,
                      rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out, void* ws,
                      int64_t tail_cap) {
  const int64_t ncell = (int64_t)nsub * nchan;
  const int64_t chunks = (ncell + kChunk - 1) / kChunk;
  ClipJob j{};
  j.nsub = nsub;
  j.nchan = nchan;
  j.max_iter = max_iter;
  j.nparts = (int)(chunks < 1 ? 1 : (chunks > kMaxParts ? kMaxParts : chunks));
  j.kappa = kappa;
  j.stat = stat;
  j.status = status;
  j.protect = protect_chan;
  j.state = state;
  j.mask = mask;
  j.out = out;
  j.ws = ws;
  j.tail_cap = tail_cap > 0 ? tail_cap : clip_tail_cap(ncell);
  return j;
}

hipError_t launch_clip(const ClipJob& j, hipStream_t s) {
  const int64_t ncell = (int64_t)j.nsub * j.nchan;
  const unsigned nmask = (unsigned)((ncell + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(clip_plan_kernel<false>, dim3(1), dim3(kPlanThreads), 0, s, j, nullptr);
  hipLaunchKernelGGL(clip_scan_kernel<false>, dim3((unsigned)j.nparts), dim3(kGridThreads), 0, s,
                     j, nullptr);
  hipLaunchKernelGGL(clip_iter_kernel<false>, dim3(1), dim3(kIterThreads), 0, s, j, nullptr);
  if (nmask > 0)
    hipLaunchKernelGGL(clip_mask_kernel<false>, dim3(nmask), dim3(kGridThreads), 0, s, j, nullptr);
  return hipGetLastError();
}

hipError_t launch_clip_batch(const ClipJob* jobs, const ClipJob* host_jobs, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int maxparts = 1;
  int64_t maxcell = 0;
  for (int i = 0; i < n; ++i) {
    if (host_jobs[i].nparts > maxparts) maxparts = host_jobs[i].nparts;
    const int64_t c = (int64_t)host_jobs[i].nsub * host_jobs[i].nchan;
    if (c > maxcell) maxcell = c;
  }
  const unsigned nmask = (unsigned)((maxcell + kChunk - 1) / kChunk);
  ClipJob none{};
  hipLaunchKernelGGL(clip_plan_kernel<true>, dim3((unsigned)n), dim3(kPlanThreads), 0, s, none, jobs);
  hipLaunchKernelGGL(clip_scan_kernel<true>, dim3((unsigned)maxparts, (unsigned)n),
                     dim3(kGridThreads), 0, s, none, jobs);
  hipLaunchKernelGGL(clip_iter_kernel<true>, dim3((unsigned)n), dim3(kIterThreads), 0, s, none, jobs);
  if (nmask > 0)
    hipLaunchKernelGGL(clip_mask_kernel<true>, dim3(nmask, (unsigned)n), dim3(kGridThreads), 0, s,
                       none, jobs);
  return hipGetLastError();
}

hipError_t launch_clip_scoped(const ClipJob& g, int scopes, int fit, rfi_flag_stats* chan_out,
                              rfi_flag_stats* sub_out, hipStream_t s) {
  const int64_t ncell = (int64_t)g.nsub * g.nchan;
  SegArgs a{g.nsub, g.nchan, g.max_iter, fit, g.kappa, g.stat, g.status, g.protect, g.mask,
            nullptr, 0};
  if (scopes & 1) {
    if (fit == 0) {
      hipError_t e = launch_clip(g, s);
      if (e != hipSuccess) return e;
    } else {
      a.out = g.out;
      a.write = 1;
      hipLaunchKernelGGL((segclip_kernel<2, kSegThreadsAll>), dim3(1), dim3(kSegThreadsAll), 0, s,
                         a);
    }
  } else if (ncell > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>((ncell + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid), dim3(256), 0, s, g.mask, ncell);
  }
  a.write = 0;
  if ((scopes & 2) && g.nsub > 0) {
    a.out = chan_out;
    hipLaunchKernelGGL((segclip_kernel<0, kSegThreads>), dim3((unsigned)g.nchan), dim3(kSegThreads),
                       0, s, a);
  }
  if ((scopes & 4) && g.nsub > 0) {
    a.out = sub_out;
    hipLaunchKernelGGL((segclip_kernel<1, kSegThreads>), dim3((unsigned)g.nsub), dim3(kSegThreads),
                       0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fit(int n, const int64_t* N, const uint64_t* Q1, const uint64_t* Q2,
                      double kappa, double* mu, double* sigma, double* thr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fit_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, N, Q1, Q2,
                     kappa, mu, sigma, thr);
  return hipGetLastError();
}

size_t eigvec_workspace_size(int nbeam, int64_t ncell) {
  return (size_t)nbeam * eigvec_blocks(ncell) * 3 * sizeof(double);
}

hipError_t launch_eigvec_flag(int nbeam, int nsub, int nchan, const float* v1,
                              const uint8_t* mask, const uint8_t* status,
                              const uint8_t* protect_chan, double kappa_v,
                              uint8_t* beam_mask, double* beam_mu, double* beam_sigma, void* ws,
                              hipStream_t s) {
  const int64_t ncell = (int64_t)nsub * nchan;
  const int nblk = eigvec_blocks(ncell);
  double* part = (double*)ws;
  hipLaunchKernelGGL(eigvec_stats_kernel, dim3(nblk, nbeam), dim3(kVT), 0, s, nsub, nchan, nblk,
                     v1, mask, status, protect_chan, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eigvec_mask_kernel, dim3(nblk, nbeam), dim3(kVT), 0, s, nsub, nchan, nblk,
                     v1, mask, (const double*)part, kappa_v, beam_mask, beam_mu, beam_sigma);
  return hipGetLastError();
}

}  // namespace rfi

// ---------------------------------------------------------------------------
// rfi_flag_noalloc: the clip with its workspace in a fixed device array of
// this library, for callers that cannot allocate.
namespace rfi {
namespace {

constexpr int64_t kNoAllocCells = (int64_t)1 << 20;
constexpr size_t kNoAllocBytes = kTailOff + (size_t)kNoAllocCells * sizeof(int64_t);

// One copy per GPU, alive until the process ends. Host code must not pass
// this name to a kernel: it is a host-side stand-in, not a device address;
// the device address comes from hipGetSymbolAddress, per device, below.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDev = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDev] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
hipError_t scratch_for(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace rfi

extern "C" rfi_status rfi_flag_noalloc(int32_t nsub, int32_t nchan, const double* stat,
                                       const uint8_t* status, const uint8_t* protect_chan,
                                       double kappa, int32_t max_iter, rfi_stream_state* state,
                                       uint8_t* mask, rfi_flag_stats* out, rfi_stream_t stream) {
  rfi::clear_error();
  if (nsub < 0 || nchan < 1) return rfi::fail(RFI_E_INVALID, "rfi_flag_noalloc: bad nsub/nchan");
  if ((int64_t)nsub * nchan > rfi::kNoAllocCells)
    return rfi::fail(RFI_E_INVALID,
                     "rfi_flag_noalloc: %lld cells exceed the fixed workspace's %lld "
                     "(use rfi_flag with a caller workspace)",
                     (long long)nsub * nchan, (long long)rfi::kNoAllocCells);
  if (nsub > 0 && (!stat || !status || !mask))
    return rfi::fail(RFI_E_INVALID, "rfi_flag_noalloc: NULL input or output");
  if (!(kappa >= 0.0)) return rfi::fail(RFI_E_INVALID, "rfi_flag_noalloc: kappa must be >= 0");
  if (max_iter < 1) return rfi::fail(RFI_E_INVALID, "rfi_flag_noalloc: max_iter %d < 1", max_iter);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rfi::check_hip(e, "rfi_flag_noalloc: hipGetDevice");
  if (dev < 0 || dev >= rfi::kMaxDev)
    return rfi::fail(RFI_E_DEVICE, "rfi_flag_noalloc: device %d out of range", dev);
  void* ws = nullptr;
  if ((e = rfi::scratch_for(dev, &ws)) != hipSuccess)
    return rfi::check_hip(e, "rfi_flag_noalloc: scratch address");
  const rfi::ClipJob j = rfi::make_clip_job(nsub, nchan, stat, status, protect_chan, kappa,
                                            max_iter, state, mask, out, ws, rfi::kNoAllocCells);
  return rfi::check_hip(rfi::launch_clip(j, (hipStream_t)stream), "rfi_flag_noalloc launch");
}
