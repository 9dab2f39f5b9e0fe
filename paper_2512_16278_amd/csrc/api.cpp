// C ABI entry points of librfi: argument validation and kernel dispatch.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"
#include "rfi.h"

namespace rfi {

namespace {
thread_local std::string g_err;
}

void clear_error() { g_err.clear(); }

rfi_status fail(rfi_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

rfi_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return RFI_OK;
  return fail(RFI_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

rfi_status validate_block(const rfi_block* blk, int64_t t0, int32_t L, int32_t nsub,
                          const char* who, BeamPtrs* bp, int32_t max_L) {
  if (!blk) return fail(RFI_E_INVALID, "%s: blk is NULL", who);
  const int n = blk->nbeam;
  if (n < 2 || n > RFI_MAX_BEAMS)
    return fail(RFI_E_INVALID, "%s: nbeam %d outside 2..%d", who, n, RFI_MAX_BEAMS);
  if (blk->nchan < 1) return fail(RFI_E_INVALID, "%s: nchan %d < 1", who, blk->nchan);
  if (blk->row_stride < blk->nchan || blk->row_stride % 16 != 0)
    return fail(RFI_E_INVALID, "%s: row_stride %lld must be >= nchan and a multiple of 16", who,
                (long long)blk->row_stride);
  if (L < 1) return fail(RFI_E_INVALID, "%s: L %d < 1", who, L);
  if (L > max_L)
    return fail(RFI_E_OVERFLOW, "%s: L %d exceeds the exact bound %d of this path", who, L,
                max_L);
  if (nsub < 0) return fail(RFI_E_INVALID, "%s: nsub %d < 0", who, nsub);
  if (t0 < 0 || t0 + (int64_t)nsub * L > blk->nsamp)
    return fail(RFI_E_INVALID, "%s: samples [%lld, %lld) outside the block of %lld", who,
                (long long)t0, (long long)(t0 + (int64_t)nsub * L), (long long)blk->nsamp);
  if ((int64_t)nsub * blk->nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "%s: nsub * nchan exceeds 2^30 cells", who);
  std::memset(bp, 0, sizeof(*bp));
  for (int b = 0; b < n; ++b) {
    if (!blk->beam[b]) return fail(RFI_E_INVALID, "%s: beam %d is NULL", who, b);
    if (((uintptr_t)blk->beam[b]) % 16 != 0)
      return fail(RFI_E_INVALID, "%s: beam %d not 16-byte aligned", who, b);
    bp->p[b] = blk->beam[b];
  }
  return RFI_OK;
}

rfi_status resolve_eig(int nbeam, const rfi_eig_params* p, rfi_eig_params* out,
                       const char* who) {
  rfi_eig_params prm{32, 12, 1, RFI_EIG_AUTO};
  if (p) prm = *p;
  if (prm.precision != 32 && prm.precision != 64)
    return fail(RFI_E_INVALID, "%s: precision %d not 32 or 64", who, prm.precision);
  if (prm.max_sweeps < 1 || prm.max_sweeps > 30)
    return fail(RFI_E_INVALID, "%s: max_sweeps %d outside 1..30", who, prm.max_sweeps);
  if (prm.solver == RFI_EIG_AUTO)
    prm.solver = prm.precision == 64 ? RFI_EIG_WAVE
                                     : (nbeam <= 20 ? RFI_EIG_LANE_TRI : RFI_EIG_TRIDIAG);
  if ((prm.solver == RFI_EIG_LANE || prm.solver == RFI_EIG_LANE_TRI) &&
      (prm.precision != 32 || nbeam > 20))
    return fail(RFI_E_INVALID, "%s: the per-lane solvers are FP32 and nbeam <= 20", who);
  if (prm.solver != RFI_EIG_LANE && prm.solver != RFI_EIG_WAVE &&
      prm.solver != RFI_EIG_TRIDIAG && prm.solver != RFI_EIG_LANE_TRI)
    return fail(RFI_E_INVALID, "%s: unknown solver %d", who, prm.solver);
  *out = prm;
  return RFI_OK;
}

hipError_t launch_eig(const EigArgs& a, const rfi_eig_params& p, hipStream_t s, int lane_wg) {
  switch (p.solver) {
    case RFI_EIG_LANE: return launch_eig_lane(a, s, lane_wg);
    case RFI_EIG_LANE_TRI: return launch_eig_lane(a, s, lane_wg, true);
    case RFI_EIG_TRIDIAG: return launch_eig_tri(a, s);
    default: return launch_eig_wave(a, p.precision, s);
  }
}

}  // namespace rfi

using rfi::check_hip;
using rfi::fail;

extern "C" {

const char* rfi_last_error(void) { return rfi::g_err.c_str(); }

const char* rfi_version(void) { return "librfi 0.1 (gfx950)"; }

rfi_status rfi_ccm_accumulate(const rfi_block* blk, int64_t t0, int32_t L, int32_t nsub,
                              int32_t* sum_x, int32_t* sum_xy, int32_t* count,
                              int32_t accumulate, int32_t variant, rfi_stream_t stream) {
  rfi::clear_error();
  rfi::BeamPtrs bp;
  const rfi_status st = rfi::validate_block(blk, t0, L, nsub, "rfi_ccm_accumulate", &bp);
  if (st != RFI_OK) return st;
  const int n = blk->nbeam;
  if (!sum_x || !sum_xy || !count)
    return fail(RFI_E_INVALID, "rfi_ccm_accumulate: NULL output");
  if (nsub == 0) return RFI_OK;
  int v = variant;
  if (v == RFI_CCM_AUTO) v = RFI_CCM_MFMA;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (v == RFI_CCM_MFMA) {
    e = rfi::launch_ccm_mfma(bp, n, blk->nchan, blk->row_stride, t0, L, nsub, sum_x, sum_xy,
                             count, accumulate ? 1 : 0, 0, s);
  } else if (v == RFI_CCM_VALU) {
    if (n > 20) return fail(RFI_E_INVALID, "rfi_ccm_accumulate: VALU variant needs nbeam <= 20");
    e = rfi::launch_ccm_valu(bp, n, blk->nchan, blk->row_stride, t0, L, nsub, sum_x, sum_xy,
                             count, accumulate ? 1 : 0, s);
  } else {
    return fail(RFI_E_INVALID, "rfi_ccm_accumulate: unknown variant %d", variant);
  }
  return check_hip(e, "rfi_ccm_accumulate launch");
}

int32_t rfi_ccm_tile_variants(int32_t nbeam) {
  return nbeam < 2 || nbeam > RFI_MAX_BEAMS ? 0 : rfi::ccm_tile_variants(nbeam);
}

rfi_status rfi_eig_batched(int32_t nbeam, int32_t nsub, int32_t nchan, const int32_t* sum_x,
                           const int32_t* sum_xy, const int32_t* count, const rfi_eig_params* p,
                           float* eigvals, double* stat, float* v1, uint8_t* status,
                           rfi_stream_t stream) {
  rfi::clear_error();
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS)
    return fail(RFI_E_INVALID, "rfi_eig_batched: nbeam %d outside 2..%d", nbeam, RFI_MAX_BEAMS);
  if (nsub < 0 || nchan < 1) return fail(RFI_E_INVALID, "rfi_eig_batched: bad nsub/nchan");
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "rfi_eig_batched: nsub * nchan exceeds 2^30 cells");
  if (!sum_x || !sum_xy || !count || !stat || !status)
    return fail(RFI_E_INVALID, "rfi_eig_batched: NULL input or output");
  rfi_eig_params prm;
  const rfi_status st = rfi::resolve_eig(nbeam, p, &prm, "rfi_eig_batched");
  if (st != RFI_OK) return st;
  if (nsub == 0) return RFI_OK;
  rfi::EigArgs a{nbeam, nsub, nchan, sum_x, sum_xy, count, prm.max_sweeps, prm.refine ? 1 : 0,
                 eigvals, stat, v1, status, (int64_t)nsub * nchan};
  hipStream_t s = (hipStream_t)stream;
  return check_hip(rfi::launch_eig(a, prm, s, 256), "rfi_eig_batched launch");
}

size_t rfi_ccm_long_workspace_size(int32_t nbeam, int32_t nchan, int32_t nsub) {
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nchan < 1 || nsub < 0) return 0;
  return rfi::ccm_long_tmp_bytes(nbeam, nchan, nsub);
}

rfi_status rfi_ccm_accumulate_long(const rfi_block* blk, int64_t t0, int32_t L, int32_t nsub,
                                   int64_t* sums, int32_t* count, void* workspace,
                                   rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_ccm_accumulate_long";
  rfi::BeamPtrs bp;
  const rfi_status st = rfi::validate_block(blk, t0, L, nsub, who, &bp, RFI_MAX_COUNT_LONG);
  if (st != RFI_OK) return st;
  if (nsub == 0) return RFI_OK;
  if (!sums || !count) return fail(RFI_E_INVALID, "%s: NULL output", who);
  if (!workspace || (uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "%s: workspace NULL or not 256-byte aligned", who);
  return check_hip(rfi::launch_ccm_long(bp, blk->nbeam, blk->nchan, blk->row_stride, t0, L, nsub,
                                        sums, count, workspace, (hipStream_t)stream),
                   "rfi_ccm_accumulate_long launch");
}

rfi_status rfi_eig_batched_long(int32_t nbeam, int32_t nsub, int32_t nchan, const int64_t* sums,
                                const int32_t* count, float* eigvals, double* stat, float* v1,
                                uint8_t* status, rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_eig_batched_long";
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS)
    return fail(RFI_E_INVALID, "%s: nbeam %d outside 2..%d", who, nbeam, RFI_MAX_BEAMS);
  if (nsub < 0 || nchan < 1) return fail(RFI_E_INVALID, "%s: bad nsub/nchan", who);
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "%s: nsub * nchan exceeds 2^30 cells", who);
  if (nsub == 0) return RFI_OK;
  if (!sums || !count || !stat || !status) return fail(RFI_E_INVALID, "%s: NULL input or output", who);
  rfi::EigArgs a{nbeam, nsub, nchan, (const int32_t*)sums, nullptr, count, 12, 1,
                 eigvals, stat, v1, status, (int64_t)nsub * nchan, 2};
  return check_hip(rfi::launch_eig_tri(a, (hipStream_t)stream), "rfi_eig_batched_long launch");
}

size_t rfi_bandpass_workspace_size(int32_t nbeam, int32_t nchan, int32_t nsub) {
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nchan < 1 || nsub < 0) return 0;
  return rfi::bandpass_workspace_size(nbeam, nchan, nsub);
}

rfi_status rfi_bandpass_arpls(int32_t nbeam, int32_t nsub, int32_t nchan, const int32_t* sum_x,
                              const int32_t* count, double lam, double ratio, int32_t itermax,
                              double* z, int32_t* passes, void* workspace, rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_bandpass_arpls";
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nsub < 0 || nchan < 1)
    return fail(RFI_E_INVALID, "%s: bad sizes", who);
  if ((int64_t)nsub * nchan > (int64_t)1 << 30 || (int64_t)nsub * nbeam > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "%s: nsub * nchan or nsub * nbeam exceeds 2^30", who);
  if (!(lam > 0.0) || !(ratio >= 0.0) || itermax < 1)
    return fail(RFI_E_INVALID, "%s: lam must be > 0, ratio >= 0, itermax >= 1", who);
  if (nsub == 0) return RFI_OK;
  if (!sum_x || !count || !z || !workspace)
    return fail(RFI_E_INVALID, "%s: NULL input, output or workspace", who);
  return check_hip(rfi::launch_arpls(nbeam, nsub, nchan, sum_x, count, lam, ratio, itermax, z,
                                     passes, workspace, (hipStream_t)stream),
                   "rfi_bandpass_arpls launch");
}

rfi_status rfi_eig_noncentred(int32_t nbeam, int32_t nsub, int32_t nchan, const int32_t* sum_x,
                              const int32_t* sum_xy, const int32_t* count, const double* z,
                              float* eigvals, double* stat, float* v1, uint8_t* status,
                              rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_eig_noncentred";
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS)
    return fail(RFI_E_INVALID, "%s: nbeam %d outside 2..%d", who, nbeam, RFI_MAX_BEAMS);
  if (nsub < 0 || nchan < 1) return fail(RFI_E_INVALID, "%s: bad nsub/nchan", who);
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "%s: nsub * nchan exceeds 2^30 cells", who);
  if (nsub == 0) return RFI_OK;
  if (!sum_x || !sum_xy || !count || !stat || !status)
    return fail(RFI_E_INVALID, "%s: NULL input or output", who);
  rfi::EigArgs a{nbeam, nsub, nchan, sum_x, sum_xy, count, 12, 1, eigvals, stat, v1, status,
                 (int64_t)nsub * nchan, 0};
  return check_hip(rfi::launch_eig_tri_nc(a, z, (hipStream_t)stream), "rfi_eig_noncentred launch");
}

rfi_status rfi_beam_offsets(int32_t nbeam, int64_t nsamp, int64_t row_stride, int64_t* offsets,
                            int64_t* total) {
  rfi::clear_error();
  if (nbeam < 1 || nbeam > RFI_MAX_BEAMS || nsamp < 0 || row_stride < 1 || row_stride % 16 ||
      !offsets || !total)
    return fail(RFI_E_INVALID, "rfi_beam_offsets: bad arguments");
  constexpr int64_t kPage = 4096, kStep = 64;
  const int64_t lim = (int64_t)1 << 62;
  if (nsamp > lim / row_stride) return fail(RFI_E_OVERFLOW, "rfi_beam_offsets: beam too large");
  const int64_t bytes = nsamp * row_stride;
  // a beam plus the largest stagger (63 steps) fits in its pitch
  const int64_t pitch = (bytes + kPage - 1) / kPage * kPage + kPage;
  if (pitch > lim / nbeam) return fail(RFI_E_OVERFLOW, "rfi_beam_offsets: block too large");
  for (int b = 0; b < nbeam; ++b) offsets[b] = b * pitch + kStep * (b % 64);
  *total = offsets[nbeam - 1] + bytes;
  return RFI_OK;
}

size_t rfi_flag_workspace_size(int32_t nsub, int32_t nchan) {
  if (nsub < 0 || nchan < 1) return 0;
  return rfi::clip_workspace_size((int64_t)nsub * nchan);
}

rfi_status rfi_flag(int32_t nsub, int32_t nchan, const double* stat, const uint8_t* status,
                    const uint8_t* protect_chan, double kappa, int32_t max_iter,
                    rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out,
                    void* workspace, rfi_stream_t stream) {
  rfi::clear_error();
  if (nsub < 0 || nchan < 1) return fail(RFI_E_INVALID, "rfi_flag: bad nsub/nchan");
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "rfi_flag: nsub * nchan exceeds 2^30 cells");
  if (nsub > 0 && (!stat || !status || !mask))
    return fail(RFI_E_INVALID, "rfi_flag: NULL input or output");
  if (!(kappa >= 0.0)) return fail(RFI_E_INVALID, "rfi_flag: kappa must be >= 0");
  if (max_iter < 1) return fail(RFI_E_INVALID, "rfi_flag: max_iter %d < 1", max_iter);
  if (!workspace) return fail(RFI_E_INVALID, "rfi_flag: workspace is NULL");
  if ((uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "rfi_flag: workspace not 256-byte aligned");
  const rfi::ClipJob j = rfi::make_clip_job(nsub, nchan, stat, status, protect_chan, kappa,
                                            max_iter, state, mask, out, workspace);
  return check_hip(rfi::launch_clip(j, (hipStream_t)stream), "rfi_flag launch");
}

rfi_status rfi_flag_scoped(int32_t nsub, int32_t nchan, const double* stat, const uint8_t* status,
                           const uint8_t* protect_chan, double kappa, int32_t max_iter,
                           int32_t scopes, int32_t fit, uint8_t* mask, rfi_flag_stats* out,
                           rfi_flag_stats* chan_out, rfi_flag_stats* sub_out, void* workspace,
                           rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_flag_scoped";
  if (nsub < 0 || nchan < 1) return fail(RFI_E_INVALID, "%s: bad nsub/nchan", who);
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "%s: nsub * nchan exceeds 2^30 cells", who);
  if (nsub > 0 && (!stat || !status || !mask))
    return fail(RFI_E_INVALID, "%s: NULL input or output", who);
  if (!(kappa >= 0.0)) return fail(RFI_E_INVALID, "%s: kappa must be >= 0", who);
  if (max_iter < 1) return fail(RFI_E_INVALID, "%s: max_iter %d < 1", who, max_iter);
  if (scopes < 1 || scopes > 7) return fail(RFI_E_INVALID, "%s: scopes %d not in 1..7", who, scopes);
  if (fit != RFI_FIT_MOMENTS && fit != RFI_FIT_HISTOGRAM)
    return fail(RFI_E_INVALID, "%s: unknown fit %d", who, fit);
  if ((scopes & RFI_SCOPE_GLOBAL) && fit == RFI_FIT_MOMENTS &&
      (!workspace || (uintptr_t)workspace % 256 != 0))
    return fail(RFI_E_INVALID, "%s: workspace NULL or not 256-byte aligned", who);
  const rfi::ClipJob j = rfi::make_clip_job(nsub, nchan, stat, status, protect_chan, kappa,
                                            max_iter, nullptr, mask, out, workspace);
  return check_hip(rfi::launch_clip_scoped(j, scopes, fit, chan_out, sub_out, (hipStream_t)stream),
                   "rfi_flag_scoped launch");
}

rfi_status rfi_clip_fit(int32_t n, const int64_t* N, const uint64_t* Q1, const uint64_t* Q2,
                        double kappa, double* mu, double* sigma, double* thr,
                        rfi_stream_t stream) {
  rfi::clear_error();
  if (n < 0) return fail(RFI_E_INVALID, "rfi_clip_fit: n %d < 0", n);
  if (n > 0 && (!N || !Q1 || !Q2 || !mu || !sigma || !thr))
    return fail(RFI_E_INVALID, "rfi_clip_fit: NULL array");
  if (!(kappa >= 0.0)) return fail(RFI_E_INVALID, "rfi_clip_fit: kappa must be >= 0");
  return check_hip(rfi::launch_fit(n, N, Q1, Q2, kappa, mu, sigma, thr, (hipStream_t)stream),
                   "rfi_clip_fit launch");
}

size_t rfi_eigvec_workspace_size(int32_t nbeam, int32_t nsub, int32_t nchan) {
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nsub < 0 || nchan < 1) return 0;
  return rfi::eigvec_workspace_size(nbeam, (int64_t)nsub * nchan);
}

rfi_status rfi_eigvec_flag(int32_t nbeam, int32_t nsub, int32_t nchan, const float* v1,
                           const uint8_t* mask, const uint8_t* status,
                           const uint8_t* protect_chan, double kappa_v, uint8_t* beam_mask,
                           double* beam_mu, double* beam_sigma, void* workspace,
                           rfi_stream_t stream) {
  rfi::clear_error();
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nsub < 0 || nchan < 1)
    return fail(RFI_E_INVALID, "rfi_eigvec_flag: bad sizes");
  if ((int64_t)nsub * nchan > (int64_t)1 << 30)
    return fail(RFI_E_INVALID, "rfi_eigvec_flag: nsub * nchan exceeds 2^30 cells");
  if (!v1 || !mask || !status || !beam_mask)
    return fail(RFI_E_INVALID, "rfi_eigvec_flag: NULL input or output");
  if (!workspace) return fail(RFI_E_INVALID, "rfi_eigvec_flag: workspace is NULL");
  if ((uintptr_t)workspace % 8 != 0)
    return fail(RFI_E_INVALID, "rfi_eigvec_flag: workspace not 8-byte aligned");
  if (!(kappa_v >= 0.0)) return fail(RFI_E_INVALID, "rfi_eigvec_flag: kappa_v must be >= 0");
  return check_hip(rfi::launch_eigvec_flag(nbeam, nsub, nchan, v1, mask, status, protect_chan,
                                           kappa_v, beam_mask, beam_mu, beam_sigma, workspace,
                                           (hipStream_t)stream),
                   "rfi_eigvec_flag launch");
}

}  // extern "C"
