// Whole-block path: sums (Eq. 1) -> eigen stage and statistic (Eq. 2) -> clip,
// with sub-interval groups pipelined over two HIP streams.
//
// The sums of a group go to one slot of a ring of kRing slots in the
// caller's workspace. On the caller's stream the CCM kernel fills slot
// g % kRing (after the eigen stage of group g - kRing has released it); on
// the helper stream the eigen stage of group g waits for that CCM and writes
// the group's rows of stat / status / eigvals / v1.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "pipeline.h"
#include "rfi.h"

namespace rfi {

namespace {

constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t slot_bytes(int nbeam, int nchan, int group, bool longL = false);

// Sub-intervals per group when the caller leaves it to the library: the whole
// block while its sums fit in kAutoSums bytes, else the largest group whose
// ring of kRing slots does. Running the eigen stage of one group beside the
// sums of the next measured slower on gfx950 than running the two stages one
// after the other over the whole block (both are then limited by the same
// vector ALU issue), so groups serve to bound the workspace, not to overlap.
constexpr size_t kAutoSums = (size_t)1 << 30;
int auto_group(int nbeam, int nchan, int nsub, bool longL) {
  if (nsub <= 1) return 1;
  if (slot_bytes(nbeam, nchan, nsub, longL) <= kAutoSums) return nsub;
  int g = (int)(kAutoSums / kRing / slot_bytes(nbeam, nchan, 1, longL));
  return g < 1 ? 1 : (g > nsub ? nsub : g);
}

size_t slot_bytes(int nbeam, int nchan, int group, bool longL) {
  const size_t cells = (size_t)group * nchan;
  if (longL)   // int64 records, the int32 chunk scratch, counts
    return up(cells * (nbeam + npair_of(nbeam)) * 8) + up(ccm_long_tmp_bytes(nbeam, nchan, group)) +
           up((size_t)group * 4);
  return up(cells * nbeam * 4) + up(cells * npair_of(nbeam) * 4) + up((size_t)group * 4);
}

}  // namespace

rfi_status resolve_process(int nbeam, int nchan, const rfi_process_params* p, ProcessPlan* pl,
                           const char* who, const rfi_tune_entry* te) {
  if (!p) return fail(RFI_E_INVALID, "%s: params is NULL", who);
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nchan < 1)
    return fail(RFI_E_INVALID, "%s: bad nbeam %d / nchan %d", who, nbeam, nchan);
  if (p->group < 0) return fail(RFI_E_INVALID, "%s: group %d < 0", who, p->group);
  if (p->nsub < 0) return fail(RFI_E_INVALID, "%s: nsub %d < 0", who, p->nsub);
  if (!(p->kappa >= 0.0)) return fail(RFI_E_INVALID, "%s: kappa must be >= 0", who);
  if (p->max_iter < 0) return fail(RFI_E_INVALID, "%s: max_iter %d < 0", who, p->max_iter);
  rfi_status st = check_tune_entry(te, nbeam, who);
  if (st != RFI_OK) return st;
  rfi_eig_params ep{p->eig_precision ? p->eig_precision : 32,
                    p->max_sweeps ? p->max_sweeps : 12, 1, te ? te->eig_solver : RFI_EIG_AUTO};
  if ((st = resolve_eig(nbeam, &ep, &pl->eig, who)) != RFI_OK) return st;
  pl->L = p->L;
  pl->longL = p->L > RFI_MAX_COUNT;
  // long sub-intervals: the FP64 tridiagonal solver on the int64 sums (their
  // cells read n L > 66,050 bytes each: the eigen stage is never the bound)
  if (pl->longL) pl->eig.solver = RFI_EIG_TRIDIAG;
  pl->ct = te ? CcmTune{te->ccm_tile, te->ccm_stages, te->ccm_group_bytes} : CcmTune{};
  pl->eig_wg = te ? te->eig_wg : 0;
  pl->nbeam = nbeam;
  pl->nchan = nchan;
  pl->nsub = p->nsub;
  pl->group = p->group ? (p->group < p->nsub ? p->group : (p->nsub < 1 ? 1 : p->nsub))
                       : auto_group(nbeam, nchan, p->nsub, pl->longL);
  pl->max_iter = p->max_iter ? p->max_iter : 50;
  pl->kappa = p->kappa;
  pl->flag_ws = up(clip_workspace_size((int64_t)p->nsub * nchan));
  pl->slot = slot_bytes(nbeam, nchan, pl->group, pl->longL);
  const int ngroup = (p->nsub + pl->group - 1) / pl->group;
  pl->nslot = ngroup < kRing ? (ngroup < 1 ? 1 : ngroup) : kRing;
  pl->ws_bytes = pl->flag_ws + (size_t)pl->nslot * pl->slot;
  return RFI_OK;
}

hipError_t PipeEvents::init() {
  if (ready) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  for (int i = 0; i < kRing; ++i) {
    if ((e = hipEventCreateWithFlags(&ccm[i], hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&eig[i], hipEventDisableTiming)) != hipSuccess) return e;
  }
  if ((e = hipEventCreateWithFlags(&start, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) return e;
  ready = true;
  return hipSuccess;
}

void PipeEvents::destroy() {
  if (!ready) return;
  for (int i = 0; i < kRing; ++i) {
    (void)hipEventDestroy(ccm[i]);
    (void)hipEventDestroy(eig[i]);
  }
  (void)hipEventDestroy(start);
  (void)hipEventDestroy(done);
  (void)hipStreamDestroy(aux);
  ready = false;
}

hipError_t enqueue_eig_groups(const BeamPtrs& bp, int64_t row_stride, int64_t t0, int L,
                              const ProcessPlan& pl, double* stat, uint8_t* status,
                              float* eigvals, float* v1, int64_t out_stride, void* ring,
                              PipeEvents& ev, hipStream_t s) {
  if (pl.nsub == 0) return hipSuccess;
  hipError_t e;
  if ((e = hipEventRecord(ev.start, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ev.aux, ev.start, 0)) != hipSuccess) return e;
  const int ngroup = (pl.nsub + pl.group - 1) / pl.group;
  const size_t cells_cap = (size_t)pl.group * pl.nchan;
  for (int g = 0; g < ngroup; ++g) {
    const int slot = g % pl.nslot;
    const int k0 = g * pl.group;
    const int ks = pl.nsub - k0 < pl.group ? pl.nsub - k0 : pl.group;
    char* base = (char*)ring + (size_t)slot * pl.slot;
    const int64_t off = (int64_t)k0 * pl.nchan;
    if (pl.longL) {
      // the slot is free once the eigen stage of its previous group has run
      if (g >= pl.nslot && (e = hipStreamWaitEvent(s, ev.eig[slot], 0)) != hipSuccess) return e;
      const int nrow = pl.nbeam + npair_of(pl.nbeam);
      int64_t* rec = (int64_t*)base;
      char* tmp = base + up(cells_cap * nrow * 8);
      int32_t* cnt = (int32_t*)(tmp + up(ccm_long_tmp_bytes(pl.nbeam, pl.nchan, pl.group)));
      e = launch_ccm_long(bp, pl.nbeam, pl.nchan, row_stride, t0 + (int64_t)k0 * L, L, ks, rec,
                          cnt, tmp, s, &pl.ct);
      if (e != hipSuccess) return e;
      if ((e = hipEventRecord(ev.ccm[slot], s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(ev.aux, ev.ccm[slot], 0)) != hipSuccess) return e;
      EigArgs a{pl.nbeam, ks, pl.nchan, (const int32_t*)rec, nullptr, cnt, pl.eig.max_sweeps, 1,
                eigvals ? eigvals + off : nullptr, stat + off, v1 ? v1 + off : nullptr,
                status + off, out_stride, 2};
      if ((e = launch_eig(a, pl.eig, ev.aux)) != hipSuccess) return e;
      if ((e = hipEventRecord(ev.eig[slot], ev.aux)) != hipSuccess) return e;
      continue;
    }
    int32_t* sx = (int32_t*)base;
    int32_t* sxy = (int32_t*)(base + up(cells_cap * pl.nbeam * 4));
    int32_t* cnt = (int32_t*)(base + up(cells_cap * pl.nbeam * 4) +
                              up(cells_cap * npair_of(pl.nbeam) * 4));
    // the slot is free once the eigen stage of its previous group has run
    if (g >= pl.nslot && (e = hipStreamWaitEvent(s, ev.eig[slot], 0)) != hipSuccess) return e;
    // the per-wave tridiagonal solver reads one cell record per wave
    const int layout = pl.eig.solver == RFI_EIG_TRIDIAG ? 1 : 0;
    e = launch_ccm_mfma(bp, pl.nbeam, pl.nchan, row_stride, t0 + (int64_t)k0 * L, L, ks, sx, sxy,
                        cnt, 0, 0, s, &pl.ct, layout);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(ev.ccm[slot], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(ev.aux, ev.ccm[slot], 0)) != hipSuccess) return e;
    EigArgs a{pl.nbeam, ks, pl.nchan, sx, sxy, cnt, pl.eig.max_sweeps, 1,
              eigvals ? eigvals + off : nullptr, stat + off, v1 ? v1 + off : nullptr,
              status + off, out_stride, layout};
    e = launch_eig(a, pl.eig, ev.aux, pl.eig_wg ? pl.eig_wg : 256);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(ev.eig[slot], ev.aux)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(ev.done, ev.aux)) != hipSuccess) return e;
  return hipStreamWaitEvent(s, ev.done, 0);
}

}  // namespace rfi

namespace {

// Helper streams and events of rfi_process_block, one set per device,
// created on first use and kept until the process ends.
constexpr int kMaxDev = 64;
std::mutex g_mu;
rfi::PipeEvents g_ev[kMaxDev];

}  // namespace

using rfi::fail;

extern "C" {

size_t rfi_process_workspace_size(int32_t nbeam, int32_t nchan, const rfi_process_params* p) {
  rfi::ProcessPlan pl;
  if (rfi::resolve_process(nbeam, nchan, p, &pl, "rfi_process_workspace_size") != RFI_OK)
    return 0;
  return pl.ws_bytes;
}

rfi_status rfi_process_block(const rfi_block* blk, const rfi_process_params* p,
                             const uint8_t* protect_chan, rfi_stream_state* state, double* stat,
                             uint8_t* status, uint8_t* mask, float* eigvals, float* v1,
                             rfi_flag_stats* out, void* workspace, rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_process_block";
  if (!p) return fail(RFI_E_INVALID, "%s: params is NULL", who);
  rfi::BeamPtrs bp;
  rfi_status st = rfi::validate_block(blk, p->t0, p->L, p->nsub, who, &bp, RFI_MAX_COUNT_LONG);
  if (st != RFI_OK) return st;
  rfi::ProcessPlan pl;
  if ((st = rfi::resolve_process(blk->nbeam, blk->nchan, p, &pl, who)) != RFI_OK) return st;
  if (pl.nsub == 0) return RFI_OK;   // nothing to do; outputs may be empty (NULL)
  if (!stat || !status || !mask) return fail(RFI_E_INVALID, "%s: NULL output", who);
  if (p->beam_mask && !v1)
    return fail(RFI_E_INVALID, "%s: the per-beam mask needs the v1 output", who);
  if (p->beam_mask && !(p->kappa_v >= 0.0))
    return fail(RFI_E_INVALID, "%s: kappa_v must be >= 0", who);
  const bool scoped = p->scopes != 0 || p->fit != 0;
  if (p->scopes < 0 || p->scopes > 7)
    return fail(RFI_E_INVALID, "%s: scopes %d not in 0..7", who, p->scopes);
  if (p->fit != RFI_FIT_MOMENTS && p->fit != RFI_FIT_HISTOGRAM)
    return fail(RFI_E_INVALID, "%s: unknown fit %d", who, p->fit);
  if (scoped && state)
    return fail(RFI_E_INVALID, "%s: the pooled stream state needs the global moment clip "
                "(scopes 0, fit 0)", who);
  if (!workspace) return fail(RFI_E_INVALID, "%s: workspace is NULL", who);
  if ((uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "%s: workspace not 256-byte aligned", who);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rfi::check_hip(e, "rfi_process_block: hipGetDevice");
  if (dev < 0 || dev >= kMaxDev) return fail(RFI_E_DEVICE, "%s: device %d out of range", who, dev);
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  rfi::PipeEvents& ev = g_ev[dev];
  if ((e = ev.init()) != hipSuccess) return rfi::check_hip(e, "rfi_process_block: helper stream");
  const int64_t ncell = (int64_t)pl.nsub * pl.nchan;
  e = rfi::enqueue_eig_groups(bp, blk->row_stride, p->t0, p->L, pl, stat, status, eigvals, v1,
                              ncell, (char*)workspace + pl.flag_ws, ev, s);
  if (e != hipSuccess) return rfi::check_hip(e, "rfi_process_block: sums / eigen launch");
  const rfi::ClipJob cj = rfi::make_clip_job(pl.nsub, pl.nchan, stat, status, protect_chan,
                                             pl.kappa, pl.max_iter, state, mask, out, workspace);
  e = scoped ? rfi::launch_clip_scoped(cj, p->scopes ? p->scopes : RFI_SCOPE_GLOBAL, p->fit,
                                       nullptr, nullptr, s)
             : rfi::launch_clip(cj, s);
  if (e != hipSuccess) return rfi::check_hip(e, "rfi_process_block: clip launch");
  // the per-beam stage's partial sums reuse the clip's workspace (the clip
  // has run by then: same stream), which is always larger
  if (p->beam_mask)
    e = rfi::launch_eigvec_flag(blk->nbeam, pl.nsub, pl.nchan, v1, mask, status, protect_chan,
                                p->kappa_v, p->beam_mask, nullptr, nullptr, workspace, s);
  return rfi::check_hip(e, "rfi_process_block: per-beam stage launch");
}

}  // extern "C"
