// Batched uneven blocks: the whole path for many blocks with one launch per
// kernel class (rfi_process_batch), its capture into a HIP graph, and the
// autotuner of the per-class launch choices (rfi_tune_batch).
//
// Workspace layout: one descriptor area, uploaded by one host-to-device copy,
// then the sums of every block (sum_x, sum_xy, count; 256-byte aligned):
//   [beam pointer tables][CcmItem x nitem][EigArgs x nitem][cell0 x (nitem +
//   nclass)][ClipJob x nitem] | sums and clip workspace of item 0 | of item 1 | ...
// Items are ordered by sums class for the sums launches (each class a
// contiguous run of CcmItem sorted by first workgroup) and by solver class
// for the eigen launches (each a contiguous run of EigArgs with ascending
// first cells).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <vector>

#include "internal.h"
#include "rfi.h"

namespace rfi {
namespace {

constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct ItemPlan {
  int idx;                 // position in the caller's array
  BeamPtrs bp;
  int nbeam, nchan;
  int64_t ncell;
  CcmClass cc;
  CcmTune ct;              // sums-engine choices of the item's shape class
  int solver, precision;   // eigen class (solver, precision)
  int lane_cls;            // template class of the per-lane or per-wave tridiagonal solver
  int wg;                  // per-lane solver workgroup
  size_t sums_off;         // byte offset of the item's sums in the workspace
  size_t clip_off;         // byte offset of the item's clip workspace
  bool longL;              // L > RFI_MAX_COUNT: its own sums (int64 records of time
                           // chunks) and FP64 tridiagonal launches, the batched clip
};

struct EigClass {
  int lane_cls, solver, precision, wg, max_nbeam;
  std::vector<int> items;  // indices into plans
  bool v1 = false;         // some item asks for v1
};

struct CcmLaunchClass {
  int nbeam;               // any member's beam count
  CcmTune ct;
  std::vector<int> items;  // indices into plans
};

// Shape class of a beam count: the sums engine's 16-row block count.
inline int shape_class(int nbeam) { return (nbeam + 1 + 15) / 16; }
inline int class_lo(int sc) { return std::max(2, 16 * (sc - 1)); }
inline int class_hi(int sc) { return 16 * sc - 1; }

struct BatchPlan {
  std::vector<ItemPlan> plans;
  rfi_eig_params eig;      // sweeps, precision (solver per item)
  int max_iter = 50;
  double kappa = 3.0, kappa_v = 1.0;
  // descriptor area
  size_t tab_off = 0, ccm_off = 0, eig_off = 0, cell0_off = 0, flag_off = 0, desc_bytes = 0;
  size_t ws_bytes = 0;
  std::vector<CcmLaunchClass> ccm_classes;
  std::vector<EigClass> eig_classes;
  std::vector<char> host;  // descriptor bytes (device addresses resolved for ws)
  std::vector<rfi_batch_item> items;  // the caller's items (host copy)
  std::vector<ClipJob> clip_jobs;  // host copy of the clip descriptors (grid sizes)
};

rfi_status plan_batch(int nitem, const rfi_batch_item* items, const rfi_batch_params* p,
                      BatchPlan* bpn, const char* who) {
  if (nitem < 0) return fail(RFI_E_INVALID, "%s: nitem < 0", who);
  if (nitem > 0 && !items) return fail(RFI_E_INVALID, "%s: items is NULL", who);
  rfi_batch_params prm{32, 12, 50, 0, 3.0, nullptr, 1.0};
  if (p) prm = *p;
  if (prm.tune && (prm.tune->n < 0 || prm.tune->n > RFI_TUNE_MAX))
    return fail(RFI_E_INVALID, "%s: tune table with %d entries", who, prm.tune->n);
  if (prm.eig_precision == 0) prm.eig_precision = 32;
  if (prm.max_sweeps == 0) prm.max_sweeps = 12;
  if (prm.max_iter == 0) prm.max_iter = 50;
  if (!(prm.kappa >= 0.0)) return fail(RFI_E_INVALID, "%s: kappa must be >= 0", who);
  if (prm.max_iter < 1) return fail(RFI_E_INVALID, "%s: max_iter < 1", who);
  bpn->max_iter = prm.max_iter;
  bpn->kappa = prm.kappa;
  bpn->kappa_v = prm.kappa_v;
  bpn->items.assign(items, items + nitem);
  size_t tab_bytes = 0;
  for (int i = 0; i < nitem; ++i) {
    const rfi_batch_item& it = items[i];
    if (!it.blk) return fail(RFI_E_INVALID, "%s: item %d has no block", who, i);
    ItemPlan ip{};
    ip.idx = i;
    rfi_status st = validate_block(it.blk, it.t0, it.L, it.nsub, who, &ip.bp, RFI_MAX_COUNT_LONG);
    if (st != RFI_OK) return st;
    ip.longL = it.L > RFI_MAX_COUNT;
    if (it.nsub == 0) continue;
    if (!it.stat || !it.status || !it.mask)
      return fail(RFI_E_INVALID, "%s: item %d has a NULL output", who, i);
    if (it.beam_mask && !it.v1)
      return fail(RFI_E_INVALID, "%s: item %d: the per-beam mask needs v1", who, i);
    if (it.beam_mask && !(prm.kappa_v >= 0.0))
      return fail(RFI_E_INVALID, "%s: kappa_v must be >= 0", who);
    const rfi_tune_entry* te = find_tune(prm.tune, it.blk->nbeam);
    rfi_eig_params ep{prm.eig_precision, prm.max_sweeps, 1, te ? te->eig_solver : RFI_EIG_AUTO};
    rfi_eig_params res;
    if ((st = resolve_eig(it.blk->nbeam, &ep, &res, who)) != RFI_OK) return st;
    bpn->eig = res;
    ip.nbeam = it.blk->nbeam;
    ip.nchan = it.blk->nchan;
    ip.ncell = (int64_t)it.nsub * it.blk->nchan;
    ip.ct = CcmTune{te ? te->ccm_tile : 0, te ? te->ccm_stages : 0, te ? te->ccm_group_bytes : 0};
    if ((st = check_tune_entry(te, ip.nbeam, who)) != RFI_OK) return st;
    if (ccm_class(ip.nbeam, &ip.cc, &ip.ct) != hipSuccess)
      return fail(RFI_E_INVALID, "%s: item %d: no sums instance for %d beams", who, i, ip.nbeam);
    // long sub-intervals: the FP64 tridiagonal solver on the int64 sums (as
    // rfi_process_block; their cells read n L > 66,050 bytes each)
    ip.solver = ip.longL ? RFI_EIG_TRIDIAG : res.solver;
    ip.precision = res.precision;
    const bool lane = res.solver == RFI_EIG_LANE || res.solver == RFI_EIG_LANE_TRI;
    ip.lane_cls = lane                            ? eig_lane_class(ip.nbeam)
                  : res.solver == RFI_EIG_TRIDIAG ? eig_tri_class(ip.nbeam)
                                                  : 0;
    ip.wg = te && te->eig_wg ? te->eig_wg : 256;
    tab_bytes += (size_t)ip.nbeam * sizeof(void*);
    bpn->plans.push_back(ip);
  }
  const int n = (int)bpn->plans.size();
  // items that share a stream state would race in the batched clip (one
  // workgroup per block reads and writes the state at the same time)
  {
    std::vector<const rfi_stream_state*> st;
    for (const ItemPlan& ip : bpn->plans)
      if (items[ip.idx].state) st.push_back(items[ip.idx].state);
    std::sort(st.begin(), st.end());
    if (std::adjacent_find(st.begin(), st.end()) != st.end())
      return fail(RFI_E_INVALID, "%s: two items share one stream state; run consecutive blocks "
                  "of a stream in separate batches", who);
  }
  // classes
  std::map<long long, std::vector<int>> ccm;
  // (solver template class or 0, solver, precision, workgroup)
  std::map<std::tuple<int, int, int, int>, std::vector<int>> eig;
  for (int k = 0; k < n; ++k) {
    const ItemPlan& ip = bpn->plans[k];
    if (ip.longL) continue;           // launched on its own (enqueue_long)
    ccm[ip.cc.key].push_back(k);
    const bool lane = ip.solver == RFI_EIG_LANE || ip.solver == RFI_EIG_LANE_TRI;
    eig[{ip.lane_cls, ip.solver, ip.precision, lane ? ip.wg : 0}].push_back(k);
  }
  for (auto& kv : ccm)
    bpn->ccm_classes.push_back({bpn->plans[kv.second[0]].nbeam, bpn->plans[kv.second[0]].ct,
                                kv.second});
  for (auto& kv : eig) {
    EigClass ec{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                std::get<3>(kv.first), 0, kv.second};
    for (int k : kv.second) {
      ec.max_nbeam = std::max(ec.max_nbeam, bpn->plans[k].nbeam);
      if (items[bpn->plans[k].idx].v1) ec.v1 = true;
    }
    bpn->eig_classes.push_back(ec);
  }
  // layout
  size_t o = 0;
  bpn->tab_off = o;
  o = up(o + tab_bytes);
  bpn->ccm_off = o;
  o = up(o + (size_t)n * sizeof(CcmItem));
  bpn->eig_off = o;
  o = up(o + (size_t)n * sizeof(EigArgs));
  bpn->cell0_off = o;
  o = up(o + (size_t)(n + bpn->eig_classes.size()) * sizeof(int64_t));
  bpn->flag_off = o;
  o = up(o + (size_t)n * sizeof(ClipJob));
  bpn->desc_bytes = o;
  for (ItemPlan& ip : bpn->plans) {
    ip.sums_off = o;
    const int nsub = items[ip.idx].nsub;
    if (ip.longL)   // int64 cell records, the int32 chunk scratch, counts
      o += up((size_t)(ip.nbeam + npair_of(ip.nbeam)) * ip.ncell * 8) +
           up(ccm_long_tmp_bytes(ip.nbeam, ip.nchan, nsub)) + up((size_t)nsub * 4);
    else
      o += up((size_t)ip.nbeam * ip.ncell * 4) + up((size_t)npair_of(ip.nbeam) * ip.ncell * 4) +
           up((size_t)nsub * 4);
    ip.clip_off = o;
    o += up(clip_workspace_size(ip.ncell));
  }
  bpn->ws_bytes = std::max<size_t>(o, kAlign);
  return RFI_OK;
}

// Fill the descriptor bytes for a workspace at device address ws.
void fill_descriptors(const rfi_batch_item* items, BatchPlan* bpn, char* ws) {
  std::vector<char>& h = bpn->host;
  h.assign(bpn->desc_bytes, 0);
  auto dptr = [&](size_t off) { return ws + off; };
  size_t tab = bpn->tab_off;
  std::vector<const uint8_t* const*> tabs(bpn->plans.size());
  for (size_t k = 0; k < bpn->plans.size(); ++k) {
    const ItemPlan& ip = bpn->plans[k];
    std::memcpy(h.data() + tab, ip.bp.p, (size_t)ip.nbeam * sizeof(void*));
    tabs[k] = (const uint8_t* const*)dptr(tab);
    tab += (size_t)ip.nbeam * sizeof(void*);
  }
  auto sums = [&](const ItemPlan& ip, int32_t** sx, int32_t** sxy, int32_t** cnt) {
    char* b = dptr(ip.sums_off);
    *sx = (int32_t*)b;
    *sxy = (int32_t*)(b + up((size_t)ip.nbeam * ip.ncell * 4));
    *cnt = (int32_t*)(b + up((size_t)ip.nbeam * ip.ncell * 4) +
                      up((size_t)npair_of(ip.nbeam) * ip.ncell * 4));
  };
  // sums descriptors, class by class
  CcmItem* ci = (CcmItem*)(h.data() + bpn->ccm_off);
  int pos = 0;
  for (auto& cls : bpn->ccm_classes) {
    int wg = 0;
    for (int k : cls.items) {
      const ItemPlan& ip = bpn->plans[k];
      const rfi_batch_item& it = items[ip.idx];
      CcmItem& c = ci[pos++];
      c.beams = tabs[k];
      c.row_stride = it.blk->row_stride;
      c.t0 = it.t0;
      sums(ip, &c.sum_x, &c.sum_xy, &c.count);
      c.nbeam = ip.nbeam;
      c.nchan = ip.nchan;
      c.L = it.L;
      c.nsub = it.nsub;
      c.nct = (ip.nchan + ip.cc.cw - 1) / ip.cc.cw;
      c.nh = ip.cc.nh;
      c.wg0 = wg;
      c.layout = ip.solver == RFI_EIG_TRIDIAG ? 1 : 0;
      wg += (c.nsub * c.nct + 7) / 8 * 8;
    }
  }
  // eigen descriptors, class by class, with the first global cell of each
  EigArgs* ea = (EigArgs*)(h.data() + bpn->eig_off);
  int64_t* c0 = (int64_t*)(h.data() + bpn->cell0_off);
  pos = 0;
  int cpos = 0;
  for (EigClass& ec : bpn->eig_classes) {
    int64_t cell = 0;
    for (int k : ec.items) {
      const ItemPlan& ip = bpn->plans[k];
      const rfi_batch_item& it = items[ip.idx];
      EigArgs& a = ea[pos++];
      int32_t *sx, *sxy, *cnt;
      sums(ip, &sx, &sxy, &cnt);
      a = EigArgs{ip.nbeam, it.nsub, ip.nchan, sx, sxy, cnt, bpn->eig.max_sweeps, 1,
                  nullptr, it.stat, it.v1, it.status, ip.ncell,
                  ip.solver == RFI_EIG_TRIDIAG ? 1 : 0};
      c0[cpos++] = cell;
      cell += ip.ncell;
    }
    c0[cpos++] = cell;      // total of the class
  }
  ClipJob* fi = (ClipJob*)(h.data() + bpn->flag_off);
  bpn->clip_jobs.resize(bpn->plans.size());
  for (size_t k = 0; k < bpn->plans.size(); ++k) {
    const ItemPlan& ip = bpn->plans[k];
    const rfi_batch_item& it = items[ip.idx];
    fi[k] = make_clip_job(it.nsub, ip.nchan, it.stat, it.status, it.protect_chan, bpn->kappa,
                          bpn->max_iter, it.state, it.mask, it.out, dptr(ip.clip_off));
    bpn->clip_jobs[k] = fi[k];
  }
}

// The batch's launches on s, in three parts; desc is the host copy of the
// descriptors (pinned for graph capture, where the copy node reads it at
// every replay).
hipError_t enqueue_desc(const BatchPlan& bpn, const void* desc, char* ws, hipStream_t s) {
  return hipMemcpyAsync(ws, desc, bpn.desc_bytes, hipMemcpyHostToDevice, s);
}

hipError_t enqueue_ccm(const BatchPlan& bpn, const void* desc, char* ws, hipStream_t s) {
  const CcmItem* ci = (const CcmItem*)(ws + bpn.ccm_off);
  const CcmItem* hci = (const CcmItem*)((const char*)desc + bpn.ccm_off);
  int pos = 0;
  for (const CcmLaunchClass& cls : bpn.ccm_classes) {
    const int m = (int)cls.items.size();
    const CcmItem& last = hci[pos + m - 1];
    const int total = last.wg0 + (last.nsub * last.nct + 7) / 8 * 8;
    hipError_t e = launch_ccm_batch(cls.nbeam, &cls.ct, ci + pos, m, total, s);
    if (e != hipSuccess) return e;
    pos += m;
  }
  return hipSuccess;
}

hipError_t enqueue_eig(const BatchPlan& bpn, const void* desc, char* ws, hipStream_t s) {
  const EigArgs* ea = (const EigArgs*)(ws + bpn.eig_off);
  const int64_t* c0 = (const int64_t*)(ws + bpn.cell0_off);
  const int64_t* hc0 = (const int64_t*)((const char*)desc + bpn.cell0_off);
  int pos = 0, cpos = 0;
  for (const EigClass& ec : bpn.eig_classes) {
    const int m = (int)ec.items.size();
    const int64_t total = hc0[cpos + m];
    hipError_t e;
    if (ec.solver == RFI_EIG_LANE || ec.solver == RFI_EIG_LANE_TRI)
      e = launch_eig_lane_batch(ec.lane_cls, ea + pos, c0 + cpos, m, total, s, ec.wg,
                                ec.solver == RFI_EIG_LANE_TRI);
    else if (ec.solver == RFI_EIG_TRIDIAG)
      e = launch_eig_tri_batch(ec.lane_cls, ea + pos, c0 + cpos, m, total, s, ec.v1);
    else
      e = launch_eig_wave_batch(ec.precision, ec.max_nbeam, ea + pos, c0 + cpos, m, total, s);
    if (e != hipSuccess) return e;
    pos += m;
    cpos += m + 1;
  }
  return hipSuccess;
}

// The items with long sub-intervals: exact int64 sums of time chunks, then the
// FP64 tridiagonal solver on them (the launches of rfi_process_block's long
// route, on the batch's stream).
hipError_t enqueue_long(const BatchPlan& bpn, char* ws, hipStream_t s) {
  for (const ItemPlan& ip : bpn.plans) {
    if (!ip.longL) continue;
    const rfi_batch_item& it = bpn.items[ip.idx];
    char* b = ws + ip.sums_off;
    int64_t* rec = (int64_t*)b;
    char* tmp = b + up((size_t)(ip.nbeam + npair_of(ip.nbeam)) * ip.ncell * 8);
    int32_t* cnt = (int32_t*)(tmp + up(ccm_long_tmp_bytes(ip.nbeam, ip.nchan, it.nsub)));
    hipError_t e = launch_ccm_long(ip.bp, ip.nbeam, ip.nchan, it.blk->row_stride, it.t0, it.L,
                                   it.nsub, rec, cnt, tmp, s, &ip.ct);
    if (e != hipSuccess) return e;
    EigArgs a{ip.nbeam, it.nsub, ip.nchan, (const int32_t*)rec, nullptr, cnt, bpn.eig.max_sweeps,
              1, nullptr, it.stat, it.v1, it.status, ip.ncell, 2};
    if ((e = launch_eig_tri(a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_batch(const BatchPlan& bpn, const void* desc, char* ws, hipStream_t s) {
  const int n = (int)bpn.plans.size();
  if (n == 0) return hipSuccess;
  hipError_t e = enqueue_desc(bpn, desc, ws, s);
  if (e == hipSuccess) e = enqueue_ccm(bpn, desc, ws, s);
  if (e == hipSuccess) e = enqueue_eig(bpn, desc, ws, s);
  if (e == hipSuccess) e = enqueue_long(bpn, ws, s);
  if (e != hipSuccess) return e;
  e = launch_clip_batch((const ClipJob*)(ws + bpn.flag_off), bpn.clip_jobs.data(), n, s);
  // per-beam stages, after every clip: their partial sums reuse each block's
  // clip workspace (always larger)
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    const ItemPlan& ip = bpn.plans[k];
    const rfi_batch_item& it = bpn.items[ip.idx];
    if (!it.beam_mask) continue;
    e = launch_eigvec_flag(ip.nbeam, it.nsub, ip.nchan, it.v1, it.mask, it.status,
                           it.protect_chan, bpn.kappa_v, it.beam_mask, nullptr, nullptr,
                           ws + ip.clip_off, s);
  }
  return e;
}

// Median time (ms) of three runs of fn on s after one warm-up; -1 on a
// launch error; the warm-up time alone when it exceeds `cutoff` ms.
float time_ms(const std::function<hipError_t()>& fn, hipStream_t s, float cutoff) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess) return -1.f;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1.f;
  }
  float res = -1.f, t[3] = {0, 0, 0};
  int run = 0;
  for (; run < 4; ++run) {
    if (hipEventRecord(a, s) != hipSuccess || fn() != hipSuccess ||
        hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
      break;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (run == 0 && ms > cutoff) {
      res = ms;
      run = 5;
      break;
    }
    if (run > 0) t[run - 1] = ms;
  }
  if (run == 4) {
    std::sort(t, t + 3);
    res = t[1];
  }
  (void)hipGetLastError();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return res;
}

}  // namespace

const rfi_tune_entry* find_tune(const rfi_tune_table* t, int nbeam) {
  if (!t) return nullptr;
  for (int i = 0; i < std::min<int>(t->n, RFI_TUNE_MAX); ++i)
    if (t->e[i].nbeam_lo <= nbeam && nbeam <= t->e[i].nbeam_hi) return &t->e[i];
  return nullptr;
}

rfi_status check_tune_entry(const rfi_tune_entry* te, int nbeam, const char* who) {
  if (!te) return RFI_OK;
  if (te->ccm_stages < 0 || te->ccm_stages > 4 || te->ccm_group_bytes < 0 ||
      te->ccm_group_bytes > 16384 || te->ccm_tile < 0 || te->ccm_tile >= ccm_tile_variants(nbeam))
    return fail(RFI_E_INVALID, "%s: tune entry for %d beams out of range", who, nbeam);
  if (te->eig_wg != 0 && te->eig_wg != 64 && te->eig_wg != 128 && te->eig_wg != 256)
    return fail(RFI_E_INVALID, "%s: tune entry eig_wg %d not 0, 64, 128 or 256", who, te->eig_wg);
  return RFI_OK;
}

}  // namespace rfi

struct rfi_batch_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* desc = nullptr;      // pinned host copy of the descriptors
};

using rfi::fail;

extern "C" {

size_t rfi_batch_workspace_size(int32_t nitem, const rfi_batch_item* items,
                                const rfi_batch_params* p) {
  rfi::clear_error();
  rfi::BatchPlan bpn;
  if (rfi::plan_batch(nitem, items, p, &bpn, "rfi_batch_workspace_size") != RFI_OK) return 0;
  return bpn.ws_bytes;
}

rfi_status rfi_process_batch(int32_t nitem, const rfi_batch_item* items,
                             const rfi_batch_params* p, void* workspace, rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_process_batch";
  rfi::BatchPlan bpn;
  rfi_status st = rfi::plan_batch(nitem, items, p, &bpn, who);
  if (st != RFI_OK) return st;
  if (bpn.plans.empty()) return RFI_OK;
  if (!workspace || (uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "%s: workspace NULL or not 256-byte aligned", who);
  rfi::fill_descriptors(items, &bpn, (char*)workspace);
  // pageable source: the runtime stages it before the call returns
  return rfi::check_hip(rfi::enqueue_batch(bpn, bpn.host.data(), (char*)workspace,
                                           (hipStream_t)stream),
                        who);
}

rfi_status rfi_tune_batch(int32_t nitem, const rfi_batch_item* items, const rfi_batch_params* p,
                          void* workspace, rfi_tune_table* table, rfi_stream_t stream) {
  rfi::clear_error();
  const char* who = "rfi_tune_batch";
  if (!table) return fail(RFI_E_INVALID, "%s: table is NULL", who);
  std::memset(table, 0, sizeof(*table));
  rfi_batch_params base{32, 12, 50, 0, 3.0, nullptr};
  if (p) base = *p;
  base.tune = nullptr;
  rfi::BatchPlan full;
  rfi_status st = rfi::plan_batch(nitem, items, &base, &full, who);
  if (st != RFI_OK) return st;
  if (full.plans.empty()) return RFI_OK;
  if (!workspace || (uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "%s: workspace NULL or not 256-byte aligned", who);
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  // the items of each shape class
  std::map<int, std::vector<rfi_batch_item>> by_class;
  std::map<int, int> max_nbeam;
  for (const rfi::ItemPlan& ip : full.plans) {
    if (ip.longL) continue;      // long sub-intervals take their own fixed route
    const int sc = rfi::shape_class(ip.nbeam);
    by_class[sc].push_back(items[ip.idx]);
    max_nbeam[sc] = std::max(max_nbeam[sc], ip.nbeam);
  }
  const int precision = full.eig.precision;
  int ne = 0;
  for (auto& kv : by_class) {
    if (ne >= RFI_TUNE_MAX) break;
    const int sc = kv.first;
    std::vector<rfi_batch_item>& sub = kv.second;
    rfi_tune_entry cur{};
    cur.nbeam_lo = rfi::class_lo(sc);
    cur.nbeam_hi = rfi::class_hi(sc);
    rfi_tune_table one{};
    one.n = 1;
    // plan the class's items with the entry `e`; run one part of it
    auto measure = [&](const rfi_tune_entry& e, int part, float cutoff) -> float {
      one.e[0] = e;
      rfi_batch_params q = base;
      q.tune = &one;
      rfi::BatchPlan bp;
      if (rfi::plan_batch((int32_t)sub.size(), sub.data(), &q, &bp, who) != RFI_OK) return -1.f;
      rfi::fill_descriptors(sub.data(), &bp, ws);
      if (rfi::enqueue_desc(bp, bp.host.data(), ws, s) != hipSuccess) return -1.f;
      if (part == 1) {
        // sums first (the eigen stage reads them), then the eigen launches
        if (rfi::enqueue_ccm(bp, bp.host.data(), ws, s) != hipSuccess) return -1.f;
        return rfi::time_ms([&] { return rfi::enqueue_eig(bp, bp.host.data(), ws, s); }, s,
                            cutoff);
      }
      return rfi::time_ms([&] { return rfi::enqueue_ccm(bp, bp.host.data(), ws, s); }, s, cutoff);
    };
    const float big = 1e30f;
    // a candidate replaces the incumbent only when clearly faster (timing noise)
    constexpr float kGain = 0.98f;
    const float ccm_def = measure(cur, 0, big);
    const float eig_def = measure(cur, 1, big);
    if (ccm_def < 0.f || eig_def < 0.f) {
      (void)hipGetLastError();
      return fail(RFI_E_DEVICE, "%s: default launch of class %d-%d failed", who, cur.nbeam_lo,
                  cur.nbeam_hi);
    }
    // sums: tile variant x ring depth, then the XCD group size
    rfi_tune_entry best = cur;
    float best_ccm = ccm_def;
    std::vector<long long> seen;
    {
      rfi::CcmClass c0;
      if (rfi::ccm_class(kv.second.empty() ? 19 : max_nbeam[sc], &c0, nullptr) == hipSuccess)
        seen.push_back(c0.key);
    }
    for (int tile = 0; tile < rfi::ccm_tile_variants(max_nbeam[sc]); ++tile) {
      for (int stages = 4; stages >= 2; --stages) {
        rfi_tune_entry e = cur;
        e.ccm_tile = tile;
        e.ccm_stages = stages;
        rfi::CcmTune ct{tile, stages, 0};
        rfi::CcmClass cc;
        if (rfi::ccm_class(max_nbeam[sc], &cc, &ct) != hipSuccess) continue;
        if (std::find(seen.begin(), seen.end(), cc.key) != seen.end()) continue;
        seen.push_back(cc.key);
        const float t = measure(e, 0, 4.f * best_ccm);
        if (t > 0.f && t < kGain * best_ccm) {
          best_ccm = t;
          best.ccm_tile = tile;
          best.ccm_stages = stages;
        }
      }
    }
    for (int gb : {256, 512, 2048, 4096, 8192}) {
      rfi_tune_entry e = best;
      e.ccm_group_bytes = gb;
      const float t = measure(e, 0, 4.f * best_ccm);
      if (t > 0.f && t < kGain * best_ccm) {
        best_ccm = t;
        best.ccm_group_bytes = gb;
      }
    }
    // eigen: the solvers that apply to every block of the class
    float best_eig = eig_def;
    std::vector<std::pair<int, int>> cands;  // (solver, wg)
    if (precision == 32 && max_nbeam[sc] <= 20) {
      cands = {{RFI_EIG_LANE, 256},     {RFI_EIG_LANE, 128},     {RFI_EIG_LANE, 64},
               {RFI_EIG_LANE_TRI, 256}, {RFI_EIG_LANE_TRI, 128}, {RFI_EIG_LANE_TRI, 64},
               {RFI_EIG_TRIDIAG, 0}};
    } else if (precision == 64) {
      cands = {{RFI_EIG_TRIDIAG, 0}, {RFI_EIG_WAVE, 0}};
    }
    // (FP32 above 20 beams: the tridiagonal solver only; the FP32 Jacobi wave
    // solver there is the precision split's reference, 50-100x slower, and
    // even one warm-up of it costs seconds on a large class)
    const int def_solver = precision == 64 ? RFI_EIG_WAVE
                           : (max_nbeam[sc] <= 20 ? RFI_EIG_LANE_TRI : RFI_EIG_TRIDIAG);
    for (auto& c : cands) {
      if (c.first == def_solver && (c.second == 0 || c.second == 256)) continue;  // measured
      rfi_tune_entry e = best;
      e.eig_solver = c.first;
      e.eig_wg = c.second;
      const float t = measure(e, 1, 4.f * best_eig);
      if (t > 0.f && t < kGain * best_eig) {
        best_eig = t;
        best.eig_solver = c.first;
        best.eig_wg = c.second;
      }
    }
    best.ms_default = (double)ccm_def + eig_def;
    best.ms_tuned = (double)best_ccm + best_eig;
    table->e[ne++] = best;
  }
  table->n = ne;
  return rfi::check_hip(hipGetLastError(), who);
}

rfi_status rfi_batch_graph_create(int32_t nitem, const rfi_batch_item* items,
                                  const rfi_batch_params* p, void* workspace,
                                  rfi_batch_graph** out) {
  rfi::clear_error();
  const char* who = "rfi_batch_graph_create";
  if (!out) return fail(RFI_E_INVALID, "%s: out is NULL", who);
  *out = nullptr;
  rfi::BatchPlan bpn;
  rfi_status st = rfi::plan_batch(nitem, items, p, &bpn, who);
  if (st != RFI_OK) return st;
  if (!workspace || (uintptr_t)workspace % 256 != 0)
    return fail(RFI_E_INVALID, "%s: workspace NULL or not 256-byte aligned", who);
  rfi::fill_descriptors(items, &bpn, (char*)workspace);
  std::unique_ptr<rfi_batch_graph> g(new rfi_batch_graph);
  hipError_t e = hipHostMalloc(&g->desc, std::max<size_t>(bpn.desc_bytes, 1), 0);
  if (e != hipSuccess) return rfi::check_hip(e, who);
  std::memcpy(g->desc, bpn.host.data(), bpn.desc_bytes);
  hipStream_t cs = nullptr;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
    (void)hipHostFree(g->desc);
    return rfi::check_hip(e, who);
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t ee = rfi::enqueue_batch(bpn, g->desc, (char*)workspace, cs);
    e = hipStreamEndCapture(cs, &g->graph);
    if (ee != hipSuccess) e = ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipHostFree(g->desc);
    return rfi::check_hip(e, who);
  }
  *out = g.release();
  return RFI_OK;
}

rfi_status rfi_batch_graph_launch(rfi_batch_graph* g, rfi_stream_t stream) {
  rfi::clear_error();
  if (!g) return fail(RFI_E_INVALID, "rfi_batch_graph_launch: NULL graph");
  return rfi::check_hip(hipGraphLaunch(g->exec, (hipStream_t)stream), "rfi_batch_graph_launch");
}

void rfi_batch_graph_destroy(rfi_batch_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->desc) (void)hipHostFree(g->desc);
  delete g;
}

}  // extern "C"
