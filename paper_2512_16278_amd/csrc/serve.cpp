// Serving runtime: continuous batching of observation blocks from many
// streams on one device (the session API of rfi.h).
//
// A scheduler thread owns the device work. Queued blocks are admitted in
// submission order whenever an execution slot is free and the HBM budget
// allows; a block of a stream never overtakes an earlier queued block of the
// same stream, but blocks of other streams may pass a block that does not
// fit yet (no head-of-line blocking). Each slot is a non-blocking HIP stream
// with its own helper stream, workspace and clip summary buffers, so admitted
// blocks of different streams run concurrently. Blocks of one stream are
// chained by a per-stream event, because each reads and writes that stream's
// device state: the pooled clip state and fit history, and the carry of the
// partial sub-interval. Completion is event-driven: behind each block's work
// the slot's stream runs a host function that rings the scheduler's doorbell
// (a flag under a mutex that no thread holds across a HIP call, so the HIP
// runtime's callback thread never waits on a thread that waits on HIP).
// Result buffers come from a session pool of power-of-two size classes and go
// back to it on release. A block whose launches fail part-way keeps its slot
// until what was enqueued has run, and fails its stream: later blocks of that
// stream are refused (its carry and clip state are no longer defined).
//
// Per block (all on the slot's stream, after the stream's previous block):
//   1. if the stream carries c samples of a sub-interval, the first L - c
//      samples are added into the carry sums and, when that completes it,
//      the eigen stage runs on that one row of cells (row 0 of the block);
//   2. the full sub-intervals that follow run through the grouped sums ->
//      eigen pipeline of the whole-block call;
//   3. the remaining samples start a new carry;
//   4. the clip over all of the block's cells, pooled with the stream state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "pipeline.h"
#include "rfi.h"

namespace rfi {
namespace {

using Clock = std::chrono::steady_clock;
constexpr int kMaxSlots = 64;
constexpr int64_t kDefaultBudget = (int64_t)64 << 30;
constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct StreamCtx {
  int id = 0;
  rfi_stream_config cfg{};
  uint8_t* protect = nullptr;        // device copy of the preserved-channel flags
  rfi_stream_state* state = nullptr; // device
  int32_t* carry = nullptr;          // device: sum_x [nbeam][nchan], sum_xy [npair][nchan], count;
                                     // long sub-intervals: int64 records [nchan][nbeam + npair], count
  int64_t carry_samples = 0;         // samples in the carry after the last admitted block
  hipEvent_t last = nullptr;         // completion of the stream's last admitted block
  bool has_last = false;
  bool failed = false;               // a block's launches failed part-way: state undefined
  int queued = 0, inflight = 0;
  bool tuned = false;                // te holds the session's tune entry for nbeam
  rfi_tune_entry te{};
  const rfi_tune_entry* tune() const { return tuned ? &te : nullptr; }
  // sub-intervals past the int32 bound: the carry's sums are int64 cell
  // records, summed by the long route (time chunks widened into int64)
  bool longL() const { return cfg.L > RFI_MAX_COUNT; }
  size_t carry_rows() const { return (size_t)(cfg.nbeam + npair_of(cfg.nbeam)) * cfg.nchan; }
  int32_t* carry_sx() const { return carry; }
  int32_t* carry_sxy() const { return carry + (size_t)cfg.nbeam * cfg.nchan; }
  int64_t* carry_rec() const { return (int64_t*)carry; }
  int32_t* carry_cnt() const {
    return longL() ? (int32_t*)(carry_rec() + carry_rows()) : carry + carry_rows();
  }
  size_t carry_bytes() const {
    return longL() ? carry_rows() * sizeof(int64_t) + sizeof(int32_t)
                   : (carry_rows() + 1) * sizeof(int32_t);
  }
};

enum class RState { Queued, Running, Done };

struct Request {
  uint64_t ticket = 0, tag = 0;
  int stream_id = 0;
  rfi_block blk{};
  RState st = RState::Queued;
  rfi_status status = RFI_OK;
  int nsub = 0, carried = 0;
  int64_t carry_after = 0;
  int64_t charge_run = 0, charge_res = 0;
  void* res = nullptr;               // stat | cell status | mask, one pooled buffer
  size_t res_cls = 0;                // its pool size class
  double* stat = nullptr;
  uint8_t* cstat = nullptr;
  uint8_t* mask = nullptr;
  float* v1 = nullptr;               // per-beam stage outputs (streams with beam_stage)
  uint8_t* bmask = nullptr;
  bool beams = false;                // the stream has the per-beam stage
  rfi_flag_stats flag{};
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  rfi_status pending = RFI_OK;       // failure to report once the enqueued work has run
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;         // recorded behind the running block's work
  bool poll = false;                 // no host function behind it: query the event
  PipeEvents ev;
  void* ws = nullptr;
  size_t ws_size = 0;
  rfi_flag_stats* dstats = nullptr;  // device
  rfi_flag_stats* hstats = nullptr;  // pinned host
  Request* req = nullptr;
};

// Argument of the host function behind a block's work (one per slot).
struct SlotBell {
  rfi_session* s;
  int slot;
};

// The device stays current for the calling thread only inside the guard.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace
}  // namespace rfi

struct rfi_session {
  int device = 0;
  int max_slots = 8;
  int64_t budget = rfi::kDefaultBudget;
  bool has_tune = false;  // session copy of the caller's tune table
  rfi_tune_table tune{};
  std::mutex mu;
  std::condition_variable cv_done;   // a block finished, for waiters
  // doorbell of the scheduler: new work, a freed budget, stop, or a slot's
  // host function. db_mu is never held across a HIP call.
  std::mutex db_mu;
  std::condition_variable db_cv;
  bool db_rung = false;
  std::vector<unsigned char> db_slot;   // per slot: its host function has run
  std::vector<rfi::SlotBell> bells;     // host-function arguments, one per slot
  // result buffers by power-of-two size class, and the bytes they hold idle
  std::map<size_t, std::vector<void*>> pool;
  int64_t pool_idle = 0;
  std::thread sched;
  bool stop = false;
  std::deque<rfi::Request*> queue;
  std::map<uint64_t, std::unique_ptr<rfi::Request>> reqs;
  std::map<int, std::unique_ptr<rfi::StreamCtx>> streams;
  std::vector<rfi::Slot> slots;
  int running = 0;
  int64_t charged = 0;
  uint64_t next_ticket = 1;
  int next_stream = 1;
  rfi::Clock::time_point t0;
  hipStream_t free_stream = nullptr;  // stream-ordered frees of released memory

  double now_us() const {
    return std::chrono::duration<double, std::micro>(rfi::Clock::now() - t0).count();
  }
  void scheduler();
  bool admit(rfi::Request* r);        // false: does not fit now
  rfi_status enqueue(rfi::Request* r, rfi::Slot& sl, rfi::StreamCtx& st, bool* launched);
  void finish(rfi::Slot& sl, bool ok);
  void ring(int slot = -1) {
    {
      std::lock_guard<std::mutex> g(db_mu);
      db_rung = true;
      if (slot >= 0) db_slot[slot] = 1;
    }
    db_cv.notify_one();
  }
  hipError_t res_get(size_t n, hipStream_t s, void** p, size_t* cls);
  void res_put(void* p, size_t cls);
};

// Host function behind a block's work on its slot's stream.
static void slot_bell(void* arg) {
  const rfi::SlotBell* b = (const rfi::SlotBell*)arg;
  b->s->ring(b->slot);
}

hipError_t rfi_session::res_get(size_t n, hipStream_t s, void** p, size_t* cls) {
  size_t c = (size_t)1 << 16;
  while (c < n) c <<= 1;
  *cls = c;
  auto it = pool.find(c);
  if (it != pool.end() && !it->second.empty()) {
    *p = it->second.back();
    it->second.pop_back();
    pool_idle -= (int64_t)c;
    return hipSuccess;
  }
  return hipMallocAsync(p, c, s);
}

void rfi_session::res_put(void* p, size_t cls) {
  // keep at most a quarter of the budget idle in the pool
  if (pool_idle + (int64_t)cls > budget / 4) {
    (void)hipFreeAsync(p, free_stream);
    return;
  }
  pool[cls].push_back(p);
  pool_idle += (int64_t)cls;
}

namespace rfi {
namespace {

// Cells, carry and buffer sizes of a block given the stream's carry.
struct BlockPlan {
  int64_t t_full = 0;   // first sample of the full sub-intervals
  int carried = 0;      // the carry sub-interval completes in this block
  int64_t carry_add = 0;  // samples added to the carry before t_full
  int nfull = 0;
  int64_t rem = 0;      // samples after the full sub-intervals
  int64_t carry_after = 0;
  int nsub = 0;
  ProcessPlan pl;       // for max(nfull, 1) sub-intervals
  size_t ws = 0, res = 0;
};

rfi_status plan_block(const StreamCtx& st, int64_t nsamp, BlockPlan* b, const char* who) {
  const int64_t L = st.cfg.L, c = st.carry_samples;
  int64_t t = 0;
  if (c > 0) {
    const int64_t need = L - c;
    if (nsamp >= need) {
      b->carried = 1;
      b->carry_add = need;
      t = need;
    } else {
      b->carry_add = nsamp;
      t = nsamp;
    }
  }
  b->t_full = t;
  const bool open_carry = c > 0 && !b->carried;
  b->nfull = open_carry ? 0 : (int)((nsamp - t) / L);
  b->rem = open_carry ? 0 : nsamp - t - (int64_t)b->nfull * L;
  b->carry_after = open_carry ? c + nsamp : b->rem;
  b->nsub = b->carried + b->nfull;
  if ((int64_t)b->nsub * st.cfg.nchan > ((int64_t)1 << 30))
    return fail(RFI_E_INVALID, "%s: block has more than 2^30 cells", who);
  rfi_process_params p{};
  p.L = (int32_t)L;
  p.nsub = b->nfull > 0 ? b->nfull : 1;
  p.eig_precision = st.cfg.eig_precision;
  p.max_sweeps = st.cfg.max_sweeps;
  p.max_iter = st.cfg.max_iter;
  p.kappa = st.cfg.kappa;
  rfi_status s = resolve_process(st.cfg.nbeam, st.cfg.nchan, &p, &b->pl, who, st.tune());
  if (s != RFI_OK) return s;
  // the clip covers all nsub rows (the carried one included)
  b->pl.flag_ws = up(clip_workspace_size((int64_t)b->nsub * st.cfg.nchan));
  b->pl.ws_bytes = b->pl.flag_ws + (size_t)b->pl.nslot * b->pl.slot;
  b->ws = b->pl.ws_bytes;
  // the carry of a long sub-interval is summed through the int32 chunk
  // scratch of the long route, placed after the pipeline's workspace
  if (st.longL()) b->ws += up(ccm_long_tmp_bytes(st.cfg.nbeam, st.cfg.nchan, 1));
  const size_t ncell = (size_t)b->nsub * st.cfg.nchan;
  b->res = ncell ? up(ncell * 8) + up(ncell) + up(ncell) : 0;
  if (ncell && st.cfg.beam_stage)
    b->res += up(ncell * st.cfg.nbeam * 4) + up(ncell * st.cfg.nbeam);
  return RFI_OK;
}

int64_t input_bytes(const rfi_block& blk) {
  return (int64_t)blk.nbeam * blk.nsamp * blk.row_stride;
}

}  // namespace
}  // namespace rfi

using rfi::fail;

// On failure, *launched tells whether work of this block was already enqueued.
rfi_status rfi_session::enqueue(rfi::Request* r, rfi::Slot& sl, rfi::StreamCtx& st,
                                bool* launched) {
  using namespace rfi;
  hipError_t e;
  *launched = false;
  BlockPlan b;
  rfi_status rs = plan_block(st, r->blk.nsamp, &b, "rfi_submit");
  if (rs != RFI_OK) return rs;
  BeamPtrs bp;
  std::memset(&bp, 0, sizeof(bp));
  for (int i = 0; i < r->blk.nbeam; ++i) bp.p[i] = r->blk.beam[i];
  const int n = st.cfg.nbeam, F = st.cfg.nchan, L = st.cfg.L;
  const int64_t stride = r->blk.row_stride;
  hipStream_t s = sl.s;
  auto dev = [&](hipError_t err, const char* what) {
    return err == hipSuccess ? RFI_OK : check_hip(err, what);
  };
  if (st.has_last && (e = hipStreamWaitEvent(s, st.last, 0)) != hipSuccess)
    return dev(e, "rfi_submit: stream order");
  if (sl.ws_size < b.ws) {
    if (sl.ws) (void)hipFreeAsync(sl.ws, s);
    sl.ws = nullptr;
    sl.ws_size = 0;
    if ((e = hipMallocAsync(&sl.ws, b.ws, s)) != hipSuccess) return dev(e, "rfi_submit: workspace");
    sl.ws_size = b.ws;
  }
  if (b.res) {
    if ((e = res_get(b.res, s, &r->res, &r->res_cls)) != hipSuccess)
      return dev(e, "rfi_submit: results");
    const size_t ncell = (size_t)b.nsub * F;
    r->stat = (double*)r->res;
    r->cstat = (uint8_t*)r->res + up(ncell * 8);
    r->mask = r->cstat + up(ncell);
    if (st.cfg.beam_stage) {
      r->v1 = (float*)(r->mask + up(ncell));
      r->bmask = (uint8_t*)r->v1 + up(ncell * n * 4);
    }
  }
  // from here on a failure leaves work of this block enqueued behind it (the
  // stream-order wait and the allocations above change no state)
  *launched = true;
  // 1. complete (or extend) the carried sub-interval
  void* ltmp = (char*)sl.ws + b.pl.ws_bytes;     // long carries only
  if (b.carry_add > 0) {
    e = st.longL() ? launch_ccm_long(bp, n, F, stride, 0, (int)b.carry_add, 1, st.carry_rec(),
                                     st.carry_cnt(), ltmp, s, &b.pl.ct, 1)
                   : launch_ccm_mfma(bp, n, F, stride, 0, (int)b.carry_add, 1, st.carry_sx(),
                                     st.carry_sxy(), st.carry_cnt(), 1, 0, s, &b.pl.ct);
    if (e != hipSuccess) return dev(e, "rfi_submit: carry sums");
  }
  if (b.carried) {
    EigArgs a{n, 1, F, st.longL() ? (const int32_t*)st.carry_rec() : st.carry_sx(),
              st.longL() ? nullptr : st.carry_sxy(), st.carry_cnt(), b.pl.eig.max_sweeps, 1,
              nullptr, r->stat, r->v1, r->cstat, (int64_t)b.nsub * F, st.longL() ? 2 : 0};
    e = launch_eig(a, b.pl.eig, s, b.pl.eig_wg ? b.pl.eig_wg : 256);
    if (e != hipSuccess) return dev(e, "rfi_submit: carry eigen stage");
  }
  // 2. full sub-intervals
  if (b.nfull > 0) {
    ProcessPlan pl = b.pl;
    char* ws = (char*)sl.ws;
    e = enqueue_eig_groups(bp, stride, b.t_full, L, pl, r->stat + (size_t)b.carried * F,
                           r->cstat + (size_t)b.carried * F, nullptr,
                           r->v1 ? r->v1 + (size_t)b.carried * F : nullptr,
                           (int64_t)b.nsub * F, ws + pl.flag_ws, sl.ev, s);
    if (e != hipSuccess) return dev(e, "rfi_submit: sums / eigen stage");
  }
  // 3. new carry
  if (b.rem > 0) {
    const int64_t tr = b.t_full + (int64_t)b.nfull * L;
    e = st.longL() ? launch_ccm_long(bp, n, F, stride, tr, (int)b.rem, 1, st.carry_rec(),
                                     st.carry_cnt(), ltmp, s, &b.pl.ct, 0)
                   : launch_ccm_mfma(bp, n, F, stride, tr, (int)b.rem, 1, st.carry_sx(),
                                     st.carry_sxy(), st.carry_cnt(), 0, 0, s, &b.pl.ct);
    if (e != hipSuccess) return dev(e, "rfi_submit: new carry");
  }
  // 4. clip, pooled with the stream state
  if (b.nsub > 0) {
    const ClipJob cj = make_clip_job(b.nsub, F, r->stat, r->cstat, st.protect, st.cfg.kappa,
                                     b.pl.max_iter, st.state, r->mask, sl.dstats, sl.ws);
    e = launch_clip(cj, s);
    if (e != hipSuccess) return dev(e, "rfi_submit: clip");
    // per-beam stage: its partial sums reuse the clip's workspace (larger)
    if (r->bmask) {
      e = launch_eigvec_flag(n, b.nsub, F, r->v1, r->mask, r->cstat, st.protect, st.cfg.kappa_v,
                             r->bmask, nullptr, nullptr, sl.ws, s);
      if (e != hipSuccess) return dev(e, "rfi_submit: per-beam stage");
    }
    if ((e = hipMemcpyAsync(sl.hstats, sl.dstats, sizeof(rfi_flag_stats), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      return dev(e, "rfi_submit: clip summary");
  }
  if ((e = hipEventRecord(st.last, s)) != hipSuccess) return dev(e, "rfi_submit: event");
  st.has_last = true;
  r->nsub = b.nsub;
  r->carried = b.carried;
  r->carry_after = b.carry_after;
  st.carry_samples = b.carry_after;
  return RFI_OK;
}

bool rfi_session::admit(rfi::Request* r) {
  using namespace rfi;
  StreamCtx& st = *streams.at(r->stream_id);
  BlockPlan b;
  if (st.failed || plan_block(st, r->blk.nsamp, &b, "rfi_submit") != RFI_OK) {
    r->status = st.failed ? RFI_E_DEVICE : RFI_E_INVALID;
    r->st = RState::Done;
    r->t_admit = r->t_done = now_us();
    st.queued--;
    cv_done.notify_all();
    return true;
  }
  const int64_t run = input_bytes(r->blk) + (int64_t)b.ws;
  const int64_t res = (int64_t)b.res;
  if (charged + run + res > budget && running > 0) return false;
  int si = -1;
  for (int i = 0; i < (int)slots.size(); ++i)
    if (!slots[i].req) { si = i; break; }
  if (si < 0) return false;
  Slot& sl = slots[si];
  r->t_admit = now_us();
  st.queued--;
  bool launched = false;
  const rfi_status rs = enqueue(r, sl, st, &launched);
  r->charge_run = run;
  r->charge_res = res;
  charged += run + res;
  if (rs != RFI_OK && !launched) {
    // nothing of this block reached the device
    r->status = rs;
    r->st = RState::Done;
    r->t_done = now_us();
    charged -= r->charge_run;
    r->charge_run = 0;
    cv_done.notify_all();
    return true;
  }
  if (rs != RFI_OK) {
    // part of the block is enqueued: it keeps the slot (and its buffers stay
    // alive) until that work has run, and the stream's carry and clip state
    // are no longer defined
    r->pending = rs;
    st.failed = true;
  }
  // completion: the slot's event, and a host function that rings the doorbell
  sl.poll = false;
  if (hipEventRecord(sl.done, sl.s) != hipSuccess) {
    (void)hipStreamSynchronize(sl.s);   // cannot track it: wait here (error path)
    sl.poll = true;
  } else if (hipLaunchHostFunc(sl.s, slot_bell, &bells[si]) != hipSuccess) {
    sl.poll = true;                      // fall back to querying the event
  }
  r->st = RState::Running;
  r->slot = si;
  sl.req = r;
  st.inflight++;
  running++;
  return true;
}

void rfi_session::finish(rfi::Slot& sl, bool ok) {
  using namespace rfi;
  Request* r = sl.req;
  StreamCtx& st = *streams.at(r->stream_id);
  if (!ok) {
    r->status = RFI_E_DEVICE;
  } else if (r->pending != RFI_OK) {
    r->status = r->pending;
  } else if (r->nsub > 0) {
    r->flag = *sl.hstats;
  }
  r->st = RState::Done;
  r->t_done = now_us();
  r->slot = -1;
  sl.req = nullptr;
  charged -= r->charge_run;
  r->charge_run = 0;
  st.inflight--;
  running--;
  cv_done.notify_all();
}

void rfi_session::scheduler() {
  using namespace rfi;
  (void)hipSetDevice(device);
  std::vector<unsigned char> rung(slots.size(), 0);
  for (;;) {
    bool any_poll = false;
    {
      std::lock_guard<std::mutex> g(db_mu);
      db_rung = false;
      rung.swap(db_slot);
      std::fill(db_slot.begin(), db_slot.end(), 0);
    }
    std::unique_lock<std::mutex> lk(mu);
    // completions: slots whose host function has run, and slots without one
    for (int i = 0; i < (int)slots.size(); ++i) {
      Slot& sl = slots[i];
      if (!sl.req || !(rung[i] || sl.poll)) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) finish(sl, true);
      else if (q != hipErrorNotReady) finish(sl, false);
      else if (rung[i]) sl.poll = true;    // rung before the event reads done: query again
    }
    // admissions: submission order; a stream's later block waits behind its
    // earlier queued one, other streams may pass
    std::vector<int> blocked;
    for (auto it = queue.begin(); it != queue.end();) {
      Request* r = *it;
      if (std::find(blocked.begin(), blocked.end(), r->stream_id) != blocked.end()) {
        ++it;
        continue;
      }
      if (admit(r)) {
        it = queue.erase(it);
      } else {
        blocked.push_back(r->stream_id);
        ++it;
      }
    }
    if (stop && queue.empty() && running == 0) break;
    for (const Slot& sl : slots) any_poll |= sl.req && sl.poll;
    lk.unlock();
    std::unique_lock<std::mutex> dl(db_mu);
    if (any_poll)
      db_cv.wait_for(dl, std::chrono::microseconds(200), [&] { return db_rung; });
    else
      db_cv.wait(dl, [&] { return db_rung; });
  }
}

extern "C" {

rfi_status rfi_session_create(const rfi_session_config* cfg, rfi_session** out) {
  rfi::clear_error();
  const char* who = "rfi_session_create";
  if (!out) return fail(RFI_E_INVALID, "%s: out is NULL", who);
  *out = nullptr;
  rfi_session_config c{0, 8, rfi::kDefaultBudget, nullptr};
  if (cfg) c = *cfg;
  if (c.tune && (c.tune->n < 0 || c.tune->n > RFI_TUNE_MAX))
    return fail(RFI_E_INVALID, "%s: tune table with %d entries", who, c.tune->n);
  if (c.max_inflight == 0) c.max_inflight = 8;
  if (c.hbm_budget == 0) c.hbm_budget = rfi::kDefaultBudget;
  if (c.max_inflight < 1 || c.max_inflight > rfi::kMaxSlots)
    return fail(RFI_E_INVALID, "%s: max_inflight %d outside 1..%d", who, c.max_inflight,
                rfi::kMaxSlots);
  if (c.hbm_budget < 0) return fail(RFI_E_INVALID, "%s: negative budget", who);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(RFI_E_DEVICE, "%s: no HIP device", who);
  if (c.device < 0 || c.device >= ndev)
    return fail(RFI_E_INVALID, "%s: device %d outside 0..%d", who, c.device, ndev - 1);
  std::unique_ptr<rfi_session> s(new rfi_session);
  s->device = c.device;
  s->max_slots = c.max_inflight;
  s->budget = c.hbm_budget;
  if (c.tune) {
    s->tune = *c.tune;
    s->has_tune = true;
  }
  s->t0 = rfi::Clock::now();
  rfi::DeviceGuard g(s->device);
  s->slots.resize(s->max_slots);
  s->db_slot.assign(s->max_slots, 0);
  s->bells.resize(s->max_slots);
  for (int i = 0; i < s->max_slots; ++i) s->bells[i] = rfi::SlotBell{s.get(), i};
  for (rfi::Slot& sl : s->slots) {
    if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
        (e = sl.ev.init()) != hipSuccess ||
        (e = hipMalloc((void**)&sl.dstats, sizeof(rfi_flag_stats))) != hipSuccess ||
        (e = hipHostMalloc((void**)&sl.hstats, sizeof(rfi_flag_stats), 0)) != hipSuccess) {
      rfi_session_destroy(s.release());
      return rfi::check_hip(e, "rfi_session_create: slot");
    }
  }
  if ((e = hipStreamCreateWithFlags(&s->free_stream, hipStreamNonBlocking)) != hipSuccess) {
    rfi_session_destroy(s.release());
    return rfi::check_hip(e, "rfi_session_create: stream");
  }
  rfi_session* raw = s.release();
  raw->sched = std::thread([raw] { raw->scheduler(); });
  *out = raw;
  return RFI_OK;
}

void rfi_session_destroy(rfi_session* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (rfi::Request* r : s->queue) {
      r->status = RFI_E_CANCELLED;
      r->st = rfi::RState::Done;
      s->streams.at(r->stream_id)->queued--;
    }
    s->queue.clear();
    s->stop = true;
  }
  s->ring();
  if (s->sched.joinable()) s->sched.join();
  rfi::DeviceGuard g(s->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : s->reqs)
    if (kv.second->res) (void)hipFree(kv.second->res);
  for (auto& kv : s->pool)
    for (void* p : kv.second) (void)hipFree(p);
  for (auto& kv : s->streams) {
    rfi::StreamCtx& st = *kv.second;
    if (st.protect) (void)hipFree(st.protect);
    if (st.state) (void)hipFree(st.state);
    if (st.carry) (void)hipFree(st.carry);
    if (st.last) (void)hipEventDestroy(st.last);
  }
  for (rfi::Slot& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.ws) (void)hipFree(sl.ws);
    if (sl.dstats) (void)hipFree(sl.dstats);
    if (sl.hstats) (void)hipHostFree(sl.hstats);
    sl.ev.destroy();
    if (sl.s) (void)hipStreamDestroy(sl.s);
  }
  if (s->free_stream) (void)hipStreamDestroy(s->free_stream);
  delete s;
}

rfi_status rfi_stream_open(rfi_session* s, const rfi_stream_config* c, int32_t* stream_id) {
  rfi::clear_error();
  const char* who = "rfi_stream_open";
  if (!s || !c || !stream_id) return fail(RFI_E_INVALID, "%s: NULL argument", who);
  rfi_stream_config cfg = *c;
  if (cfg.eig_precision == 0) cfg.eig_precision = 32;
  if (cfg.max_sweeps == 0) cfg.max_sweeps = 12;
  if (cfg.max_iter == 0) cfg.max_iter = 50;
  if (cfg.L < 1 || cfg.L > RFI_MAX_COUNT_LONG)
    return fail(RFI_E_INVALID, "%s: L %d outside 1..%d", who, cfg.L, RFI_MAX_COUNT_LONG);
  if (!(cfg.kappa >= 0.0)) return fail(RFI_E_INVALID, "%s: kappa must be >= 0", who);
  if (cfg.beam_stage != 0 && cfg.beam_stage != 1)
    return fail(RFI_E_INVALID, "%s: beam_stage must be 0 or 1", who);
  if (cfg.beam_stage && !(cfg.kappa_v >= 0.0))
    return fail(RFI_E_INVALID, "%s: kappa_v must be >= 0", who);
  if (cfg.max_iter < 1) return fail(RFI_E_INVALID, "%s: max_iter %d < 1", who, cfg.max_iter);
  rfi::ProcessPlan pl;
  rfi_process_params p{};
  p.L = cfg.L;
  p.nsub = 1;
  p.eig_precision = cfg.eig_precision;
  p.max_sweeps = cfg.max_sweeps;
  p.max_iter = cfg.max_iter;
  p.kappa = cfg.kappa;
  const rfi_tune_entry* te = s->has_tune ? rfi::find_tune(&s->tune, cfg.nbeam) : nullptr;
  rfi_status rs = rfi::resolve_process(cfg.nbeam, cfg.nchan, &p, &pl, who, te);
  if (rs != RFI_OK) return rs;
  std::unique_ptr<rfi::StreamCtx> st(new rfi::StreamCtx);
  st->cfg = cfg;
  if (te) {
    st->tuned = true;
    st->te = *te;
  }
  st->cfg.protect_chan = nullptr;
  rfi::DeviceGuard g(s->device);
  hipError_t e;
  auto bad = [&](hipError_t err) {
    if (st->protect) (void)hipFree(st->protect);
    if (st->state) (void)hipFree(st->state);
    if (st->carry) (void)hipFree(st->carry);
    if (st->last) (void)hipEventDestroy(st->last);
    return rfi::check_hip(err, "rfi_stream_open");
  };
  if ((e = hipMalloc((void**)&st->state, sizeof(rfi_stream_state))) != hipSuccess ||
      (e = hipMemset(st->state, 0, sizeof(rfi_stream_state))) != hipSuccess ||
      (e = hipMalloc((void**)&st->carry, st->carry_bytes())) != hipSuccess ||
      (e = hipMemset(st->carry, 0, st->carry_bytes())) != hipSuccess ||
      (e = hipEventCreateWithFlags(&st->last, hipEventDisableTiming)) != hipSuccess)
    return bad(e);
  if (c->protect_chan) {
    if ((e = hipMalloc((void**)&st->protect, cfg.nchan)) != hipSuccess ||
        (e = hipMemcpy(st->protect, c->protect_chan, cfg.nchan, hipMemcpyHostToDevice)) !=
            hipSuccess)
      return bad(e);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  st->id = s->next_stream++;
  *stream_id = st->id;
  s->streams[st->id] = std::move(st);
  return RFI_OK;
}

rfi_status rfi_submit(rfi_session* s, int32_t stream_id, const rfi_block* blk, uint64_t user_tag,
                      uint64_t* ticket) {
  rfi::clear_error();
  const char* who = "rfi_submit";
  if (!s || !blk || !ticket) return fail(RFI_E_INVALID, "%s: NULL argument", who);
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->streams.find(stream_id);
  if (it == s->streams.end()) return fail(RFI_E_INVALID, "%s: unknown stream %d", who, stream_id);
  rfi::StreamCtx& st = *it->second;
  if (blk->nbeam != st.cfg.nbeam || blk->nchan != st.cfg.nchan)
    return fail(RFI_E_INVALID, "%s: block shape %d x %d differs from the stream's %d x %d", who,
                blk->nbeam, blk->nchan, st.cfg.nbeam, st.cfg.nchan);
  if (blk->nsamp < 0) return fail(RFI_E_INVALID, "%s: nsamp < 0", who);
  rfi::BeamPtrs bp;
  rfi_status rs = rfi::validate_block(blk, 0, st.cfg.L, 0, who, &bp, RFI_MAX_COUNT_LONG);
  if (rs != RFI_OK) return rs;
  if (rfi::input_bytes(*blk) > s->budget)
    return fail(RFI_E_BUDGET, "%s: block of %lld bytes exceeds the budget of %lld", who,
                (long long)rfi::input_bytes(*blk), (long long)s->budget);
  std::unique_ptr<rfi::Request> r(new rfi::Request);
  r->beams = st.cfg.beam_stage != 0;
  r->ticket = s->next_ticket++;
  r->tag = user_tag;
  r->stream_id = stream_id;
  r->blk = *blk;
  r->t_submit = s->now_us();
  *ticket = r->ticket;
  st.queued++;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  lk.unlock();
  s->ring();
  return RFI_OK;
}

static void fill_result(const rfi::Request& r, rfi_result* out) {
  std::memset(out, 0, sizeof(*out));
  out->ticket = r.ticket;
  out->user_tag = r.tag;
  out->stream_id = r.stream_id;
  out->status = r.status;
  out->nsub = r.nsub;
  out->nchan = r.blk.nchan;
  out->carried = r.carried;
  out->carry_samples = r.carry_after;
  out->stat = r.stat;
  out->cell_status = r.cstat;
  out->mask = r.mask;
  out->flag = r.flag;
  out->t_submit_us = r.t_submit;
  out->t_admit_us = r.t_admit;
  out->t_done_us = r.t_done;
  out->v1 = r.v1;
  out->beam_mask = r.bmask;
}

rfi_status rfi_poll(rfi_session* s, uint64_t ticket, rfi_result* r) {
  rfi::clear_error();
  if (!s || !r) return fail(RFI_E_INVALID, "rfi_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_poll: unknown ticket %llu",
                                       (unsigned long long)ticket);
  if (it->second->st != rfi::RState::Done) return RFI_E_NOT_READY;
  fill_result(*it->second, r);
  return RFI_OK;
}

rfi_status rfi_wait(rfi_session* s, uint64_t ticket, int64_t timeout_us, rfi_result* r) {
  rfi::clear_error();
  if (!s || !r) return fail(RFI_E_INVALID, "rfi_wait: NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_wait: unknown ticket %llu",
                                       (unsigned long long)ticket);
  rfi::Request* q = it->second.get();
  auto ready = [&] { return q->st == rfi::RState::Done; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(RFI_E_TIMEOUT, "rfi_wait: ticket %llu not done after %lld us",
                (unsigned long long)ticket, (long long)timeout_us);
  }
  fill_result(*q, r);
  return RFI_OK;
}

rfi_status rfi_cancel(rfi_session* s, uint64_t ticket) {
  rfi::clear_error();
  if (!s) return fail(RFI_E_INVALID, "rfi_cancel: NULL session");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_cancel: unknown ticket");
  rfi::Request* r = it->second.get();
  if (r->st != rfi::RState::Queued) return RFI_E_NOT_READY;
  s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
  s->streams.at(r->stream_id)->queued--;
  r->status = RFI_E_CANCELLED;
  r->st = rfi::RState::Done;
  r->t_admit = r->t_done = s->now_us();
  s->cv_done.notify_all();
  return RFI_OK;
}

rfi_status rfi_result_copy(rfi_session* s, uint64_t ticket, double* stat, uint8_t* cell_status,
                           uint8_t* mask) {
  rfi::clear_error();
  if (!s) return fail(RFI_E_INVALID, "rfi_result_copy: NULL session");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_result_copy: unknown ticket");
  rfi::Request* r = it->second.get();
  if (r->st != rfi::RState::Done)
    return fail(RFI_E_NOT_READY, "rfi_result_copy: ticket still queued or running");
  const size_t n = (size_t)r->nsub * r->blk.nchan;
  if (n == 0 || !r->res) return RFI_OK;
  rfi::DeviceGuard g(s->device);
  hipError_t e = hipSuccess;
  if (stat) e = hipMemcpy(stat, r->stat, n * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess && cell_status)
    e = hipMemcpy(cell_status, r->cstat, n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && mask) e = hipMemcpy(mask, r->mask, n, hipMemcpyDeviceToHost);
  return rfi::check_hip(e, "rfi_result_copy");
}

rfi_status rfi_result_copy_beams(rfi_session* s, uint64_t ticket, float* v1, uint8_t* beam_mask) {
  rfi::clear_error();
  if (!s) return fail(RFI_E_INVALID, "rfi_result_copy_beams: NULL session");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_result_copy_beams: unknown ticket");
  rfi::Request* r = it->second.get();
  if (r->st != rfi::RState::Done)
    return fail(RFI_E_NOT_READY, "rfi_result_copy_beams: ticket still queued or running");
  if (!r->beams)
    return fail(RFI_E_INVALID, "rfi_result_copy_beams: the stream has no per-beam stage");
  const size_t n = (size_t)r->nsub * r->blk.nchan * r->blk.nbeam;
  if (n == 0 || !r->bmask) return RFI_OK;
  rfi::DeviceGuard g(s->device);
  hipError_t e = hipSuccess;
  if (v1) e = hipMemcpy(v1, r->v1, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && beam_mask) e = hipMemcpy(beam_mask, r->bmask, n, hipMemcpyDeviceToHost);
  return rfi::check_hip(e, "rfi_result_copy_beams");
}

rfi_status rfi_result_release(rfi_session* s, uint64_t ticket) {
  rfi::clear_error();
  if (!s) return fail(RFI_E_INVALID, "rfi_result_release: NULL session");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(RFI_E_INVALID, "rfi_result_release: unknown ticket");
  rfi::Request* r = it->second.get();
  if (r->st != rfi::RState::Done)
    return fail(RFI_E_NOT_READY, "rfi_result_release: ticket still queued or running");
  rfi::DeviceGuard g(s->device);
  if (r->res) s->res_put(r->res, r->res_cls);
  s->charged -= r->charge_res;
  s->reqs.erase(it);
  lk.unlock();
  s->ring();   // budget freed
  return RFI_OK;
}

// Wait (holding lk) until the stream has nothing queued or running.
static rfi::StreamCtx* idle_stream(rfi_session* s, std::unique_lock<std::mutex>& lk, int id,
                                   const char* who) {
  auto it = s->streams.find(id);
  if (it == s->streams.end()) {
    fail(RFI_E_INVALID, "%s: unknown stream %d", who, id);
    return nullptr;
  }
  rfi::StreamCtx* st = it->second.get();
  s->cv_done.wait(lk, [&] { return st->queued == 0 && st->inflight == 0; });
  return st;
}

rfi_status rfi_stream_close(rfi_session* s, int32_t stream_id) {
  rfi::clear_error();
  if (!s) return fail(RFI_E_INVALID, "rfi_stream_close: NULL session");
  std::unique_lock<std::mutex> lk(s->mu);
  rfi::StreamCtx* st = idle_stream(s, lk, stream_id, "rfi_stream_close");
  if (!st) return RFI_E_INVALID;
  rfi::DeviceGuard g(s->device);
  (void)hipEventSynchronize(st->last);
  if (st->protect) (void)hipFree(st->protect);
  (void)hipFree(st->state);
  (void)hipFree(st->carry);
  (void)hipEventDestroy(st->last);
  s->streams.erase(stream_id);
  return RFI_OK;
}

namespace {
struct ExportHeader {
  uint32_t magic, version;
  int32_t nbeam, nchan, L, pad;
  int64_t carry_samples;
};
constexpr uint32_t kMagic = 0x52464953u;   // "RFIS"
}  // namespace

rfi_status rfi_stream_export(rfi_session* s, int32_t stream_id, void* host_buf, size_t* nbytes) {
  rfi::clear_error();
  const char* who = "rfi_stream_export";
  if (!s || !nbytes) return fail(RFI_E_INVALID, "%s: NULL argument", who);
  std::unique_lock<std::mutex> lk(s->mu);
  rfi::StreamCtx* st = idle_stream(s, lk, stream_id, who);
  if (!st) return RFI_E_INVALID;
  const size_t need = sizeof(ExportHeader) + sizeof(rfi_stream_state) + st->carry_bytes();
  if (!host_buf) {
    *nbytes = need;
    return RFI_OK;
  }
  if (*nbytes < need) return fail(RFI_E_INVALID, "%s: buffer of %zu bytes < %zu", who, *nbytes, need);
  rfi::DeviceGuard g(s->device);
  hipError_t e = hipEventSynchronize(st->last);
  ExportHeader h{kMagic, 1, st->cfg.nbeam, st->cfg.nchan, st->cfg.L, 0, st->carry_samples};
  char* p = (char*)host_buf;
  std::memcpy(p, &h, sizeof(h));
  if (e == hipSuccess)
    e = hipMemcpy(p + sizeof(h), st->state, sizeof(rfi_stream_state), hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(p + sizeof(h) + sizeof(rfi_stream_state), st->carry, st->carry_bytes(),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return rfi::check_hip(e, who);
  *nbytes = need;
  return RFI_OK;
}

rfi_status rfi_stream_import(rfi_session* s, int32_t stream_id, const void* host_buf,
                             size_t nbytes) {
  rfi::clear_error();
  const char* who = "rfi_stream_import";
  if (!s || !host_buf) return fail(RFI_E_INVALID, "%s: NULL argument", who);
  std::unique_lock<std::mutex> lk(s->mu);
  rfi::StreamCtx* st = idle_stream(s, lk, stream_id, who);
  if (!st) return RFI_E_INVALID;
  const size_t need = sizeof(ExportHeader) + sizeof(rfi_stream_state) + st->carry_bytes();
  ExportHeader h;
  if (nbytes < sizeof(h)) return fail(RFI_E_INVALID, "%s: buffer too small", who);
  std::memcpy(&h, host_buf, sizeof(h));
  if (h.magic != kMagic || h.version != 1 || h.nbeam != st->cfg.nbeam ||
      h.nchan != st->cfg.nchan || h.L != st->cfg.L || nbytes != need || h.carry_samples < 0 ||
      h.carry_samples >= st->cfg.L)
    return fail(RFI_E_INVALID, "%s: checkpoint does not match the stream", who);
  rfi::DeviceGuard g(s->device);
  const char* p = (const char*)host_buf;
  hipError_t e = hipEventSynchronize(st->last);
  if (e == hipSuccess)
    e = hipMemcpy(st->state, p + sizeof(h), sizeof(rfi_stream_state), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(st->carry, p + sizeof(h) + sizeof(rfi_stream_state), st->carry_bytes(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return rfi::check_hip(e, who);
  st->carry_samples = h.carry_samples;
  return RFI_OK;
}

}  // extern "C"
