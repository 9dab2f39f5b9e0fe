// A fake device for host-only tests of the serving runtime (csrc/serve.cpp).
//
// TEST INFRASTRUCTURE ONLY: it replaces the HIP runtime calls and the
// library's kernel launchers that serve.cpp uses, so that the scheduler
// (admission, HBM budget, per-stream ordering, carries, cancel, close,
// allocation and launch failures) runs on the CPU, under ThreadSanitizer.
//
// Model: "device memory" is host memory; every stream is a worker thread
// that runs its operations in order (work items that sleep and then apply a
// side effect, event records, waits on events, copies, host functions).
// The launchers' side effects are simple functions of their inputs, so a
// driver can check which data each block read and in which order the blocks
// of one stream ran:
//   - sums launch (carry): count[0] = L or count[0] += L;
//   - eigen stage of the carried row: stat[j] = 100000 + count[0];
//   - eigen stage of full sub-intervals: stat[k nchan + j] = beam 0's byte at
//     (t0 + k L, j), status = 0;
//   - clip: out->iterations = state->nblocks (then nblocks + 1), out->nfit =
//     ncell, mask = (stat > 200).
// Failure injection: fake_fail_alloc_in(k) makes the k-th allocation from now
// fail; fake_fail_launch_in(k) the k-th launcher call from now.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "pipeline.h"

// ---------------------------------------------------------------------------
// knobs for the driver
static std::atomic<int> g_fail_alloc{0};     // > 0: countdown to a failing allocation
static std::atomic<int> g_fail_launch{0};    // > 0: countdown to a failing launcher call
static std::atomic<int> g_work_us{200};      // duration of one work item
static std::atomic<int> g_errors{0};         // inconsistencies seen by the fake kernels

extern "C" void fake_fail_alloc_in(int k) { g_fail_alloc = k; }
extern "C" void fake_fail_launch_in(int k) { g_fail_launch = k; }
extern "C" void fake_set_work_us(int us) { g_work_us = us; }
extern "C" int fake_errors() { return g_errors.load(); }

static bool take(std::atomic<int>& c) {
  int v = c.load();
  while (v > 0) {
    if (c.compare_exchange_weak(v, v - 1)) return v == 1;
  }
  return false;
}

// ---------------------------------------------------------------------------
// events and streams
struct ihipEvent_t {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0, completed = 0;
};

namespace {

struct Op {
  enum Kind { Work, Record, Wait, Host } kind;
  std::function<void()> fn;   // Work effect / Host function
  int us = 0;
  ihipEvent_t* ev = nullptr;
  uint64_t gen = 0;
};

}  // namespace

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Op> q;
  bool stop = false;
  std::thread th;
  void run() {
    for (;;) {
      Op op;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) return;
        op = std::move(q.front());
        q.pop_front();
      }
      switch (op.kind) {
        case Op::Work:
          if (op.us > 0) std::this_thread::sleep_for(std::chrono::microseconds(op.us));
          if (op.fn) op.fn();
          break;
        case Op::Host:
          op.fn();
          break;
        case Op::Record: {
          std::lock_guard<std::mutex> g(op.ev->mu);
          if (op.gen > op.ev->completed) op.ev->completed = op.gen;
          op.ev->cv.notify_all();
          break;
        }
        case Op::Wait: {
          std::unique_lock<std::mutex> g(op.ev->mu);
          op.ev->cv.wait(g, [&] { return op.ev->completed >= op.gen; });
          break;
        }
      }
    }
  }
  void push(Op op) {
    {
      std::lock_guard<std::mutex> g(mu);
      q.push_back(std::move(op));
    }
    cv.notify_one();
  }
};

namespace {

std::mutex g_streams_mu;
std::vector<ihipStream_t*> g_streams;
ihipStream_t* g_null = nullptr;

ihipStream_t* new_stream() {
  ihipStream_t* s = new ihipStream_t;
  s->th = std::thread([s] { s->run(); });
  std::lock_guard<std::mutex> g(g_streams_mu);
  g_streams.push_back(s);
  return s;
}

ihipStream_t* resolve(hipStream_t s) {
  if (s) return s;
  std::lock_guard<std::mutex> g(g_streams_mu);
  if (!g_null) {
    g_null = new ihipStream_t;
    g_null->th = std::thread([] { g_null->run(); });
  }
  return g_null;
}

uint64_t record(ihipEvent_t* e, ihipStream_t* s) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> g(e->mu);
    gen = ++e->recorded;
  }
  Op op{Op::Record};
  op.ev = e;
  op.gen = gen;
  s->push(std::move(op));
  return gen;
}

void sync_stream(ihipStream_t* s) {
  ihipEvent_t e;
  const uint64_t gen = record(&e, s);
  std::unique_lock<std::mutex> g(e.mu);
  e.cv.wait(g, [&] { return e.completed >= gen; });
}

void work(hipStream_t s, std::function<void()> fn) {
  Op op{Op::Work};
  op.fn = std::move(fn);
  op.us = g_work_us.load();
  resolve(s)->push(std::move(op));
}

}  // namespace

// ---------------------------------------------------------------------------
// the HIP runtime calls serve.cpp makes
extern "C" {

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new_stream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->th.join();
  std::lock_guard<std::mutex> g(g_streams_mu);
  for (auto& p : g_streams)
    if (p == s) p = nullptr;
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  sync_stream(resolve(s));
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  std::vector<ihipStream_t*> all;
  {
    std::lock_guard<std::mutex> g(g_streams_mu);
    for (auto* p : g_streams)
      if (p) all.push_back(p);
  }
  for (auto* p : all) sync_stream(p);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> g(e->mu);
    gen = e->recorded;
  }
  Op op{Op::Wait};
  op.ev = e;
  op.gen = gen;
  resolve(s)->push(std::move(op));
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) {
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  record(e, resolve(s));
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> g(e->mu);
  return e->completed >= e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> g(e->mu);
  const uint64_t gen = e->recorded;
  e->cv.wait(g, [&] { return e->completed >= gen; });
  return hipSuccess;
}

hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* arg) {
  Op op{Op::Host};
  op.fn = [fn, arg] { fn(arg); };
  resolve(s)->push(std::move(op));
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t n) {
  if (take(g_fail_alloc)) return hipErrorOutOfMemory;
  *p = std::calloc(n ? n : 1, 1);
  return hipSuccess;
}
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipFreeAsync(void* p, hipStream_t s) {
  Op op{Op::Work};
  op.fn = [p] { std::free(p); };
  resolve(s)->push(std::move(op));
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemset(void* p, int v, size_t n) {
  std::memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
  Op op{Op::Work};
  op.fn = [d, s, n] { std::memcpy(d, s, n); };
  resolve(st)->push(std::move(op));
  return hipSuccess;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// the library pieces serve.cpp calls
namespace rfi {

static thread_local char t_err[512];

void clear_error() { t_err[0] = 0; }
rfi_status fail(rfi_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return code;
}
rfi_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return RFI_OK;
  fail(RFI_E_DEVICE, "%s: fake device error %d", what, (int)e);
  return e == hipErrorOutOfMemory ? RFI_E_NOMEM : RFI_E_DEVICE;
}

rfi_status validate_block(const rfi_block* blk, int64_t, int32_t L, int32_t, const char* who,
                          BeamPtrs* bp, int32_t max_L) {
  if (!blk || blk->nbeam < 2 || blk->nbeam > RFI_MAX_BEAMS || blk->nchan < 1 ||
      blk->nsamp < 0 || blk->row_stride < blk->nchan || L < 1 || L > max_L)
    return fail(RFI_E_INVALID, "%s: bad block", who);
  std::memset(bp, 0, sizeof(*bp));
  for (int b = 0; b < blk->nbeam; ++b) {
    if (!blk->beam[b]) return fail(RFI_E_INVALID, "%s: NULL beam", who);
    bp->p[b] = (const uint8_t*)blk->beam[b];
  }
  return RFI_OK;
}

const rfi_tune_entry* find_tune(const rfi_tune_table* t, int nbeam) {
  if (!t) return nullptr;
  for (int i = 0; i < t->n; ++i)
    if (nbeam >= t->e[i].nbeam_lo && nbeam <= t->e[i].nbeam_hi) return &t->e[i];
  return nullptr;
}

rfi_status resolve_process(int nbeam, int nchan, const rfi_process_params* p, ProcessPlan* pl,
                           const char* who, const rfi_tune_entry*) {
  if (nbeam < 2 || nbeam > RFI_MAX_BEAMS || nchan < 1 || p->nsub < 0)
    return fail(RFI_E_INVALID, "%s: bad sizes", who);
  pl->nbeam = nbeam;
  pl->nchan = nchan;
  pl->nsub = p->nsub;
  pl->group = p->nsub > 0 ? p->nsub : 1;
  pl->nslot = 1;
  pl->L = p->L;
  pl->max_iter = p->max_iter ? p->max_iter : 50;
  pl->kappa = p->kappa;
  pl->slot = (size_t)pl->group * nchan * 8;
  pl->flag_ws = 256;
  pl->ws_bytes = pl->flag_ws + pl->slot;
  return RFI_OK;
}

size_t clip_workspace_size(int64_t ncell) { return 256 + (size_t)ncell * 8; }

ClipJob make_clip_job(int nsub, int nchan, const double* stat, const uint8_t* status,
                      const uint8_t* protect, double kappa, int max_iter,
                      rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out, void* ws,
                      int64_t) {
  ClipJob j{};
  j.nsub = nsub;
  j.nchan = nchan;
  j.max_iter = max_iter;
  j.kappa = kappa;
  j.stat = stat;
  j.status = status;
  j.protect = protect;
  j.state = state;
  j.mask = mask;
  j.out = out;
  j.ws = ws;
  return j;
}

hipError_t PipeEvents::init() {
  ready = true;
  return hipSuccess;
}
void PipeEvents::destroy() { ready = false; }

hipError_t launch_ccm_mfma(const BeamPtrs&, int, int, int64_t, int64_t, int L, int nsub,
                           int32_t*, int32_t*, int32_t* count, int accumulate, int, hipStream_t s,
                           const CcmTune*, int, int64_t, int) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  if (nsub != 1) g_errors++;
  work(s, [=] { count[0] = accumulate ? count[0] + L : L; });
  return hipSuccess;
}

size_t ccm_long_tmp_bytes(int, int, int) { return 256; }

hipError_t launch_ccm_long(const BeamPtrs&, int, int, int64_t, int64_t, int L, int nsub, int64_t*,
                           int32_t* count, void* tmp, hipStream_t s, const CcmTune*,
                           int accumulate) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  if (nsub != 1 || !tmp) g_errors++;
  work(s, [=] { count[0] = accumulate ? count[0] + L : L; });
  return hipSuccess;
}

hipError_t launch_eig(const EigArgs& a, const rfi_eig_params&, hipStream_t s, int) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  const EigArgs g = a;
  work(s, [g] {
    for (int j = 0; j < g.nchan; ++j) {
      g.stat[j] = 100000.0 + g.count[0];
      g.status[j] = 0;
    }
  });
  return hipSuccess;
}

hipError_t enqueue_eig_groups(const BeamPtrs& bp, int64_t row_stride, int64_t t0, int L,
                              const ProcessPlan& pl, double* stat, uint8_t* status, float*,
                              float*, int64_t, void*, PipeEvents& ev, hipStream_t s) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  if (!ev.ready) g_errors++;
  const uint8_t* b0 = bp.p[0];
  const int nsub = pl.nsub, F = pl.nchan;
  work(s, [=] {
    for (int k = 0; k < nsub; ++k)
      for (int j = 0; j < F; ++j) {
        stat[(int64_t)k * F + j] = b0[(t0 + (int64_t)k * L) * row_stride + j];
        status[(int64_t)k * F + j] = 0;
      }
  });
  return hipSuccess;
}

hipError_t launch_eigvec_flag(int nbeam, int nsub, int nchan, const float*, const uint8_t* mask,
                              const uint8_t*, const uint8_t*, double, uint8_t* beam_mask,
                              double*, double*, void* ws, hipStream_t s) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  if (!ws) g_errors++;
  const int64_t n = (int64_t)nsub * nchan;
  work(s, [=] {
    for (int b = 0; b < nbeam; ++b)
      for (int64_t c = 0; c < n; ++c) beam_mask[b * n + c] = mask[c];
  });
  return hipSuccess;
}

hipError_t launch_clip(const ClipJob& j, hipStream_t s) {
  if (take(g_fail_launch)) return hipErrorLaunchFailure;
  const ClipJob c = j;
  work(s, [c] {
    const int64_t n = (int64_t)c.nsub * c.nchan;
    int64_t nf = 0;
    for (int64_t i = 0; i < n; ++i) {
      c.mask[i] = c.stat[i] > 200.0;
      nf += c.mask[i];
    }
    c.out->iterations = (int32_t)c.state->nblocks;
    c.out->converged = 1;
    c.out->nflag = nf;
    c.out->nfit = n;
    c.state->nblocks++;
  });
  return hipSuccess;
}

}  // namespace rfi

extern "C" const char* rfi_last_error(void) { return rfi::t_err; }
