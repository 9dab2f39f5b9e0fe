// Internal pieces of the pipelined whole-block path, shared by
// rfi_process_block and the serving session.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "internal.h"
#include "rfi.h"

namespace rfi {

constexpr int kRing = 3;   // sum slots in flight between the two streams

// Sizes and settings of one whole-block call, defaults applied.
struct ProcessPlan {
  int nbeam = 0, nchan = 0, nsub = 0, group = 1, nslot = 1, max_iter = 50;
  int L = 0;
  bool longL = false;    // L > RFI_MAX_COUNT: int64 sums in time chunks, FP64 tridiagonal solver
  double kappa = 3.0;
  rfi_eig_params eig{32, 12, 1, RFI_EIG_AUTO};
  CcmTune ct{};          // sums-engine choices (zeros = the engine's defaults)
  int eig_wg = 0;        // per-lane solver workgroup (0 = default)
  size_t flag_ws = 0;    // bytes of the clip workspace (first in the workspace)
  size_t slot = 0;       // bytes of one ring slot of sums
  size_t ws_bytes = 0;   // total workspace
};

// te: tuned launch choices for this beam count (solver, sums tile, ring depth,
// XCD grouping, per-lane workgroup), or NULL for the defaults.
rfi_status resolve_process(int nbeam, int nchan, const rfi_process_params* p, ProcessPlan* pl,
                           const char* who, const rfi_tune_entry* te = nullptr);

// Helper stream and the events that order the ring between the two streams.
struct PipeEvents {
  bool ready = false;
  hipStream_t aux = nullptr;
  hipEvent_t ccm[kRing] = {}, eig[kRing] = {}, start = nullptr, done = nullptr;
  hipError_t init();
  void destroy();
};

// Enqueue sums + eigen stage for pl.nsub sub-intervals starting at t0, in
// groups, on s and ev.aux; later work on s waits for all of it. Rows of the
// per-cell outputs: stat/status[cell], eigvals/v1[i * out_stride + cell].
hipError_t enqueue_eig_groups(const BeamPtrs& bp, int64_t row_stride, int64_t t0, int L,
                              const ProcessPlan& pl, double* stat, uint8_t* status,
                              float* eigvals, float* v1, int64_t out_stride, void* ring,
                              PipeEvents& ev, hipStream_t s);

}  // namespace rfi
