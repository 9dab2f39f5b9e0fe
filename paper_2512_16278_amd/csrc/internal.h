// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfi.h"

namespace rfi {

// Device pointers of a block's beams, passed to kernels by value.
struct BeamPtrs {
  const uint8_t* p[RFI_MAX_BEAMS];
};

inline int npair_of(int n) { return n * (n + 1) / 2; }

// One block of a batched sums launch (device descriptor). The block's
// workgroups are [wg0, wg0 + 8 ceil(nsub * nct / 8)); wg0 is a multiple of 8.
struct CcmItem {
  const uint8_t* const* beams;   // device table [nbeam] of beam pointers
  int64_t row_stride, t0;
  int32_t* sum_x;
  int32_t* sum_xy;
  int32_t* count;
  int32_t nbeam, nchan, L, nsub;
  int32_t nct, nh, wg0, layout;  // layout: as the sums engine's argument
};
// Launch choices of the MFMA sums engine (all 0 = defaults): tile = variant
// index of the beam count's tile shapes (< ccm_tile_variants), stages = cap
// of the load ring depth (2..4), group_bytes = contiguous row bytes of the
// tiles given to one XCD in turn.
struct CcmTune {
  int tile, stages, group_bytes;
};
int ccm_tile_variants(int nbeam);
// Instance class of the MFMA sums engine for a beam count: blocks of one
// class share a batched launch; cw = channels per tile, nh = epilogue passes.
struct CcmClass {
  long long key;
  int cw, nh, group_bytes;
};
hipError_t ccm_class(int nbeam, CcmClass* c, const CcmTune* t = nullptr);
// Batched sums launch over the items of one class (items in device memory,
// sorted by wg0); nbeam_of_class is any member's beam count, t its choices.
hipError_t launch_ccm_batch(int nbeam_of_class, const CcmTune* t, const CcmItem* items,
                            int nitem, int total_wg, hipStream_t s);

// Kernel launchers (return a HIP error code; arguments already validated).
// kstride: samples from the start of one sub-interval to the next (0 = L:
// back to back; longer strides sum one time chunk of long sub-intervals);
// ksplit > 1: launch sub-interval k starts at t0 + (k / ksplit) kstride +
// (k mod ksplit) L (ksplit consecutive chunks of L samples per stride).
hipError_t launch_ccm_mfma(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, int shared_cu, hipStream_t s,
                           const CcmTune* t = nullptr, int layout = 0, int64_t kstride = 0,
                           int ksplit = 1);
// Sums layouts: 0 = the C ABI's rows (sum_x[b][cell], sum_xy[pair][cell]);
// 1 = one record per cell, sum_x[cell * (nbeam + npair) + row] with rows b
// then nbeam + pair (sum_xy unused): what a one-cell-per-wave consumer reads
// with coalesced loads.
hipError_t launch_ccm_valu(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int32_t* sum_x, int32_t* sum_xy,
                           int32_t* count, int accumulate, hipStream_t s);

// Sums of sub-intervals longer than RFI_MAX_COUNT (up to RFI_MAX_COUNT_LONG):
// int64 cell records rec[cell * (nbeam + npair) + row] (rows b, then nbeam +
// pair), count[k] = L (accumulate: both added to what rec and count hold);
// tmp: ccm_long_tmp_bytes of device scratch.
size_t ccm_long_tmp_bytes(int nbeam, int nchan, int nsub);
hipError_t launch_ccm_long(const BeamPtrs& bp, int nbeam, int nchan, int64_t row_stride,
                           int64_t t0, int L, int nsub, int64_t* rec, int32_t* count, void* tmp,
                           hipStream_t s, const CcmTune* t = nullptr, int accumulate = 0);

struct EigArgs {
  int nbeam, nsub, nchan;
  const int32_t* sum_x;
  const int32_t* sum_xy;
  const int32_t* count;
  int max_sweeps, refine;
  float* eigvals;
  double* stat;
  float* v1;
  uint8_t* status;
  int64_t out_stride;  // cell stride of the eigvals / v1 rows (>= nsub * nchan)
  int layout;          // sums layout (1: cell records; 2: int64 cell records of long
                       // sub-intervals, in sum_x; the tridiagonal solver only)
};
// FP32, nbeam <= 20; wg = lanes (cells) per workgroup: 64, 128 or 256; tri
// = Householder + Sturm instead of Jacobi for the first kernel
hipError_t launch_eig_lane(const EigArgs& a, hipStream_t s, int wg = 256, bool tri = false);
hipError_t launch_eig_wave(const EigArgs& a, int precision, hipStream_t s);  // any nbeam
hipError_t launch_eig_tri(const EigArgs& a, hipStream_t s);               // any nbeam, FP64
// The eigen stage of one block with resolved parameters (solver, precision).
hipError_t launch_eig(const EigArgs& a, const rfi_eig_params& p, hipStream_t s, int lane_wg = 256);
// Batched eigen stage over the cells of several blocks, one index space:
// items[i] (device) describes block i, cell0[i] (device, ascending) is its
// first global cell, total the number of cells. The per-lane solver takes
// one template class of beam counts (eig_lane_class(n), 0 = none); the
// per-wave solver any beam counts up to max_nbeam.
int eig_lane_class(int n);
hipError_t launch_eig_lane_batch(int cls, const EigArgs* items, const int64_t* cell0, int nitem,
                                 int64_t total, hipStream_t s, int wg = 256, bool tri = false);
hipError_t launch_eig_wave_batch(int precision, int max_nbeam, const EigArgs* items,
                                 const int64_t* cell0, int nitem, int64_t total, hipStream_t s);
// The per-wave tridiagonal solver: template class of a beam count (local
// block size of its 8 x 8 lane grid; 0 = none) and its batched launch over
// items of one class.
int eig_tri_class(int n);
hipError_t launch_eig_tri_batch(int cls, const EigArgs* items, const int64_t* cell0, int nitem,
                                int64_t total, hipStream_t s, bool v1 = false);

// ArPLS bandpass of every (beam, sub-interval) from the channel sums (rows
// layout sum_x[b][cell]); z [nbeam][ncell] FP64; passes [nsub][nbeam] or NULL;
// ws: bandpass_workspace_size bytes.
size_t bandpass_workspace_size(int nbeam, int nchan, int nsub);
hipError_t launch_arpls(int nbeam, int nsub, int nchan, const int32_t* sum_x,
                        const int32_t* count, double lam, double ratio, int itermax, double* z,
                        int32_t* passes, void* ws, hipStream_t s);
// The FP64 tridiagonal solver on the non-centred matrix of the bandpass-
// subtracted power (zb [nbeam][ncell] or NULL), sums in the rows layout.
hipError_t launch_eig_tri_nc(const EigArgs& a, const double* zb, hipStream_t s);

// One clip problem (device descriptor): the cells of one block, its outputs
// and its workspace (clip_workspace_size bytes, 256-byte aligned, holding at
// most tail_cap tail entries).
struct ClipJob {
  int32_t nsub, nchan, max_iter, nparts;
  double kappa;
  const double* stat;
  const uint8_t* status;
  const uint8_t* protect;
  rfi_stream_state* state;
  uint8_t* mask;
  rfi_flag_stats* out;
  void* ws;
  int64_t tail_cap;
};
// Tail capacity the library gives a block of ncell cells, and the workspace
// bytes for it (or for an explicit capacity).
int64_t clip_tail_cap(int64_t ncell);
size_t clip_workspace_size(int64_t ncell);
size_t clip_workspace_size_for_cap(int64_t tail_cap);
// Descriptor with the scan's workgroup count filled in (tail_cap 0: the
// default capacity for the block).
ClipJob make_clip_job(int nsub, int nchan, const double* stat, const uint8_t* status,
                      const uint8_t* protect_chan, double kappa, int max_iter,
                      rfi_stream_state* state, uint8_t* mask, rfi_flag_stats* out, void* ws,
                      int64_t tail_cap = 0);
// The clip of one block (four launches on s).
hipError_t launch_clip(const ClipJob& j, hipStream_t s);
// The clips of n blocks: jobs in device memory, host_jobs the same
// descriptors on the host (grid sizes).
hipError_t launch_clip_batch(const ClipJob* jobs, const ClipJob* host_jobs, int n, hipStream_t s);
// Clip scopes: scopes bit 1 = the global clip of g (the four-launch clip for
// fit 0, a one-workgroup clip for the histogram fit 1), bit 2 = one clip per
// channel, bit 4 = one clip per sub-interval; g.mask gets the union (zeroed
// first when bit 1 is absent); chan_out [nchan] / sub_out [nsub] nullable.
hipError_t launch_clip_scoped(const ClipJob& g, int scopes, int fit, rfi_flag_stats* chan_out,
                              rfi_flag_stats* sub_out, hipStream_t s);
// The clip's exact fit for given moment sums (device arrays of n entries;
// Q1, Q2 as little-endian 64-bit limb pairs).
hipError_t launch_fit(int n, const int64_t* N, const uint64_t* Q1, const uint64_t* Q2,
                      double kappa, double* mu, double* sigma, double* thr, hipStream_t s);
// Per-beam eigenvector stage: ws holds eigvec_workspace_size bytes of
// per-workgroup partial sums.
size_t eigvec_workspace_size(int nbeam, int64_t ncell);
hipError_t launch_eigvec_flag(int nbeam, int nsub, int nchan, const float* v1,
                              const uint8_t* mask, const uint8_t* status,
                              const uint8_t* protect_chan, double kappa_v,
                              uint8_t* beam_mask, double* beam_mu, double* beam_sigma, void* ws,
                              hipStream_t s);

// Error reporting shared by the entry points (thread-local message).
void clear_error();
rfi_status fail(rfi_status code, const char* fmt, ...);
rfi_status check_hip(hipError_t e, const char* what);
// Argument checks shared by the entry points; fill bp on success.
// max_L: the longest sub-interval the caller's path takes (RFI_MAX_COUNT, or
// RFI_MAX_COUNT_LONG where int64 sums are used).
rfi_status validate_block(const rfi_block* blk, int64_t t0, int32_t L, int32_t nsub,
                          const char* who, BeamPtrs* bp, int32_t max_L = RFI_MAX_COUNT);
// Eigen parameters with defaults applied and the solver resolved.
rfi_status resolve_eig(int nbeam, const rfi_eig_params* p, rfi_eig_params* out, const char* who);
// Entry of a tune table whose beam range holds nbeam (NULL if none or no table).
const rfi_tune_entry* find_tune(const rfi_tune_table* t, int nbeam);
// Range checks of one entry's launch choices for nbeam beams (not the solver,
// which resolve_eig checks).
rfi_status check_tune_entry(const rfi_tune_entry* te, int nbeam, const char* who);

}  // namespace rfi
