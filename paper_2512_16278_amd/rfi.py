"""Thin ctypes binding of librfi (include/rfi.h) and librfi_synth (include/rfi_synth.h).

Argument marshalling only: every step runs in the HIP library. Tensors are
PyTorch device tensors (used for device memory and streams); their data
pointers and the current HIP stream are passed straight through the C ABI.
Loading fails loudly if the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))

RFI_OK = 0
RFI_E_INVALID, RFI_E_OVERFLOW, RFI_E_NOMEM, RFI_E_BUDGET = -1, -2, -3, -4
RFI_E_DEVICE, RFI_E_NOT_READY, RFI_E_CANCELLED, RFI_E_TIMEOUT = -5, -6, -7, -8
RFI_CELL_DEGENERATE, RFI_CELL_NOT_CONVERGED, RFI_CELL_PROTECTED = 1, 2, 4
RFI_CELL_REFINE_FAILED, RFI_CELL_BAD_COUNT = 8, 16
RFI_MAX_BEAMS = 79
RFI_MAX_COUNT = 33025
RFI_MAX_COUNT_LONG = 262143
RFI_HIST_CAP = 1024
RFI_CCM_AUTO, RFI_CCM_MFMA, RFI_CCM_VALU = 0, 1, 2
RFI_EIG_AUTO, RFI_EIG_LANE, RFI_EIG_WAVE, RFI_EIG_TRIDIAG, RFI_EIG_LANE_TRI = 0, 1, 2, 3, 4
RFI_SCOPE_GLOBAL, RFI_SCOPE_CHANNEL, RFI_SCOPE_SUBINT = 1, 2, 4
RFI_FIT_MOMENTS, RFI_FIT_HISTOGRAM = 0, 1


class RfiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librfi error {code}: {msg}")
        self.code = code


class rfi_block(C.Structure):
    _fields_ = [("nbeam", C.c_int32), ("nchan", C.c_int32), ("nsamp", C.c_int64),
                ("row_stride", C.c_int64), ("beam", C.c_void_p * RFI_MAX_BEAMS)]


class rfi_eig_params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_sweeps", C.c_int32), ("refine", C.c_int32),
                ("solver", C.c_int32)]


class rfi_flag_stats(C.Structure):
    _fields_ = [("mu", C.c_double), ("sigma", C.c_double), ("thr", C.c_double),
                ("iterations", C.c_int32), ("converged", C.c_int32), ("nflag", C.c_int64),
                ("nfit", C.c_int64)]


class rfi_hist_entry(C.Structure):
    _fields_ = [("mu", C.c_double), ("sigma", C.c_double), ("thr", C.c_double),
                ("iterations", C.c_int32), ("converged", C.c_int32)]


class rfi_stream_state(C.Structure):
    _fields_ = [("n", C.c_int64), ("q1", C.c_uint64 * 2), ("q2", C.c_uint64 * 2),
                ("nblocks", C.c_int64), ("hist", rfi_hist_entry * RFI_HIST_CAP)]


class rfi_process_params(C.Structure):
    _fields_ = [("t0", C.c_int64), ("L", C.c_int32), ("nsub", C.c_int32), ("group", C.c_int32),
                ("eig_precision", C.c_int32), ("max_sweeps", C.c_int32), ("max_iter", C.c_int32),
                ("kappa", C.c_double), ("kappa_v", C.c_double), ("beam_mask", C.c_void_p),
                ("scopes", C.c_int32), ("fit", C.c_int32)]


class rfi_batch_item(C.Structure):
    _fields_ = [("blk", C.POINTER(rfi_block)), ("t0", C.c_int64), ("L", C.c_int32),
                ("nsub", C.c_int32), ("protect_chan", C.c_void_p), ("state", C.c_void_p),
                ("stat", C.c_void_p), ("status", C.c_void_p), ("mask", C.c_void_p),
                ("out", C.c_void_p), ("v1", C.c_void_p), ("beam_mask", C.c_void_p)]


class rfi_tune_entry(C.Structure):
    _fields_ = [("nbeam_lo", C.c_int32), ("nbeam_hi", C.c_int32), ("ccm_tile", C.c_int32),
                ("ccm_stages", C.c_int32), ("ccm_group_bytes", C.c_int32),
                ("eig_solver", C.c_int32), ("eig_wg", C.c_int32), ("pad", C.c_int32),
                ("ms_default", C.c_double), ("ms_tuned", C.c_double)]


RFI_TUNE_MAX = 8


class rfi_tune_table(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("e", rfi_tune_entry * RFI_TUNE_MAX)]


def tune_table_dict(t: rfi_tune_table) -> list:
    """Entries of a tune table as dicts."""
    return [{f: getattr(t.e[i], f) for f, _ in rfi_tune_entry._fields_ if f != "pad"}
            for i in range(t.n)]


class rfi_batch_params(C.Structure):
    _fields_ = [("eig_precision", C.c_int32), ("max_sweeps", C.c_int32), ("max_iter", C.c_int32),
                ("pad", C.c_int32), ("kappa", C.c_double), ("tune", C.POINTER(rfi_tune_table)),
                ("kappa_v", C.c_double)]


class rfi_session_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_inflight", C.c_int32), ("hbm_budget", C.c_int64),
                ("tune", C.POINTER(rfi_tune_table))]


class rfi_stream_config(C.Structure):
    _fields_ = [("nbeam", C.c_int32), ("nchan", C.c_int32), ("L", C.c_int32),
                ("eig_precision", C.c_int32), ("max_sweeps", C.c_int32), ("max_iter", C.c_int32),
                ("kappa", C.c_double), ("protect_chan", C.c_void_p), ("beam_stage", C.c_int32),
                ("pad", C.c_int32), ("kappa_v", C.c_double)]


class rfi_result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("user_tag", C.c_uint64), ("stream_id", C.c_int32),
                ("status", C.c_int32), ("nsub", C.c_int32), ("nchan", C.c_int32),
                ("carried", C.c_int32), ("carry_samples", C.c_int64), ("stat", C.c_void_p),
                ("cell_status", C.c_void_p), ("mask", C.c_void_p), ("flag", rfi_flag_stats),
                ("t_submit_us", C.c_double), ("t_admit_us", C.c_double),
                ("t_done_us", C.c_double), ("v1", C.c_void_p), ("beam_mask", C.c_void_p)]


class rfi_synth_spec(C.Structure):
    _fields_ = [("nbeam", C.c_int32), ("nchan", C.c_int32), ("nsamp", C.c_int64),
                ("row_stride", C.c_int64), ("key0", C.c_uint32), ("key1", C.c_uint32),
                ("cdf", C.c_void_p), ("sin_of_chan", C.c_void_p), ("sin_meta", C.c_void_p),
                ("sin_tab", C.c_void_p), ("sin_gain", C.c_void_p), ("pmax", C.c_int32),
                ("nburst", C.c_int32), ("burst_meta", C.c_void_p), ("burst_amp", C.c_void_p),
                ("npulse", C.c_int32), ("pulse_meta", C.c_void_p), ("pulse_delay", C.c_void_p)]


_LIB = None
_SYN = None


def lib_path(name: str = "librfi.so") -> str:
    return os.path.join(PKG, name)


def _load(name):
    path = lib_path(name)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                           f"(python -c 'import __graft_entry__ as g; g.build()')")
    return C.CDLL(path)


def lib():
    """The loaded librfi (ctypes.CDLL), with argument types declared."""
    global _LIB
    if _LIB is None:
        L = _load("librfi.so")
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.rfi_ccm_accumulate.argtypes = [C.POINTER(rfi_block), i64, i32, i32, vp, vp, vp, i32, i32, vp]
        L.rfi_eig_batched.argtypes = [i32, i32, i32, vp, vp, vp, C.POINTER(rfi_eig_params),
                                      vp, vp, vp, vp, vp]
        L.rfi_flag.argtypes = [i32, i32, vp, vp, vp, dbl, i32, vp, vp, vp, vp, vp]
        L.rfi_flag_workspace_size.argtypes = [i32, i32]
        L.rfi_beam_offsets.argtypes = [i32, i64, i64, vp, vp]
        L.rfi_flag_workspace_size.restype = C.c_size_t
        L.rfi_clip_fit.argtypes = [i32, vp, vp, vp, dbl, vp, vp, vp, vp]
        L.rfi_flag_scoped.argtypes = [i32, i32, vp, vp, vp, dbl, i32, i32, i32, vp, vp, vp, vp, vp,
                                      vp]
        L.rfi_ccm_long_workspace_size.argtypes = [i32, i32, i32]
        L.rfi_ccm_long_workspace_size.restype = C.c_size_t
        L.rfi_ccm_accumulate_long.argtypes = [C.POINTER(rfi_block), i64, i32, i32, vp, vp, vp, vp]
        L.rfi_eig_batched_long.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.rfi_flag_noalloc.argtypes = [i32, i32, vp, vp, vp, dbl, i32, vp, vp, vp, vp]
        L.rfi_bandpass_workspace_size.argtypes = [i32, i32, i32]
        L.rfi_bandpass_workspace_size.restype = C.c_size_t
        L.rfi_bandpass_arpls.argtypes = [i32, i32, i32, vp, vp, dbl, dbl, i32, vp, vp, vp, vp]
        L.rfi_eig_noncentred.argtypes = [i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rfi_eigvec_flag.argtypes = [i32, i32, i32, vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp]
        L.rfi_eigvec_workspace_size.argtypes = [i32, i32, i32]
        L.rfi_eigvec_workspace_size.restype = C.c_size_t
        L.rfi_process_workspace_size.argtypes = [i32, i32, C.POINTER(rfi_process_params)]
        L.rfi_process_workspace_size.restype = C.c_size_t
        L.rfi_process_block.argtypes = [C.POINTER(rfi_block), C.POINTER(rfi_process_params),
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        u64 = C.c_uint64
        L.rfi_session_create.argtypes = [C.POINTER(rfi_session_config), C.POINTER(vp)]
        L.rfi_session_destroy.argtypes = [vp]
        L.rfi_session_destroy.restype = None
        L.rfi_stream_open.argtypes = [vp, C.POINTER(rfi_stream_config), C.POINTER(i32)]
        L.rfi_stream_close.argtypes = [vp, i32]
        L.rfi_submit.argtypes = [vp, i32, C.POINTER(rfi_block), u64, C.POINTER(u64)]
        L.rfi_poll.argtypes = [vp, u64, C.POINTER(rfi_result)]
        L.rfi_wait.argtypes = [vp, u64, i64, C.POINTER(rfi_result)]
        L.rfi_cancel.argtypes = [vp, u64]
        L.rfi_result_release.argtypes = [vp, u64]
        L.rfi_result_copy.argtypes = [vp, u64, vp, vp, vp]
        L.rfi_result_copy_beams.argtypes = [vp, u64, vp, vp]
        L.rfi_batch_workspace_size.argtypes = [i32, C.POINTER(rfi_batch_item),
                                               C.POINTER(rfi_batch_params)]
        L.rfi_batch_workspace_size.restype = C.c_size_t
        L.rfi_process_batch.argtypes = [i32, C.POINTER(rfi_batch_item),
                                        C.POINTER(rfi_batch_params), vp, vp]
        L.rfi_batch_graph_create.argtypes = [i32, C.POINTER(rfi_batch_item),
                                             C.POINTER(rfi_batch_params), vp, C.POINTER(vp)]
        L.rfi_batch_graph_launch.argtypes = [vp, vp]
        L.rfi_tune_batch.argtypes = [i32, C.POINTER(rfi_batch_item), C.POINTER(rfi_batch_params),
                                     vp, C.POINTER(rfi_tune_table), vp]
        L.rfi_ccm_tile_variants.argtypes = [i32]
        L.rfi_ccm_tile_variants.restype = i32
        L.rfi_batch_graph_destroy.argtypes = [vp]
        L.rfi_batch_graph_destroy.restype = None
        L.rfi_stream_export.argtypes = [vp, i32, vp, C.POINTER(C.c_size_t)]
        L.rfi_stream_import.argtypes = [vp, i32, vp, C.c_size_t]
        for f in ("rfi_ccm_accumulate", "rfi_ccm_accumulate_long", "rfi_eig_batched_long",
                  "rfi_flag_scoped",
                  "rfi_eig_batched", "rfi_flag", "rfi_clip_fit",
                  "rfi_flag_noalloc", "rfi_bandpass_arpls", "rfi_eig_noncentred",
                  "rfi_eigvec_flag",
                  "rfi_process_block", "rfi_session_create", "rfi_stream_open",
                  "rfi_stream_close", "rfi_submit", "rfi_poll", "rfi_wait", "rfi_cancel",
                  "rfi_result_release", "rfi_stream_export", "rfi_stream_import",
                  "rfi_result_copy", "rfi_result_copy_beams", "rfi_process_batch",
                  "rfi_batch_graph_create",
                  "rfi_batch_graph_launch", "rfi_tune_batch"):
            getattr(L, f).restype = i32
        L.rfi_last_error.restype = C.c_char_p
        L.rfi_version.restype = C.c_char_p
        _LIB = L
    return _LIB


def synth_lib():
    global _SYN
    if _SYN is None:
        S = _load("librfi_synth.so")
        S.rfi_synth_fill.argtypes = [C.POINTER(rfi_synth_spec), C.c_int32, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_void_p]
        S.rfi_synth_fill.restype = C.c_int32
        S.rfi_stream_read_sink_words.restype = C.c_int32
        S.rfi_stream_read.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        S.rfi_stream_read.restype = C.c_int32
        _SYN = S
    return _SYN


def _check(code):
    if code != RFI_OK:
        raise RfiError(code, lib().rfi_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def rfi_beam_offsets(nbeam, nsamp, row_stride):
    """(offsets, total): rfi_beam_offsets' staggered beam placement."""
    offs = (C.c_int64 * int(nbeam))()
    tot = C.c_int64()
    _check(lib().rfi_beam_offsets(int(nbeam), int(nsamp), int(row_stride), offs, C.byref(tot)))
    return [int(o) for o in offs], int(tot.value)


def alloc_beams(nbeam, nsamp, row_stride, device="cuda"):
    """(storage, beams): one device allocation holding nbeam uint8
    [nsamp, row_stride] beams placed by rfi_beam_offsets (from a 4 KB-aligned
    base inside the storage); beams is the list of per-beam views."""
    import torch
    offs, tot = rfi_beam_offsets(nbeam, nsamp, row_stride)
    raw = torch.empty(tot + 4096, dtype=torch.uint8, device=device)
    pad = (-raw.data_ptr()) % 4096
    n = int(nsamp) * int(row_stride)
    beams = [raw[pad + o: pad + o + n].view(int(nsamp), int(row_stride)) for o in offs]
    return raw, beams


def make_block(data, nchan=None) -> rfi_block:
    """rfi_block for a device uint8 tensor [nbeam, nsamp, row_stride] (or a
    list of per-beam [nsamp, row_stride] tensors) holding nchan channels per
    row (default: the whole row)."""
    blk = rfi_block()
    beams = list(data) if isinstance(data, (list, tuple)) else [data[b] for b in range(data.shape[0])]
    blk.nbeam = len(beams)
    blk.nsamp = beams[0].shape[0]
    blk.row_stride = beams[0].stride(0)
    blk.nchan = beams[0].shape[1] if nchan is None else int(nchan)
    for b, t in enumerate(beams):
        blk.beam[b] = t.data_ptr()
    return blk


def rfi_ccm_accumulate(blk: rfi_block, t0, L, nsub, sum_x, sum_xy, count, accumulate=0,
                       variant=RFI_CCM_AUTO, stream=None):
    _check(lib().rfi_ccm_accumulate(C.byref(blk), int(t0), int(L), int(nsub), _ptr(sum_x),
                                    _ptr(sum_xy), _ptr(count), int(accumulate), int(variant),
                                    _stream(stream)))


def rfi_ccm_long_workspace_size(nbeam, nchan, nsub):
    return int(lib().rfi_ccm_long_workspace_size(int(nbeam), int(nchan), int(nsub)))


def rfi_ccm_accumulate_long(blk: rfi_block, t0, L, nsub, sums, count, workspace, stream=None):
    """int64 cell-record sums of long sub-intervals (L <= RFI_MAX_COUNT_LONG)."""
    _check(lib().rfi_ccm_accumulate_long(C.byref(blk), int(t0), int(L), int(nsub), _ptr(sums),
                                         _ptr(count), _ptr(workspace), _stream(stream)))


def rfi_eig_batched_long(nbeam, nsub, nchan, sums, count, stat, status, eigvals=None, v1=None,
                         stream=None):
    _check(lib().rfi_eig_batched_long(int(nbeam), int(nsub), int(nchan), _ptr(sums), _ptr(count),
                                      _ptr(eigvals), _ptr(stat), _ptr(v1), _ptr(status),
                                      _stream(stream)))


def rfi_eig_batched(nbeam, nsub, nchan, sum_x, sum_xy, count, stat, status, eigvals=None,
                    v1=None, precision=32, max_sweeps=12, refine=1, solver=RFI_EIG_AUTO,
                    stream=None):
    p = rfi_eig_params(precision, max_sweeps, refine, solver)
    _check(lib().rfi_eig_batched(int(nbeam), int(nsub), int(nchan), _ptr(sum_x), _ptr(sum_xy),
                                 _ptr(count), C.byref(p), _ptr(eigvals), _ptr(stat), _ptr(v1),
                                 _ptr(status), _stream(stream)))


def rfi_bandpass_workspace_size(nbeam, nchan, nsub):
    return int(lib().rfi_bandpass_workspace_size(int(nbeam), int(nchan), int(nsub)))


def rfi_bandpass_arpls(nbeam, nsub, nchan, sum_x, count, z, workspace=None, passes=None,
                       lam=1e5, ratio=0.05, itermax=100, stream=None):
    """ArPLS baselines z [nbeam, nsub * nchan] (FP64) from the channel sums;
    the workspace is allocated with torch when not given."""
    if workspace is None:
        import torch
        workspace = torch.empty(max(rfi_bandpass_workspace_size(nbeam, nchan, nsub), 1),
                                dtype=torch.uint8, device=z.device)
    _check(lib().rfi_bandpass_arpls(int(nbeam), int(nsub), int(nchan), _ptr(sum_x), _ptr(count),
                                    float(lam), float(ratio), int(itermax), _ptr(z), _ptr(passes),
                                    _ptr(workspace), _stream(stream)))


def rfi_eig_noncentred(nbeam, nsub, nchan, sum_x, sum_xy, count, z, stat, status, eigvals=None,
                       v1=None, stream=None):
    _check(lib().rfi_eig_noncentred(int(nbeam), int(nsub), int(nchan), _ptr(sum_x), _ptr(sum_xy),
                                    _ptr(count), _ptr(z), _ptr(eigvals), _ptr(stat), _ptr(v1),
                                    _ptr(status), _stream(stream)))


def rfi_flag_workspace_size(nsub, nchan):
    return int(lib().rfi_flag_workspace_size(int(nsub), int(nchan)))


def flag_workspace(nsub, nchan, device="cuda"):
    """A device buffer of rfi_flag_workspace_size bytes (torch's allocator
    aligns it to 256 bytes)."""
    import torch
    return torch.empty(max(rfi_flag_workspace_size(nsub, nchan), 1), dtype=torch.uint8,
                       device=device)


def rfi_flag(nsub, nchan, stat, status, mask, protect_chan=None, kappa=3.0, max_iter=50,
             state=None, out=None, workspace=None, stream=None):
    """rfi_flag; workspace=None takes a buffer from torch for this call (the
    library itself allocates nothing)."""
    if workspace is None:
        workspace = flag_workspace(nsub, nchan, stat.device)
    _check(lib().rfi_flag(int(nsub), int(nchan), _ptr(stat), _ptr(status), _ptr(protect_chan),
                          float(kappa), int(max_iter), _ptr(state), _ptr(mask), _ptr(out),
                          _ptr(workspace), _stream(stream)))


def rfi_flag_noalloc(nsub, nchan, stat, status, mask, protect_chan=None, kappa=3.0, max_iter=50,
                     state=None, out=None, stream=None):
    """rfi_flag on the library's fixed workspace (no allocation anywhere)."""
    _check(lib().rfi_flag_noalloc(int(nsub), int(nchan), _ptr(stat), _ptr(status),
                                  _ptr(protect_chan), float(kappa), int(max_iter), _ptr(state),
                                  _ptr(mask), _ptr(out), _stream(stream)))


RFI_FLAG_NOALLOC_MAX_CELLS = 1 << 20


def rfi_flag_scoped(nsub, nchan, stat, status, mask, scopes=RFI_SCOPE_GLOBAL,
                    fit=RFI_FIT_MOMENTS, protect_chan=None, kappa=3.0, max_iter=50, out=None,
                    chan_out=None, sub_out=None, workspace=None, stream=None):
    """rfi_flag_scoped; workspace=None takes a buffer from torch when the
    global moment clip needs one."""
    if workspace is None and (scopes & RFI_SCOPE_GLOBAL) and fit == RFI_FIT_MOMENTS:
        workspace = flag_workspace(nsub, nchan, stat.device)
    _check(lib().rfi_flag_scoped(int(nsub), int(nchan), _ptr(stat), _ptr(status),
                                 _ptr(protect_chan), float(kappa), int(max_iter), int(scopes),
                                 int(fit), _ptr(mask), _ptr(out), _ptr(chan_out), _ptr(sub_out),
                                 _ptr(workspace), _stream(stream)))


def rfi_clip_fit(N, Q1, Q2, mu, sigma, thr, kappa=3.0, stream=None):
    """The clip's exact moment fit on device arrays (N int64 [n]; Q1, Q2
    uint64-as-int64 [n, 2] limb pairs; mu, sigma, thr float64 [n])."""
    _check(lib().rfi_clip_fit(int(N.numel()), _ptr(N), _ptr(Q1), _ptr(Q2), float(kappa), _ptr(mu),
                              _ptr(sigma), _ptr(thr), _stream(stream)))


def process_params(L, nsub, t0=0, group=0, eig_precision=32, max_sweeps=12, max_iter=50,
                   kappa=3.0, kappa_v=1.0, beam_mask=None, scopes=0,
                   fit=RFI_FIT_MOMENTS) -> rfi_process_params:
    """beam_mask: a device uint8 tensor [nbeam, ncell] to run the per-beam stage into;
    scopes / fit: the clip of rfi_flag_scoped instead of the global moment clip."""
    return rfi_process_params(int(t0), int(L), int(nsub), int(group), int(eig_precision),
                              int(max_sweeps), int(max_iter), float(kappa), float(kappa_v),
                              None if beam_mask is None else beam_mask.data_ptr(), int(scopes),
                              int(fit))


def rfi_process_workspace_size(nbeam, nchan, p: rfi_process_params):
    return int(lib().rfi_process_workspace_size(int(nbeam), int(nchan), C.byref(p)))


def rfi_process_block(blk: rfi_block, p: rfi_process_params, stat, status, mask, workspace,
                      protect_chan=None, state=None, eigvals=None, v1=None, out=None,
                      stream=None):
    _check(lib().rfi_process_block(C.byref(blk), C.byref(p), _ptr(protect_chan), _ptr(state),
                                   _ptr(stat), _ptr(status), _ptr(mask), _ptr(eigvals), _ptr(v1),
                                   _ptr(out), _ptr(workspace), _stream(stream)))


def rfi_eigvec_workspace_size(nbeam, nsub, nchan):
    return int(lib().rfi_eigvec_workspace_size(int(nbeam), int(nsub), int(nchan)))


def rfi_eigvec_flag(nbeam, nsub, nchan, v1, mask, status, beam_mask, protect_chan=None,
                    kappa_v=1.0, beam_mu=None, beam_sigma=None, workspace=None, stream=None):
    """rfi_eigvec_flag; workspace=None takes a buffer from torch."""
    if workspace is None:
        import torch
        workspace = torch.empty(max(rfi_eigvec_workspace_size(nbeam, nsub, nchan), 8),
                                dtype=torch.uint8, device=v1.device)
    _check(lib().rfi_eigvec_flag(int(nbeam), int(nsub), int(nchan), _ptr(v1), _ptr(mask),
                                 _ptr(status), _ptr(protect_chan), float(kappa_v), _ptr(beam_mask),
                                 _ptr(beam_mu), _ptr(beam_sigma), _ptr(workspace),
                                 _stream(stream)))


# --- batched uneven blocks --------------------------------------------------------

class Batch:
    """Items for rfi_process_batch / rfi_batch_graph_*. Each item is
    (block, t0, L, nsub, stat, status, mask[, out, state, protect_chan]) with
    device tensors; the ctypes structures are kept alive here."""

    def __init__(self, items, eig_precision=32, max_sweeps=12, max_iter=50, kappa=3.0,
                 tune: "rfi_tune_table | None" = None, kappa_v=1.0):
        self._blocks = [it["blk"] for it in items]
        n = len(items)
        self.n = n
        self.arr = (rfi_batch_item * max(n, 1))()
        for i, it in enumerate(items):
            a = self.arr[i]
            a.blk = C.pointer(self._blocks[i])
            a.t0 = int(it.get("t0", 0))
            a.L = int(it["L"])
            a.nsub = int(it["nsub"])
            a.protect_chan = _ptr(it.get("protect_chan"))
            a.state = _ptr(it.get("state"))
            a.stat = _ptr(it["stat"])
            a.status = _ptr(it["status"])
            a.mask = _ptr(it["mask"])
            a.out = _ptr(it.get("out"))
            a.v1 = _ptr(it.get("v1"))
            a.beam_mask = _ptr(it.get("beam_mask"))
        self.tune_table = tune
        self.p = rfi_batch_params(int(eig_precision), int(max_sweeps), int(max_iter), 0,
                                  float(kappa), C.pointer(tune) if tune is not None else None,
                                  float(kappa_v))

    def workspace_size(self):
        return int(lib().rfi_batch_workspace_size(self.n, self.arr, C.byref(self.p)))

    def run(self, workspace, stream=None):
        _check(lib().rfi_process_batch(self.n, self.arr, C.byref(self.p), _ptr(workspace),
                                       _stream(stream)))

    def tune(self, workspace, stream=None) -> rfi_tune_table:
        """rfi_tune_batch on these items: the per-class launch choices (the
        table is not applied; pass it as Batch(..., tune=table))."""
        t = rfi_tune_table()
        _check(lib().rfi_tune_batch(self.n, self.arr, C.byref(self.p), _ptr(workspace), C.byref(t),
                                    _stream(stream)))
        return t

    def graph(self, workspace):
        return BatchGraph(self, workspace)


class BatchGraph:
    def __init__(self, batch: Batch, workspace):
        self.h = C.c_void_p()
        _check(lib().rfi_batch_graph_create(batch.n, batch.arr, C.byref(batch.p), _ptr(workspace),
                                            C.byref(self.h)))

    def launch(self, stream=None):
        _check(lib().rfi_batch_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            lib().rfi_batch_graph_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- serving session ------------------------------------------------------------

class Session:
    """Thin wrapper of an rfi_session (continuous batching of blocks)."""

    def __init__(self, device=0, max_inflight=8, hbm_budget=0,
                 tune: "rfi_tune_table | None" = None):
        self.h = C.c_void_p()
        cfg = rfi_session_config(int(device), int(max_inflight), int(hbm_budget),
                                 C.pointer(tune) if tune is not None else None)
        _check(lib().rfi_session_create(C.byref(cfg), C.byref(self.h)))

    def close(self):
        if self.h:
            lib().rfi_session_destroy(self.h)
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def open_stream(self, nbeam, nchan, L, kappa=3.0, max_iter=50, eig_precision=32,
                    max_sweeps=12, protect_chan=None, beam_stage=False, kappa_v=1.0) -> int:
        keep = None
        pp = None
        if protect_chan is not None:
            keep = np.ascontiguousarray(np.asarray(protect_chan, dtype=np.uint8))
            pp = keep.ctypes.data
        cfg = rfi_stream_config(int(nbeam), int(nchan), int(L), int(eig_precision),
                                int(max_sweeps), int(max_iter), float(kappa), pp,
                                1 if beam_stage else 0, 0, float(kappa_v))
        sid = C.c_int32()
        _check(lib().rfi_stream_open(self.h, C.byref(cfg), C.byref(sid)))
        return sid.value

    def close_stream(self, sid):
        _check(lib().rfi_stream_close(self.h, int(sid)))

    def submit(self, sid, blk: rfi_block, tag=0) -> int:
        t = C.c_uint64()
        _check(lib().rfi_submit(self.h, int(sid), C.byref(blk), int(tag), C.byref(t)))
        return t.value

    def poll(self, ticket):
        r = rfi_result()
        code = lib().rfi_poll(self.h, int(ticket), C.byref(r))
        if code == RFI_E_NOT_READY:
            return None
        _check(code)
        return r

    def wait(self, ticket, timeout_us=-1) -> rfi_result:
        r = rfi_result()
        _check(lib().rfi_wait(self.h, int(ticket), int(timeout_us), C.byref(r)))
        return r

    def cancel(self, ticket) -> int:
        return int(lib().rfi_cancel(self.h, int(ticket)))

    def release(self, ticket):
        _check(lib().rfi_result_release(self.h, int(ticket)))

    def export_stream(self, sid) -> bytes:
        n = C.c_size_t(0)
        _check(lib().rfi_stream_export(self.h, int(sid), None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().rfi_stream_export(self.h, int(sid), buf, C.byref(n)))
        return buf.raw[: n.value]

    def import_stream(self, sid, raw: bytes):
        buf = C.create_string_buffer(raw, len(raw))
        _check(lib().rfi_stream_import(self.h, int(sid), buf, len(raw)))


def result_arrays(sess: "Session", r: rfi_result):
    """Host copies (stat, cell status, mask) of a done ticket's results."""
    n = r.nsub * r.nchan
    stat = np.zeros(n, dtype=np.float64)
    cst = np.zeros(n, dtype=np.uint8)
    mask = np.zeros(n, dtype=np.uint8)
    _check(lib().rfi_result_copy(sess.h, r.ticket, stat.ctypes.data, cst.ctypes.data,
                                 mask.ctypes.data))
    return stat, cst, mask


def result_beams(sess: "Session", r: rfi_result, nbeam: int):
    """Host copies (v1 [nbeam, ncell], beam mask [nbeam, ncell]) of a done
    ticket of a stream opened with beam_stage."""
    n = r.nsub * r.nchan
    v1 = np.zeros((nbeam, n), dtype=np.float32)
    bm = np.zeros((nbeam, n), dtype=np.uint8)
    _check(lib().rfi_result_copy_beams(sess.h, r.ticket, v1.ctypes.data, bm.ctypes.data))
    return v1, bm


def flag_stats_from_bytes(raw: bytes) -> dict:
    s = rfi_flag_stats.from_buffer_copy(raw)
    return dict(mu=s.mu, sigma=s.sigma, thr=s.thr, iterations=s.iterations,
                converged=s.converged, nflag=s.nflag, nfit=s.nfit)


def stream_state_from_bytes(raw: bytes) -> rfi_stream_state:
    return rfi_stream_state.from_buffer_copy(raw)


# --- measurement and input infrastructure ----------------------------------------

def stream_read_sink_words() -> int:
    return int(synth_lib().rfi_stream_read_sink_words())


def stream_read(t, sink, nbytes=None, stream=None):
    """Read nbytes (default: all) of device tensor t once (HBM roofline reference)."""
    n = t.numel() * t.element_size() if nbytes is None else int(nbytes)
    r = synth_lib().rfi_stream_read(C.c_void_p(t.data_ptr()), n, _ptr(sink), _stream(stream))
    if r != 0:
        raise RuntimeError(f"rfi_stream_read failed ({r})")


class DeviceSynth:
    """Device copies of a SynthSpec's integer tables and rfi_synth_fill calls."""

    def __init__(self, spec, device="cuda"):
        import torch
        from . import synth as _s
        tabs = _s.device_tables(spec)
        self.spec = spec
        self._keep = {}

        def dev(a, dtype):
            t = torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).to(device)
            self._keep[id(t)] = t
            return t

        cdf = dev(tabs["cdf"].astype(np.uint32).view(np.int32), np.int32)
        self.c = rfi_synth_spec()
        c = self.c
        c.nbeam, c.nchan, c.nsamp = spec.nbeam, spec.nchan, spec.nsamp
        c.key0, c.key1 = spec.key
        c.cdf = cdf.data_ptr()
        c.sin_of_chan = dev(tabs["sin_of_chan"], np.int32).data_ptr()
        c.sin_meta = dev(tabs["sin_meta"], np.int64).data_ptr()
        c.sin_tab = dev(tabs["sin_tab"], np.int32).data_ptr()
        c.sin_gain = dev(tabs["sin_gain"], np.int32).data_ptr()
        c.pmax = int(tabs["pmax"])
        c.nburst = int(tabs["nburst"])
        c.burst_meta = dev(tabs["burst_meta"], np.int64).data_ptr()
        c.burst_amp = dev(tabs["burst_amp"], np.int32).data_ptr()
        c.npulse = int(tabs["npulse"])
        c.pulse_meta = dev(tabs["pulse_meta"], np.int64).data_ptr()
        c.pulse_delay = dev(tabs["pulse_delay"], np.int32).data_ptr()

    def fill(self, beam_tensor, beam, t_lo=0, t_hi=None, stream=None):
        """Write rows [t_lo, t_hi) of `beam` into beam_tensor[t_lo:t_hi] (a
        device uint8 [nsamp, row_stride] tensor)."""
        t_hi = self.spec.nsamp if t_hi is None else t_hi
        self.c.row_stride = beam_tensor.stride(0)
        dst = beam_tensor.data_ptr() + t_lo * beam_tensor.stride(0)
        r = synth_lib().rfi_synth_fill(C.byref(self.c), int(beam), int(t_lo), int(t_hi),
                                       C.c_void_p(dst), _stream(stream))
        if r != 0:
            raise RuntimeError(f"rfi_synth_fill failed ({r})")
