"""CPU-only checks of the C ABI: the library loads, exports every function
that include/*.h declares, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2512_16278_amd")


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rfi_[a-z0-9_]+)\s*\(", txt)))


def _lib(name):
    path = os.path.join(PKG, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not built (run __graft_entry__.build())")
    return C.CDLL(path)


def test_every_declared_symbol_is_exported():
    for header, lib in (("rfi.h", "librfi.so"), ("rfi_synth.h", "librfi_synth.so")):
        L = _lib(lib)
        names = _declared(header)
        assert names
        for n in names:
            assert hasattr(L, n), f"{lib} does not export {n}"


def test_argument_errors_are_synchronous():
    from paper_2512_16278_amd import rfi
    L = rfi.lib()
    assert b"gfx950" in L.rfi_version()
    with pytest.raises(rfi.RfiError) as e:
        rfi._check(L.rfi_ccm_accumulate(None, 0, 16, 1, None, None, None, 0, 0, None))
    assert e.value.code == rfi.RFI_E_INVALID
    blk = rfi.rfi_block()
    blk.nbeam, blk.nchan, blk.nsamp, blk.row_stride = 19, 64, 1024, 64
    for b in range(19):
        blk.beam[b] = 16 * (b + 1)          # never dereferenced: validation fails first
    bad = [
        dict(L=0), dict(L=40000), dict(t0=-1), dict(nsub=5, L=256),
    ]
    for kw in bad:
        args = dict(t0=0, L=64, nsub=1)
        args.update(kw)
        code = L.rfi_ccm_accumulate(C.byref(blk), args["t0"], args["L"], args["nsub"],
                                    None, None, None, 0, 0, None)
        assert code in (rfi.RFI_E_INVALID, rfi.RFI_E_OVERFLOW), kw
        assert L.rfi_last_error()
    assert L.rfi_ccm_accumulate(C.byref(blk), 0, 40000, 1, None, None, None, 0, 0, None) == rfi.RFI_E_OVERFLOW
    blk.row_stride = 72                          # not a multiple of 16
    assert L.rfi_ccm_accumulate(C.byref(blk), 0, 64, 1, C.c_void_p(16), C.c_void_p(16),
                                C.c_void_p(16), 0, 0, None) == rfi.RFI_E_INVALID
    blk.row_stride = 64
    blk.nbeam = 80
    assert L.rfi_ccm_accumulate(C.byref(blk), 0, 64, 1, C.c_void_p(16), C.c_void_p(16),
                                C.c_void_p(16), 0, 0, None) == rfi.RFI_E_INVALID
    p = rfi.rfi_eig_params(48, 12, 1, 0)
    assert L.rfi_eig_batched(19, 1, 64, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16),
                             C.byref(p), None, C.c_void_p(16), None, C.c_void_p(16), None) == rfi.RFI_E_INVALID
    p = rfi.rfi_eig_params(64, 12, 1, rfi.RFI_EIG_LANE)
    assert L.rfi_eig_batched(19, 1, 64, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16),
                             C.byref(p), None, C.c_void_p(16), None, C.c_void_p(16), None) == rfi.RFI_E_INVALID
    assert L.rfi_flag(1, 64, C.c_void_p(16), C.c_void_p(16), None, -1.0, 50, None,
                      C.c_void_p(16), None, None, None) == rfi.RFI_E_INVALID
    assert L.rfi_flag(1, 64, C.c_void_p(16), C.c_void_p(16), None, 3.0, 0, None,
                      C.c_void_p(16), None, None, None) == rfi.RFI_E_INVALID
    assert rfi.rfi_flag_workspace_size(99, 4096) > 0
    # long sub-intervals: int64 path up to RFI_MAX_COUNT_LONG
    assert rfi.rfi_ccm_long_workspace_size(19, 4096, 1) > 0
    assert rfi.rfi_ccm_long_workspace_size(1, 4096, 1) == 0
    blk.nbeam, blk.nsamp = 19, 300000
    assert L.rfi_ccm_accumulate_long(C.byref(blk), 0, rfi.RFI_MAX_COUNT_LONG + 1, 1, C.c_void_p(256),
                                     C.c_void_p(256), C.c_void_p(256), None) == rfi.RFI_E_OVERFLOW
    assert L.rfi_ccm_accumulate_long(C.byref(blk), 0, 203450, 1, C.c_void_p(256), C.c_void_p(256),
                                     None, None) == rfi.RFI_E_INVALID
    assert L.rfi_ccm_accumulate(C.byref(blk), 0, 203450, 1, C.c_void_p(256), C.c_void_p(256),
                                C.c_void_p(256), 0, 0, None) == rfi.RFI_E_OVERFLOW
    assert L.rfi_eig_batched_long(1, 1, 64, None, None, None, None, None, None, None) == rfi.RFI_E_INVALID
    assert rfi.rfi_process_workspace_size(19, 4096, rfi.process_params(203450, 1)) > 0
    blk.nsamp = 1024
    # the clip needs a caller workspace (the library allocates nothing), 256-byte aligned
    assert L.rfi_flag(1, 64, C.c_void_p(16), C.c_void_p(16), None, 3.0, 50, None,
                      C.c_void_p(16), None, None, None) == rfi.RFI_E_INVALID
    assert b"workspace" in L.rfi_last_error()
    assert L.rfi_flag(1, 64, C.c_void_p(16), C.c_void_p(16), None, 3.0, 50, None,
                      C.c_void_p(16), None, C.c_void_p(272), None) == rfi.RFI_E_INVALID
    assert L.rfi_clip_fit(-1, None, None, None, 3.0, None, None, None, None) == rfi.RFI_E_INVALID
    assert L.rfi_clip_fit(4, None, None, None, 3.0, None, None, None, None) == rfi.RFI_E_INVALID
    assert L.rfi_flag_noalloc(1 << 11, 1 << 10, C.c_void_p(256), C.c_void_p(256), None, 3.0,
                              50, None, C.c_void_p(256), None, None) == rfi.RFI_E_INVALID
    # per-beam stage: workspace required
    assert 0 < rfi.rfi_eigvec_workspace_size(19, 99, 4096) <= 79 * 256 * 24
    assert rfi.rfi_eigvec_workspace_size(1, 99, 4096) == 0
    assert L.rfi_eigvec_flag(19, 1, 64, C.c_void_p(256), C.c_void_p(256), C.c_void_p(256), None,
                             1.0, C.c_void_p(256), None, None, None, None) == rfi.RFI_E_INVALID
    assert b"workspace" in L.rfi_last_error()
    # ArPLS bandpass and the non-centred matrix: argument checks before any launch
    assert rfi.rfi_bandpass_workspace_size(19, 4096, 1) == 7 * 19 * 4096 * 8
    assert rfi.rfi_bandpass_workspace_size(1, 4096, 1) == 0
    v = C.c_void_p(256)
    assert L.rfi_bandpass_arpls(19, 1, 64, v, v, 0.0, 0.05, 100, v, None, v, None) == rfi.RFI_E_INVALID
    assert L.rfi_bandpass_arpls(19, 1, 64, v, v, 1e5, -0.1, 100, v, None, v, None) == rfi.RFI_E_INVALID
    assert L.rfi_bandpass_arpls(19, 1, 64, v, v, 1e5, 0.05, 0, v, None, v, None) == rfi.RFI_E_INVALID
    assert L.rfi_bandpass_arpls(19, 1, 64, v, v, 1e5, 0.05, 100, v, None, None, None) == rfi.RFI_E_INVALID
    assert L.rfi_bandpass_arpls(19, 0, 64, None, None, 1e5, 0.05, 100, None, None, None, None) == rfi.RFI_OK
    assert L.rfi_eig_noncentred(80, 1, 64, v, v, v, None, None, v, None, v, None) == rfi.RFI_E_INVALID
    assert L.rfi_eig_noncentred(19, 1, 64, v, None, v, None, None, v, None, v, None) == rfi.RFI_E_INVALID


def test_struct_layouts_match_header():
    from paper_2512_16278_amd import rfi
    assert C.sizeof(rfi.rfi_block) == 24 + 8 * rfi.RFI_MAX_BEAMS
    assert C.sizeof(rfi.rfi_flag_stats) == 48
    assert C.sizeof(rfi.rfi_hist_entry) == 32
    assert C.sizeof(rfi.rfi_stream_state) == 48 + 32 * rfi.RFI_HIST_CAP
    hdr = open(os.path.join(ROOT, "include", "rfi.h")).read()
    assert f"#define RFI_MAX_BEAMS {rfi.RFI_MAX_BEAMS}" in hdr
    assert f"#define RFI_HIST_CAP {rfi.RFI_HIST_CAP}" in hdr
    assert f"#define RFI_MAX_COUNT {rfi.RFI_MAX_COUNT}" in hdr


def test_struct_layouts_match_c_compiler(tmp_path):
    """sizeof / offsetof of the ABI structures as gcc sees include/rfi.h equal
    the ctypes mirrors of the binding."""
    import shutil
    import subprocess
    from paper_2512_16278_amd import rfi
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    checks = {
        "rfi_tune_entry": rfi.rfi_tune_entry, "rfi_tune_table": rfi.rfi_tune_table,
        "rfi_batch_params": rfi.rfi_batch_params, "rfi_batch_item": rfi.rfi_batch_item,
        "rfi_block": rfi.rfi_block, "rfi_flag_stats": rfi.rfi_flag_stats,
        "rfi_stream_state": rfi.rfi_stream_state, "rfi_eig_params": rfi.rfi_eig_params,
        "rfi_process_params": rfi.rfi_process_params,
        "rfi_session_config": rfi.rfi_session_config,
        "rfi_stream_config": rfi.rfi_stream_config, "rfi_result": rfi.rfi_result,
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rfi.h"', "int main(void) {"]
    for name, st in checks.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for name, st in checks.items():
        assert int(got[name]) == C.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)


def test_tune_arguments():
    from paper_2512_16278_amd import rfi
    L = rfi.lib()
    assert [L.rfi_ccm_tile_variants(n) for n in (1, 2, 15, 16, 19, 31, 36, 72, 79, 80)] == \
        [0, 1, 1, 3, 3, 3, 1, 1, 1, 0]
    blk = rfi.rfi_block()
    blk.nbeam, blk.nchan, blk.nsamp, blk.row_stride = 19, 64, 1024, 64
    for b in range(19):
        blk.beam[b] = 256 * (b + 1)          # never dereferenced
    items = (rfi.rfi_batch_item * 1)()
    items[0].blk = C.pointer(blk)
    items[0].L, items[0].nsub = 256, 2
    items[0].stat = items[0].status = items[0].mask = 256
    t = rfi.rfi_tune_table()
    p = rfi.rfi_batch_params(32, 12, 50, 0, 3.0, C.pointer(t))
    assert L.rfi_batch_workspace_size(1, items, C.byref(p)) > 0      # empty table
    t.n = 1
    t.e[0].nbeam_lo, t.e[0].nbeam_hi = 16, 31
    for field, val in (("ccm_tile", 3), ("ccm_stages", 5), ("ccm_group_bytes", 1 << 20),
                       ("eig_wg", 96), ("eig_solver", 9)):
        setattr(t.e[0], field, val)
        assert L.rfi_batch_workspace_size(1, items, C.byref(p)) == 0, field
        assert L.rfi_last_error()
        setattr(t.e[0], field, 0)
    t.e[0].ccm_tile, t.e[0].eig_wg, t.e[0].eig_solver = 2, 64, rfi.RFI_EIG_TRIDIAG
    assert L.rfi_batch_workspace_size(1, items, C.byref(p)) > 0
    t.n = 99
    assert L.rfi_batch_workspace_size(1, items, C.byref(p)) == 0
    # two items on one stream state would race in the batched clip: refused
    p2 = rfi.rfi_batch_params(32, 12, 50, 0, 3.0, None)
    items2 = (rfi.rfi_batch_item * 2)()
    for i in range(2):
        items2[i].blk = C.pointer(blk)
        items2[i].L, items2[i].nsub = 256, 2
        items2[i].stat = items2[i].status = items2[i].mask = 256
        items2[i].state = 4096
    assert L.rfi_batch_workspace_size(2, items2, C.byref(p2)) == 0
    assert b"stream state" in L.rfi_last_error()
    items2[1].state = 8192
    assert L.rfi_batch_workspace_size(2, items2, C.byref(p2)) > 0
    assert L.rfi_tune_batch(1, items, C.byref(p), None, None, None) == rfi.RFI_E_INVALID
    out = rfi.rfi_tune_table()
    assert L.rfi_tune_batch(1, items, C.byref(p), None, C.byref(out), None) == rfi.RFI_E_INVALID


def test_process_block_argument_errors():
    from paper_2512_16278_amd import rfi
    L = rfi.lib()
    p = rfi.process_params(256, 4)
    assert rfi.rfi_process_workspace_size(19, 4096, p) > 0
    bad = rfi.process_params(256, 4, group=-1)
    assert rfi.rfi_process_workspace_size(19, 4096, bad) == 0
    assert rfi.rfi_process_workspace_size(1, 4096, p) == 0
    assert L.rfi_process_block(None, C.byref(p), None, None, None, None, None, None, None,
                               None, None, None) == rfi.RFI_E_INVALID
    blk = rfi.rfi_block()
    blk.nbeam, blk.nchan, blk.nsamp, blk.row_stride = 19, 64, 1024, 64
    for b in range(19):
        blk.beam[b] = 16 * (b + 1)          # never dereferenced: validation fails first
    args = [C.c_void_p(256)] * 3
    assert L.rfi_process_block(C.byref(blk), None, None, None, *args, None, None, None,
                               C.c_void_p(256), None) == rfi.RFI_E_INVALID
    # workspace missing / misaligned
    assert L.rfi_process_block(C.byref(blk), C.byref(p), None, None, *args, None, None, None,
                               None, None) == rfi.RFI_E_INVALID
    assert L.rfi_process_block(C.byref(blk), C.byref(p), None, None, *args, None, None, None,
                               C.c_void_p(272), None) == rfi.RFI_E_INVALID
    # samples outside the block; kappa < 0
    assert L.rfi_process_block(C.byref(blk), C.byref(rfi.process_params(256, 5)), None, None,
                               *args, None, None, None, C.c_void_p(256), None) == rfi.RFI_E_INVALID
    assert L.rfi_process_block(C.byref(blk), C.byref(rfi.process_params(256, 4, kappa=-1)),
                               None, None, *args, None, None, None, C.c_void_p(256),
                               None) == rfi.RFI_E_INVALID
    assert b"kappa" in L.rfi_last_error()


def test_session_without_device_or_with_bad_arguments():
    """Session calls validate their arguments before touching a device; with
    no device the session cannot be created."""
    from paper_2512_16278_amd import rfi
    L = rfi.lib()
    h = C.c_void_p()
    cfg = rfi.rfi_session_config(0, 65, 0)                      # too many slots
    assert L.rfi_session_create(C.byref(cfg), C.byref(h)) == rfi.RFI_E_INVALID
    assert L.rfi_session_create(None, None) == rfi.RFI_E_INVALID
    t = C.c_uint64()
    r = rfi.rfi_result()
    assert L.rfi_submit(None, 1, None, 0, C.byref(t)) == rfi.RFI_E_INVALID
    assert L.rfi_poll(None, 1, C.byref(r)) == rfi.RFI_E_INVALID
    assert L.rfi_wait(None, 1, 0, C.byref(r)) == rfi.RFI_E_INVALID
    assert L.rfi_cancel(None, 1) == rfi.RFI_E_INVALID
    assert L.rfi_result_release(None, 1) == rfi.RFI_E_INVALID
    L.rfi_session_destroy(None)
    import torch
    if not torch.cuda.is_available():
        cfg = rfi.rfi_session_config(0, 4, 0)
        assert L.rfi_session_create(C.byref(cfg), C.byref(h)) == rfi.RFI_E_DEVICE


def test_beam_offsets_stagger():
    """rfi_beam_offsets: beam b starts 64 (b mod 64) bytes past a 4 KB
    boundary, 16-byte aligned, and no two beams overlap."""
    from paper_2512_16278_amd import rfi
    for nbeam, nsamp, stride in ((19, 203450, 4096), (72, 1000, 1024), (1, 0, 16), (79, 3, 4112)):
        offs, tot = rfi.rfi_beam_offsets(nbeam, nsamp, stride)
        n = nsamp * stride
        assert len(offs) == nbeam
        for b, o in enumerate(offs):
            assert o % 4096 == 64 * (b % 64)
            assert o % 16 == 0
            assert o + n <= tot
            if b:
                assert offs[b - 1] + n <= o
        assert tot == offs[-1] + n
    L = rfi.lib()
    o, t = (C.c_int64 * 80)(), C.c_int64()
    for args in ((0, 10, 4096), (80, 10, 4096), (19, -1, 4096), (19, 10, 0), (19, 10, 4100)):
        assert L.rfi_beam_offsets(*args, o, C.byref(t)) == rfi.RFI_E_INVALID
    assert L.rfi_beam_offsets(19, 10, 4096, None, C.byref(t)) == rfi.RFI_E_INVALID
    assert L.rfi_beam_offsets(79, 1 << 50, 4096, o, C.byref(t)) == rfi.RFI_E_OVERFLOW


def test_batch_accepts_long_sub_intervals():
    """Batch items take L up to RFI_MAX_COUNT_LONG (the long route of the
    whole-block call); the workspace grows by the int64 records and the chunk
    scratch; beyond the bound the item is refused."""
    from paper_2512_16278_amd import rfi
    L = rfi.lib()
    blk = rfi.rfi_block()
    blk.nbeam, blk.nchan, blk.nsamp, blk.row_stride = 19, 40, 300000, 48
    for b in range(19):
        blk.beam[b] = 256 * (b + 1)          # never dereferenced
    items = (rfi.rfi_batch_item * 1)()
    items[0].blk = C.pointer(blk)
    items[0].stat = items[0].status = items[0].mask = 256
    p = rfi.rfi_batch_params(32, 12, 50, 0, 3.0, None)
    items[0].L, items[0].nsub = rfi.RFI_MAX_COUNT, 2
    short = L.rfi_batch_workspace_size(1, items, C.byref(p))
    items[0].L = rfi.RFI_MAX_COUNT + 1
    long_ = L.rfi_batch_workspace_size(1, items, C.byref(p))
    assert short > 0 and long_ > short
    nrow = 19 + 19 * 20 // 2
    assert long_ - short >= 2 * 40 * nrow * 4       # int64 records instead of int32 sums
    items[0].L, items[0].nsub = rfi.RFI_MAX_COUNT_LONG + 1, 1
    assert L.rfi_batch_workspace_size(1, items, C.byref(p)) == 0
    assert L.rfi_last_error()
