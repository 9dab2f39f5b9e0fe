#!/usr/bin/env python3
"""Throughput of the whole per-block path on one MI355X.

Workload: FAST-shaped block, 19 beams x 4096 channels of uint8 total power,
49.152 us samples, 10 s of data (203,450 samples), 2048-sample sub-intervals
(99 full sub-intervals; the 698-sample tail is not a full cell), synthetic
(seeded, generated on the GPU, device-resident before timing). One step is
one pass of the whole path over the block, by default the three calls

    rfi_ccm_accumulate -> rfi_eig_batched -> rfi_flag

with HIP events recorded between them on the launch stream in every timed
step, or, with --path fused, the single call rfi_process_block (the same
kernels behind one entry point; also timed below the main figure).

Metric: beam-sample GB/s = nbeam * nchan * nsub * L bytes / step time.
The roofline object is for the dominant kernel (the sums kernel, one launch
per step over the whole block): achieved = its algorithmic bytes per launch
(n L input bytes per cell x nsub * nchan cells; the int32 sums it writes are
intermediate, reported apart) / its mean launch time from the events of the
timed steps. The CPU baseline times the FP64 oracle on a bounded sample, on
one thread and on all host cores (one worker process per channel strip).
Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
FP32_VALU_PEAK = 78.6e12       # non-packed FP32 FMA: 256 CU x 64 lanes x 2 x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_strip(task):
    """Worker of the all-core CPU baseline: regenerate channels [c_lo, c_hi)
    of the first nsub sub-intervals (not timed), then run the oracle's
    per-cell part on them (BLAS limited to one thread by the environment)."""
    seconds, nsub, c_lo, c_hi = task
    from oracle import pipeline
    from paper_2512_16278_amd import synth
    spec = synth.fast_spec(seconds=seconds)
    x = synth.generate(spec, 0, nsub * spec.L, c_lo, c_hi)
    t0 = time.time()
    cr = pipeline.cells(x, spec.L, nsub)
    t1 = time.time()
    return c_lo, cr.stat, cr.degenerate, t0, t1, int(x.size)


def cpu_baseline(spec, seconds: float, nsub_sample: int, nchan_single: int, nchan_all: int):
    """The FP64 oracle, as it stands, on bounded samples of the same block
    (bytes regenerated on the CPU, generation not timed):

    * one thread (BLAS pools limited to 1): the whole path -- sums,
      correlation, eigen, statistic, clip -- on channels 0..nchan_single-1 of
      the first nsub_sample sub-intervals;
    * all host cores: one worker process per channel strip of channels
      0..nchan_all-1 (BLAS 1 thread each) runs the per-cell part, the parent
      clips the gathered statistic; wall time from the first worker's start
      to the last one's end, plus the clip.
    """
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import threadpoolctl
    from oracle import clip, pipeline
    from paper_2512_16278_amd import synth
    L = spec.L
    host = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    x = synth.generate(spec, 0, nsub_sample * L, 0, nchan_single)
    log(f"cpu baseline: sample generated in {time.perf_counter() - t0:.1f} s; "
        f"one thread on {x.size / 1e6:.0f} MB")
    with threadpoolctl.threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pipeline.block(x, L, nsub_sample)
        dt1 = time.perf_counter() - t0
    single = {"value": x.size / dt1 / 1e9, "unit": "GB/s", "cores": 1, "seconds": round(dt1, 2),
              "sample": f"channels 0..{nchan_single - 1} x {nsub_sample} sub-int(s) of {L} "
                        f"samples x {spec.nbeam} beams ({x.size / 1e6:.0f} MB)"}
    del x
    workers = max(1, min(host, 16))
    edges = np.linspace(0, nchan_all, workers + 1).astype(int)
    tasks = [(seconds, nsub_sample, int(edges[i]), int(edges[i + 1])) for i in range(workers)
             if edges[i + 1] > edges[i]]
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:
        os.environ[k] = "1"
    try:
        # a worker that dies raises here instead of being replaced
        with ProcessPoolExecutor(len(tasks), mp_context=mp.get_context("spawn")) as pool:
            parts = list(pool.map(_oracle_strip, tasks))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    parts.sort(key=lambda p: p[0])
    stat = np.concatenate([p[1] for p in parts], axis=1)
    deg = np.concatenate([p[2] for p in parts], axis=1)
    with threadpoolctl.threadpool_limits(limits=1):
        t0 = time.perf_counter()
        clip.clip_iterative(stat, pipeline.eligible_cells(deg), 3.0, 50)
        dclip = time.perf_counter() - t0
    wall = max(p[4] for p in parts) - min(p[3] for p in parts) + dclip
    nbytes = sum(p[5] for p in parts)
    return {
        "value": nbytes / wall / 1e9, "unit": "GB/s", "cores": len(tasks), "kind": "oracle",
        "sample": f"channels 0..{nchan_all - 1} x {nsub_sample} sub-int(s) of {L} samples x "
                  f"{spec.nbeam} beams ({nbytes / 1e6:.0f} MB, {nsub_sample * nchan_all} cells) "
                  f"in {len(tasks)} channel strips, one worker process each, BLAS 1 thread; "
                  f"the parent clips the gathered statistic",
        "seconds": round(wall, 2), "host_cores": host, "single_thread": single,
    }


MIX_NBEAM = (7, 19, 36, 72)
MIX_NCHAN = (1024, 4096, 8192)
MIX_L = (512, 1024, 4096)


def precision_split(dev, spec, data, blk, nsub, ev_time):
    """Precision split on the FAST-shaped block: exact int32 sums by the int8
    MFMA engine vs the dot4 VALU engine (bit-exact, timed); FP32 Jacobi, FP32
    Householder + Sturm and FP64 Jacobi on the GPU (timed), each against the
    FP64 oracle on sampled cells (per-cell eigenvalue error, residual of the
    dominant pair), and statistic and mask differences from the FP64 Jacobi
    over every cell."""
    import torch
    from oracle import pipeline
    from paper_2512_16278_amd import rfi, synth
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    ncell = nsub * nc
    npair = nb * (nb + 1) // 2
    sums = {}
    times = {}
    for name, var in (("mfma", rfi.RFI_CCM_MFMA), ("valu", rfi.RFI_CCM_VALU)):
        sx = torch.empty((nb, ncell), dtype=torch.int32, device=dev)
        sxy = torch.empty((npair, ncell), dtype=torch.int32, device=dev)
        cnt = torch.empty(nsub, dtype=torch.int32, device=dev)
        times[f"ccm_{name}_ms"] = ev_time(lambda: rfi.rfi_ccm_accumulate(
            blk, 0, L, nsub, sx, sxy, cnt, variant=var))
        sums[name] = (sx, sxy, cnt)
    exact = bool(torch.equal(sums["mfma"][0], sums["valu"][0]) and
                 torch.equal(sums["mfma"][1], sums["valu"][1]))
    del sums["valu"]
    sx, sxy, cnt = sums["mfma"]
    # (name, precision, solver): the FP32 per-lane Jacobi, the FP32 per-lane
    # Householder + Sturm solver (the default below 21 beams), the FP64 Jacobi
    runs = (("fp32", 32, rfi.RFI_EIG_LANE), ("fp32_householder", 32, rfi.RFI_EIG_LANE_TRI),
            ("fp64", 64, rfi.RFI_EIG_WAVE))
    res = {}
    for name, prec, solver in runs:
        stat = torch.empty(ncell, dtype=torch.float64, device=dev)
        status = torch.empty(ncell, dtype=torch.uint8, device=dev)
        ev = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
        v1 = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
        mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
        times[f"eig_{name}_ms"] = ev_time(lambda: rfi.rfi_eig_batched(
            nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1, precision=prec,
            solver=solver))
        times[f"eig_{name}_stat_only_ms"] = ev_time(lambda: rfi.rfi_eig_batched(
            nb, nsub, nc, sx, sxy, cnt, stat, status, precision=prec, solver=solver))
        rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, eigvals=ev, v1=v1,
                            precision=prec, solver=solver)
        rfi.rfi_flag(nsub, nc, stat, status, mask)
        torch.cuda.synchronize()
        res[name] = dict(stat=stat.cpu().numpy().reshape(nsub, nc),
                         ev=ev.cpu().numpy().reshape(nb, nsub, nc),
                         v1=v1.cpu().numpy().reshape(nb, nsub, nc),
                         status=status.cpu().numpy(), mask=mask.cpu().numpy())
    mask_diff = int(np.count_nonzero(res["fp32"]["mask"] != res["fp64"]["mask"]))
    # sampled cells against the oracle
    k, c_hi = 0, 256
    x = synth.generate(spec, k * L, (k + 1) * L, 0, c_hi)
    cr = pipeline.cells(x, L, 1)
    w_ref = cr.w[0]                                  # [c, n], |lambda| descending
    r_ref = cr.r[0]                                  # [c, n, n]
    out = {"sums_bit_exact_mfma_vs_valu": exact, "mask_disagreements_fp32_vs_fp64": mask_diff,
           "cells": ncell, "sample": f"sub-interval {k}, channels 0..{c_hi - 1} ({c_hi} cells)"}
    for name, prec, solver in runs:
        ev = res[name]["ev"][:, k, :c_hi].T.astype(np.float64)       # [c, n]
        v = res[name]["v1"][:, k, :c_hi].T.astype(np.float64)
        lam1 = w_ref[:, :1]
        nrel = np.abs(ev - w_ref) / np.abs(lam1)
        erel = np.abs(ev - w_ref) / np.abs(w_ref)
        s_err = np.abs(res[name]["stat"][k, :c_hi] - cr.stat[0])
        resid = np.linalg.norm(np.einsum("cab,cb->ca", r_ref, v) - ev[:, :1] * v, axis=1)
        out[name] = {
            "eig_norm_rel_max": float(nrel.max()), "eig_elem_rel_max": float(erel.max()),
            "stat_abs_max": float(s_err.max()), "resid_max": float(resid.max()),
            "not_converged": int(np.count_nonzero(res[name]["status"] & rfi.RFI_CELL_NOT_CONVERGED)),
            # over every cell of the block, against the FP64 Jacobi
            "stat_vs_fp64_all_cells_max": float(np.abs(res[name]["stat"] - res["fp64"]["stat"]).max()),
            "mask_vs_fp64_all_cells": int(np.count_nonzero(res[name]["mask"] != res["fp64"]["mask"])),
        }
    out.update({k2: round(v2, 4) for k2, v2 in times.items()})
    return out


def widened_rows(dev, spec, data, blk, nsub, sx, sxy, cnt, stat, status, mask, ev_time, peak):
    """The calls beyond the three-step path, on the same FAST-shaped block,
    each timed with HIP events on the launch stream (median of 3 after one
    warm-up): the per-beam eigenvector stage, the clip scopes (moment and
    histogram fits), the ArPLS bandpass and the non-centred statistic, and the
    whole 10 s block as one long sub-interval. Bytes are the algorithmic ones
    each call must move (inputs read once, outputs written once)."""
    import torch
    from paper_2512_16278_amd import rfi
    nb, nc, L = spec.nbeam, spec.nchan, spec.L
    ncell = nsub * nc
    out = {}

    def rec(name, ms, nbytes, note):
        out[name] = {"ms": round(ms, 4), "bytes": int(nbytes),
                     "gbs": round(nbytes / (ms / 1e3) / 1e9, 1),
                     "hbm_frac": round(nbytes / (ms / 1e3) / 1e9 / peak, 4), "note": note}

    # per-beam stage on the block's v1 and mask
    v1 = torch.empty((nb, ncell), dtype=torch.float32, device=dev)
    rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, v1=v1)
    rfi.rfi_flag(nsub, nc, stat, status, mask)
    bm = torch.empty((nb, ncell), dtype=torch.uint8, device=dev)
    vws = torch.empty(rfi.rfi_eigvec_workspace_size(nb, nsub, nc), dtype=torch.uint8, device=dev)
    ms = ev_time(lambda: rfi.rfi_eigvec_flag(nb, nsub, nc, v1, mask, status, bm, kappa_v=1.0,
                                             workspace=vws))
    rec("eigvec_stage", ms, nb * ncell * 4 + 2 * ncell + nb * ncell,
        "rfi_eigvec_flag: |v1| fit per beam, beam mask")
    del v1, bm
    # clip scopes
    ws = rfi.flag_workspace(nsub, nc, dev)
    m2 = torch.empty_like(mask)
    for fitname, fit in (("moments", rfi.RFI_FIT_MOMENTS), ("histogram", rfi.RFI_FIT_HISTOGRAM)):
        ms = ev_time(lambda: rfi.rfi_flag_scoped(nsub, nc, stat, status, m2, scopes=7, fit=fit,
                                                 workspace=ws))
        rec(f"scopes_{fitname}", ms, ncell * (8 + 1 + 1),
            f"rfi_flag_scoped: global + per channel + per sub-interval, {fitname} fit")
    del ws, m2
    # ArPLS bandpass from the channel sums, then the non-centred statistic
    z = torch.empty((nb, ncell), dtype=torch.float64, device=dev)
    bws = torch.empty(rfi.rfi_bandpass_workspace_size(nb, nc, nsub), dtype=torch.uint8,
                      device=dev)
    passes = torch.empty((nsub, nb), dtype=torch.int32, device=dev)
    ms = ev_time(lambda: rfi.rfi_bandpass_arpls(nb, nsub, nc, sx, cnt, z, workspace=bws,
                                                passes=passes), reps=1)
    pm = passes.float().mean().item()
    rec("arpls", ms, nb * ncell * (4 + 8),
        f"rfi_bandpass_arpls: {nb * nsub} systems of {nc} channels, mean {pm:.1f} passes")
    del bws
    st2 = torch.empty_like(stat)
    ss2 = torch.empty_like(status)
    npair = nb * (nb + 1) // 2
    ms = ev_time(lambda: rfi.rfi_eig_noncentred(nb, nsub, nc, sx, sxy, cnt, z, st2, ss2))
    rec("noncentred_stat", ms, (nb + npair) * ncell * 4 + nb * ncell * 8 + ncell * 9,
        "rfi_eig_noncentred: FP64 tridiagonal solver on the raw-moment matrix")
    del z, st2, ss2
    # the whole block as one sub-interval of 10 s (Table 1's longest)
    Ll = spec.nsamp
    p = rfi.process_params(Ll, 1)
    pws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, p), dtype=torch.uint8, device=dev)
    sl = torch.empty(nc, dtype=torch.float64, device=dev)
    ssl = torch.empty(nc, dtype=torch.uint8, device=dev)
    msl = torch.empty(nc, dtype=torch.uint8, device=dev)
    ms = ev_time(lambda: rfi.rfi_process_block(blk, p, sl, ssl, msl, pws))
    rec("long_subint", ms, nb * nc * Ll,
        f"rfi_process_block with L = {Ll} (one 10 s sub-interval, {nc} cells): int32 time "
        f"chunks widened to int64, FP64 tridiagonal solver")
    del pws
    torch.cuda.empty_cache()
    return out


def mix_items(dev, nblocks=24, seed=11):
    """The seeded uneven mix (beam counts 7/19/36/72, channels 1024/4096/8192,
    L 512/1024/4096, 0.1-2 s each) as views into per-channel-count pools of
    generated beams: (items, bytes per beam count, total bytes, pools)."""
    import torch
    from paper_2512_16278_amd import rfi, synth
    rng = np.random.default_rng(seed)
    pools = {}
    for F in MIX_NCHAN:
        spec = synth.mixed_spec(seed + F, max(MIX_NBEAM), F, 512, 2.1)
        _, t = rfi.alloc_beams(spec.nbeam, spec.nsamp, F, dev)   # per-beam views
        ds = rfi.DeviceSynth(spec, dev)
        for b in range(spec.nbeam):
            ds.fill(t[b], b)
        pools[F] = t
    items, blocks, nbytes = [], [], 0
    per_class = {}
    for _ in range(nblocks):
        nb, F, L = int(rng.choice(MIX_NBEAM)), int(rng.choice(MIX_NCHAN)), int(rng.choice(MIX_L))
        nsamp = int(rng.uniform(0.1, 2.0) / synth.TSAMP)
        nsub = nsamp // L
        if nsub == 0:
            continue
        start = int(rng.integers(0, pools[F][0].shape[0] - nsamp))
        pool = pools[F]
        blk = rfi.make_block([pool[b][start:start + nsamp] for b in range(nb)], F)
        n = nsub * F
        it = dict(blk=blk, L=L, nsub=nsub,
                  stat=torch.empty(n, dtype=torch.float64, device=dev),
                  status=torch.empty(n, dtype=torch.uint8, device=dev),
                  mask=torch.empty(n, dtype=torch.uint8, device=dev))
        items.append(it)
        nbytes += nb * F * nsub * L
        per_class[nb] = per_class.get(nb, 0) + nb * F * nsub * L
    return items, per_class, nbytes, pools


def batch_class_run(dev, nbeam, reps=3, nblocks=24, seed=11):
    """The blocks of one beam count of the uneven mix as one rfi_process_batch,
    run reps times (a short workload for counter profiles of that class)."""
    import torch
    from paper_2512_16278_amd import rfi
    items, per_class, _, pools = mix_items(dev, nblocks, seed)
    sub = [it for it in items if it["blk"].nbeam == nbeam]
    if not sub:
        raise SystemExit(f"no block of {nbeam} beams in the mix")
    cb = rfi.Batch(sub)
    ws = torch.empty(cb.workspace_size(), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        cb.run(ws)
        b.record(stream)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    cells = sum(it["nsub"] * it["blk"].nchan for it in sub)
    del pools
    return {"nbeam": nbeam, "blocks": len(sub), "cells": cells,
            "bytes_gb": round(per_class[nbeam] / 1e9, 2), "ms": [round(t, 3) for t in ts],
            "ns_per_cell": round(float(np.median(ts)) * 1e6 / cells, 2)}


def batch_bench(dev, nblocks=24, seed=11):
    """Uneven blocks (beam counts 7/19/36/72, channels 1024/4096/8192, L
    512/1024/4096, 0.1-2 s each) through (a) one rfi_process_block per
    block on one stream, (b) one rfi_process_batch, (c) one replay of the
    batch's HIP graph. Same blocks, same outputs; throughput in beam-sample
    GB/s of the full sub-intervals."""
    import torch
    from paper_2512_16278_amd import rfi
    items, per_class, nbytes, pools = mix_items(dev, nblocks, seed)
    stream = torch.cuda.current_stream()
    wss = []
    for it in items:
        p = rfi.process_params(it["L"], it["nsub"])
        nbm = it["blk"].nbeam
        wss.append((p, torch.empty(rfi.rfi_process_workspace_size(nbm, it["blk"].nchan, p),
                                   dtype=torch.uint8, device=dev)))

    def separate():
        for it, (p, ws) in zip(items, wss):
            rfi.rfi_process_block(it["blk"], p, it["stat"], it["status"], it["mask"], ws)

    bt = rfi.Batch(items)
    bws = torch.empty(bt.workspace_size(), dtype=torch.uint8, device=dev)
    g = bt.graph(bws)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    t_sep = timed(separate)
    t_bat = timed(lambda: bt.run(bws))
    t_gr = timed(lambda: g.launch())
    g.close()
    # autotuner: per shape class, on the block with the most cells of the class
    sample = {}
    for it in items:
        nb = it["blk"].nbeam
        c = (nb + 16) // 16
        if c not in sample or it["nsub"] * it["blk"].nchan > sample[c]["nsub"] * sample[c]["blk"].nchan:
            sample[c] = it
    st = rfi.Batch(list(sample.values()))
    sws = torch.empty(st.workspace_size(), dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    table = st.tune(sws)
    tune_s = time.perf_counter() - t0
    del sws
    tb = rfi.Batch(items, tune=table)
    tws = bws if tb.workspace_size() <= bws.numel() else torch.empty(
        tb.workspace_size(), dtype=torch.uint8, device=dev)
    tg = tb.graph(tws)
    t_tg = timed(lambda: tg.launch())
    tg.close()
    # per beam-count class: its blocks alone as one batch; the bound that binds
    # it: HBM (its bytes at 8 TB/s) or, for the FP64 tridiagonal solver above
    # 20 beams, the FP64 vector issue of the reduction ((4/3) n^3 flop per cell
    # at 78.6 TFLOP/s, the floor a perfect kernel would need)
    classes = []
    for nbk in sorted(per_class):
        sub = [it for it in items if it["blk"].nbeam == nbk]
        cb = rfi.Batch(sub)
        cws = bws if cb.workspace_size() <= bws.numel() else torch.empty(
            cb.workspace_size(), dtype=torch.uint8, device=dev)
        tc = timed(lambda: cb.run(cws))
        cells = sum(it["nsub"] * it["blk"].nchan for it in sub)
        hbm_ms = per_class[nbk] / 8e12 * 1e3
        fp64_ms = cells * (4.0 / 3.0) * nbk ** 3 / 78.6e12 * 1e3 if nbk > 20 else 0.0
        classes.append({"nbeam": nbk, "blocks": len(sub), "bytes_gb": round(per_class[nbk] / 1e9, 2),
                        "cells": cells, "ms": round(tc, 3),
                        "gbs": round(per_class[nbk] / tc / 1e6, 1),
                        "hbm_frac": round(hbm_ms / tc, 4),
                        "ns_per_cell": round(tc * 1e6 / cells, 2),
                        "bound": "fp64" if fp64_ms > hbm_ms else "hbm",
                        "bound_frac": round(max(hbm_ms, fp64_ms) / tc, 4)})
    out = {"blocks": len(items), "bytes_gb": round(nbytes / 1e9, 2),
           "classes": classes,
           "bytes_by_nbeam_gb": {str(k): round(v / 1e9, 2) for k, v in sorted(per_class.items())},
           "separate_ms": round(t_sep, 3), "batch_ms": round(t_bat, 3), "graph_ms": round(t_gr, 3),
           "tuned_graph_ms": round(t_tg, 3),
           "separate_gbs": round(nbytes / t_sep / 1e6, 1), "graph_gbs": round(nbytes / t_gr / 1e6, 1),
           "tuned_graph_gbs": round(nbytes / t_tg / 1e6, 1), "tune_s": round(tune_s, 2),
           "tune_table": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in e.items()}
                          for e in rfi.tune_table_dict(table)]}
    del pools
    torch.cuda.empty_cache()
    return out


def serve_bench(dev, rates, nblocks, nstreams=8, seed=7, slots=8, budget=64 << 30):
    """Serving loop: Poisson arrivals of uneven blocks from nstreams streams.

    Each stream has one shape class (nbeam, nchan, L) drawn from the uneven
    mix; its blocks last U(0.1, 2) s (49.152 us samples) and are windows into
    a device-resident pool of synthetic data (pre-generated on the GPU: host
    generation at TB/s is impossible). For every arrival rate the same trace
    runs through a session with `slots` execution slots (continuous batching)
    and through a one-slot session (one block at a time). Throughput counts
    every ingested beam-sample; latency is submit -> results ready.
    """
    import torch
    from paper_2512_16278_amd import rfi, synth
    rng = np.random.default_rng(seed)
    pool_s = 2.2
    pools = {}
    for F in MIX_NCHAN:
        spec = synth.mixed_spec(seed + F, max(MIX_NBEAM), F, 512, pool_s)
        _, t = rfi.alloc_beams(spec.nbeam, spec.nsamp, F, dev)   # per-beam views
        ds = rfi.DeviceSynth(spec, dev)
        for b in range(spec.nbeam):
            ds.fill(t[b], b)
        pools[F] = t
    torch.cuda.synchronize()
    shapes = [(int(rng.choice(MIX_NBEAM)), int(rng.choice(MIX_NCHAN)), int(rng.choice(MIX_L)))
              for _ in range(nstreams)]
    log(f"serving: {nstreams} streams {shapes}; pools {sum(t.numel() for p in pools.values() for t in p) / 1e9:.1f} GB")

    def trace(rate):
        r = np.random.default_rng(seed + int(rate))
        t = np.cumsum(r.exponential(1.0 / rate, size=nblocks))
        out = []
        for ta in t:
            si = int(r.integers(nstreams))
            nb, F, L = shapes[si]
            nsamp = int(r.uniform(0.1, 2.0) / synth.TSAMP)
            start = int(r.integers(0, pools[F][0].shape[0] - nsamp))
            out.append((float(ta), si, start, nsamp))
        return out

    def run(tr, nslot):
        with rfi.Session(max_inflight=nslot, hbm_budget=budget) as S:
            sids = [S.open_stream(nb, F, L) for nb, F, L in shapes]
            blks = []
            for ta, si, start, nsamp in tr:
                nb, F, L = shapes[si]
                pool = pools[F]
                blks.append(rfi.make_block([pool[b][start:start + nsamp] for b in range(nb)], F))
            tickets = []
            t0 = time.perf_counter()
            for (ta, si, start, nsamp), blk in zip(tr, blks):
                while time.perf_counter() - t0 < ta:
                    pass
                tickets.append(S.submit(sids[si], blk))
            lat, byts, t_first, t_last = [], 0, None, 0.0
            for (ta, si, start, nsamp), tk in zip(tr, tickets):
                r = S.wait(tk)
                if r.status != rfi.RFI_OK:
                    raise RuntimeError(f"serving block failed ({r.status})")
                lat.append((r.t_done_us - r.t_submit_us) / 1e3)
                t_first = r.t_submit_us if t_first is None else min(t_first, r.t_submit_us)
                t_last = max(t_last, r.t_done_us)
                nb, F, L = shapes[si]
                byts += nb * F * nsamp
                S.release(tk)
        lat = np.array(lat)
        span = (t_last - t_first) / 1e6
        return {"gbs": round(byts / span / 1e9, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "span_s": round(span, 3)}

    out = {"streams": [list(s) for s in shapes], "blocks_per_rate": nblocks, "slots": slots,
           "budget_gb": budget / 2**30, "rates": []}
    run(trace(rates[0])[:4], slots)                    # warm-up (code objects, pools)
    for rate in rates:
        tr = trace(rate)
        a = run(tr, slots)
        b = run(tr, 1)
        log(f"serving rate {rate}/s: batched {a}  one-at-a-time {b}")
        out["rates"].append({"rate_per_s": rate, "batched": a, "one_at_a_time": b})
    del pools
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="mfma", choices=["mfma", "valu"])
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--cpu-sample-subints", type=int, default=1)
    ap.add_argument("--cpu-sample-chans", type=int, default=1024,
                    help="channels of the one-thread oracle sample")
    ap.add_argument("--cpu-sample-chans-all", type=int, default=4096,
                    help="channels of the all-core oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--path", default="stages", choices=["fused", "stages"])
    ap.add_argument("--group", type=int, default=0, help="sub-intervals per pipeline group")
    ap.add_argument("--serve-rates", default="200,2000",
                    help="arrival rates (blocks/s) of the serving run; empty = skip it")
    ap.add_argument("--serve-blocks", type=int, default=40, help="blocks per serving rate")
    ap.add_argument("--no-precision-split", action="store_true")
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the timings of the per-beam stage, scopes, bandpass and long "
                         "sub-interval calls")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch comparison")
    ap.add_argument("--no-placement", action="store_true",
                    help="skip the sums call on the aligned beam placement")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving loop and print its JSON")
    ap.add_argument("--batch-class", type=int, default=0,
                    help="only run the uneven mix's blocks of this beam count as one batch "
                         "(three runs; a short workload for counter profiles)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the uneven-batch comparison and print its JSON")
    ap.add_argument("--quick", action="store_true",
                    help="time the steps only (no latency, stage split or CPU baseline)")
    ap.add_argument("--profile-run", action="store_true",
                    help="for counter collection: one copy, one streaming read, one three-call "
                         "step and one whole-block step, then the JSON line of those")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (cells are "
              "independent; several GPUs would each take a channel range)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_16278_amd import rfi, synth

    dev = torch.device("cuda:0")
    if args.batch_class:
        print(json.dumps({"batch_class": batch_class_run(dev, args.batch_class)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_bench(dev)}), flush=True)
        return
    if args.serve_only:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        print(json.dumps({"serving": serve_bench(dev, rates, args.serve_blocks)}), flush=True)
        return
    spec = synth.fast_spec(seconds=args.seconds)
    nb, nc, ns, L = spec.nbeam, spec.nchan, spec.nsamp, spec.L
    nsub = ns // L
    ncell = nsub * nc
    npair = nb * (nb + 1) // 2
    stride = (nc + 15) // 16 * 16
    log(f"workload: {nb} beams x {nc} ch x {ns} samples, L={L}, {nsub} sub-ints, "
        f"{spec.nbytes() / 1e9:.2f} GB")
    # beams placed by rfi_beam_offsets (beam b 64 b bytes past a 4 KB
    # boundary); the aligned placement is timed beside it below
    data, beams = rfi.alloc_beams(nb, ns, stride, dev)
    ds = rfi.DeviceSynth(spec, dev)
    for b in range(nb):
        ds.fill(beams[b], b)
    torch.cuda.synchronize()
    log("input generated on the GPU")

    # untimed plain copy of a known 1 GiB: the reference point that scales the
    # HBM byte counters of a profiler run (FETCH_SIZE / WRITE_SIZE per byte)
    calib = data.view(-1)[: 1 << 30].clone()
    del calib
    torch.cuda.synchronize()

    # measured streaming-read peak: the whole input read once by a plain
    # 16-byte-load kernel (median of 5, HIP events on the launch stream)
    sink = torch.empty(rfi.stream_read_sink_words(), dtype=torch.int32, device=dev)
    rd = []
    for _ in range(1 if args.profile_run else 6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        rfi.stream_read(data, sink)
        b.record()
        torch.cuda.synchronize()
        rd.append(a.elapsed_time(b))
    rd = rd[1:] if len(rd) > 1 else rd
    read_gbs = data.numel() / (float(np.median(rd)) / 1e3) / 1e9
    log(f"streaming read of {data.numel() / 1e9:.2f} GB: {read_gbs:.0f} GB/s")

    blk = rfi.make_block(beams, nc)
    sx = torch.empty((nb, ncell), dtype=torch.int32, device=dev)
    sxy = torch.empty((npair, ncell), dtype=torch.int32, device=dev)
    cnt = torch.empty(nsub, dtype=torch.int32, device=dev)
    stat = torch.empty(ncell, dtype=torch.float64, device=dev)
    status = torch.empty(ncell, dtype=torch.uint8, device=dev)
    mask = torch.empty(ncell, dtype=torch.uint8, device=dev)
    fstats = torch.zeros(48, dtype=torch.uint8, device=dev)
    fws = torch.empty(rfi.rfi_flag_workspace_size(nsub, nc), dtype=torch.uint8, device=dev)
    variant = rfi.RFI_CCM_MFMA if args.variant == "mfma" else rfi.RFI_CCM_VALU
    stream = torch.cuda.current_stream()

    pp = rfi.process_params(L, nsub, group=args.group, eig_precision=args.precision)
    pws = torch.empty(rfi.rfi_process_workspace_size(nb, nc, pp), dtype=torch.uint8, device=dev)

    def step_stages(evs=None):
        # evs: four events recorded on the launch stream around the three calls
        if evs is not None:
            evs[0].record(stream)
        rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx, sxy, cnt, variant=variant)
        if evs is not None:
            evs[1].record(stream)
        rfi.rfi_eig_batched(nb, nsub, nc, sx, sxy, cnt, stat, status, precision=args.precision)
        if evs is not None:
            evs[2].record(stream)
        rfi.rfi_flag(nsub, nc, stat, status, mask, out=fstats, workspace=fws)
        if evs is not None:
            evs[3].record(stream)

    def step_fused(evs=None):
        rfi.rfi_process_block(blk, pp, stat, status, mask, pws, out=fstats)

    step = step_fused if args.path == "fused" else step_stages
    if args.profile_run:
        step_stages()
        step_fused()
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "stream_read_gbs": round(read_gbs, 1)}), flush=True)
        return
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # timed region: K steps back to back between two synchronisations; in the
    # three-call path every step also records events between its calls (on
    # the launch stream), which time the dominant kernel live
    mk = lambda: torch.cuda.Event(enable_timing=True)          # noqa: E731
    sev = [[mk() for _ in range(4)] for _ in range(args.steps)]
    t_start, t_end = mk(), mk()
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(args.steps):
        step(sev[i] if args.path == "stages" else None)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps ({args.path}): {ms_step:.3f} ms/step")
    if args.quick:
        nbytes_q = nb * nc * nsub * L
        print(json.dumps({"quick": True, "ms_per_step": round(ms_step, 4),
                          "value": round(nbytes_q / (ms_step / 1e3) / 1e9, 2),
                          "stream_read_gbs": round(read_gbs, 1), "group": args.group,
                          "path": args.path}), flush=True)
        return

    # block latency: each step alone, from an event before it to one after it
    lat = []
    e0, e1 = mk(), mk()
    for _ in range(max(10, min(args.steps, 30))):
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)

    # per-call times: from the timed steps themselves in the three-call path,
    # else from separate three-call steps
    if args.path != "stages":
        sev = [[mk() for _ in range(4)] for _ in range(max(3, min(args.steps, 10)))]
        for evs in sev:
            step_stages(evs)
        torch.cuda.synchronize()
    st = np.array([[evs[i].elapsed_time(evs[i + 1]) for i in range(3)] for evs in sev])
    ms_ccm, ms_eig, ms_flag = st.mean(axis=0)
    med = np.median(st, axis=0)
    log(f"calls (mean ms): ccm {ms_ccm:.3f}  eig {ms_eig:.3f}  flag {ms_flag:.3f}")
    # the other entry point over the same block, for comparison
    other = step_fused if args.path == "stages" else step_stages
    for _ in range(2):
        other()
    torch.cuda.synchronize()
    o0, o1 = mk(), mk()
    o0.record(stream)
    for _ in range(args.steps):
        other()
    o1.record(stream)
    torch.cuda.synchronize()
    ms_other = o0.elapsed_time(o1) / args.steps
    # the timed path's own outputs, for the summary
    step()
    torch.cuda.synchronize()

    nbytes_in = nb * nc * nsub * L
    value = nbytes_in / (ms_step / 1e3) / 1e9
    sums_bytes = 4 * (nb + npair) * ncell
    flags = rfi.flag_stats_from_bytes(fstats.cpu().numpy().tobytes())
    # HBM bytes of the sums kernel from the committed counter summary, while
    # the kernel's source is the one those counters were taken on
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "ccm_traffic_fast19x4096.json")
    if os.path.exists(tpath):
        from paper_2512_16278_amd import prof_summary
        rec = json.load(open(tpath))
        if rec.get("source_sha256") == prof_summary.source_hash() and rec.get("traffic_bytes"):
            traffic = int(rec["traffic_bytes"])
    if ms_ccm >= ms_eig:
        ccm_gbs = nbytes_in / (ms_ccm / 1e3) / 1e9
        roof = {"kernel": "ccm_mfma_kernel (64-channel tiles, one launch per block)"
                          if variant == rfi.RFI_CCM_MFMA else "ccm_valu_kernel",
                "bound": "hbm", "achieved": round(ccm_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ccm_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "ms": round(float(ms_ccm), 4), "algorithmic_bytes": nbytes_in,
                "sums_write_bytes": sums_bytes,
                "derivation": f"{nb} beams x {L} samples = {nb * L} input bytes per cell x "
                              f"{ncell} cells per launch / mean launch time over the "
                              f"{len(sev)} event-timed steps / {HBM_PEAK_GBS:.0f} GB/s"}
    else:
        # algorithmic FP32 flops of the Jacobi: per sweep n(n-1)/2 rotations of
        # 6(n-2) + 12 flops; 6 sweeps (the typical count on noise-dominated cells)
        flop = ncell * 6 * (nb * (nb - 1) / 2) * (6 * (nb - 2) + 12)
        ach = flop / (ms_eig / 1e3)
        roof = {"kernel": "eig_lane_jacobi", "bound": "alu", "achieved": round(ach / 1e12, 2),
                "peak": FP32_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VALU_PEAK, 4), "traffic": None,
                "ms": round(float(ms_eig), 4)}

    def ev_time(fn, reps=3):
        ts = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts[1:]))

    # the same block with every beam at the same offset modulo 4 KB (one
    # [nbeam][nsamp][row] tensor): the sums call alone, median of 5
    layout = None
    if not (args.profile_run or args.no_placement):
        alias = torch.empty((nb, ns, stride), dtype=torch.uint8, device=dev)
        for b in range(nb):
            ds.fill(alias[b], b)
        ablk = rfi.make_block(alias, nc)
        sx2, sxy2, cnt2 = torch.empty_like(sx), torch.empty_like(sxy), torch.empty_like(cnt)
        ms_alias = ev_time(lambda: rfi.rfi_ccm_accumulate(ablk, 0, L, nsub, sx2, sxy2, cnt2,
                                                          variant=variant), reps=5)
        ms_stag = ev_time(lambda: rfi.rfi_ccm_accumulate(blk, 0, L, nsub, sx2, sxy2, cnt2,
                                                         variant=variant), reps=5)
        same = bool(torch.equal(sx2, sx) and torch.equal(sxy2, sxy))
        layout = {"placement": "beam b at 64 (b mod 64) bytes past a 4 KB boundary "
                               "(rfi_beam_offsets)",
                  "ccm_ms_staggered": round(ms_stag, 4), "ccm_ms_aligned": round(ms_alias, 4),
                  "aligned_note": "all beams at the same offset modulo 4 KB",
                  "sums_equal": same}
        del alias, sx2, sxy2, cnt2
        torch.cuda.empty_cache()
        log(f"placement: {layout}")

    widened = None
    if not args.no_widened:
        widened = widened_rows(dev, spec, data, blk, nsub, sx, sxy, cnt, stat, status, mask,
                               ev_time, HBM_PEAK_GBS)
        log(f"widened rows: {widened}")

    psplit = None
    if not args.no_precision_split:
        del sx, sxy
        torch.cuda.empty_cache()
        psplit = precision_split(dev, spec, data, blk, nsub, ev_time)
        log(f"precision split: {psplit}")

    serving = None
    batch = None
    if args.serve_rates or not args.no_batch:
        del data, beams
        torch.cuda.empty_cache()
    if not args.no_batch:
        batch = batch_bench(dev)
        log(f"uneven batch: {batch}")
    if args.serve_rates:
        torch.cuda.empty_cache()
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        serving = serve_bench(dev, rates, args.serve_blocks)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(spec, args.seconds, args.cpu_sample_subints, args.cpu_sample_chans,
                           args.cpu_sample_chans_all)
        log(f"cpu baseline: {cpu['value'] * 1e3:.2f} MB/s on {cpu['cores']} workers, "
            f"{cpu['single_thread']['value'] * 1e3:.2f} MB/s on one thread")

    out = {
        "metric": "beam-sample GB/s through CCM+eigen+flag at 1 GPU; p50/p99 block latency",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int8 MFMA -> int32 sums, f64 correlation, f32 eigen + f64 refinement, f64 clip",
        "data": "synthetic (seeded FAST-shaped, generated on the GPU)",
        "config": {"workload": f"FAST-shaped block: {nb} beams x {nc} channels x {ns} samples "
                               f"(10 s at 49.152 us), L={L}, {nsub} sub-ints, "
                               f"{nbytes_in / 1e9:.2f} GB", "nbeam": nb, "nchan": nc,
                   "L": L, "nsub": nsub, "path": args.path, "ccm": args.variant,
                   "eigen": ("fp32 householder+sturm, fp64 refinement" if args.precision == 32
                             else "fp64 jacobi")},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms": {"path": "three calls", "mean": {"ccm": round(float(ms_ccm), 4),
                      "eig": round(float(ms_eig), 4), "flag": round(float(ms_flag), 4)},
                      "median": {"ccm": round(float(med[0]), 4), "eig": round(float(med[1]), 4),
                                 "flag": round(float(med[2]), 4)}},
        ("fused_ms_per_step" if args.path == "stages" else "stages_ms_per_step"):
            round(ms_other, 4),
        "hbm_frac_whole_path": round(value / HBM_PEAK_GBS, 4),
        "stream_read_gbs": round(read_gbs, 1),
        "frac_of_measured_read": round(value / read_gbs, 4),
        "flagged_cells": int(flags["nflag"]), "clip_iterations": int(flags["iterations"]),
        "roofline": roof,
        "placement": layout,
        "widened": widened,
        "precision_split": psplit,
        "batch": batch,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
